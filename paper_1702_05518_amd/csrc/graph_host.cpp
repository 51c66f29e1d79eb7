// graph_host.cpp -- host half of libgmrf: graph validation, coloring checks,
// connected components, the color-slab permutation, the chunks of the
// one-launch sweep and the greedy coloring.  No HIP calls here, so every
// check runs (and is tested) without a GPU.
//
// The coloring is the pre-computation of Sec. 2.3: the sites of one color
// must share no edge, and each color becomes a contiguous slab so a color pass
// reads and writes one dense range of the site arrays.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>
#include <numeric>
#include <string>

#include "internal.hpp"

namespace gmrf {

namespace {

thread_local std::string g_error;

std::string edge_str(int64_t i, int64_t j)
{
    char buf[96];
    std::snprintf(buf, sizeof buf, "(%lld, %lld)", (long long)i, (long long)j);
    return buf;
}

int64_t count_components(int64_t n, const std::vector<int64_t> &rp, const int32_t *col)
{
    // union-find with path halving
    std::vector<int64_t> parent(n);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int64_t v) {
        while (parent[v] != v) {
            parent[v] = parent[parent[v]];
            v = parent[v];
        }
        return v;
    };
    int64_t comps = n;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            int64_t a = find(i), b = find(col[e]);
            if (a != b) {
                parent[std::max(a, b)] = std::min(a, b);
                --comps;
            }
        }
    return comps;
}

// Hop distances from a set of sources (one per connected component, the
// components being disjoint each is a plain breadth-first search from its
// source).
std::vector<int32_t> hop_distances(int64_t n, const std::vector<int64_t> &rp, const int32_t *col,
                                   const std::vector<int64_t> &sources)
{
    std::vector<int32_t> d(n, -1);
    std::vector<int64_t> queue;
    queue.reserve(n);
    for (int64_t s : sources) {
        d[s] = 0;
        queue.push_back(s);
    }
    for (size_t head = 0; head < queue.size(); ++head) {
        const int64_t v = queue[head];
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int64_t u = col[e];
            if (d[u] < 0) {
                d[u] = d[v] + 1;
                queue.push_back(u);
            }
        }
    }
    return d;
}

// The site of each component that maximises score (ties: smallest id).
template <typename F>
std::vector<int64_t> argmax_per_component(int64_t n, const std::vector<int32_t> &comp,
                                          int64_t ncomp, F score)
{
    std::vector<int64_t> best(ncomp, -1);
    std::vector<int64_t> val(ncomp, std::numeric_limits<int64_t>::min());
    for (int64_t i = 0; i < n; ++i) {
        const int64_t v = score(i);
        if (v > val[comp[i]]) {
            val[comp[i]] = v;
            best[comp[i]] = i;
        }
    }
    return best;
}

// Sizes of the chunk a set of owned sites would make: its staged sites
// (R, the owned sites closed under "lower-colored neighbour", and H, the
// other neighbours of R), |R| and the neighbour entries of R.  mark and hmark
// are scratch stamped with `tag`.
struct ChunkSize {
    int64_t nloc, nr, nadj;
};

ChunkSize chunk_size(const std::vector<int64_t> &rp, const int32_t *col, const int32_t *color,
                     const std::vector<int64_t> &owned, std::vector<int64_t> &mark,
                     std::vector<int64_t> &hmark, int64_t tag, std::vector<int64_t> &stack)
{
    ChunkSize cs{0, 0, 0};
    stack.clear();
    for (int64_t u : owned) {
        mark[u] = tag;
        stack.push_back(u);
    }
    std::vector<int64_t> R;
    while (!stack.empty()) {
        const int64_t u = stack.back();
        stack.pop_back();
        R.push_back(u);
        cs.nadj += rp[u + 1] - rp[u];
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e)
            if (color[col[e]] < color[u] && mark[col[e]] != tag) {
                mark[col[e]] = tag;
                stack.push_back(col[e]);
            }
    }
    cs.nr = (int64_t)R.size();
    cs.nloc = cs.nr;
    for (int64_t u : R)
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e)
            if (mark[col[e]] != tag && hmark[col[e]] != tag) {
                hmark[col[e]] = tag;
                cs.nloc++;
            }
    cs.nadj = (cs.nadj + 7) / 8 * 8;     // padded as the chunk tables pad it
    return cs;
}

// The chunks of the one-launch sweep, as cells of sites, and a locality
// order in which every cell is one run (cells in order, each in
// breadth-first order from its seed).
//  1. Coordinates: in each connected component, the hop distances from three
//     sites -- the farthest from the component's smallest id (s1), the
//     farthest from s1 (s2), the farthest from both (s3).  On a planar mesh
//     they behave like coordinates of the embedding.
//  2. Seeds: recursive bisection of each component on the coordinate with
//     the widest spread, down to boxes of kChunkSites sites; a box's seed is
//     its member nearest the box's mean coordinates.
//  3. Cells: a breadth-first search from all seeds at once gives each site
//     to the nearest seed (graph distance), a cell closing at 5/4 of the
//     chunk size; sites left over seed further cells.  Cells below a quarter
//     of the chunk size join their smallest neighbouring cell.
//  4. A cell whose chunk would outgrow either LDS cap (FP64 or FP32 values)
//     is split in two by distance from two far-apart members, until every
//     chunk fits or the cell is small (under 8 sites; at most ten rounds).
// The cells are compact (a ball of the graph), which keeps the recomputed
// closure and the read-only halo of each chunk small.
void chunk_cells(int64_t n, const std::vector<int64_t> &rp, const int32_t *col,
                 const int32_t *color, std::vector<int32_t> &cell, std::vector<int64_t> &order)
{
    std::vector<int32_t> comp(n, -1);
    std::vector<int64_t> seeds;
    {
        std::vector<int64_t> queue;
        queue.reserve(n);
        for (int64_t s = 0; s < n; ++s) {
            if (comp[s] >= 0)
                continue;
            const int32_t id = (int32_t)seeds.size();
            seeds.push_back(s);
            comp[s] = id;
            queue.clear();
            queue.push_back(s);
            for (size_t head = 0; head < queue.size(); ++head) {
                const int64_t v = queue[head];
                for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
                    if (comp[col[e]] < 0) {
                        comp[col[e]] = id;
                        queue.push_back(col[e]);
                    }
            }
        }
    }
    const int64_t ncomp = (int64_t)seeds.size();
    const std::vector<int32_t> d0 = hop_distances(n, rp, col, seeds);
    const std::vector<int64_t> s1 = argmax_per_component(n, comp, ncomp,
                                                         [&](int64_t i) { return d0[i]; });
    const std::vector<int32_t> d1 = hop_distances(n, rp, col, s1);
    const std::vector<int64_t> s2 = argmax_per_component(n, comp, ncomp,
                                                         [&](int64_t i) { return d1[i]; });
    const std::vector<int32_t> d2 = hop_distances(n, rp, col, s2);
    const std::vector<int64_t> s3 = argmax_per_component(
        n, comp, ncomp, [&](int64_t i) { return std::min(d1[i], d2[i]); });
    const std::vector<int32_t> d3 = hop_distances(n, rp, col, s3);
    const int32_t *dim[3] = {d1.data(), d2.data(), d3.data()};

    // 2. recursive bisection into boxes, one seed each
    std::vector<int64_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return comp[a] < comp[b]; });
    std::vector<std::pair<int64_t, int64_t>> stack, boxes;
    for (int64_t lo = 0, i = 1; i <= n; ++i)
        if (i == n || comp[idx[i]] != comp[idx[lo]]) {
            stack.push_back({lo, i});
            lo = i;
        }
    std::reverse(stack.begin(), stack.end());
    while (!stack.empty()) {
        const auto [a, b] = stack.back();
        stack.pop_back();
        const int64_t parts = (b - a + kChunkSites - 1) / kChunkSites;
        if (parts <= 1) {
            boxes.push_back({a, b});
            continue;
        }
        int best = 0;
        int64_t spread = -1;
        for (int d = 0; d < 3; ++d) {
            int32_t mn = std::numeric_limits<int32_t>::max(), mx = -1;
            for (int64_t i = a; i < b; ++i) {
                mn = std::min(mn, dim[d][idx[i]]);
                mx = std::max(mx, dim[d][idx[i]]);
            }
            if ((int64_t)mx - mn > spread) {
                spread = (int64_t)mx - mn;
                best = d;
            }
        }
        const int64_t left = (parts / 2) * kChunkSites;
        const int32_t *v = dim[best];
        std::nth_element(idx.begin() + a, idx.begin() + a + left, idx.begin() + b,
                         [&](int64_t x, int64_t y) { return v[x] != v[y] ? v[x] < v[y] : x < y; });
        stack.push_back({a + left, b});
        stack.push_back({a, a + left});
    }

    // 3. capacity-bounded cells around the seeds
    const int64_t cap = kChunkSites + kChunkSites / 4;
    cell.assign(n, -1);
    std::vector<int64_t> size, queue;
    queue.reserve(n);
    auto grow = [&](size_t head) {
        for (; head < queue.size(); ++head) {
            const int64_t v = queue[head];
            const int32_t c = cell[v];
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
                if (cell[col[e]] < 0 && size[c] < cap) {
                    cell[col[e]] = c;
                    size[c]++;
                    queue.push_back(col[e]);
                }
        }
    };
    for (const auto &bx : boxes) {
        double m[3] = {0.0, 0.0, 0.0};
        for (int64_t i = bx.first; i < bx.second; ++i)
            for (int d = 0; d < 3; ++d)
                m[d] += dim[d][idx[i]];
        int64_t seed = idx[bx.first];
        double bd = std::numeric_limits<double>::max();
        for (int64_t i = bx.first; i < bx.second; ++i) {
            double dd = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double z = dim[d][idx[i]] - m[d] / (double)(bx.second - bx.first);
                dd += z * z;
            }
            if (dd < bd) {
                bd = dd;
                seed = idx[i];
            }
        }
        cell[seed] = (int32_t)size.size();
        size.push_back(1);
        queue.push_back(seed);
    }
    grow(0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t s0 = idx[i];               // leftovers, in box order
        if (cell[s0] >= 0)
            continue;
        const size_t head = queue.size();
        cell[s0] = (int32_t)size.size();
        size.push_back(1);
        queue.push_back(s0);
        grow(head);
    }
    auto members = [&]() {
        std::vector<std::vector<int64_t>> mem(size.size());
        for (int64_t v : queue)
            mem[cell[v]].push_back(v);
        return mem;
    };
    {
        std::vector<std::vector<int64_t>> mem = members();
        for (size_t c = 0; c < mem.size(); ++c) {
            if (mem[c].empty() || (int64_t)mem[c].size() >= kChunkSites / 4)
                continue;
            int32_t to = -1;
            for (int64_t v : mem[c])
                for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
                    const int32_t d = cell[col[e]];
                    if (d != (int32_t)c && (to < 0 || mem[d].size() < mem[to].size()))
                        to = d;
                }
            if (to < 0)
                continue;                            // a small component: stays a cell
            for (int64_t v : mem[c]) {
                cell[v] = to;
                mem[to].push_back(v);
            }
            mem[c].clear();
        }
        // renumber the cells in order of their first member in the search
        // order, each cell's members in that order
        std::vector<int32_t> renum(mem.size(), -1);
        int32_t nc = 0;
        for (int64_t v : queue)
            if (renum[cell[v]] < 0)
                renum[cell[v]] = nc++;
        for (int64_t i = 0; i < n; ++i)
            cell[i] = renum[cell[i]];
        size.assign(nc, 0);
        for (int64_t i = 0; i < n; ++i)
            size[cell[i]]++;
    }

    // 4. split cells whose chunk would outgrow the LDS limit
    std::vector<int64_t> mark(n, -1), hmark(n, -1), scratch, dist(n, -1);
    int64_t tag = 0;
    std::vector<int32_t> check(size.size());            // cells to check in this pass
    std::iota(check.begin(), check.end(), 0);
    for (int round = 0; round < 10 && !check.empty(); ++round) {
        std::vector<std::vector<int64_t>> mem(size.size());
        for (int64_t v : queue)
            mem[cell[v]].push_back(v);
        std::vector<int32_t> next;
        for (const int32_t c : check) {
            if ((int64_t)mem[c].size() < 8)
                continue;
            const ChunkSize cs = chunk_size(rp, col, color, mem[c], mark, hmark, ++tag, scratch);
            if (chunk_fits_lds(cs.nloc, cs.nr, cs.nadj))
                continue;
            // two far-apart members: the farthest from the first member, then
            // the farthest from that (hop distances inside the cell)
            auto bfs_in_cell = [&](int64_t from) {
                for (int64_t v : mem[c])
                    dist[v] = -1;
                std::vector<int64_t> q{from};
                dist[from] = 0;
                for (size_t h = 0; h < q.size(); ++h)
                    for (int64_t e = rp[q[h]]; e < rp[q[h] + 1]; ++e) {
                        const int64_t u = col[e];
                        if (cell[u] == (int32_t)c && dist[u] < 0) {
                            dist[u] = dist[q[h]] + 1;
                            q.push_back(u);
                        }
                    }
                return q.back();
            };
            const int64_t pa = bfs_in_cell(mem[c][0]);
            const int64_t pb = bfs_in_cell(pa);
            std::vector<int64_t> da(mem[c].size());
            bfs_in_cell(pa);
            for (size_t i = 0; i < mem[c].size(); ++i)
                da[i] = dist[mem[c][i]];
            bfs_in_cell(pb);
            const int32_t fresh = (int32_t)size.size();
            size.push_back(0);
            for (size_t i = 0; i < mem[c].size(); ++i)
                if (dist[mem[c][i]] >= 0 && (da[i] < 0 || dist[mem[c][i]] < da[i])) {
                    cell[mem[c][i]] = fresh;
                    size[fresh]++;
                    size[c]--;
                }
            next.push_back(c);
            next.push_back(fresh);
        }
        check.swap(next);
    }
    // the order: cells by first member in the search order, members in it
    std::vector<int32_t> renum(size.size(), -1);
    int32_t nc = 0;
    for (int64_t v : queue)
        if (renum[cell[v]] < 0)
            renum[cell[v]] = nc++;
    std::vector<int64_t> start(nc + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        cell[i] = renum[cell[i]];
        start[cell[i] + 1]++;
    }
    for (int32_t c = 0; c < nc; ++c)
        start[c + 1] += start[c];
    order.assign(n, 0);
    for (int64_t v : queue)
        order[start[cell[v]]++] = v;
}

// Chunks of the one-launch sweep.  A color's sites are conditionally
// independent given the others (Sec. 2.3), so a block can produce the new
// values of the sites it owns if it also recomputes, color by color, every
// site whose new value they read: the owned sites' lower-colored neighbours,
// theirs, and so on (R_b); every other neighbour of R_b is read at its value
// from before the sweep (H_b).  The random numbers are keyed by site, so a
// recomputed site is bitwise its owner's value.  Chunk b owns the sites of
// cell b (chunk_cells; cell: by original id).  Sets chunks_ok (and fills the
// tables) only if every chunk fits the LDS and index limits.
void build_chunks(HostGraph *g, const std::vector<int32_t> &cell)
{
    const int64_t n = g->n;
    const int32_t k = g->k;
    g->chunks_ok = false;
    if (k > kFusedMaxColors)
        return;
    g->nchunks = 1 + *std::max_element(cell.begin(), cell.end());
    std::vector<int32_t> colpos(n), chunk(n);
    for (int32_t c = 0; c < k; ++c)
        for (int32_t p = g->slab_offsets[c]; p < g->slab_offsets[c + 1]; ++p)
            colpos[p] = c;
    // owned sites of each chunk, ascending slab position (so by color)
    std::vector<int32_t> own_off(g->nchunks + 1, 0), own(n);
    for (int64_t p = 0; p < n; ++p) {
        chunk[p] = cell[g->orig_of_slab[p]];
        own_off[chunk[p] + 1]++;
    }
    for (int32_t b = 0; b < g->nchunks; ++b)
        own_off[b + 1] += own_off[b];
    {
        std::vector<int32_t> fill(own_off.begin(), own_off.end() - 1);
        for (int64_t p = 0; p < n; ++p)
            own[fill[chunk[p]]++] = (int32_t)p;
    }
    std::vector<int32_t> mark(n, -1), hmark(n, -1), slot(n, -1);
    std::vector<int32_t> R, H, stack;
    g->ch_loc.assign(1, 0);
    g->ch_row.assign(1, 0);
    g->ch_adj.assign(1, 0);
    g->ch_meta.clear();
    g->loc_site.clear();
    g->loc_id.clear();
    g->loc_row.clear();
    g->loc_adj.clear();
    g->max_local = g->max_r = g->max_adj = 0;
    g->max_image4 = g->max_image8 = 0;
    for (int32_t b = 0; b < g->nchunks; ++b) {
        R.clear();
        H.clear();
        stack.clear();
        for (int32_t q = own_off[b]; q < own_off[b + 1]; ++q) {
            mark[own[q]] = b;
            stack.push_back(own[q]);
        }
        while (!stack.empty()) {
            const int32_t u = stack.back();
            stack.pop_back();
            R.push_back(u);
            for (int32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
                const int32_t v = g->col[e];
                if (colpos[v] < colpos[u] && mark[v] != b) {
                    mark[v] = b;
                    stack.push_back(v);
                }
            }
        }
        // R by color, the owned sites first within a color, then by position
        std::sort(R.begin(), R.end(), [&](int32_t a, int32_t c) {
            if (colpos[a] != colpos[c])
                return colpos[a] < colpos[c];
            const bool oa = chunk[a] == b, oc = chunk[c] == b;
            return oa != oc ? oa : a < c;
        });
        for (int32_t u : R)
            for (int32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
                const int32_t v = g->col[e];
                if (mark[v] != b && hmark[v] != b) {
                    hmark[v] = b;
                    H.push_back(v);
                }
            }
        std::sort(H.begin(), H.end());
        const int64_t nloc = (int64_t)R.size() + (int64_t)H.size();
        int64_t nadj = 0;
        for (int32_t u : R)
            nadj += g->row_ptr[u + 1] - g->row_ptr[u];
        nadj = (nadj + 7) / 8 * 8;       // padded to whole 16-byte vectors
        if (nadj > kMaxLocalAdj || !chunk_fits_lds(nloc, (int64_t)R.size(), nadj))
            return;                      // this graph sweeps by color passes only
        g->max_local = std::max(g->max_local, (int32_t)nloc);
        g->max_r = std::max(g->max_r, (int32_t)R.size());
        g->max_adj = std::max(g->max_adj, (int32_t)nadj);
        g->max_image4 = std::max(g->max_image4, chunk_lds_bytes(nloc, (int64_t)R.size(), nadj, 4));
        g->max_image8 = std::max(g->max_image8, chunk_lds_bytes(nloc, (int64_t)R.size(), nadj, 8));
        int32_t s = 0;
        for (int32_t u : R)
            slot[u] = s++;
        for (int32_t v : H)
            slot[v] = s++;
        // metadata: R color offsets, owned counts per color, and where each
        // color's owned run starts in its slab (the owned sites of a color
        // are consecutive slab positions: slabs follow the locality order)
        std::vector<int32_t> roff(k + 1, 0), owned(k, 0), ostart(k, 0);
        for (int32_t u : R) {
            roff[colpos[u] + 1]++;
            if (chunk[u] == b) {
                if (owned[colpos[u]]++ == 0)
                    ostart[colpos[u]] = u;
            }
        }
        for (int32_t c = 0; c < k; ++c)
            roff[c + 1] += roff[c];
        g->ch_meta.insert(g->ch_meta.end(), roff.begin(), roff.end());
        g->ch_meta.insert(g->ch_meta.end(), owned.begin(), owned.end());
        g->ch_meta.insert(g->ch_meta.end(), ostart.begin(), ostart.end());
        g->loc_site.insert(g->loc_site.end(), R.begin(), R.end());
        g->loc_site.insert(g->loc_site.end(), H.begin(), H.end());
        for (int32_t u : R)
            g->loc_id.push_back((uint32_t)g->orig_of_slab[u]);
        for (int32_t v : H)
            g->loc_id.push_back((uint32_t)g->orig_of_slab[v]);
        uint16_t off = 0;
        for (int32_t u : R) {
            g->loc_row.push_back(off);
            for (int32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e)
                g->loc_adj.push_back((uint16_t)slot[g->col[e]]);
            off = (uint16_t)(off + (g->row_ptr[u + 1] - g->row_ptr[u]));
        }
        g->loc_row.push_back(off);
        // each chunk's rows and neighbours start on a 16-byte boundary, so the
        // kernel stages them with 16-byte loads
        while (g->loc_row.size() % 8)
            g->loc_row.push_back(0);
        while (g->loc_adj.size() % 8)
            g->loc_adj.push_back(0);
        g->ch_loc.push_back((int32_t)g->loc_site.size());
        g->ch_row.push_back((int32_t)g->loc_row.size());
        g->ch_adj.push_back((int32_t)g->loc_adj.size());
    }
    g->chunks_ok = true;
}

int build_lattice(const gmrf_graph_desc *d, HostGraph *g)
{
    const int64_t rows = d->lat_rows, cols = d->lat_cols;
    if (rows < 1 || cols < 1)
        return fail(GMRF_E_INVALID_ARG, "lattice: rows and cols must be >= 1");
    if (d->lat_stencil != 4 && d->lat_stencil != 8)
        return fail(GMRF_E_INVALID_ARG, "lattice: lat_stencil must be 0, 4 or 8");
    if (rows * cols > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(GMRF_E_GRAPH, "lattice: rows * cols must fit in int32");
    if (d->n != rows * cols)
        return fail(GMRF_E_INVALID_ARG, "lattice: n must equal lat_rows * lat_cols");
    const int32_t k = d->lat_stencil == 4 ? 2 : 4;
    if (d->num_colors != 0 && d->num_colors != k)
        return fail(GMRF_E_COLORING, "lattice: the parity coloring of this stencil has " +
                                         std::to_string(k) + " colors");
    if (d->color) {
        for (int64_t r = 0; r < rows; ++r)
            for (int64_t c = 0; c < cols; ++c) {
                const int32_t want =
                    d->lat_stencil == 4 ? (int32_t)((r + c) % 2) : (int32_t)(2 * (r % 2) + c % 2);
                if (d->color[r * cols + c] != want)
                    return fail(GMRF_E_COLORING,
                                "lattice: color of site " + std::to_string(r * cols + c) +
                                    " differs from the parity coloring of the stencil");
            }
    }
    g->n = d->n;
    g->k = k;
    g->rows = (int32_t)rows;
    g->cols = (int32_t)cols;
    g->stencil = d->lat_stencil;
    g->components = 1;   // both stencils connect every lattice
    g->isolated = d->n == 1 ? 1 : 0;
    const int64_t horiz = rows * (cols - 1), vert = (rows - 1) * cols;
    const int64_t diag = d->lat_stencil == 8 ? 2 * (rows - 1) * (cols - 1) : 0;
    g->nnz = 2 * (horiz + vert + diag);
    return GMRF_OK;
}

} // namespace

void set_error(const std::string &msg) { g_error = msg; }
void clear_error() { g_error.clear(); }
int fail(int status, const std::string &msg)
{
    g_error = msg;
    return status;
}
const char *error_cstr() { return g_error.c_str(); }

size_t graph_device_bytes(const HostGraph &g)
{
    if (g.stencil != 0)
        return 0;
    // at least one column entry: a site without neighbours still loads entry 0
    // (clamped gathers), which must hold a valid site index
    size_t bytes = align_up(sizeof(int32_t) * (size_t)(g.n + 1)) +
                   align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(g.nnz, 1)) +
                   align_up(sizeof(int32_t) * (size_t)g.n);
    if (g.chunks_ok)
        bytes += align_up(sizeof(int32_t) * g.ch_loc.size()) +
                 align_up(sizeof(int32_t) * g.ch_row.size()) +
                 align_up(sizeof(int32_t) * g.ch_adj.size()) +
                 align_up(sizeof(int32_t) * g.ch_meta.size()) +
                 align_up(sizeof(int32_t) * g.loc_site.size()) +
                 align_up(sizeof(uint32_t) * g.loc_id.size()) +
                 align_up(sizeof(uint16_t) * g.loc_row.size()) +
                 align_up(sizeof(uint16_t) * std::max<size_t>(g.loc_adj.size(), 1));
    return bytes;
}

int build_host_graph(const gmrf_graph_desc *d, HostGraph *g)
{
    if (!d || !g)
        return fail(GMRF_E_INVALID_ARG, "graph: NULL description");
    if (!(d->rho > -1.0 && d->rho <= 1.0) || !std::isfinite(d->rho))
        return fail(GMRF_E_INVALID_ARG, "graph: rho must lie in (-1, 1]");
    g->rho = d->rho;
    if (d->n < 1)
        return fail(GMRF_E_INVALID_ARG, "graph: n must be >= 1");
    if (d->lat_stencil != 0)
        return build_lattice(d, g);

    const int64_t n = d->n;
    if (n > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(GMRF_E_GRAPH, "graph: n must fit in int32");
    if (!d->row_ptr || !d->color)
        return fail(GMRF_E_INVALID_ARG, "graph: row_ptr and color are required");
    const int64_t *rp = d->row_ptr;
    if (rp[0] != 0)
        return fail(GMRF_E_GRAPH, "graph: row_ptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i])
            return fail(GMRF_E_GRAPH, "graph: row_ptr decreases at row " + std::to_string(i));
    const int64_t nnz = rp[n];
    if (nnz > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(GMRF_E_GRAPH, "graph: more than 2^31 - 1 adjacency entries");
    if (nnz > 0 && !d->col_idx)
        return fail(GMRF_E_INVALID_ARG, "graph: col_idx is required");
    const int32_t *col = d->col_idx;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int64_t j = col[e];
            if (j < 0 || j >= n)
                return fail(GMRF_E_GRAPH, "graph: neighbour id out of range in row " +
                                              std::to_string(i));
            if (j == i)
                return fail(GMRF_E_GRAPH, "graph: self loop at site " + std::to_string(i));
            if (e > rp[i] && col[e - 1] >= j)
                return fail(GMRF_E_GRAPH, "graph: row " + std::to_string(i) +
                                              " is not strictly ascending (duplicate or unsorted)");
        }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int64_t j = col[e];
            if (!std::binary_search(col + rp[j], col + rp[j + 1], (int32_t)i))
                return fail(GMRF_E_GRAPH, "graph: asymmetric edge " + edge_str(i, j));
        }
    const int32_t k = d->num_colors;
    if (k < 1)
        return fail(GMRF_E_COLORING, "graph: num_colors must be >= 1");
    for (int64_t i = 0; i < n; ++i)
        if (d->color[i] < 0 || d->color[i] >= k)
            return fail(GMRF_E_COLORING, "graph: color of site " + std::to_string(i) +
                                             " outside 0 .. num_colors - 1");
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] > i && d->color[i] == d->color[col[e]])
                return fail(GMRF_E_COLORING, "graph: improper coloring, edge " +
                                                 edge_str(i, col[e]) + " inside color " +
                                                 std::to_string(d->color[i]));

    g->n = n;
    g->k = k;
    g->nnz = nnz;
    g->stencil = 0;
    std::vector<int64_t> rpv(rp, rp + n + 1);
    g->components = count_components(n, rpv, col);
    g->isolated = 0;
    for (int64_t i = 0; i < n; ++i)
        g->isolated += rp[i + 1] == rp[i];

    // Color slabs.  Inside a slab the sites follow the locality order of the
    // chunks (chunk_cells), so the threads of one wavefront touch nearby
    // sites and their neighbour gathers share cache lines, and each chunk's
    // sites of one color are one contiguous run of the slab.  The order is
    // internal: random numbers are keyed by original ids and neighbour sums
    // run in original-id order.
    std::vector<int32_t> cell;
    std::vector<int64_t> visit;
    chunk_cells(n, rpv, col, d->color, cell, visit);
    g->slab_offsets.assign(k + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        g->slab_offsets[d->color[i] + 1]++;
    for (int32_t c = 0; c < k; ++c)
        g->slab_offsets[c + 1] += g->slab_offsets[c];
    g->orig_of_slab.resize(n);
    g->slab_of_orig.resize(n);
    std::vector<int32_t> fill(g->slab_offsets.begin(), g->slab_offsets.end() - 1);
    for (int64_t v = 0; v < n; ++v) {
        const int64_t i = visit[v];
        const int32_t pos = fill[d->color[i]]++;
        g->orig_of_slab[pos] = (int32_t)i;
        g->slab_of_orig[i] = pos;
    }
    // permuted CSR: row of slab position p = neighbours of orig_of_slab[p],
    // kept in ascending original id (the summation order of the sweep)
    g->row_ptr.resize(n + 1);
    g->col.resize(nnz);
    g->row_ptr[0] = 0;
    for (int64_t p = 0; p < n; ++p) {
        const int64_t i = g->orig_of_slab[p];
        int64_t w = g->row_ptr[p];
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            g->col[w++] = g->slab_of_orig[col[e]];
        g->row_ptr[p + 1] = (int32_t)w;
    }
    build_chunks(g, cell);
    return GMRF_OK;
}

int greedy_coloring_host(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *color,
                         int32_t *k)
{
    if (n < 0 || (n > 0 && (!row_ptr || !color)) || !k)
        return fail(GMRF_E_INVALID_ARG, "greedy_coloring: bad arguments");
    if (n > 0 && row_ptr[n] > 0 && !col)
        return fail(GMRF_E_INVALID_ARG, "greedy_coloring: col_idx is required");
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (col[e] < 0 || col[e] >= n)
                return fail(GMRF_E_GRAPH, "greedy_coloring: neighbour id out of range");
    // First fit in ascending id order: site i takes the smallest color not
    // held by an already-colored neighbour.  This equals peeling maximal
    // independent sets smallest-id-first: site i lands in color j exactly
    // when colors 0..j-1 each hold a lower neighbour and color j does not.
    std::vector<int64_t> seen(n + 1, -1);
    int32_t kk = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (col[e] < i)
                seen[color[col[e]]] = i;
        int32_t c = 0;
        while (seen[c] == i)
            ++c;
        color[i] = c;
        kk = std::max(kk, c + 1);
    }
    *k = kk;
    return GMRF_OK;
}

} // namespace gmrf
