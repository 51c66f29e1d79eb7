// graph_host.cpp -- host half of libgmrf: graph validation, coloring checks,
// connected components, the color-slab permutation and the greedy coloring.
// No HIP calls here, so every check runs (and is tested) without a GPU.
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

// Breadth-first visit order of all sites: each component from its smallest
// unvisited id, neighbours queued in ascending id order.
std::vector<int64_t> breadth_first_order(int64_t n, const std::vector<int64_t> &rp,
                                         const int32_t *col)
{
    std::vector<int64_t> order;
    order.reserve(n);
    std::vector<unsigned char> seen(n, 0);
    for (int64_t s = 0; s < n; ++s) {
        if (seen[s])
            continue;
        seen[s] = 1;
        size_t head = order.size();
        order.push_back(s);
        while (head < order.size()) {
            const int64_t v = order[head++];
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
                const int64_t u = col[e];
                if (!seen[u]) {
                    seen[u] = 1;
                    order.push_back(u);
                }
            }
        }
    }
    return order;
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

size_t graph_device_bytes(int64_t n, int64_t nnz, bool lattice)
{
    if (lattice)
        return 0;
    // at least one column entry: a site without neighbours still loads entry 0
    // (clamped gathers), which must hold a valid site index
    return align_up(sizeof(int32_t) * (size_t)(n + 1)) +
           align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)) +
           align_up(sizeof(int32_t) * (size_t)n);
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

    // Color slabs.  Inside a slab the sites follow a breadth-first order of
    // the graph (components by smallest id, neighbours by ascending id), so
    // the threads of one wavefront touch nearby sites and their neighbour
    // gathers share cache lines.  The order is internal: random numbers are
    // keyed by original ids and neighbour sums run in original-id order.
    const std::vector<int64_t> visit = breadth_first_order(n, rpv, col);
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
