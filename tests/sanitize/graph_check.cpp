// graph_check.cpp -- host-only driver of the graph builder (graph_host.cpp),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py.  Reads graphs from a binary file, builds the host
// form of each and checks the invariants of the color slabs and of the
// chunk tables of the chunked sweep (Sec. 2.3: every chunk's closure R under
// lower-color neighbours, owned sites, local adjacency).  Exit status 0 when
// every check holds; the first failed check is printed.
//
// File layout, repeated per graph: int64 n, int64 nnz, int32 k, double rho,
// int64 row_ptr[n + 1], int32 col[nnz], int32 color[n].
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <vector>

#include "internal.hpp"

using namespace gmrf;

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "graph %d: check failed: %s (line %d)\n", gi, #cond, \
                         __LINE__);                                                  \
            return 1;                                                                \
        }                                                                            \
    } while (0)

static int chunked = 0;

static int check_graph(int gi, int64_t n, int32_t k, double rho, const std::vector<int64_t> &rp,
                       const std::vector<int32_t> &cl, const std::vector<int32_t> &color)
{
    gmrf_graph_desc d{};
    d.n = n;
    d.row_ptr = rp.data();
    d.col_idx = cl.data();
    d.color = color.data();
    d.num_colors = k;
    d.rho = rho;
    HostGraph g;
    CHECK(build_host_graph(&d, &g) == GMRF_OK);
    // slabs: a permutation, grouped by color
    CHECK((int64_t)g.orig_of_slab.size() == n && (int64_t)g.slab_of_orig.size() == n);
    for (int64_t p = 0; p < n; ++p)
        CHECK(g.slab_of_orig[g.orig_of_slab[p]] == p);
    for (int32_t c = 0; c < k; ++c)
        for (int32_t p = g.slab_offsets[c]; p < g.slab_offsets[c + 1]; ++p)
            CHECK(color[g.orig_of_slab[p]] == c);
    int64_t isolated = 0;
    for (int64_t i = 0; i < n; ++i)
        isolated += rp[i + 1] == rp[i];
    CHECK(g.isolated == isolated);
    if (!g.chunks_ok)
        return 0;
    ++chunked;
    std::vector<int32_t> colpos(n);
    for (int32_t c = 0; c < k; ++c)
        for (int32_t p = g.slab_offsets[c]; p < g.slab_offsets[c + 1]; ++p)
            colpos[p] = c;
    std::vector<int> owner(n, -1);
    int64_t img4 = 0, img8 = 0;
    for (int32_t b = 0; b < g.nchunks; ++b) {
        const int32_t l0 = g.ch_loc[b], nloc = g.ch_loc[b + 1] - l0;
        const int32_t *m = g.ch_meta.data() + (size_t)b * (3 * k + 1);
        const int32_t nr = m[k];
        const int32_t r0 = g.ch_row[b], a0 = g.ch_adj[b], nadj = g.ch_adj[b + 1] - a0;
        CHECK(nloc >= nr && nr >= 1 && nloc <= g.max_local && nr <= g.max_r);
        CHECK(r0 % 8 == 0 && a0 % 8 == 0 && nadj % 8 == 0 && nadj <= g.max_adj);
        CHECK(chunk_fits_lds(nloc, nr, nadj));
        CHECK(chunk_lds_bytes(nloc, nr, nadj, 4) <= g.max_image4);
        CHECK(chunk_lds_bytes(nloc, nr, nadj, 8) <= g.max_image8);
        img4 = std::max(img4, chunk_lds_bytes(nloc, nr, nadj, 4));
        img8 = std::max(img8, chunk_lds_bytes(nloc, nr, nadj, 8));
        CHECK(m[0] == 0);
        std::vector<int32_t> slot_of(n, -1);
        for (int32_t s = 0; s < nloc; ++s) {
            const int32_t p = g.loc_site[l0 + s];
            CHECK(p >= 0 && p < n && slot_of[p] < 0);
            CHECK((int64_t)g.loc_id[l0 + s] == g.orig_of_slab[p]);
            slot_of[p] = s;
        }
        for (int32_t c = 0; c < k; ++c) {
            CHECK(m[c] <= m[c + 1]);
            const int32_t own = m[k + 1 + c], ost = m[2 * k + 1 + c];
            CHECK(own >= 0 && own <= m[c + 1] - m[c]);
            for (int32_t o = 0; o < own; ++o) {
                // owned run: the first own R sites of the color, consecutive slab positions
                CHECK(g.loc_site[l0 + m[c] + o] == ost + o);
                CHECK(owner[ost + o] < 0);
                owner[ost + o] = b;
            }
            for (int32_t s = m[c]; s < m[c + 1]; ++s)
                CHECK(colpos[g.loc_site[l0 + s]] == c);
        }
        for (int32_t s = 0; s < nr; ++s) {
            const int32_t u = g.loc_site[l0 + s];
            const int32_t e0 = g.loc_row[r0 + s], e1 = g.loc_row[r0 + s + 1];
            CHECK(e0 <= e1 && e1 - e0 == g.row_ptr[u + 1] - g.row_ptr[u]);
            for (int32_t e = 0; e < e1 - e0; ++e) {
                const int32_t v = g.col[g.row_ptr[u] + e];
                const int32_t l = g.loc_adj[a0 + e0 + e];
                CHECK(l < nloc && g.loc_site[l0 + l] == v);   // same neighbour, same order
                if (colpos[v] < colpos[u])
                    CHECK(l < nr);                            // closure under lower colors
            }
        }
        CHECK(g.loc_row[r0 + nr] <= nadj);
    }
    for (int64_t p = 0; p < n; ++p)
        CHECK(owner[p] >= 0);                                 // every site owned once
    CHECK(img4 == g.max_image4 && img8 == g.max_image8);   // the launch reserves the largest
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 2) {
        std::fprintf(stderr, "usage: graph_check FILE\n");
        return 2;
    }
    std::ifstream f(argv[1], std::ios::binary);
    int gi = 0, rc = 0;
    for (;; ++gi) {
        int64_t n = 0, nnz = 0;
        int32_t k = 0;
        double rho = 1.0;
        if (!f.read((char *)&n, 8))
            break;
        f.read((char *)&nnz, 8);
        f.read((char *)&k, 4);
        f.read((char *)&rho, 8);
        std::vector<int64_t> rp(n + 1);
        std::vector<int32_t> cl(nnz), color(n);
        f.read((char *)rp.data(), 8 * (n + 1));
        f.read((char *)cl.data(), 4 * nnz);
        f.read((char *)color.data(), 4 * n);
        if (!f)
            return 2;
        rc |= check_graph(gi, n, k, rho, rp, cl, color);
    }
    std::printf("checked %d graphs, %d with chunk tables\n", gi, chunked);
    return rc;
}
