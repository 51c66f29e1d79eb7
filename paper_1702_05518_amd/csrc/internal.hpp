// internal.hpp -- library-private types shared by the host graph builder and
// the HIP side of libgmrf.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "gmrf.h"

namespace gmrf {

// Thread-local error message behind gmrf_last_error().
void set_error(const std::string &msg);
void clear_error();
int fail(int status, const std::string &msg);

// Host form of a validated graph (built by graph_host.cpp, no HIP calls).
struct HostGraph {
    int64_t n = 0;
    int32_t k = 0;
    int64_t components = 0;
    int64_t isolated = 0;         // sites without neighbours
    int64_t nnz = 0;              // directed adjacency entries (2 |E|)
    double rho = 1.0;
    int32_t rows = 0, cols = 0;   // lattice shape
    int32_t stencil = 0;          // 0 = general graph, 4 or 8 = lattice
    // General graphs: sites permuted into color slabs (color, then the
    // chunk order).  slab_offsets[c] .. slab_offsets[c+1] is
    // color c.
    std::vector<int32_t> slab_offsets;   // k + 1
    std::vector<int32_t> orig_of_slab;   // slab position -> original id
    std::vector<int32_t> slab_of_orig;   // original id -> slab position
    std::vector<int32_t> row_ptr;        // permuted CSR, n + 1
    std::vector<int32_t> col;            // slab positions, each row in ascending ORIGINAL id
    // Chunks for the one-launch sweep of a general graph (built by
    // build_chunks): chunk b owns about kChunkSites sites of compact extent
    // and stages, in LDS slot order, R_b (its owned sites and every site
    // whose new value they need this sweep, by color, owned first within a
    // color) and then H_b (the other neighbours of R_b, read-only).
    int32_t nchunks = 0;
    int32_t max_local = 0;               // most staged sites of any chunk
    int32_t max_r = 0;                   // most recomputed (R) sites of any chunk
    int32_t max_adj = 0;                 // most local neighbour entries of any chunk
    int64_t max_image4 = 0, max_image8 = 0;   // largest chunk LDS image, FP32 / FP64 values
    bool chunks_ok = false;              // every chunk within the LDS and index limits
    std::vector<int32_t> ch_loc;         // nchunks + 1: first staged site of each chunk
    std::vector<int32_t> ch_row;         // nchunks + 1: first local row offset of each chunk
    std::vector<int32_t> ch_adj;         // nchunks + 1: first local neighbour of each chunk
    std::vector<int32_t> ch_meta;        // per chunk, 3k + 1: R color offsets (k + 1), owned
                                         // counts (k), first slab position of the owned run of
                                         // each color (k)
    std::vector<int32_t> loc_site;       // slab position of every staged site
    std::vector<uint32_t> loc_id;        // original id of every staged site
    std::vector<uint16_t> loc_row;       // per chunk, |R_b| + 1 offsets into its local neighbours
    std::vector<uint16_t> loc_adj;       // local slots of the neighbours of each R_b site,
                                         // ascending original id
};

// Owned sites per chunk, and the limits of a chunk: its LDS image (staged
// values, y and normal variates of the R sites, local rows and neighbours)
// with FP64 and with FP32 values, and 16-bit local offsets.  A block lays out
// its own chunk's image; a launch reserves the largest image of the graph
// (at most kFusedLaunchLds).  The FP64 cap keeps four blocks of the chunked
// sweep kernel (with its static LDS) within a CU's 160 KB; the FP32 cap
// (six blocks fit from 25,000 B) splits the largest few percent of the
// chunks further, whose closures set the tail of a sweep (measured on
// Delaunay graphs: 1M sites 36.9 -> 33.2 us, 15k sites 15.8 -> 14.8 us).
constexpr int32_t kChunkSites = 512;
constexpr int64_t kFusedLdsBytes = 38000;
constexpr int64_t kFusedLdsBytes32 = 21800;
constexpr int64_t kFusedLaunchLds = 65536;
constexpr int64_t kMaxLocalAdj = 65535;
constexpr int32_t kFusedMaxColors = 32;  // colorings with more colors sweep by color passes

// Bytes of a chunk's LDS image with real_bytes-byte values (the layout of
// the chunked sweep kernel: values of the staged sites, then y and the
// sweep's normal variate of each R site, then the R sites' local row offsets
// and neighbours, each part 16-byte aligned).
inline int64_t chunk_lds_bytes(int64_t nloc, int64_t nr, int64_t nadj, int64_t real_bytes)
{
    auto al = [](int64_t b) { return (b + 15) / 16 * 16; };
    return al(real_bytes * nloc) + 2 * al(real_bytes * nr) + al(2 * (nr + 1)) + al(2 * nadj);
}

// Does a chunk's image fit both caps?
inline bool chunk_fits_lds(int64_t nloc, int64_t nr, int64_t nadj)
{
    return chunk_lds_bytes(nloc, nr, nadj, 8) <= kFusedLdsBytes &&
           chunk_lds_bytes(nloc, nr, nadj, 4) <= kFusedLdsBytes32;
}

// Validate a description and build its host form; returns a gmrf_status.
int build_host_graph(const gmrf_graph_desc *d, HostGraph *out);

// First-fit greedy coloring in ascending id order.
int greedy_coloring_host(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *color,
                         int32_t *k);

// Bytes of the device form of a graph (a built host form).
size_t graph_device_bytes(const HostGraph &g);

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

} // namespace gmrf
