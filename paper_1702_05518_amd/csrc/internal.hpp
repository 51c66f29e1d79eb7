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
    int64_t nnz = 0;              // directed adjacency entries (2 |E|)
    double rho = 1.0;
    int32_t rows = 0, cols = 0;   // lattice shape
    int32_t stencil = 0;          // 0 = general graph, 4 or 8 = lattice
    // General graphs: sites permuted into color slabs (color, then a
    // breadth-first locality order).  slab_offsets[c] .. slab_offsets[c+1] is
    // color c.
    std::vector<int32_t> slab_offsets;   // k + 1
    std::vector<int32_t> orig_of_slab;   // slab position -> original id
    std::vector<int32_t> slab_of_orig;   // original id -> slab position
    std::vector<int32_t> row_ptr;        // permuted CSR, n + 1
    std::vector<int32_t> col;            // slab positions, each row in ascending ORIGINAL id
};

// Validate a description and build its host form; returns a gmrf_status.
int build_host_graph(const gmrf_graph_desc *d, HostGraph *out);

// First-fit greedy coloring in ascending id order.
int greedy_coloring_host(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *color,
                         int32_t *k);

// Bytes of the device form of a graph.
size_t graph_device_bytes(int64_t n, int64_t nnz, bool lattice);

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

} // namespace gmrf
