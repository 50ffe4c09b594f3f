// Host-side internals shared by the graph, run and server translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "hpmocd.h"
#include "internal.hpp"

struct hpmocd_graph {
    int32_t n = 0;
    int64_t m2 = 0;
    int32_t max_deg = 0;
    int device = 0;
    int32_t *d_rp = nullptr, *d_col = nullptr, *d_small = nullptr, *d_large = nullptr;
    int32_t *d_up_rp = nullptr, *d_up_col = nullptr;
    int32_t n_small = 0, n_large = 0;
    int32_t class_end[hpm::N_DEG_CLASSES] = {};
    int32_t large_max_deg = 0;
    bool owns_device = true;  // false when the arrays live in a server's device arena
};

namespace hpm {

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return HPMOCD_ERR_HIP;    \
    } while (0)

// Waits for stream s when it leaves scope: an entry point that returns early on an error
// leaves no kernel running on memory its caller may free next (on success s is already
// drained, so the wait costs nothing).
struct DrainOnExit {
    hipStream_t s;
    ~DrainOnExit() { (void)hipStreamSynchronize(s); }
};

// A validated graph on the host: sorted adjacency and the mutation kernels' degree classes.
struct HostGraph {
    int32_t n = 0;
    int64_t m2 = 0;
    int32_t max_deg = 0;
    std::vector<int32_t> rp, col, small, large;
    std::vector<int32_t> up_rp, up_col;  // neighbours u > v of each v
    int32_t class_end[N_DEG_CLASSES] = {};
    int32_t large_max_deg = 0;
};
int prepare_graph(int32_t n, const int32_t *row_ptr, const int32_t *col, HostGraph *out);
// device bytes of a graph placed in one block (each array 256-byte aligned)
size_t graph_block_bytes(int32_t n, int64_t m2, int32_t n_small, int32_t n_large);
// Copies the graph to the device: into `block` (graph_block_bytes, stream-ordered copies on
// s; the host arrays must outlive them) or, with block == nullptr, into allocations of its
// own (synchronous copies).
int place_graph(const HostGraph &h, void *block, hipStream_t s, hpmocd_graph *g);

DevGraph dev_graph(const hpmocd_graph *g);
int check_params(const hpmocd_params *p);
int check_device(const hpmocd_graph *g);

}  // namespace hpm
