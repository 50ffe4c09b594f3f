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
    uint64_t hash = 0;        // FNV-1a over n and the sorted CSR
};

namespace hpm {

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return HPMOCD_ERR_HIP;    \
    } while (0)

// Runs an entry point's body: no exception leaves the C ABI. The library throws only when
// host resources run out (an allocation, a thread), which is reported as HPMOCD_ERR_NOMEM;
// stream-draining guards inside the body run while the exception unwinds.
template <class F>
int c_guard(F &&f) noexcept
{
    try {
        return f();
    } catch (...) {
        return HPMOCD_ERR_NOMEM;
    }
}

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
    uint64_t hash = 0;
};
int prepare_graph(int32_t n, const int32_t *row_ptr, const int32_t *col, HostGraph *out);
// A region of page-locked host memory used as staging for stream-ordered copies: a copy
// from pageable memory is staged by the runtime through its own buffers while the stream
// waits, one chunk at a time; from page-locked memory it is a plain DMA. take() hands out
// 256-byte-aligned pieces until the region is full (nullptr: copy from pageable memory
// instead). The owner resets `used` once the copies that read the pieces have completed.
struct Pinned {
    char *base = nullptr;
    size_t size = 0, used = 0;
    void *take(size_t bytes)
    {
        const size_t b = (bytes + 255) / 256 * 256;
        if (!base || used + b > size) return nullptr;
        void *p = base + used;
        used += b;
        return p;
    }
    // host source for a copy of `bytes` from src: a staged copy in this region when it fits
    const void *stage(const void *src, size_t bytes);
};

// device bytes of a graph placed in one block (each array 256-byte aligned)
size_t graph_block_bytes(int32_t n, int64_t m2, int32_t n_small, int32_t n_large);
// Copies the graph to the device: into `block` (graph_block_bytes, stream-ordered copies on
// s; the host arrays must outlive them) or, with block == nullptr, into allocations of its
// own (synchronous copies).
int place_graph(const HostGraph &h, void *block, hipStream_t s, hpmocd_graph *g,
                Pinned *stage = nullptr);
// A host-to-device copy not yet issued.
struct PendingCopy {
    void *dst;
    const void *src;
    size_t bytes;
};
// place_graph into `block` without issuing the copies: the arrays are staged (when they fit
// the staging region) and the copies appended to `copies`, so that a caller placing several
// graphs issues every copy only after all the host-side staging is done and the stream does
// not wait on it between copies.
void place_graph_deferred(const HostGraph &h, void *block, hpmocd_graph *g, Pinned *stage,
                          std::vector<PendingCopy> &copies);

DevGraph dev_graph(const hpmocd_graph *g);
int check_params(const hpmocd_params *p);
int check_device(const hpmocd_graph *g);

}  // namespace hpm
