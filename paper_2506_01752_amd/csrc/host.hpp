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
    int32_t n_small = 0, n_large = 0;
    int32_t class_end[hpm::N_DEG_CLASSES] = {};
    int32_t large_max_deg = 0;
};

namespace hpm {

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return HPMOCD_ERR_HIP;    \
    } while (0)

DevGraph dev_graph(const hpmocd_graph *g);
int check_params(const hpmocd_params *p);
int check_device(const hpmocd_graph *g);

}  // namespace hpm
