// Graph creation and validation (section 2.1: a simple undirected graph), parameter checks
// and status strings of libhpmocd.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "host.hpp"

namespace hpm {

constexpr int64_t MAX_ARCS_EXACT = 94906265;  // largest 2m with (2m)^2 <= 2^53

DevGraph dev_graph(const hpmocd_graph *g)
{
    DevGraph d;
    d.n = g->n;
    d.m2 = g->m2;
    d.row_ptr = g->d_rp;
    d.col = g->d_col;
    d.small_nodes = g->d_small;
    d.n_small = g->n_small;
    d.large_nodes = g->d_large;
    d.n_large = g->n_large;
    for (int k = 0; k < N_DEG_CLASSES; ++k) d.class_end[k] = g->class_end[k];
    d.large_max_deg = g->large_max_deg;
    return d;
}

int check_params(const hpmocd_params *p)
{
    if (!p) return HPMOCD_ERR_ARG;
    if (p->pop_size < 1 || p->pop_size > HPMOCD_MAX_POP) return HPMOCD_ERR_ARG;
    if (p->generations < 0) return HPMOCD_ERR_ARG;
    if (p->parents_per_child < 1 || p->parents_per_child > HPMOCD_MAX_PARENTS) return HPMOCD_ERR_ARG;
    if (!(p->crossover_p >= 0.0 && p->crossover_p <= 1.0)) return HPMOCD_ERR_ARG;
    if (!(p->mutation_p >= 0.0 && p->mutation_p <= 1.0)) return HPMOCD_ERR_ARG;
    return HPMOCD_OK;
}

int check_device(const hpmocd_graph *g)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return HPMOCD_ERR_HIP;
    return dev == g->device ? HPMOCD_OK : HPMOCD_ERR_ARG;
}

}  // namespace hpm

using namespace hpm;

extern "C" {

const char *hpmocd_strerror(int status)
{
    switch (status) {
    case HPMOCD_OK: return "ok";
    case HPMOCD_ERR_ARG: return "invalid argument";
    case HPMOCD_ERR_CSR_ASYM: return "CSR is not symmetric";
    case HPMOCD_ERR_SELF_LOOP: return "graph has a self-loop";
    case HPMOCD_ERR_DUP_EDGE: return "graph has a repeated edge";
    case HPMOCD_ERR_RANGE: return "row_ptr or column index out of range";
    case HPMOCD_ERR_EMPTY: return "graph has no edge";
    case HPMOCD_ERR_TOO_LARGE: return "(2m)^2 exceeds 2^53";
    case HPMOCD_ERR_WORKSPACE: return "workspace too small";
    case HPMOCD_ERR_HIP: return "HIP runtime error";
    case HPMOCD_ERR_BUDGET: return "device-memory budget exceeded";
    case HPMOCD_ERR_NOMEM: return "host allocation failed";
    default: return "unknown status";
    }
}

int hpmocd_graph_create(int32_t n, const int32_t *row_ptr, const int32_t *col,
                        hpmocd_graph **out)
{
    if (!out || !row_ptr || n < 1) return HPMOCD_ERR_ARG;
    if (row_ptr[0] != 0) return HPMOCD_ERR_RANGE;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return HPMOCD_ERR_RANGE;
    const int64_t m2 = row_ptr[n];
    if (m2 == 0) return HPMOCD_ERR_EMPTY;
    if (!col) return HPMOCD_ERR_ARG;
    if (m2 > MAX_ARCS_EXACT) return HPMOCD_ERR_TOO_LARGE;
    std::vector<int32_t> c;
    try {
        c.assign(col, col + m2);
    } catch (...) {
        return HPMOCD_ERR_NOMEM;
    }
    int32_t max_deg = 0;
    for (int32_t v = 0; v < n; ++v) {
        const int32_t rs = row_ptr[v], re = row_ptr[v + 1];
        max_deg = std::max(max_deg, re - rs);
        for (int32_t e = rs; e < re; ++e) {
            if (c[e] < 0 || c[e] >= n) return HPMOCD_ERR_RANGE;
            if (c[e] == v) return HPMOCD_ERR_SELF_LOOP;
        }
        std::sort(c.begin() + rs, c.begin() + re);
        for (int32_t e = rs + 1; e < re; ++e)
            if (c[e] == c[e - 1]) return HPMOCD_ERR_DUP_EDGE;
    }
    for (int32_t v = 0; v < n; ++v)
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t u = c[e];
            if (!std::binary_search(c.begin() + row_ptr[u], c.begin() + row_ptr[u + 1], v))
                return HPMOCD_ERR_CSR_ASYM;
        }
    // node classes for the mutation kernels (counting sort by degree)
    std::vector<int32_t> small, large;
    {
        std::vector<int64_t> cnt((size_t)max_deg + 2, 0);
        for (int32_t v = 0; v < n; ++v) ++cnt[(size_t)(row_ptr[v + 1] - row_ptr[v]) + 1];
        for (size_t d = 1; d < cnt.size(); ++d) cnt[d] += cnt[d - 1];
        std::vector<int32_t> by_deg(n);
        for (int32_t v = 0; v < n; ++v) by_deg[cnt[(size_t)(row_ptr[v + 1] - row_ptr[v])]++] = v;
        for (int32_t v : by_deg) {
            const int32_t d = row_ptr[v + 1] - row_ptr[v];
            if (d >= 1 && d <= SMALL_DEG_MAX) small.push_back(v);
        }
        for (auto it = by_deg.rbegin(); it != by_deg.rend(); ++it) {
            const int32_t d = row_ptr[*it + 1] - row_ptr[*it];
            if (d > SMALL_DEG_MAX) large.push_back(*it);
        }
    }
    hpmocd_graph *g = new (std::nothrow) hpmocd_graph;
    if (!g) return HPMOCD_ERR_NOMEM;
    g->n = n;
    g->m2 = m2;
    g->max_deg = max_deg;
    g->n_small = (int32_t)small.size();
    g->n_large = (int32_t)large.size();
    for (int k = 0; k < N_DEG_CLASSES; ++k) {
        int32_t e = 0;
        for (int32_t v : small)
            if (row_ptr[v + 1] - row_ptr[v] <= DEG_CLASS_MAX[k]) ++e;
        g->class_end[k] = e;
    }
    g->large_max_deg = large.empty() ? 0 : row_ptr[large[0] + 1] - row_ptr[large[0]];
    bool ok = hipGetDevice(&g->device) == hipSuccess;
    ok = ok && hipMalloc(&g->d_rp, sizeof(int32_t) * ((size_t)n + 1)) == hipSuccess;
    ok = ok && hipMalloc(&g->d_col, sizeof(int32_t) * (size_t)m2) == hipSuccess;
    ok = ok && hipMalloc(&g->d_small, sizeof(int32_t) * std::max<size_t>(1, small.size())) == hipSuccess;
    ok = ok && hipMalloc(&g->d_large, sizeof(int32_t) * std::max<size_t>(1, large.size())) == hipSuccess;
    ok = ok && hipMemcpy(g->d_rp, row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(g->d_col, c.data(), sizeof(int32_t) * (size_t)m2, hipMemcpyHostToDevice) == hipSuccess;
    if (ok && !small.empty())
        ok = hipMemcpy(g->d_small, small.data(), sizeof(int32_t) * small.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (ok && !large.empty())
        ok = hipMemcpy(g->d_large, large.data(), sizeof(int32_t) * large.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        hpmocd_graph_destroy(g);
        return HPMOCD_ERR_HIP;
    }
    *out = g;
    return HPMOCD_OK;
}

void hpmocd_graph_destroy(hpmocd_graph *g)
{
    if (!g) return;
    if (g->d_rp) (void)hipFree(g->d_rp);
    if (g->d_col) (void)hipFree(g->d_col);
    if (g->d_small) (void)hipFree(g->d_small);
    if (g->d_large) (void)hipFree(g->d_large);
    delete g;
}

int hpmocd_graph_info(const hpmocd_graph *g, int32_t *n, int64_t *arcs, int32_t *max_deg)
{
    if (!g) return HPMOCD_ERR_ARG;
    if (n) *n = g->n;
    if (arcs) *arcs = g->m2;
    if (max_deg) *max_deg = g->max_deg;
    return HPMOCD_OK;
}

}  // extern "C"
