// Graph creation and validation (section 2.1: a simple undirected graph), parameter checks
// and status strings of libhpmocd.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "host.hpp"

namespace hpm {

constexpr int64_t MAX_ARCS_EXACT = 94906265;  // largest 2m with (2m)^2 <= 2^53

int prepare_graph(int32_t n, const int32_t *row_ptr, const int32_t *col, HostGraph *out)
{
    if (!out || !row_ptr || n < 1) return HPMOCD_ERR_ARG;
    if (row_ptr[0] != 0) return HPMOCD_ERR_RANGE;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return HPMOCD_ERR_RANGE;
    const int64_t m2 = row_ptr[n];
    if (m2 == 0) return HPMOCD_ERR_EMPTY;
    if (!col) return HPMOCD_ERR_ARG;
    if (m2 > MAX_ARCS_EXACT) return HPMOCD_ERR_TOO_LARGE;
    HostGraph &h = *out;
    try {
        h.rp.assign(row_ptr, row_ptr + (size_t)n + 1);
        h.col.assign(col, col + m2);
    } catch (...) {
        return HPMOCD_ERR_NOMEM;
    }
    std::vector<int32_t> &c = h.col;
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
    // Symmetry: with every row sorted and free of repeats, the arcs are symmetric exactly when
    // the transpose equals them. Each node's in-degree must equal its degree; the transpose's
    // rows are then filled by walking the sources in ascending order, which leaves every row
    // sorted, and compared with the rows as given (a sequential pass instead of one binary
    // search into a random row per arc).
    try {
        std::vector<int32_t> pos(row_ptr, row_ptr + n);
        for (int64_t e = 0; e < m2; ++e) ++pos[c[e]];
        for (int32_t u = 0; u < n; ++u)
            if (pos[u] != row_ptr[u + 1]) return HPMOCD_ERR_CSR_ASYM;  // in-degree != degree
        std::copy(row_ptr, row_ptr + n, pos.begin());
        std::vector<int32_t> t((size_t)m2);
        for (int32_t v = 0; v < n; ++v)
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) t[pos[c[e]]++] = v;
        if (std::memcmp(t.data(), c.data(), sizeof(int32_t) * (size_t)m2) != 0)
            return HPMOCD_ERR_CSR_ASYM;
    } catch (...) {
        return HPMOCD_ERR_NOMEM;
    }
    // upper arcs (u > v) for the fitness scan, and node classes for the mutation kernels
    // (counting sort by degree)
    try {
        h.up_rp.assign((size_t)n + 1, 0);
        h.up_col.reserve((size_t)(m2 / 2));
        for (int32_t v = 0; v < n; ++v) {
            auto b = std::upper_bound(c.begin() + row_ptr[v], c.begin() + row_ptr[v + 1], v);
            h.up_col.insert(h.up_col.end(), b, c.begin() + row_ptr[v + 1]);
            h.up_rp[(size_t)v + 1] = (int32_t)h.up_col.size();
        }
        std::vector<int64_t> cnt((size_t)max_deg + 2, 0);
        for (int32_t v = 0; v < n; ++v) ++cnt[(size_t)(row_ptr[v + 1] - row_ptr[v]) + 1];
        for (size_t d = 1; d < cnt.size(); ++d) cnt[d] += cnt[d - 1];
        std::vector<int32_t> by_deg(n);
        for (int32_t v = 0; v < n; ++v) by_deg[cnt[(size_t)(row_ptr[v + 1] - row_ptr[v])]++] = v;
        for (int32_t v : by_deg) {
            const int32_t d = row_ptr[v + 1] - row_ptr[v];
            if (d >= 1 && d <= SMALL_DEG_MAX) h.small.push_back(v);
        }
        for (auto it = by_deg.rbegin(); it != by_deg.rend(); ++it) {
            const int32_t d = row_ptr[*it + 1] - row_ptr[*it];
            if (d > SMALL_DEG_MAX) h.large.push_back(*it);
        }
    } catch (...) {
        return HPMOCD_ERR_NOMEM;
    }
    h.n = n;
    h.m2 = m2;
    h.max_deg = max_deg;
    // small is in ascending degree order: each class ends where the degrees pass its bound
    for (int k = 0; k < N_DEG_CLASSES; ++k)
        h.class_end[k] = (int32_t)(std::upper_bound(h.small.begin(), h.small.end(), DEG_CLASS_MAX[k],
                                                    [&](int32_t d, int32_t v) {
                                                        return d < row_ptr[v + 1] - row_ptr[v];
                                                    }) -
                                   h.small.begin());
    h.large_max_deg = h.large.empty() ? 0 : row_ptr[h.large[0] + 1] - row_ptr[h.large[0]];
    // fingerprint: FNV-1a (Fowler, Noll, Vo), 64-bit, over the bytes of n, row_ptr and the
    // sorted col
    uint64_t x = 0xcbf29ce484222325ull;
    auto mix = [&x](const void *data, size_t bytes) {
        const unsigned char *b = (const unsigned char *)data;
        for (size_t i = 0; i < bytes; ++i) x = (x ^ b[i]) * 0x100000001b3ull;
    };
    mix(&n, sizeof(n));
    mix(h.rp.data(), sizeof(int32_t) * h.rp.size());
    mix(h.col.data(), sizeof(int32_t) * h.col.size());
    h.hash = x;
    return HPMOCD_OK;
}

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

size_t graph_block_bytes(int32_t n, int64_t m2, int32_t n_small, int32_t n_large)
{
    return 2 * al256(4 * ((size_t)n + 1)) + al256(4 * (size_t)m2) +
           al256(4 * std::max<size_t>(1, (size_t)(m2 / 2))) +
           al256(4 * std::max<size_t>(1, (size_t)n_small)) +
           al256(4 * std::max<size_t>(1, (size_t)n_large));
}

const void *Pinned::stage(const void *src, size_t bytes)
{
    void *p = take(bytes);
    if (!p) return src;
    std::memcpy(p, src, bytes);
    return p;
}

static void graph_fields(const HostGraph &h, hpmocd_graph *g)
{
    g->n = h.n;
    g->m2 = h.m2;
    g->max_deg = h.max_deg;
    g->n_small = (int32_t)h.small.size();
    g->n_large = (int32_t)h.large.size();
    for (int k = 0; k < N_DEG_CLASSES; ++k) g->class_end[k] = h.class_end[k];
    g->large_max_deg = h.large_max_deg;
    g->hash = h.hash;
}

void place_graph_deferred(const HostGraph &h, void *block, hpmocd_graph *g, Pinned *stage,
                          std::vector<PendingCopy> &copies)
{
    graph_fields(h, g);
    (void)hipGetDevice(&g->device);
    const size_t b_rp = 4 * ((size_t)h.n + 1), b_col = 4 * (size_t)h.m2;
    const size_t b_small = 4 * std::max<size_t>(1, h.small.size());
    const size_t b_large = 4 * std::max<size_t>(1, h.large.size());
    char *p = (char *)block;
    g->owns_device = false;
    g->d_rp = (int32_t *)p;
    p += al256(b_rp);
    g->d_col = (int32_t *)p;
    p += al256(b_col);
    g->d_small = (int32_t *)p;
    p += al256(b_small);
    g->d_large = (int32_t *)p;
    p += al256(b_large);
    g->d_up_rp = (int32_t *)p;
    p += al256(b_rp);
    g->d_up_col = (int32_t *)p;
    auto add = [&](void *dst, const void *src, size_t bytes) {
        if (!bytes) return;
        if (stage) src = stage->stage(src, bytes);
        copies.push_back(PendingCopy{dst, src, bytes});
    };
    add(g->d_rp, h.rp.data(), b_rp);
    add(g->d_col, h.col.data(), b_col);
    add(g->d_up_rp, h.up_rp.data(), b_rp);
    add(g->d_up_col, h.up_col.data(), 4 * h.up_col.size());
    add(g->d_small, h.small.data(), 4 * h.small.size());
    add(g->d_large, h.large.data(), 4 * h.large.size());
}

int place_graph(const HostGraph &h, void *block, hipStream_t s, hpmocd_graph *g, Pinned *stage)
{
    graph_fields(h, g);
    if (hipGetDevice(&g->device) != hipSuccess) return HPMOCD_ERR_HIP;
    const size_t b_rp = 4 * ((size_t)h.n + 1), b_col = 4 * (size_t)h.m2;
    const size_t b_up = 4 * std::max<size_t>(1, h.up_col.size());
    const size_t b_small = 4 * std::max<size_t>(1, h.small.size());
    const size_t b_large = 4 * std::max<size_t>(1, h.large.size());
    if (block) {
        std::vector<PendingCopy> copies;
        place_graph_deferred(h, block, g, stage, copies);
        for (const PendingCopy &c : copies)
            if (hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyHostToDevice, s) != hipSuccess)
                return HPMOCD_ERR_HIP;
        return HPMOCD_OK;
    }
    g->owns_device = true;
    bool ok = hipMalloc(&g->d_rp, b_rp) == hipSuccess;
    ok = ok && hipMalloc(&g->d_col, b_col) == hipSuccess;
    ok = ok && hipMalloc(&g->d_small, b_small) == hipSuccess;
    ok = ok && hipMalloc(&g->d_large, b_large) == hipSuccess;
    ok = ok && hipMalloc(&g->d_up_rp, b_rp) == hipSuccess;
    ok = ok && hipMalloc(&g->d_up_col, b_up) == hipSuccess;
    // copies on a private non-blocking stream: a null-stream copy would synchronise with
    // (and invalidate) a hipGraph capture running in another thread
    hipStream_t st = nullptr;
    ok = ok && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    const hipMemcpyKind h2d = hipMemcpyHostToDevice;
    ok = ok && hipMemcpyAsync(g->d_rp, h.rp.data(), b_rp, h2d, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(g->d_up_rp, h.up_rp.data(), b_rp, h2d, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(g->d_up_col, h.up_col.data(), 4 * h.up_col.size(), h2d, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(g->d_col, h.col.data(), b_col, h2d, st) == hipSuccess;
    if (ok && !h.small.empty())
        ok = hipMemcpyAsync(g->d_small, h.small.data(), 4 * h.small.size(), h2d, st) == hipSuccess;
    if (ok && !h.large.empty())
        ok = hipMemcpyAsync(g->d_large, h.large.data(), 4 * h.large.size(), h2d, st) == hipSuccess;
    if (st) {
        ok = hipStreamSynchronize(st) == hipSuccess && ok;
        (void)hipStreamDestroy(st);
    }
    return ok ? HPMOCD_OK : HPMOCD_ERR_HIP;
}

DevGraph dev_graph(const hpmocd_graph *g)
{
    DevGraph d;
    d.n = g->n;
    d.m2 = g->m2;
    d.row_ptr = g->d_rp;
    d.col = g->d_col;
    d.up_rp = g->d_up_rp;
    d.up_col = g->d_up_col;
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
    case HPMOCD_ERR_RANGE: return "row_ptr, column index or label out of range";
    case HPMOCD_ERR_EMPTY: return "graph has no edge";
    case HPMOCD_ERR_TOO_LARGE: return "(2m)^2 exceeds 2^53";
    case HPMOCD_ERR_WORKSPACE: return "workspace too small";
    case HPMOCD_ERR_HIP: return "HIP runtime error";
    case HPMOCD_ERR_BUDGET: return "device-memory budget exceeded";
    case HPMOCD_ERR_NOMEM: return "host allocation failed";
    case HPMOCD_ERR_CANCELLED: return "request cancelled";
    case HPMOCD_ERR_TIMEOUT: return "wait timed out";
    case HPMOCD_ERR_SCRATCH: return "problem exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
    }
}

int hpmocd_graph_create(int32_t n, const int32_t *row_ptr, const int32_t *col,
                        hpmocd_graph **out)
{
    return c_guard([&]() -> int {
        if (!out) return HPMOCD_ERR_ARG;
        HostGraph h;
        int rc = prepare_graph(n, row_ptr, col, &h);
        if (rc) return rc;
        hpmocd_graph *g = new (std::nothrow) hpmocd_graph;
        if (!g) return HPMOCD_ERR_NOMEM;
        if ((rc = place_graph(h, nullptr, nullptr, g))) {
            hpmocd_graph_destroy(g);
            return rc;
        }
        *out = g;
        return HPMOCD_OK;
    });
}

void hpmocd_graph_destroy(hpmocd_graph *g)
{
    if (!g) return;
    if (!g->owns_device) {
        delete g;
        return;
    }
    if (g->d_rp) (void)hipFree(g->d_rp);
    if (g->d_col) (void)hipFree(g->d_col);
    if (g->d_small) (void)hipFree(g->d_small);
    if (g->d_large) (void)hipFree(g->d_large);
    if (g->d_up_rp) (void)hipFree(g->d_up_rp);
    if (g->d_up_col) (void)hipFree(g->d_up_col);
    delete g;
}

int hpmocd_graph_hash(const hpmocd_graph *g, uint64_t *hash)
{
    if (!g || !hash) return HPMOCD_ERR_ARG;
    *hash = g->hash;
    return HPMOCD_OK;
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
