// Host side of libhpmocd: graph validation and upload, workspace carving, the generation
// loop (optionally replayed from a hipGraph), tracing, front extraction and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "hpmocd.h"
#include "internal.hpp"
#include "philox.hpp"

using namespace hpm;

struct hpmocd_graph {
    int32_t n = 0;
    int64_t m2 = 0;
    int32_t max_deg = 0;
    int device = 0;
    int32_t *d_rp = nullptr, *d_col = nullptr, *d_small = nullptr, *d_large = nullptr;
    int32_t n_small = 0, n_large = 0;
    int32_t class_end[N_DEG_CLASSES] = {};
    int32_t large_max_deg = 0;
};

namespace {

constexpr size_t ALIGN = 256;
constexpr int64_t MAX_ARCS_EXACT = 94906265;  // largest 2m with (2m)^2 <= 2^53

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
int32_t round16(int32_t x) { return (x + 15) / 16 * 16; }

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return HPMOCD_ERR_HIP;    \
    } while (0)

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

// Sub-allocations of the caller's workspace.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <class T>
    T *take(size_t count)
    {
        T *p = base ? (T *)(base + off) : nullptr;
        off += align_up(sizeof(T) * count);
        return p;
    }
};

struct RunLayout {
    int32_t ld = 0;
    size_t plane = 0;  // bytes of one node-major [n][ld] int32 plane
    int32_t *pool[2] = {nullptr, nullptr};
    int32_t *q[2] = {nullptr, nullptr};
    int32_t *C = nullptr;
    int32_t *D = nullptr;       // plain histogram (only when the binned one does not apply)
    HistPlan hp;
    uint32_t *run = nullptr, *off = nullptr;  // binned histogram work areas
    DevState st{};
    size_t bytes = 0;
};

RunLayout carve_run(void *ws, int32_t n, int32_t pop, int32_t es, int32_t max_deg)
{
    RunLayout L;
    L.hp = hist_plan(n, pop, max_deg);
    L.ld = round16(pop);
    L.plane = (size_t)n * (size_t)L.ld * sizeof(int32_t);
    Carver cv(ws);
    const size_t cells = (size_t)n * (size_t)L.ld;
    L.pool[0] = cv.take<int32_t>(cells);
    L.pool[1] = cv.take<int32_t>(cells);
    L.q[0] = cv.take<int32_t>(cells);
    L.q[1] = cv.take<int32_t>(cells);
    L.C = cv.take<int32_t>(cells);
    if (L.hp.enabled) {
        L.run = cv.take<uint32_t>(L.hp.entries);
        L.off = cv.take<uint32_t>(L.hp.offsets);
    } else {
        L.D = cv.take<int32_t>(cells);
    }
    DevState &s = L.st;
    s.gen = cv.take<int32_t>(1);
    s.ps_id = cv.take<int32_t>(pop);
    s.ps_A = cv.take<int64_t>(pop);
    s.ps_S = cv.take<int64_t>(pop);
    s.ps_f1 = cv.take<double>(pop);
    s.ps_f2 = cv.take<double>(pop);
    s.pos_id = cv.take<int32_t>(pop);
    s.pos_A = cv.take<int64_t>(pop);
    s.pos_S = cv.take<int64_t>(pop);
    s.tr_rank = cv.take<int32_t>(pop);
    s.tr_crowd = cv.take<double>(pop);
    s.par_id = cv.take<int32_t>((size_t)pop * es);
    s.gate = cv.take<int32_t>(pop);
    s.Aq = cv.take<unsigned long long>(pop);
    s.Sq = cv.take<unsigned long long>(pop);
    s.fr_count = cv.take<int32_t>(1);
    s.fr_id = cv.take<int32_t>(pop);
    s.fr_A = cv.take<int64_t>(pop);
    s.fr_S = cv.take<int64_t>(pop);
    s.fr_f1 = cv.take<double>(pop);
    s.fr_f2 = cv.take<double>(pop);
    L.bytes = cv.off;
    return L;
}

GaConst ga_const(const hpmocd_params *p, int32_t ld)
{
    GaConst c;
    c.pop = p->pop_size;
    c.ld = ld;
    c.es = p->parents_per_child;
    c.seed = p->seed;
    c.thr_c = bernoulli_threshold(p->crossover_p);
    c.thr_m = bernoulli_threshold(p->mutation_p);
    // nodes per wave group in the small-degree mutation kernel: enough candidate (node,
    // offspring) pairs to fill about 1.5 waves of mutations, within the LDS list capacity
    int g = 1;
    if (p->mutation_p > 0.0) g = (int)std::ceil(96.0 / (p->pop_size * p->mutation_p));
    g = std::max(1, std::min(g, 1024 / p->pop_size));
    c.mut_group = g;
    return c;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
};

// One generation's kernels. pool/q index cur -> nxt.
hipError_t generation(const DevGraph &g, const GaConst &c, const RunLayout &L, int cur,
                      hipStream_t s, std::vector<EventPair> *ev)
{
    const int nxt = 1 - cur;
    hipError_t e;
    auto mark = [&](int k, bool end) {
        if (!ev) return;
        (void)hipEventRecord(end ? (*ev)[k].b : (*ev)[k].a, s);
    };
    mark(0, false);
    if ((e = launch_rank_parents(c, g.m2, L.st, s)) != hipSuccess) return e;
    mark(0, true);
    mark(1, false);
    if ((e = launch_crossover(g, c, L.st, L.pool[cur], L.q[cur], L.pool[nxt], L.C, L.q[nxt], s)) !=
        hipSuccess)
        return e;
    if ((e = launch_mutation(g, c, L.st, L.C, L.q[nxt], s)) != hipSuccess) return e;
    mark(1, true);
    mark(2, false);
    if ((e = launch_fitness(g, L.q[nxt], c.ld, c.pop, L.hp, L.run, L.off, L.D, L.st.Aq, L.st.Sq,
                            s)) != hipSuccess)
        return e;
    mark(2, true);
    mark(3, false);
    if (!L.hp.enabled && (e = launch_fill_zero(L.D, L.plane, s)) != hipSuccess) return e;
    mark(3, true);
    mark(4, false);
    if ((e = launch_select(c, g.m2, L.st, s)) != hipSuccess) return e;
    mark(4, true);
    return hipSuccess;
}

// Host copy of P (selection order) as rows, for the trace callback.
int emit_state(const hpmocd_graph *G, const GaConst &c, const RunLayout &L, int cur, int32_t gen,
               hipStream_t s, hpmocd_trace_fn fn, void *user, bool with_labels)
{
    const int32_t n = G->n, pop = c.pop, ld = c.ld;
    const size_t plane_cells = with_labels ? (size_t)n * ld : 0;
    std::vector<int32_t> pool(plane_cells), q(plane_cells), ids(pop), rank(pop);
    std::vector<int64_t> A(pop), S(pop);
    std::vector<double> f1(pop), f2(pop), crowd(pop);
    HIP_TRY(hipStreamSynchronize(s));
    if (with_labels && gen > 0)
        HIP_TRY(hipMemcpy(pool.data(), L.pool[cur], L.plane, hipMemcpyDeviceToHost));
    if (with_labels) HIP_TRY(hipMemcpy(q.data(), L.q[cur], L.plane, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ids.data(), L.st.ps_id, sizeof(int32_t) * pop, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(A.data(), L.st.ps_A, sizeof(int64_t) * pop, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(S.data(), L.st.ps_S, sizeof(int64_t) * pop, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(f1.data(), L.st.ps_f1, sizeof(double) * pop, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(f2.data(), L.st.ps_f2, sizeof(double) * pop, hipMemcpyDeviceToHost));
    if (gen > 0) {
        HIP_TRY(hipMemcpy(rank.data(), L.st.tr_rank, sizeof(int32_t) * pop, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(crowd.data(), L.st.tr_crowd, sizeof(double) * pop, hipMemcpyDeviceToHost));
    }
    std::vector<int32_t> rows(with_labels ? (size_t)pop * n : 0);
    for (int32_t i = 0; with_labels && i < pop; ++i) {
        const int32_t id = ids[i];
        const int32_t *src = id < pop ? pool.data() + id : q.data() + (id - pop);
        int32_t *dst = rows.data() + (size_t)i * n;
        for (int32_t v = 0; v < n; ++v) dst[v] = src[(size_t)v * ld];
    }
    hpmocd_state_view view;
    view.g = gen;
    view.pop_size = pop;
    view.n_nodes = n;
    view.labels = with_labels ? rows.data() : nullptr;
    view.A = A.data();
    view.S = S.data();
    view.f1 = f1.data();
    view.f2 = f2.data();
    view.rank = gen > 0 ? rank.data() : nullptr;
    view.crowd = gen > 0 ? crowd.data() : nullptr;
    fn(&view, user);
    return HPMOCD_OK;
}

struct EventSet {
    std::vector<hipEvent_t> all;
    ~EventSet()
    {
        for (hipEvent_t e : all) (void)hipEventDestroy(e);
    }
    hipEvent_t make()
    {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        all.push_back(e);
        return e;
    }
};

float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

}  // namespace

namespace {
struct EvalLayout {
    int32_t ld = 0;
    size_t plane = 0;
    HistPlan hp;
    uint32_t *run = nullptr, *off = nullptr;
    int32_t *lab = nullptr, *D = nullptr;
    unsigned long long *A = nullptr, *S = nullptr;
    double *f1 = nullptr, *f2 = nullptr;
    size_t bytes = 0;
};
EvalLayout carve_eval(void *ws, int32_t n, int32_t n_ind, int32_t max_deg)
{
    EvalLayout L;
    L.ld = round16(n_ind);
    L.plane = (size_t)n * (size_t)L.ld * sizeof(int32_t);
    L.hp = hist_plan(n, n_ind, max_deg);
    Carver cv(ws);
    L.lab = cv.take<int32_t>((size_t)n * L.ld);
    if (L.hp.enabled) {
        L.run = cv.take<uint32_t>(L.hp.entries);
        L.off = cv.take<uint32_t>(L.hp.offsets);
    } else {
        L.D = cv.take<int32_t>((size_t)n * L.ld);
    }
    L.A = cv.take<unsigned long long>(n_ind);
    L.S = cv.take<unsigned long long>(n_ind);
    L.f1 = cv.take<double>(n_ind);
    L.f2 = cv.take<double>(n_ind);
    L.bytes = cv.off;
    return L;
}
}  // namespace

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

int hpmocd_workspace_size(const hpmocd_graph *g, const hpmocd_params *p, size_t *bytes)
{
    if (!g || !bytes) return HPMOCD_ERR_ARG;
    int rc = check_params(p);
    if (rc) return rc;
    *bytes = carve_run(nullptr, g->n, p->pop_size, p->parents_per_child, g->max_deg).bytes;
    return HPMOCD_OK;
}

void hpmocd_front_free(hpmocd_front *f)
{
    if (!f) return;
    std::free(f->labels);
    std::free(f->intra_arcs);
    std::free(f->sum_deg_sq);
    std::free(f->f1);
    std::free(f->f2);
    std::free(f);
}

int hpmocd_run_ex(const hpmocd_graph *G, const hpmocd_params *p, void *ws, size_t ws_bytes,
                  void *stream, int flags, hpmocd_profile *prof, hpmocd_trace_fn trace,
                  void *user, hpmocd_front **out)
{
    if (!G || !out || !ws) return HPMOCD_ERR_ARG;
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_device(G))) return rc;
    const int32_t pop = p->pop_size, T = p->generations, n = G->n;
    RunLayout L = carve_run(ws, n, pop, p->parents_per_child, G->max_deg);
    if (ws_bytes < L.bytes) return HPMOCD_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const DevGraph dg = dev_graph(G);
    const GaConst c = ga_const(p, L.ld);
    const bool time_kernels = (flags & HPMOCD_TIME_KERNELS) != 0 && prof;
    const bool trace_labels = (flags & HPMOCD_TRACE_NO_LABELS) == 0;
    const bool use_graph = !(flags & (HPMOCD_NO_GRAPH | HPMOCD_TIME_KERNELS)) && !trace &&
                           s != nullptr && T >= 2;

    EventSet evs;
    hipEvent_t e_start = nullptr, e_loop0 = nullptr, e_loop1 = nullptr, e_end = nullptr;
    hipEvent_t e_fit0 = nullptr, e_fit1 = nullptr, e_sw1 = nullptr;
    // kernel-group events for every generation are created before the run starts, and read
    // only after it ends, so timing adds no host synchronisation to the loop
    std::vector<std::vector<EventPair>> gen_events;
    if (time_kernels) {
        gen_events.assign((size_t)T, std::vector<EventPair>(5));
        for (auto &v : gen_events)
            for (auto &pr : v) {
                pr.a = evs.make();
                pr.b = evs.make();
                if (!pr.a || !pr.b) return HPMOCD_ERR_HIP;
            }
    }
    if (prof) {
        e_start = evs.make();
        e_loop0 = evs.make();
        e_loop1 = evs.make();
        e_end = evs.make();
        e_fit0 = evs.make();
        e_fit1 = evs.make();
        e_sw1 = evs.make();
        if (!e_start || !e_loop0 || !e_loop1 || !e_end || !e_fit0 || !e_fit1 || !e_sw1)
            return HPMOCD_ERR_HIP;
        HIP_TRY(hipEventRecord(e_start, s));
    }

    // initial population (Alg. 1 phases 1-2) into offspring buffer 0
    if (!L.hp.enabled) HIP_TRY(launch_fill_zero(L.D, L.plane, s));
    HIP_TRY(launch_fill_zero(L.st.Aq, sizeof(unsigned long long) * pop, s));
    HIP_TRY(launch_fill_zero(L.st.Sq, sizeof(unsigned long long) * pop, s));
    HIP_TRY(launch_init(dg, c, L.q[0], s));
    if (prof) HIP_TRY(hipEventRecord(e_fit0, s));
    HIP_TRY(launch_fitness(dg, L.q[0], c.ld, pop, L.hp, L.run, L.off, L.D, L.st.Aq, L.st.Sq, s));
    if (prof) HIP_TRY(hipEventRecord(e_fit1, s));
    if (!L.hp.enabled) HIP_TRY(launch_fill_zero(L.D, L.plane, s));
    if (prof) HIP_TRY(hipEventRecord(e_sw1, s));
    HIP_TRY(launch_init_state(c, G->m2, L.st, s));
    int cur = 0;
    if (trace && (rc = emit_state(G, c, L, cur, 0, s, trace, user, trace_labels))) return rc;

    double fit_ms = 0, sweep_ms = 0, var_ms = 0, sel_ms = 0;
    if (prof) HIP_TRY(hipEventRecord(e_loop0, s));
    int32_t gdone = 0;
    if (use_graph) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e1 = generation(dg, c, L, 0, s, nullptr);
        hipError_t e2 = e1 == hipSuccess ? generation(dg, c, L, 1, s, nullptr) : e1;
        hipError_t ec = hipStreamEndCapture(s, &graph);
        if (e1 != hipSuccess || e2 != hipSuccess || ec != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return HPMOCD_ERR_HIP;
        }
        hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return HPMOCD_ERR_HIP;
        hipError_t el = hipSuccess;
        for (int32_t k = 0; k < T / 2 && el == hipSuccess; ++k) el = hipGraphLaunch(exec, s);
        (void)hipGraphExecDestroy(exec);
        if (el != hipSuccess) return HPMOCD_ERR_HIP;
        gdone = (T / 2) * 2;
        cur = 0;
    }
    for (int32_t gen = gdone + 1; gen <= T; ++gen) {
        std::vector<EventPair> *ev = time_kernels ? &gen_events[(size_t)(gen - 1)] : nullptr;
        HIP_TRY(generation(dg, c, L, cur, s, ev));
        cur = 1 - cur;
        if (trace && (rc = emit_state(G, c, L, cur, gen, s, trace, user, trace_labels))) return rc;
    }
    if (prof) HIP_TRY(hipEventRecord(e_loop1, s));

    // phase 4: first front, in crowded order
    HIP_TRY(launch_final(c, G->m2, L.st, s));
    int32_t k = 0;
    HIP_TRY(hipMemcpyAsync(&k, L.st.fr_count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (k < 1 || k > pop) return HPMOCD_ERR_HIP;
    HIP_TRY(launch_extract(n, c.ld, pop, L.pool[cur], L.q[cur], L.st.fr_id, k, L.C, s));
    hpmocd_front *f = (hpmocd_front *)std::calloc(1, sizeof(hpmocd_front));
    if (!f) return HPMOCD_ERR_NOMEM;
    f->n_solutions = k;
    f->n_nodes = n;
    f->labels = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)k * n);
    f->intra_arcs = (int64_t *)std::malloc(sizeof(int64_t) * k);
    f->sum_deg_sq = (int64_t *)std::malloc(sizeof(int64_t) * k);
    f->f1 = (double *)std::malloc(sizeof(double) * k);
    f->f2 = (double *)std::malloc(sizeof(double) * k);
    if (!f->labels || !f->intra_arcs || !f->sum_deg_sq || !f->f1 || !f->f2) {
        hpmocd_front_free(f);
        return HPMOCD_ERR_NOMEM;
    }
    bool ok = hipMemcpyAsync(f->labels, L.C, sizeof(int32_t) * (size_t)k * n, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(f->intra_arcs, L.st.fr_A, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(f->sum_deg_sq, L.st.fr_S, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(f->f1, L.st.fr_f1, sizeof(double) * k, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(f->f2, L.st.fr_f2, sizeof(double) * k, hipMemcpyDeviceToHost, s) == hipSuccess;
    if (prof) ok = ok && hipEventRecord(e_end, s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        hpmocd_front_free(f);
        return HPMOCD_ERR_HIP;
    }
    // Alg. 3: first maximiser of Q = (1 - f1) - f2
    double best = -INFINITY;
    int32_t sel = 0;
    for (int32_t i = 0; i < k; ++i) {
        const double qv = (1.0 - f->f1[i]) - f->f2[i];
        if (qv > best) {
            best = qv;
            sel = i;
        }
    }
    f->selected = sel;
    if (time_kernels) {
        for (auto &ev : gen_events) {
            sel_ms += elapsed(ev[0].a, ev[0].b) + elapsed(ev[4].a, ev[4].b);
            var_ms += elapsed(ev[1].a, ev[1].b);
            fit_ms += elapsed(ev[2].a, ev[2].b);
            sweep_ms += elapsed(ev[3].a, ev[3].b);
        }
    }
    if (prof) {
        prof->total_ms = elapsed(e_start, e_end);
        prof->loop_ms = elapsed(e_loop0, e_loop1);
        prof->fitness_ms = time_kernels ? fit_ms + elapsed(e_fit0, e_fit1) : 0.0;
        prof->sweep_ms = time_kernels ? sweep_ms + elapsed(e_fit1, e_sw1) : 0.0;
        prof->variation_ms = time_kernels ? var_ms : 0.0;
        prof->select_ms = time_kernels ? sel_ms : 0.0;
        prof->fitness_launches = (int64_t)T + 1;
        prof->individual_evals = (int64_t)pop * ((int64_t)T + 1);
    }
    *out = f;
    return HPMOCD_OK;
}

int hpmocd_run(const hpmocd_graph *g, const hpmocd_params *p, void *ws, size_t ws_bytes,
               void *stream, hpmocd_front **out)
{
    return hpmocd_run_ex(g, p, ws, ws_bytes, stream, 0, nullptr, nullptr, nullptr, out);
}


int hpmocd_eval_workspace_size(const hpmocd_graph *g, int32_t n_ind, size_t *bytes)
{
    if (!g || !bytes || n_ind < 1) return HPMOCD_ERR_ARG;
    *bytes = carve_eval(nullptr, g->n, n_ind, g->max_deg).bytes;
    return HPMOCD_OK;
}

int hpmocd_eval(const hpmocd_graph *G, const int32_t *d_labels, int32_t n_ind, void *ws,
                size_t ws_bytes, void *stream, int64_t *A, int64_t *S, double *f1, double *f2,
                double *kernel_ms)
{
    if (!G || !d_labels || n_ind < 1 || !ws || !A || !S || !f1 || !f2) return HPMOCD_ERR_ARG;
    int rc = check_device(G);
    if (rc) return rc;
    EvalLayout L = carve_eval(ws, G->n, n_ind, G->max_deg);
    if (ws_bytes < L.bytes) return HPMOCD_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const DevGraph dg = dev_graph(G);
    if (!L.hp.enabled) HIP_TRY(launch_fill_zero(L.D, L.plane, s));
    HIP_TRY(launch_fill_zero(L.A, sizeof(unsigned long long) * n_ind, s));
    HIP_TRY(launch_fill_zero(L.S, sizeof(unsigned long long) * n_ind, s));
    HIP_TRY(launch_transpose_in(d_labels, G->n, n_ind, L.ld, L.lab, s));
    EventSet evs;
    hipEvent_t a = nullptr, b = nullptr;
    if (kernel_ms) {
        a = evs.make();
        b = evs.make();
        if (!a || !b) return HPMOCD_ERR_HIP;
        HIP_TRY(hipEventRecord(a, s));
    }
    HIP_TRY(launch_fitness(dg, L.lab, L.ld, n_ind, L.hp, L.run, L.off, L.D, L.A, L.S, s));
    if (kernel_ms) HIP_TRY(hipEventRecord(b, s));
    HIP_TRY(launch_finalize(G->m2, n_ind, L.A, L.S, L.f1, L.f2, s));
    std::vector<unsigned long long> hA(n_ind), hS(n_ind);
    HIP_TRY(hipMemcpyAsync(hA.data(), L.A, sizeof(unsigned long long) * n_ind, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hS.data(), L.S, sizeof(unsigned long long) * n_ind, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(f1, L.f1, sizeof(double) * n_ind, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(f2, L.f2, sizeof(double) * n_ind, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int32_t i = 0; i < n_ind; ++i) {
        A[i] = (int64_t)hA[i];
        S[i] = (int64_t)hS[i];
    }
    if (kernel_ms) *kernel_ms = elapsed(a, b);
    return HPMOCD_OK;
}

}  // extern "C"
