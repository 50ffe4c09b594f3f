// Runs of Alg. 1 on the device: workspace carving, the batch runner (many populations, each
// on its own graph, advanced together by multi-item launches), hipGraph replay of the
// generation loop, the autotuner, tracing, front extraction and the run/eval entry points.
// A single run is a batch of one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <condition_variable>
#include <initializer_list>
#include <mutex>
#include <thread>
#include <vector>

#include <sys/mman.h>

#include "host.hpp"
#include "philox.hpp"
#include "run.hpp"

namespace hpm {

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }
int32_t round16(int32_t x) { return (x + 15) / 16 * 16; }

namespace {

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

}  // namespace

RunLayout carve_run(void *ws, int32_t n, int32_t pop, int32_t es, int32_t max_deg,
                    const Tuning &t, bool both_histograms)
{
    RunLayout L;
    L.hp = hist_plan(n, pop, max_deg, t.hist_min_log2, t.hist_rbits, t.hist_narrow != 0);
    L.ld = round16(pop);
    L.plane = (size_t)n * (size_t)L.ld * sizeof(int32_t);
    Carver cv(ws);
    const size_t cells = (size_t)n * (size_t)L.ld;
    L.pool[0] = cv.take<int32_t>(cells);
    L.pool[1] = cv.take<int32_t>(cells);
    L.q[0] = cv.take<int32_t>(cells);
    L.q[1] = cv.take<int32_t>(cells);
    L.C = cv.take<int32_t>(cells);
    size_t entries = L.hp.enabled ? L.hp.entries : 0, offsets = L.hp.enabled ? L.hp.offsets : 0;
    if (both_histograms)
        for (int32_t rb : HIST_RBITS_CHOICES)  // every binned plan the autotuner may pick
            for (bool narrow : {false, true}) {
                const HistPlan h = hist_plan(n, pop, max_deg, 0, rb, narrow);
                if (!h.enabled) continue;
                entries = std::max(entries, h.entries);
                offsets = std::max(offsets, h.offsets);
            }
    if (entries) {
        L.run = cv.take<uint32_t>(entries);
        L.off = cv.take<uint32_t>(offsets);
    }
    if (!L.hp.enabled || both_histograms) L.D = cv.take<int32_t>(cells);
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
    s.fr_sel = cv.take<int32_t>(1);
    s.fr_id = cv.take<int32_t>(pop);
    s.fr_A = cv.take<int64_t>(pop);
    s.fr_S = cv.take<int64_t>(pop);
    s.fr_f1 = cv.take<double>(pop);
    s.fr_f2 = cv.take<double>(pop);
    L.bytes = cv.off;
    return L;
}

int32_t mut_target_for(const Tuning &t, int64_t nodes)
{
    if (t.mut_target_items > 0) return t.mut_target_items;
    return nodes >= (int64_t(1) << 18) ? 96 : 48;  // measured best at 1M and at 1k-40k nodes
}

GaConst ga_const(const hpmocd_params *p, int32_t ld, int32_t mut_target)
{
    GaConst c;
    c.pop = p->pop_size;
    c.ld = ld;
    c.es = p->parents_per_child;
    c.seed = p->seed;
    c.thr_c = bernoulli_threshold(p->crossover_p);
    c.thr_m = bernoulli_threshold(p->mutation_p);
    // nodes per wave group in the small-degree mutation kernels: enough candidate (node,
    // offspring) pairs to fill about mut_target mutations, within the LDS list capacity
    int g = 1;
    if (p->mutation_p > 0.0) g = (int)std::ceil(mut_target / (p->pop_size * p->mutation_p));
    g = std::max(1, std::min(g, 1024 / p->pop_size));
    c.mut_group = g;
    return c;
}

void Pop::setup(const hpmocd_graph *graph, const hpmocd_params &params, void *ws,
                const Tuning &t, int64_t batch_nodes, bool both_histograms)
{
    G = graph;
    p = params;
    L = carve_run(ws, G->n, p.pop_size, p.parents_per_child, G->max_deg, t, both_histograms);
    c = ga_const(&p, L.ld, mut_target_for(t, std::max<int64_t>(batch_nodes, G->n)));
    dg = dev_graph(G);
    shape(t, batch_nodes);
    cur = 0;
}

void Pop::shape(const Tuning &t, int64_t batch_nodes)
{
    const int64_t npw = batch_nodes / std::max<int64_t>(1, t.fit_target_waves);
    fit_npw = (int32_t)std::max<int64_t>(1, std::min<int64_t>(64, npw));
    const int64_t nb = batch_nodes / std::max<int64_t>(1, t.xo_target_blocks);
    // the crossover stages its nodes' two rows in LDS beside its tables: 64 KB in all, and
    // at most 16 nodes per workgroup (measured at |V| = 1M: 8, 16, 24, 32, 64 nodes ->
    // 0.62, 0.56, 0.57, 0.58, 0.82 ms of crossover per generation)
    const int64_t tables = 4 * ((((int64_t)2 + p.parents_per_child) * p.pop_size + 3) & ~3);
    const int64_t lds_nodes = std::max<int64_t>(1, (65536 - tables) / (8 * (int64_t)L.ld));
    xo_nb = (int32_t)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(16, lds_nodes), nb));
}

Item Pop::item(int which) const
{
    Item it{};
    it.g = dg;
    it.c = c;
    it.st = L.st;
    it.hp = L.hp;
    it.D = L.D;
    it.D_bytes = L.D ? L.plane : 0;
    it.run = L.run;
    it.off = L.off;
    it.fit_pop = c.pop;
    it.fit_ld = L.ld;
    it.fit_A = L.st.Aq;
    it.fit_S = L.st.Sq;
    it.fit_npw = fit_npw;
    it.xo_nb = xo_nb;
    it.C = L.C;
    if (which == ITEM_INIT) {
        it.q_cur = L.q[0];
        it.lab = L.q[0];
        it.pool_cur = L.pool[0];
        it.pool_new = L.pool[1];
        it.q_next = L.q[1];
    } else {
        const int a = which == ITEM_PARITY0 ? 0 : 1, b = 1 - a;
        it.pool_cur = L.pool[a];
        it.q_cur = L.q[a];
        it.pool_new = L.pool[b];
        it.q_next = L.q[b];
        it.lab = L.q[b];
    }
    return it;
}

size_t meta_bytes(int32_t count)
{
    return align_up(sizeof(Item) * (size_t)count) +
           align_up(sizeof(int32_t) * (size_t)N_KINDS * ((size_t)count + 1));
}

int Meta::upload(const Item *host_items, int32_t n_items, void *region, hipStream_t s,
                 Pinned *stage)
{
    count = n_items;
    items = (Item *)region;
    starts = (int32_t *)((char *)region + align_up(sizeof(Item) * (size_t)count));
    const size_t n_starts = (size_t)N_KINDS * ((size_t)count + 1);
    Item *hi = &h_item1;
    int32_t *st = h_starts1;
    if (count == 1) {
        h_item1 = host_items[0];
    } else {
        h_items.assign(host_items, host_items + count);
        h_starts.assign(n_starts, 0);
        hi = h_items.data();
        st = h_starts.data();
    }
    for (int k = 0; k < N_KINDS; ++k) {
        int32_t *row = st + (size_t)k * (count + 1);
        int64_t acc = 0;
        lds[k] = 0;
        aux[k] = 0;
        for (int32_t i = 0; i < count; ++i) {
            row[i] = (int32_t)acc;
            acc += kind_blocks((Kind)k, host_items[i]);
            lds[k] = std::max(lds[k], kind_lds((Kind)k, host_items[i]));
            aux[k] = std::max(aux[k], kind_aux((Kind)k, host_items[i]));
        }
        row[count] = (int32_t)acc;
        if (acc > 0x7fffffff) return HPMOCD_ERR_ARG;
        totals[k] = (int32_t)acc;
    }
    const void *src_items = hi, *src_starts = st;
    if (stage) {
        src_items = stage->stage(hi, sizeof(Item) * (size_t)count);
        src_starts = stage->stage(st, sizeof(int32_t) * n_starts);
    }
    HIP_TRY(hipMemcpyAsync(items, src_items, sizeof(Item) * (size_t)count, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(starts, src_starts, sizeof(int32_t) * n_starts, hipMemcpyHostToDevice, s));
    return HPMOCD_OK;
}

hipError_t Meta::launch(Kind k, hipStream_t s) const
{
    return launch_kind(k, span(k), totals[k], lds[k], aux[k], s);
}

hipError_t Meta::one(OneKernel which, hipStream_t s) const
{
    return launch_one(which, span(K_ONE), count, s);
}

// Fitness of a population. k_fitness (A) only reads the labels, so with a fork it runs
// beside k_hist: k_bin first (bandwidth-bound, like the arc scan), then the arc scan on a
// side stream next to k_hist, whose dependent offset -> run -> LDS chains leave most of the
// memory bandwidth free; both join back into s.
hipError_t launch_fitness_kinds(const Meta &m, hipStream_t s, const Fork *fk)
{
    hipError_t e;
    if ((e = m.launch(K_BIN, s)) != hipSuccess) return e;
    hipStream_t scan = s;
    if (fk && m.totals[K_HIST] > 0) {
        if ((e = hipEventRecord(fk->fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(fk->side[0], fk->fork, 0)) != hipSuccess) return e;
        scan = fk->side[0];
    }
    // k_hist first: its workgroups need 64 KB of LDS each and would otherwise find the CUs
    // full of arc-scan waves
    if ((e = m.launch(K_HIST, s)) != hipSuccess) return e;
    if ((e = m.launch(K_FIT, scan)) != hipSuccess) return e;
    if (scan != s) {
        if ((e = hipEventRecord(fk->join[0], scan)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, fk->join[0], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_init_seq(const Meta &m, hipStream_t s, const Fork *fk)
{
    hipError_t e;
    if ((e = m.launch(K_CLEAR, s)) != hipSuccess) return e;  // plain histograms start at zero
    if ((e = m.one(ONE_ZERO_ACC, s)) != hipSuccess) return e;
    if ((e = m.launch(K_INIT, s)) != hipSuccess) return e;
    if ((e = launch_fitness_kinds(m, s, fk)) != hipSuccess) return e;
    if ((e = m.launch(K_CLEAR, s)) != hipSuccess) return e;
    return m.one(ONE_INIT_STATE, s);
}

int Fork::init()
{
    for (int i = 0; i < 2; ++i) {
        if (!side[i]) HIP_TRY(hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking));
        if (!join[i]) HIP_TRY(hipEventCreateWithFlags(&join[i], hipEventDisableTiming));
    }
    if (!fork) HIP_TRY(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    return HPMOCD_OK;
}

Fork::~Fork()
{
    for (int i = 0; i < 2; ++i) {
        if (side[i]) {
            (void)hipStreamSynchronize(side[i]);  // work left unjoined by an error path
            (void)hipStreamDestroy(side[i]);
        }
        if (join[i]) (void)hipEventDestroy(join[i]);
    }
    if (fork) (void)hipEventDestroy(fork);
}

// Mutation launches of one generation. With a fork, three branches joined back into s: degree
// class <= 16 on s; 33-64, then 17-32 on the first side stream; the wave classes from the
// highest degree down, then the large nodes, on the second. Longest items first within a
// branch: a branch's last kernel then has short items to fill the chip with. At |V| = 1M,
// pop 100, this order ran 337 generations/s against 329 for ascending order in each branch
// (the fork as a whole: 287 with every class on s).
static hipError_t launch_mutation(const Meta &m, hipStream_t s, const Fork *fk)
{
    hipError_t e;
    if (!fk) {
        for (int k = 0; k < N_DEG_CLASSES; ++k)
            if ((e = m.launch((Kind)(K_MUT0 + k), s)) != hipSuccess) return e;
        return m.launch(K_MUTL, s);
    }
    static_assert(N_DEG_CLASSES == 8, "branch plan below covers classes 0-7");
    static const int side0[] = {2, 1}, side1[] = {6, 5, 4, 3, 7};
    if ((e = hipEventRecord(fk->fork, s)) != hipSuccess) return e;
    for (int i = 0; i < 2; ++i)
        if ((e = hipStreamWaitEvent(fk->side[i], fk->fork, 0)) != hipSuccess) return e;
    if ((e = m.launch(K_MUT0, s)) != hipSuccess) return e;
    for (int k : side0)
        if ((e = m.launch((Kind)(K_MUT0 + k), fk->side[0])) != hipSuccess) return e;
    for (int k : side1)
        if ((e = m.launch((Kind)(K_MUT0 + k), fk->side[1])) != hipSuccess) return e;
    if ((e = m.launch(K_MUTL, fk->side[1])) != hipSuccess) return e;
    for (int i = 0; i < 2; ++i) {
        if ((e = hipEventRecord(fk->join[i], fk->side[i])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, fk->join[i], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_generation(const Meta &m, hipStream_t s, const EventPair *ev, const Fork *fk)
{
    hipError_t e;
    auto mark = [&](int k, bool end) {
        if (ev) (void)hipEventRecord(end ? ev[k].b : ev[k].a, s);
    };
    mark(0, false);
    if ((e = m.one(ONE_RANK_PARENTS, s)) != hipSuccess) return e;
    mark(0, true);
    mark(1, false);
    mark(5, false);
    if ((e = m.launch(K_XO, s)) != hipSuccess) return e;
    mark(5, true);
    if ((e = launch_mutation(m, s, fk)) != hipSuccess) return e;
    mark(1, true);
    mark(2, false);
    if ((e = launch_fitness_kinds(m, s, fk)) != hipSuccess) return e;
    mark(2, true);
    mark(3, false);
    if ((e = m.launch(K_CLEAR, s)) != hipSuccess) return e;
    mark(3, true);
    mark(4, false);
    if ((e = m.one(ONE_SELECT, s)) != hipSuccess) return e;
    mark(4, true);
    return hipSuccess;
}

float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

EventSet::~EventSet()
{
    for (hipEvent_t e : all) (void)hipEventDestroy(e);
}

hipEvent_t EventSet::make()
{
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    all.push_back(e);
    return e;
}

// Host copy of one population (selection order) for the trace callback.
int emit_state(const Pop &P, int32_t gen, hipStream_t s, hpmocd_trace_fn fn, void *user,
               bool with_labels)
{
    const int32_t n = P.G->n, pop = P.c.pop, ld = P.c.ld;
    const RunLayout &L = P.L;
    const int cur = P.cur;
    const size_t plane_cells = with_labels ? (size_t)n * ld : 0;
    std::vector<int32_t> pool(plane_cells), q(plane_cells), ids(pop), rank(pop);
    std::vector<int64_t> A(pop), S(pop);
    std::vector<double> f1(pop), f2(pop), crowd(pop);
    const hipMemcpyKind d2h = hipMemcpyDeviceToHost;
    if (with_labels && gen > 0) HIP_TRY(hipMemcpyAsync(pool.data(), L.pool[cur], L.plane, d2h, s));
    if (with_labels) HIP_TRY(hipMemcpyAsync(q.data(), L.q[cur], L.plane, d2h, s));
    HIP_TRY(hipMemcpyAsync(ids.data(), L.st.ps_id, sizeof(int32_t) * pop, d2h, s));
    HIP_TRY(hipMemcpyAsync(A.data(), L.st.ps_A, sizeof(int64_t) * pop, d2h, s));
    HIP_TRY(hipMemcpyAsync(S.data(), L.st.ps_S, sizeof(int64_t) * pop, d2h, s));
    HIP_TRY(hipMemcpyAsync(f1.data(), L.st.ps_f1, sizeof(double) * pop, d2h, s));
    HIP_TRY(hipMemcpyAsync(f2.data(), L.st.ps_f2, sizeof(double) * pop, d2h, s));
    if (gen > 0) {
        HIP_TRY(hipMemcpyAsync(rank.data(), L.st.tr_rank, sizeof(int32_t) * pop, d2h, s));
        HIP_TRY(hipMemcpyAsync(crowd.data(), L.st.tr_crowd, sizeof(double) * pop, d2h, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
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

// Front of one population after its final ranking (k_final has run): device -> host.
namespace {

// Device-to-host copies of large results (a front's labels: up to N_p x n int32, 400 MB at
// |V| = 1M, pop 100; a batch's fronts together). From pageable memory the runtime stages such
// a copy through small buffers of its own at a few GB/s. Here the pieces to copy are packed
// into BOUNCE_BUFS page-locked chunks per device (allocated on first use, kept until the
// process ends): the calling thread keeps the DMA engine fed, one chunk after another, while
// up to COPY_THREADS helper threads copy completed chunks out on the host, each taking every
// COPY_THREADS-th chunk. One thread copying out into freshly mapped memory ran at about 14
// GB/s, well below the link. Calls from several threads take turns.
constexpr size_t BOUNCE_CHUNK = (size_t)8 << 20;
constexpr int BOUNCE_BUFS = 8;
constexpr int COPY_THREADS = 4;
constexpr size_t BOUNCE_MIN = (size_t)4 << 20;  // less in all goes direct
constexpr int BOUNCE_DEVICES = 64;
struct Bounce {
    std::mutex mu;
    bool tried = false;
    char *buf[BOUNCE_BUFS] = {};
    hipEvent_t ev[BOUNCE_BUFS] = {};
};
Bounce g_bounce[BOUNCE_DEVICES];

bool bounce_ready(Bounce *b)
{
    if (!b->tried) {
        b->tried = true;
        bool ok = true;
        for (int i = 0; i < BOUNCE_BUFS; ++i) {
            ok = ok && hipHostMalloc((void **)&b->buf[i], BOUNCE_CHUNK, hipHostMallocDefault) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming) == hipSuccess;
        }
        if (!ok) {
            for (int i = 0; i < BOUNCE_BUFS; ++i) {
                if (b->buf[i]) (void)hipHostFree(b->buf[i]);
                if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
                b->buf[i] = nullptr;
                b->ev[i] = nullptr;
            }
        }
    }
    return b->buf[0] != nullptr;
}

// Hand-off between the thread that issues the chunk copies and the helpers that copy the
// chunks out: chunk i may be issued once chunk i - BOUNCE_BUFS (the buffer's previous
// content) has been copied out.
struct ChunkBoard {
    std::mutex mu;
    std::condition_variable cv;
    size_t issued = 0;
    std::vector<char> out;  // per chunk: copied out
    bool failed = false;
};

// one piece of a chunk: bytes [off, off + len) of the chunk go to dst, from src on the device
struct Piece {
    char *dst;
    const char *src;
    size_t len, off;
};

}  // namespace

// Copies every segment from device memory to host memory in stream order on s; returns with
// the copies complete.
hipError_t copy_segments(const HostSeg *segs, size_t count, hipStream_t s)
{
    size_t total = 0;
    for (size_t i = 0; i < count; ++i) total += segs[i].bytes;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    Bounce *b = (dev >= 0 && dev < BOUNCE_DEVICES && total >= BOUNCE_MIN) ? &g_bounce[dev] : nullptr;
    std::unique_lock<std::mutex> lock;
    if (b) {
        lock = std::unique_lock<std::mutex>(b->mu);
        if (!bounce_ready(b)) b = nullptr;
    }
    if (!b) {
        for (size_t i = 0; i < count; ++i)
            if (segs[i].bytes &&
                (e = hipMemcpyAsync(segs[i].dst, segs[i].src, segs[i].bytes, hipMemcpyDeviceToHost, s)) != hipSuccess) {
                (void)hipStreamSynchronize(s);
                return e;
            }
        return hipStreamSynchronize(s);
    }
    // pack the segments into chunks, each piece 256-byte aligned in its chunk
    std::vector<std::vector<Piece>> chunks(1);
    size_t fill = 0;
    for (size_t i = 0; i < count; ++i) {
        for (size_t done = 0; done < segs[i].bytes;) {
            fill = (fill + 255) / 256 * 256;
            if (fill >= BOUNCE_CHUNK) {
                chunks.emplace_back();
                fill = 0;
            }
            const size_t len = std::min(segs[i].bytes - done, BOUNCE_CHUNK - fill);
            chunks.back().push_back({(char *)segs[i].dst + done, (const char *)segs[i].src + done, len, fill});
            fill += len;
            done += len;
        }
    }
    const size_t nchunk = chunks.size();
    ChunkBoard bd;
    bd.out.assign(nchunk, 0);
    std::vector<hipError_t> werr;
    auto helper = [&](size_t first, size_t step, hipError_t *err) {
        for (size_t j = first; j < nchunk; j += step) {
            {
                std::unique_lock<std::mutex> lk(bd.mu);
                bd.cv.wait(lk, [&] { return bd.issued > j || bd.failed; });
                if (bd.failed) return;
            }
            const hipError_t ee = hipEventSynchronize(b->ev[j % BOUNCE_BUFS]);
            if (ee == hipSuccess)
                for (const Piece &pc : chunks[j]) std::memcpy(pc.dst, b->buf[j % BOUNCE_BUFS] + pc.off, pc.len);
            std::lock_guard<std::mutex> lk(bd.mu);
            if (ee != hipSuccess) {
                *err = ee;
                bd.failed = true;
            } else {
                bd.out[j] = 1;
            }
            bd.cv.notify_all();
            if (ee != hipSuccess) return;
        }
    };
    auto issue = [&](size_t i, char *buf) {
        hipError_t ee = hipSuccess;
        for (const Piece &pc : chunks[i])
            if ((ee = hipMemcpyAsync(buf + pc.off, pc.src, pc.len, hipMemcpyDeviceToHost, s)) != hipSuccess) break;
        return ee;
    };
    const size_t want = std::min<size_t>(COPY_THREADS, nchunk);
    werr.assign(want, hipSuccess);
    std::vector<std::thread> th;
    try {
        for (size_t t = 0; t < want; ++t) th.emplace_back(helper, t, want, &werr[t]);
    } catch (...) {  // no thread to spare: stop the helpers that did start
        std::lock_guard<std::mutex> lk(bd.mu);
        bd.failed = true;
        bd.cv.notify_all();
    }
    if (th.size() < want) {  // and copy one chunk at a time
        for (auto &x : th) x.join();
        for (size_t i = 0; i < nchunk; ++i) {
            if ((e = issue(i, b->buf[0])) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess) {
                (void)hipStreamSynchronize(s);
                return e;
            }
            for (const Piece &pc : chunks[i]) std::memcpy(pc.dst, b->buf[0] + pc.off, pc.len);
        }
        return hipSuccess;
    }
    for (size_t i = 0; i < nchunk && e == hipSuccess; ++i) {
        {
            std::unique_lock<std::mutex> lk(bd.mu);
            bd.cv.wait(lk, [&] { return i < BOUNCE_BUFS || bd.out[i - BOUNCE_BUFS] || bd.failed; });
            if (bd.failed) break;
        }
        e = issue(i, b->buf[i % BOUNCE_BUFS]);
        if (e == hipSuccess) e = hipEventRecord(b->ev[i % BOUNCE_BUFS], s);
        std::lock_guard<std::mutex> lk(bd.mu);
        if (e != hipSuccess) bd.failed = true;
        else bd.issued = i + 1;
        bd.cv.notify_all();
    }
    for (auto &x : th) x.join();
    if (e != hipSuccess || bd.failed) {
        (void)hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        for (hipError_t x : werr)
            if (x != hipSuccess) return x;
        return hipErrorUnknown;
    }
    return hipSuccess;
}

hipError_t copy_to_host(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const HostSeg seg{dst, src, bytes};
    return copy_segments(&seg, 1, s);
}

// Small device-to-host copies issued together; drains s whatever happens, so that no copy
// outlives host buffers of the caller's frame on an error return.
hipError_t copy_small(std::initializer_list<HostSeg> segs, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (const HostSeg &g : segs)
        if (e == hipSuccess && g.bytes) e = hipMemcpyAsync(g.dst, g.src, g.bytes, hipMemcpyDeviceToHost, s);
    const hipError_t es = hipStreamSynchronize(s);
    return e != hipSuccess ? e : es;
}

namespace {

// Host memory for fronts' labels. A large buffer is 2 MB-aligned with transparent huge pages
// requested, and once freed it is kept (up to LABEL_CACHE_COUNT buffers, LABEL_CACHE_BYTES in
// all) for the next front it fits: copying a front into memory that is already mapped skips
// the kernel's zeroing of every fresh page, which cost more than the copy itself.
constexpr size_t LABEL_LARGE = (size_t)32 << 20;
constexpr int LABEL_CACHE_COUNT = 2;
constexpr size_t LABEL_CACHE_BYTES = (size_t)2 << 30;
struct LabelCache {
    std::mutex mu;
    std::vector<std::pair<void *, size_t>> live;  // large buffers handed out, and their sizes
    std::vector<std::pair<void *, size_t>> idle;  // freed ones kept for reuse, oldest first
};
LabelCache &label_cache()
{
    static LabelCache *c = new LabelCache;  // never destroyed: frees may come at exit
    return *c;
}

}  // namespace

void *alloc_labels(size_t bytes)
{
    if (bytes < LABEL_LARGE) return std::malloc(bytes ? bytes : 1);
    constexpr size_t HUGE_PAGE = (size_t)2 << 20;
    const size_t rounded = (bytes + HUGE_PAGE - 1) / HUGE_PAGE * HUGE_PAGE;
    LabelCache &c = label_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    size_t best = c.idle.size();
    for (size_t i = 0; i < c.idle.size(); ++i)  // the smallest kept buffer that fits, if not
        if (c.idle[i].second >= rounded && c.idle[i].second <= 2 * rounded &&  // twice too big
            (best == c.idle.size() || c.idle[i].second < c.idle[best].second))
            best = i;
    void *p = nullptr;
    size_t size = rounded;
    if (best < c.idle.size()) {
        p = c.idle[best].first;
        size = c.idle[best].second;
        c.idle.erase(c.idle.begin() + (std::ptrdiff_t)best);
    } else {
        p = std::aligned_alloc(HUGE_PAGE, rounded);
        if (!p) return nullptr;
        (void)madvise(p, rounded, MADV_HUGEPAGE);
    }
    try {
        c.live.emplace_back(p, size);
    } catch (...) {
        std::free(p);
        return nullptr;
    }
    return p;
}

void host_copy(void *dst, const void *src, size_t bytes)
{
    constexpr size_t PART_MIN = (size_t)8 << 20;
    const size_t parts = std::min<size_t>(COPY_THREADS, bytes / PART_MIN);
    if (parts < 2) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const size_t step = (bytes / parts + 4095) / 4096 * 4096;
    auto part = [=](size_t i) {
        const size_t off = std::min(bytes, i * step), len = std::min(step, bytes - off);
        std::memcpy((char *)dst + off, (const char *)src + off, len);
    };
    std::vector<std::thread> th;
    size_t started = 1;  // part 0 is this thread's
    try {
        for (; started < parts; ++started) th.emplace_back(part, started);
    } catch (...) {
    }
    part(0);
    for (size_t i = started; i < parts; ++i) part(i);  // parts no thread could be started for
    for (auto &x : th) x.join();
}

void free_labels(void *p)
{
    if (!p) return;
    LabelCache &c = label_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    size_t i = 0;
    while (i < c.live.size() && c.live[i].first != p) ++i;
    if (i == c.live.size()) {  // a small buffer from malloc
        std::free(p);
        return;
    }
    const std::pair<void *, size_t> e = c.live[i];
    c.live.erase(c.live.begin() + (std::ptrdiff_t)i);
    if (e.second > LABEL_CACHE_BYTES) {
        std::free(p);
        return;
    }
    try {
        c.idle.push_back(e);
    } catch (...) {
        std::free(p);
        return;
    }
    size_t total = 0;
    for (const auto &x : c.idle) total += x.second;
    while (!c.idle.empty() && ((int)c.idle.size() > LABEL_CACHE_COUNT || total > LABEL_CACHE_BYTES)) {
        total -= c.idle.front().second;
        std::free(c.idle.front().first);
        c.idle.erase(c.idle.begin());
    }
}

int extract_front(const Pop &P, hipStream_t s, hpmocd_front **out, Pinned *stage)
{
    if (!stage) {
        const Pop *pp = &P;
        return extract_fronts(&pp, 1, s, out);
    }
    const RunLayout &L = P.L;
    const int32_t n = P.G->n, pop = P.c.pop;
    int32_t ks[2] = {0, 0};  // front size and Alg. 3's choice (both computed by k_final)
    hipError_t e = hipMemcpyAsync(&ks[0], L.st.fr_count, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&ks[1], L.st.fr_sel, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess || e != hipSuccess) return HPMOCD_ERR_HIP;  // ks in scope
    const int32_t k = ks[0];
    if (k < 1 || k > pop || ks[1] < 0 || ks[1] >= k) return HPMOCD_ERR_HIP;
    HIP_TRY(launch_extract(n, P.c.ld, pop, L.pool[P.cur], L.q[P.cur], L.st.fr_id, k, L.C, s));
    hpmocd_front *f = (hpmocd_front *)std::calloc(1, sizeof(hpmocd_front));
    if (!f) return HPMOCD_ERR_NOMEM;
    f->n_solutions = k;
    f->n_nodes = n;
    const size_t lab_bytes = sizeof(int32_t) * (size_t)k * n;
    f->labels = (int32_t *)alloc_labels(lab_bytes);
    f->intra_arcs = (int64_t *)std::malloc(sizeof(int64_t) * k);
    f->sum_deg_sq = (int64_t *)std::malloc(sizeof(int64_t) * k);
    f->f1 = (double *)std::malloc(sizeof(double) * k);
    f->f2 = (double *)std::malloc(sizeof(double) * k);
    if (!f->labels || !f->intra_arcs || !f->sum_deg_sq || !f->f1 || !f->f2) {
        hpmocd_front_free(f);
        return HPMOCD_ERR_NOMEM;
    }
    void *lab_dst = f->labels;
    if (stage) {
        stage->used = 0;
        if (void *q = stage->take(lab_bytes)) lab_dst = q;
    }
    bool ok = hipMemcpyAsync(f->intra_arcs, L.st.fr_A, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(f->sum_deg_sq, L.st.fr_S, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(f->f1, L.st.fr_f1, sizeof(double) * k, hipMemcpyDeviceToHost, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(f->f2, L.st.fr_f2, sizeof(double) * k, hipMemcpyDeviceToHost, s) == hipSuccess;
    if (lab_dst != f->labels) {  // into the caller's page-locked staging, then out of it
        ok = ok && hipMemcpyAsync(lab_dst, L.C, lab_bytes, hipMemcpyDeviceToHost, s) == hipSuccess;
        ok = ok && hipStreamSynchronize(s) == hipSuccess;
        if (ok) host_copy(f->labels, lab_dst, lab_bytes);
    } else {
        ok = ok && copy_to_host(f->labels, L.C, lab_bytes, s) == hipSuccess;
    }
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        hpmocd_front_free(f);
        return HPMOCD_ERR_HIP;
    }
    f->selected = ks[1];
    *out = f;
    return HPMOCD_OK;
}

int extract_fronts(const Pop *const *pops, int32_t count, hipStream_t s, hpmocd_front **outs)
{
    for (int32_t i = 0; i < count; ++i) outs[i] = nullptr;
    if (count <= 0) return HPMOCD_OK;
    // every population's front size and Alg. 3's choice (k_final), in one round trip; for
    // many populations into page-locked memory, since a copy into pageable memory returns
    // only once it is done
    int32_t *ks = nullptr;
    std::vector<int32_t> ks_pageable;
    if (count < 8 ||
        hipHostMalloc((void **)&ks, sizeof(int32_t) * 2 * (size_t)count, hipHostMallocDefault) != hipSuccess) {
        ks = nullptr;
        try {
            ks_pageable.assign(2 * (size_t)count, 0);
        } catch (...) {
            return HPMOCD_ERR_NOMEM;
        }
    }
    struct HostFree {  // drains s first: no copy into ks is left in flight, whatever return
        int32_t *p;
        hipStream_t s;
        ~HostFree()
        {
            (void)hipStreamSynchronize(s);
            if (p) (void)hipHostFree(p);
        }
    } ks_guard{ks, s};
    int32_t *kv = ks ? ks : ks_pageable.data();
    for (int32_t i = 0; i < count; ++i) {  // ks_guard drains s on an early return
        const RunLayout &L = pops[i]->L;
        HIP_TRY(hipMemcpyAsync(&kv[2 * i], L.st.fr_count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&kv[2 * i + 1], L.st.fr_sel, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    for (int32_t i = 0; i < count; ++i) {
        const int32_t k = kv[2 * i], sel = kv[2 * i + 1];
        if (k < 1 || k > pops[i]->c.pop || sel < 0 || sel >= k) return HPMOCD_ERR_HIP;
    }
    // each front's rows into its population's C plane (free after the last generation)
    for (int32_t i = 0; i < count; ++i) {
        const Pop &P = *pops[i];
        const RunLayout &L = P.L;
        HIP_TRY(launch_extract(P.G->n, P.c.ld, P.c.pop, L.pool[P.cur], L.q[P.cur], L.st.fr_id,
                               kv[2 * i], L.C, s));
    }
    auto fail = [&](int rc) {
        for (int32_t i = 0; i < count; ++i) {
            hpmocd_front_free(outs[i]);
            outs[i] = nullptr;
        }
        return rc;
    };
    std::vector<HostSeg> segs;
    try {
        segs.reserve(5 * (size_t)count);
    } catch (...) {
        return HPMOCD_ERR_NOMEM;
    }
    for (int32_t i = 0; i < count; ++i) {
        const Pop &P = *pops[i];
        const RunLayout &L = P.L;
        const int32_t k = kv[2 * i], n = P.G->n;
        hpmocd_front *f = (hpmocd_front *)std::calloc(1, sizeof(hpmocd_front));
        if (!f) return fail(HPMOCD_ERR_NOMEM);
        outs[i] = f;
        f->n_solutions = k;
        f->n_nodes = n;
        f->selected = kv[2 * i + 1];
        const size_t lab_bytes = sizeof(int32_t) * (size_t)k * n;
        f->labels = (int32_t *)alloc_labels(lab_bytes);
        f->intra_arcs = (int64_t *)std::malloc(sizeof(int64_t) * k);
        f->sum_deg_sq = (int64_t *)std::malloc(sizeof(int64_t) * k);
        f->f1 = (double *)std::malloc(sizeof(double) * k);
        f->f2 = (double *)std::malloc(sizeof(double) * k);
        if (!f->labels || !f->intra_arcs || !f->sum_deg_sq || !f->f1 || !f->f2) return fail(HPMOCD_ERR_NOMEM);
        segs.push_back({f->labels, L.C, lab_bytes});
        segs.push_back({f->intra_arcs, L.st.fr_A, sizeof(int64_t) * k});
        segs.push_back({f->sum_deg_sq, L.st.fr_S, sizeof(int64_t) * k});
        segs.push_back({f->f1, L.st.fr_f1, sizeof(double) * k});
        segs.push_back({f->f2, L.st.fr_f2, sizeof(double) * k});
    }
    if (copy_segments(segs.data(), segs.size(), s) != hipSuccess) return fail(HPMOCD_ERR_HIP);
    return HPMOCD_OK;
}

bool enqueue_front(const Pop &P, hipStream_t s, Pinned *stage, StagedFront *sf, hipError_t *err)
{
    const RunLayout &L = P.L;
    const int32_t n = P.G->n, pop = P.c.pop;
    const size_t lab = sizeof(int32_t) * (size_t)pop * n;
    const size_t need = 256 + (lab + 255) / 256 * 256 + 4 * ((8 * (size_t)pop + 255) / 256 * 256);
    *err = hipSuccess;
    if (!stage || stage->used + need > stage->size) return false;
    sf->ks = (int32_t *)stage->take(2 * sizeof(int32_t));
    sf->labels = (int32_t *)stage->take(lab);
    sf->A = (int64_t *)stage->take(8 * (size_t)pop);
    sf->S = (int64_t *)stage->take(8 * (size_t)pop);
    sf->f1 = (double *)stage->take(8 * (size_t)pop);
    sf->f2 = (double *)stage->take(8 * (size_t)pop);
    const hipMemcpyKind d2h = hipMemcpyDeviceToHost;
    hipError_t e = launch_extract(n, P.c.ld, pop, L.pool[P.cur], L.q[P.cur], L.st.fr_id, pop, L.C,
                                  s, L.st.fr_count);
    if (e == hipSuccess) e = hipMemcpyAsync(sf->ks, L.st.fr_count, sizeof(int32_t), d2h, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sf->ks + 1, L.st.fr_sel, sizeof(int32_t), d2h, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sf->labels, L.C, lab, d2h, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sf->A, L.st.fr_A, 8 * (size_t)pop, d2h, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sf->S, L.st.fr_S, 8 * (size_t)pop, d2h, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sf->f1, L.st.fr_f1, 8 * (size_t)pop, d2h, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sf->f2, L.st.fr_f2, 8 * (size_t)pop, d2h, s);
    *err = e;
    return true;
}

int front_from_staged(const Pop &P, const StagedFront &sf, hpmocd_front **out)
{
    const int32_t n = P.G->n, pop = P.c.pop;
    const int32_t k = sf.ks[0], sel = sf.ks[1];
    if (k < 1 || k > pop || sel < 0 || sel >= k) return HPMOCD_ERR_HIP;
    hpmocd_front *f = (hpmocd_front *)std::calloc(1, sizeof(hpmocd_front));
    if (!f) return HPMOCD_ERR_NOMEM;
    f->n_solutions = k;
    f->n_nodes = n;
    f->labels = (int32_t *)alloc_labels(sizeof(int32_t) * (size_t)k * n);
    f->intra_arcs = (int64_t *)std::malloc(sizeof(int64_t) * k);
    f->sum_deg_sq = (int64_t *)std::malloc(sizeof(int64_t) * k);
    f->f1 = (double *)std::malloc(sizeof(double) * k);
    f->f2 = (double *)std::malloc(sizeof(double) * k);
    if (!f->labels || !f->intra_arcs || !f->sum_deg_sq || !f->f1 || !f->f2) {
        hpmocd_front_free(f);
        return HPMOCD_ERR_NOMEM;
    }
    host_copy(f->labels, sf.labels, sizeof(int32_t) * (size_t)k * n);
    std::memcpy(f->intra_arcs, sf.A, sizeof(int64_t) * k);
    std::memcpy(f->sum_deg_sq, sf.S, sizeof(int64_t) * k);
    std::memcpy(f->f1, sf.f1, sizeof(double) * k);
    std::memcpy(f->f2, sf.f2, sizeof(double) * k);
    f->selected = sel;
    *out = f;
    return HPMOCD_OK;
}

// ---------------------------------------------------------------------------------------
// Batch: the populations, their workspace and the three item tables (init, parity 0, 1).
// ---------------------------------------------------------------------------------------
struct BatchLayout {
    std::vector<size_t> pop_off;  // byte offset of each population's region
    size_t meta_off[3] = {0, 0, 0};
    size_t bytes = 0;
};

static BatchLayout batch_layout(const hpmocd_graph *const *graphs, int32_t count,
                                const hpmocd_params *params, const Tuning &t, bool both)
{
    BatchLayout B;
    size_t off = 0;
    for (int32_t i = 0; i < count; ++i) {
        B.pop_off.push_back(off);
        off += align_up(carve_run(nullptr, graphs[i]->n, params[i].pop_size,
                                  params[i].parents_per_child, graphs[i]->max_deg,
                                  t, both)
                            .bytes);
    }
    for (int k = 0; k < 3; ++k) {
        B.meta_off[k] = off;
        off += meta_bytes(count);
    }
    B.bytes = off;
    return B;
}

static int check_batch(const hpmocd_graph *const *graphs, int32_t count,
                       const hpmocd_params *params)
{
    if (!graphs || !params || count < 1) return HPMOCD_ERR_ARG;
    for (int32_t i = 0; i < count; ++i) {
        if (!graphs[i]) return HPMOCD_ERR_ARG;
        int rc = check_params(&params[i]);
        if (rc) return rc;
        // one generation count and one ensemble size per batch (shared launches)
        if (params[i].generations != params[0].generations ||
            params[i].parents_per_child != params[0].parents_per_child)
            return HPMOCD_ERR_ARG;
    }
    return HPMOCD_OK;
}

int Batch::setup(const hpmocd_graph *const *graphs, int32_t count, const hpmocd_params *params,
                 void *ws, size_t ws_bytes, const Tuning &t, bool both, hipStream_t s)
{
    tuning = t;
    if (int rc = fork.init()) return rc;
    BatchLayout B = batch_layout(graphs, count, params, t, both);
    if (ws_bytes < B.bytes) return HPMOCD_ERR_WORKSPACE;
    int64_t total_nodes = 0;
    for (int32_t i = 0; i < count; ++i) total_nodes += graphs[i]->n;
    pops.assign(count, Pop{});
    for (int32_t i = 0; i < count; ++i)
        pops[i].setup(graphs[i], params[i], (char *)ws + B.pop_off[i], t, total_nodes, both);
    for (int w = 0; w < 3; ++w) {
        std::vector<Item> items;
        for (const Pop &P : pops) items.push_back(P.item(w == 0 ? ITEM_INIT : (w == 1 ? ITEM_PARITY0 : ITEM_PARITY1)));
        int rc = meta[w].upload(items, (char *)ws + B.meta_off[w], s);
        if (rc) return rc;
    }
    return HPMOCD_OK;
}

// Runs generations [first, last] of every population. Uses hipGraph replay of the
// two-generation parity cycle when allowed; otherwise launches kernels one by one.
int Batch::generations(int32_t first, int32_t last, hipStream_t s, bool use_graph,
                       std::vector<std::vector<EventPair>> *ev, hpmocd_trace_fn trace,
                       void *user, bool trace_labels)
{
    int32_t gen = first;
    if (use_graph && last - first + 1 >= 2 && !trace && !ev) {
        const int p0 = pops.empty() ? 0 : pops[0].cur;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e1 = launch_generation(meta[1 + p0], s, nullptr, &fork);
        hipError_t e2 = e1 == hipSuccess ? launch_generation(meta[1 + (1 - p0)], s, nullptr, &fork) : e1;
        hipError_t ec = hipStreamEndCapture(s, &graph);
        if (e1 != hipSuccess || e2 != hipSuccess || ec != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return HPMOCD_ERR_HIP;
        }
        hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return HPMOCD_ERR_HIP;
        const int32_t pairs = (last - first + 1) / 2;
        hipError_t el = hipSuccess;
        for (int32_t k = 0; k < pairs && el == hipSuccess; ++k) el = hipGraphLaunch(exec, s);
        (void)hipGraphExecDestroy(exec);
        if (el != hipSuccess) return HPMOCD_ERR_HIP;
        gen += 2 * pairs;
    }
    for (; gen <= last; ++gen) {
        const int par = pops.empty() ? 0 : pops[0].cur;
        const EventPair *evp = ev ? (*ev)[(size_t)(gen - 1)].data() : nullptr;
        HIP_TRY(launch_generation(meta[1 + par], s, evp, &fork));
        for (Pop &P : pops) P.cur = 1 - P.cur;
        if (trace) {
            int rc = emit_state(pops[0], gen, s, trace, user, trace_labels);
            if (rc) return rc;
        }
    }
    // after a graph replay every population has advanced an even number of generations,
    // so its parity is unchanged
    return HPMOCD_OK;
}

// Autotuner: coordinate descent over the launch-shape knobs, each candidate timed on one
// generation of this very batch (results discarded; every choice gives identical results,
// only the work decomposition changes).
static int autotune(const hpmocd_graph *const *graphs, int32_t count, const hpmocd_params *params,
                    void *ws, size_t ws_bytes, hipStream_t s, Tuning *best, double *probe_ms)
{
    std::vector<hpmocd_params> probe(params, params + count);
    for (auto &p : probe) p.generations = 1;
    EventSet evs;
    hipEvent_t a = evs.make(), b = evs.make();
    if (!a || !b) return HPMOCD_ERR_HIP;
    // The layout of the populations does not depend on the knobs (both histogram areas are
    // carved at their largest), so the initial populations are made once and every candidate
    // then times one generation on whatever the previous one left, at the buffer parity that
    // left; the state always holds valid labels and ids.
    // Knob values often give the same launch shapes (e.g. every crossover target that rounds
    // to 16 nodes per workgroup): a candidate whose shapes were timed already is not run again.
    bool initialised = false;
    int parity = 0;
    std::vector<std::pair<uint64_t, double>> seen;
    double spent = 0;  // GPU time of the candidates actually run
    auto time_it = [&](const Tuning &t, double *ms) -> int {
        Batch bt;
        int rc = bt.setup(graphs, count, probe.data(), ws, ws_bytes, t, true, s);
        if (rc) return rc;
        uint64_t sig = 1469598103934665603ull;  // FNV-1a over what the knobs change per population
        auto mix = [&](int64_t v) {
            for (int b = 0; b < 8; ++b) {
                sig ^= (uint64_t)(v >> (8 * b)) & 0xFFu;
                sig *= 1099511628211ull;
            }
        };
        for (const Pop &P : bt.pops) {
            mix(P.L.hp.enabled);
            mix(P.L.hp.rbits);
            mix(P.L.hp.nb);
            mix(P.fit_npw);
            mix(P.xo_nb);
            mix(P.c.mut_group);
        }
        for (const auto &x : seen)
            if (x.first == sig) {
                *ms = x.second;
                return HPMOCD_OK;
            }
        if (!initialised) {
            HIP_TRY(launch_init_seq(bt.meta[0], s, &bt.fork));
            initialised = true;
        }
        for (Pop &P : bt.pops) P.cur = parity;
        HIP_TRY(hipEventRecord(a, s));
        rc = bt.generations(1, 1, s, false, nullptr, nullptr, nullptr, false);
        if (rc) return rc;
        parity = bt.pops.empty() ? 0 : bt.pops[0].cur;
        HIP_TRY(hipEventRecord(b, s));
        HIP_TRY(hipEventSynchronize(b));
        *ms = elapsed(a, b);
        seen.emplace_back(sig, *ms);
        spent += *ms;
        return HPMOCD_OK;
    };
    Tuning cur = *best;
    double cur_ms = 0;
    int rc = time_it(cur, &cur_ms);
    if (rc) return rc;
    const int32_t fit_c[] = {2048, 8192, 16384, 65536};
    const int32_t xo_c[] = {512, 2048, 8192};
    const int32_t mut_c[] = {48, 96, 192};
    const int32_t hist_c[] = {16, 20, 24, 31};
    const int32_t narrow_c[] = {0, 1};
    for (int knob = 0; knob < 6; ++knob) {
        const int32_t *vals = knob == 0 ? fit_c : knob == 1 ? xo_c : knob == 2 ? mut_c
                              : knob == 3 ? hist_c : knob == 4 ? HIST_RBITS_CHOICES : narrow_c;
        const int nv = knob == 0 || knob == 3 ? 4 : (knob == 5 ? 2 : 3);
        for (int i = 0; i < nv; ++i) {
            Tuning t = cur;
            int32_t *field = knob == 0 ? &t.fit_target_waves : knob == 1 ? &t.xo_target_blocks
                             : knob == 2 ? &t.mut_target_items
                             : knob == 3 ? &t.hist_min_log2
                             : knob == 4 ? &t.hist_rbits : &t.hist_narrow;
            if (*field == vals[i]) continue;
            *field = vals[i];
            double ms = 0;
            if ((rc = time_it(t, &ms))) return rc;
            if (ms < cur_ms) {
                cur = t;
                cur_ms = ms;
            }
        }
    }
    *best = cur;
    if (probe_ms) *probe_ms = spent;
    return HPMOCD_OK;
}

// Runs started from several host threads take turns (whole runs are serialised per
// process): four threads each capturing, instantiating and replaying their own hipGraph at
// once crashed the process with a segmentation fault, and no cause was found in this
// library's code. Recursive: a trace callback may start a run of its own.
std::recursive_mutex &run_mutex()
{
    static std::recursive_mutex mu;
    return mu;
}

int run_batch(const hpmocd_graph *const *graphs, int32_t count, const hpmocd_params *params,
              void *ws, size_t ws_bytes, void *stream, int flags, hpmocd_profile *prof,
              hpmocd_trace_fn trace, void *user, hpmocd_front **outs)
{
    std::lock_guard<std::recursive_mutex> serial(run_mutex());
    int rc = check_batch(graphs, count, params);
    if (rc) return rc;
    if (!ws || !outs) return HPMOCD_ERR_ARG;
    if (trace && count != 1) return HPMOCD_ERR_ARG;
    for (int32_t i = 0; i < count; ++i)
        if ((rc = check_device(graphs[i]))) return rc;
    hipStream_t s = (hipStream_t)stream;
    DrainOnExit drain{s};
    const int32_t T = params[0].generations;
    const bool autotune_on = (flags & HPMOCD_AUTOTUNE) != 0;
    Tuning t = default_tuning(count);
    int64_t nodes = 0;
    for (int32_t i = 0; i < count; ++i) nodes += graphs[i]->n;
    t.mut_target_items = mut_target_for(t, nodes);  // explicit, so the profile reports it
    double probe_ms = 0;
    if (autotune_on && (rc = autotune(graphs, count, params, ws, ws_bytes, s, &t, &probe_ms)))
        return rc;
    Batch B;
    if ((rc = B.setup(graphs, count, params, ws, ws_bytes, t, autotune_on, s))) return rc;
    const bool time_kernels = (flags & HPMOCD_TIME_KERNELS) != 0 && prof;
    const bool trace_labels = (flags & HPMOCD_TRACE_NO_LABELS) == 0;
    const bool use_graph = !(flags & (HPMOCD_NO_GRAPH | HPMOCD_TIME_KERNELS)) && !trace &&
                           s != nullptr;

    EventSet evs;
    std::vector<std::vector<EventPair>> gen_events;
    if (time_kernels) {
        gen_events.assign((size_t)T, std::vector<EventPair>(6));
        for (auto &v : gen_events)
            for (auto &pr : v) {
                pr.a = evs.make();
                pr.b = evs.make();
                if (!pr.a || !pr.b) return HPMOCD_ERR_HIP;
            }
    }
    hipEvent_t e_start = nullptr, e_loop0 = nullptr, e_loop1 = nullptr, e_end = nullptr;
    hipEvent_t e_fit0 = nullptr, e_fit1 = nullptr;
    if (prof) {
        e_start = evs.make();
        e_loop0 = evs.make();
        e_loop1 = evs.make();
        e_end = evs.make();
        e_fit0 = evs.make();
        e_fit1 = evs.make();
        if (!e_start || !e_loop0 || !e_loop1 || !e_end || !e_fit0 || !e_fit1) return HPMOCD_ERR_HIP;
        HIP_TRY(hipEventRecord(e_start, s));
    }
    // initial populations (Alg. 1 phases 1-2)
    const Meta &mi = B.meta[0];
    HIP_TRY(mi.launch(K_CLEAR, s));
    HIP_TRY(mi.one(ONE_ZERO_ACC, s));
    HIP_TRY(mi.launch(K_INIT, s));
    if (prof) HIP_TRY(hipEventRecord(e_fit0, s));
    HIP_TRY(launch_fitness_kinds(mi, s, &B.fork));
    if (prof) HIP_TRY(hipEventRecord(e_fit1, s));
    HIP_TRY(mi.launch(K_CLEAR, s));
    HIP_TRY(mi.one(ONE_INIT_STATE, s));
    if (trace && (rc = emit_state(B.pops[0], 0, s, trace, user, trace_labels))) return rc;

    if (prof) HIP_TRY(hipEventRecord(e_loop0, s));
    if ((rc = B.generations(1, T, s, use_graph, time_kernels ? &gen_events : nullptr, trace, user,
                            trace_labels)))
        return rc;
    if (prof) HIP_TRY(hipEventRecord(e_loop1, s));

    // phase 4: first front of every population
    HIP_TRY(B.meta[1].one(ONE_FINAL, s));
    {
        std::vector<const Pop *> pp;
        try {
            for (const Pop &P : B.pops) pp.push_back(&P);
        } catch (...) {
            return HPMOCD_ERR_NOMEM;
        }
        if ((rc = extract_fronts(pp.data(), count, s, outs))) return rc;
    }
    if (prof) {
        HIP_TRY(hipEventRecord(e_end, s));
        HIP_TRY(hipEventSynchronize(e_end));
        double fit_ms = 0, sweep_ms = 0, var_ms = 0, sel_ms = 0, xo_ms = 0;
        for (auto &ev : gen_events) {
            sel_ms += elapsed(ev[0].a, ev[0].b) + elapsed(ev[4].a, ev[4].b);
            var_ms += elapsed(ev[1].a, ev[1].b);
            xo_ms += elapsed(ev[5].a, ev[5].b);
            fit_ms += elapsed(ev[2].a, ev[2].b);
            sweep_ms += elapsed(ev[3].a, ev[3].b);
        }
        int64_t inds = 0;
        for (const Pop &P : B.pops) inds += (int64_t)P.c.pop * ((int64_t)T + 1);
        prof->total_ms = elapsed(e_start, e_end);
        prof->loop_ms = elapsed(e_loop0, e_loop1);
        prof->fitness_ms = time_kernels ? fit_ms + elapsed(e_fit0, e_fit1) : 0.0;
        prof->sweep_ms = time_kernels ? sweep_ms : 0.0;
        prof->variation_ms = time_kernels ? var_ms : 0.0;
        prof->crossover_ms = time_kernels ? xo_ms : 0.0;
        prof->select_ms = time_kernels ? sel_ms : 0.0;
        prof->fitness_launches = (int64_t)T + 1;
        prof->individual_evals = inds;
        prof->tune_fit_target_waves = B.tuning.fit_target_waves;
        prof->tune_xo_target_blocks = B.tuning.xo_target_blocks;
        prof->tune_mut_target_items = B.tuning.mut_target_items;
        prof->tune_hist_min_log2 = B.tuning.hist_min_log2;
        prof->tune_hist_rbits = B.tuning.hist_rbits;
        prof->tune_hist_narrow = B.tuning.hist_narrow;
        prof->tune_probe_ms = probe_ms;
    }
    return HPMOCD_OK;
}

size_t batch_workspace(const hpmocd_graph *const *graphs, int32_t count,
                       const hpmocd_params *params, bool both)
{
    return batch_layout(graphs, count, params, default_tuning(count), both).bytes;
}

Tuning default_tuning(int32_t count)
{
    Tuning t;
    t.hist_narrow = count > 1 ? 0 : 1;
    return t;
}

}  // namespace hpm

using namespace hpm;

extern "C" {

void hpmocd_front_free(hpmocd_front *f)
{
    if (!f) return;
    free_labels(f->labels);
    std::free(f->intra_arcs);
    std::free(f->sum_deg_sq);
    std::free(f->f1);
    std::free(f->f2);
    std::free(f);
}

int hpmocd_workspace_size(const hpmocd_graph *g, const hpmocd_params *p, size_t *bytes)
{
    return c_guard([&]() -> int {
        if (!g || !bytes) return HPMOCD_ERR_ARG;
        int rc = check_params(p);
        if (rc) return rc;
        *bytes = batch_workspace(&g, 1, p, false);
        return HPMOCD_OK;
    });
}

int hpmocd_run_ex(const hpmocd_graph *G, const hpmocd_params *p, void *ws, size_t ws_bytes,
                  void *stream, int flags, hpmocd_profile *prof, hpmocd_trace_fn trace,
                  void *user, hpmocd_front **out)
{
    return c_guard([&]() -> int {
        if (!G || !out || !p) return HPMOCD_ERR_ARG;
        if (flags & HPMOCD_AUTOTUNE) return HPMOCD_ERR_ARG;  // batches only
        hpmocd_front *f = nullptr;
        int rc = run_batch(&G, 1, p, ws, ws_bytes, stream, flags, prof, trace, user, &f);
        if (rc == HPMOCD_OK) *out = f;
        return rc;
    });
}

int hpmocd_run(const hpmocd_graph *g, const hpmocd_params *p, void *ws, size_t ws_bytes,
               void *stream, hpmocd_front **out)
{
    return c_guard([&]() -> int {
        return hpmocd_run_ex(g, p, ws, ws_bytes, stream, 0, nullptr, nullptr, nullptr, out);
    });
}

int hpmocd_run_traced(const hpmocd_graph *g, const hpmocd_params *p, void *ws, size_t ws_bytes,
                      void *stream, hpmocd_trace_fn on_generation, void *user,
                      hpmocd_front **out)
{
    return c_guard([&]() -> int {
        if (!on_generation) return HPMOCD_ERR_ARG;
        return hpmocd_run_ex(g, p, ws, ws_bytes, stream, 0, nullptr, on_generation, user, out);
    });
}

int hpmocd_batch_workspace_size(const hpmocd_graph *const *graphs, int32_t count,
                                const hpmocd_params *params, int flags, size_t *bytes)
{
    return c_guard([&]() -> int {
        if (!bytes) return HPMOCD_ERR_ARG;
        int rc = check_batch(graphs, count, params);
        if (rc) return rc;
        *bytes = batch_workspace(graphs, count, params, (flags & HPMOCD_AUTOTUNE) != 0);
        return HPMOCD_OK;
    });
}

int hpmocd_run_batch(const hpmocd_graph *const *graphs, int32_t count,
                     const hpmocd_params *params, void *ws, size_t ws_bytes, void *stream,
                     int flags, hpmocd_profile *profile, hpmocd_front **outs)
{
    return c_guard([&]() -> int {
        return run_batch(graphs, count, params, ws, ws_bytes, stream, flags, profile, nullptr,
                         nullptr, outs);
    });
}

// ---------------------------------------------------------------------------------------
// checkpoint / resume
// ---------------------------------------------------------------------------------------
void hpmocd_snapshot_free(hpmocd_snapshot *sn)
{
    if (!sn) return;
    std::free(sn->labels);
    std::free(sn->A);
    std::free(sn->S);
    std::free(sn);
}

int hpmocd_run_to(const hpmocd_graph *G, const hpmocd_params *p, int32_t stop_gen, void *ws,
                  size_t ws_bytes, void *stream, hpmocd_snapshot **out)
{
    return c_guard([&]() -> int {
        if (!G || !p || !out || !ws) return HPMOCD_ERR_ARG;
        int rc = check_params(p);
        if (rc) return rc;
        if (stop_gen < 0 || stop_gen > p->generations) return HPMOCD_ERR_ARG;
        if ((rc = check_device(G))) return rc;
        std::lock_guard<std::recursive_mutex> serial(run_mutex());
        hipStream_t s = (hipStream_t)stream;
        DrainOnExit drain{s};
        Batch B;
        if ((rc = B.setup(&G, 1, p, ws, ws_bytes, Tuning{}, false, s))) return rc;
        HIP_TRY(launch_init_seq(B.meta[0], s, &B.fork));
        if ((rc = B.generations(1, stop_gen, s, s != nullptr, nullptr, nullptr, nullptr, false)))
            return rc;
        // members in selection order, gathered into row-major rows (C is free here)
        const Pop &P = B.pops[0];
        const int32_t n = G->n, pop = p->pop_size;
        HIP_TRY(launch_extract(n, P.c.ld, pop, P.L.pool[P.cur], P.L.q[P.cur], P.L.st.ps_id, pop,
                               P.L.C, s));
        hpmocd_snapshot *sn = (hpmocd_snapshot *)std::calloc(1, sizeof(hpmocd_snapshot));
        if (!sn) return HPMOCD_ERR_NOMEM;
        sn->g = stop_gen;
        sn->pop_size = pop;
        sn->n_nodes = n;
        sn->params = *p;
        sn->graph_hash = G->hash;
        sn->labels = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)pop * n);
        sn->A = (int64_t *)std::malloc(sizeof(int64_t) * pop);
        sn->S = (int64_t *)std::malloc(sizeof(int64_t) * pop);
        if (!sn->labels || !sn->A || !sn->S) {
            hpmocd_snapshot_free(sn);
            return HPMOCD_ERR_NOMEM;
        }
        const hipMemcpyKind d2h = hipMemcpyDeviceToHost;
        bool ok = copy_to_host(sn->labels, P.L.C, sizeof(int32_t) * (size_t)pop * n, s) == hipSuccess;
        ok = ok && hipMemcpyAsync(sn->A, P.L.st.ps_A, sizeof(int64_t) * pop, d2h, s) == hipSuccess;
        ok = ok && hipMemcpyAsync(sn->S, P.L.st.ps_S, sizeof(int64_t) * pop, d2h, s) == hipSuccess;
        ok = ok && hipStreamSynchronize(s) == hipSuccess;
        if (!ok) {
            hpmocd_snapshot_free(sn);
            return HPMOCD_ERR_HIP;
        }
        *out = sn;
        return HPMOCD_OK;
    });
}

int hpmocd_resume(const hpmocd_graph *G, const hpmocd_params *p, const hpmocd_snapshot *sn,
                  void *ws, size_t ws_bytes, void *stream, hpmocd_front **out)
{
    return c_guard([&]() -> int {
        if (!G || !p || !sn || !out || !ws || !sn->labels || !sn->A || !sn->S) return HPMOCD_ERR_ARG;
        int rc = check_params(p);
        if (rc) return rc;
        const int32_t n = G->n, pop = p->pop_size, T = p->generations;
        if (sn->n_nodes != n || sn->pop_size != pop || sn->g < 0 || sn->g > T) return HPMOCD_ERR_ARG;
        std::lock_guard<std::recursive_mutex> serial(run_mutex());
        // the snapshot belongs to this graph and these parameters (the generation count may grow)
        const hpmocd_params &q = sn->params;
        if (sn->graph_hash != G->hash || q.pop_size != pop || q.seed != p->seed ||
            q.crossover_p != p->crossover_p || q.mutation_p != p->mutation_p ||
            q.parents_per_child != p->parents_per_child)
            return HPMOCD_ERR_ARG;
        for (size_t i = 0; i < (size_t)pop * n; ++i)
            if (sn->labels[i] < 0 || sn->labels[i] >= n) return HPMOCD_ERR_RANGE;
        const int64_t m2 = G->m2;
        std::vector<int32_t> ids(pop);
        for (int32_t i = 0; i < pop; ++i) {
            if (sn->A[i] < 0 || sn->A[i] > m2 || sn->S[i] < 0 || sn->S[i] > m2 * m2)
                return HPMOCD_ERR_RANGE;
            ids[i] = i;  // member i lives in column i of the committed pool
        }
        if ((rc = check_device(G))) return rc;
        hipStream_t s = (hipStream_t)stream;
        DrainOnExit drain{s};
        Batch B;
        if ((rc = B.setup(&G, 1, p, ws, ws_bytes, Tuning{}, false, s))) return rc;
        Pop &P = B.pops[0];
        P.cur = 0;
        const DevState &st = P.L.st;
        const int32_t gen = sn->g + 1;  // the device generation counter after selection of g
        const hipMemcpyKind h2d = hipMemcpyHostToDevice;
        HIP_TRY(hipMemcpyAsync(P.L.C, sn->labels, sizeof(int32_t) * (size_t)pop * n, h2d, s));
        HIP_TRY(launch_transpose_in(P.L.C, n, pop, P.c.ld, P.L.pool[0], nullptr, s));  // checked above
        HIP_TRY(hipMemcpyAsync(st.ps_id, ids.data(), sizeof(int32_t) * pop, h2d, s));
        HIP_TRY(hipMemcpyAsync(st.ps_A, sn->A, sizeof(int64_t) * pop, h2d, s));
        HIP_TRY(hipMemcpyAsync(st.ps_S, sn->S, sizeof(int64_t) * pop, h2d, s));
        // f1, f2 from A, S by the kernels' own divisions (eq. objectives)
        HIP_TRY(launch_finalize(m2, pop, (const unsigned long long *)st.ps_A,
                                (const unsigned long long *)st.ps_S, st.ps_f1, st.ps_f2, s));
        HIP_TRY(hipMemcpyAsync(st.gen, &gen, sizeof(int32_t), h2d, s));
        // re-evaluate the members with the fitness kernels (eq. objectives) through a one-item
        // table in the init table's place (no initialisation runs on resume): the stored A and S
        // must be those of the stored labels
        {
            Item ev = P.item(ITEM_PARITY0);
            ev.lab = P.L.pool[0];
            Meta mv;
            if ((rc = mv.upload(&ev, 1, (void *)B.meta[0].items, s))) return rc;
            HIP_TRY(mv.launch(K_CLEAR, s));
            HIP_TRY(mv.one(ONE_ZERO_ACC, s));
            HIP_TRY(launch_fitness_kinds(mv, s, nullptr));
            std::vector<int64_t> A(pop), S(pop);
            HIP_TRY(copy_small({{A.data(), ev.fit_A, sizeof(int64_t) * pop},
                                {S.data(), ev.fit_S, sizeof(int64_t) * pop}}, s));
            for (int32_t i = 0; i < pop; ++i)
                if (A[i] != sn->A[i] || S[i] != sn->S[i]) return HPMOCD_ERR_ARG;
        }
        HIP_TRY(B.meta[1].launch(K_CLEAR, s));  // the plain histogram plane starts at zero
        if ((rc = B.generations(sn->g + 1, T, s, s != nullptr, nullptr, nullptr, nullptr, false)))
            return rc;
        HIP_TRY(B.meta[1 + P.cur].one(ONE_FINAL, s));
        rc = extract_front(P, s, out);  // synchronises s: the host arrays above outlive the copies
        return rc;
    });
}

}  // extern "C"

namespace hpm {

int eval_on(const hpmocd_graph *G, const int32_t *d_labels, int32_t n_ind, void *ws,
            hipStream_t s, int64_t *A, int64_t *S, double *f1, double *f2, double *kernel_ms)
{
    DrainOnExit drain{s};
    const int32_t ld = round16(n_ind);
    const size_t plane = (size_t)G->n * ld * 4;
    char *p = (char *)ws;
    int32_t *lab = (int32_t *)p;
    p += align_up(plane);
    Item it{};
    it.g = dev_graph(G);
    const Tuning t;
    it.hp = hist_plan(G->n, n_ind, G->max_deg, t.hist_min_log2, t.hist_rbits,
                      t.hist_narrow != 0, true);  // caller's labels: any range
    if (it.hp.enabled) {
        it.run = (uint32_t *)p;
        p += align_up(it.hp.entries * 4);
        it.off = (uint32_t *)p;
        p += align_up(it.hp.offsets * 4);
    } else {
        it.D = (int32_t *)p;
        it.D_bytes = plane;
        p += align_up(plane);
    }
    unsigned long long *dA = (unsigned long long *)p;
    p += align_up(8 * (size_t)n_ind);
    unsigned long long *dS = (unsigned long long *)p;
    p += align_up(8 * (size_t)n_ind);
    double *df1 = (double *)p;
    p += align_up(8 * (size_t)n_ind);
    double *df2 = (double *)p;
    p += align_up(8 * (size_t)n_ind);
    int32_t *d_bad = (int32_t *)p;
    p += align_up(sizeof(int32_t));
    it.lab = lab;
    it.fit_pop = n_ind;
    it.fit_ld = ld;
    it.fit_A = dA;
    it.fit_S = dS;
    it.fit_npw = (int32_t)std::max<int64_t>(1, std::min<int64_t>(64, G->n / t.fit_target_waves));
    it.xo_nb = 1;
    it.c.pop = n_ind;
    Meta m;
    int rc = m.upload(&it, 1, p, s);
    if (rc) return rc;
    // everything the kernels accumulate into starts at zero: the plain histogram plane, the
    // A / S accumulators and the label-range flag (the binned areas are overwritten whole)
    HIP_TRY(m.launch(K_CLEAR, s));
    HIP_TRY(m.one(ONE_ZERO_ACC, s));
    HIP_TRY(hipMemsetAsync(d_bad, 0, sizeof(int32_t), s));
    HIP_TRY(launch_transpose_in(d_labels, G->n, n_ind, ld, lab, d_bad, s));
    EventSet evs;
    hipEvent_t a = nullptr, b = nullptr;
    if (kernel_ms) {
        a = evs.make();
        b = evs.make();
        if (!a || !b) return HPMOCD_ERR_HIP;
        HIP_TRY(hipEventRecord(a, s));
    }
    HIP_TRY(launch_fitness_kinds(m, s, nullptr));
    if (kernel_ms) HIP_TRY(hipEventRecord(b, s));
    HIP_TRY(launch_finalize(G->m2, n_ind, dA, dS, df1, df2, s));
    // A and S are non-negative counts below 2^63: the unsigned accumulators' bits are the
    // int64 values, copied straight into the caller's arrays
    int32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad) return HPMOCD_ERR_RANGE;  // evaluated with those labels replaced by 0
    HIP_TRY(copy_small({{A, dA, sizeof(int64_t) * n_ind}, {S, dS, sizeof(int64_t) * n_ind},
                        {f1, df1, sizeof(double) * n_ind}, {f2, df2, sizeof(double) * n_ind}}, s));
    if (kernel_ms) *kernel_ms = elapsed(a, b);
    return HPMOCD_OK;
}

}  // namespace hpm

extern "C" {

// ---------------------------------------------------------------------------------------
// fitness alone (eval)
// ---------------------------------------------------------------------------------------
int hpmocd_eval_workspace_size(const hpmocd_graph *g, int32_t n_ind, size_t *bytes)
{
    return c_guard([&]() -> int {
        if (!g || !bytes || n_ind < 1) return HPMOCD_ERR_ARG;
        const int32_t ld = round16(n_ind);
        const Tuning t;
        const HistPlan hp = hist_plan(g->n, n_ind, g->max_deg, t.hist_min_log2, t.hist_rbits,
                                      t.hist_narrow != 0, true);
        size_t b = align_up((size_t)g->n * ld * 4);  // transposed labels
        b += hp.enabled ? align_up(hp.entries * 4) + align_up(hp.offsets * 4) : align_up((size_t)g->n * ld * 4);
        b += 2 * align_up(8 * (size_t)n_ind) + 2 * align_up(8 * (size_t)n_ind);
        b += align_up(sizeof(int32_t));  // out-of-range label flag
        b += meta_bytes(1);
        *bytes = b;
        return HPMOCD_OK;
    });
}

int hpmocd_eval(const hpmocd_graph *G, const int32_t *d_labels, int32_t n_ind, void *ws,
                size_t ws_bytes, void *stream, int64_t *A, int64_t *S, double *f1, double *f2,
                double *kernel_ms)
{
    return c_guard([&]() -> int {
        if (!G || !d_labels || n_ind < 1 || !ws || !A || !S || !f1 || !f2) return HPMOCD_ERR_ARG;
        int rc = check_device(G);
        if (rc) return rc;
        size_t need = 0;
        hpmocd_eval_workspace_size(G, n_ind, &need);
        if (ws_bytes < need) return HPMOCD_ERR_WORKSPACE;
        return eval_on(G, d_labels, n_ind, ws, (hipStream_t)stream, A, S, f1, f2, kernel_ms);
    });
}

}  // extern "C"
