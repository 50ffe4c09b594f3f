// Batch runner internals (host side): populations, their workspace layout, item tables and
// launch-shape tuning. Used by the run, eval and server translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <initializer_list>
#include <vector>

#include "host.hpp"

namespace hpm {

size_t align_up(size_t x);
int32_t round16(int32_t x);

// Launch-shape knobs. Every value gives identical results; they only change how the work is
// cut into workgroups (the autotuner picks them per batch).
struct Tuning {
    int32_t fit_target_waves = 2048;   // arc-scan waves wanted over the batch
    int32_t xo_target_blocks = 2048;   // crossover/init workgroups wanted over the batch
    int32_t mut_target_items = 0;      // mutations queued per wave group (small degrees);
                                       // 0: by size (96 from 2^18 nodes, else 48)
    int32_t hist_min_log2 = 20;        // binned histogram from 2^k (node, individual) pairs
    int32_t hist_rbits = 14;           // binned histogram tiles of up to 2^k labels
    int32_t hist_narrow = 1;           // small graphs: narrower tiles, smaller chunks
};

// Default shapes for a batch of `count` populations. A lone small graph needs narrower
// histogram tiles and smaller chunks to occupy the device; in a batch the populations fill it
// together, and the extra workgroups and offsets only cost.
Tuning default_tuning(int32_t count);
// the mutation queue target a tuning resolves to for a launch over `nodes` nodes
int32_t mut_target_for(const Tuning &t, int64_t nodes);

// tile sizes (log2 labels per tile) the autotuner tries for the binned histogram
constexpr int32_t HIST_RBITS_CHOICES[3] = {12, 13, 14};

struct RunLayout {
    int32_t ld = 0;
    size_t plane = 0;  // bytes of one node-major [n][ld] int32 plane
    int32_t *pool[2] = {nullptr, nullptr};
    int32_t *q[2] = {nullptr, nullptr};
    int32_t *C = nullptr;
    int32_t *D = nullptr;                     // plain histogram plane
    HistPlan hp;
    uint32_t *run = nullptr, *off = nullptr;  // binned histogram areas
    DevState st{};
    size_t bytes = 0;
};

// both_histograms: room for the plain plane and for the binned areas of every tile size the
// autotuner may try
RunLayout carve_run(void *ws, int32_t n, int32_t pop, int32_t es, int32_t max_deg,
                    const Tuning &t, bool both_histograms);
GaConst ga_const(const hpmocd_params *p, int32_t ld, int32_t mut_target);

enum ItemWhich { ITEM_INIT = 0, ITEM_PARITY0, ITEM_PARITY1 };

// One population on one graph.
struct Pop {
    const hpmocd_graph *G = nullptr;
    hpmocd_params p{};
    RunLayout L;
    GaConst c{};
    DevGraph dg{};
    int32_t fit_npw = 1, xo_nb = 1;
    int cur = 0;  // buffer parity: pool[cur] / q[cur] hold the current population
    void setup(const hpmocd_graph *graph, const hpmocd_params &params, void *ws, const Tuning &t,
               int64_t batch_nodes, bool both_histograms);
    // launch shapes of this population's items for a batch of batch_nodes nodes in total
    void shape(const Tuning &t, int64_t batch_nodes);
    Item item(int which) const;
};

// Device tables of one set of items: the items and, per launch kind, the block offsets.
// upload() copies them on the given stream (never the null stream, which would synchronise
// with, and break, a hipGraph capture in another thread); the host copies stay in the Meta,
// so it must outlive the copies (the stream is synchronised before a Meta goes away).
struct Meta {
    std::vector<Item> h_items;
    std::vector<int32_t> h_starts;
    Item h_item1{};                       // staging of a one-item table (no host allocation)
    int32_t h_starts1[2 * N_KINDS] = {};
    Item *items = nullptr;
    int32_t *starts = nullptr;
    int32_t count = 0;
    int32_t totals[N_KINDS] = {};
    size_t lds[N_KINDS] = {};
    int32_t aux[N_KINDS] = {};
    Span span(Kind k) const { return Span{items, starts + (size_t)k * (count + 1), count}; }
    // stage: optional page-locked staging for the two copies
    int upload(const Item *host_items, int32_t n_items, void *region, hipStream_t s,
               Pinned *stage = nullptr);
    int upload(const std::vector<Item> &host_items, void *region, hipStream_t s,
               Pinned *stage = nullptr)
    {
        return upload(host_items.data(), (int32_t)host_items.size(), region, s, stage);
    }
    hipError_t launch(Kind k, hipStream_t s) const;
    hipError_t one(OneKernel which, hipStream_t s) const;
};
size_t meta_bytes(int32_t count);

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
};
struct EventSet {
    std::vector<hipEvent_t> all;
    ~EventSet();
    hipEvent_t make();
};
float elapsed(hipEvent_t a, hipEvent_t b);

// Two side streams and their events: the mutation classes touch disjoint nodes, so they run
// as parallel branches of the generation (bandwidth-bound per-lane classes beside
// latency-bound per-wave classes); inside a hipGraph capture they become parallel nodes.
// Streams at the default priority.
struct Fork {
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
    int init();
    Fork() = default;
    Fork(const Fork &) = delete;
    Fork &operator=(const Fork &) = delete;
    ~Fork();
};

hipError_t launch_fitness_kinds(const Meta &m, hipStream_t s, const Fork *fk);
hipError_t launch_init_seq(const Meta &m, hipStream_t s, const Fork *fk);
// fk == nullptr: every kernel on s, one after another
hipError_t launch_generation(const Meta &m, hipStream_t s, const EventPair *ev, const Fork *fk);
int emit_state(const Pop &P, int32_t gen, hipStream_t s, hpmocd_trace_fn fn, void *user,
               bool with_labels);
// stage: optional page-locked staging for the labels' device-to-host copy (reset by the
// call, which synchronises s)
int extract_front(const Pop &P, hipStream_t s, hpmocd_front **out, Pinned *stage = nullptr);
// Fronts of several populations after their final ranking (k_final has run), one stream
// drain for all of them; on error no front is returned.
int extract_fronts(const Pop *const *pops, int32_t count, hipStream_t s, hpmocd_front **outs);
// device-to-host copies: bytes from src (device) to dst (host); returns with all complete
struct HostSeg {
    void *dst;
    const void *src;
    size_t bytes;
};
hipError_t copy_segments(const HostSeg *segs, size_t count, hipStream_t s);
hipError_t copy_to_host(void *dst, const void *src, size_t bytes, hipStream_t s);
// small copies issued together; drains s whatever happens (also on an error)
hipError_t copy_small(std::initializer_list<HostSeg> segs, hipStream_t s);
// host buffers of fronts' labels (hpmocd_front_free releases them with free_labels)
void *alloc_labels(size_t bytes);
void free_labels(void *p);
// memcpy of a large host buffer split over a few threads (one thread for small ones)
void host_copy(void *dst, const void *src, size_t bytes);

// The front of a ranked population without host synchronisation: every copy is enqueued on
// s into page-locked host memory taken from `stage` (all N_p candidate rows, the device
// count deciding how many are filled), so nothing waits on the host in the middle of the
// stream. front_from_staged builds the front once s has passed that point. Returns false
// (nothing enqueued) when the staging region lacks room.
struct StagedFront {
    int32_t *ks = nullptr;       // front size, Alg. 3's choice
    int32_t *labels = nullptr;   // N_p x n
    int64_t *A = nullptr, *S = nullptr;
    double *f1 = nullptr, *f2 = nullptr;
};
bool enqueue_front(const Pop &P, hipStream_t s, Pinned *stage, StagedFront *sf, hipError_t *err);
int front_from_staged(const Pop &P, const StagedFront &sf, hpmocd_front **out);

// Fitness of n_ind device label rows with the eval workspace at ws (hpmocd_eval_workspace_size
// bytes, contents on entry irrelevant); results to host arrays. No device or host allocation
// unless kernel_ms is requested (its events).
int eval_on(const hpmocd_graph *G, const int32_t *d_labels, int32_t n_ind, void *ws,
            hipStream_t s, int64_t *A, int64_t *S, double *f1, double *f2, double *kernel_ms);

// A whole batched run (init, T generations, fronts); a single run is a batch of one.
int run_batch(const hpmocd_graph *const *graphs, int32_t count, const hpmocd_params *params,
              void *ws, size_t ws_bytes, void *stream, int flags, hpmocd_profile *prof,
              hpmocd_trace_fn trace, void *user, hpmocd_front **outs);
size_t batch_workspace(const hpmocd_graph *const *graphs, int32_t count,
                       const hpmocd_params *params, bool both);

struct Batch {
    std::vector<Pop> pops;
    Meta meta[3];  // init, parity 0, parity 1
    Tuning tuning;
    Fork fork;
    int setup(const hpmocd_graph *const *graphs, int32_t count, const hpmocd_params *params,
              void *ws, size_t ws_bytes, const Tuning &t, bool both, hipStream_t s);
    int generations(int32_t first, int32_t last, hipStream_t s, bool use_graph,
                    std::vector<std::vector<EventPair>> *ev, hpmocd_trace_fn trace, void *user,
                    bool trace_labels);
};

}  // namespace hpm
