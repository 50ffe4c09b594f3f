/*
 * hpmocd.h - C ABI of the MI355X (gfx950) implementation of the HP-MOCD community search
 * (arXiv 2506.01752): an NSGA-II over node-label partitions of an undirected, unweighted
 * graph that minimises the two objectives of section 4.1 (eq. "objectives").
 *
 * Conventions (every entry point):
 *  - Status is an int: HPMOCD_OK (0) or a negative HPMOCD_ERR_* code; hpmocd_strerror()
 *    names it. No C++ exception crosses this boundary. Output arguments are written only
 *    on success.
 *  - Host inputs are read during the call and copied; the caller keeps ownership.
 *  - Device workspace and the HIP stream (a hipStream_t passed as void*, NULL = the null
 *    stream) belong to the caller; the library launches its kernels on that stream and
 *    synchronises it before returning results to the host.
 *  - Objects returned through an out-pointer (graphs, fronts) belong to the library until
 *    released with their *_destroy / *_free function.
 *  - Results are deterministic: a run is a pure function of (graph, params).
 */
#ifndef HPMOCD_H
#define HPMOCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HPMOCD_OK 0
#define HPMOCD_ERR_ARG -1        /* null pointer or parameter out of range */
#define HPMOCD_ERR_CSR_ASYM -2   /* arc (u,v) present without (v,u) */
#define HPMOCD_ERR_SELF_LOOP -3  /* arc (v,v); section 2.1 excludes self-loops */
#define HPMOCD_ERR_DUP_EDGE -4   /* repeated arc; the graph is simple (section 2.1) */
#define HPMOCD_ERR_RANGE -5      /* row_ptr not monotone from 0, or a column or label outside [0,n) */
#define HPMOCD_ERR_EMPTY -6      /* no edge: f1 = 0/0 is undefined */
#define HPMOCD_ERR_TOO_LARGE -7  /* (2m)^2 > 2^53: f2's denominator would not be exact */
#define HPMOCD_ERR_WORKSPACE -8  /* workspace smaller than the size the library asked for */
#define HPMOCD_ERR_HIP -9        /* a HIP runtime call failed */
#define HPMOCD_ERR_BUDGET -10    /* request does not fit the device-memory budget */
#define HPMOCD_ERR_NOMEM -11     /* host allocation failed */
#define HPMOCD_ERR_CANCELLED -12 /* server request cancelled (or the server shut down first) */
#define HPMOCD_ERR_TIMEOUT -13   /* server wait timed out; the request is still pending */
#define HPMOCD_ERR_SCRATCH -14   /* problem larger than hpmocd_eval_noalloc's fixed scratch */

/* Largest population: the selection kernels rank 2 * pop_size points in one workgroup. */
#define HPMOCD_MAX_POP 512
/* Largest ensemble (parents per child, E_S of Alg. 1). */
#define HPMOCD_MAX_PARENTS 8

/* Graph G = (V, E) of section 2.1: simple, undirected, unweighted. Opaque; device resident. */
typedef struct hpmocd_graph hpmocd_graph;

/* Parameters of Alg. 1: HP-MOCD(G, N_p, T, C_P, M_P, E_S) plus the seed of the counter-based
 * random stream (Philox4x32-10 keyed by the seed, counter = (node or slot, individual,
 * generation, purpose)). */
typedef struct {
    int32_t pop_size;          /* N_p, 1 .. HPMOCD_MAX_POP */
    int32_t generations;       /* T >= 0 */
    double crossover_p;        /* C_P in [0,1]: majority-vote crossover happens w.p. C_P (Alg. 2) */
    double mutation_p;         /* M_P in [0,1]: per-node neighbour-plurality mutation (sec. 4.3.2) */
    int32_t parents_per_child; /* E_S, 1 .. HPMOCD_MAX_PARENTS (the paper uses 4) */
    uint64_t seed;
} hpmocd_params;

/* First front F_1 of the final population (Alg. 1, phase 4), host memory owned by the
 * library. Rows are in crowded-comparison order (rank, then crowding distance descending,
 * then position); identical partitions are kept. Labels are node ids in [0, n): node v's
 * community is named by the id of some node. */
typedef struct {
    int32_t n_solutions;       /* k = |F_1| >= 1 */
    int32_t n_nodes;           /* n */
    int32_t *labels;           /* k x n, row-major */
    int64_t *intra_arcs;       /* A = 2 sum_c |E(c)| per solution */
    int64_t *sum_deg_sq;       /* S = sum_c (sum_{v in c} deg v)^2 per solution */
    double *f1;                /* (2m - A) / 2m, one binary64 division (eq. objectives) */
    double *f2;                /* S / (2m)^2, one binary64 division */
    int32_t selected;          /* Alg. 3: first index maximising (1 - f1) - f2 */
} hpmocd_front;

/* Per-generation observables handed to a trace callback (host copies, valid during the
 * callback only). At g = 0 they describe the initial population; at g >= 1 the population
 * after environmental selection of generation g, in selection order. rank/crowd are those
 * computed at the start of generation g on P^(g-1) (NULL at g = 0), in that step's order. */
typedef struct {
    int32_t g, pop_size, n_nodes;
    const int32_t *labels;     /* pop_size x n, row-major */
    const int64_t *A, *S;
    const double *f1, *f2;
    const int32_t *rank;
    const double *crowd;
} hpmocd_state_view;

typedef void (*hpmocd_trace_fn)(const hpmocd_state_view *state, void *user);

/* Stream-ordered timings of a run (milliseconds of device time, from HIP events recorded on
 * the caller's stream). Kernel-group times are filled only with HPMOCD_TIME_KERNELS. */
typedef struct {
    double total_ms;           /* init through front extraction */
    double loop_ms;            /* generations 1..T */
    double fitness_ms;         /* edge-scan fitness kernels (all launches) */
    double sweep_ms;           /* clearing the community-degree histogram after each scan */
    double variation_ms;       /* crossover + mutation kernels */
    double select_ms;          /* ranking / crowding / selection kernels */
    int64_t fitness_launches;  /* number of edge-scan launches */
    int64_t individual_evals;  /* N_p (T + 1), summed over a batch */
    int32_t tune_fit_target_waves;  /* launch shapes used (autotuned with HPMOCD_AUTOTUNE) */
    int32_t tune_xo_target_blocks;
    int32_t tune_mut_target_items;
    int32_t tune_hist_min_log2;
    int32_t tune_hist_rbits;
    int32_t tune_hist_narrow;  /* 1: narrower histogram tiles and chunks on small graphs */
    double tune_probe_ms;      /* device time spent probing shapes (0 without autotuning) */
    double crossover_ms;       /* the crossover kernels' part of variation_ms */
} hpmocd_profile;

#define HPMOCD_NO_GRAPH 1      /* launch each kernel (no hipGraph replay of the loop) */
#define HPMOCD_TIME_KERNELS 2  /* record events around every kernel group (implies NO_GRAPH) */
#define HPMOCD_TRACE_NO_LABELS 4 /* trace callback gets labels = NULL (objectives only) */
#define HPMOCD_AUTOTUNE 8      /* batches: time candidate launch shapes on the batch first */

/* Builds the device graph from a symmetric CSR (row_ptr[n+1], col[row_ptr[n]]).
 * Validates it (codes above; section 2.1 requires a simple undirected graph), sorts every
 * adjacency list ascending, and copies it to the current HIP device (synchronously).
 * n >= 1; isolated nodes are allowed. */
int hpmocd_graph_create(int32_t n, const int32_t *row_ptr, const int32_t *col,
                        hpmocd_graph **out);
void hpmocd_graph_destroy(hpmocd_graph *g);
/* n, number of arcs (2m) and the largest degree. Any out-pointer may be NULL. */
int hpmocd_graph_info(const hpmocd_graph *g, int32_t *n, int64_t *arcs, int32_t *max_deg);
/* 64-bit fingerprint of the graph (FNV-1a over n and the sorted CSR): equal graphs, given in
 * any adjacency order, have equal fingerprints. */
int hpmocd_graph_hash(const hpmocd_graph *g, uint64_t *hash);

/* Bytes of device workspace hpmocd_run needs for these parameters (256-byte aligned). */
int hpmocd_workspace_size(const hpmocd_graph *g, const hpmocd_params *p, size_t *bytes);

/* Alg. 1 end to end on the device: initialisation, T generations of tournament ->
 * crossover (Alg. 2) -> mutation (sec. 4.3.2) -> evaluation (eq. objectives) ->
 * environmental selection, then the first front and the Alg. 3 choice. d_workspace must be
 * device memory of at least hpmocd_workspace_size bytes; its contents on entry do not
 * matter. The front is returned in *out (free with hpmocd_front_free). Runs called from
 * several host threads at once take turns: the library runs one at a time per process (as
 * are hpmocd_run_batch, hpmocd_run_to and hpmocd_resume); many graphs at once is what
 * hpmocd_run_batch and the server are for. */
int hpmocd_run(const hpmocd_graph *g, const hpmocd_params *p, void *d_workspace,
               size_t ws_bytes, void *stream, hpmocd_front **out);

/* hpmocd_run with options: flags (HPMOCD_NO_GRAPH, HPMOCD_TIME_KERNELS), an optional profile
 * to fill, and an optional per-generation trace callback (forces NO_GRAPH and copies the
 * population to the host every generation: tests only). Results equal hpmocd_run's. */
int hpmocd_run_ex(const hpmocd_graph *g, const hpmocd_params *p, void *d_workspace,
                  size_t ws_bytes, void *stream, int flags, hpmocd_profile *profile,
                  hpmocd_trace_fn trace, void *user, hpmocd_front **out);

/* hpmocd_run with a per-generation trace (tests only): on_generation receives the initial
 * population (g = 0) and the population after every generation's environmental selection,
 * copied to the host (kernels launched one by one, a device-to-host copy per generation).
 * The front equals hpmocd_run's. Same as hpmocd_run_ex with flags 0 and no profile. */
int hpmocd_run_traced(const hpmocd_graph *g, const hpmocd_params *p, void *d_workspace,
                      size_t ws_bytes, void *stream, hpmocd_trace_fn on_generation, void *user,
                      hpmocd_front **out);

void hpmocd_front_free(hpmocd_front *f);

/* Batched form: `count` independent runs of Alg. 1, each on its own graph with its own
 * population and parameters (params[i]; all with the same generations and
 * parents_per_child), advanced together: every kernel launch covers all of the batch's
 * populations, and the generation loop is replayed from one hipGraph. With HPMOCD_AUTOTUNE
 * the launch shapes (arc-scan waves, crossover workgroups, mutation queue length, histogram
 * choice) are first timed on two generations of this batch and the fastest kept; results do
 * not depend on the shapes. Each run's front equals its hpmocd_run front bit for bit.
 * outs[count] receives one front per run (free each with hpmocd_front_free). The workspace
 * size depends on the flags (autotuning needs room for both histogram variants). */
int hpmocd_batch_workspace_size(const hpmocd_graph *const *graphs, int32_t count,
                                const hpmocd_params *params, int flags, size_t *bytes);
int hpmocd_run_batch(const hpmocd_graph *const *graphs, int32_t count,
                     const hpmocd_params *params, void *d_workspace, size_t ws_bytes,
                     void *stream, int flags, hpmocd_profile *profile, hpmocd_front **outs);

/* Checkpoint / resume. A snapshot is the population of a run after environmental selection
 * of generation g (g = 0: the initial population) in selection order, which is all a run
 * carries from one generation to the next: the random draws are a function of (seed, g,
 * individual, node) and need no saved state. Host memory owned by the library. */
typedef struct {
    int32_t g;            /* generations completed */
    int32_t pop_size, n_nodes;
    int32_t *labels;      /* pop_size x n_nodes, row-major, in selection order */
    int64_t *A, *S;       /* objectives' integer numerators of each member */
    hpmocd_params params; /* the run's parameters (generations may differ on resume) */
    uint64_t graph_hash;  /* fingerprint of the graph (hpmocd_graph_hash) */
} hpmocd_snapshot;

/* Runs initialisation and generations 1..stop_gen (0 <= stop_gen <= p->generations) and
 * returns the snapshot in *out instead of a front. Workspace as for hpmocd_run. */
int hpmocd_run_to(const hpmocd_graph *g, const hpmocd_params *p, int32_t stop_gen,
                  void *d_workspace, size_t ws_bytes, void *stream, hpmocd_snapshot **out);
/* Continues a run from a snapshot taken with the same graph and parameters: generations
 * snap->g + 1 .. p->generations, then the front. The result equals the uninterrupted
 * hpmocd_run bit for bit. Validation: sizes, g <= T, labels in [0, n), the graph's
 * fingerprint and every parameter but the generation count equal to the snapshot's
 * (HPMOCD_ERR_ARG otherwise) before any device work; then the fitness kernels re-evaluate
 * the snapshot's labels, and A or S differing from the stored values gives HPMOCD_ERR_ARG
 * (the objectives would not belong to the labels). */
int hpmocd_resume(const hpmocd_graph *g, const hpmocd_params *p, const hpmocd_snapshot *snap,
                  void *d_workspace, size_t ws_bytes, void *stream, hpmocd_front **out);
void hpmocd_snapshot_free(hpmocd_snapshot *s);

/* Fitness alone (eq. objectives) for n_ind partitions given as device memory, row-major
 * n_ind x n int32 labels in [0, n). Writes A, S, f1, f2 (host arrays of n_ind). A label
 * outside [0, n) gives HPMOCD_ERR_RANGE (found while the labels are read; the outputs are then
 * not written). */
int hpmocd_eval_workspace_size(const hpmocd_graph *g, int32_t n_ind, size_t *bytes);
int hpmocd_eval(const hpmocd_graph *g, const int32_t *d_labels, int32_t n_ind,
                void *d_workspace, size_t ws_bytes, void *stream, int64_t *A, int64_t *S,
                double *f1, double *f2, double *kernel_ms);

/* hpmocd_eval for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same kernels and
 * results, bit for bit, with the workspace taken from a fixed device array of
 * HPMOCD_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on until the
 * process ends, instead of a caller workspace. The call allocates no device memory (no
 * hipMalloc, no hipFree, no allocating library routine). d_labels: device memory, row-major
 * n_ind x n int32 labels in [0, n), on the graph's device, which must be current. A, S, f1,
 * f2: host arrays of n_ind, written only on success. Errors: HPMOCD_ERR_ARG (null pointer,
 * n_ind < 1, another device current), HPMOCD_ERR_SCRATCH when hpmocd_eval_workspace_size
 * (g, n_ind) exceeds HPMOCD_NOALLOC_SCRATCH_BYTES (e.g. 40,000 nodes x 100 partitions fits,
 * 1,000,000 x 100 does not), HPMOCD_ERR_RANGE for a label outside [0, n), HPMOCD_ERR_HIP.
 * Every call on one device shares that device's array (each call clears what it
 * accumulates into): calls that overlap on one device, from several host threads or on
 * several streams, race and must be serialised by the caller. */
#define HPMOCD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hpmocd_eval_noalloc(const hpmocd_graph *g, const int32_t *d_labels, int32_t n_ind,
                        void *stream, int64_t *A, int64_t *S, double *f1, double *f2);

/* Served form: a community-detection service over one device. Requests (a CSR graph plus
 * Alg. 1 parameters) are submitted from any host thread and return at once with a ticket;
 * a scheduler thread owned by the server admits them in arrival order while two limits
 * hold: at most max_active resident requests, and their device bytes (graph + populations +
 * histogram + state, reported by submit) within hbm_budget, all carved from one device arena
 * the caller provides. Continuous batching: every scheduler step initialises the requests
 * just admitted and advances every resident request by one generation in shared launches
 * (requests at different generations, on different graphs, in the same kernels); a request
 * that has run its T generations is ranked (Alg. 1 phase 4), its front copied to the host
 * and its memory released, so requests that arrived meanwhile take its place at the next
 * step. Populations stay on the device for the whole run. A request's front equals its
 * hpmocd_run front bit for bit, whatever else shares the device.
 *
 * The arena must hold hpmocd_server_arena_overhead(max_active) bytes of tables plus the
 * budget; it and the stream belong to the caller and must outlive the server. All requests
 * of a server share parents_per_child (one crossover kernel shape per step). */
typedef struct hpmocd_server hpmocd_server;

#define HPMOCD_SERVER_FIFO 1  /* baseline: one request at a time, each run as hpmocd_run */
#define HPMOCD_SERVER_MAX_ACTIVE 4096

typedef struct {
    size_t hbm_budget;          /* device bytes resident requests may hold together */
    int32_t max_active;         /* 1 .. HPMOCD_SERVER_MAX_ACTIVE */
    int32_t parents_per_child;  /* E_S of every request */
    int32_t flags;              /* HPMOCD_SERVER_FIFO or 0 */
    size_t host_stage_bytes;    /* page-locked host staging per in-flight step (a third for
                                 * graph and table uploads, two thirds for fronts; copies that
                                 * do not fit go from or to pageable memory); 0 = 384 MB */
} hpmocd_server_config;

/* Life of one request, seconds on the server's monotonic clock (0 = server creation). */
typedef struct {
    double submit_s, admit_s, done_s;  /* done = front on the host */
    int64_t device_bytes;              /* bytes it held while resident */
    int32_t steps;                     /* scheduler steps it was resident for */
    int32_t max_mix;                   /* most requests resident together during its run */
} hpmocd_request_info;

typedef struct {
    int64_t steps, admitted, completed, cancelled;
    int32_t peak_active;
    int64_t peak_bytes;
    double busy_s;                     /* scheduler time spent in steps (host clock) */
} hpmocd_server_stats;

#define HPMOCD_REQ_QUEUED 0
#define HPMOCD_REQ_RUNNING 1
#define HPMOCD_REQ_DONE 2

size_t hpmocd_server_arena_overhead(int32_t max_active);
/* Starts the scheduler thread on the calling thread's current device. d_arena: device memory
 * of arena_bytes >= overhead + hbm_budget. */
int hpmocd_server_create(const hpmocd_server_config *cfg, void *d_arena, size_t arena_bytes,
                         void *stream, hpmocd_server **out);
/* Validates and copies the graph (as hpmocd_graph_create) and queues the request.
 * HPMOCD_ERR_BUDGET if it could never fit the budget. *ticket identifies it; *device_bytes
 * (may be NULL) receives the bytes it will hold. */
int hpmocd_server_submit(hpmocd_server *s, int32_t n, const int32_t *row_ptr, const int32_t *col,
                         const hpmocd_params *p, int64_t *ticket, size_t *device_bytes);
/* *state = HPMOCD_REQ_QUEUED / RUNNING / DONE. */
int hpmocd_server_poll(hpmocd_server *s, int64_t ticket, int32_t *state);
/* Blocks until the request is done or timeout_s passes (< 0: no limit). On completion
 * returns the request's status and releases the ticket; on HPMOCD_OK *out receives the front
 * (free with hpmocd_front_free) and *info (may be NULL) its timings. Several threads may wait
 * on one ticket: the first to see it done consumes it, the others return HPMOCD_ERR_ARG, as
 * does any later call with that ticket. */
int hpmocd_server_wait(hpmocd_server *s, int64_t ticket, double timeout_s, hpmocd_front **out,
                       hpmocd_request_info *info);
/* A queued request is dropped at once, a resident one at the next step; its wait returns
 * HPMOCD_ERR_CANCELLED. */
int hpmocd_server_cancel(hpmocd_server *s, int64_t ticket);
int hpmocd_server_stats_get(hpmocd_server *s, hpmocd_server_stats *out);
/* Stops the scheduler after its current step; requests not done are cancelled and their
 * tickets released. No other call on s may be in progress or follow. */
void hpmocd_server_destroy(hpmocd_server *s);

const char *hpmocd_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* HPMOCD_H */
