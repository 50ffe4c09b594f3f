// Internal declarations shared by the host driver and the kernel launchers (not part of the
// C ABI).
//
// Device data layout:
//  * graph: symmetric CSR (row_ptr[n+1], col[2m], int32), neighbour lists ascending;
//  * populations are NODE-MAJOR: the label of individual j at node v lives at
//    base[v * ld + j], ld = pop_size rounded up to 16 (64-byte rows). One CSR arc (v,u)
//    then needs the single contiguous row base[u * ld .. u * ld + pop) for every individual
//    at once, so the CSR is streamed once per generation instead of once per individual.
//  * community-degree histograms D are node-major the same way: D[c * ld + j].
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hpmocd.h"

namespace hpm {

constexpr int HPMOCD_MAX_PARENTS_DEV = HPMOCD_MAX_PARENTS;
constexpr int HPMOCD_MAX_POP_DEV = HPMOCD_MAX_POP;

// Mutation work classes by degree (upper bounds). Degrees 1..32: one (node, offspring) item
// per lane, neighbour labels sorted in registers. Degrees 33..512: one item per wave, the
// labels spread 1, 2, 4 or 8 per lane and sorted across the wave. Higher degrees: one item
// per wave with an LDS sort (up to LARGE_SORT_CAP neighbours) or, above that, an exact scan.
constexpr int N_DEG_CLASSES = 8;
constexpr int DEG_CLASS_MAX[N_DEG_CLASSES] = {16, 32, 64, 128, 256, 512, 1024, 2048};
constexpr int SMALL_DEG_MAX = 2048;
constexpr int LARGE_SORT_CAP = 4096;
constexpr int SEL_THREADS = 1024;   // selection kernels: one workgroup, one thread per point

struct DevGraph {
    int32_t n;
    int64_t m2;                // 2m = number of arcs
    const int32_t *row_ptr;
    const int32_t *col;
    // upper arcs: the neighbours u > v of every node v, ascending (each undirected edge once)
    const int32_t *up_rp;
    const int32_t *up_col;
    const int32_t *small_nodes;  // nodes with 1 <= deg <= SMALL_DEG_MAX, ascending degree
    int32_t n_small;
    int32_t class_end[N_DEG_CLASSES];  // end of each degree class within small_nodes
    const int32_t *large_nodes;  // nodes with deg > SMALL_DEG_MAX, descending degree
    int32_t n_large;
    int32_t large_max_deg;       // largest degree (0 when there is no large node)
};

// Generation state kept on the device (small arrays; the populations are passed apart).
// Member ids: id < pop refers to column id of the committed pool; id >= pop to column
// id - pop of the offspring buffer.
struct DevState {
    int32_t *gen;        // current generation number g (read by every kernel)
    int32_t *ps_id;      // P after selection, in selection order: member ids
    int64_t *ps_A, *ps_S;
    double *ps_f1, *ps_f2;
    int32_t *pos_id;     // P reordered at the start of a generation (crowded order)
    int64_t *pos_A, *pos_S;
    int32_t *tr_rank;    // rank / crowding of that reordered P (trace output)
    double *tr_crowd;
    int32_t *par_id;     // [pop][E_S] parent ids of every offspring
    int32_t *gate;       // per offspring: -1 = majority crossover, k = copy of parent k
    unsigned long long *Aq, *Sq;  // fitness accumulators of the offspring
    int32_t *fr_count;   // final front: size, Alg. 3's choice, ids and objectives
    int32_t *fr_sel;
    int32_t *fr_id;
    int64_t *fr_A, *fr_S;
    double *fr_f1, *fr_f2;
};

struct GaConst {
    int32_t pop;
    int32_t ld;
    int32_t es;
    uint64_t seed;
    uint64_t thr_c;   // crossover threshold (Bernoulli as integer compare)
    uint64_t thr_m;   // mutation threshold
    int32_t mut_group;  // nodes per wave group in the small-degree mutation kernel
};

// Plan of the binned community-degree histogram (see kernels.hip): labels are split into
// tiles of 2^rbits values; pass 1 bins every (label, degree) pair of a chunk of nb nodes and
// a group of 16 individuals into runs per (tile, individual); pass 2 builds each tile's
// histogram in LDS. Used when every degree fits the entry's 32 - rbits bits, nb >= 64 and the
// problem has at least 2^min_log2 (node, individual) pairs.
constexpr int HB_CG = 16;  // individuals per bin group
struct HistPlan {
    // Label l goes to tile l div 2^rbits at index l mod 2^rbits (contiguous tiles, T =
    // ceil(n / 2^rbits), tile_bits = -1), or to tile l mod T at index l div T (interleaved
    // tiles, T = 2^tile_bits); an index is below 2^rbits either way.
    int32_t rbits = 0;
    int32_t tiles = 0;     // T
    int32_t tile_bits = -1;
    int32_t nb = 0;        // nodes per pass-1 chunk
    int32_t nchunks = 0, ngroups = 0;
    bool enabled = false;
    size_t entries = 0;    // uint32 entries of the run area
    size_t offsets = 0;    // uint32 offsets (per chunk and group: tiles * 16 + 1)
};
// narrow: on small graphs, narrower tiles and smaller chunks so that pass 2 alone fills the
// device. interleave: tiles interleave the label values, for labels that may come from a
// narrow range (partitions handed in by a caller, e.g. community indices 0..k-1); the
// search's own labels are node ids spread over [0, n), for which contiguous tiles suffice.
HistPlan hist_plan(int32_t n, int32_t pop, int32_t max_deg, int32_t min_log2, int32_t max_rbits,
                   bool narrow, bool interleave = false);

// One population on one graph, as the kernels see it (lives in device memory). A run is a
// batch of one item; the batched form puts many graphs, each with its own population, into
// the same launches.
struct Item {
    DevGraph g;
    GaConst c;
    DevState st;
    HistPlan hp;
    const int32_t *pool_cur, *q_cur;     // parent planes of a generation (q_cur: init target)
    int32_t *pool_new, *C, *q_next;      // crossover / mutation outputs
    const int32_t *lab;                  // plane the fitness kernels evaluate
    int32_t fit_pop, fit_ld;             // individuals evaluated and their row stride
    unsigned long long *fit_A, *fit_S;   // accumulators the fitness kernels add into
    int32_t *D;                          // plain histogram plane (hp disabled)
    size_t D_bytes;
    uint32_t *run, *off;                 // binned histogram areas (hp enabled)
    int32_t fit_npw;                     // nodes per wave of the arc scan
    int32_t xo_nb;                       // nodes per workgroup of init / crossover
};

// A multi-item launch: item i owns blocks [start[i], start[i + 1]) of a one-dimensional grid.
struct Span {
    const Item *items;
    const int32_t *start;
    int32_t count;
};

// Launch kinds; a kind's per-item block count depends only on the item's geometry.
enum Kind : int {
    K_INIT = 0,
    K_FIT,
    K_BIN,
    K_HIST,
    K_CLEAR,
    K_ONE,  // one workgroup per item (selection kernels)
    K_XO,
    K_MUT0,  // + class index, N_DEG_CLASSES kinds
    K_MUTL = K_MUT0 + N_DEG_CLASSES,
    N_KINDS
};
int32_t kind_blocks(Kind k, const Item &it);  // host side
size_t kind_lds(Kind k, const Item &it);       // dynamic LDS bytes the kind needs (host side)

// ---- multi-item launchers (kernels.hip); `blocks` is the total over the span -------------
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
int32_t kind_aux(Kind k, const Item &it);     // template / size argument of the kind
hipError_t launch_kind(Kind k, const Span &sp, int32_t blocks, size_t lds, int32_t aux,
                       hipStream_t s);
// k_dev (may be null): a device count; rows at or beyond it are skipped (k is then an upper
// bound that sizes the launch)
hipError_t launch_extract(int32_t n, int32_t ld, int32_t pop, const int32_t *pool,
                          const int32_t *q, const int32_t *ids, int32_t k, int32_t *out,
                          hipStream_t s, const int32_t *k_dev = nullptr);
// bad (may be null): a device flag set to 1 if a label lies outside [0, n); such labels are
// stored as 0
hipError_t launch_transpose_in(const int32_t *rows, int32_t n, int32_t n_ind, int32_t ld,
                               int32_t *out, int32_t *bad, hipStream_t s);
hipError_t launch_finalize(int64_t m2, int32_t n_ind, const unsigned long long *A,
                           const unsigned long long *S, double *f1, double *f2,
                           hipStream_t s);

// which selection kernel a K_ONE launch runs
enum OneKernel : int { ONE_INIT_STATE = 0, ONE_RANK_PARENTS, ONE_SELECT, ONE_FINAL, ONE_ZERO_ACC };
hipError_t launch_one(OneKernel which, const Span &sp, int32_t count, hipStream_t s);

}  // namespace hpm
