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

constexpr int SMALL_DEG_MAX = 32;   // mutation of nodes up to this degree: one lane per node
constexpr int LARGE_SORT_CAP = 4096;  // larger nodes: LDS sort up to this degree, then a scan
constexpr int SEL_THREADS = 1024;   // selection kernels: one workgroup, one thread per point

struct DevGraph {
    int32_t n;
    int64_t m2;                // 2m = number of arcs
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *small_nodes;  // nodes with 1 <= deg <= SMALL_DEG_MAX, ascending degree
    int32_t n_small;
    const int32_t *large_nodes;  // nodes with deg > SMALL_DEG_MAX, descending degree
    int32_t n_large;
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
    int32_t *fr_count;   // final front: size, ids and objectives
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

// ---- launchers (kernels.hip) -----------------------------------------------------------
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_init(const DevGraph &g, const GaConst &c, int32_t *Q, hipStream_t s);
hipError_t launch_fitness(const DevGraph &g, const int32_t *lab, int32_t ld, int32_t pop,
                          int32_t *D, unsigned long long *A, hipStream_t s);
hipError_t launch_sweep(int32_t n, const int32_t *lab_unused, int32_t ld, int32_t pop,
                        int32_t *D, unsigned long long *S, hipStream_t s);
hipError_t launch_init_state(const GaConst &c, int64_t m2, const DevState &st, hipStream_t s);
hipError_t launch_rank_parents(const GaConst &c, int64_t m2, const DevState &st,
                               hipStream_t s);
hipError_t launch_crossover(const DevGraph &g, const GaConst &c, const DevState &st,
                            const int32_t *pool_cur, const int32_t *q_cur, int32_t *pool_new,
                            int32_t *C, int32_t *q_next, hipStream_t s);
hipError_t launch_mutation(const DevGraph &g, const GaConst &c, const DevState &st,
                           const int32_t *C, int32_t *q_next, hipStream_t s);
hipError_t launch_select(const GaConst &c, int64_t m2, const DevState &st, hipStream_t s);
hipError_t launch_final(const GaConst &c, int64_t m2, const DevState &st, hipStream_t s);
hipError_t launch_extract(int32_t n, int32_t ld, int32_t pop, const int32_t *pool,
                          const int32_t *q, const int32_t *ids, int32_t k, int32_t *out,
                          hipStream_t s);
hipError_t launch_transpose_in(const int32_t *rows, int32_t n, int32_t n_ind, int32_t ld,
                               int32_t *out, hipStream_t s);
hipError_t launch_finalize(int64_t m2, int32_t n_ind, const unsigned long long *A,
                           const unsigned long long *S, double *f1, double *f2,
                           hipStream_t s);

}  // namespace hpm
