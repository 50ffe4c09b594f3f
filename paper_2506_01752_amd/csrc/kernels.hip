// HIP kernels of the HP-MOCD hot path for gfx950 (CDNA4, wave64).
//
// Everything here is integer work except the two objective divisions and the crowding
// distance (binary64, no contraction). No kernel uses MFMA: nothing is a dense contraction.
// The populations and the community-degree histograms are node-major (see internal.hpp).
#include <climits>

#include "internal.hpp"
#include "philox.hpp"

namespace hpm {

// ---------------------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------------------
// Division of 0 <= x < 2^32 by a run-time constant d >= 1 with one high multiply
// (Granlund & Montgomery, "Division by invariant integers using multiplication", 1994).
struct FastDiv {
    uint32_t d, m, s;
    FastDiv() = default;
    explicit FastDiv(uint32_t div) : d(div)
    {
        s = 0;
        while ((1ull << s) < div) ++s;
        m = (uint32_t)((((1ull << 32) * ((1ull << s) - div)) / div) + 1);
    }
    __device__ __forceinline__ uint32_t div(uint32_t x) const
    {
        return (uint32_t)(((uint64_t)__umulhi(x, m) + x) >> s);
    }
};

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// number of set bits of a 64-lane mask below this lane
__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                           __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Orders this wave's LDS accesses: earlier writes are visible to later reads of other lanes.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double f1_of(int64_t k1, int64_t m2) { return (double)k1 / (double)m2; }
__device__ __forceinline__ double f2_of(int64_t k2, int64_t m2)
{
    return (double)k2 / (double)(m2 * m2);
}

// ---------------------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------------------
__global__ void k_fill_zero(uint4 *p, size_t n16, unsigned char *tail, size_t ntail)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    const size_t n16 = bytes / 16, ntail = bytes % 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    k_fill_zero<<<(unsigned)blocks, 256, 0, s>>>((uint4 *)p, n16, (unsigned char *)p + n16 * 16,
                                                 ntail);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// initialisation (Alg. 1 InitializePopulation): node v of individual j takes its own id or
// the id of a uniformly drawn neighbour (sorted adjacency), one Philox block per (v, j).
// ---------------------------------------------------------------------------------------
constexpr int NODE_BLOCK = 32;  // nodes per workgroup in the per-(node, individual) kernels

__global__ __launch_bounds__(256) void k_init(DevGraph g, GaConst c, int32_t *__restrict__ Q,
                                              FastDiv divpop)
{
    const int64_t v0 = (int64_t)blockIdx.x * NODE_BLOCK;
    const int nv = (int)min((int64_t)NODE_BLOCK, (int64_t)g.n - v0);
    const uint32_t items = (uint32_t)nv * (uint32_t)c.pop;
    for (uint32_t f = threadIdx.x; f < items; f += blockDim.x) {
        const uint32_t q = divpop.div(f);
        const uint32_t j = f - q * (uint32_t)c.pop;
        const int32_t v = (int32_t)(v0 + q);
        const int32_t rs = g.row_ptr[v];
        const uint32_t d = (uint32_t)(g.row_ptr[v + 1] - rs);
        const u32x4 w = philox(c.seed, (uint32_t)v, j, 0u, TAG_INIT);
        const uint32_t k = pick(w.a, d + 1u);
        Q[(size_t)v * c.ld + j] = (k == d) ? v : g.col[rs + (int32_t)k];
    }
}

hipError_t launch_init(const DevGraph &g, const GaConst &c, int32_t *Q, hipStream_t s)
{
    const unsigned blocks = (unsigned)((g.n + NODE_BLOCK - 1) / NODE_BLOCK);
    k_init<<<blocks, 256, 0, s>>>(g, c, Q, FastDiv((uint32_t)c.pop));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// fitness (section 4.1, eq. objectives): one wave walks a run of consecutive nodes; its
// lanes hold two individuals each (columns 2l, 2l+1 of a 128-column chunk). For every arc
// (v,u) the wave reads the node-major row of u once (a contiguous 8-byte-per-lane load),
// compares with v's row and counts intra arcs per lane. v, its arc range and the neighbour
// ids are wave-uniform (scalar loads). D[label][col] += deg(v) by device-scope atomics.
// ---------------------------------------------------------------------------------------
constexpr int FIT_NODES_PER_WAVE = 32;
constexpr int FIT_UNROLL = 8;

__global__ __launch_bounds__(256) void k_fitness(DevGraph g, const int32_t *__restrict__ lab,
                                                 int32_t ld, int32_t pop, int32_t nchunks,
                                                 int32_t *__restrict__ D,
                                                 unsigned long long *__restrict__ A)
{
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int chunk = wave % nchunks;
    const int64_t v0 = (int64_t)(wave / nchunks) * FIT_NODES_PER_WAVE;
    if (v0 >= g.n) return;
    const int64_t v1 = min(v0 + FIT_NODES_PER_WAVE, (int64_t)g.n);
    const int c0 = chunk * 128 + 2 * lane;
    const bool act0 = c0 < pop, act1 = c0 + 1 < pop;
    int cnt0 = 0, cnt1 = 0;
    if (act0) {
        for (int64_t v = v0; v < v1; ++v) {
            const int32_t rs = g.row_ptr[v], re = g.row_ptr[v + 1];
            const int2 own = *(const int2 *)(lab + (size_t)v * ld + c0);
            int32_t e = rs;
            for (; e + FIT_UNROLL <= re; e += FIT_UNROLL) {
                int32_t u[FIT_UNROLL];
#pragma unroll
                for (int k = 0; k < FIT_UNROLL; ++k) u[k] = g.col[e + k];
                int2 x[FIT_UNROLL];
#pragma unroll
                for (int k = 0; k < FIT_UNROLL; ++k)
                    x[k] = *(const int2 *)(lab + (size_t)u[k] * ld + c0);
#pragma unroll
                for (int k = 0; k < FIT_UNROLL; ++k) {
                    cnt0 += x[k].x == own.x;
                    cnt1 += x[k].y == own.y;
                }
            }
            for (; e < re; ++e) {
                const int2 x = *(const int2 *)(lab + (size_t)g.col[e] * ld + c0);
                cnt0 += x.x == own.x;
                cnt1 += x.y == own.y;
            }
            const int32_t d = re - rs;
            if (d > 0) {
                atomicAdd(D + (size_t)own.x * ld + c0, d);
                if (act1) atomicAdd(D + (size_t)own.y * ld + c0 + 1, d);
            }
        }
        atomicAdd(A + c0, (unsigned long long)cnt0);
        if (act1) atomicAdd(A + c0 + 1, (unsigned long long)cnt1);
    }
}

hipError_t launch_fitness(const DevGraph &g, const int32_t *lab, int32_t ld, int32_t pop,
                          int32_t *D, unsigned long long *A, hipStream_t s)
{
    const int nchunks = (pop + 127) / 128;
    const int64_t waves = ((int64_t)g.n + FIT_NODES_PER_WAVE - 1) / FIT_NODES_PER_WAVE * nchunks;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    k_fitness<<<blocks, 256, 0, s>>>(g, lab, ld, pop, nchunks, D, A);
    return hipGetLastError();
}

// S = sum_c D_c^2 per individual: a coalesced sweep over the node-major histogram that also
// clears it for the next evaluation.
constexpr int SWEEP_ROWS_PER_WAVE = 128;

__global__ __launch_bounds__(256) void k_sweep(int32_t n, int32_t ld, int32_t pop,
                                               int32_t nchunks, int32_t *__restrict__ D,
                                               unsigned long long *__restrict__ S)
{
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int chunk = wave % nchunks;
    const int64_t r0 = (int64_t)(wave / nchunks) * SWEEP_ROWS_PER_WAVE;
    if (r0 >= n) return;
    const int64_t r1 = min(r0 + SWEEP_ROWS_PER_WAVE, (int64_t)n);
    const int c0 = chunk * 128 + 2 * lane;
    if (c0 >= pop) return;
    unsigned long long s0 = 0, s1 = 0;
    int64_t r = r0;
    for (; r + 4 <= r1; r += 4) {
        int2 x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = *(const int2 *)(D + (size_t)(r + k) * ld + c0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s0 += (unsigned long long)((int64_t)x[k].x * x[k].x);
            s1 += (unsigned long long)((int64_t)x[k].y * x[k].y);
            *(int2 *)(D + (size_t)(r + k) * ld + c0) = make_int2(0, 0);
        }
    }
    for (; r < r1; ++r) {
        const int2 x = *(const int2 *)(D + (size_t)r * ld + c0);
        s0 += (unsigned long long)((int64_t)x.x * x.x);
        s1 += (unsigned long long)((int64_t)x.y * x.y);
        *(int2 *)(D + (size_t)r * ld + c0) = make_int2(0, 0);
    }
    atomicAdd(S + c0, s0);
    if (c0 + 1 < pop) atomicAdd(S + c0 + 1, s1);
}

hipError_t launch_sweep(int32_t n, const int32_t *, int32_t ld, int32_t pop, int32_t *D,
                        unsigned long long *S, hipStream_t s)
{
    const int nchunks = (pop + 127) / 128;
    const int64_t waves = ((int64_t)n + SWEEP_ROWS_PER_WAVE - 1) / SWEEP_ROWS_PER_WAVE * nchunks;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    k_sweep<<<blocks, 256, 0, s>>>(n, ld, pop, nchunks, D, S);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// NSGA-II selection routines (Alg. 1: FastNonDominatedSort, CrowdingDistanceAssignment,
// SortByRankAndDistance, EnvironmentalSelection) for N <= 1024 points in one workgroup.
// Dominance on exact integer keys k1 = 2m - A, k2 = S; crowding in binary64 on
// f1 = k1 / 2m, f2 = k2 / (2m)^2; order by (rank, crowding desc, position).
// ---------------------------------------------------------------------------------------
struct SelSmem {
    long long k1[SEL_THREADS];
    long long k2[SEL_THREADS];
    double crowd[SEL_THREADS];
    int rank[SEL_THREADS];
    int list[SEL_THREADS];
    int sorted[SEL_THREADS];
    int nlist;
};

__device__ __forceinline__ bool dom(long long b1, long long b2, long long a1, long long a2)
{
    return b1 <= a1 && b2 <= a2 && (b1 < a1 || b2 < a2);
}

// On return: sh.rank[i], sh.crowd[i] for i < N and sh.list[q] = index of the point at
// crowded-comparison position q.
__device__ void rank_crowd_order(int N, int64_t m2, SelSmem &sh)
{
    const int i = threadIdx.x;
    const bool act = i < N;
    const long long a1 = act ? sh.k1[i] : 0, a2 = act ? sh.k2[i] : 0;

    // domination counts, then peel fronts (Deb's fast non-dominated sort)
    int cnt = 0;
    if (act)
        for (int j = 0; j < N; ++j) cnt += dom(sh.k1[j], sh.k2[j], a1, a2);
    int myrank = (act && cnt == 0) ? 1 : 0;
    if (act) sh.rank[i] = myrank;
    __syncthreads();
    for (int r = 1;; ++r) {
        if (i == 0) sh.nlist = 0;
        __syncthreads();
        if (act && myrank == r) sh.list[atomicAdd(&sh.nlist, 1)] = i;
        __syncthreads();
        const int nf = sh.nlist;
        if (nf == 0) break;
        if (act && myrank == 0) {
            for (int a = 0; a < nf; ++a) {
                const int j = sh.list[a];
                cnt -= dom(sh.k1[j], sh.k2[j], a1, a2);
            }
            if (cnt == 0) {
                myrank = r + 1;
                sh.rank[i] = myrank;
            }
        }
        __syncthreads();
    }

    // crowding distance per front
    int off = 0, l = 0;
    if (act)
        for (int j = 0; j < N; ++j) {
            const int rj = sh.rank[j];
            off += rj < myrank;
            l += rj == myrank;
        }
    const bool interior_front = act && l > 2;
    double cd = 0.0;
    for (int o = 0; o < 2; ++o) {
        const long long mykey = o == 0 ? a1 : a2;
        int pos = 0;
        if (interior_front) {
            for (int j = 0; j < N; ++j) {
                if (sh.rank[j] != myrank) continue;
                const long long kj = o == 0 ? sh.k1[j] : sh.k2[j];
                pos += (kj < mykey) || (kj == mykey && j < i);
            }
            sh.sorted[off + pos] = i;
        }
        __syncthreads();
        if (interior_front) {
            if (pos == 0 || pos == l - 1) {
                cd = __builtin_inf();
            } else {
                const int first = sh.sorted[off], last = sh.sorted[off + l - 1];
                const int lo = sh.sorted[off + pos - 1], hi = sh.sorted[off + pos + 1];
                double vf, vl, vlo, vhi;
                if (o == 0) {
                    vf = f1_of(sh.k1[first], m2);
                    vl = f1_of(sh.k1[last], m2);
                    vlo = f1_of(sh.k1[lo], m2);
                    vhi = f1_of(sh.k1[hi], m2);
                } else {
                    vf = f2_of(sh.k2[first], m2);
                    vl = f2_of(sh.k2[last], m2);
                    vlo = f2_of(sh.k2[lo], m2);
                    vhi = f2_of(sh.k2[hi], m2);
                }
                const double den = vl - vf;
                if (den != 0.0) cd = cd + (vhi - vlo) / den;
            }
        }
        __syncthreads();
    }
    if (act && l <= 2) cd = __builtin_inf();
    if (act) sh.crowd[i] = cd;
    __syncthreads();

    // crowded-comparison order
    if (act) {
        int p = 0;
        for (int j = 0; j < N; ++j) {
            const int rj = sh.rank[j];
            const double cj = sh.crowd[j];
            p += (rj < myrank) || (rj == myrank && (cj > cd || (cj == cd && j < i)));
        }
        sh.list[p] = i;
    }
    __syncthreads();
}

__global__ __launch_bounds__(SEL_THREADS) void k_init_state(GaConst c, int64_t m2, DevState st)
{
    const int i = threadIdx.x;
    if (i < c.pop) {
        const int64_t A = (int64_t)st.Aq[i], S = (int64_t)st.Sq[i];
        st.ps_id[i] = c.pop + i;
        st.ps_A[i] = A;
        st.ps_S[i] = S;
        st.ps_f1[i] = f1_of(m2 - A, m2);
        st.ps_f2[i] = f2_of(S, m2);
    }
    if (i == 0) *st.gen = 1;
}

hipError_t launch_init_state(const GaConst &c, int64_t m2, const DevState &st, hipStream_t s)
{
    k_init_state<<<1, SEL_THREADS, 0, s>>>(c, m2, st);
    return hipGetLastError();
}

// Start of generation g: rank, crowd and reorder P^(g-1); draw the E_S binary tournaments
// of every offspring and its crossover gate; clear the offspring fitness accumulators.
__global__ __launch_bounds__(SEL_THREADS) void k_rank_parents(GaConst c, int64_t m2, DevState st)
{
    __shared__ SelSmem sh;
    const int i = threadIdx.x, N = c.pop;
    if (i < N) {
        sh.k1[i] = m2 - st.ps_A[i];
        sh.k2[i] = st.ps_S[i];
    }
    __syncthreads();
    rank_crowd_order(N, m2, sh);
    if (i < N) {
        const int src = sh.list[i];
        const int id = st.ps_id[src];
        st.pos_id[i] = id;
        st.pos_A[i] = st.ps_A[src];
        st.pos_S[i] = st.ps_S[src];
        st.tr_rank[i] = sh.rank[src];
        st.tr_crowd[i] = sh.crowd[src];
        sh.sorted[i] = id;
    }
    __syncthreads();
    const uint32_t g = (uint32_t)*st.gen;
    const int es = c.es;
    for (int t = i; t < N * es; t += blockDim.x) {
        const int j = t / es, k = t - (t / es) * es;
        const u32x4 w = philox(c.seed, (uint32_t)k, (uint32_t)j, g, TAG_SEL);
        const uint32_t a = pick(w.a, (uint32_t)N), b = pick(w.b, (uint32_t)N);
        st.par_id[j * es + k] = sh.sorted[a < b ? a : b];  // lower position wins
    }
    for (int j = i; j < N; j += blockDim.x) {
        const u32x4 w = philox(c.seed, GATE_X, (uint32_t)j, g, TAG_SEL);
        st.gate[j] = ((uint64_t)w.a < c.thr_c) ? -1 : (int)pick(w.b, (uint32_t)es);
        st.Aq[j] = 0ull;
        st.Sq[j] = 0ull;
    }
}

hipError_t launch_rank_parents(const GaConst &c, int64_t m2, const DevState &st, hipStream_t s)
{
    k_rank_parents<<<1, SEL_THREADS, 0, s>>>(c, m2, st);
    return hipGetLastError();
}

// End of generation g: R = P (reordered) ++ Q, keep the first pop in crowded order.
__global__ __launch_bounds__(SEL_THREADS) void k_select(GaConst c, int64_t m2, DevState st)
{
    __shared__ SelSmem sh;
    const int i = threadIdx.x, np = c.pop, N = 2 * c.pop;
    if (i < np) {
        sh.k1[i] = m2 - st.pos_A[i];
        sh.k2[i] = st.pos_S[i];
    } else if (i < N) {
        sh.k1[i] = m2 - (int64_t)st.Aq[i - np];
        sh.k2[i] = (int64_t)st.Sq[i - np];
    }
    __syncthreads();
    rank_crowd_order(N, m2, sh);
    if (i < np) {
        const int src = sh.list[i];
        const int64_t A = src < np ? st.pos_A[src] : (int64_t)st.Aq[src - np];
        const int64_t S = src < np ? st.pos_S[src] : (int64_t)st.Sq[src - np];
        st.ps_id[i] = src;  // < pop: committed pool column; >= pop: offspring column
        st.ps_A[i] = A;
        st.ps_S[i] = S;
        st.ps_f1[i] = f1_of(m2 - A, m2);
        st.ps_f2[i] = f2_of(S, m2);
    }
    if (i == 0) *st.gen += 1;
}

hipError_t launch_select(const GaConst &c, int64_t m2, const DevState &st, hipStream_t s)
{
    k_select<<<1, SEL_THREADS, 0, s>>>(c, m2, st);
    return hipGetLastError();
}

// Phase 4 of Alg. 1: the rank-1 members of the final population in crowded order.
__global__ __launch_bounds__(SEL_THREADS) void k_final(GaConst c, int64_t m2, DevState st)
{
    __shared__ SelSmem sh;
    const int i = threadIdx.x, N = c.pop;
    if (i < N) {
        sh.k1[i] = m2 - st.ps_A[i];
        sh.k2[i] = st.ps_S[i];
    }
    __syncthreads();
    rank_crowd_order(N, m2, sh);
    if (i < N) {
        const int src = sh.list[i];
        if (sh.rank[src] == 1) {  // rank-1 members come first in crowded order
            const int64_t A = st.ps_A[src], S = st.ps_S[src];
            st.fr_id[i] = st.ps_id[src];
            st.fr_A[i] = A;
            st.fr_S[i] = S;
            st.fr_f1[i] = f1_of(m2 - A, m2);
            st.fr_f2[i] = f2_of(S, m2);
        }
    }
    if (i == 0) {
        int k = 0;
        for (int j = 0; j < N; ++j) k += sh.rank[j] == 1;
        *st.fr_count = k;
    }
}

hipError_t launch_final(const GaConst &c, int64_t m2, const DevState &st, hipStream_t s)
{
    k_final<<<1, SEL_THREADS, 0, s>>>(c, m2, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// crossover (Alg. 2) + commit of the reordered parents into the next pool.
// Thread per (node, offspring). Label of member id at node v:
//   id < pop ? pool_cur[v][id] : q_cur[v][id - pop].
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_crossover(int32_t n, GaConst c, DevState st,
                                                   const int32_t *__restrict__ pool_cur,
                                                   const int32_t *__restrict__ q_cur,
                                                   int32_t *__restrict__ pool_new,
                                                   int32_t *__restrict__ C,
                                                   int32_t *__restrict__ q_next, FastDiv divpop)
{
    extern __shared__ int xs[];  // [pop] pos_id, [pop] gate, [pop * es] par_id
    const int pop = c.pop, es = c.es, ld = c.ld;
    int *s_pos = xs, *s_gate = xs + pop, *s_par = xs + 2 * pop;
    for (int t = threadIdx.x; t < pop; t += blockDim.x) {
        s_pos[t] = st.pos_id[t];
        s_gate[t] = st.gate[t];
    }
    for (int t = threadIdx.x; t < pop * es; t += blockDim.x) s_par[t] = st.par_id[t];
    __syncthreads();
    const uint32_t g = (uint32_t)*st.gen;
    const int64_t v0 = (int64_t)blockIdx.x * NODE_BLOCK;
    const int nv = (int)min((int64_t)NODE_BLOCK, (int64_t)n - v0);
    const uint32_t items = (uint32_t)nv * (uint32_t)pop;
    for (uint32_t f = threadIdx.x; f < items; f += blockDim.x) {
        const uint32_t q = divpop.div(f);
        const int j = (int)(f - q * (uint32_t)pop);
        const int64_t v = v0 + q;
        const size_t row = (size_t)v * ld;
        const int32_t *prow = pool_cur + row;
        const int32_t *qrow = q_cur + row - pop;  // indexed by id >= pop
        int id = s_pos[j];
        pool_new[row + j] = id < pop ? prow[id] : qrow[id];
        const int gk = s_gate[j];
        int out;
        if (gk >= 0) {
            id = s_par[j * es + gk];
            out = id < pop ? prow[id] : qrow[id];
        } else {
            int L[HPMOCD_MAX_PARENTS_DEV];
#pragma unroll
            for (int k = 0; k < HPMOCD_MAX_PARENTS_DEV; ++k) {
                if (k < es) {
                    const int pid = s_par[j * es + k];
                    L[k] = pid < pop ? prow[pid] : qrow[pid];
                } else {
                    L[k] = 0;
                }
            }
            // plurality over the ensemble; ties drawn uniformly over the tied labels taken in
            // ascending order (eq. arg_max)
            int cnt[HPMOCD_MAX_PARENTS_DEV];
            int best = 0;
#pragma unroll
            for (int k = 0; k < HPMOCD_MAX_PARENTS_DEV; ++k) {
                int ck = 0;
#pragma unroll
                for (int t = 0; t < HPMOCD_MAX_PARENTS_DEV; ++t) ck += (t < es) && L[t] == L[k];
                cnt[k] = (k < es) ? ck : 0;
                best = max(best, cnt[k]);
            }
            bool cand[HPMOCD_MAX_PARENTS_DEV];
            int nt = 0;
#pragma unroll
            for (int k = 0; k < HPMOCD_MAX_PARENTS_DEV; ++k) {
                bool first = true;
#pragma unroll
                for (int t = 0; t < k; ++t) first = first && L[t] != L[k];
                cand[k] = (k < es) && first && cnt[k] == best;
                nt += cand[k];
            }
            int want = 0;
            if (nt > 1) want = (int)pick(philox(c.seed, (uint32_t)v, (uint32_t)j, g, TAG_XOV).a,
                                         (uint32_t)nt);
            out = 0;
#pragma unroll
            for (int k = 0; k < HPMOCD_MAX_PARENTS_DEV; ++k) {
                int below = 0;
#pragma unroll
                for (int t = 0; t < HPMOCD_MAX_PARENTS_DEV; ++t) below += cand[t] && L[t] < L[k];
                if (cand[k] && below == want) out = L[k];
            }
        }
        C[row + j] = out;
        q_next[row + j] = out;
    }
}

hipError_t launch_crossover(const DevGraph &g, const GaConst &c, const DevState &st,
                            const int32_t *pool_cur, const int32_t *q_cur, int32_t *pool_new,
                            int32_t *C, int32_t *q_next, hipStream_t s)
{
    const unsigned blocks = (unsigned)((g.n + NODE_BLOCK - 1) / NODE_BLOCK);
    const size_t smem = sizeof(int) * (size_t)c.pop * (size_t)(2 + c.es);
    k_crossover<<<blocks, 256, smem, s>>>(g.n, c, st, pool_cur, q_cur, pool_new, C, q_next,
                                          FastDiv((uint32_t)c.pop));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// mutation (section 4.3.2): node v of offspring j mutates when its MUT draw falls below
// the threshold and deg v > 0; it then takes the plurality label of its neighbours in the
// post-crossover child C (its own label excluded), ties drawn with the second MUT word over
// the tied labels in ascending order. Reads only C, writes only q_next (synchronous).
// ---------------------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void bitonic_regs(int (&a)[K])
{
#pragma unroll
    for (int k = 2; k <= K; k <<= 1)
#pragma unroll
        for (int jj = k >> 1; jj > 0; jj >>= 1)
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const int l = i ^ jj;
                if (l > i) {
                    const int x = a[i], y = a[l];
                    const bool up = (i & k) == 0;
                    a[i] = up ? min(x, y) : max(x, y);
                    a[l] = up ? max(x, y) : min(x, y);
                }
            }
}

// Plurality of d <= K labels held by this lane (one mutation per lane).
template <int K>
__device__ __forceinline__ int lane_plurality(const int32_t *__restrict__ C, int ld, int j,
                                              const int32_t *__restrict__ nbr, int d, uint32_t r)
{
    int a[K];
#pragma unroll
    for (int i = 0; i < K; ++i) a[i] = (i < d) ? C[(size_t)nbr[i] * ld + j] : INT_MAX;
    bitonic_regs<K>(a);
    int best = 0, nt = 0, cur = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (i < d) {
            cur = (i > 0 && a[i] == a[i - 1]) ? cur + 1 : 1;
            const bool end = (i == d - 1) || (i + 1 < K && a[i + 1] != a[i]);
            if (end) {
                if (cur > best) {
                    best = cur;
                    nt = 1;
                } else if (cur == best) {
                    ++nt;
                }
            }
        }
    }
    const int want = nt > 1 ? (int)pick(r, (uint32_t)nt) : 0;
    int res = a[0], seen = 0;
    cur = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (i < d) {
            cur = (i > 0 && a[i] == a[i - 1]) ? cur + 1 : 1;
            const bool end = (i == d - 1) || (i + 1 < K && a[i + 1] != a[i]);
            if (end && cur == best) {
                if (seen == want) res = a[i];
                ++seen;
            }
        }
    }
    return res;
}

constexpr int MUT_WAVES = 4;
constexpr int MUT_LIST_CAP = 1024;  // mutation items one wave can queue (group * pop)

__global__ __launch_bounds__(256) void k_mutate_small(DevGraph g, GaConst c, DevState st,
                                                      const int32_t *__restrict__ C,
                                                      int32_t *__restrict__ q_next,
                                                      FastDiv divpop)
{
    __shared__ uint2 items[MUT_WAVES][MUT_LIST_CAP];
    const int wv = threadIdx.x >> 6, lane = lane_id();
    const uint32_t gen = (uint32_t)*st.gen;
    const int pop = c.pop, G = c.mut_group;
    const int ngroups = (g.n_small + G - 1) / G;
    for (int grp = blockIdx.x * MUT_WAVES + wv; grp < ngroups; grp += gridDim.x * MUT_WAVES) {
        const int base = grp * G;
        const int gn = min(G, g.n_small - base);
        const uint32_t total = (uint32_t)gn * (uint32_t)pop;
        int count = 0;
        for (uint32_t f0 = 0; f0 < total; f0 += 64) {
            const uint32_t f = f0 + (uint32_t)lane;
            bool mut = false;
            uint32_t r = 0, key = 0;
            if (f < total) {
                const uint32_t gv = divpop.div(f);
                const uint32_t j = f - gv * (uint32_t)pop;
                const int32_t node = g.small_nodes[base + (int)gv];
                const u32x4 w = philox(c.seed, (uint32_t)node, j, gen, TAG_MUT);
                mut = (uint64_t)w.a < c.thr_m;
                r = w.b;
                key = (gv << 16) | j;
            }
            const uint64_t bal = __ballot(mut);
            if (mut) items[wv][count + lanes_below(bal)] = make_uint2(key, r);
            count += __popcll(bal);
        }
        wave_lds_sync();
        for (int b = 0; b < count; b += 64) {
            const int idx = b + lane;
            const bool has = idx < count;
            const uint2 it = has ? items[wv][idx] : make_uint2(0u, 0u);
            const int32_t node = g.small_nodes[base + (int)(it.x >> 16)];
            const int j = (int)(it.x & 0xFFFFu);
            const int32_t rs = g.row_ptr[node];
            const int d = has ? g.row_ptr[node + 1] - rs : 0;
            const int dmax = wave_max(d);
            const int32_t *nbr = g.col + rs;
            int res;
            if (dmax <= 4)
                res = lane_plurality<4>(C, c.ld, j, nbr, d, it.y);
            else if (dmax <= 8)
                res = lane_plurality<8>(C, c.ld, j, nbr, d, it.y);
            else if (dmax <= 16)
                res = lane_plurality<16>(C, c.ld, j, nbr, d, it.y);
            else
                res = lane_plurality<32>(C, c.ld, j, nbr, d, it.y);
            if (has) q_next[(size_t)node * c.ld + j] = res;
        }
        wave_lds_sync();
    }
}

// Nodes above SMALL_DEG_MAX: one wave per node; each mutating offspring's neighbour labels
// are sorted in LDS (bitonic), and the plurality is read off the runs.
__device__ __forceinline__ int upper_bound_lds(const int *buf, int lo, int hi, int x)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (buf[mid] <= x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(64) void k_mutate_large(DevGraph g, GaConst c, DevState st,
                                                     const int32_t *__restrict__ C,
                                                     int32_t *__restrict__ q_next)
{
    __shared__ uint2 items[HPMOCD_MAX_POP_DEV];
    __shared__ int buf[LARGE_SORT_CAP];
    __shared__ int result;
    const int lane = threadIdx.x;
    const uint32_t gen = (uint32_t)*st.gen;
    const int pop = c.pop, ld = c.ld;
    for (int t = blockIdx.x; t < g.n_large; t += gridDim.x) {
        const int32_t node = g.large_nodes[t];
        const int32_t rs = g.row_ptr[node];
        const int d = g.row_ptr[node + 1] - rs;
        int count = 0;
        for (int j0 = 0; j0 < pop; j0 += 64) {
            const int j = j0 + lane;
            bool mut = false;
            uint32_t r = 0;
            if (j < pop) {
                const u32x4 w = philox(c.seed, (uint32_t)node, (uint32_t)j, gen, TAG_MUT);
                mut = (uint64_t)w.a < c.thr_m;
                r = w.b;
            }
            const uint64_t bal = __ballot(mut);
            if (mut) items[count + lanes_below(bal)] = make_uint2((uint32_t)j, r);
            count += __popcll(bal);
        }
        __syncthreads();
        for (int it = 0; it < count; ++it) {
            const int j = (int)items[it].x;
            const uint32_t r = items[it].y;
            if (d <= LARGE_SORT_CAP) {
                int P = 64;
                while (P < d) P <<= 1;
                for (int i = lane; i < P; i += 64)
                    buf[i] = i < d ? C[(size_t)g.col[rs + i] * ld + j] : INT_MAX;
                __syncthreads();
                for (int k = 2; k <= P; k <<= 1)
                    for (int jj = k >> 1; jj > 0; jj >>= 1) {
                        for (int i = lane; i < P; i += 64) {
                            const int l = i ^ jj;
                            if (l > i) {
                                const int x = buf[i], y = buf[l];
                                const bool up = (i & k) == 0;
                                if (up ? (x > y) : (x < y)) {
                                    buf[i] = y;
                                    buf[l] = x;
                                }
                            }
                        }
                        __syncthreads();
                    }
                int mybest = 0;
                for (int i = lane; i < d; i += 64)
                    if (i == 0 || buf[i] != buf[i - 1])
                        mybest = max(mybest, upper_bound_lds(buf, i, d, buf[i]) - i);
                const int best = wave_max(mybest);
                int nt = 0;
                for (int i0 = 0; i0 < d; i0 += 64) {
                    const int i = i0 + lane;
                    const bool q = i < d && (i == 0 || buf[i] != buf[i - 1]) &&
                                   upper_bound_lds(buf, i, d, buf[i]) - i == best;
                    nt += __popcll(__ballot(q));
                }
                int want = nt > 1 ? (int)pick(r, (uint32_t)nt) : 0;
                for (int i0 = 0; i0 < d; i0 += 64) {
                    const int i = i0 + lane;
                    const bool q = i < d && (i == 0 || buf[i] != buf[i - 1]) &&
                                   upper_bound_lds(buf, i, d, buf[i]) - i == best;
                    const uint64_t bal = __ballot(q);
                    const int cntq = __popcll(bal);
                    if (want < cntq) {
                        if (q && lanes_below(bal) == want) result = buf[i];
                        break;
                    }
                    want -= cntq;
                }
            } else {
                // degree above the LDS sort capacity: walk the distinct labels in ascending
                // order by repeated minimum extraction (slow, exact)
                int best = 0, nt = 0, prev = -1;
                for (;;) {
                    int mn = INT_MAX;
                    for (int i = lane; i < d; i += 64) {
                        const int x = C[(size_t)g.col[rs + i] * ld + j];
                        if (x > prev) mn = min(mn, x);
                    }
                    mn = wave_min(mn);
                    if (mn == INT_MAX) break;
                    int cn = 0;
                    for (int i = lane; i < d; i += 64) cn += C[(size_t)g.col[rs + i] * ld + j] == mn;
                    cn = wave_sum(cn);
                    if (cn > best) {
                        best = cn;
                        nt = 1;
                    } else if (cn == best) {
                        ++nt;
                    }
                    prev = mn;
                }
                const int want = nt > 1 ? (int)pick(r, (uint32_t)nt) : 0;
                int seen = 0;
                prev = -1;
                for (;;) {
                    int mn = INT_MAX;
                    for (int i = lane; i < d; i += 64) {
                        const int x = C[(size_t)g.col[rs + i] * ld + j];
                        if (x > prev) mn = min(mn, x);
                    }
                    mn = wave_min(mn);
                    if (mn == INT_MAX) break;
                    int cn = 0;
                    for (int i = lane; i < d; i += 64) cn += C[(size_t)g.col[rs + i] * ld + j] == mn;
                    cn = wave_sum(cn);
                    if (cn == best) {
                        if (seen == want) {
                            if (lane == 0) result = mn;
                            break;
                        }
                        ++seen;
                    }
                    prev = mn;
                }
            }
            __syncthreads();
            if (lane == 0) q_next[(size_t)node * ld + j] = result;
            __syncthreads();
        }
    }
}

hipError_t launch_mutation(const DevGraph &g, const GaConst &c, const DevState &st,
                           const int32_t *C, int32_t *q_next, hipStream_t s)
{
    if (c.thr_m == 0) return hipSuccess;  // no node can mutate
    if (g.n_small > 0) {
        const int ngroups = (g.n_small + c.mut_group - 1) / c.mut_group;
        int blocks = (ngroups + MUT_WAVES - 1) / MUT_WAVES;
        if (blocks > 4096) blocks = 4096;
        k_mutate_small<<<blocks, 64 * MUT_WAVES, 0, s>>>(g, c, st, C, q_next,
                                                          FastDiv((uint32_t)c.pop));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (g.n_large > 0) {
        int blocks = g.n_large < 8192 ? g.n_large : 8192;
        k_mutate_large<<<blocks, 64, 0, s>>>(g, c, st, C, q_next);
        return hipGetLastError();
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------------------
// front extraction, eval-path helpers
// ---------------------------------------------------------------------------------------
__global__ void k_extract(int32_t n, int32_t ld, int32_t pop, const int32_t *__restrict__ pool,
                          const int32_t *__restrict__ q, const int32_t *__restrict__ ids,
                          int32_t k, int32_t *__restrict__ out)
{
    const int row = blockIdx.y;
    const int id = ids[row];
    const int32_t *src = id < pop ? pool + id : q + (id - pop);
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        out[(size_t)row * n + v] = src[(size_t)v * ld];
}

hipError_t launch_extract(int32_t n, int32_t ld, int32_t pop, const int32_t *pool,
                          const int32_t *q, const int32_t *ids, int32_t k, int32_t *out,
                          hipStream_t s)
{
    if (k == 0) return hipSuccess;
    unsigned bx = (unsigned)((n + 255) / 256);
    if (bx > 1024) bx = 1024;
    k_extract<<<dim3(bx, (unsigned)k), 256, 0, s>>>(n, ld, pop, pool, q, ids, k, out);
    return hipGetLastError();
}

// rows [n_ind][n] -> node-major [n][ld], 32x32 tiles through LDS
__global__ void k_transpose_in(const int32_t *__restrict__ rows, int32_t n, int32_t n_ind,
                               int32_t ld, int32_t *__restrict__ out)
{
    __shared__ int tile[32][33];
    const int64_t v0 = (int64_t)blockIdx.x * 32;
    const int i0 = blockIdx.y * 32;
    for (int r = threadIdx.y; r < 32; r += blockDim.y) {
        const int i = i0 + r;
        const int64_t v = v0 + threadIdx.x;
        if (i < n_ind && v < n) tile[r][threadIdx.x] = rows[(size_t)i * n + v];
    }
    __syncthreads();
    for (int r = threadIdx.y; r < 32; r += blockDim.y) {
        const int64_t v = v0 + r;
        const int i = i0 + threadIdx.x;
        if (i < n_ind && v < n) out[(size_t)v * ld + i] = tile[threadIdx.x][r];
    }
}

hipError_t launch_transpose_in(const int32_t *rows, int32_t n, int32_t n_ind, int32_t ld,
                               int32_t *out, hipStream_t s)
{
    dim3 grid((unsigned)((n + 31) / 32), (unsigned)((n_ind + 31) / 32));
    k_transpose_in<<<grid, dim3(32, 8), 0, s>>>(rows, n, n_ind, ld, out);
    return hipGetLastError();
}

__global__ void k_finalize(int64_t m2, int32_t n_ind, const unsigned long long *A,
                           const unsigned long long *S, double *f1, double *f2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_ind) {
        f1[i] = f1_of(m2 - (int64_t)A[i], m2);
        f2[i] = f2_of((int64_t)S[i], m2);
    }
}

hipError_t launch_finalize(int64_t m2, int32_t n_ind, const unsigned long long *A,
                           const unsigned long long *S, double *f1, double *f2, hipStream_t s)
{
    k_finalize<<<(unsigned)((n_ind + 255) / 256), 256, 0, s>>>(m2, n_ind, A, S, f1, f2);
    return hipGetLastError();
}

}  // namespace hpm
