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
    __host__ __device__ explicit FastDiv(uint32_t div) : d(div)
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

// Buffer pointers read from the item tables are generic to the compiler: it would emit flat
// memory instructions (which also count against the LDS/scalar counter) and keep
// wave-uniform loads such as CSR row offsets off the scalar unit. Every hot kernel re-types
// the buffers it touches as global-address-space pointers first.
#define GLB __attribute__((address_space(1)))
#define LDSP __attribute__((address_space(3)))
template <class T> __device__ __forceinline__ GLB T *glb(T *p) { return (GLB T *)p; }

// device-scope relaxed atomic addition on global memory, returning the old value
template <class T> __device__ __forceinline__ T gatomic_add(GLB T *p, T v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// DevGraph with global-address-space pointers (degree-class bounds are read from the item
// table directly: a private copy indexed at run time would live in scratch memory)
struct GGraph {
    int32_t n;
    int64_t m2;
    const GLB int32_t *row_ptr;
    const GLB int32_t *col;
    const GLB int32_t *up_rp;
    const GLB int32_t *up_col;
    const GLB int32_t *small_nodes;
    const GLB int32_t *large_nodes;
    int32_t n_small, n_large, large_max_deg;
};
__device__ __forceinline__ GGraph gview(const DevGraph &g)
{
    GGraph v;
    v.n = g.n;
    v.m2 = g.m2;
    v.row_ptr = glb(g.row_ptr);
    v.col = glb(g.col);
    v.up_rp = glb(g.up_rp);
    v.up_col = glb(g.up_col);
    v.small_nodes = glb(g.small_nodes);
    v.large_nodes = glb(g.large_nodes);
    v.n_small = g.n_small;
    v.n_large = g.n_large;
    v.large_max_deg = g.large_max_deg;
    return v;
}

// DevState fields the variation kernels read
struct GState {
    const GLB int32_t *gen;
    const GLB int32_t *pos_id;
    const GLB int32_t *par_id;
    const GLB int32_t *gate;
};
__device__ __forceinline__ GState gview(const DevState &s)
{
    GState v;
    v.gen = glb(s.gen);
    v.pos_id = glb(s.pos_id);
    v.par_id = glb(s.par_id);
    v.gate = glb(s.gate);
    return v;
}

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

// The item that owns this workgroup in a multi-item launch, with the workgroup's index
// among the item's blocks and the item's block count (all wave-uniform).
__device__ __forceinline__ int item_of(const Span &sp, int &lb, int &nblk)
{
    const int b = (int)blockIdx.x;
    int lo = 0, hi = sp.count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sp.start[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    lb = b - sp.start[lo];
    nblk = sp.start[lo + 1] - sp.start[lo];
    return lo;
}

// Workgroups are dealt to the eight XCDs round-robin by block id, and each XCD has its own
// L2. This renumbers an item's blocks so that the blocks one XCD runs form one contiguous
// range of logical indices (a bijection on [0, nblk)): kernels whose neighbouring logical
// blocks share cache lines then share them inside one L2.
__device__ __forceinline__ int xcd_remap(int lb, int nblk)
{
    const int x = lb & 7, q = lb >> 3;
    const int per = nblk >> 3, rem = nblk & 7;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + q;
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
constexpr int NODE_BLOCK = 32;  // nodes per workgroup in the init kernel

__global__ __launch_bounds__(256) void k_init(Span sp)
{
    int lb, nblk;
    const Item &it = sp.items[item_of(sp, lb, nblk)];
    const GGraph g = gview(it.g);
    const GaConst c = it.c;
    GLB int32_t *__restrict__ Q = glb(const_cast<int32_t *>(it.q_cur));
    const FastDiv divpop((uint32_t)c.pop);
    const int64_t v0 = (int64_t)lb * NODE_BLOCK;
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

// ---------------------------------------------------------------------------------------
// fitness (section 4.1, eq. objectives): one wave walks a run of consecutive nodes; its
// lanes hold two individuals each (columns 2l, 2l+1 of a 128-column chunk). The graph is
// symmetric, so A (intra arcs) is twice the number of intra edges: the wave visits each
// undirected edge once, as the upper arc (v,u) with u > v, reads the node-major row of u (a
// contiguous 8-byte-per-lane load), compares with v's row and counts per lane; the count is
// doubled at the end. v, its arc range and the neighbour ids are wave-uniform (scalar loads).
// Community degree sums, small problems only (larger ones use the binned histogram below):
// D[label][col] += deg(v) by device-scope atomics whose returned old value gives S exactly,
// since sum over the additions of (old + d)^2 - old^2 telescopes to sum_c D_c^2 whatever
// order the atomics take.
// ---------------------------------------------------------------------------------------
constexpr int FIT_ARCS = 16;   // arcs in flight per wave in the scan phase
constexpr int FIT_WAVES = 4;   // waves per k_fitness workgroup
constexpr int FIT_NODES = 8;   // nodes per batch in the histogram phase

__device__ __forceinline__ unsigned long long sq_step(int old, int d)
{
    return 2ull * (unsigned long long)(unsigned)old * (unsigned)d +
           (unsigned long long)(unsigned)d * (unsigned)d;
}

// Phase 1 walks the wave's upper-arc range [up_rp[v0], up_rp[v1]) as one flat stream, 16
// arcs at a time: for each arc (s,u) it loads the rows of u and of its source s (the source
// row is re-read from L1) and counts equal labels. Phase 2 then adds deg(v) into the histogram
// for 8 nodes at a time. Keeping the histogram atomics out of phase 1 matters: vector
// memory counters drain in order, so an atomic issued between two gathers would make the
// second wait for the atomic's round trip.
struct FitSums {
    int c0 = -1;  // first of the lane's two columns; -1 when the lane has none
    unsigned long long a0 = 0, a1 = 0, s0 = 0, s1 = 0;
};

__device__ __forceinline__ FitSums fitness_wave(const Item &it, int lb)
{
    FitSums out;
    const GGraph g = gview(it.g);
    const GLB int32_t *__restrict__ lab = glb(it.lab);
    const int32_t ld = it.fit_ld, pop = it.fit_pop, npw = it.fit_npw;
    const int nchunks = (pop + 127) / 128;
    GLB int32_t *__restrict__ D = glb(it.D);
    const int atomics_phase = it.hp.enabled ? 0 : 1;
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(lb * FIT_WAVES + (int)(threadIdx.x >> 6));
    const int chunk = wave % nchunks;
    const int32_t v0 = (int32_t)min((int64_t)(wave / nchunks) * npw, (int64_t)g.n);
    if (v0 >= g.n) return out;
    const int32_t v1 = (int32_t)min((int64_t)v0 + npw, (int64_t)g.n);
    const int c0 = chunk * 128 + 2 * lane;
    const bool act1 = c0 + 1 < pop;
    if (c0 >= pop) return out;
    const GLB int32_t *__restrict__ lc = lab + c0;

    // phase 1: intra-community arcs
    int cnt0 = 0, cnt1 = 0;
    const int32_t a0 = g.up_rp[v0], a1 = g.up_rp[v1];
    int32_t src = v0, src_end = g.up_rp[v0 + 1];
    for (int32_t e = a0; e < a1; e += FIT_ARCS) {
        int32_t u[FIT_ARCS], sv[FIT_ARCS];
#pragma unroll
        for (int k = 0; k < FIT_ARCS; ++k) {
            const int32_t ek = min(e + k, a1 - 1);
            while (ek >= src_end) {  // uniform: advance to the arc's source node
                ++src;
                src_end = g.up_rp[src + 1];
            }
            u[k] = g.up_col[ek];
            sv[k] = src;
        }
        int2 x[FIT_ARCS], y[FIT_ARCS];
#pragma unroll
        for (int k = 0; k < FIT_ARCS; ++k) {
            x[k] = *(const int2 *)(lc + (size_t)u[k] * ld);
            y[k] = *(const int2 *)(lc + (size_t)sv[k] * ld);
        }
#pragma unroll
        for (int k = 0; k < FIT_ARCS; ++k) {
            const bool ok = e + k < a1;
            cnt0 += ok && x[k].x == y[k].x;
            cnt1 += ok && x[k].y == y[k].y;
        }
    }

    // phase 2: community degree sums and S (telescoping squares)
    unsigned long long s0 = 0, s1 = 0;
    if (atomics_phase)
    for (int32_t vb = v0; vb < v1; vb += FIT_NODES) {
        int2 own[FIT_NODES];
        int32_t d[FIT_NODES];
#pragma unroll
        for (int k = 0; k < FIT_NODES; ++k) {
            const int32_t v = min(vb + k, v1 - 1);
            d[k] = (vb + k < v1) ? g.row_ptr[v + 1] - g.row_ptr[v] : 0;
            own[k] = *(const int2 *)(lc + (size_t)v * ld);
        }
        int o0[FIT_NODES], o1[FIT_NODES];
#pragma unroll
        for (int k = 0; k < FIT_NODES; ++k) {
            o0[k] = o1[k] = 0;
            if (d[k] > 0) {
                o0[k] = gatomic_add(D + (size_t)own[k].x * ld + c0, d[k]);
                if (act1) o1[k] = gatomic_add(D + (size_t)own[k].y * ld + c0 + 1, d[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < FIT_NODES; ++k) {
            s0 += sq_step(o0[k], d[k]);
            s1 += sq_step(o1[k], d[k]);
        }
    }
    // every intra edge {v,u} stands for the two intra arcs (v,u) and (u,v)
    out.c0 = c0;
    out.a0 = 2ull * (unsigned)cnt0;
    out.a1 = act1 ? 2ull * (unsigned)cnt1 : 0ull;
    out.s0 = s0;
    out.s1 = act1 ? s1 : 0ull;
    return out;
}

// The waves' per-column sums are added up per workgroup in LDS first, so that A (and, on the
// plain path, S) takes one global atomic per (workgroup, column) instead of one per (wave,
// column): those atomics land on a few hundred addresses and execute at the memory side, one
// after another per address, which on small graphs (many waves of a few nodes each) cost more
// than the scan itself.
__global__ __launch_bounds__(64 * FIT_WAVES) void k_fitness(Span sp)
{
    int lb, nblk;
    const Item &it = sp.items[item_of(sp, lb, nblk)];
    extern __shared__ unsigned long long fit_red[];  // [fit_ld] A, then [fit_ld] S (plain path)
    const int ldf = it.fit_ld, pop = it.fit_pop;
    const bool plain = !it.hp.enabled;
    const int nred = plain ? 2 * ldf : ldf;
    for (int i = threadIdx.x; i < nred; i += blockDim.x) fit_red[i] = 0ull;
    __syncthreads();
    const FitSums f = fitness_wave(it, lb);
    if (f.c0 >= 0) {
        atomicAdd(&fit_red[f.c0], f.a0);
        atomicAdd(&fit_red[f.c0 + 1], f.a1);  // c0 + 1 < ld: ld is a multiple of 16
        if (plain) {
            atomicAdd(&fit_red[ldf + f.c0], f.s0);
            atomicAdd(&fit_red[ldf + f.c0 + 1], f.s1);
        }
    }
    __syncthreads();
    GLB unsigned long long *__restrict__ A = glb(it.fit_A);
    GLB unsigned long long *__restrict__ S = glb(it.fit_S);
    for (int i = threadIdx.x; i < pop; i += blockDim.x) {
        if (fit_red[i]) gatomic_add(A + i, fit_red[i]);
        if (plain && fit_red[ldf + i]) gatomic_add(S + i, fit_red[ldf + i]);
    }
}

// ---------------------------------------------------------------------------------------
// Binned community-degree histogram. Atomics on global memory are executed at the memory
// side on this part whatever the histogram's footprint, at a few times 10^10 per second, so
// the n x pop scattered additions of the plain histogram dominate the evaluation. Instead:
//  pass 1 (k_bin): a workgroup takes nb nodes x 16 individuals, counts the (label tile,
//   individual) bucket of every pair in LDS, scans the counts, and writes the pairs as
//   packed words (label's index within its tile | deg << rbits) grouped by bucket into its
//   own area, plus the bucket offsets;
//  pass 2 (k_hist): a workgroup per (tile, individual) gathers that bucket's runs from every
//   chunk into an LDS histogram of 2^rbits counters and adds sum D_c^2 to S.
// Every addition happens in LDS; the only global atomic is one per pass-2 workgroup.
// ---------------------------------------------------------------------------------------
// largest chunk of the binned histogram (nodes per k_bin workgroup)
constexpr int BIN_MAX_NODES = 1024;
// small graphs: narrower tiles (down to 2^12 labels) until pass 2 has this many (tile,
// individual) workgroups, and chunks small enough that pass 2's threads each get one
constexpr int HIST_MIN_WGS = 512;
constexpr int HIST_MIN_CHUNKS = 256;
// interleaved tiles only while k_bin's counters take at most this many LDS words
constexpr int HIST_INTERLEAVE_MAX_COUNTERS = 4096;

HistPlan hist_plan(int32_t n, int32_t pop, int32_t max_deg, int32_t min_log2, int32_t max_rbits,
                   bool narrow, bool interleave)
{
    HistPlan p;
    int rb = 0;
    const int rb_max = max_rbits < 10 ? 10 : (max_rbits > 14 ? 14 : max_rbits);
    while ((1 << rb) < n && rb < rb_max) ++rb;  // tiles of up to 16384 labels (64 KB of LDS)
    while (narrow && rb > 12 && (((int64_t)n + (1 << rb) - 1) >> rb) * pop < HIST_MIN_WGS) --rb;
    p.rbits = rb;
    p.tiles = (int32_t)(((int64_t)n + (1 << rb) - 1) >> rb);
    // Interleaved tiles (label l in tile l mod T at index l div T, T the power of two at or
    // above the contiguous count) spread labels from a narrow range, such as community
    // indices 0..k-1, over every tile; with contiguous tiles they would all fall in the
    // first, whose k_hist workgroups would then do all the work. Kept contiguous where the
    // rounding would take too much of k_bin's LDS from its chunk.
    if (interleave) {
        int tb = 0;
        while ((1 << tb) < p.tiles) ++tb;
        if ((1 << tb) * HB_CG <= HIST_INTERLEAVE_MAX_COUNTERS) {
            p.tile_bits = tb;
            p.tiles = 1 << tb;
        }
    }
    const int counters = p.tiles * HB_CG;
    // 64 KB of LDS: counters, staging (16 words a node), scan partials, degrees (1 a node)
    const int budget_words = 16384 - 64;
    int nb = (budget_words - counters - 2) / (HB_CG + 1);
    nb = nb / 64 * 64;
    if (nb > BIN_MAX_NODES) nb = BIN_MAX_NODES;
    const int nb_par = (int)((n / HIST_MIN_CHUNKS) / 64 * 64);
    if (narrow && nb > nb_par) nb = nb_par < 64 ? 64 : nb_par;
    p.nb = nb;
    // the plain histogram's n * pop global atomics are cheap for small problems, where the
    // two extra launches would cost more than they save
    p.enabled = nb >= 64 && (int64_t)max_deg < ((int64_t)1 << (32 - rb)) &&
                (int64_t)n * pop >= ((int64_t)1 << min_log2);
    if (!p.enabled) return p;
    p.nchunks = (n + nb - 1) / nb;
    p.ngroups = (pop + HB_CG - 1) / HB_CG;
    p.entries = (size_t)p.ngroups * p.nchunks * (size_t)nb * HB_CG;
    p.offsets = (size_t)p.ngroups * p.nchunks * (size_t)(counters + 1);
    return p;
}

// block-wide exclusive scan of one value per thread (blockDim = 256); returns the prefix
// and writes the block total to *total
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *wsum, uint32_t *total)
{
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        if (w < wv) base += wsum[w];
        tot += wsum[w];
    }
    *total = tot;
    return base + x - v;
}

// A k_bin workgroup holds its whole chunk (at most BIN_MAX_NODES x 16 items), BIN_IPT items
// per thread in registers, so that both passes use one read of the labels. The launch takes
// as many threads as its largest chunk has nodes (rounded up to whole waves, at most
// BIN_THREADS): small graphs' 64-node chunks get one-wave workgroups.
constexpr int BIN_THREADS = 1024;
constexpr int BIN_IPT = BIN_MAX_NODES * HB_CG / BIN_THREADS;
static_assert(BIN_IPT == HB_CG, "a chunk of nb nodes needs nb threads");

// k_bin workgroups launched per item at most, for 1024-thread workgroups: the part's 256 CUs
// hold one each (the registers of the chunk-in-registers form, with the next unit's labels
// in flight beside this one's, leave no room for a second), and each workgroup runs unit
// after unit. Smaller workgroups (small graphs' shorter chunks) get proportionally more.
constexpr int BIN_RESIDENT = 256;

__global__ __launch_bounds__(BIN_THREADS) void k_bin(Span sp)
{
    int lb, nblk;
    const Item &it = sp.items[item_of(sp, lb, nblk)];
    const GGraph g = gview(it.g);
    const GLB int32_t *__restrict__ lab = glb(it.lab);
    const int32_t ld = it.fit_ld, pop = it.fit_pop;
    const HistPlan p = it.hp;
    GLB uint32_t *__restrict__ run = glb(it.run);
    GLB uint32_t *__restrict__ off = glb(it.off);
    extern __shared__ uint32_t bl[];
    const int counters = p.tiles * HB_CG;
    uint32_t *cnt = bl;                             // [counters + 1]
    uint32_t *stage = bl + counters + 1;            // [nb * 16]
    uint32_t *wsum = stage + (size_t)p.nb * HB_CG;  // [BIN_THREADS / 64]
    uint32_t *degl = wsum + BIN_THREADS / 64;       // [nb] the chunk's degrees
    const uint32_t rmask = (1u << p.rbits) - 1u;
    const uint32_t ntiles = (uint32_t)p.tiles;
    // Units u = chunk * ngroups + group. Blocks are dealt to the eight XCDs round-robin; the
    // blocks of one XCD take one contiguous range of units and walk it side by side, so that
    // at any time they hold neighbouring units: the groups of one chunk read the same label
    // rows (16 columns each) together, through one L2.
    const int units = p.nchunks * p.ngroups;
    const int xcd = lb & 7, per = nblk >> 3, rem = nblk & 7;
    const int bx = per + (xcd < rem ? 1 : 0);
    const int l0 = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    const int u_end = (int)((int64_t)(l0 + bx) * units / nblk);
    int u = (int)((int64_t)l0 * units / nblk) + (lb >> 3);
    // a unit's labels (16 items per thread, item itm = 16 * (v - v0) + jl: a wave reads four
    // 64-byte row segments) and its nodes' degrees are loaded one unit ahead, so that the next
    // unit's loads are in flight while this one is counted, scanned and written out
    uint32_t xv[BIN_IPT], xn[BIN_IPT];
    uint32_t dv = 0, dn = 0;
    // thread t holds column t % 16 of nodes v0 + t / 16 + k * rows (blockDim.x is a multiple
    // of 64)
    const int col = (int)(threadIdx.x & (HB_CG - 1)), row = (int)(threadIdx.x >> 4);
    const int rows = (int)(blockDim.x >> 4);
    auto fetch = [&](int uu, uint32_t(&xr)[BIN_IPT], uint32_t &dr) {
        const int chunk = uu / p.ngroups, grp = uu - chunk * p.ngroups;
        const int32_t v0 = chunk * p.nb;
        const int nv = min(p.nb, g.n - v0);
        const bool colok = col < min(HB_CG, pop - grp * HB_CG);
        const GLB int32_t *src = lab + (size_t)(v0 + row) * ld + grp * HB_CG + col;
#pragma unroll
        for (int k = 0; k < BIN_IPT; ++k)
            xr[k] = (colok && k * rows + row < nv) ? (uint32_t)src[(size_t)(k * rows) * ld] : 0u;
        const int t = (int)threadIdx.x;
        dr = t < nv ? (uint32_t)(g.row_ptr[v0 + t + 1] - g.row_ptr[v0 + t]) : 0u;
    };
    if (u < u_end) fetch(u, xv, dv);
    for (; u < u_end; u += bx) {
        if (u + bx < u_end) fetch(u + bx, xn, dn);
        const int chunk = u / p.ngroups, grp = u - chunk * p.ngroups;
        const int32_t v0 = chunk * p.nb;
        const int nv = min(p.nb, g.n - v0);
        const bool colok = col < min(HB_CG, pop - grp * HB_CG);
        // each label as (tile << rbits | index within its tile): with contiguous tiles, the
        // label itself
        if (p.tile_bits >= 0) {
#pragma unroll
            for (int k = 0; k < BIN_IPT; ++k)
                xv[k] = ((xv[k] & (ntiles - 1u)) << p.rbits) | (xv[k] >> p.tile_bits);
        }
        for (int i = threadIdx.x; i <= counters; i += blockDim.x) cnt[i] = 0;
        if ((int)threadIdx.x < nv) degl[threadIdx.x] = dv;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BIN_IPT; ++k)
            if (colok && k * rows + row < nv) atomicAdd(&cnt[(xv[k] >> p.rbits) * HB_CG + col], 1u);
        __syncthreads();
        // exclusive scan of the counters: each thread scans a contiguous slice
        const int per_t = (counters + (int)blockDim.x - 1) / (int)blockDim.x;
        const int a = min((int)threadIdx.x * per_t, counters), b = min(a + per_t, counters);
        uint32_t sum = 0;
        for (int i = a; i < b; ++i) sum += cnt[i];
        uint32_t total;
        uint32_t acc = block_exclusive_scan(sum, wsum, &total);
        __syncthreads();
        for (int i = a; i < b; ++i) {
            const uint32_t v = cnt[i];
            cnt[i] = acc;
            acc += v;
        }
        if (threadIdx.x == 0) cnt[counters] = total;
        __syncthreads();
        GLB uint32_t *o = off + ((size_t)chunk * p.ngroups + grp) * (size_t)(counters + 1);
        for (int i = threadIdx.x; i <= counters; i += blockDim.x) o[i] = cnt[i];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BIN_IPT; ++k)
            if (colok && k * rows + row < nv) {
                const uint32_t pos = atomicAdd(&cnt[(xv[k] >> p.rbits) * HB_CG + col], 1u);
                stage[pos] = (xv[k] & rmask) | (degl[k * rows + row] << p.rbits);
            }
        __syncthreads();
        GLB uint32_t *dst = run + ((size_t)grp * p.nchunks + chunk) * ((size_t)p.nb * HB_CG);
        for (uint32_t i = threadIdx.x; i < total; i += blockDim.x) dst[i] = stage[i];
        // the next unit rewrites cnt and degl only after its first barrier, which every thread
        // reaches after its copy-out above; stage only after three more
#pragma unroll
        for (int k = 0; k < BIN_IPT; ++k) xv[k] = xn[k];
        dv = dn;
    }
}

constexpr int HIST_UNROLL = 16;

__global__ __launch_bounds__(256) void k_hist(Span sp)
{
    int lb, nblk;
    const Item &it = sp.items[item_of(sp, lb, nblk)];
    const HistPlan p = it.hp;
    const GLB uint32_t *__restrict__ run = glb(it.run);
    const GLB uint32_t *__restrict__ off = glb(it.off);
    GLB unsigned long long *__restrict__ S = glb(it.fit_S);
    extern __shared__ uint32_t hist[];  // [2^rbits], the whole 64 KB at most
    // the arc scan runs beside this kernel; its waves are bandwidth-bound while these wait on
    // chains of dependent loads, so these take the higher issue priority on a shared CU
    __builtin_amdgcn_s_setprio(3);
    // individuals of one tile side by side: the 16 of a group read adjacent run offsets
    const int lg = xcd_remap(lb, nblk);
    const int t = lg / it.fit_pop, j = lg % it.fit_pop;
    const int grp = j / HB_CG, jl = j % HB_CG;
    const int counters = p.tiles * HB_CG;
    const int bucket = t * HB_CG + jl;
    const int R = 1 << p.rbits;
    for (int i = threadIdx.x; i < R; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const size_t span = (size_t)p.nb * HB_CG;
    // each thread owns chunks w = tid + 256 k; the run bounds of up to 8 of them are loaded
    // together, then the runs are read HIST_UNROLL words at a time
    constexpr int WPT = 8;
    for (int w0 = 0; w0 < p.nchunks; w0 += (int)blockDim.x * WPT) {
        uint32_t b0[WPT], b1[WPT];
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int w = w0 + k * (int)blockDim.x + (int)threadIdx.x;
            b0[k] = b1[k] = 0;
            if (w < p.nchunks) {
                const GLB uint32_t *o = off + ((size_t)w * p.ngroups + grp) * (size_t)(counters + 1) + bucket;
                b0[k] = o[0];
                b1[k] = o[1];
            }
        }
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const int w = w0 + k * (int)blockDim.x + (int)threadIdx.x;
            const GLB uint32_t *src = run + ((size_t)grp * p.nchunks + (size_t)(w < p.nchunks ? w : 0)) * span;
            for (uint32_t e = b0[k]; e < b1[k]; e += HIST_UNROLL) {
                uint32_t x[HIST_UNROLL];
#pragma unroll
                for (int q = 0; q < HIST_UNROLL; ++q) x[q] = (e + q < b1[k]) ? src[e + q] : 0u;
#pragma unroll
                for (int q = 0; q < HIST_UNROLL; ++q)
                    if (e + q < b1[k]) atomicAdd(&hist[x[q] & (uint32_t)(R - 1)], x[q] >> p.rbits);
            }
        }
    }
    __syncthreads();
    unsigned long long sq = 0;
    for (int i = threadIdx.x; i < R; i += blockDim.x) {
        const unsigned long long h = hist[i];
        sq += h * h;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
    if (lane_id() == 0 && sq != 0) gatomic_add(S + j, sq);  // one atomic per wave
}

// clears the plain histogram plane of every item (write-only stream)
__global__ __launch_bounds__(256) void k_clear(Span sp)
{
    int lb, nblk;
    const Item &it = sp.items[item_of(sp, lb, nblk)];
    uint4 *p = (uint4 *)it.D;
    const size_t n16 = it.D_bytes / 16;
    for (size_t i = (size_t)lb * blockDim.x + threadIdx.x; i < n16; i += (size_t)nblk * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
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

// Sum over a group of T consecutive lanes (T a power of two dividing 64); every lane of the
// wave must call it.
__device__ __forceinline__ int group_sum(int v, int T)
{
    for (int o = T >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// On return: sh.rank[i], sh.crowd[i] for i < N and sh.list[q] = index of the point at
// crowded-comparison position q. Point i is served by the T threads [i*T, i*T + T) (T a
// power of two with N*T <= blockDim, at most 64); each O(N) scan is split over the group.
__device__ void rank_crowd_order(int N, int64_t m2, SelSmem &sh)
{
    int T = 1;
    while (T < 64 && N * T * 2 <= (int)blockDim.x) T <<= 1;
    const int i = threadIdx.x / T, sub = threadIdx.x % T;
    const bool act = i < N;
    const bool owner = act && sub == 0;
    const long long a1 = act ? sh.k1[i] : 0, a2 = act ? sh.k2[i] : 0;

    // domination counts, then peel fronts (Deb's fast non-dominated sort)
    int cnt = 0;
    if (act) {
#pragma unroll 4
        for (int j = sub; j < N; j += T) cnt += dom(sh.k1[j], sh.k2[j], a1, a2);
    }
    cnt = group_sum(cnt, T);
    int myrank = (act && cnt == 0) ? 1 : 0;
    if (owner) sh.rank[i] = myrank;
    __syncthreads();
    for (int r = 1;; ++r) {
        if (threadIdx.x == 0) sh.nlist = 0;
        __syncthreads();
        if (owner && myrank == r) sh.list[atomicAdd(&sh.nlist, 1)] = i;
        __syncthreads();
        const int nf = sh.nlist;
        if (nf == 0) break;
        int dec = 0;
        if (act && myrank == 0) {
#pragma unroll 4
            for (int a = sub; a < nf; a += T) {
                const int j = sh.list[a];
                dec += dom(sh.k1[j], sh.k2[j], a1, a2);
            }
        }
        dec = group_sum(dec, T);
        if (act && myrank == 0) {
            cnt -= dec;
            if (cnt == 0) {
                myrank = r + 1;
                if (owner) sh.rank[i] = myrank;
            }
        }
        __syncthreads();
    }

    // crowding distance per front
    int off = 0, l = 0;
    if (act) {
#pragma unroll 4
        for (int j = sub; j < N; j += T) {
            const int rj = sh.rank[j];
            off += rj < myrank;
            l += rj == myrank;
        }
    }
    off = group_sum(off, T);
    l = group_sum(l, T);
    const bool interior_front = act && l > 2;
    double cd = 0.0;
    for (int o = 0; o < 2; ++o) {
        const long long mykey = o == 0 ? a1 : a2;
        int pos = 0;
        if (interior_front) {
#pragma unroll 4
            for (int j = sub; j < N; j += T) {
                const long long kj = o == 0 ? sh.k1[j] : sh.k2[j];
                pos += sh.rank[j] == myrank && ((kj < mykey) || (kj == mykey && j < i));
            }
        }
        pos = group_sum(pos, T);
        if (interior_front && sub == 0) sh.sorted[off + pos] = i;
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
    if (owner) sh.crowd[i] = cd;
    __syncthreads();

    // crowded-comparison order
    int p = 0;
    if (act) {
#pragma unroll 4
        for (int j = sub; j < N; j += T) {
            const int rj = sh.rank[j];
            const double cj = sh.crowd[j];
            p += (rj < myrank) || (rj == myrank && (cj > cd || (cj == cd && j < i)));
        }
    }
    p = group_sum(p, T);
    if (owner) sh.list[p] = i;
    __syncthreads();
}

// The selection kernels run one workgroup per item: block b serves item b.
__global__ __launch_bounds__(SEL_THREADS) void k_init_state(Span sp)
{
    const Item &it = sp.items[blockIdx.x];
    const GaConst c = it.c;
    const DevState st = it.st;
    const int64_t m2 = it.g.m2;
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

// Start of generation g: rank, crowd and reorder P^(g-1); draw the E_S binary tournaments
// of every offspring and its crossover gate; clear the offspring fitness accumulators.
__global__ __launch_bounds__(SEL_THREADS) void k_rank_parents(Span sp)
{
    __shared__ SelSmem sh;
    const Item &it = sp.items[blockIdx.x];
    const GaConst c = it.c;
    const DevState st = it.st;
    const int64_t m2 = it.g.m2;
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

// End of generation g: R = P (reordered) ++ Q, keep the first pop in crowded order.
__global__ __launch_bounds__(SEL_THREADS) void k_select(Span sp)
{
    __shared__ SelSmem sh;
    const Item &it = sp.items[blockIdx.x];
    const GaConst c = it.c;
    const DevState st = it.st;
    const int64_t m2 = it.g.m2;
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

// Phase 4 of Alg. 1: the rank-1 members of the final population in crowded order.
__global__ __launch_bounds__(SEL_THREADS) void k_final(Span sp)
{
    __shared__ SelSmem sh;
    const Item &it = sp.items[blockIdx.x];
    const GaConst c = it.c;
    const DevState st = it.st;
    const int64_t m2 = it.g.m2;
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
        // Alg. 3: the first front member (crowded order) of largest Q = (1 - f1) - f2
        double best = -__builtin_inf();
        int sel = 0;
        for (int q = 0; q < k; ++q) {
            const int src = sh.list[q];
            const double qv = (1.0 - f1_of(sh.k1[src], m2)) - f2_of(sh.k2[src], m2);
            if (qv > best) {
                best = qv;
                sel = q;
            }
        }
        *st.fr_count = k;
        *st.fr_sel = sel;
    }
}

// Clears the offspring accumulators before the initial population's evaluation.
__global__ __launch_bounds__(SEL_THREADS) void k_zero_acc(Span sp)
{
    const Item &it = sp.items[blockIdx.x];
    for (int i = threadIdx.x; i < it.fit_pop; i += blockDim.x) {
        it.fit_A[i] = 0ull;
        it.fit_S[i] = 0ull;
    }
}

hipError_t launch_one(OneKernel which, const Span &sp, int32_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    switch (which) {
    case ONE_ZERO_ACC: k_zero_acc<<<count, SEL_THREADS, 0, s>>>(sp); break;
    case ONE_INIT_STATE: k_init_state<<<count, SEL_THREADS, 0, s>>>(sp); break;
    case ONE_RANK_PARENTS: k_rank_parents<<<count, SEL_THREADS, 0, s>>>(sp); break;
    case ONE_SELECT: k_select<<<count, SEL_THREADS, 0, s>>>(sp); break;
    default: k_final<<<count, SEL_THREADS, 0, s>>>(sp); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// crossover (Alg. 2) + commit of the reordered parents into the next pool.
// Thread per (node, offspring). Label of member id at node v:
//   id < pop ? pool_cur[v][id] : q_cur[v][id - pop].
// ---------------------------------------------------------------------------------------
// Plurality over an ensemble of ES labels; ties drawn uniformly over the tied labels taken
// in ascending order (eq. arg_max). The draw is made only when there is a tie.
template <int ES>
__device__ __forceinline__ int ensemble_plurality(const int (&L)[ES], uint64_t seed, uint32_t v,
                                                  uint32_t j, uint32_t g)
{
    int cnt[ES];
    int best = 0;
#pragma unroll
    for (int k = 0; k < ES; ++k) {
        int ck = 0;
#pragma unroll
        for (int t = 0; t < ES; ++t) ck += L[t] == L[k];
        cnt[k] = ck;
        best = max(best, ck);
    }
    bool cand[ES];
    int nt = 0;
#pragma unroll
    for (int k = 0; k < ES; ++k) {
        bool first = true;
#pragma unroll
        for (int t = 0; t < k; ++t) first = first && L[t] != L[k];
        cand[k] = first && cnt[k] == best;
        nt += cand[k];
    }
    if (nt == 1) {
        int out = L[0];
#pragma unroll
        for (int k = ES - 1; k >= 0; --k)
            if (cand[k]) out = L[k];
        return out;
    }
    const int want = (int)pick(philox(seed, v, j, g, TAG_XOV).a, (uint32_t)nt);
    int out = L[0];
#pragma unroll
    for (int k = 0; k < ES; ++k) {
        int below = 0;
#pragma unroll
        for (int t = 0; t < ES; ++t) below += cand[t] && L[t] < L[k];
        if (cand[k] && below == want) out = L[k];
    }
    return out;
}

// ints of k_crossover's LDS tables (pos_id, gate, par_id), rounded up to 16 bytes
__host__ __device__ inline int xo_table_ints(int pop, int es) { return ((2 + es) * pop + 3) & ~3; }

template <int ES>
__global__ __launch_bounds__(256) void k_crossover(Span sp)
{
    int lb, nblk;
    const Item &it = sp.items[item_of(sp, lb, nblk)];
    const int32_t n = it.g.n, nblock = it.xo_nb;
    const GaConst c = it.c;
    const GState st = gview(it.st);
    const GLB int32_t *__restrict__ pool_cur = glb(it.pool_cur);
    const GLB int32_t *__restrict__ q_cur = glb(it.q_cur);
    GLB int32_t *__restrict__ pool_new = glb(it.pool_new);
    GLB int32_t *__restrict__ C = glb(it.C);
    GLB int32_t *__restrict__ q_next = glb(it.q_next);
    const FastDiv divpop((uint32_t)c.pop);
    // LDS: [pop] pos_id, [pop] gate, [pop * ES] par_id, then (16-byte aligned) the block's
    // rows of the committed pool and of the offspring plane, [nblock * ld] each
    extern __shared__ __align__(16) int xs[];
    const int pop = c.pop, ld = c.ld;
    int *s_pos = xs, *s_gate = xs + pop, *s_par = xs + 2 * pop;
    int *s_pool = xs + xo_table_ints(pop, ES), *s_q = s_pool + (size_t)nblock * ld;
    for (int t = threadIdx.x; t < pop; t += blockDim.x) {
        s_pos[t] = st.pos_id[t];
        s_gate[t] = st.gate[t];
    }
    for (int t = threadIdx.x; t < pop * ES; t += blockDim.x) s_par[t] = st.par_id[t];
    const uint32_t g = (uint32_t)*st.gen;
    const int64_t v0 = (int64_t)lb * nblock;
    const int nv = (int)min((int64_t)nblock, (int64_t)n - v0);
    const uint32_t items = (uint32_t)nv * (uint32_t)pop;
    {   // consecutive nodes' rows are one contiguous span: 16-byte loads (ld is a multiple of 16)
        const int4 *gp = (const int4 *)(pool_cur + (size_t)v0 * ld);
        const int4 *gq = (const int4 *)(q_cur + (size_t)v0 * ld);
        int4 *lp = (int4 *)s_pool, *lq = (int4 *)s_q;
        const int n4 = nv * ld / 4;
        for (int t = threadIdx.x; t < n4; t += blockDim.x) {
            lp[t] = gp[t];
            lq[t] = gq[t];
        }
    }
    __syncthreads();
    // XO_ITEMS (node, offspring) items per thread at once: all their loads are issued
    // before any plurality is resolved
    constexpr int XO_ITEMS = 4;
    for (uint32_t base = 0; base < items; base += blockDim.x * XO_ITEMS) {
        int commit[XO_ITEMS], L[XO_ITEMS][ES];
        bool has[XO_ITEMS];
        size_t row[XO_ITEMS];
        int jj[XO_ITEMS], gk[XO_ITEMS];
        uint32_t vv[XO_ITEMS];
#pragma unroll
        for (int t = 0; t < XO_ITEMS; ++t) {
            const uint32_t f = base + t * blockDim.x + threadIdx.x;
            has[t] = f < items;
            const uint32_t fq = has[t] ? f : 0u;
            const uint32_t q = divpop.div(fq);
            jj[t] = (int)(fq - q * (uint32_t)pop);
            vv[t] = (uint32_t)(v0 + q);
            row[t] = (size_t)vv[t] * ld;
            const int *prow = s_pool + (size_t)q * ld;
            const int *qrow = s_q + (size_t)q * ld - pop;  // indexed by id >= pop
            const int id = s_pos[jj[t]];
            commit[t] = id < pop ? prow[id] : qrow[id];
            gk[t] = s_gate[jj[t]];
#pragma unroll
            for (int k = 0; k < ES; ++k) {
                const int pid = s_par[jj[t] * ES + (gk[t] >= 0 ? gk[t] : k)];
                L[t][k] = pid < pop ? prow[pid] : qrow[pid];
            }
        }
#pragma unroll
        for (int t = 0; t < XO_ITEMS; ++t) {
            if (!has[t]) continue;
            const int out = gk[t] >= 0 ? L[t][0]
                                       : ensemble_plurality<ES>(L[t], c.seed, vv[t], (uint32_t)jj[t], g);
            pool_new[row[t] + jj[t]] = commit[t];
            C[row[t] + jj[t]] = out;
            q_next[row[t] + jj[t]] = out;
        }
    }
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
template <int K, class NbrPtr>
__device__ __forceinline__ int lane_plurality(const GLB int32_t *__restrict__ C, int ld, int j,
                                              NbrPtr nbr, int d, uint32_t r)
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

// Lane class kernel: nodes list[0..count) all have 1 <= deg <= KMAX. A wave takes a group of
// G consecutive nodes, draws the MUT word of every (node, offspring) pair, queues the pairs
// that mutate in LDS (and, behind them, the group's neighbour lists), then resolves them one
// per lane. For KMAX == 16 the register array
// size is picked per batch (4, 8 or 16) from the batch's largest degree.
template <int KMAX, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_mutate_lanes(Span sp, int cls)
{
    int lb, nblk;
    const Item &it = sp.items[item_of(sp, lb, nblk)];
    const GGraph g = gview(it.g);
    const GaConst c = it.c;
    const GState st = gview(it.st);
    const GLB int32_t *__restrict__ C = glb(it.C);
    GLB int32_t *__restrict__ q_next = glb(it.q_next);
    const int32_t cstart = cls == 0 ? 0 : it.g.class_end[cls - 1];
    const GLB int32_t *__restrict__ list = g.small_nodes + cstart;
    const int32_t count_nodes = it.g.class_end[cls] - cstart;
    const FastDiv divpop((uint32_t)c.pop);
    __shared__ uint2 items[WAVES][MUT_LIST_CAP];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = lane_id();
    const uint32_t gen = (uint32_t)*st.gen;
    const int pop = c.pop, G = c.mut_group;
    const int ngroups = (count_nodes + G - 1) / G;
    for (int grp = lb * WAVES + wv; grp < ngroups; grp += nblk * WAVES) {
        const int base = grp * G;
        const int gn = min(G, count_nodes - base);
        const uint32_t total = (uint32_t)gn * (uint32_t)pop;
        // the group's node ids, one per lane, shared by shuffles (groups of up to 64 nodes)
        const int32_t lane_node = lane < gn ? list[base + lane] : 0;
        int count = 0;
        for (uint32_t f0 = 0; f0 < total; f0 += 64) {
            const uint32_t f = f0 + (uint32_t)lane;
            const uint32_t gv = divpop.div(f);
            const int32_t shared_node = __shfl(lane_node, (int)(gv & 63u));
            bool mut = false;
            uint32_t r = 0, key = 0;
            if (f < total) {
                const uint32_t j = f - gv * (uint32_t)pop;
                const int32_t node = G <= 64 ? shared_node : list[base + (int)gv];
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
        // The group's node ids, degrees and neighbour lists, staged once in the free part of
        // the queue (when it has room: not when nearly every pair mutates), so that the
        // gathers below read neighbour ids from LDS instead of requesting each node's
        // adjacency line again for every neighbour position (k_mutate_lanes<16> 1034 -> 911
        // us, <32> 593 -> 510 us at |V| = 1M, pop 100).
        LDSP int32_t *s_node = (LDSP int32_t *)&items[wv][count];
        LDSP int32_t *s_rs = s_node + gn, *s_deg = s_rs + gn, *s_nbr = s_deg + gn;
        const bool staged = count + (gn * (KMAX + 3) + 1) / 2 <= MUT_LIST_CAP;
        if (staged) {
            for (int t = lane; t < gn; t += 64) {
                const int32_t v = t < 64 ? lane_node : list[base + t];
                const int32_t rs = g.row_ptr[v];
                s_node[t] = v;
                s_rs[t] = rs;
                s_deg[t] = g.row_ptr[v + 1] - rs;
            }
            wave_lds_sync();
            for (int t = lane; t < gn * KMAX; t += 64) {
                const int gv = t / KMAX, k = t % KMAX;
                s_nbr[t] = k < s_deg[gv] ? g.col[s_rs[gv] + k] : 0;
            }
            wave_lds_sync();
        }
        for (int b = 0; b < count; b += 64) {
            const int idx = b + lane;
            const bool has = idx < count;
            const uint2 it = has ? items[wv][idx] : make_uint2(0u, 0u);
            const int gv = (int)(it.x >> 16);
            const int j = (int)(it.x & 0xFFFFu);
            // plurality of the item's d neighbour labels, the register array sized per batch
            auto resolve = [&](auto nbr, int d) {
                if constexpr (KMAX == 16) {
                    const int dmax = wave_max(d);
                    if (dmax <= 4) return lane_plurality<4>(C, c.ld, j, nbr, d, it.y);
                    if (dmax <= 8) return lane_plurality<8>(C, c.ld, j, nbr, d, it.y);
                    return lane_plurality<16>(C, c.ld, j, nbr, d, it.y);
                } else {
                    return lane_plurality<KMAX>(C, c.ld, j, nbr, d, it.y);
                }
            };
            int32_t node;
            int res;
            if (staged) {
                node = s_node[gv];
                res = resolve(s_nbr + gv * KMAX, has ? s_deg[gv] : 0);
            } else {
                node = list[base + gv];
                const int32_t rs = g.row_ptr[node];
                res = resolve(g.col + rs, has ? g.row_ptr[node + 1] - rs : 0);
            }
            if (has) q_next[(size_t)node * c.ld + j] = res;
        }
        wave_lds_sync();
    }
}

// One item per wave: the d <= 64E neighbour labels sit E per lane at positions
// p = lane + 64k, are sorted across the wave with a bitonic network (partners in other
// lanes via shuffles, in the same lane via register swaps), and the plurality is read off
// the runs with ballots.
template <int E>
__device__ __forceinline__ void wave_bitonic(int (&a)[E])
{
    const int lane = lane_id();
#pragma unroll
    for (int kk = 2; kk <= 64 * E; kk <<= 1) {
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            if (jj >= 64) {
                const int js = jj / 64;
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int kp = k ^ js;
                    if (kp > k) {
                        const bool up = ((64 * k) & kk) == 0;
                        const int x = a[k], y = a[kp];
                        a[k] = up ? min(x, y) : max(x, y);
                        a[kp] = up ? max(x, y) : min(x, y);
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int p = lane + 64 * k;
                    const int y = __shfl_xor(a[k], jj);
                    const bool up = (p & kk) == 0;
                    const bool lower = (lane & jj) == 0;
                    a[k] = (lower == up) ? min(a[k], y) : max(a[k], y);
                }
            }
        }
    }
}

// Plurality of the d labels a[] holds (position lane + 64k, INT_MAX beyond d); sorts a.
template <int E>
__device__ __forceinline__ int wave_resolve(int (&a)[E], int d, uint32_t r)
{
    const int lane = lane_id();
    wave_bitonic<E>(a);
    uint64_t St[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int p = lane + 64 * k;
        int prev = __shfl_up(a[k], 1);
        if (k > 0) {
            const int wrap = __shfl(a[k - 1], 63);
            if (lane == 0) prev = wrap;
        }
        St[k] = __ballot(p < d && (p == 0 || a[k] != prev));
    }
    const uint64_t above = lane == 63 ? 0ull : (~0ull << (lane + 1));
    int len[E];
    int mybest = 0;
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int p = lane + 64 * k;
        int end = d;
        const uint64_t rest = St[k] & above;
        if (rest) {
            end = 64 * k + __builtin_ctzll(rest);
        } else {
#pragma unroll
            for (int k2 = E - 1; k2 > k; --k2)
                if (St[k2]) end = 64 * k2 + __builtin_ctzll(St[k2]);
        }
        end = min(end, d);
        len[k] = ((St[k] >> lane) & 1ull) ? end - p : 0;
        mybest = max(mybest, len[k]);
    }
    const int best = wave_max(mybest);
    uint64_t Tm[E];
    int nt = 0;
#pragma unroll
    for (int k = 0; k < E; ++k) {
        Tm[k] = __ballot(len[k] == best);
        nt += __popcll(Tm[k]);
    }
    int want = nt > 1 ? (int)pick(r, (uint32_t)nt) : 0;
    int res = 0;
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int c = __popcll(Tm[k]);
        if (want >= 0 && want < c) {
            const bool sel = ((Tm[k] >> lane) & 1ull) && lanes_below(Tm[k]) == want;
            const int src = __builtin_ctzll(__ballot(sel));
            res = __shfl(a[k], src);
        }
        want -= c;
    }
    return res;
}

// Degree class (64(E/2), 64E]: a wave takes one node and a slice of its offspring, draws
// their MUT words, queues the mutating ones in LDS and resolves them in batches: the labels
// of a batch's items are gathered together (each lane reads the batch's columns of one
// neighbour row back to back, so a row line is fetched once per batch, not once per item),
// then each item is sorted and resolved in turn.
//
// Waves per node in the wave classes: a node's offspring are split into this many slices so
// that one wave resolves about `per` mutations (a node has pop * M_P of them on average). One
// wave per node left the few high-degree nodes' waves resolving ten or more wave-wide sorts
// one after another while the rest of the chip idled. The count is a power of two up to
// MUT_WAVES, so all slices of a node fall in one workgroup and its waves read the node's
// neighbour rows at the same time, through one L2, instead of from up to three XCDs.
__host__ __device__ inline int mut_slices(int cls, int pop, uint64_t thr_m)
{
    if (cls < 2) return 1;
    const int per = cls == 2 ? 8 : (cls == 3 ? 4 : (cls == 4 ? 2 : 1));
    const int expect = (int)(((uint64_t)pop * thr_m) >> 32);  // floor(pop * M_P)
    int sl = 1;
    while (sl < MUT_WAVES && sl * 2 <= expect / per && sl * 2 <= pop) sl *= 2;
    return sl;
}

// items per gather batch: B x E labels held per lane
template <int E>
struct WaveBatch {
    static constexpr int B = E <= 4 ? 8 : (E == 8 ? 4 : (E == 16 ? 2 : 1));
};

template <int E>
__global__ __launch_bounds__(256) void k_mutate_wave(Span sp, int cls)
{
    int lb, nblk;
    const Item &it = sp.items[item_of(sp, lb, nblk)];
    const GGraph g = gview(it.g);
    const GaConst c = it.c;
    const GState st = gview(it.st);
    const GLB int32_t *__restrict__ C = glb(it.C);
    GLB int32_t *__restrict__ q_next = glb(it.q_next);
    const int32_t cstart = cls == 0 ? 0 : it.g.class_end[cls - 1];
    const GLB int32_t *__restrict__ list = g.small_nodes + cstart;
    const int32_t count_nodes = it.g.class_end[cls] - cstart;
    __shared__ uint2 items[MUT_WAVES][HPMOCD_MAX_POP_DEV];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = lane_id();
    const uint32_t gen = (uint32_t)*st.gen;
    const int pop = c.pop, ld = c.ld;
    const int slices = mut_slices(cls, pop, c.thr_m);
    const int span = (pop + slices - 1) / slices;
    const int units = count_nodes * slices;  // (node, slice of its offspring)
    for (int t = lb * MUT_WAVES + wv; t < units; t += nblk * MUT_WAVES) {
        const int32_t node = list[t / slices];
        const int jlo = (t % slices) * span, jhi = min(pop, jlo + span);
        const int32_t rs = g.row_ptr[node];
        const int d = g.row_ptr[node + 1] - rs;
        const GLB int32_t *nbr = g.col + rs;
        int count = 0;
        for (int j0 = jlo; j0 < jhi; j0 += 64) {
            const int j = j0 + lane;
            bool mut = false;
            uint32_t r = 0;
            if (j < jhi) {
                const u32x4 w = philox(c.seed, (uint32_t)node, (uint32_t)j, gen, TAG_MUT);
                mut = (uint64_t)w.a < c.thr_m;
                r = w.b;
            }
            const uint64_t bal = __ballot(mut);
            if (mut) items[wv][count + lanes_below(bal)] = make_uint2((uint32_t)j, r);
            count += __popcll(bal);
        }
        wave_lds_sync();
        constexpr int B = WaveBatch<E>::B;
        // the node's neighbour ids: for E <= 2 read once for all its batches (a node's
        // mutations span two batches of 8 there); wider classes reload them per batch rather
        // than hold E more registers
        constexpr int EH = E <= 2 ? E : 1;
        int32_t nid[EH];
#pragma unroll
        for (int k = 0; k < EH; ++k) nid[k] = (E <= 2 && lane + 64 * k < d) ? nbr[lane + 64 * k] : 0;
        for (int i0 = 0; i0 < count; i0 += B) {
            const int nb = min(B, count - i0);
            int jb[B];
#pragma unroll
            for (int b = 0; b < B; ++b) jb[b] = b < nb ? (int)items[wv][i0 + b].x : 0;
            int a[B][E];
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int p = lane + 64 * k;
                int32_t id;
                if constexpr (E <= 2)
                    id = nid[k];
                else
                    id = p < d ? nbr[p] : 0;
                const size_t row = (size_t)id * ld;
#pragma unroll
                for (int b = 0; b < B; ++b) a[b][k] = (p < d && b < nb) ? C[row + jb[b]] : INT_MAX;
            }
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (b < nb) {
                    const int out = wave_resolve<E>(a[b], d, items[wv][i0 + b].y);
                    if (lane == 0) q_next[(size_t)node * ld + jb[b]] = out;
                }
            }
        }
        wave_lds_sync();
    }
}

// Nodes above the wave classes: a workgroup per node; its four waves take the node's
// mutating offspring in turn, each sorting the neighbour labels in its own LDS buffer
// (bitonic), then reading the plurality off the runs.
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

// plurality of d labels sorted ascending in buf (wave-cooperative)
__device__ int sorted_plurality(const int *buf, int d, uint32_t r, int *res_slot)
{
    const int lane = lane_id();
    int mybest = 0;
    for (int i = lane; i < d; i += 64)
        if (i == 0 || buf[i] != buf[i - 1]) mybest = max(mybest, upper_bound_lds(buf, i, d, buf[i]) - i);
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
            if (q && lanes_below(bal) == want) *res_slot = buf[i];
            break;
        }
        want -= cntq;
    }
    wave_lds_sync();
    return *res_slot;
}

// exact plurality by walking the distinct labels in ascending order (any degree, slow)
__device__ int scan_plurality(const GLB int32_t *__restrict__ C, int ld, int j,
                              const GLB int32_t *__restrict__ nbr, int d, uint32_t r)
{
    const int lane = lane_id();
    int best = 0, nt = 0, prev = -1;
    for (;;) {
        int mn = INT_MAX;
        for (int i = lane; i < d; i += 64) {
            const int x = C[(size_t)nbr[i] * ld + j];
            if (x > prev) mn = min(mn, x);
        }
        mn = wave_min(mn);
        if (mn == INT_MAX) break;
        int cn = 0;
        for (int i = lane; i < d; i += 64) cn += C[(size_t)nbr[i] * ld + j] == mn;
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
            const int x = C[(size_t)nbr[i] * ld + j];
            if (x > prev) mn = min(mn, x);
        }
        mn = wave_min(mn);
        if (mn == INT_MAX) break;
        int cn = 0;
        for (int i = lane; i < d; i += 64) cn += C[(size_t)nbr[i] * ld + j] == mn;
        cn = wave_sum(cn);
        if (cn == best) {
            if (seen == want) return mn;
            ++seen;
        }
        prev = mn;
    }
    return prev;  // not reached
}

__global__ __launch_bounds__(128) void k_mutate_large(Span sp, int pmax)
{
    int lb, nblk;
    const Item &it = sp.items[item_of(sp, lb, nblk)];
    const GGraph g = gview(it.g);
    const GaConst c = it.c;
    const GState st = gview(it.st);
    const GLB int32_t *__restrict__ C = glb(it.C);
    GLB int32_t *__restrict__ q_next = glb(it.q_next);
    extern __shared__ int lds[];
    uint2 *items = (uint2 *)lds;                    // [pop]
    int *res = lds + 2 * HPMOCD_MAX_POP_DEV;        // [MUT_WAVES]
    int *cnt_sh = res + MUT_WAVES;                  // [1]
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = lane_id();
    const int nwaves = (int)(blockDim.x >> 6);
    int *buf = cnt_sh + 4 + wv * pmax;              // [pmax] per wave
    const uint32_t gen = (uint32_t)*st.gen;
    const int pop = c.pop, ld = c.ld;
    for (int t = lb; t < g.n_large; t += nblk) {
        const int32_t node = g.large_nodes[t];
        const int32_t rs = g.row_ptr[node];
        const int d = g.row_ptr[node + 1] - rs;
        const GLB int32_t *nbr = g.col + rs;
        if (threadIdx.x == 0) *cnt_sh = 0;
        __syncthreads();
        for (int j = threadIdx.x; j < pop; j += blockDim.x) {
            const u32x4 w = philox(c.seed, (uint32_t)node, (uint32_t)j, gen, TAG_MUT);
            if ((uint64_t)w.a < c.thr_m) items[atomicAdd(cnt_sh, 1)] = make_uint2((uint32_t)j, w.b);
        }
        __syncthreads();
        const int count = *cnt_sh;
        for (int it = wv; it < count; it += nwaves) {
            const int j = (int)items[it].x;
            const uint32_t r = items[it].y;
            int out;
            if (d <= pmax) {
                int P = 64;
                while (P < d) P <<= 1;
                for (int i = lane; i < P; i += 64) buf[i] = i < d ? C[(size_t)nbr[i] * ld + j] : INT_MAX;
                wave_lds_sync();
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
                        wave_lds_sync();
                    }
                out = sorted_plurality(buf, d, r, res + wv);
            } else {
                out = scan_plurality(C, ld, j, nbr, d, r);
            }
            if (lane == 0) q_next[(size_t)node * ld + j] = out;
            wave_lds_sync();
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// front extraction, eval-path helpers
// ---------------------------------------------------------------------------------------
// Front rows ids[0..k) of a population (id < pop: column id of pool, else column id - pop of
// q) into individual-major out[k][n]. A workgroup moves EX_NODES nodes x EX_ROWS rows through
// LDS: first each lane takes one row and the waves walk the nodes, so that one wave's loads
// fall in a node's two label rows; then each lane takes one node and the waves walk the
// rows, so that every store writes EX_NODES consecutive labels of one output row. (One
// thread per output label, each reading its 4-byte label from its own line, took 1.83 ms for
// a 100 x 1M front; this takes 0.36 ms.)
constexpr int EX_NODES = 64, EX_ROWS = 128, EX_THREADS = 256;

__global__ __launch_bounds__(EX_THREADS) void k_extract(int32_t n, int32_t ld, int32_t pop,
                                                        const int32_t *__restrict__ pool,
                                                        const int32_t *__restrict__ q,
                                                        const int32_t *__restrict__ ids, int32_t k,
                                                        const int32_t *__restrict__ k_dev,
                                                        int32_t *__restrict__ out)
{
    __shared__ int32_t tile[EX_ROWS][EX_NODES + 1];  // +1: lanes of phase 1 hit distinct banks
    const int kk = k_dev ? min(k, *k_dev) : k;  // rows beyond the device-side count hold nothing
    const int r0 = blockIdx.y * EX_ROWS;
    if (r0 >= kk) return;
    const int64_t v0 = (int64_t)blockIdx.x * EX_NODES;
    const int nv = (int)min((int64_t)EX_NODES, (int64_t)n - v0);
    {
        constexpr int GROUPS = EX_THREADS / EX_ROWS;
        const int rr = threadIdx.x % EX_ROWS, grp = threadIdx.x / EX_ROWS;
        if (r0 + rr < kk) {
            const int id = ids[r0 + rr];
            const int32_t *src = (id < pop ? pool + id : q + (id - pop)) + (size_t)v0 * ld;
            for (int t = grp; t < nv; t += GROUPS) tile[rr][t] = src[(size_t)t * ld];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x % EX_NODES;
    const int rows = min(EX_ROWS, kk - r0);
    if (lane < nv)
        for (int rr = threadIdx.x / EX_NODES; rr < rows; rr += EX_THREADS / EX_NODES)
            out[(size_t)(r0 + rr) * n + v0 + lane] = tile[rr][lane];
}

hipError_t launch_extract(int32_t n, int32_t ld, int32_t pop, const int32_t *pool,
                          const int32_t *q, const int32_t *ids, int32_t k, int32_t *out,
                          hipStream_t s, const int32_t *k_dev)
{
    if (k == 0 || n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + EX_NODES - 1) / EX_NODES), (unsigned)((k + EX_ROWS - 1) / EX_ROWS));
    k_extract<<<grid, EX_THREADS, 0, s>>>(n, ld, pop, pool, q, ids, k, k_dev, out);
    return hipGetLastError();
}

// rows [n_ind][n] -> node-major [n][ld] through LDS, 64 individuals x 64 nodes per 256-thread
// workgroup: each wave reads one individual's 256-byte run of 64 labels per step and writes
// one node's 64 columns. With `bad`, a label outside [0, n) is stored as 0 (the kernels
// downstream index by label) and *bad set to 1.
__global__ __launch_bounds__(256) void k_transpose_in(const int32_t *__restrict__ rows, int32_t n,
                                                      int32_t n_ind, int32_t ld,
                                                      int32_t *__restrict__ out,
                                                      int32_t *__restrict__ bad)
{
    __shared__ int tile[64][65];
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int i0 = blockIdx.y * 64;
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    bool seen_bad = false;
    for (int r = w; r < 64; r += 4) {
        const int i = i0 + r;
        const int64_t v = v0 + lane;
        if (i < n_ind && v < n) {
            int32_t x = rows[(size_t)i * n + v];
            if (bad && (x < 0 || x >= n)) {
                seen_bad = true;
                x = 0;
            }
            tile[r][lane] = x;
        }
    }
    if (seen_bad) *bad = 1;
    __syncthreads();
    for (int r = w; r < 64; r += 4) {
        const int64_t v = v0 + r;
        const int i = i0 + lane;
        if (i < n_ind && v < n) out[(size_t)v * ld + i] = tile[lane][r];
    }
}

hipError_t launch_transpose_in(const int32_t *rows, int32_t n, int32_t n_ind, int32_t ld,
                               int32_t *out, int32_t *bad, hipStream_t s)
{
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((n_ind + 63) / 64));
    k_transpose_in<<<grid, 256, 0, s>>>(rows, n, n_ind, ld, out, bad);
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

namespace hpm {

// ---------------------------------------------------------------------------------------
// launch geometry of every kind, per item (host side)
// ---------------------------------------------------------------------------------------
static int32_t ceil_div(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

static int32_t large_pmax(const Item &it)
{
    int pmax = 64;
    while (pmax < it.g.large_max_deg && pmax < LARGE_SORT_CAP) pmax <<= 1;
    return pmax;
}

int32_t kind_blocks(Kind k, const Item &it)
{
    const DevGraph &g = it.g;
    switch (k) {
    case K_INIT: return ceil_div(g.n, NODE_BLOCK);
    case K_FIT: return ceil_div((int64_t)ceil_div(g.n, it.fit_npw) * ((it.fit_pop + 127) / 128), FIT_WAVES);
    case K_BIN: {
        if (!it.hp.enabled) return 0;
        // as many workgroups as fit at once: 256 of 1024 threads, more of fewer
        const int32_t threads = (it.hp.nb + 63) / 64 * 64;
        return std::min(it.hp.nchunks * it.hp.ngroups, BIN_RESIDENT * (BIN_THREADS / threads));
    }
    case K_HIST: return it.hp.enabled ? it.hp.tiles * it.fit_pop : 0;
    case K_CLEAR: {
        if (it.hp.enabled) return 0;
        const int32_t b = ceil_div((int64_t)(it.D_bytes / 16), 256);
        return b < 1 ? 1 : (b > 2048 ? 2048 : b);
    }
    case K_ONE: return 1;
    case K_XO: return ceil_div(g.n, it.xo_nb);
    case K_MUTL:
        if (it.c.thr_m == 0 || g.n_large == 0) return 0;
        return g.n_large < 8192 ? g.n_large : 8192;
    default: break;
    }
    const int cls = (int)k - (int)K_MUT0;
    if (cls < 0 || cls >= N_DEG_CLASSES || it.c.thr_m == 0) return 0;
    const int32_t start = cls == 0 ? 0 : it.g.class_end[cls - 1];
    const int32_t cnt = it.g.class_end[cls] - start;
    if (cnt <= 0) return 0;
    if (DEG_CLASS_MAX[cls] <= 32) {
        const int32_t b = ceil_div(ceil_div(cnt, it.c.mut_group), MUT_WAVES);
        return b > 8192 ? 8192 : b;
    }
    const int32_t b = ceil_div((int64_t)cnt * mut_slices(cls, it.c.pop, it.c.thr_m), MUT_WAVES);
    return b > 16384 ? 16384 : b;
}

size_t kind_lds(Kind k, const Item &it)
{
    switch (k) {
    case K_FIT: return sizeof(unsigned long long) * (size_t)it.fit_ld * (it.hp.enabled ? 1 : 2);
    case K_BIN:
        return it.hp.enabled ? sizeof(uint32_t) * ((size_t)it.hp.tiles * HB_CG + 1 +
                                                   (size_t)it.hp.nb * HB_CG + BIN_THREADS / 64 +
                                                   (size_t)it.hp.nb)
                             : 0;
    case K_HIST: return it.hp.enabled ? sizeof(uint32_t) * ((size_t)1 << it.hp.rbits) : 0;
    case K_XO:
        return sizeof(int) * ((size_t)xo_table_ints(it.c.pop, it.c.es) + 2 * (size_t)it.xo_nb * it.c.ld);
    case K_MUTL:
        return sizeof(int) * (2 * (size_t)HPMOCD_MAX_POP_DEV + MUT_WAVES + 4 +
                              2 * (size_t)large_pmax(it));
    default: return 0;
    }
}

int32_t kind_aux(Kind k, const Item &it)
{
    if (k == K_XO) return it.c.es;
    if (k == K_BIN) return it.hp.enabled ? (it.hp.nb + 63) / 64 * 64 : 0;  // threads
    if (k == K_MUTL) return large_pmax(it);
    return 0;
}

hipError_t launch_kind(Kind k, const Span &sp, int32_t blocks, size_t lds, int32_t aux,
                       hipStream_t s)
{
    if (blocks <= 0) return hipSuccess;
    const unsigned nb = (unsigned)blocks;
    switch (k) {
    case K_INIT: k_init<<<nb, 256, 0, s>>>(sp); break;
    case K_FIT: k_fitness<<<nb, 64 * FIT_WAVES, lds, s>>>(sp); break;
    case K_BIN: {
        const unsigned threads = (unsigned)(aux < 64 ? 64 : (aux > BIN_THREADS ? BIN_THREADS : aux));
        k_bin<<<nb, threads, lds, s>>>(sp);
        break;
    }
    case K_HIST: k_hist<<<nb, 256, lds, s>>>(sp); break;
    case K_CLEAR: k_clear<<<nb, 256, 0, s>>>(sp); break;
    case K_XO:
        switch (aux) {
        case 1: k_crossover<1><<<nb, 256, lds, s>>>(sp); break;
        case 2: k_crossover<2><<<nb, 256, lds, s>>>(sp); break;
        case 3: k_crossover<3><<<nb, 256, lds, s>>>(sp); break;
        case 4: k_crossover<4><<<nb, 256, lds, s>>>(sp); break;
        case 5: k_crossover<5><<<nb, 256, lds, s>>>(sp); break;
        case 6: k_crossover<6><<<nb, 256, lds, s>>>(sp); break;
        case 7: k_crossover<7><<<nb, 256, lds, s>>>(sp); break;
        case 8: k_crossover<8><<<nb, 256, lds, s>>>(sp); break;
        default: return hipErrorInvalidValue;
        }
        break;
    case K_MUTL: k_mutate_large<<<nb, 128, lds, s>>>(sp, aux); break;
    default: {
        const int cls = (int)k - (int)K_MUT0;
        switch (cls) {
        case 0: k_mutate_lanes<16, MUT_WAVES><<<nb, 64 * MUT_WAVES, 0, s>>>(sp, cls); break;
        case 1: k_mutate_lanes<32, MUT_WAVES><<<nb, 64 * MUT_WAVES, 0, s>>>(sp, cls); break;
        case 2: k_mutate_wave<1><<<nb, 64 * MUT_WAVES, 0, s>>>(sp, cls); break;
        case 3: k_mutate_wave<2><<<nb, 64 * MUT_WAVES, 0, s>>>(sp, cls); break;
        case 4: k_mutate_wave<4><<<nb, 64 * MUT_WAVES, 0, s>>>(sp, cls); break;
        case 5: k_mutate_wave<8><<<nb, 64 * MUT_WAVES, 0, s>>>(sp, cls); break;
        case 6: k_mutate_wave<16><<<nb, 64 * MUT_WAVES, 0, s>>>(sp, cls); break;
        case 7: k_mutate_wave<32><<<nb, 64 * MUT_WAVES, 0, s>>>(sp, cls); break;
        default: return hipErrorInvalidValue;
        }
    }
    }
    return hipGetLastError();
}

}  // namespace hpm
