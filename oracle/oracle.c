/*
 * HP-MOCD reference oracle: a plain, serial, obviously-correct CPU implementation of the
 * NSGA-II community search of "A High-Performance Evolutionary Multiobjective Community
 * Detection Algorithm" (HP-MOCD, arXiv 2506.01752).
 *
 * THIS FILE IS TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it. The product path (the HIP library) never calls it and shares
 * no code with it: this file has its own Philox, its own evaluation, its own sorting.
 *
 * Precision: every count is an exact integer (int64); the two objectives are each one IEEE
 * binary64 division of exact integers; crowding distance is binary64 subtraction, division
 * and addition in a fixed order. Build with -ffp-contract=off and without fast-math.
 *
 * Readings of points the paper leaves open (each one is listed in the design notes):
 *  - objectives as exact numerators: f1 = (2m - A) / 2m, f2 = S / (2m)^2 (section 4.1, eq.
 *    "objectives"), with A = number of intra-community arcs (= 2 * sum_c |E(c)|) and
 *    S = sum_c (sum_{v in c} deg v)^2;
 *  - counter-based randomness: Philox4x32-10, key = seed, counter = (x, individual,
 *    generation, tag); range draw pick(r, k) = (r * k) >> 32; Bernoulli(p) = r < floor(p 2^32);
 *  - initialisation: each node takes its own id or the id of a uniformly drawn neighbour
 *    (the paper only says "random partitions"; parity unpinned);
 *  - tournament: binary, with replacement, under the crowded-comparison order;
 *  - crossover: ensemble of E_S parents, gate r < thr(C_P) (section 4.3.1, eq. "arg_max");
 *    ties broken by an index drawn over the tied labels in ascending order;
 *  - mutation: synchronous over the post-crossover child, neighbours only, same tie rule
 *    (section 4.3.2);
 *  - dominance on exact integer keys (2m - A, S), which orders exactly like (f1, f2);
 *  - crowding distance per front after Deb et al. 2002, +inf at both ends and for fronts of
 *    at most two members, nothing added when an objective's range is zero;
 *  - order: rank ascending, crowding descending, position ascending.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
static int thread_id(void) { return omp_get_thread_num(); }
#else
static int thread_id(void) { return 0; }
#endif

#define OR_TAG_INIT 0u
#define OR_TAG_SEL 1u
#define OR_TAG_XOV 2u
#define OR_TAG_MUT 3u
#define OR_GATE_X 0xFFFFFFFFu

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10, written from Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as */
/* easy as 1, 2, 3" (SC'11): each round multiplies counter words 0 and 2 by two fixed       */
/* 32-bit constants, xors the high halves with the other two words and the key, and swaps; */
/* the key is bumped by the two Weyl constants between rounds.                             */
/* ------------------------------------------------------------------------------------ */
void or_philox(uint64_t seed, uint32_t x, uint32_t ind, uint32_t gen, uint32_t tag,
               uint32_t out[4])
{
    uint32_t c0 = x, c1 = ind, c2 = gen, c3 = tag;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform index in [0, k) from a 32-bit draw: floor(r * k / 2^32) */
uint32_t or_pick(uint32_t r, uint32_t k) { return (uint32_t)(((uint64_t)r * (uint64_t)k) >> 32); }

/* Bernoulli threshold: the event is r < thr(p) */
uint64_t or_thr(double p)
{
    if (p >= 1.0) return (uint64_t)1 << 32;
    if (p <= 0.0) return 0;
    return (uint64_t)floor(p * 4294967296.0);
}

/* ------------------------------------------------------------------------------------ */
/* Graph: symmetric CSR; the oracle keeps its own copy with every adjacency list sorted.    */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    int64_t m2; /* number of arcs = 2|E| */
    int32_t *row_ptr;
    int32_t *col;
} or_graph;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void graph_copy(or_graph *g, int32_t n, const int32_t *row_ptr, const int32_t *col)
{
    g->n = n;
    g->m2 = row_ptr[n];
    g->row_ptr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->m2 > 0 ? g->m2 : 1));
    memcpy(g->row_ptr, row_ptr, sizeof(int32_t) * (size_t)(n + 1));
    if (g->m2 > 0) memcpy(g->col, col, sizeof(int32_t) * (size_t)g->m2);
    for (int32_t v = 0; v < n; ++v)
        qsort(g->col + g->row_ptr[v], (size_t)(g->row_ptr[v + 1] - g->row_ptr[v]),
              sizeof(int32_t), cmp_i32);
}

static void graph_free(or_graph *g)
{
    free(g->row_ptr);
    free(g->col);
}

/* ------------------------------------------------------------------------------------ */
/* Evaluation (section 4.1, eq. "objectives").                                            */
/*   A  = #{arcs (v,u) : L[u] == L[v]}            (twice the intra-community edge count)  */
/*   D_c = sum_{v : L[v] == c} deg(v);  S = sum_c D_c^2                                    */
/*   f1 = (2m - A) / 2m  (= 1 - sum_c |E(c)| / m),  f2 = S / (2m)^2                        */
/* ------------------------------------------------------------------------------------ */
static void eval_graph(const or_graph *g, const int32_t *lab, int64_t *D, int64_t *A_out,
                       int64_t *S_out, double *f1, double *f2)
{
    int64_t A = 0;
    for (int32_t v = 0; v < g->n; ++v)
        for (int32_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e)
            if (lab[g->col[e]] == lab[v]) ++A;
    memset(D, 0, sizeof(int64_t) * (size_t)g->n);
    for (int32_t v = 0; v < g->n; ++v) D[lab[v]] += g->row_ptr[v + 1] - g->row_ptr[v];
    int64_t S = 0;
    for (int32_t c = 0; c < g->n; ++c) S += D[c] * D[c];
    *A_out = A;
    *S_out = S;
    *f1 = (double)(g->m2 - A) / (double)g->m2;
    *f2 = (double)S / (double)(g->m2 * g->m2);
}

void or_eval(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *lab,
             int64_t *A, int64_t *S, double *f1, double *f2)
{
    or_graph g;
    graph_copy(&g, n, row_ptr, col);
    int64_t *D = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    eval_graph(&g, lab, D, A, S, f1, f2);
    free(D);
    graph_free(&g);
}

/* k partitions (k x n, row-major) against one copy of the graph */
void or_eval_batch(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *lab,
                   int32_t k, int64_t *A, int64_t *S, double *f1, double *f2)
{
    or_graph g;
    graph_copy(&g, n, row_ptr, col);
    int64_t *D = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < k; ++i)
        eval_graph(&g, lab + (size_t)i * (size_t)n, D, A + i, S + i, f1 + i, f2 + i);
    free(D);
    graph_free(&g);
}

/* ------------------------------------------------------------------------------------ */
/* Plurality with a random tie-break (eq. "arg_max"): among vals[0..k), take the labels of */
/* maximal multiplicity, in ascending order, and return the one at index pick(r, #ties).   */
/* `vals` is sorted in place. The draw r is only needed when there is a tie, so it is      */
/* produced by a callback; being counter-based, drawing it lazily changes nothing.         */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;
    uint32_t x, ind, gen, tag;
    int lane; /* which 32-bit output word is the tie-break draw */
} draw_spec;

static uint32_t draw(const draw_spec *d)
{
    uint32_t w[4];
    or_philox(d->seed, d->x, d->ind, d->gen, d->tag, w);
    return w[d->lane];
}

static int32_t plurality(int32_t *vals, int32_t k, const draw_spec *tie)
{
    qsort(vals, (size_t)k, sizeof(int32_t), cmp_i32);
    int32_t best = 0, nties = 0;
    for (int32_t i = 0; i < k;) {
        int32_t j = i;
        while (j < k && vals[j] == vals[i]) ++j;
        if (j - i > best) {
            best = j - i;
            nties = 1;
        } else if (j - i == best) {
            ++nties;
        }
        i = j;
    }
    int32_t want = nties == 1 ? 0 : (int32_t)or_pick(draw(tie), (uint32_t)nties);
    for (int32_t i = 0, seen = 0; i < k;) {
        int32_t j = i;
        while (j < k && vals[j] == vals[i]) ++j;
        if (j - i == best) {
            if (seen == want) return vals[i];
            ++seen;
        }
        i = j;
    }
    return -1; /* unreachable for k > 0 */
}

/* ------------------------------------------------------------------------------------ */
/* Initialisation (Alg. 1, InitializePopulation): node v of individual i takes a uniform   */
/* choice among {its sorted neighbours} followed by {itself}.                               */
/* ------------------------------------------------------------------------------------ */
static void init_individual(const or_graph *g, uint64_t seed, int32_t i, int32_t *lab)
{
    uint32_t w[4];
    for (int32_t v = 0; v < g->n; ++v) {
        int32_t d = g->row_ptr[v + 1] - g->row_ptr[v];
        or_philox(seed, (uint32_t)v, (uint32_t)i, 0u, OR_TAG_INIT, w);
        uint32_t j = or_pick(w[0], (uint32_t)d + 1u);
        lab[v] = (j == (uint32_t)d) ? v : g->col[g->row_ptr[v] + (int32_t)j];
    }
}

void or_init_individual(int32_t n, const int32_t *row_ptr, const int32_t *col, uint64_t seed,
                        int32_t i, int32_t *lab)
{
    or_graph g;
    graph_copy(&g, n, row_ptr, col);
    init_individual(&g, seed, i, lab);
    graph_free(&g);
}

/* ------------------------------------------------------------------------------------ */
/* Tournament selection (Alg. 1 TournamentSelection, size k = 2) for parent slot k of     */
/* offspring j at generation g. The population is already in crowded-comparison order     */
/* (rank ascending, crowding descending, position ascending), so of two contestants the   */
/* one at the lower position is the better one (equal positions: the same member). The   */
/* contestants are drawn independently and with replacement from the SEL draw of counter  */
/* (k, j, g). Returns the winner's position in [0, np).                                   */
/* ------------------------------------------------------------------------------------ */
int32_t or_tournament(uint64_t seed, uint32_t gen, uint32_t j, uint32_t k, int32_t np)
{
    uint32_t w[4];
    or_philox(seed, k, j, gen, OR_TAG_SEL, w);
    uint32_t a = or_pick(w[0], (uint32_t)np), b = or_pick(w[1], (uint32_t)np);
    return (int32_t)(a < b ? a : b);
}

/* ------------------------------------------------------------------------------------ */
/* Crossover gate (section 4.3.1, Alg. 2): a uniform x is drawn and the ensemble crossover */
/* happens when x <= C_P, i.e. with probability C_P; otherwise the child is a copy of one  */
/* of its E_S parents, chosen uniformly. x is the first word of the SEL draw of counter    */
/* (0xFFFFFFFF, j, g), read as the integer event w0 < floor(C_P 2^32); the second word      */
/* picks the copied parent. Returns -1 for crossover, else the copied parent slot.         */
/* ------------------------------------------------------------------------------------ */
int32_t or_gate(uint64_t seed, uint32_t gen, uint32_t j, double crossover_p, int32_t es)
{
    uint32_t w[4];
    or_philox(seed, OR_GATE_X, j, gen, OR_TAG_SEL, w);
    if ((uint64_t)w[0] < or_thr(crossover_p)) return -1;
    return (int32_t)or_pick(w[1], (uint32_t)es);
}

/* ------------------------------------------------------------------------------------ */
/* Crossover (section 4.3.1, Alg. 2) of offspring j at generation g from E_S parent rows.  */
/* gate_copy < 0: majority vote per node; gate_copy = k: copy of parent k.                 */
/* ------------------------------------------------------------------------------------ */
static void crossover(int32_t n, int32_t es, const int32_t *const *par, int32_t gate_copy,
                      uint64_t seed, uint32_t g, uint32_t j, int32_t *child)
{
    if (gate_copy >= 0) {
        memcpy(child, par[gate_copy], sizeof(int32_t) * (size_t)n);
        return;
    }
    int32_t vals[64];
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t k = 0; k < es; ++k) vals[k] = par[k][v];
        draw_spec tie = {seed, (uint32_t)v, j, g, OR_TAG_XOV, 0};
        child[v] = plurality(vals, es, &tie);
    }
}

void or_crossover(int32_t n, int32_t es, const int32_t *parents /* es x n */, int32_t gate_copy,
                  uint64_t seed, uint32_t g, uint32_t j, int32_t *child)
{
    const int32_t *rows[64];
    for (int32_t k = 0; k < es; ++k) rows[k] = parents + (size_t)k * (size_t)n;
    crossover(n, es, rows, gate_copy, seed, g, j, child);
}

/* ------------------------------------------------------------------------------------ */
/* Mutation (section 4.3.2): node v is selected when r0 < thr(M_P) and it has neighbours; */
/* it then takes the plurality label of its neighbours in the post-crossover child C      */
/* (own label not counted), ties broken with r1. Synchronous: all reads come from C.       */
/* ------------------------------------------------------------------------------------ */
int32_t or_neighbour_plurality(int32_t n, const int32_t *row_ptr, const int32_t *col,
                               const int32_t *C, int32_t v, uint64_t seed, uint32_t gen,
                               uint32_t j)
{
    (void)n;
    int32_t d = row_ptr[v + 1] - row_ptr[v];
    if (d == 0) return C[v];
    int32_t *vals = (int32_t *)malloc(sizeof(int32_t) * (size_t)d);
    for (int32_t e = 0; e < d; ++e) vals[e] = C[col[row_ptr[v] + e]];
    draw_spec tie = {seed, (uint32_t)v, j, gen, OR_TAG_MUT, 1};
    int32_t out = plurality(vals, d, &tie);
    free(vals);
    return out;
}

static void mutate(const or_graph *g, const int32_t *C, uint64_t thr, uint64_t seed, uint32_t gen,
                   uint32_t j, int32_t *out, int32_t *scratch)
{
    for (int32_t v = 0; v < g->n; ++v) {
        int32_t d = g->row_ptr[v + 1] - g->row_ptr[v];
        uint32_t w[4];
        or_philox(seed, (uint32_t)v, j, gen, OR_TAG_MUT, w);
        if ((uint64_t)w[0] < thr && d > 0) {
            for (int32_t e = 0; e < d; ++e) scratch[e] = C[g->col[g->row_ptr[v] + e]];
            draw_spec tie = {seed, (uint32_t)v, j, gen, OR_TAG_MUT, 1};
            out[v] = plurality(scratch, d, &tie);
        } else {
            out[v] = C[v];
        }
    }
}

void or_mutate(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *C,
               double mutation_p, uint64_t seed, uint32_t gen, uint32_t j, int32_t *out)
{
    or_graph g;
    graph_copy(&g, n, row_ptr, col);
    int32_t maxd = 1;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] - row_ptr[v] > maxd) maxd = row_ptr[v + 1] - row_ptr[v];
    int32_t *scratch = (int32_t *)malloc(sizeof(int32_t) * (size_t)maxd);
    mutate(&g, C, or_thr(mutation_p), seed, gen, j, out, scratch);
    free(scratch);
    graph_free(&g);
}

/* ------------------------------------------------------------------------------------ */
/* One offspring (Alg. 1 steps inside a generation): E_S tournaments over the population   */
/* P in crowded order (rows P[0..np)), the crossover gate, the crossover and the mutation. */
/* Writes the child to out and, when parent_pos is not NULL, the E_S winners' positions    */
/* and the gate's result.                                                                 */
/* ------------------------------------------------------------------------------------ */
static void offspring(const or_graph *g, const int32_t *const *P, int32_t np, int32_t es,
                      double crossover_p, uint64_t thr_m, uint64_t seed, uint32_t gen,
                      uint32_t j, int32_t *C, int32_t *scratch, int32_t *out,
                      int32_t *parent_pos, int32_t *gate_out)
{
    const int32_t *par[8];
    for (int32_t k = 0; k < es; ++k) {
        int32_t q = or_tournament(seed, gen, j, (uint32_t)k, np);
        par[k] = P[q];
        if (parent_pos) parent_pos[k] = q;
    }
    int32_t gate_copy = or_gate(seed, gen, j, crossover_p, es);
    if (gate_out) *gate_out = gate_copy;
    crossover(g->n, es, par, gate_copy, seed, gen, j, C);
    mutate(g, C, thr_m, seed, gen, j, out, scratch);
}

/* offspring j of generation gen from the population rows `pop` (np x n, crowded order) */
void or_offspring(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *pop,
                  int32_t np, int32_t es, double crossover_p, double mutation_p, uint64_t seed,
                  uint32_t gen, uint32_t j, int32_t *child, int32_t *parent_pos,
                  int32_t *gate_out)
{
    or_graph g;
    graph_copy(&g, n, row_ptr, col);
    int32_t maxd = 1;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] - row_ptr[v] > maxd) maxd = row_ptr[v + 1] - row_ptr[v];
    const int32_t **rows = (const int32_t **)malloc(sizeof(int32_t *) * (size_t)np);
    for (int32_t q = 0; q < np; ++q) rows[q] = pop + (size_t)q * (size_t)n;
    int32_t *scratch = (int32_t *)malloc(sizeof(int32_t) * (size_t)maxd);
    int32_t *C = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    offspring(&g, rows, np, es, crossover_p, or_thr(mutation_p), seed, gen, j, C, scratch,
              child, parent_pos, gate_out);
    free(C);
    free(scratch);
    free(rows);
    graph_free(&g);
}

/* ------------------------------------------------------------------------------------ */
/* Fast non-dominated sort (NSGA-II, Deb et al. 2002; Alg. 1 FastNonDominatedSort).        */
/* Objectives are minimised; dominance is read on the exact integer keys k1 = 2m - A,      */
/* k2 = S (section 2.2 definition of dominance). rank = 1 for the first front.             */
/* ------------------------------------------------------------------------------------ */
static int dominates(int64_t a1, int64_t a2, int64_t b1, int64_t b2)
{
    return a1 <= b1 && a2 <= b2 && (a1 < b1 || a2 < b2);
}

void or_rank(int32_t N, const int64_t *k1, const int64_t *k2, int32_t *rank)
{
    int32_t *ndom = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
    int32_t *front = (int32_t *)malloc(sizeof(int32_t) * ((size_t)N + 1));
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * ((size_t)N + 1));
    for (int32_t p = 0; p < N; ++p)
        for (int32_t q = 0; q < N; ++q)
            if (q != p && dominates(k1[q], k2[q], k1[p], k2[p])) ++ndom[p];
    int32_t nf = 0;
    for (int32_t p = 0; p < N; ++p)
        if (ndom[p] == 0) {
            rank[p] = 1;
            front[nf++] = p;
        }
    int32_t r = 1;
    while (nf > 0) {
        int32_t nn = 0;
        for (int32_t a = 0; a < nf; ++a) {
            int32_t p = front[a];
            for (int32_t q = 0; q < N; ++q)
                if (dominates(k1[p], k2[p], k1[q], k2[q]) && --ndom[q] == 0) {
                    rank[q] = r + 1;
                    next[nn++] = q;
                }
        }
        memcpy(front, next, sizeof(int32_t) * (size_t)nn);
        nf = nn;
        ++r;
    }
    free(ndom);
    free(front);
    free(next);
}

/* ------------------------------------------------------------------------------------ */
/* Crowding distance (NSGA-II, Deb et al. 2002; Alg. 1 CrowdingDistanceAssignment).        */
/* ------------------------------------------------------------------------------------ */
static const int64_t *g_sort_key;
static int cmp_key_pos(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_sort_key[x] != g_sort_key[y]) return g_sort_key[x] < g_sort_key[y] ? -1 : 1;
    return (x > y) - (x < y);
}

void or_crowding(int32_t N, const int32_t *rank, const int64_t *k1, const int64_t *k2,
                 const double *f1, const double *f2, double *crowd)
{
    int32_t *mem = (int32_t *)malloc(sizeof(int32_t) * ((size_t)N + 1));
    for (int32_t i = 0; i < N; ++i) crowd[i] = 0.0;
    int32_t maxr = 0;
    for (int32_t i = 0; i < N; ++i)
        if (rank[i] > maxr) maxr = rank[i];
    for (int32_t r = 1; r <= maxr; ++r) {
        int32_t l = 0;
        for (int32_t i = 0; i < N; ++i)
            if (rank[i] == r) mem[l++] = i;
        if (l == 0) continue;
        if (l <= 2) {
            for (int32_t a = 0; a < l; ++a) crowd[mem[a]] = INFINITY;
            continue;
        }
        for (int obj = 0; obj < 2; ++obj) {
            const int64_t *key = obj == 0 ? k1 : k2;
            const double *o = obj == 0 ? f1 : f2;
            g_sort_key = key;
            qsort(mem, (size_t)l, sizeof(int32_t), cmp_key_pos);
            double den = o[mem[l - 1]] - o[mem[0]];
            crowd[mem[0]] = INFINITY;
            crowd[mem[l - 1]] = INFINITY;
            if (den != 0.0)
                for (int32_t a = 1; a < l - 1; ++a)
                    crowd[mem[a]] = crowd[mem[a]] + (o[mem[a + 1]] - o[mem[a - 1]]) / den;
        }
    }
    free(mem);
}

/* ------------------------------------------------------------------------------------ */
/* Crowded-comparison order (Alg. 1 SortByRankAndDistance): rank ascending, crowding       */
/* descending, original position ascending. order[q] = index of the member at position q. */
/* ------------------------------------------------------------------------------------ */
static const int32_t *g_ord_rank;
static const double *g_ord_crowd;
static int cmp_crowded(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_ord_rank[x] != g_ord_rank[y]) return g_ord_rank[x] < g_ord_rank[y] ? -1 : 1;
    if (g_ord_crowd[x] > g_ord_crowd[y]) return -1;
    if (g_ord_crowd[x] < g_ord_crowd[y]) return 1;
    return (x > y) - (x < y);
}

void or_order(int32_t N, const int32_t *rank, const double *crowd, int32_t *order)
{
    for (int32_t i = 0; i < N; ++i) order[i] = i;
    g_ord_rank = rank;
    g_ord_crowd = crowd;
    qsort(order, (size_t)N, sizeof(int32_t), cmp_crowded);
}

/* ------------------------------------------------------------------------------------ */
/* The whole run (Alg. 1).                                                                */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t pop_size;
    int32_t generations;
    double crossover_p;
    double mutation_p;
    int32_t parents_per_child;
    uint64_t seed;
} or_params;

typedef struct {
    int32_t g, pop_size, n_nodes;
    const int32_t *labels; /* pop_size x n_nodes, P after environmental selection, in order */
    const int64_t *A, *S;
    const double *f1, *f2;
    const int32_t *rank;  /* rank of P^(g-1) members from the start of generation g (NULL at g=0) */
    const double *crowd;  /* crowding of the same (NULL at g=0); both in that reordered order */
} or_state_view;

typedef void (*or_callback)(const or_state_view *, void *);

typedef struct {
    int32_t *row; /* n labels */
    int64_t A, S;
    double f1, f2;
} member;

/* rank, crowd and order a set of members; returns order[] (caller frees) and rank/crowd of
 * each member in the original index space */
static int32_t *rank_crowd_order(const member *const *set, int32_t N, int64_t m2, int32_t *rank,
                                 double *crowd)
{
    int64_t *k1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int64_t *k2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    double *f1 = (double *)malloc(sizeof(double) * (size_t)N);
    double *f2 = (double *)malloc(sizeof(double) * (size_t)N);
    for (int32_t i = 0; i < N; ++i) {
        k1[i] = m2 - set[i]->A;
        k2[i] = set[i]->S;
        f1[i] = set[i]->f1;
        f2[i] = set[i]->f2;
    }
    or_rank(N, k1, k2, rank);
    or_crowding(N, rank, k1, k2, f1, f2, crowd);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    or_order(N, rank, crowd, order);
    free(k1);
    free(k2);
    free(f1);
    free(f2);
    return order;
}

static void emit(or_callback cb, void *user, int32_t g, int32_t n, const member *const *P,
                 int32_t np, const int32_t *rank, const double *crowd, int32_t *buf_lab,
                 int64_t *bA, int64_t *bS, double *bf1, double *bf2)
{
    for (int32_t i = 0; i < np; ++i) {
        memcpy(buf_lab + (size_t)i * (size_t)n, P[i]->row, sizeof(int32_t) * (size_t)n);
        bA[i] = P[i]->A;
        bS[i] = P[i]->S;
        bf1[i] = P[i]->f1;
        bf2[i] = P[i]->f2;
    }
    or_state_view s;
    s.g = g;
    s.pop_size = np;
    s.n_nodes = n;
    s.labels = buf_lab;
    s.A = bA;
    s.S = bS;
    s.f1 = bf1;
    s.f2 = bf2;
    s.rank = rank;
    s.crowd = crowd;
    cb(&s, user);
}

/* Returns 0 on success, -1 on a bad argument. Outputs: the rank-1 members of P^(T) in
 * crowded-comparison order (duplicates kept): *n_front rows in front_labels (capacity
 * pop_size x n), their A, S, f1, f2; *selected = first index maximising (1 - f1) - f2
 * (Alg. 3, strict improvement). */
int or_run(int32_t n, const int32_t *row_ptr, const int32_t *col, const or_params *prm,
           int32_t threads, or_callback cb, void *user, int32_t *n_front,
           int32_t *front_labels, int64_t *fA, int64_t *fS, double *ff1, double *ff2,
           int32_t *selected)
{
    /* threads > 1 only spreads independent individuals over OpenMP threads; every
     * individual is computed exactly as in the serial loop, so results do not change */
    if (threads < 1) threads = 1;
    const int32_t np = prm->pop_size, T = prm->generations, es = prm->parents_per_child;
    if (n <= 0 || np < 1 || T < 0 || es < 1 || es > 8) return -1;
    if (row_ptr[n] <= 0) return -1;
    or_graph G;
    graph_copy(&G, n, row_ptr, col);
    const uint64_t seed = prm->seed, thr_m = or_thr(prm->mutation_p);
    int32_t maxd = 1;
    for (int32_t v = 0; v < n; ++v)
        if (G.row_ptr[v + 1] - G.row_ptr[v] > maxd) maxd = G.row_ptr[v + 1] - G.row_ptr[v];

    member *store = (member *)malloc(sizeof(member) * (size_t)(2 * np));
    for (int32_t i = 0; i < 2 * np; ++i)
        store[i].row = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    const member **P = (const member **)malloc(sizeof(member *) * (size_t)np);
    const member **R = (const member **)malloc(sizeof(member *) * (size_t)(2 * np));
    const int32_t **Prow = (const int32_t **)malloc(sizeof(int32_t *) * (size_t)np);
    member **freeq = (member **)malloc(sizeof(member *) * (size_t)np);
    int64_t *Dall = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * (size_t)threads);
    int32_t *scall = (int32_t *)malloc(sizeof(int32_t) * (size_t)maxd * (size_t)threads);
    int32_t *Call = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)threads);
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * np));
    double *crowd = (double *)malloc(sizeof(double) * (size_t)(2 * np));
    int32_t *prank = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
    double *pcrowd = (double *)malloc(sizeof(double) * (size_t)np);
    int32_t *buf_lab = NULL;
    int64_t *bA = NULL, *bS = NULL;
    double *bf1 = NULL, *bf2 = NULL;
    if (cb) {
        buf_lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)np * (size_t)n);
        bA = (int64_t *)malloc(sizeof(int64_t) * (size_t)np);
        bS = (int64_t *)malloc(sizeof(int64_t) * (size_t)np);
        bf1 = (double *)malloc(sizeof(double) * (size_t)np);
        bf2 = (double *)malloc(sizeof(double) * (size_t)np);
    }

    /* Phase 1-2 of Alg. 1: initial population and its evaluation */
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
    for (int32_t i = 0; i < np; ++i) {
        int t = thread_id();
        member *m = &store[i];
        init_individual(&G, seed, i, m->row);
        eval_graph(&G, m->row, Dall + (size_t)t * (size_t)n, &m->A, &m->S, &m->f1, &m->f2);
        P[i] = m;
    }
    if (cb) emit(cb, user, 0, n, P, np, NULL, NULL, buf_lab, bA, bS, bf1, bf2);

    /* Phase 3: generations */
    for (int32_t gen = 1; gen <= T; ++gen) {
        /* step 1: rank, crowd and reorder P^(gen-1) on its own */
        int32_t *order = rank_crowd_order(P, np, G.m2, rank, crowd);
        const member **tmp = (const member **)malloc(sizeof(member *) * (size_t)np);
        for (int32_t q = 0; q < np; ++q) {
            tmp[q] = P[order[q]];
            prank[q] = rank[order[q]];
            pcrowd[q] = crowd[order[q]];
        }
        memcpy(P, tmp, sizeof(member *) * (size_t)np);
        free(tmp);
        free(order);

        for (int32_t q = 0; q < np; ++q) Prow[q] = P[q]->row;

        /* the storage slots not holding a member of P receive the offspring */
        int32_t nfree = 0;
        for (int32_t i = 0; i < 2 * np; ++i) {
            int used = 0;
            for (int32_t q = 0; q < np; ++q)
                if (P[q] == &store[i]) used = 1;
            if (!used) freeq[nfree++] = &store[i];
        }

        /* steps 2-5: offspring j = tournament -> crossover -> mutation -> evaluation */
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
        for (int32_t j = 0; j < np; ++j) {
            int t = thread_id();
            int32_t *C = Call + (size_t)t * (size_t)n;
            int32_t *scratch = scall + (size_t)t * (size_t)maxd;
            int64_t *D = Dall + (size_t)t * (size_t)n;
            member *q = freeq[j];
            offspring(&G, Prow, np, es, prm->crossover_p, thr_m, seed, (uint32_t)gen,
                      (uint32_t)j, C, scratch, q->row, NULL, NULL);
            eval_graph(&G, q->row, D, &q->A, &q->S, &q->f1, &q->f2);
        }

        /* step 6: R = P ++ Q, keep the first pop_size in crowded-comparison order */
        for (int32_t q = 0; q < np; ++q) R[q] = P[q];
        for (int32_t j = 0; j < np; ++j) R[np + j] = freeq[j];
        order = rank_crowd_order(R, 2 * np, G.m2, rank, crowd);
        for (int32_t q = 0; q < np; ++q) P[q] = R[order[q]];
        free(order);
        if (cb) emit(cb, user, gen, n, P, np, prank, pcrowd, buf_lab, bA, bS, bf1, bf2);
    }

    /* Phase 4: front of P^(T) and the recommended solution (Alg. 3) */
    int32_t *order = rank_crowd_order(P, np, G.m2, rank, crowd);
    int32_t k = 0;
    double best = -INFINITY;
    int32_t sel = 0;
    for (int32_t q = 0; q < np; ++q) {
        const member *m = P[order[q]];
        if (rank[order[q]] != 1) continue;
        memcpy(front_labels + (size_t)k * (size_t)n, m->row, sizeof(int32_t) * (size_t)n);
        fA[k] = m->A;
        fS[k] = m->S;
        ff1[k] = m->f1;
        ff2[k] = m->f2;
        double qv = (1.0 - m->f1) - m->f2;
        if (qv > best) {
            best = qv;
            sel = k;
        }
        ++k;
    }
    free(order);
    *n_front = k;
    *selected = sel;

    for (int32_t i = 0; i < 2 * np; ++i) free(store[i].row);
    free(store);
    free(P);
    free(R);
    free(Prow);
    free(freeq);
    free(Dall);
    free(scall);
    free(Call);
    free(rank);
    free(crowd);
    free(prank);
    free(pcrowd);
    free(buf_lab);
    free(bA);
    free(bS);
    free(bf1);
    free(bf2);
    graph_free(&G);
    return 0;
}
