/* Host-sanitizer driver for the oracle: compiles oracle.c into one executable with
 * AddressSanitizer and UndefinedBehaviorSanitizer and exercises every entry point on small
 * graphs (cliques with a bridge, a path, a star with isolated nodes, a random graph) and
 * edge parameters. Exit status 0 = no finding (sanitizer findings abort). */
#include "../../oracle/oracle.c"

#include <stdio.h>

static void csr(int32_t n, const int32_t (*e)[2], int32_t m, int32_t *rp, int32_t *col)
{
    memset(rp, 0, sizeof(int32_t) * (size_t)(n + 1));
    for (int32_t i = 0; i < m; ++i) {
        rp[e[i][0] + 1]++;
        rp[e[i][1] + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) rp[v + 1] += rp[v];
    int32_t *fill = calloc((size_t)n, sizeof(int32_t));
    for (int32_t i = 0; i < m; ++i) {
        const int32_t a = e[i][0], b = e[i][1];
        col[rp[a] + fill[a]++] = b;
        col[rp[b] + fill[b]++] = a;
    }
    for (int32_t v = 0; v < n; ++v) qsort(col + rp[v], (size_t)(rp[v + 1] - rp[v]), sizeof(int32_t), cmp_i32);
    free(fill);
}

static int gens_seen;
static void count_gen(const or_state_view *s, void *u)
{
    (void)u;
    gens_seen += s->pop_size > 0;
}

static int run_case(int32_t n, const int32_t (*e)[2], int32_t m, int32_t pop, int32_t T,
                    double cp, double mp, int32_t es, uint64_t seed)
{
    int32_t *rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *col = malloc(sizeof(int32_t) * (size_t)(2 * m));
    csr(n, e, m, rp, col);
    or_params prm = {pop, T, cp, mp, es, seed};
    int32_t nf = 0, sel = -1;
    int32_t *fl = malloc(sizeof(int32_t) * (size_t)pop * n);
    int64_t *fA = malloc(sizeof(int64_t) * pop), *fS = malloc(sizeof(int64_t) * pop);
    double *f1 = malloc(sizeof(double) * pop), *f2 = malloc(sizeof(double) * pop);
    gens_seen = 0;
    int rc = or_run(n, rp, col, &prm, 1, count_gen, NULL, &nf, fl, fA, fS, f1, f2, &sel);
    int bad = rc != 0 || nf < 1 || nf > pop || sel < 0 || sel >= nf || gens_seen != T + 1;
    /* evaluation, init, crossover, mutation and the selection routines directly */
    int64_t A, S;
    double g1, g2;
    or_eval(n, rp, col, fl, &A, &S, &g1, &g2);
    bad |= A != fA[0] || S != fS[0];
    int32_t *lab = malloc(sizeof(int32_t) * (size_t)n * 3);
    for (int32_t i = 0; i < 3; ++i) or_init_individual(n, rp, col, seed, i, lab + (size_t)i * n);
    int32_t *child = malloc(sizeof(int32_t) * (size_t)n), *mut = malloc(sizeof(int32_t) * (size_t)n);
    or_crossover(n, 3, lab, -1, seed, 1, 0, child);
    or_mutate(n, rp, col, child, 0.5, seed, 1, 0, mut);
    for (int32_t v = 0; v < n; ++v) (void)or_neighbour_plurality(n, rp, col, child, v, seed, 1, 2);
    int32_t rank[8], order[8];
    int64_t k1[8], k2[8];
    double crowd[8], o1[8], o2[8];
    for (int i = 0; i < 8; ++i) {
        k1[i] = (i * 7) % 5;
        k2[i] = (i * 3) % 4;
        o1[i] = (double)k1[i] / 5.0;
        o2[i] = (double)k2[i] / 4.0;
    }
    or_rank(8, k1, k2, rank);
    or_crowding(8, rank, k1, k2, o1, o2, crowd);
    or_order(8, rank, crowd, order);
    free(rp); free(col); free(fl); free(fA); free(fS); free(f1); free(f2);
    free(lab); free(child); free(mut);
    return bad;
}

int main(void)
{
    int32_t e[4096][2];
    int32_t m = 0;
    /* two 6-cliques joined by one bridge */
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < 6; ++i)
            for (int j = i + 1; j < 6; ++j) e[m][0] = 6 * c + i, e[m][1] = 6 * c + j, ++m;
    e[m][0] = 5, e[m][1] = 6, ++m;
    int bad = run_case(12, e, m, 16, 6, 0.9, 0.2, 4, 1);
    bad |= run_case(12, e, m, 1, 3, 1.0, 1.0, 8, 2);    /* one individual, every node mutates */
    bad |= run_case(12, e, m, 5, 0, 0.0, 0.0, 1, 3);    /* T = 0 */
    m = 0;                                              /* path of 30 */
    for (int i = 0; i + 1 < 30; ++i) e[m][0] = i, e[m][1] = i + 1, ++m;
    bad |= run_case(30, e, m, 12, 5, 0.8, 0.3, 3, 4);
    m = 0;                                              /* star of 20 plus 9 isolated nodes */
    for (int i = 1; i < 20; ++i) e[m][0] = 0, e[m][1] = i, ++m;
    bad |= run_case(29, e, m, 10, 4, 0.9, 0.5, 4, 5);
    m = 0;                                              /* random simple graph, 300 nodes */
    uint32_t x = 12345;
    char *seen = calloc(300 * 300, 1);
    while (m < 1500) {
        x = x * 1664525u + 1013904223u;
        const int a = (int)((x >> 8) % 300);
        x = x * 1664525u + 1013904223u;
        const int b = (int)((x >> 8) % 300);
        if (a == b || seen[a * 300 + b]) continue;
        seen[a * 300 + b] = seen[b * 300 + a] = 1;
        e[m][0] = a, e[m][1] = b, ++m;
    }
    free(seen);
    bad |= run_case(300, e, m, 24, 6, 0.9, 0.1, 4, 6);
    printf(bad ? "FAIL\n" : "ok\n");
    return bad;
}
