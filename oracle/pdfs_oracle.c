/*
 * Plain CPU oracle for P-DFS + greedy weighted set cover.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * shares no code, header or table with it.
 *
 * What it computes (Sec. II-B, Sec. III-B/C, Alg. 1 and Alg. 2 of the paper):
 *
 *  - Preprocessing order (Sec. III-B, artifact Task 2): gene rows are
 *    visited from most sparse to least sparse.  Reading adopted: ascending
 *    combined (tumour + normal) mutation count, ties by caller index.
 *  - BEST(U) = one step-4 argmax of Alg. 1, done the P-DFS way (Alg. 2):
 *    a depth-first walk over g1 < g2 < ... < gh in the sorted order, keeping
 *    the running tumour intersection y_l = U & x_g1 & ... & x_gl and
 *    backtracking as soon as it is empty.  At depth h a non-empty y_h is a
 *    candidate; its score is S = p*TP + q*TN with TP = |y_h|,
 *    FP = |n_g1 & ... & n_gh| over all normals, TN = N_n - FP (the normals
 *    that do not carry the whole combination; with bit 8 of the mode set,
 *    the literal wording of T- in Sec. II-C instead: TN = normals carrying
 *    none of the genes, FP = |n_g1 | ... | n_gh|).  S is the
 *    numerator of F = (alpha*TP + TN)/(N_t + N_n) scaled by q, with
 *    alpha = p/q; the denominator is the same for every candidate of a round
 *    so it never changes the argmax.  The strict ">" of the maximum search
 *    keeps the first candidate in walk order, i.e. the lexicographically
 *    smallest tuple in sorted-index space.
 *  - Loop bounds follow Alg. 2: depth l ranges up to G-h+l (1-based).
 *  - Modes:  EMPTY = Alg. 2 (prune on empty intersection at every depth);
 *            NONE  = exhaustive enumeration (the pruning-off baseline), TP=0
 *                    tuples are visited but never selected;
 *            BOUND = EMPTY plus the score-bound test of Sec. III-E:
 *                    a prefix with |y_l| = c can at best reach
 *                    p*c + q*N_n; in lexicographic walk order every later
 *                    tuple loses ties, so the prefix is dropped when a best
 *                    exists and that bound is <= its score.
 *  - Greedy WSC (Alg. 1): repeat BEST, append the winner, remove the tumour
 *    samples it covers (DelCols on tumour columns only); stop when the
 *    covered count reaches the target, when no combination covers any
 *    uncovered tumour sample, or at the round cap.
 *
 * Counters per depth l (1..h): visited = nodes whose intersection was
 * computed, nonempty = those with y_l != 0, bound_pruned = prefixes dropped
 * by the bound test.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_H 9

enum { OR_MODE_NONE = 0, OR_MODE_EMPTY = 1, OR_MODE_BOUND = 2 };

static int64_t count_bits(const uint64_t *v, int words) {
    int64_t c = 0;
    for (int w = 0; w < words; w++) c += __builtin_popcountll(v[w]);
    return c;
}

/* ------------------------------------------------------------ ordering */
typedef struct {
    int64_t key;
    int32_t gene;
} or_sort_item;

static int cmp_sort_item(const void *a, const void *b) {
    const or_sort_item *x = (const or_sort_item *)a, *y = (const or_sort_item *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->gene < y->gene ? -1 : (x->gene > y->gene);
}

/* perm[i] = caller gene placed at sorted position i (sparsest first). */
void oracle_order(int32_t G, int32_t wt, const uint64_t *T, int32_t wn,
                  const uint64_t *N, int32_t *perm) {
    or_sort_item *it = (or_sort_item *)malloc(sizeof(or_sort_item) * (size_t)(G > 0 ? G : 1));
    for (int32_t g = 0; g < G; g++) {
        it[g].key = count_bits(T + (size_t)g * wt, wt) +
                    (wn > 0 ? count_bits(N + (size_t)g * wn, wn) : 0);
        it[g].gene = g;
    }
    qsort(it, (size_t)G, sizeof(or_sort_item), cmp_sort_item);
    for (int32_t i = 0; i < G; i++) perm[i] = it[i].gene;
    free(it);
}

/* ------------------------------------------------------------ P-DFS */
typedef struct {
    int32_t G, wt, wn, n_normal, h, mode;
    int32_t tn_literal;         /* TN = normals carrying none of the genes */
    const uint64_t *T, *N;
    const int32_t *perm;
    int64_t p, q;
    uint64_t *y;                /* (h+1) rows of wt words; y[0] = U */
    uint64_t *z;                /* scratch row of wn words for the normals */
    int32_t idx[OR_MAX_H];      /* current sorted indices, depth 1..h */
    int found;
    int64_t best_s, best_tp, best_fp;
    int32_t best[OR_MAX_H];
    uint64_t visited[OR_MAX_H + 1], nonempty[OR_MAX_H + 1], bound_pruned[OR_MAX_H + 1];
} or_dfs;

static void score_leaf(or_dfs *st, int64_t tp) {
    int64_t fp = 0;
    if (st->wn > 0 && st->n_normal > 0) {
        const uint64_t *n0 = st->N + (size_t)st->perm[st->idx[0]] * st->wn;
        for (int w = 0; w < st->wn; w++) st->z[w] = n0[w];
        for (int l = 1; l < st->h; l++) {
            const uint64_t *nl = st->N + (size_t)st->perm[st->idx[l]] * st->wn;
            /* FP: normals carrying every gene of the tuple (AND), or under the
             * literal reading of T- any of them (OR) */
            if (st->tn_literal)
                for (int w = 0; w < st->wn; w++) st->z[w] |= nl[w];
            else
                for (int w = 0; w < st->wn; w++) st->z[w] &= nl[w];
        }
        fp = count_bits(st->z, st->wn);
    }
    int64_t tn = st->n_normal - fp;
    int64_t s = st->p * tp + st->q * tn;
    if (!st->found || s > st->best_s) {
        st->found = 1;
        st->best_s = s;
        st->best_tp = tp;
        st->best_fp = fp;
        for (int l = 0; l < st->h; l++) st->best[l] = st->idx[l];
    }
}

/* Fill depth l (1-based) with sorted indices lo..G-h+l-1 (depth 1 may be
 * cut to the share [lo, hi1)). */
static void descend(or_dfs *st, int l, int32_t lo, int32_t hi1) {
    int32_t hi = st->G - st->h + l - 1;
    if (l == 1 && hi1 - 1 < hi) hi = hi1 - 1;
    const uint64_t *prev = st->y + (size_t)(l - 1) * st->wt;
    uint64_t *cur = st->y + (size_t)l * st->wt;
    for (int32_t i = lo; i <= hi; i++) {
        const uint64_t *row = st->T + (size_t)st->perm[i] * st->wt;
        for (int w = 0; w < st->wt; w++) cur[w] = prev[w] & row[w];
        st->idx[l - 1] = i;
        st->visited[l]++;
        int64_t c = count_bits(cur, st->wt);
        if (c > 0) st->nonempty[l]++;
        if (l == st->h) {
            if (c > 0) score_leaf(st, c);
            continue;
        }
        if (c == 0 && st->mode != OR_MODE_NONE) continue;
        if (st->mode == OR_MODE_BOUND && st->found &&
            st->p * c + st->q * (int64_t)st->n_normal <= st->best_s) {
            st->bound_pruned[l]++;
            continue;
        }
        descend(st, l + 1, i + 1, 0);
    }
}

/*
 * One argmax round.  U: wt words (uncovered tumour samples).  Returns 1 and
 * fills best_idx (sorted indices), tp, fp when a combination with TP >= 1
 * exists, 0 otherwise, -1 on bad arguments.  counters: 3 x (OR_MAX_H+1)
 * uint64, added to (visited, nonempty, bound_pruned), index = depth.
 */
static int best_share(int32_t G, int32_t n_tumor, int32_t n_normal, int32_t wt,
                      const uint64_t *T, int32_t wn, const uint64_t *N,
                      const int32_t *perm, int32_t h, int64_t p, int64_t q,
                      const uint64_t *U, int32_t mode, int32_t g1_lo, int32_t g1_hi,
                      int32_t *best_idx, int64_t *tp, int64_t *fp, uint64_t *counters);

int oracle_best(int32_t G, int32_t n_tumor, int32_t n_normal, int32_t wt,
                const uint64_t *T, int32_t wn, const uint64_t *N,
                const int32_t *perm, int32_t h, int64_t p, int64_t q,
                const uint64_t *U, int32_t mode, int32_t *best_idx,
                int64_t *tp, int64_t *fp, uint64_t *counters) {
    return best_share(G, n_tumor, n_normal, wt, T, wn, N, perm, h, p, q, U, mode, 0, G,
                      best_idx, tp, fp, counters);
}

/*
 * The same search restricted to first genes g1 in [g1_lo, g1_hi) (sorted
 * positions): one rank's share when the outer loop is split into intervals
 * (Sec. III-D).  Used to time a bounded sample of a round.
 */
int oracle_best_share(int32_t G, int32_t n_tumor, int32_t n_normal, int32_t wt,
                      const uint64_t *T, int32_t wn, const uint64_t *N,
                      const int32_t *perm, int32_t h, int64_t p, int64_t q,
                      const uint64_t *U, int32_t mode, int32_t g1_lo, int32_t g1_hi,
                      int32_t *best_idx, int64_t *tp, int64_t *fp, uint64_t *counters) {
    return best_share(G, n_tumor, n_normal, wt, T, wn, N, perm, h, p, q, U, mode, g1_lo, g1_hi,
                      best_idx, tp, fp, counters);
}

static int best_share(int32_t G, int32_t n_tumor, int32_t n_normal, int32_t wt,
                      const uint64_t *T, int32_t wn, const uint64_t *N,
                      const int32_t *perm, int32_t h, int64_t p, int64_t q,
                      const uint64_t *U, int32_t mode, int32_t g1_lo, int32_t g1_hi,
                      int32_t *best_idx, int64_t *tp, int64_t *fp, uint64_t *counters) {
    if (h < 1 || h > OR_MAX_H || h > G || q < 1 || p < 0 || n_tumor < 1) return -1;
    if (g1_lo < 0) g1_lo = 0;
    if (g1_hi > G) g1_hi = G;
    (void)n_tumor;
    or_dfs st;
    memset(&st, 0, sizeof(st));
    st.G = G; st.wt = wt; st.wn = wn; st.n_normal = n_normal; st.h = h;
    st.mode = mode & 0xff;                  /* bit 8: literal-T- reading */
    st.tn_literal = (mode >> 8) & 1;
    st.T = T; st.N = N; st.perm = perm; st.p = p; st.q = q;
    st.y = (uint64_t *)calloc((size_t)(h + 1) * wt, sizeof(uint64_t));
    st.z = (uint64_t *)calloc((size_t)(wn > 0 ? wn : 1), sizeof(uint64_t));
    memcpy(st.y, U, sizeof(uint64_t) * (size_t)wt);
    descend(&st, 1, g1_lo, g1_hi);
    if (counters) {
        for (int l = 0; l <= OR_MAX_H; l++) {
            counters[l] += st.visited[l];
            counters[(OR_MAX_H + 1) + l] += st.nonempty[l];
            counters[2 * (OR_MAX_H + 1) + l] += st.bound_pruned[l];
        }
    }
    free(st.y);
    free(st.z);
    if (!st.found) return 0;
    for (int l = 0; l < h; l++) best_idx[l] = st.best[l];
    *tp = st.best_tp;
    *fp = st.best_fp;
    return 1;
}

/*
 * Greedy WSC (Alg. 1) over BEST rounds.
 *   target <= 0 means all n_tumor samples; max_rounds <= 0 means no cap.
 *   U0: initial uncovered mask (wt words) or NULL for all samples.
 *   Per round r (0-based) writes: genes[r*h + l] caller ids (sorted order),
 *   sidx[r*h + l] sorted indices, rec[r*6 + k] =
 *   {tp, fp, tn, score_num, score_den, uncovered_before}.
 *   Writes the final uncovered mask to U_out (wt words) if not NULL.
 * Returns the number of rounds run (rounds beyond cap are run and counted but
 * not written), or -1 on bad arguments.
 */
int oracle_wsc(int32_t G, int32_t n_tumor, int32_t n_normal, int32_t wt,
               const uint64_t *T, int32_t wn, const uint64_t *N, int32_t h,
               int64_t p, int64_t q, int32_t target, int32_t max_rounds,
               const uint64_t *U0, int32_t mode, int32_t cap, int32_t *genes,
               int32_t *sidx, int64_t *rec, uint64_t *counters, uint64_t *U_out) {
    if (h < 1 || h > OR_MAX_H || h > G || q < 1 || p < 0 || n_tumor < 1 || wt < (n_tumor + 63) / 64)
        return -1;
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)G);
    oracle_order(G, wt, T, wn, N, perm);
    uint64_t *U = (uint64_t *)calloc((size_t)wt, sizeof(uint64_t));
    uint64_t *cov = (uint64_t *)calloc((size_t)wt, sizeof(uint64_t));
    if (U0) {
        memcpy(U, U0, sizeof(uint64_t) * (size_t)wt);
    } else {
        for (int32_t s = 0; s < n_tumor; s++) U[s >> 6] |= 1ULL << (s & 63);
    }
    const int32_t K = target > 0 ? target : n_tumor;
    int rounds = 0;
    int32_t best[OR_MAX_H];
    for (;;) {
        int64_t uncovered = count_bits(U, wt);
        if (n_tumor - uncovered >= K) break;
        if (max_rounds > 0 && rounds >= max_rounds) break;
        int64_t tp = 0, fp = 0;
        int found = oracle_best(G, n_tumor, n_normal, wt, T, wn, N, perm, h, p, q, U,
                                mode, best, &tp, &fp, counters);
        if (found <= 0) break;
        if (rounds < cap) {
            for (int l = 0; l < h; l++) {
                genes[rounds * h + l] = perm[best[l]];
                sidx[rounds * h + l] = best[l];
            }
            int64_t tn = n_normal - fp;
            rec[rounds * 6 + 0] = tp;
            rec[rounds * 6 + 1] = fp;
            rec[rounds * 6 + 2] = tn;
            rec[rounds * 6 + 3] = p * tp + q * tn;
            rec[rounds * 6 + 4] = q * (uncovered + n_normal);
            rec[rounds * 6 + 5] = uncovered;
        }
        /* C <- C u C(gamma*);  X <- DelCols(X, gamma*) on tumour columns. */
        for (int w = 0; w < wt; w++) cov[w] = U[w];
        for (int l = 0; l < h; l++) {
            const uint64_t *row = T + (size_t)perm[best[l]] * wt;
            for (int w = 0; w < wt; w++) cov[w] &= row[w];
        }
        for (int w = 0; w < wt; w++) U[w] &= ~cov[w];
        rounds++;
    }
    if (U_out) memcpy(U_out, U, sizeof(uint64_t) * (size_t)wt);
    free(perm);
    free(U);
    free(cov);
    return rounds;
}
