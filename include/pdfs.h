/*
 * pdfs.h -- C ABI of the MI355X P-DFS / greedy weighted-set-cover library.
 *
 * The library finds h-hit gene combinations the way the paper's pruned
 * depth-first search does (Sec. III-C, Alg. 2) inside the standard greedy
 * weighted-set-cover loop (Sec. II-C, Alg. 1), on one AMD Instinct GPU.
 *
 * Problem (Sec. II-B, Eq. 1): tumour matrix T (G genes x N_t samples) and
 * normal matrix N (G x N_n), both 0/1.  A combination gamma of h distinct
 * genes covers a sample when every gene of gamma is mutated in it.  With the
 * still-uncovered tumour samples U of the current round:
 *     TP = |cover_T(gamma) & U|,  FP = |cover_N(gamma)|,  TN = N_n - FP,
 *     S  = p*TP + q*TN            (integer numerator of the score)
 * F(gamma) = (alpha*TP + TN) / (|U| + N_n) with alpha = p/q (Sec. II-C), so
 * F = S / (q*(|U| + N_n)); the denominator is shared by all candidates of a
 * round, so candidates are ranked by S, exactly, in integers.
 * Each round picks, among the combinations with TP >= 1, the largest S; ties
 * go to the lexicographically smallest tuple of sorted gene indices (the
 * order a sequential depth-first maximum search with a strict ">" keeps).
 * Genes are sorted once, sparsest first (Sec. III-B): ascending combined
 * tumour+normal mutation count, ties by caller index.  The round's cover is
 * then removed from U (DelCols of Alg. 1, tumour columns only) and the loop
 * repeats until the covered count reaches the target, no combination has
 * TP >= 1, or the round cap is hit.
 *
 * Bit layout: a matrix is row-major uint64 words, one row per gene; sample s
 * of gene g is bit (s & 63) of word row[g*stride + (s >> 6)].  Bits past the
 * sample count must be 0 (PDFS_ERR_INVALID_ARG otherwise).
 *
 * Errors: every call returns an int32 status; nothing is thrown across the
 * ABI.  Negative values are errors, 0 is success, positive values are
 * informational.  pdfs_strerror() names a status; pdfs_last_error() gives the
 * detail of the last failing call on a context.
 *
 * Threading: a context may be used by one host thread at a time; distinct
 * contexts are independent.  Work is issued on the stream given at creation
 * (NULL = the device's null stream); calls return after their results are on
 * the host.
 */
#ifndef PDFS_H
#define PDFS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define PDFS_OK 0
#define PDFS_NO_COMBO 1            /* no h-subset covers an uncovered sample   */
#define PDFS_PENDING 2             /* server: request not finished yet         */
#define PDFS_ERR_INVALID_ARG (-1)  /* bad argument, layout or pad bits          */
#define PDFS_ERR_UNSUPPORTED (-2)  /* valid but outside what the GPU path runs  */
#define PDFS_ERR_OUT_OF_MEMORY (-3)/* device allocation or admission failure    */
#define PDFS_ERR_DEVICE (-4)       /* HIP runtime / kernel error                */
#define PDFS_ERR_TRUNCATED (-5)    /* output array too small; *n_out = needed   */

/* ------------------------------------------------------------ pruning modes */
/* PDFS_PRUNE_EMPTY: the paper's rule (Alg. 2) -- a prefix whose running tumour
 *   intersection is empty is not extended.
 * PDFS_PRUNE_BOUND: EMPTY plus the score bound of Sec. III-E -- a prefix
 *   covering c uncovered tumour samples can reach at most p*c + q*N_n, so it
 *   is not extended when that cannot beat the best combination found so far.
 *   Exact: it returns the same combinations as EMPTY.  The default.
 * PDFS_PRUNE_NONE: exhaustive enumeration (the pruning-off baseline the paper
 *   compares against, Sec. IV): every gene is walked and every prefix is
 *   extended, empty or not; leaves with TP = 0 are visited but never chosen,
 *   so the combinations equal EMPTY's and only the visited counters grow
 *   (to the full loop-bound counts of Alg. 2).  Its first use on a context
 *   regrows the row-indexed buffers to G rows. */
#define PDFS_PRUNE_NONE 0
#define PDFS_PRUNE_EMPTY 1
#define PDFS_PRUNE_BOUND 2

#define PDFS_MAX_H 9

typedef struct pdfs_ctx pdfs_ctx;

/* Input cohort.  tumor: G rows x tumor_stride_words uint64 (stride >=
 * ceil(n_tumor/64)); normal: G rows x normal_stride_words (stride >=
 * ceil(n_normal/64); may be NULL when n_normal == 0).  on_device != 0 means
 * both pointers are device pointers on the context's device.  The library
 * copies the data; the caller keeps ownership and may free it on return. */
typedef struct {
    int32_t G;
    int32_t n_tumor;   /* >= 1   */
    int32_t n_normal;  /* >= 0   */
    int32_t on_device;
    const uint64_t *tumor;
    const uint64_t *normal;
    int64_t tumor_stride_words;
    int64_t normal_stride_words;
} pdfs_matrix;

/* pdfs_options.flags */
#define PDFS_OPT_TIME_KERNELS 1   /* time the pair-table and DFS launches with HIP
                                     events on the context's stream (pdfs_stats) */
#define PDFS_OPT_TN_LITERAL 8     /* TN counts the normals carrying none of the
                                     combination's genes (the literal wording of
                                     T- in Sec. II-C; FP = normals carrying any);
                                     default: normals not carrying all of them */
#define PDFS_OPT_GRAPHS 2         /* capture one round as a HIP graph per row width
                                     and replay it (needs a non-NULL stream; ignored
                                     together with PDFS_OPT_TIME_KERNELS) */

typedef struct {
    int32_t prune_mode; /* PDFS_PRUNE_*                                  */
    int32_t device;     /* HIP device ordinal                            */
    void *stream;       /* hipStream_t on that device, or NULL           */
    int32_t flags;      /* PDFS_OPT_* bits                               */
    int32_t pair_cap;   /* initial capacity of the round's pair list
                           (pairs); <= 0: the default, max(2^21, 128 x
                           the active genes of the first round), at most
                           every pair.  A round that emits more pairs
                           grows the list to its count + 1/4 and is run
                           again, so this only trades memory for an
                           occasional repeated round. */
} pdfs_options;

/* One chosen combination (one greedy round). */
typedef struct {
    int32_t h;
    int32_t genes[PDFS_MAX_H];      /* caller gene ids, in sorted order          */
    int32_t sorted_idx[PDFS_MAX_H]; /* the same genes as sorted (sparsest-first) indices */
    int32_t tp;                     /* tumour samples covered among U            */
    int32_t fp;                     /* normal samples covered                    */
    int32_t tn;                     /* n_normal - fp                             */
    int32_t uncovered_before;       /* |U| at the start of the round             */
    int32_t newly_covered;          /* tumour samples the round adds to the cover
                                       (U loses exactly the tp samples)         */
    int64_t score_num;              /* S = p*tp + q*tn                           */
    int64_t score_den;              /* q*(uncovered_before + n_normal); F = num/den */
} pdfs_combo;

/* Per-depth counters, index = depth (1..h), summed over rounds.
 * visited[l]: depth-l nodes whose running intersection was formed (the loop
 *   bounds of Alg. 2: depth l ranges over sorted indices up to G-h+l-1,
 *   0-based); nonempty[l]: those with a non-empty tumour intersection;
 *   bound_pruned[l]: non-empty prefixes dropped by the score bound.
 * Under PDFS_PRUNE_EMPTY the counts are exact and order-independent.  Under
 * PDFS_PRUNE_BOUND they depend on how fast the incumbent rises and are for
 * information only. */
typedef struct {
    uint64_t visited[PDFS_MAX_H + 1];
    uint64_t nonempty[PDFS_MAX_H + 1];
    uint64_t bound_pruned[PDFS_MAX_H + 1];
    int32_t rounds;
    int32_t reserved;
    int64_t ns_total;   /* host wall time of the call, nanoseconds */
    /* Filled when the context was created with PDFS_OPT_TIME_KERNELS:
     * index 0 = int8-MFMA pair-table kernel, 1 = depth-first stage (depths
     * 3..h), 2 = the part of index 1 spent in the depth-4 tile kernel (h = 4
     * under PDFS_PRUNE_EMPTY: depth-3 prefixes with long depth-4 candidate
     * streams are listed, bucketed by their third gene and expanded in
     * tiles; 0 otherwise). */
    int64_t kernel_ns[3];        /* summed HIP-event durations            */
    int32_t kernel_launches[3];  /* launches timed                        */
    /* Work the kernels had to do, counted inside them (always filled):
     * pair_macs  = active pairs x |U| (one multiply-add per sample);
     * dfs_visits[l] = depth-l (l = 3, 4) candidate intersections over active
     *   genes; dfs_leaves = non-empty leaves (each compared with its
     *   lane's best); dfs_fp_leaves = leaves whose
     *   normal intersection had to be counted; dfs_visit_words3/4 = depth-3/4
     *   visits times ceil(|U|/64) of their round, summed (so words / visits
     *   is the mean row length in 64-bit words). */
    uint64_t pair_macs;
    uint64_t dfs_visits[PDFS_MAX_H + 1];
    uint64_t dfs_leaves;
    uint64_t dfs_fp_leaves;
    uint64_t dfs_visit_words3;   /* sum of visits x ceil(|U|/64), depth 3 */
    uint64_t dfs_visit_words4;   /* same for depth 4 */
} pdfs_stats;

/* Copies the cohort to the device, sorts genes sparsest first and sets up the
 * round workspace.  *out receives the context (NULL on failure).  Errors:
 * INVALID_ARG (shapes, strides, pad bits, n_tumor < 1, G < 1), OUT_OF_MEMORY,
 * DEVICE. */
int32_t pdfs_create(const pdfs_matrix *m, const pdfs_options *opt, pdfs_ctx **out);

/* Releases the context and its device memory.  NULL is ignored. */
void pdfs_destroy(pdfs_ctx *ctx);

/* Changes the pruning mode of later calls. */
int32_t pdfs_set_prune_mode(pdfs_ctx *ctx, int32_t prune_mode);

/* One argmax round (step 4 of Alg. 1, done as Alg. 2): the best h-subset
 * against the uncovered mask `uncovered` (host pointer, ceil(n_tumor/64)
 * words, NULL = every tumour sample).  alpha = alpha_p / alpha_q with
 * alpha_q >= 1.  Returns PDFS_OK with *out filled, PDFS_NO_COMBO when no
 * subset has TP >= 1 (out->h = 0), or an error.  stats may be NULL; it is
 * overwritten.  h: 1..PDFS_MAX_H (h = 5..9 expand every depth below the
 * pair level wave-wide through per-depth prefix rings; the answers are the
 * same in every prune mode). */
int32_t pdfs_best_combo(pdfs_ctx *ctx, int32_t h, uint32_t alpha_p, uint32_t alpha_q,
                        const uint64_t *uncovered, pdfs_combo *out, pdfs_stats *stats);

/* The greedy weighted-set-cover loop (Alg. 1).  target_covered <= 0 means
 * every tumour sample; max_rounds <= 0 means no cap.  initial_uncovered (host
 * pointer, ceil(n_tumor/64) words) resumes from a previous state; NULL starts
 * with every sample uncovered.  Rounds are written to out[0..cap); *n_out is
 * the number of rounds.  If more than cap rounds were needed the call returns
 * PDFS_ERR_TRUNCATED with *n_out = rounds needed (the first cap are written).
 * final_uncovered (host, may be NULL) receives the mask after the last round.
 * stats may be NULL.  The first call with h >= 5 on a context allocates the
 * deep walk's prefix rings (about 0.8 GB at 1000 tumour samples), kept until
 * pdfs_destroy; PDFS_ERR_OUT_OF_MEMORY if that fails.  PDFS_ERR_DEVICE also
 * reports a device-side consistency failure (a corrupt result slot, or the
 * deep walk's scheduler making no progress), with the run stopped. */
int32_t pdfs_wsc_run(pdfs_ctx *ctx, int32_t h, uint32_t alpha_p, uint32_t alpha_q,
                     int32_t target_covered, int32_t max_rounds,
                     const uint64_t *initial_uncovered, pdfs_combo *out, int32_t cap,
                     int32_t *n_out, uint64_t *final_uncovered, pdfs_stats *stats);

const char *pdfs_strerror(int32_t status);
const char *pdfs_last_error(const pdfs_ctx *ctx);

/* ------------------------------------------------------- allocation-free round
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * The round of pdfs_best_combo (same arguments, results and statistics, on a
 * context made beforehand by pdfs_create, which does allocate) with every
 * per-round buffer -- uncovered-sample list, active list, re-packed and
 * unpacked rows, pair, work and item lists, argmax slots, counter rows, round
 * state -- taken from one static device array of PDFS_NOALLOC_SCRATCH_BYTES
 * instead of the context's workspace.  The library holds that array on every
 * device it has created a context on, until the process ends.  The call makes
 * no device allocation or free and calls no allocating library routine; it
 * copies the mask in, launches on the context's stream and waits for the
 * result.  Limits: h <= 4 (PDFS_ERR_UNSUPPORTED otherwise); a round whose
 * fixed workspace (rows, unpacked rows and lists for the context's gene count
 * and row width) exceeds the array is rejected with PDFS_ERR_UNSUPPORTED
 * before any work; the pair and item lists take the rest of the array (up to
 * every active pair), and a round whose non-empty pairs do not fit returns
 * PDFS_ERR_OUT_OF_MEMORY.  pdfs_last_error() names the sizes.  Every call on
 * a device shares that device's array (the round state, slots and counters are
 * cleared by each call): calls that overlap on one device race. */
#define PDFS_NOALLOC_SCRATCH_BYTES (64u << 20)
int32_t pdfs_best_combo_noalloc(pdfs_ctx *ctx, int32_t h, uint32_t alpha_p, uint32_t alpha_q,
                                const uint64_t *uncovered, pdfs_combo *out, pdfs_stats *stats);

/* Measurement support (not part of the method): the integer VALU rate the
 * device sustains for the depth-first kernels' per-word instruction pair
 * (an AND with a wave-uniform row word, then a popcount-accumulate), in
 * lane-operations per second, measured by a short probe kernel on `device`
 * (a few ms; allocates and frees a small buffer).  The achieved rate of the
 * depth-first stage is reported against both this and the datasheet peak.
 * Returns PDFS_OK, PDFS_ERR_INVALID_ARG (NULL output), PDFS_ERR_DEVICE or
 * PDFS_ERR_OUT_OF_MEMORY. */
int32_t pdfs_measure_int_peak(int32_t device, double *lane_ops_per_s);

/* ------------------------------------------------------------- batched
 * Many independent cohorts (instances) solved together: each instance keeps
 * its own context, rounds stay device-resident, one round per row width is
 * captured as a HIP graph and replayed, and the instances' rounds run
 * concurrently on a small set of streams (one per hardware queue) while a
 * single host thread feeds them.  Results are those of pdfs_wsc_run on each
 * instance alone.  The split granularity (depth-3 candidates per work item,
 * seed pairs in bound mode) is chosen per instance class by the tuner below
 * when the batch is created with PDFS_OPT_AUTOTUNE. */
#define PDFS_OPT_AUTOTUNE 4
/* Two ways to run a batch; by default each run takes the one that measures
 * faster for its pruning mode.
 * One launch per round step over all instances (default under
 * PDFS_PRUNE_BOUND; only for batches of up to 64 instances, all with h in
 * {3, 4}, under PDFS_PRUNE_EMPTY or PDFS_PRUNE_BOUND): every light step
 * covers every instance with a block row each, each depth-first step drains
 * one shared work queue of all live instances' work items (the ordering of
 * Sec. III-D's request-driven chunks), and the round's launches are one
 * captured HIP graph replayed until every instance's stop flag is set; the
 * row width of a chunk of rounds is the largest any live instance needs.
 * Each instance's own launches concurrently on the batch's streams (default
 * otherwise): under PDFS_PRUNE_EMPTY a round of a large instance fills the
 * device by itself, and instances that run independently overlap one
 * instance's narrow tail rounds with another's wide ones, where one launch
 * per step makes every instance wait for the slowest at each step.
 * PDFS_OPT_BATCH_STREAMS asks for the streams, PDFS_OPT_BATCH_ONE_LAUNCH for
 * one launch per step where the batch allows it (streams otherwise); both
 * together are PDFS_ERR_INVALID_ARG. */
#define PDFS_OPT_BATCH_STREAMS 16
#define PDFS_OPT_BATCH_ONE_LAUNCH 32

typedef struct pdfs_batch pdfs_batch;

/* Ingests n instances (host or device matrices as in pdfs_create).
 * opt->stream is ignored: the batch owns its streams. */
int32_t pdfs_batch_create(const pdfs_matrix *inst, int32_t n, const pdfs_options *opt,
                          pdfs_batch **out);
/* Runs the greedy loop on every instance.  h[i], target[i] (<= 0: all),
 * outs[i] (caps[i] records), n_outs[i] = rounds of instance i.  stats (may
 * be NULL) receives the sums over instances.  Returns the first error, or
 * PDFS_ERR_TRUNCATED if some instance needed more than caps[i] rounds. */
int32_t pdfs_batch_run(pdfs_batch *b, const int32_t *h, uint32_t alpha_p, uint32_t alpha_q,
                       const int32_t *target, pdfs_combo *const *outs, const int32_t *caps,
                       int32_t *n_outs, pdfs_stats *stats);
void pdfs_batch_destroy(pdfs_batch *b);
/* Detail of the last failing call on b (which instance failed and why);
 * b = NULL gives the detail of a failed pdfs_batch_create on this thread.
 * The string stays valid until the next call on b. */
const char *pdfs_batch_last_error(const pdfs_batch *b);

/* ------------------------------------------------------------- served
 * A request loop: solves submitted at any time are admitted when a slot and
 * device memory are free (admission by free HBM: the request's estimated
 * footprint must fit both the budget and the device's free memory), run
 * concurrently with the requests already on the device (continuous
 * batching: new requests join as others finish), keep their bit matrices and
 * uncovered masks on the device between rounds, and are released on
 * completion.  Latency is measured from submission to completion. */
typedef struct pdfs_server pdfs_server;

/* hbm_budget_bytes: device memory the server may hold (0 = 90% of free);
 * max_active: requests on the device at once (<= 0: 8). */
int32_t pdfs_server_create(const pdfs_options *opt, uint64_t hbm_budget_bytes,
                           int32_t max_active, pdfs_server **out);
/* Copies the cohort (host matrices only) and queues the solve.  *ticket
 * identifies it.  Requests larger than the budget are rejected
 * (PDFS_ERR_OUT_OF_MEMORY); invalid ones with PDFS_ERR_INVALID_ARG. */
int32_t pdfs_server_submit(pdfs_server *s, const pdfs_matrix *m, int32_t h, uint32_t alpha_p,
                           uint32_t alpha_q, int32_t target_covered, uint64_t *ticket);
/* PDFS_PENDING while queued or running; PDFS_OK with the rounds (up to cap,
 * *n_out = rounds) and latency_ns once done (the ticket is then released);
 * an error code if the solve failed; PDFS_ERR_INVALID_ARG for an unknown
 * ticket. */
int32_t pdfs_server_poll(pdfs_server *s, uint64_t ticket, pdfs_combo *out, int32_t cap,
                         int32_t *n_out, int64_t *latency_ns);
/* Blocks until every submitted request has finished. */
int32_t pdfs_server_drain(pdfs_server *s);
void pdfs_server_destroy(pdfs_server *s);
/* Detail of the last failing pdfs_server_submit / pdfs_server_poll on s (for
 * a failed solve: the ticket and the solve's own error); s = NULL gives the
 * detail of a failed pdfs_server_create on this thread.  The string is a
 * per-thread copy, valid until the calling thread's next call of this
 * function. */
const char *pdfs_server_last_error(const pdfs_server *s);

#ifdef __cplusplus
}
#endif
#endif /* PDFS_H */
