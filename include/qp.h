/*
 * qp.h -- C ABI of the MI355X all-pairs posterior engine.
 *
 * The engine computes stage I of QuickProbs 2 (Gudys & Deorowicz, "QuickProbs 2:
 * Towards rapid construction of high-quality alignments of large protein
 * families"): for every pair of sequences of a family, the posterior
 * probability that residue x_i is aligned with residue y_j, from a pair hidden
 * Markov model and from a partition function over alignments (Methods, opening
 * paragraph), combined into one matrix, kept sparse by a threshold (Methods,
 * "Selective consistency", footnote on the sparsity coefficient; "Other
 * algorithmic improvements", memory as the limit on family size), together
 * with the maximum-expected-accuracy score that stage II turns into a
 * distance (Methods, opening paragraph).
 *
 * Model (the paper names the models but does not restate them; the readings
 * are fixed here):
 *   alignment     monotone sequence of match columns M(i,j), x-gap columns and
 *                 y-gap columns using every residue once; a gap column of x is
 *                 never adjacent to a gap column of y; begin and end behave as
 *                 match columns.
 *   pair-HMM      match emission odds e_ab = p_ab / (qx_a qy_b) from the joint
 *                 p (qx, qy its marginals); G gap classes, M->gap_k delta_k,
 *                 gap_k->gap_k eps_k, gap_k->M 1-eps_k, M->M 1-2*sum(delta).
 *   partition fn  weight exp(score/T), score = sum of s_ab over matches plus
 *                 pf_gap_open + (L-1)*pf_gap_extend for every gap run of
 *                 length L (terminal runs included).
 *   posterior     P = w_hmm * P_hmm + (1 - w_hmm) * P_pf.
 *   sparse form   entries with P >= thresh, CSR per pair, rows = residues of
 *                 the first sequence, columns ascending.
 *   distance      A(i,j) = max(A(i-1,j-1) + P(i,j), A(i-1,j), A(i,j-1)) on the
 *                 dense P; EA = A(m,n) / min(m,n); dist = 1 - EA.
 *
 * Pairs.  In all-pairs mode the pairs of an n-sequence family are (i<j) in
 * row-major order, p = i*n - i*(i+1)/2 + (j-i-1); P(j,i) is P(i,j) transposed
 * (the model is symmetric in x and y).  Explicit pair lists are also accepted.
 *
 * Errors.  Every call returns qp_status; nothing throws across the ABI.  On
 * error, output pointers are set to NULL, nothing is leaked, and
 * qp_last_error() returns a message (thread-local, valid until the next call
 * on that thread).
 *
 * Threads.  Calls from different host threads are safe; calls that share a
 * plan or a server must be serialised by the caller except where stated.
 */
#ifndef QP_H
#define QP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QP_OK = 0,
    QP_EINVAL = -1,      /* invalid argument                                  */
    QP_ENOMEM = -2,      /* host or device memory could not be obtained       */
    QP_EDEVICE = -3,     /* HIP runtime error or no usable gfx950 device      */
    QP_EBUSY = -4,       /* server: result not ready (non-blocking wait)      */
    QP_ETIMEDOUT = -5,   /* server: wait timed out                            */
    QP_ECANCELED = -6,   /* server: request cancelled or server shut down     */
    QP_ENOSPC = -7       /* output capacity exceeded (device-resident calls)  */
} qp_status;

/* QP_MAX_SEQ_LEN: longest sequence accepted.  Longer sequences are refused
 * with QP_EINVAL: banded pairs with more than three 512-row bands are
 * disabled while a GPU memory fault seen on a 3000-5000 residue workload is
 * unexplained (a CPU emulation of the same launches found no out-of-bounds
 * access). */
enum { QP_ALPHA = 20, QP_MAX_GAP_CLASSES = 2, QP_MAX_SEQ_LEN = 1536 };

/* arithmetic of the dynamic programmes */
enum {
    QP_FP32_SCALED = 0,  /* FP32 values, power-of-two scale per lane strip    */
    QP_FP64 = 1          /* FP64 values, same scaling                          */
};

/*
 * Model parameters (raw; the library derives its tables on the device).
 * Residue codes are 0..19 in the order "ARNDCQEGHILKMFPSTWYV".
 * Validation (QP_EINVAL): joint entries in (0,1), summing to 1 within 1e-9 and
 * symmetric within 1e-12; 1 <= n_gap_classes <= 2; delta_k in (0, 0.5),
 * eps_k in [0, 1), 1 - 2*sum(delta) > 0; score symmetric within 1e-12 and
 * finite; temperature > 0; pf gap scores finite; w_hmm in [0,1];
 * precision one of the enum above.
 */
typedef struct {
    double joint[QP_ALPHA * QP_ALPHA];   /* p_ab, row = residue of x         */
    int32_t n_gap_classes;               /* G                                */
    double gap_open[QP_MAX_GAP_CLASSES]; /* delta_k                          */
    double gap_extend[QP_MAX_GAP_CLASSES]; /* eps_k                          */
    double score[QP_ALPHA * QP_ALPHA];   /* s_ab                             */
    double pf_gap_open;                  /* score of the first gap residue   */
    double pf_gap_extend;                /* score of each further gap residue*/
    double temperature;                  /* T                                */
    double w_hmm;                        /* weight of the HMM posterior      */
    int32_t precision;                   /* QP_FP32_SCALED or QP_FP64        */
    int32_t alphabet;                    /* residue codes 0..alphabet-1: 20
                                          * amino acids (0 reads as 20), 4
                                          * nucleotides; 2..20.  joint and
                                          * score keep their 20 x 20 layout;
                                          * joint is 0 outside the
                                          * alphabet x alphabet block       */
} qp_params;

/*
 * Host-resident result (library-owned; release with qp_result_free, never
 * with free()).  The struct and its arrays sit in one host block; blocks of
 * 1 MiB and more are pinned and reused by later results once freed.
 * Pair p covers rows row_off[p] .. row_off[p+1]-1 of row_ptr (m_p + 1 local
 * row pointers starting at 0) and entries nnz_off[p] .. nnz_off[p+1]-1 of
 * col/val.  col is the 0-based residue index in the second sequence.
 */
typedef struct {
    int32_t n_seqs;
    int64_t n_pairs;
    int64_t total_rows;     /* row_off[n_pairs]                               */
    int64_t nnz;            /* nnz_off[n_pairs]                               */
    int32_t* pair_i;        /* [n_pairs] first sequence (rows)                */
    int32_t* pair_j;        /* [n_pairs] second sequence (columns)            */
    int64_t* row_off;       /* [n_pairs + 1]                                  */
    int32_t* row_ptr;       /* [total_rows]                                   */
    int64_t* nnz_off;       /* [n_pairs + 1]                                  */
    int32_t* col;           /* [nnz]                                          */
    float* val;             /* [nnz] combined posterior                       */
    double* dist;           /* [n_pairs] 1 - EA                               */
    double* log_z;          /* [2 * n_pairs] log Z_hmm, log Z_pf per pair     */
    double device_ms;       /* device time of the posterior pipeline          */
    float thresh;           /* sparsity threshold the entries were kept at
                               (the requested one; a served family admitted
                               under a memory budget may have a larger one)  */
} qp_result;

/* Library version, (major << 16) | minor. */
int32_t qp_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* qp_last_error(void);

/* Fill *p with the defaults used by the benchmark workloads: no joint or
 * score (zeros -- the caller must provide them), G = 2 with delta =
 * (0.02, 0.005), eps = (0.5, 0.9), PF gaps -12 / -1, T = 5, w_hmm = 0.5,
 * QP_FP32_SCALED.  Never fails. */
void qp_params_default(qp_params* p);

/* Validate parameters without touching the device.  QP_OK or QP_EINVAL. */
qp_status qp_params_check(const qp_params* p);

/*
 * All-pairs posteriors of one family (the stage-I computation, Methods,
 * opening paragraph).
 *   seqs[n]   host pointers to residue codes (0..19); borrowed for the call
 *   lens[n]   sequence lengths, each >= 1
 *   n         number of sequences (n < 2 gives a result with zero pairs)
 *   params    model, see qp_params
 *   thresh    sparsity threshold in (0, 1]
 *   out       receives a library-owned result on QP_OK, NULL otherwise
 * Runs on the current HIP device on an internal stream and blocks until the
 * result is on the host.  Every plan it makes holds the guaranteed output
 * bound of its pairs (see qp_output_bound), so no run can overflow and none
 * is repeated; when the bound of the whole family exceeds a third of the
 * free device memory, the pairs are cut in order into chunks whose bounds
 * fit, run one after the other, and concatenated into one result.
 * QP_ENOMEM if a single pair's bound cannot be held.
 */
qp_status qp_posteriors(const uint8_t* const* seqs, const int32_t* lens, int32_t n,
                        const qp_params* params, float thresh, qp_result** out);

/* Same for an explicit list of pairs (pair_i[k], pair_j[k]), 0 <= index < n,
 * pair_i[k] != pair_j[k]; rows are residues of seqs[pair_i[k]].  Result pair
 * k is list entry k. */
qp_status qp_posteriors_pairs(const uint8_t* const* seqs, const int32_t* lens, int32_t n,
                              const int32_t* pair_i, const int32_t* pair_j, int64_t n_pairs,
                              const qp_params* params, float thresh, qp_result** out);

/* Release a result (NULL-safe). */
void qp_result_free(qp_result* r);

/*
 * Output size with a guarantee (the sparse output is what limits family size
 * in memory; paper: "Selective consistency", footnote on the sparsity, and
 * the closing discussion).  The posteriors of a row sum to at most one, so a
 * row keeps at most floor(1/thresh) entries at or above the threshold; the
 * kernels give each row floor(1/thresh) + 1 slots (rounding slack), at most
 * its pair's column count.
 *
 * qp_output_bound: *entries = sum over pairs of m * min(n, floor(1/thresh)+1)
 * for the family (pair_i = pair_j = NULL: all pairs i < j) or the pair list.
 *
 * qp_threshold_for_budget: *thresh = the smallest threshold whose bound is
 * at most max_entries (when even the dense output fits, the threshold at
 * which rows first keep every column).  QP_ENOSPC if even thresh = 1 (two
 * slots per row) does not fit.  Both: QP_EINVAL for invalid lengths, pairs
 * or threshold.  Host computation only.
 */
qp_status qp_output_bound(const int32_t* lens, int32_t n, const int32_t* pair_i, const int32_t* pair_j,
                          int64_t n_pairs, float thresh, int64_t* entries);
qp_status qp_threshold_for_budget(const int32_t* lens, int32_t n, const int32_t* pair_i, const int32_t* pair_j,
                                  int64_t n_pairs, int64_t max_entries, float* thresh);

/* ------------------------------------------------------------------------
 * Device-resident form.  A plan fixes the family shape (lengths, pair list,
 * parameters, threshold), owns the device workspace and output buffers and
 * a captured HIP graph of the whole pipeline.  Inputs are device pointers
 * the caller owns (for instance torch tensors); the stream is the caller's.
 * ---------------------------------------------------------------------- */
typedef struct qp_plan qp_plan;

/* Device pointers into plan-owned outputs, valid until the next run or
 * qp_plan_destroy.  Layout as qp_result. */
typedef struct {
    int64_t n_pairs;
    int64_t total_rows;
    int64_t nnz;            /* filled by qp_plan_sync                         */
    const int32_t* pair_i;
    const int32_t* pair_j;
    const int64_t* row_off;
    const int32_t* row_ptr;
    const int64_t* nnz_off;
    const int32_t* col;
    const float* val;
    const double* dist;
    const double* log_z;
} qp_device_result;

/*
 * Create a plan on the current device.
 *   lens[n]          host copy of the sequence lengths
 *   pair_i, pair_j   NULL for all pairs, else a host pair list of n_pairs
 *   nnz_capacity     capacity of the sparse output (entries); 0 lets the
 *                    library estimate it; -1 sizes it to qp_output_bound, so
 *                    no run can overflow; a run that overflows reports
 *                    QP_ENOSPC from qp_plan_sync with the entries it needed,
 *                    and a new plan with at least that capacity must be made
 * Allocates device memory (QP_ENOMEM if it cannot).
 */
qp_status qp_plan_create(const int32_t* lens, int32_t n, const int32_t* pair_i, const int32_t* pair_j,
                         int64_t n_pairs, const qp_params* params, float thresh, int64_t nnz_capacity,
                         qp_plan** plan);

/* Enqueue the whole pipeline on `stream` (a hipStream_t, NULL = legacy
 * default).  d_seqs: residue codes of all sequences concatenated; d_seq_off:
 * int64 start offset of each sequence in d_seqs ([n]); both device pointers,
 * read during the run.  Asynchronous. */
qp_status qp_plan_run(qp_plan* plan, const uint8_t* d_seqs, const int64_t* d_seq_off, void* stream);

/* Wait for the last run on its stream, check for output overflow and fill
 * *res (may be NULL).  QP_ENOSPC if the sparse output did not fit: res->nnz
 * then holds the number of entries the run produced (every other field is
 * zero) and the plan is unchanged; create a plan with nnz_capacity >= that. */
qp_status qp_plan_sync(qp_plan* plan, qp_device_result* res);

/* Copy the last run's outputs to a library-owned host result. */
qp_status qp_plan_download(qp_plan* plan, qp_result** out);

/* Average device time (ms) of the posterior kernel and of the whole
 * pipeline over the runs since the last reset, from HIP events recorded on
 * the run stream; *n_runs receives the number of runs averaged. */
qp_status qp_plan_timing(qp_plan* plan, double* kernel_ms, double* pipeline_ms, int64_t* n_runs, int32_t reset);

/* Kernel classes of a plan: 0..7 run row sequences of at most 512 in one
 * band of 64 R rows, R = 1..8 rows per lane of a 64-lane wavefront (the
 * class of a pair set by the tuning table's rows_per_lane); 8..11 cut a
 * longer row sequence into nb = ceil(m / 512) bands of 64 R rows with
 * R = 5..8 = ceil(m / (64 nb)) (R = 4, bands of 256 rows, in the
 * checkpointed form).  The tuning table's banded entry applies to all four. */
#define QP_KERNEL_CLASSES 12

/* One kernel class of the plan: pairs run with *rows_per_lane rows per lane.
 * *pairs and *cells are the pairs and m*n cells of this family in the class
 * (0 when it is absent); *kernel_ms is the average duration of the class's
 * persistent kernel over the timed runs (events recorded on the stream it
 * runs on; reset together with qp_plan_timing).  Any output pointer may be
 * NULL.  QP_EINVAL for a class outside [0, QP_KERNEL_CLASSES). */
qp_status qp_plan_class_timing(qp_plan* plan, int32_t cls, double* kernel_ms, int64_t* pairs, int64_t* cells,
                               int32_t* rows_per_lane);

/* Use (1) or stop using (0) the captured HIP graph for subsequent runs
 * (default 1). */
qp_status qp_plan_set_graph(qp_plan* plan, int32_t use_graph);

/* Run the plan in the plain per-pair form (1) or the batched form (0, the
 * default).  The per-pair form launches the pair kernel once per pair, one
 * wavefront, in pair order on the run stream, with no graph and no work
 * queue; it is the baseline the batched form is measured against.  The
 * setup, scan and gather steps and every output are the same as in the
 * batched form; qp_plan_class_timing reports nothing for per-pair runs.
 * QP_ENOMEM if the per-pair class list cannot be allocated. */
qp_status qp_plan_set_per_pair(qp_plan* plan, int32_t on);

/*
 * Tuning table (process-wide; plans copy it when they are made).  Entries
 * c = 0..7 are the single-band classes (R = c + 1 rows per lane of a 64-lane
 * wavefront), entry 8 the banded classes 8..11 together (row sequences
 * longer than 512).  A pair whose row sequence needs at least r = ceil(m/64)
 * rows per lane runs with rows_per_lane[r-1] (r..8) rows per lane; every
 * class launches waves_frac[c] (0, 1] of its occupancy-limited persistent
 * grid.
 * recompute[c] = 1 runs class c's FP32 pairs in the checkpointed form: the
 * forward sweep keeps only its state every 8 steps and the backward sweep
 * recomputes each 8-step block's forward values in registers, instead of
 * writing every cell's forward values to device memory and reading them
 * back (recompute[c] = 0); same outputs, different memory / arithmetic
 * balance.  The checkpointed form exists for classes 0..4 (1 to 5 rows per
 * lane) and for the banded classes, which it runs in bands of 256 rows (4
 * per lane) (QP_EINVAL for recompute[c] = 1 on classes 5..7);
 * the FP64 path always uses the other form.
 * Default: rows_per_lane[r-1] = r, waves_frac = 1, recompute = 1 for the
 * classes of 1 to 5 rows per lane (the banded classes are faster spilling).
 * concurrent_classes = 1 runs a plan's kernel classes side by side on forked
 * streams (one class's tail overlaps the next one's work); 0 runs them one
 * after another on the run stream, largest rows per lane first, each with
 * the whole device (and one workspace shared by all classes).  Default 1.
 * orient = 1 lets a plan sweep a pair with its second sequence as rows when
 * a cost model of the kernel classes (lane-steps of the sweep times a
 * measured cost per class) finds that cheaper and both models' tables are
 * exactly symmetric, so that P(y, x) = P(x, y)^T; the output rows are the
 * first sequence's either way.  0 sweeps every pair with the first
 * sequence as rows.  Default 1; qp_posteriors_noalloc never transposes.
 * Filled in by the project's autotuner (paper_1512_07437_amd/autotune.py)
 * from measurements per length bucket.
 */
typedef struct {
    int32_t rows_per_lane[8];
    double waves_frac[9];
    int32_t recompute[9];
    int32_t concurrent_classes;
    int32_t orient;
} qp_tuning;

/* Set the table (NULL restores the default); QP_EINVAL for a value out of
 * range, the table then unchanged. */
qp_status qp_set_tuning(const qp_tuning* t);
qp_status qp_get_tuning(qp_tuning* t);

/* Device bytes held by the plan. */
int64_t qp_plan_device_bytes(const qp_plan* plan);

void qp_plan_destroy(qp_plan* plan);

/* ------------------------------------------------------------------------
 * Allocation-free form, for callers that cannot allocate device memory:
 * code under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same kernels and outputs as a plan created with nnz_capacity =
 * -1 and run once; no device or host allocation is made on success.
 * ---------------------------------------------------------------------- */

/* Size of the fixed device workspace behind qp_posteriors_noalloc: one
 * array per device, held from the first call on that device until the
 * process ends (256 MiB). */
#define QP_NOALLOC_SCRATCH_BYTES (256 * 1024 * 1024)

/* Caller-owned device outputs (layout as qp_result) and a status word. */
typedef struct {
    int32_t* pair_i;        /* [P] P = n(n-1)/2, pairs i < j in row-major order */
    int32_t* pair_j;        /* [P]                                            */
    int64_t* row_off;       /* [P + 1]                                        */
    int32_t* row_ptr;       /* [sum over pairs of lens[i] + 1]                */
    int64_t* nnz_off;       /* [P + 1]; nnz_off[P] = entries written          */
    int32_t* col;           /* [capacity]                                     */
    float* val;             /* [capacity]                                     */
    int64_t capacity;       /* entries col / val hold: >= qp_output_bound     */
    double* dist;           /* [P]                                            */
    double* log_z;          /* [2P]                                           */
    int32_t* status;        /* [1] written at the end of the run: 0 = OK;
                               bit 2 (4): a residue code outside the
                               alphabet; bit 1 (2): a row held more entries
                               than its slots; bit 0 (1): output overflow
                               (cannot happen at capacity >= the bound)     */
} qp_noalloc_out;

/*
 * All-pairs posteriors of one family with no allocation: every workspace
 * buffer (tables, aligned sequence copy, pair schedule, output pool, per-wave
 * scratch) is carved out of the fixed QP_NOALLOC_SCRATCH_BYTES device array.
 *   d_seqs, d_seq_off  device inputs as for qp_plan_run
 *   lens[n], params, thresh  host values as for qp_plan_create
 *   out                caller-owned device outputs, sized as documented
 *   stream             hipStream_t (NULL = legacy default)
 * Asynchronous: every step is enqueued on `stream`; the outputs and
 * out->status are valid once it has been synchronised.  Fewer waves run than
 * in a plan when the per-wave scratch of the family's longest pairs does not
 * fit the remaining workspace for a full grid.  QP_ENOMEM (before anything
 * is enqueued) when the tables, pair lists, an output pool of the bound's
 * size and one block of waves do not fit the workspace; QP_EINVAL for
 * invalid inputs or out->capacity below qp_output_bound.  Every call on a
 * device shares that device's workspace and leaves its contents behind:
 * calls that overlap on one device (different streams or threads without
 * ordering) race and must be serialised by the caller.
 */
qp_status qp_posteriors_noalloc(const uint8_t* d_seqs, const int64_t* d_seq_off, const int32_t* lens, int32_t n,
                                const qp_params* params, float thresh, const qp_noalloc_out* out, void* stream);

/* ------------------------------------------------------------------------
 * Guide tree (the stage after the posteriors; paper: Methods, opening
 * paragraph -- weighted UPGMA on the pairwise distances -- and "Selective
 * consistency" -- the tree-guided distance).  Host memory, host computation.
 * ---------------------------------------------------------------------- */

/*
 * Weighted UPGMA (WPGMA) over n sequences.
 *   dist     [n(n-1)/2] distances in pair order p = i*n - i*(i+1)/2 + (j-i-1)
 *            (the dist array of qp_result); finite values
 *   merges   [2(n-1)] out: step k joins clusters merges[2k] < merges[2k+1];
 *            ids 0..n-1 are the sequences, id n+k is the cluster made at step k
 *   heights  [n-1] out: half the distance at which step k joins
 * Each step joins the two closest clusters; the joined cluster's distance to
 * any other is the plain mean of the two (each side weighs the same,
 * whatever its size).  Equal distances: the pair with the smaller smaller
 * id, then the smaller larger id.  QP_EINVAL for n outside [1, 32768], a
 * NULL array (n > 1) or a value that is not finite; QP_ENOMEM when the
 * working copy of the distances cannot be allocated.  n = 1: nothing to do.
 */
qp_status qp_guide_tree(const double* dist, int32_t n, int32_t* merges, double* heights);

/*
 * Tree-guided distance of every pair (i < j), in pair order: the number of
 * nodes (sequences and joins) of the smallest subtree holding both, i.e. of
 * the subtree under their first common join, 2L - 1 for L sequences under it.
 *   merges   [2(n-1)] a tree as qp_guide_tree writes it
 *   out      [n(n-1)/2] out
 * QP_EINVAL if a step does not join two existing, not yet joined clusters.
 */
qp_status qp_tree_distance(const int32_t* merges, int32_t n, int32_t* out);

/* ------------------------------------------------------------------------
 * Selective consistency (the stage that consumes the posteriors and the
 * guide tree; paper: Methods, "Selective consistency", and "Other
 * algorithmic improvements" for the number of passes).  Every pair's sparse
 * matrix is relaxed through the third sequences z the tree selects:
 *   Z_xy  = { z not x, y : max(d_xz, d_yz) <= tree_threshold }  (tree-guided
 *           distances as qp_tree_distance gives them)
 *   h_xy  = 1 + (amplification - 1) |Z_xy| / (n - 2)   (1 when n = 2)
 *   S'_xy = (2 h_xy S_xy + sum over z in Z_xy of S_xz S_zy) / (2 h_xy + |Z_xy|)
 * with S_ab = S_ba transposed for a > b, entries below thresh dropped; each
 * pass relaxes every pair from the previous pass's matrices (the paper uses
 * two passes below 50 sequences, one otherwise; T about 200, amplification
 * 3).  Device memory, the caller's stream; FP32 accumulation.
 * ---------------------------------------------------------------------- */
typedef struct qp_relax qp_relax;

/*
 * Workspace for one family shape (all pairs i < j of n sequences).
 *   lens[n]         host sequence lengths (validated as for qp_plan_create)
 *   in_capacity     entries of the input CSR it will be given (0: the
 *                   output bound of the family at thresh, see
 *                   qp_output_bound); the relaxed outputs are sized to that
 *                   bound, so no pass can overflow
 * QP_EINVAL for n > 2048, a negative threshold, amplification < 1, passes
 * outside [1, 8] or thresh outside (0, 1]; QP_ENOMEM when the workspace
 * cannot be allocated.
 */
qp_status qp_relax_create(const int32_t* lens, int32_t n, int64_t in_capacity, int32_t tree_threshold,
                          double amplification, int32_t passes, float thresh, qp_relax** relax);

/* Enqueue every pass on `stream`.  in: device CSR of all pairs in the
 * layout of qp_device_result (for instance what qp_plan_sync returns for an
 * all-pairs plan), holding in_nnz entries; d_tdist: device int32 [n(n-1)/2]
 * tree-guided distances in pair order.  Inputs are read during the run.
 * One run at a time per workspace (a new run waits for the last). */
qp_status qp_relax_run(qp_relax* relax, const qp_device_result* in, int64_t in_nnz, const int32_t* d_tdist,
                       void* stream);

/* Wait for the run and fill *out (may be NULL) with device pointers into
 * workspace-owned outputs (layout of qp_device_result), valid until the next
 * run or qp_relax_destroy. */
qp_status qp_relax_sync(qp_relax* relax, qp_device_result* out);

/* Copy the relaxed matrices to a library-owned host result (qp_result_free). */
qp_status qp_relax_download(qp_relax* relax, qp_result** out);

/* Device bytes held by the workspace. */
int64_t qp_relax_device_bytes(const qp_relax* relax);

void qp_relax_destroy(qp_relax* relax);

/* ------------------------------------------------------------------------
 * Serving: families arrive over time; each is admitted when the free device
 * memory budget covers its workspace and outputs and a slot is free; admitted
 * families run concurrently on a pool of streams (continuous batching), and
 * each result is identical to the result of the same family run alone.
 * ---------------------------------------------------------------------- */
typedef struct qp_server qp_server;

typedef struct {
    int64_t hbm_budget_bytes;   /* device memory the server may hold (> 0)  */
    int32_t max_slots;          /* families in flight at once (1..64)       */
    int32_t n_streams;          /* streams in the pool (1..16)              */
} qp_server_config;

typedef struct {
    double submit_s;            /* host clock at submit (seconds)           */
    double admit_s;             /* host clock when admitted                 */
    double done_s;              /* host clock when the result was ready     */
    int64_t cells;              /* sum of m*n over the family's pairs       */
    double launched_s;          /* host clock when its work was enqueued    */
    double device_s;            /* host clock when its device work was seen
                                   finished (the download follows)          */
} qp_request_times;

/* Create a server on the current device (starts one scheduler thread). */
qp_status qp_server_create(const qp_server_config* cfg, qp_server** s);

/* Submit a family; inputs are copied.  QP_ENOMEM if the family could never
 * fit in the budget.  Thread-safe. */
qp_status qp_server_submit(qp_server* s, const uint8_t* const* seqs, const int32_t* lens, int32_t n,
                           const qp_params* params, float thresh, uint64_t* ticket);

/* Wait for a ticket: timeout_ms < 0 blocks, 0 polls (QP_EBUSY if not
 * ready).  On QP_OK the result is handed over (free with qp_result_free) and
 * the ticket is retired.  Thread-safe. */
qp_status qp_server_wait(qp_server* s, uint64_t ticket, int32_t timeout_ms, qp_result** out,
                         qp_request_times* times);

/* Cancel a queued (not yet admitted) request.  QP_EBUSY if already running. */
qp_status qp_server_cancel(qp_server* s, uint64_t ticket);

/* Counters: families queued, in flight, finished; device bytes in use. */
qp_status qp_server_stats(qp_server* s, int64_t* queued, int64_t* in_flight, int64_t* finished,
                          int64_t* bytes_in_use);

/* Stop the scheduler; waits for in-flight work; pending requests are
 * cancelled. */
qp_status qp_server_destroy(qp_server* s);

#ifdef __cplusplus
}
#endif

#endif /* QP_H */
