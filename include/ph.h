/*
 * ph.h - C ABI of libpairhmm: the Pair-HMM forward algorithm and its adjoint
 * on AMD Instinct MI355X (gfx950).
 *
 * What is computed (arXiv 2411.11547, Section II-A): for a read R = r_1..r_m
 * and a haplotype H = h_1..h_n over {A,C,G,T,N}, the match/insert/delete
 * recurrences Eq. (1)-(3) with emissions Eq. (4), initialised with
 * M(i,0) = I(i,0) = D(i,0) = 0, M(0,j) = I(0,j) = 0, D(0,j) = 1/n, give the
 * likelihood L = sum_{j=1..n} (M(m,j) + I(m,j)).  Every call returns
 * log10 L for every read/haplotype pair of a list of batches
 * B_q = (R_q, H_q) (Section II-A, last paragraph; Section III-A).
 *
 * Conventions fixed by this library where the paper leaves them open:
 *  - Phred decoding per read position: Q = 10^(-q/10) for the base quality,
 *    delta = 10^(-ins/10), zeta = 10^(-del/10), eps = 10^(-gcp/10),
 *    alpha = 1 - delta - zeta, beta = 1 - eps, lam_match = 1 - Q,
 *    lam_mismatch = Q / 3.
 *  - Base codes: A=0, C=1, G=2, T=3, N=4; N on either side is a match.
 *  - D(0,0) = 1/n (the zero initialisation covers rows i >= 1 only).
 *
 * Memory: unless stated otherwise every pointer is DEVICE memory (hipMalloc
 * or torch CUDA tensors), owned by the caller, and must stay valid until the
 * work enqueued on `stream` has completed.  The plan owns its scratch.
 *
 * Streams: calls enqueue work on `stream` (a hipStream_t; NULL = the null
 * stream) and return without waiting; results are valid once the stream has
 * been synchronised.  A plan must not be used from two streams at once.
 *
 * Errors: every function returns a ph_status and never aborts or throws.
 * ph_last_error() returns a message for the most recent failure of the
 * calling thread.
 */
#ifndef PH_H
#define PH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PH_OK = 0,
    PH_ERR_INVALID = -1,       /* bad argument: NULL pointer, empty read or haplotype, bad code */
    PH_ERR_UNSUPPORTED = -2,   /* read longer than 65535 bases (forward) or 319 (adjoint) */
    PH_ERR_NOMEM = -3,         /* device or host allocation failed */
    PH_ERR_HIP = -4,           /* a HIP runtime call failed; see ph_last_error() */
    PH_ERR_PLAN_MISMATCH = -5, /* the problem does not have the shape the plan was built for */
    PH_ERR_STATE = -6          /* call order violated (e.g. backward without a checkpointed forward) */
} ph_status;

/* Per-pair status written next to each score. */
enum {
    PH_PAIR_FP32 = 0,           /* FP32 sweep, scaled sum above the underflow threshold */
    PH_PAIR_FP64 = 1,           /* recomputed by the FP64 sweep: the FP32 sum was out of range,
                                   or a read row i below the first has alpha_i < 2^-20 or
                                   eps_i delta_{i-1} / delta_i > 2^20 (the FP32 sweep's
                                   rescaled states divide by both; Phred gap-open qualities
                                   of 3 or less, a gap-open quality rising by more than 60
                                   between neighbouring bases, or explicit delta = 0) */
    PH_PAIR_FP64_FLOOR = 2,     /* FP64 sweep, but below its own range floor: unreliable */
    PH_PAIR_FP32_UNRESCUED = 3  /* FP32 below threshold in a mode without rescue */
};

/* Shape of a problem: batch structure and sequence lengths, HOST memory.
 * Reads of batch q are batch_read_begin[q] .. batch_read_begin[q+1]-1, its
 * haplotypes batch_hap_begin[q] .. batch_hap_begin[q+1]-1; read r spans
 * read_offset[r] .. read_offset[r+1]-1 of the per-base arrays, haplotype h
 * spans hap_offset[h] .. hap_offset[h+1]-1 of hap_bases. */
typedef struct {
    int32_t num_batches;
    const int32_t *batch_read_begin; /* [num_batches + 1], non-decreasing, starts at 0 */
    const int32_t *batch_hap_begin;  /* [num_batches + 1], non-decreasing, starts at 0 */
    int32_t num_reads;
    const int64_t *read_offset;      /* [num_reads + 1] */
    int32_t num_haps;
    const int64_t *hap_offset;       /* [num_haps + 1] */
} ph_shape;

/* The data of a problem, DEVICE memory, same structure as ph_shape.  The
 * CSR arrays must hold the values the plan was built from. */
typedef struct {
    int32_t num_batches;
    const int32_t *batch_read_begin; /* [num_batches + 1] */
    const int32_t *batch_hap_begin;  /* [num_batches + 1] */
    int32_t num_reads;
    const int64_t *read_offset;      /* [num_reads + 1] */
    const uint8_t *read_bases;       /* [read_offset[num_reads]] codes 0..4 */
    const uint8_t *base_qual;        /* Phred per read base */
    const uint8_t *ins_qual;         /* Phred of an insertion starting after this base */
    const uint8_t *del_qual;         /* Phred of a deletion starting after this base */
    const uint8_t *gcp_qual;         /* Phred of gap continuation */
    int32_t num_haps;
    const int64_t *hap_offset;       /* [num_haps + 1] */
    const uint8_t *hap_bases;        /* [hap_offset[num_haps]] codes 0..4 */
} ph_problem;

typedef struct {
    /* Scaled FP32 row-m sum below which a pair is recomputed in FP64.
     * The FP32 sweep starts from D(0,j) = 2^120 / n, so the default 1e-28
     * corresponds to log10 L of about -64.1.  <= 0 selects the default;
     * +inf sends every pair to the FP64 sweep. */
    double rescue_threshold;
    int use_graph;         /* 1: capture the launch sequence of ph_forward_batch (three
                              stage graphs) and of ph_backward_batch once per set of
                              buffers and replay it */
    int plain;             /* 1: one FP32 kernel sized for the longest read, pairs
                              in output order, no binning, no rescue (baseline) */
    int force_p;           /* 0 = tuned; else lanes per pair (4, 8, 16, 32 or 64) for every
                              bin (4 lanes: reads up to 63, 8 lanes: up to 127) */
    int keep_checkpoints;  /* 1: build the adjoint's tables and workspace at plan
                              time (else on the first ph_backward_batch) */
    const char *tune_table_path; /* NULL = built-in table; else a text file of
                                    "max_read_len lanes rows_per_lane" lines */
    int single_launch;     /* 1: one persistent FP32 launch drains every bin when all
                              non-empty bins use 16 lanes and 3..16 rows per lane
                              (reads up to 255); otherwise one launch per bin */
} ph_plan_opts;

typedef struct ph_plan ph_plan; /* opaque: owns scratch, queues, checkpoints, graph */

/* Fill opts with defaults. */
void ph_plan_opts_default(ph_plan_opts *opts);

/* Build a plan for problems of the given shape (HOST arrays, read once):
 * the partitioning of the pairs by read length into (lanes per pair, rows
 * per lane) configurations, each with its own work list (Section III-C).
 * The lists depend on the shape alone, so the plan builds them once, on the
 * host, and uploads them: in configurations of 16 or more lanes a tile
 * holds 64/lanes reads of one batch, each swept against a run of the
 * batch's haplotypes one after the other (a chain); the remaining pairs
 * form tiles of single pairs, longest haplotype first.  (The on-device
 * sorting of a batch list into such lists, Section III-A stage 3, serves
 * ph_forward_batch_noalloc, which has no plan.)  This is the `ph_plan` call
 * of the library's call list, named ph_plan_create because C cannot give a
 * function the name of the ph_plan type.
 * Validates the shape: batch ranges inside the read/haplotype counts, every
 * read and haplotype non-empty (PH_ERR_INVALID), every read at most 65535
 * bases (PH_ERR_UNSUPPORTED; plain mode: 1023); then sizes and allocates
 * device scratch on the current device.  Reads of up to 1023 bases are
 * binned by length; longer reads are swept in windows of 1024 rows whose
 * boundary rows (3 values per haplotype column) live in plan scratch.
 * The plan owns its scratch, streams and graphs until ph_plan_destroy.
 * *out receives the plan. */
ph_status ph_plan_create(const ph_shape *shape, const ph_plan_opts *opts, ph_plan **out);

/* Number of pairs P = sum_q |R_q| |H_q| and real cells sum_pairs m*n. */
ph_status ph_plan_info(const ph_plan *plan, int64_t *num_pairs, int64_t *num_cells,
                       int32_t *max_read_len, int32_t *max_hap_len);

/* Forward pass (Section III-B): out_log10L[P] (device, double) receives
 * log10 L of every pair, in batch-major, read, haplotype order;
 * out_status[P] (device, uint8, may be NULL) the per-pair ph status.
 * log10_params: NULL to derive parameters from the Phred arrays, else a
 * device float array [read_offset[num_reads]][7] of log10 probabilities
 * {alpha, beta, delta, eps, zeta, lam_match, lam_mismatch} per read base.
 * The problem's counts must equal the plan's (PH_ERR_PLAN_MISMATCH). */
ph_status ph_forward_batch(ph_plan *plan, const ph_problem *problem,
                           const float *log10_params, double *out_log10L,
                           uint8_t *out_status, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): the forward
 * pass of ph_forward_batch without a plan.  It allocates nothing: its
 * scratch (pair records, binning counters, FP64 queues, linear parameters)
 * is one fixed array of 7.5 MB inside the library, one copy per GPU,
 * held until the process ends.  Arguments as ph_forward_batch, with the
 * shape (HOST arrays, read during the call) in place of the plan; the
 * pairs of a plan built with the library's own bin table (tune_table_path
 * NULL, force_p 0) and the default rescue threshold, each as a single pair
 * (no chains): the same statuses, the same FP64 values, FP32 values to
 * rounding (a chain groups the FP32 partial sums of the row-m sum by other
 * column blocks).
 * Limits: at most 65536 pairs, 16384 batches, reads of 1..1023 bases, and
 * with log10_params at most 65536 read bases; larger problems give
 * PH_ERR_UNSUPPORTED before any device work.  Counts that differ between
 * shape and problem give PH_ERR_PLAN_MISMATCH.
 * The first call on each device sets up that device (the array's address,
 * constant tables) and must not itself be captured; later calls enqueue
 * kernels only.  Every call on one GPU shares that GPU's array: calls whose
 * work overlaps on the device (two streams, or two host threads) race, so
 * order them on one stream or with events. */
ph_status ph_forward_batch_noalloc(const ph_shape *shape, const ph_problem *problem,
                                   const float *log10_params, double *out_log10L,
                                   uint8_t *out_status, void *stream);

/* Viterbi score (the max-product form of Eq. (1)-(3): every sum over
 * predecessor states a maximum, and the largest M(m,j) or I(m,j) instead of
 * their sum): out_log10V[P] receives log10 of the probability of each pair's
 * most probable alignment path, with the same binning, FP64 rescue, status
 * codes, arguments and output order as ph_forward_batch.  Not available in
 * plain mode (PH_ERR_UNSUPPORTED). */
ph_status ph_viterbi_batch(ph_plan *plan, const ph_problem *problem,
                           const float *log10_params, double *out_log10V,
                           uint8_t *out_status, void *stream);

/* Adjoint pass: grad_params[read_offset[num_reads]][7] (device, float)
 * receives d(sum_p u_p log10 L_p)/d log10 theta for the seven parameters of
 * every read base, u = grad_log10L[P] (device, double).  The derivative of
 * Eq. (1)-(4) run backwards; d log10 L / d log10 theta is the posterior
 * expected number of uses of theta.  The call is self-contained: it runs its
 * own checkpointed FP32 forward (every lane's state, i.e. every K-th row,
 * at a fixed interval of columns) and then the reverse sweep, so it needs no
 * preceding ph_forward_batch and keep_checkpoints only moves the set-up of
 * its tables to plan creation (the forward call's own scores are not
 * reused: the adjoint's lane layout differs from the forward's bins).  Pairs
 * whose scaled FP32 sum falls below the plan's rescue threshold (or
 * overflows), or with a read row below the first whose beta is below 2^-20
 * (the adjoint's rescaled states divide by beta; Phred gap continuation 0
 * gives beta = 0), are redone in FP64; only pairs below the
 * FP64 floor (log10 L < about -608) get NaN gradients, and pairs with
 * u_p = 0 contribute nothing.  The gradient buffer is overwritten.  Reads
 * longer than 319 bases give PH_ERR_UNSUPPORTED.  Deterministic: each pair
 * writes its own gradient rows, and the rows of a read with several pairs
 * are summed in haplotype order in FP64, so replays give identical bits. */
ph_status ph_backward_batch(ph_plan *plan, const ph_problem *problem,
                            const float *log10_params, const double *grad_log10L,
                            float *grad_params, void *stream);

/* Check the device data of a problem against the plan: every base code in
 * 0..4.  Synchronous; PH_ERR_INVALID if a code is out of range.  The forward
 * pass itself does not read-validate device data: the kernels read codes
 * above 4 as N.  Uses a counter of its own, so the bookkeeping of the last
 * forward call (ph_plan_rescued) is left as it was. */
ph_status ph_validate(ph_plan *plan, const ph_problem *problem, void *stream);

/* Kernel-level timing of the most recent ph_forward_batch / ph_backward_batch
 * on this plan, from HIP events recorded on the call's stream around each
 * stage.  ms[0] = binning, ms[1] = FP32 sweep, ms[2] = FP64 rescue,
 * ms[3] = adjoint sweep.  Synchronises the stream. */
ph_status ph_plan_stage_ms(ph_plan *plan, float ms[4]);

/* Number of pairs sent to an FP64 sweep by the most recent forward call,
 * those of reads longer than 1023 bases (windowed sweep) included; equal to
 * the number of pairs with status PH_PAIR_FP64 or PH_PAIR_FP64_FLOOR
 * (synchronises the stream). */
ph_status ph_plan_rescued(ph_plan *plan, int64_t *count);

void ph_plan_destroy(ph_plan *plan);

/* ---- Streaming forward over host-resident batches ------------------------
 * The workflow of Section III-A: the batches are cut into subsets of whole
 * batches, subset k+1 is copied to the GPU while subset k is binned and
 * computed (one plan per subset), and each subset's scores are copied back as
 * soon as it finishes.  Copies overlap compute only when the host arrays are
 * pinned (allocate them with ph_host_alloc); pageable arrays work but their
 * copies are staged by the runtime. */
typedef struct {
    int64_t max_subset_cells; /* cells (sum of m*n) per subset; a larger batch forms a
                                 subset of its own; <= 0 selects 6e10 */
    int32_t buffer_sets;      /* device input/output buffer sets, reused in turn; 0: one per
                                 subset when all of them take at most a quarter of the free
                                 device memory (then no copy waits for compute), else 2;
                                 values are clamped to 2 .. number of subsets */
    ph_plan_opts plan;        /* options of every subset's plan */
} ph_pipeline_opts;

typedef struct ph_pipeline ph_pipeline; /* opaque: subset plans, device buffer sets, streams */

void ph_pipeline_opts_default(ph_pipeline_opts *opts);

/* Partition the shape (HOST arrays, read once) into subsets and create their
 * plans and the device buffers on the current device.  Errors as
 * ph_plan_create. */
ph_status ph_pipeline_create(const ph_shape *shape, const ph_pipeline_opts *opts, ph_pipeline **out);

ph_status ph_pipeline_info(const ph_pipeline *pipe, int32_t *num_subsets, int64_t *num_pairs,
                           int64_t *num_cells);

/* Forward pass of a problem held in HOST memory (every ph_problem array is a
 * host pointer; the CSR arrays must match the shape).  out_log10L[P] and
 * out_status[P] (may be NULL) are HOST arrays in the order of
 * ph_forward_batch.  Synchronous: returns when the scores are on the host. */
ph_status ph_pipeline_forward(ph_pipeline *pipe, const ph_problem *host_problem, double *out_log10L,
                              uint8_t *out_status);

/* Milliseconds from the first host-to-device copy to the last device-to-host
 * copy of the most recent ph_pipeline_forward, from HIP events. */
ph_status ph_pipeline_ms(ph_pipeline *pipe, float *ms);

void ph_pipeline_destroy(ph_pipeline *pipe);

/* Pinned host memory for pipeline inputs and outputs (hipHostMalloc); NULL on
 * failure. */
void *ph_host_alloc(size_t bytes);
void ph_host_free(void *ptr);

/* Message of the calling thread's most recent failure ("" if none).  It
 * takes no plan: the message is kept per thread, so it also covers calls
 * that failed before a plan existed (ph_plan_create, ph_pipeline_create). */
const char *ph_last_error(void);

/* Library version string. */
const char *ph_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PH_H */
