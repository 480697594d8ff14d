/*
 * rqa.h -- C ABI of the MI355X (gfx950) library for the hot path of averaged
 * recurrence quantification analysis (Panis, Adamek & Marwan, "Averaged
 * Recurrence Quantification Analysis", arXiv 2208.09136).
 *
 * What the library computes, for a float32 series y[0..n-1]:
 *   - delay vectors x(t) = [y(t), y(t-tau), ..., y(t-(m-1)tau)] (Methodology,
 *     Lorenz-system subsection).  Vector i (0-based) has component k equal to
 *     y[i + (m-1-k)tau]; there are nv = n - (m-1)tau vectors.
 *   - a key per pair i < j: the maximum norm max_k |d_k| (Recurrence
 *     quantification analysis section, after Eq. 1) or the squared Euclidean
 *     norm, summed left to right over k = 0..m-1, every operation rounded to
 *     binary32 and no fused multiply-add; d_k = y[i+(m-1-k)tau] -
 *     y[j+(m-1-k)tau].  Euclidean thresholds are therefore in squared units.
 *   - the recurrence matrix of Eq. 1 over the upper triangle j > i
 *     (Technical implementation on a GPU), restricted to j - i >= theiler:
 *     M = (nv-theiler)(nv-theiler+1)/2 pairs.  A pair recurs at threshold
 *     eps iff key <= eps (equal to the paper's strict Heaviside at the next
 *     float above eps).
 *   - the threshold for a preselected recurrence rate RR (Averaged RQA
 *     section): the k-th smallest key, k = ceil(RR * M) with RR quantised to
 *     1e-9 and k clamped to [1, M].
 *   - RR (Eq. 3) = C / M with C = #{key <= eps}, the diagonal-line
 *     determinism DET (Eq. 4) = (points on diagonal lines of length >= lmin)
 *     / C, and the averaged DET (the averaged-determinism equation of the
 *     Averaged RQA section) = mean of DET over the given RR targets.  Lines
 *     that touch the border of the plot count with their length inside it.
 *
 * Conventions for every call:
 *   - All functions return rqa_status; nothing throws or aborts.  On an
 *     error the outputs are left untouched and rqa_last_error() describes it.
 *   - Series pointers are DEVICE pointers on the context's device; every
 *     *_out pointer and every other array argument is HOST memory.  The
 *     caller owns all of them; the library never keeps a pointer past a call.
 *   - Calls are ordered on the context's stream and synchronise with it
 *     before returning; outputs are complete on return.
 *   - A context is not thread-safe: use one context per host thread.
 *   - n must be < 2^31.  K (number of RR targets or thresholds) is 1..128.
 */
#ifndef RQA_H
#define RQA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RQA_MAX_K 128
#define RQA_MAX_HIST_K 32          /* thresholds of one full-histogram pass over the pairs */
#define RQA_MAX_HIST_LEN (1u << 24) /* entries per full-histogram row */

typedef struct rqa_ctx rqa_ctx;

typedef enum {
    RQA_OK = 0,
    RQA_ERR_INVALID_ARG = -1, /* null pointer, zero m/tau/theiler/lmin, K out of range, bad RR or eps, unknown norm/flag */
    RQA_ERR_TOO_SHORT = -2,   /* nv <= theiler: there is no pair to evaluate */
    RQA_ERR_NONFINITE = -3,   /* a NaN or infinite sample in the series */
    RQA_ERR_DEVICE = -4,      /* a HIP runtime error; the text is in rqa_last_error() */
    RQA_ERR_NOMEM = -5,       /* device scratch could not be allocated */
    RQA_ERR_UNSUPPORTED = -6  /* a flag or shape the kernels do not implement */
} rqa_status;

typedef enum { RQA_NORM_MAX = 0, RQA_NORM_EUCLIDEAN = 1 } rqa_norm;

/* Embedding dimension m >= 1, delay tau >= 1, norm (rqa_norm), Theiler window
 * theiler >= 1 (pairs with j - i < theiler are excluded; 1 gives the paper's
 * j > i), minimal line length lmin in 1..16 (the paper uses 2). */
typedef struct {
    uint32_t m;
    uint32_t tau;
    uint32_t norm;
    uint32_t theiler;
    uint32_t lmin;
} rqa_params;

/* flags.  Every selection method gives the same exact thresholds; they
 * differ in the number of passes over the pairs. */
enum {
    RQA_SEL_AUTO = 0,    /* exact selection, the method picked by the library: RQA_SEL_SAMPLE for calls
                            of at least 2^29 pairs in all (where its set-up pays), else RQA_SEL_PLAIN */
    RQA_SEL_LEARNED = 1, /* exact selection inside a key window the network predicts (two passes);
                            series with a target outside the window fall back to RQA_SEL_PLAIN */
    RQA_FULL_HIST = 2,   /* rqa_det_curve only: also return the full line-length histogram P(l) */
    RQA_SEL_SAMPLE = 4,  /* as RQA_SEL_LEARNED with the window from sketch-sample quantiles (no network) */
    RQA_SEL_WINDOW = 8,  /* as RQA_SEL_LEARNED with the window set by rqa_set_window (for tests) */
    RQA_SEL_PLAIN = 16   /* exact selection by radix passes over all pairs (three; the line sweep
                            takes the third when DET is asked for) */
};

/* Create a context on HIP device `device`.  hip_stream is a hipStream_t on
 * that device to order all work on, or NULL for a stream the context creates
 * and owns.  The context owns its device scratch (grown on demand, freed by
 * rqa_destroy).  *out receives the context on RQA_OK. */
rqa_status rqa_create(rqa_ctx **out, int device, void *hip_stream);

/* Free a context and its scratch.  NULL is ignored. */
void rqa_destroy(rqa_ctx *ctx);

/* Exact thresholds for K target recurrence rates (Averaged RQA section: the
 * RR is preselected and eps follows from it).  Every selection method gives
 * the same exact thresholds; they differ in the number of passes.
 *   series_dev: n float32 samples (device).
 *   rr: K targets in (0, 1] (host), any order, repeats allowed.
 *   flags: one selection method (RQA_SEL_AUTO, RQA_SEL_PLAIN, RQA_SEL_SAMPLE,
 *     RQA_SEL_LEARNED or RQA_SEL_WINDOW).
 *   eps_out[K]: eps_r = the k_r-th smallest key (host).
 *   k_out[K] (or NULL): k_r.   count_out[K] (or NULL): #{key <= eps_r}.
 * Outputs follow the order of rr. */
rqa_status rqa_select_thresholds(rqa_ctx *ctx, const float *series_dev, uint64_t n,
                                 const rqa_params *p, const double *rr, uint32_t K,
                                 uint32_t flags, float *eps_out, uint64_t *k_out,
                                 uint64_t *count_out);

/* Recurrence rate and determinism at K given thresholds in one pass over the
 * pairs (Eq. 3, Eq. 4), and their mean.
 *   eps: K thresholds in key units, each >= 0 or +inf, not NaN (host).
 *   count_out[K]: C_r = #{key <= eps_r};  rr_out[K]: C_r / M;
 *   det_out[K]: DET_r (NaN when C_r = 0);  det_mean_out[1]: mean of det_out.
 * flags: 0, or RQA_FULL_HIST for the diagonal line-length histogram P_r(l)
 * behind Eq. 4 (one more pass, with whole diagonals per workgroup):
 *   hist_out[K * hist_len] (host), row r at hist_out + r * hist_len:
 *     entry l < hist_len - 1 = number of diagonal lines of exactly l
 *     recurrent pairs (maximal runs of j - i = const with key <= eps_r, every
 *     line inside the pairs j - i >= theiler); entry hist_len - 1 also takes
 *     every longer line; entry 0 is 0 (unless hist_len = 1, where it counts
 *     all lines).  So sum_l l P_r(l) = C_r when hist_len exceeds the longest
 *     line, and DET_r = sum_{l >= lmin} l P_r(l) / C_r.
 *   hist_len: 1 .. RQA_MAX_HIST_LEN.  Without the flag hist_out must be NULL
 *     and hist_len 0.
 *   Limits of the full histogram: fewer than 2^24 - 1 embedded vectors,
 *   else RQA_ERR_UNSUPPORTED.  One histogram pass over the pairs takes up to
 *   RQA_MAX_HIST_K thresholds; more run as several passes in the same call. */
rqa_status rqa_det_curve(rqa_ctx *ctx, const float *series_dev, uint64_t n,
                         const rqa_params *p, const float *eps, uint32_t K, uint32_t flags,
                         uint64_t *count_out, double *rr_out, double *det_out,
                         double *det_mean_out, uint64_t *hist_out, uint64_t hist_len);

/* The whole path for one series: exact thresholds for the K targets, then RR,
 * DET and the averaged DET at those thresholds, without a host round trip in
 * between.  Any output pointer except det_mean_out may be NULL. */
rqa_status rqa_run(rqa_ctx *ctx, const float *series_dev, uint64_t n, const rqa_params *p,
                   const double *rr, uint32_t K, uint32_t flags, float *eps_out,
                   uint64_t *k_out, uint64_t *count_out, double *rr_out, double *det_out,
                   double *det_mean_out);

/* S independent series in one launch per phase (the paper's ensemble of
 * independent series, Methodology section).
 *   concat_dev: all series back to back (device); series s is
 *     concat_dev[offsets[s] .. offsets[s+1]-1].
 *   offsets[S+1] (host), p[S] (host), rr[S*K] (host, row s for series s).
 *   eps_out, rr_out, det_out: S*K (host, row s for series s);
 *   det_mean_out: S (host).  count_out (or NULL): S*K.
 * Every series gets exactly the result a single-series rqa_run would give. */
rqa_status rqa_batch(rqa_ctx *ctx, uint32_t S, const float *concat_dev, const uint64_t *offsets,
                     const rqa_params *p, const double *rr, uint32_t K, uint32_t flags,
                     float *eps_out, double *rr_out, double *det_out, double *det_mean_out,
                     uint64_t *count_out);

/* rqa_batch plus the full diagonal line-length histogram P_r(l) at every
 * selected threshold, in the same call: the paper derives DET, the average
 * line length L and the longest line L_max from this one histogram
 * (Technical implementation on a GPU) and proposes averaging those measures
 * over the RR set like DET (Averaged RQA section).
 *   Arguments and outputs as in rqa_batch, plus
 *   hist_out[S * K * hist_len] (host): series s, target r at
 *     hist_out + (s * K + r) * hist_len, rows as rqa_det_curve returns them;
 *   hist_len: 1 .. RQA_MAX_HIST_LEN.
 * The histogram takes ceil(K / RQA_MAX_HIST_K) passes over the pairs after
 * the selection.  Series with 2^24 - 1 or more embedded vectors give
 * RQA_ERR_UNSUPPORTED.  rqa_line_measures turns the rows into L and L_max,
 * rqa_averaged_det (a running mean) into their averaged curves. */
rqa_status rqa_batch_hist(rqa_ctx *ctx, uint32_t S, const float *concat_dev, const uint64_t *offsets,
                          const rqa_params *p, const double *rr, uint32_t K, uint32_t flags,
                          float *eps_out, double *rr_out, double *det_out, double *det_mean_out,
                          uint64_t *count_out, uint64_t *hist_out, uint64_t hist_len);

/* rqa_batch without any allocation, for callers that cannot allocate memory
 * on the device: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Arguments, results and errors as in
 * rqa_batch (results are bit-identical), except:
 *   - flags: RQA_SEL_AUTO, RQA_SEL_PLAIN, RQA_SEL_SAMPLE or RQA_SEL_WINDOW;
 *     RQA_SEL_LEARNED returns RQA_ERR_UNSUPPORTED.
 *   - Device scratch comes from a static area of RQA_STATIC_SCRATCH_BYTES
 *     per GPU, which the GPU holds from the first rqa_create on it until the
 *     process ends.  A call whose scratch would not fit (it grows with S and
 *     K: about 0.7 MB per series at K = 20 with plain selection, 3 MB with
 *     RQA_SEL_SAMPLE) returns RQA_ERR_NOMEM before any work, and
 *     rqa_last_error() gives the bytes needed.
 *   - No device or pinned host memory is allocated; host staging uses the
 *     context's ordinary host memory.
 *   - Every call on one GPU shares that GPU's area and leaves its contents
 *     behind (each call clears what it needs): calls that overlap on one GPU,
 *     from any context or thread, race and must be serialised by the
 *     caller. */
#define RQA_STATIC_SCRATCH_BYTES (64u << 20)
rqa_status rqa_batch_static(rqa_ctx *ctx, uint32_t S, const float *concat_dev, const uint64_t *offsets,
                            const rqa_params *p, const double *rr, uint32_t K, uint32_t flags,
                            float *eps_out, double *rr_out, double *det_out, double *det_mean_out,
                            uint64_t *count_out);

/* Per-phase device times of the last computing call (select, det curve,
 * run, batch, sketch), in milliseconds, measured with HIP events on the
 * context stream when timing is enabled (rqa_set_timing) and summed over
 * all launches of the call.  times_out[0..n_out-1] receives: [0] selection
 * pass 1, [1] pass 2, [2] pass 3, [3] sweep, [4] everything else (checks,
 * sketch, network, scans, preparation), [5] full line-length histogram
 * pass (rqa_det_curve with RQA_FULL_HIST).  Windowed selection books its two
 * passes as passes 1 and 2; a plain fallback adds its three passes to
 * passes 1-3.  Returns the number of entries written. */
int rqa_phase_times(rqa_ctx *ctx, double *times_out, int n_out);

/* Measured VALU issue rate of the context's GPU, the denominator of the
 * library's roofline (its kernels are bound by vector-ALU issue and LDS, not
 * by HBM: the input is O(n) bytes and every count stays in LDS or L2).
 * Every lane of 8 workgroups of 256 threads per CU runs 16 independent
 * dependency chains of one instruction:
 *   kind 0: v_add_f32 (32-bit float add), 1: v_add_u32 (32-bit integer add),
 *   2: v_max_u32 (32-bit integer max), 3: v_add_u32 with one operand in a
 *   scalar register (gfx950 then issues it at the rate of kind 2).
 * A kind outside 0..3 returns RQA_ERR_INVALID_ARG.
 * *lane_ops_per_s receives executed lane-operations per second of the
 * fastest of 8 timed launches (HIP events on the context stream);
 * *ms_out (or NULL) that launch's time.  Uses the context's scratch. */
rqa_status rqa_valu_rate(rqa_ctx *ctx, uint32_t kind, double *lane_ops_per_s, double *ms_out);

/* Enable (1) or disable (0) per-phase HIP-event timing on the context. */
rqa_status rqa_set_timing(rqa_ctx *ctx, int enable);

/* Kernel launch shape overrides for later calls on this context: segment
 * length along a diagonal (a multiple of 64, at most 65536) and tiles per
 * work chunk (at most 4096).  0 selects automatic: the autotuned table of the
 * context where it has the size bucket, otherwise about 16 segments per
 * series (64..1024) and 8 tiles per chunk.  Shapes never change results. */
rqa_status rqa_set_shape(rqa_ctx *ctx, uint32_t segment, uint32_t chunk_tiles);

/* Launch-shape autotuner (batched persistent launch of the workload
 * configurations).  Times the whole path (rqa_run with default flags, so
 * with the selection method such a call takes) on the given series, as the
 * device time of its phases (the fastest of three runs after one untimed
 * run), for candidate segment lengths (powers of two from 64 to 4096) and
 * chunk sizes {2, 8, 32, 128, 512}, and records the fastest in the context's table under the size
 * bucket (log2 of the number of vectors, norm, embedding and line class, K up
 * to 32 or beyond).  segment_out/chunk_tiles_out (or NULL) receive it.
 * Arguments as in rqa_run. */
rqa_status rqa_autotune(rqa_ctx *ctx, const float *series_dev, uint64_t n, const rqa_params *p,
                        const double *rr, uint32_t K, uint32_t *segment_out, uint32_t *chunk_tiles_out);

/* Autotuner for rqa_batch: tunes the segment length of every size bucket
 * present in the batch (on up to 64 of its series), then the chunk size of
 * the whole batch, and records them for later multi-series calls.
 * Arguments as in rqa_batch. */
rqa_status rqa_autotune_batch(rqa_ctx *ctx, uint32_t S, const float *concat_dev, const uint64_t *offsets,
                              const rqa_params *p, const double *rr, uint32_t K, uint32_t *chunk_tiles_out);

/* Distance sketch of S series (the input of the threshold-bracket network;
 * an extension of the paper's method).  For series s, RQA_SKETCH_PAIRS pairs
 * are drawn with the SplitMix64 output function of counter q on stream
 * seed + s (pair index = output mod M, pairs numbered diagonal by diagonal);
 * their keys give the median `scale` (bit pattern, scale_out[s]) and the
 * counts of clamp(((bits - scale) >> 21) + 32, 0, 63) divided by
 * RQA_SKETCH_PAIRS as features 0..63; feature 64 is log2(n)/16 and feature
 * 65 is m/4.  features_out: S*RQA_SKETCH_FEATURES floats (host).  Series as in
 * rqa_batch. */
#define RQA_SKETCH_PAIRS 4096
#define RQA_SKETCH_FEATURES 66
rqa_status rqa_sketch_batch(rqa_ctx *ctx, uint32_t S, const float *concat_dev, const uint64_t *offsets,
                            const rqa_params *p, uint64_t seed, float *features_out, uint32_t *scale_out);

/* The same sketch's sampled keys, sorted: sample_out (host, S *
 * RQA_SKETCH_PAIRS) receives for series s the RQA_SKETCH_PAIRS key bit
 * patterns of its sampled pairs in ascending order (the order statistics the
 * sample window of RQA_SEL_SAMPLE is taken from; its median is scale_out of
 * rqa_sketch_batch).  Arguments and errors as rqa_sketch_batch. */
rqa_status rqa_sketch_sample(rqa_ctx *ctx, uint32_t S, const float *concat_dev, const uint64_t *offsets,
                             const rqa_params *p, uint64_t seed, uint32_t *sample_out);

/* Threshold-bracket network (an extension of the method; the paper has no
 * learned part): a perceptron 66 -> 128 -> 128 -> 20 with exact GELU hidden
 * layers mapping the sketch features to the offsets
 * t_r = (bits(eps_r) - scale) / 2^23 of the exact thresholds of the 20 target
 * rates 0.01, 0.02, ..., 0.20.  It is held by the context; its forward and
 * backward passes and Adam run in the library's own FP32 kernels.
 * Parameter layout (RQA_MLP_PARAMS floats): W1[66][128], b1[128],
 * W2[128][128], b2[128], W3[128][20], b3[20], row-major. */
#define RQA_MLP_INPUTS 66
#define RQA_MLP_OUTPUTS 20
#define RQA_MLP_PARAMS 27668
/* He-uniform weights from the SplitMix64 stream `seed`, zero biases, Adam reset. */
rqa_status rqa_mlp_init(rqa_ctx *ctx, uint64_t seed);
/* Copy parameters in (host, count = RQA_MLP_PARAMS; Adam reset) or out. */
rqa_status rqa_mlp_set_params(rqa_ctx *ctx, const float *params, uint64_t count);
rqa_status rqa_mlp_get_params(rqa_ctx *ctx, float *params, uint64_t count);
/* y_dev[B][20] = network(x_dev[B][66]); both device pointers, B <= 65536. */
rqa_status rqa_mlp_forward(rqa_ctx *ctx, const float *x_dev, uint32_t B, float *y_dev);
/* Gradient of the mean squared error against t_dev[B][20] (device) with
 * respect to the parameters, into grad_out (host, RQA_MLP_PARAMS floats);
 * loss_out (or NULL) receives the loss.  Parameters are unchanged. */
rqa_status rqa_mlp_gradients(rqa_ctx *ctx, const float *x_dev, const float *t_dev, uint32_t B,
                             float *grad_out, double *loss_out);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at learning rate lr on the
 * batch; loss_out (or NULL) receives the loss before the step. */
rqa_status rqa_mlp_train_step(rqa_ctx *ctx, const float *x_dev, const float *t_dev, uint32_t B, float lr,
                              double *loss_out);
/* Half-widths (RQA_MLP_OUTPUTS, offset units) of the bracket around each
 * predicted offset, from calibration on held-out series. */
rqa_status rqa_mlp_set_bracket(rqa_ctx *ctx, const float *delta, uint32_t n);

/* Window of the RQA_SEL_WINDOW method: key values [lo, hi] (>= 0, not NaN). */
rqa_status rqa_set_window(rqa_ctx *ctx, float lo, float hi);
/* Width z of the RQA_SEL_SAMPLE window: sample ranks q P -/+ z sqrt(P q (1-q))
 * around each target rate q (default 5). */
rqa_status rqa_set_sample_width(rqa_ctx *ctx, float z);
/* Statistics of the last selection on this context: full counting passes
 * over all pairs (3 plain, 2 windowed, 5 windowed with fallback), series
 * that fell back to plain selection, targets outside their window.  Any
 * pointer may be NULL. */
rqa_status rqa_selection_stats(rqa_ctx *ctx, uint32_t *full_passes, uint32_t *series_fallback,
                               uint32_t *targets_missed);

/* Save / load the context's autotuned table as JSON (path: host string).
 * Loading replaces the table; a malformed file leaves it unchanged. */
rqa_status rqa_tune_save(rqa_ctx *ctx, const char *path);
rqa_status rqa_tune_load(rqa_ctx *ctx, const char *path);

/* Number of persistent workgroups of every counting launch (selection passes
 * and sweep).  0 (the default) sizes each launch to one full set of resident
 * workgroups, at most one per work chunk.  A nonzero value is used as given,
 * also when it exceeds the number of chunks: the surplus workgroups find the
 * work queue empty and exit.  Applies to later calls on this context. */
rqa_status rqa_set_grid(rqa_ctx *ctx, uint32_t workgroups);

/* The averaged-DET curve over an ordered RR set (averaged-determinism
 * equation of the Averaged RQA section, with RR* running over the set):
 * curve_out[r] = (DET_0 + ... + DET_r) / (r + 1), summed left to right in
 * double, for r = 0..K-1 (curve_out[K-1] equals the mean DET of rqa_run).  A
 * NaN DET (empty plot) makes the rest of the curve NaN.  Host arrays; no
 * device work.  Returns RQA_ERR_INVALID_ARG for NULL pointers or K = 0. */
rqa_status rqa_averaged_det(const double *det, uint32_t K, double *curve_out);

/* Average diagonal line length L and longest diagonal line L_max from line
 * histograms (the histogram section of the GPU implementation derives DET,
 * L and L_max from P(l); L and L_max follow the standard RQA definitions):
 *   L_r = sum_{l >= lmin} l P_r(l) / sum_{l >= lmin} P_r(l), summed in
 *         increasing l in double (NaN without a line of length >= lmin);
 *   L_max_r = the largest l with P_r(l) > 0 (0 without a line).
 * hist: K rows of hist_len entries as rqa_det_curve returns them (host).  A
 * nonzero last entry counts as length hist_len - 1, so both are exact when
 * hist_len exceeds the longest diagonal (nv - theiler + 1 entries or more).
 * L_out[K], lmax_out[K] (host, either may be NULL).  Averaged forms over an
 * RR set: rqa_averaged_det applied to L_out (the same running mean).
 * Returns RQA_ERR_INVALID_ARG for hist NULL, K = 0, hist_len = 0 or
 * lmin = 0.  No device work. */
rqa_status rqa_line_measures(const uint64_t *hist, uint32_t K, uint64_t hist_len, uint32_t lmin,
                             double *L_out, uint64_t *lmax_out);

/* Human-readable name of a status code (static string). */
const char *rqa_status_string(rqa_status s);

/* Detail of the last failure on the calling thread (static thread-local
 * storage, valid until the next call from that thread). */
const char *rqa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RQA_H */
