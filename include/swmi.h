/*
 * swmi -- exact affine-gap Smith-Waterman on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libswmi.so.  Every entry point returns an sw_status; none aborts.
 * On failure a thread-local message is available from sw_last_error().
 *
 * The computation follows SW# (Korpar & Sikic, arXiv 1304.5966), Section 2:
 *   first phase  -- forward local-alignment pass over the whole matrix in
 *                   linear memory, giving the best score and its endpoint;
 *   second phase -- reverse pass from the endpoint with minus-infinity
 *                   borders and no zero floor, giving the start point;
 *   reconstruction -- Myers-Miller divide and conquer between start and end,
 *                   giving the alignment.
 * Affine gaps as in the paper's abstract: a gap of length k costs
 *   gap_open + (k - 1) * gap_extend.
 *
 * Conventions shared by every call:
 *  - Sequences are DNA letters "ACGTacgt" (case-insensitive), or with a
 *    substitution matrix (sw_scoring.matrix) the letters of its alphabet.  Any
 *    other byte makes the call fail with SW_EINVAL and names the offset.
 *  - A indexes rows (the reference), B indexes columns.
 *  - Coordinates are 0-based and inclusive.  When the best score is 0 the
 *    alignment is empty: start = end = -1 and the CIGAR is "".
 *  - Ties: the endpoint is the lexicographically smallest (end_a, end_b)
 *    holding the best score; the start is the lexicographically largest
 *    (start_a, start_b) from which that endpoint is reached with the best
 *    score; the alignment is the canonical Myers-Miller path (midline ties go
 *    to the smallest column, a plain crossing before a gap-spanning one).
 *  - CIGAR: run-length "=" (equal letters), "X" (unequal letters), "I" (consumes B
 *    only), "D" (consumes A only).
 *  - Host input buffers are borrowed read-only for the duration of the call;
 *    result structs are caller-owned (sw_align_result's CIGAR is freed with
 *    sw_align_result_free).
 *  - Device pointers, where taken, must be valid on the context's device and
 *    ordered on the context's stream; the call synchronizes that stream
 *    before returning results to host memory.
 */
#ifndef SWMI_H
#define SWMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SW_OK = 0,
    SW_EINVAL = -1,        /* bad argument: null pointer, bad letter, bad scoring */
    SW_ENOMEM = -2,        /* device or host allocation failed, or workspace too small */
    SW_EDEVICE = -3,       /* a HIP runtime call or kernel failed */
    SW_EUNSUPPORTED = -4,  /* arguments valid but outside what the kernels handle */
    SW_EINTERNAL = -5      /* internal consistency check failed */
} sw_status;

/* Substitution matrix (protein alignment: the library part behind the
 * swsharpp executable that the paper's Section 3 lists beside the nucleotide
 * ones; the paper gives no matrix): s(x, y) for a letter x of A
 * and a letter y of B is scores[i * size + j] where alphabet[i] == x and
 * alphabet[j] == y, letters compared case-insensitively.  The matrix need not
 * be symmetric.  Requirements, else SW_EINVAL: 1 <= size <= 31 distinct
 * letters (bytes 33..126, case-insensitively distinct), every score in
 * -127..127.  Borrowed for the duration of the call. */
typedef struct {
    const char* alphabet;   /* size letters */
    const int8_t* scores;   /* size x size, row = letter of A, column = letter of B */
    int32_t size;
    int32_t reserved;       /* 0 */
} sw_matrix;

/* Scoring (all configurations of the benchmark: 1, 3, 5, 2).
 * Requirements: 0 < match <= 127, 0 <= mismatch <= 127,
 * 0 < gap_extend <= gap_open, gap_open <= 2^20.  Otherwise SW_EINVAL.
 * With a matrix, match and mismatch are ignored and the largest entry plays
 * match's part in the bounds below (at least 1).
 * If match * min(len_a, len_b) >= 2^30 the call returns SW_EUNSUPPORTED
 * (int32 headroom).
 * Matrix scoring runs the same passes as DNA (score, start, alignment, batch,
 * row slabs, two halves, external thresholds); not with a threshold model
 * (SW_PRUNE_LEARNED without a threshold) or SW_FLAG_BOTH_STRANDS
 * (SW_EUNSUPPORTED). */
typedef struct {
    int32_t match;            /* added for equal letters */
    int32_t mismatch;         /* subtracted for unequal letters */
    int32_t gap_open;         /* cost of a gap of length 1 */
    int32_t gap_extend;       /* cost of each further gap position */
    const sw_matrix* matrix;  /* NULL: match / mismatch over ACGT */
} sw_scoring;

typedef enum {
    SW_PRUNE_NONE = 0,     /* every cell is computed */
    SW_PRUNE_BEST = 1,     /* skip tiles that cannot reach the running best (exact; paper Section 2, pruning) */
    SW_PRUNE_LEARNED = 2   /* as BEST, plus a threshold T predicted by the model; exact, with a rerun on a miss */
} sw_prune_mode;

typedef struct sw_model sw_model;

/* Progress of a long score pass: called on the calling thread after each row
 * slab with the rows of A done so far and the total. */
typedef void (*sw_progress_fn)(void* user, int64_t rows_done, int64_t rows_total);

typedef struct {
    int32_t prune_mode;        /* sw_prune_mode */
    int32_t threshold;         /* > 0: use this T instead of the model's prediction (LEARNED mode) */
    const sw_model* model;     /* LEARNED mode: threshold model (sw_model_load) */
    int32_t rows_per_lane;     /* 0 = the context's tuned value (else 8); else 4, 6 or 8 */
    int32_t waves_per_cu;      /* 0 = the context's tuned value (else 8); else 1..16 stripe waves per CU */
    int32_t band_width;        /* 0 = automatic; else columns per band, a positive multiple of 64 */
    int32_t flags;             /* SW_FLAG_* bits */
    /* Row slabs (sw_score, sw_score_dev, sw_align's score pass; paper Section 2,
     * linear memory): the score pass runs as launches over consecutive rows of A,
     * each starting from the previous one's last row of H and F, with the best
     * cell so far carried over; results are identical to one launch.  0 =
     * automatic (one launch up to 1e14 cells, else slabs of at most that);
     * > 0 = rows per slab. */
    int32_t slab_rows;
    sw_progress_fn progress;   /* optional, called after each slab (NULL: none) */
    void* progress_user;
    /* sw_batch / sw_batch_dev in SW_PRUNE_LEARNED mode: one threshold T >= 0 per
     * pair (n_pairs values, host memory, read during the call), used instead of
     * the model's predictions and of `threshold`; NULL: not used. */
    const int32_t* pair_thresholds;
} sw_options;

/* sw_batch_dev: capture the device work of the call in a HIP graph and replay
 * it on later calls with the same pairs (offsets), pointers, workspace size,
 * options, scoring, tuning and learned thresholds; other calls capture anew (the
 * context keeps one graph).  A replay skips the host planning: the graph copies
 * the launch's tables from pinned host memory kept with it, so the workspace
 * may be used for other work between replays.  Capture needs a non-null
 * stream. */
#define SW_FLAG_GRAPH 1

/* sw_score / sw_score_dev: run the score pass as the paper's two halves
 * (Section 2, last paragraphs): the upper half of A's rows forward and the
 * lower half reversed, in one launch, joined at the midline; then, when the
 * best alignment ends below the midline, the lower half forward once more
 * with the best score as threshold to find the endpoint.  Results equal the
 * single pass; sw_score_result.split_case reports the paper's case.  Needs
 * len_a >= 2; not with SW_PRUNE_LEARNED, row slabs or sw_batch
 * (SW_EUNSUPPORTED). */
#define SW_FLAG_HALVES 2

/* sw_score / sw_score_dev / sw_align: align A against both strands of B
 * (paper Section 3, both strands): B as given and its reverse complement
 * (reversed, A<->T, C<->G), both in one launch.  The result is the better
 * strand, the forward one on a tie; its strand field is 1 when it is the
 * reverse complement, and then end_b, start_b and the CIGAR refer to the
 * reverse complement of B (position p there is B's position len_b - 1 - p).
 * Not with SW_PRUNE_LEARNED, SW_FLAG_HALVES or sw_batch (SW_EUNSUPPORTED). */
#define SW_FLAG_BOTH_STRANDS 4

/* Where the two-halves pass found the maximum (paper Section 2, cases a-c). */
typedef enum {
    SW_SPLIT_NONE = 0,    /* single pass, or score 0 */
    SW_SPLIT_LOWER = 1,   /* (a) inside the lower half */
    SW_SPLIT_UPPER = 2,   /* (b) inside the upper half (the first cell holding it is there) */
    SW_SPLIT_MIDDLE = 3   /* (c) at the midpoint: the best alignment crosses the midline */
} sw_split_case;

typedef struct {
    int32_t score;             /* best local score S >= 0 */
    int32_t threshold;         /* pruning threshold T that was used (0 if none) */
    int64_t end_a;             /* endpoint row (A index), -1 if S == 0 */
    int64_t end_b;             /* endpoint column (B index), -1 if S == 0 */
    int64_t cells_computed;    /* DP cells evaluated by the score pass (pruned tiles excluded) */
    int32_t fallback;          /* 1 if T exceeded the found maximum and the plain pass was rerun */
    int32_t split_case;        /* sw_split_case (SW_FLAG_HALVES), else SW_SPLIT_NONE */
    int32_t strand;            /* 0: B as given; 1: its reverse complement (SW_FLAG_BOTH_STRANDS) */
    int32_t reserved;
} sw_score_result;

typedef struct {
    int32_t score;
    int32_t strand;            /* 0: B as given; 1: its reverse complement (SW_FLAG_BOTH_STRANDS) */
    int64_t start_a, start_b;  /* first aligned pair, -1 if score == 0 */
    int64_t end_a, end_b;      /* last aligned pair, -1 if score == 0 */
    char* cigar;               /* NUL-terminated, owned by the library: sw_align_result_free */
    int64_t cigar_len;
} sw_align_result;

typedef struct sw_context sw_context;

/* Last error message of the calling thread ("" if none).  Valid until the next call. */
const char* sw_last_error(void);

/* Library version string. */
const char* sw_version(void);

/* Creates a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  A context caches device
 * workspace and tuning; it is not thread-safe: use one per stream. */
sw_status sw_context_create(int device, void* hip_stream, sw_context** out);
sw_status sw_context_destroy(sw_context* ctx);

/* Caps the device memory the context's host-pointer calls (sw_score, sw_align,
 * sw_start, sw_batch) hold for inputs and workspace: a call that would need
 * more fails with SW_ENOMEM before any device work.  0 (the default) = no
 * limit.  Lowering the limit below what is held releases the held buffers
 * (after the context's stream is idle).  The _dev calls use the caller's
 * workspace and are not counted. */
sw_status sw_context_set_max_workspace(sw_context* ctx, size_t bytes);

/* Engine shape per workload class, set by a tuner that timed the candidates
 * on the device.  Calls whose options leave rows_per_lane / waves_per_cu at 0
 * take the class's tuned value (8 / 8 when untuned).  The class of a launch
 * follows its mean cell count per DP problem: HUGE from 1e12, LARGE from
 * 1e10, below that BATCH when the launch holds more than one problem and
 * SMALL when it holds one.  Workspace sizes depend on
 * the shape: query them after changing the tuning.
 * rows_per_lane: 0 (untuned), 4, 6 or 8; waves_per_cu: 0 (untuned) or 1..16. */
typedef enum {
    SW_TUNE_PAIR_SMALL = 0,
    SW_TUNE_PAIR_LARGE = 1,
    SW_TUNE_PAIR_HUGE = 2,
    SW_TUNE_BATCH = 3
} sw_tune_class;

sw_status sw_context_set_tuning(sw_context* ctx, int32_t tune_class, int32_t rows_per_lane,
                                int32_t waves_per_cu);
sw_status sw_context_get_tuning(const sw_context* ctx, int32_t tune_class, int32_t* rows_per_lane,
                                int32_t* waves_per_cu);

/* Column band width of the class's local passes (score pass, batches), set by
 * the tuner; calls whose options leave band_width at 0 take it.  0 = automatic:
 * the widest band whose stripe hand-off slots fit 32 GiB.  A positive multiple
 * of 64, else SW_EINVAL.  The banded global passes (start, reconstruction) size
 * their bands from the alignment and ignore it. */
sw_status sw_context_set_band_width(sw_context* ctx, int32_t tune_class, int32_t band_width);
sw_status sw_context_get_band_width(const sw_context* ctx, int32_t tune_class, int32_t* band_width);

/* First phase (paper Section 2): best local score and its endpoint.
 * a[0..len_a), b[0..len_b): host letters.  out: caller-owned. */
sw_status sw_score(sw_context* ctx, const char* a, int64_t len_a, const char* b, int64_t len_b,
                   const sw_scoring* scoring, const sw_options* options, sw_score_result* out);

/* Same as sw_score on device-resident letters (d_a, d_b on the context's
 * device).  The workspace (device, at least sw_score_workspace_size bytes,
 * owned by the caller) holds every intermediate; nothing else is allocated. */
size_t sw_score_workspace_size(sw_context* ctx, int64_t len_a, int64_t len_b, const sw_options* options);
sw_status sw_score_dev(sw_context* ctx, const uint8_t* d_a, int64_t len_a, const uint8_t* d_b,
                       int64_t len_b, const sw_scoring* scoring, const sw_options* options,
                       void* d_workspace, size_t workspace_bytes, sw_score_result* out);

/* sw_score_dev without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Every intermediate lives in a fixed
 * scratch array of SW_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device it runs on until the process ends; the call allocates nothing.  A
 * pair whose workspace (sw_score_workspace_size with the same options)
 * exceeds the scratch fails with SW_ENOMEM before any device work.  All calls
 * on one device share that device's scratch and clear what they read before
 * writing it: calls that overlap in time on one device (two streams, two
 * threads) race and must not be issued. */
#define SW_NOALLOC_SCRATCH_BYTES (256ull << 20)
sw_status sw_score_dev_noalloc(sw_context* ctx, const uint8_t* d_a, int64_t len_a, const uint8_t* d_b,
                               int64_t len_b, const sw_scoring* scoring, const sw_options* options,
                               sw_score_result* out);

/* All three phases (paper Section 2): score, start, end and the canonical
 * CIGAR.  out->cigar is allocated by the library; release it with
 * sw_align_result_free. */
sw_status sw_align(sw_context* ctx, const char* a, int64_t len_a, const char* b, int64_t len_b,
                   const sw_scoring* scoring, const sw_options* options, sw_align_result* out);
void sw_align_result_free(sw_align_result* r);

/* Second phase alone (paper Section 2): the start point of the best alignment
 * that ends at (end_a, end_b) with score `score` (as returned by sw_score). */
sw_status sw_start(sw_context* ctx, const char* a, int64_t len_a, const char* b, int64_t len_b,
                   const sw_scoring* scoring, int32_t score, int64_t end_a, int64_t end_b,
                   int64_t* start_a, int64_t* start_b);

/* Many independent pairs in one persistent launch.  Pair p is
 * seqs_a[offs_a[p] .. offs_a[p+1]) against seqs_b[offs_b[p] .. offs_b[p+1])
 * (host letters, offs_* of length n_pairs + 1, non-decreasing).
 * out[0 .. n_pairs) receives score and endpoint per pair. */
sw_status sw_batch(sw_context* ctx, const char* seqs_a, const int64_t* offs_a, const char* seqs_b,
                   const int64_t* offs_b, int32_t n_pairs, const sw_scoring* scoring,
                   const sw_options* options, sw_score_result* out);

/* The reconstruction's host part (paper Section 2: small sub-matrices are
 * aligned on the CPU): canonical Myers-Miller alignment of the whole of
 * a x b (host letters) as a global alignment whose leading / trailing deletion
 * runs open at tb / te (-1 = gap_open - gap_extend; 0 = continuing a run), gap
 * cost g + h*k otherwise.  If score_known, `score` must be the optimal global
 * score; it restricts the work to the diagonals that score can reach.  Writes
 * a NUL-terminated CIGAR of at most cap bytes.  Host only, no device use. */
sw_status sw_mm_host(const char* a, int64_t len_a, const char* b, int64_t len_b, const sw_scoring* scoring,
                     int32_t tb, int32_t te, int32_t score_known, int64_t score, char* cigar, int64_t cap,
                     int64_t* cigar_len);

/* sw_batch on device-resident letters: d_seqs_a / d_seqs_b hold the packed
 * letters on the context's device, indexed by the host offset arrays offs_a /
 * offs_b exactly as in sw_batch.  The device workspace (caller-owned, at least
 * sw_batch_workspace_size bytes) holds every intermediate.
 * Workspace sizes include the stripe hand-off slots: one per resident wave,
 * plus up to SWMI_SLOT_ROOM_BYTES more (environment variable, bytes; default
 * 8 GiB; 0 keeps the minimal ring) where slots are small, so that a batch of
 * many short pairs rarely waits for a slot to be free. */
size_t sw_batch_workspace_size(sw_context* ctx, const int64_t* offs_a, const int64_t* offs_b, int32_t n_pairs,
                               const sw_scoring* scoring, const sw_options* options);
sw_status sw_batch_dev(sw_context* ctx, const uint8_t* d_seqs_a, const int64_t* offs_a, const uint8_t* d_seqs_b,
                       const int64_t* offs_b, int32_t n_pairs, const sw_scoring* scoring,
                       const sw_options* options, void* d_workspace, size_t workspace_bytes,
                       sw_score_result* out);

/* ---- Learned pruning threshold (not in the paper; see the pruning rule of
 * Section 2, which it feeds).  A 256-128-128-1 ReLU network with BF16
 * weights and inputs and FP32 accumulation predicts y = ln(1 + S) from pair
 * features; the threshold is T = floor(0.9 * (exp(y) - 1)), or none (T = 0)
 * when T < 0.01 |A||B| / (|A| + |B|): such a threshold could skip under 2 % of
 * the cells.  A pass that finds a best below T (a miss) reports the largest H
 * it computed, S' <= S, and reruns with threshold S' (exact; it cannot miss);
 * sw_score_result.fallback flags the rerun and cells_computed counts both
 * passes.  Parameters are one
 * FP32 vector of sw_mlp_param_count() values: W1[256][128], b1[128],
 * W2[128][128], b2[128], W3[128], b3 (row-major, input index first); the BF16
 * copy (d_wbf) holds the same values rounded to nearest even.  All _dev calls
 * take device pointers, run on the context's stream and allocate nothing. */

/* Model file: "SWMLP001", int32 256, int32 128, float mean[256],
 * float inv_std[256], float params[sw_mlp_param_count()].  sw_options.model. */
sw_status sw_model_load(sw_context* ctx, const char* path, sw_model** out);
sw_status sw_model_free(sw_model* model);
int64_t sw_mlp_param_count(void);

/* Features of pair p (letters d_seqs_a[offs_a[p]..offs_a[p+1]) and likewise b;
 * offsets on the host) into d_out[p*256 .. p*256+256): [0,128) the
 * complement-folded shared 4-mer spectrum, [128,254) ln(1 + number of
 * 64-diagonal bands whose 12-mer hit count falls in each of 126 log bins),
 * [254,256) ln|A| / ln 4e6 and ln|B| / ln 4e6. */
size_t sw_features_workspace_size(sw_context* ctx, const int64_t* offs_a, const int64_t* offs_b, int32_t n_pairs);
sw_status sw_features_dev(sw_context* ctx, const uint8_t* d_seqs_a, const int64_t* offs_a, const uint8_t* d_seqs_b,
                          const int64_t* offs_b, int32_t n_pairs, float* d_out, void* d_workspace,
                          size_t workspace_bytes);
/* d_x[n][256] (BF16) = round((d_feat - mean) * inv_std). */
sw_status sw_mlp_standardize_dev(sw_context* ctx, const float* d_feat, int32_t n, const float* d_mean,
                                 const float* d_inv_std, uint16_t* d_x);
/* Forward pass: h1, h2 [n][128] (post-ReLU, BF16-rounded, stored as float), y [n]. */
sw_status sw_mlp_forward_dev(sw_context* ctx, const uint16_t* d_x, int32_t n, const uint16_t* d_wbf,
                             const float* d_params, float* d_h1, float* d_h2, float* d_y);
/* Gradient over the n samples into d_grad (same layout as the parameters):
 * quantile <= 0: of mean((y - target)^2); 0 < quantile < 1: of the mean
 * pinball loss mean(max(q (target - y), (q - 1) (target - y))), whose
 * minimiser is the q-quantile of the target (subgradient 0 at y == target);
 * quantile >= 1: SW_EINVAL.  d_scratch holds 64 + 257 * n floats.  Fixed
 * summation order. */
sw_status sw_mlp_backward_dev(sw_context* ctx, const uint16_t* d_x, int32_t n, const uint16_t* d_wbf,
                              const float* d_h1, const float* d_h2, const float* d_y, const float* d_target,
                              float quantile, float* d_scratch, float* d_grad);
/* One Adam step (bias-corrected, step >= 1) on the FP32 parameters; refreshes d_wbf. */
sw_status sw_mlp_adam_dev(sw_context* ctx, float* d_params, float* d_m, float* d_v, const float* d_grad,
                          int32_t step, float lr, float beta1, float beta2, float eps, uint16_t* d_wbf);

#ifdef __cplusplus
}
#endif

#endif /* SWMI_H */
