/*
 * fif.h -- C ABI of the MI355X (gfx950) Fast Iterative Filtering library.
 *
 * The library decomposes real signals into intrinsic mode functions (IMFs)
 * with the direct (FFT) form of Discrete Iterative Filtering of Cicone & Zhou,
 * "Numerical Analysis for Iterative Filtering with New Efficient
 * Implementations Based on FFT":
 *
 *   - Algorithm 2 (DIF), outer loop: while the residual r has at least two
 *     extrema, fix the filter length from the extrema count, extract one IMF,
 *     subtract it; the last residual is returned as the remainder;
 *   - Theorem 5 and the one-step formula of Section 4: with periodic
 *     extension the window matrix W is circulant, so the IMF after m inner
 *     steps is IDFT((1 - lambda)^m DFT(r)), lambda being the DFT of W's first
 *     column (equation "Lambdas");
 *   - Section 4, the scan over the step count: m is the smallest count whose
 *     stop quantity SD = ||s_{m+1} - s_m|| / ||s_m|| (equation "SD") is
 *     <= delta, here evaluated from the spectrum by Parseval's identity (the
 *     identity used in the proof of Theorem 2).
 *
 * Conventions shared by every entry point:
 *   - Readings: the window is the triangle of equation "triangular" (half
 *     support L, sampled at integer offsets, taps summing to 1) convolved
 *     with itself; L = ceil(2N/k) (mask_rule 0) or 2*floor(nu*N/k) (mask_rule
 *     1, equation "Unif_Mask_length"); k counts sign changes of the nonzero
 *     forward differences r_{i+1} - r_i (i = 0..N-2); the outer loop also
 *     stops when max|r - mean(r)| <= floor_tau * max|s| (rounding floor) and
 *     after max_imfs IMFs; m is capped at max_inner (flag FIF_IMF_CAP).
 *   - Signal lengths: N >= 2 whose prime factors are all <= 7; lengths above
 *     8192 must split as N1*N2 with N1, N2 <= 4096 (so N <= 2^24).
 *     Otherwise FIF_ERR_UNSUPPORTED_LENGTH and nothing is launched.
 *   - Buffers: every array argument except `lengths` of fif_plan_create is a
 *     caller-owned DEVICE pointer (HBM of the current HIP device).  The
 *     library never frees or retains them.  Packed batches put signal b at
 *     element offset off_b = sum_{c<b} N_c; its IMFs occupy
 *     imfs[max_imfs*off_b .. max_imfs*off_b + max_imfs*N_b), row j = IMF j.
 *     IMF rows at and after n_imfs[b] are zero.
 *   - Precision: the residual spectrum, lambda, (1-lambda)^m, the stop-test
 *     sums and the residual whose extrema are counted are FP64; the FP32
 *     entry points read FP32 signals (widened exactly) and round IMFs and
 *     remainders to FP32 on store.  The _f64 entry points store FP64.
 *   - Asynchrony: fif_decompose_batched* enqueue work on `stream` and return;
 *     outputs are valid once the caller synchronises that stream.
 *     fif_decompose* (single signal) synchronise the stream before return.
 *   - Errors: argument problems are detected on the host before any launch
 *     and returned as a negative fif_status; fif_last_error() then returns a
 *     thread-local message.  Per-signal problems (non-finite samples) are
 *     reported in sig_status[b] and do not stop the other signals.
 *   - Determinism: results are bitwise reproducible and do not depend on the
 *     batch a signal is decomposed in.
 */
#ifndef FIF_H
#define FIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FIF_OK = 0,
    FIF_ERR_INVALID_ARG = -1,
    FIF_ERR_UNSUPPORTED_LENGTH = -2,
    FIF_ERR_NOMEM = -3,
    FIF_ERR_DEVICE = -4,
    FIF_ERR_NONFINITE = -5,  /* only ever stored in sig_status[] */
    FIF_ERR_CAPACITY = -6,
    FIF_ERR_NOT_FOUND = -7   /* tune-cache lookup without an entry */
} fif_status;

typedef enum {
    /* eq. "triangular" triangle of half-support L, convolved with itself */
    FIF_WINDOW_TRI2 = 0,
    /* the sampled shape given in fif_options.window (see there) */
    FIF_WINDOW_SAMPLED = 1
} fif_window;

/* per-IMF flags */
#define FIF_IMF_CAP 1u          /* inner count stopped at max_inner, SD > delta */
#define FIF_IMF_REFINED 2u      /* FP64 verification moved the FP32 estimate of m */
#define FIF_IMF_UNRESOLVED 4u   /* the multi-workgroup search ran out of rounds; m is
                                   the smallest FP64-verified count found (not expected) */

/* why a signal's outer loop ended (fif_signal_info.stop_reason) */
#define FIF_STOP_MAX_IMFS 0
#define FIF_STOP_FLOOR 1
#define FIF_STOP_FEW_EXTREMA 2
#define FIF_STOP_FAILED 3

typedef struct {
    int32_t mask_rule;   /* 0: L = ceil(2N/k)  1: L = 2*floor(nu*N/k) (equation
                            "Unif_Mask_length")  2: L = ceil(N/f), f the highest
                            bin 1 <= f <= N/2 whose power is >= peak_rho times
                            the strongest of those bins (the spectral-peak rule
                            of Section 2) */
    int32_t stop_mode;   /* 0: smallest m with SD_m <= delta (equation "SD");
                               SD counts the bins with |R_j|^2 >= 1e-26 times
                               the strongest non-constant bin's (the rest is
                               rounding-level content) and is summed relative
                               to its largest weight, so a residual whose
                               counted bins all have lambda > delta (a pure
                               tone, for one) runs to max_inner (FIF_IMF_CAP)
                            1: smallest m >= 1 with ||s_{m+1} - s_m||_2 < delta
                               (equation "Discrete_Abs_StopCond"), IMF = s_m
                            2: m = N0, the smallest N0 >= 1 satisfying
                               inequality "N0_discrete" of Theorem 5 (no search);
                               mode 1 searches no count above that N0 */
    double nu;           /* mask_rule 1 constant, default 1.6 */
    int64_t max_inner;   /* cap on m, default 1000000 */
    double floor_tau;    /* rounding floor, default 1e-9 */
    double gamma;        /* > 0: thresholded IMF (equation
                            "IMF_cont_stop_threshold"): bins with
                            (1 - lambda)^m >= 1 - gamma go whole into the IMF;
                            0 (default): off; must be < 1 */
    double peak_rho;     /* mask_rule 2 fraction, in (0, 1], default 0.1 */
    const double* window;/* HOST array of window_points >= 2 samples of a window
                            shape on [0, 1] (x_i = i / (window_points - 1)), or
                            NULL (default): the triangle of equation "triangular" with the
                            closed-form eigenvalues of equation "eig2".  Section 4
                            needs only W's eigenvalues, the DFT of its first
                            column (equation "Lambdas"), so any shape can be
                            tabulated: h_q = the samples linearly interpolated at
                            x = |q|/L, |q| <= L-1; the window is h convolved with
                            itself over (sum h)^2, folded modulo N; each outer
                            step then computes lambda_j = (DFT(h)_j / sum h)^2
                            for every active signal (one extra FP64 transform
                            per step).  Samples must be finite and >= 0, the
                            first > 0; at most 65537 of them; copied at plan
                            creation.  Not with stop_mode 2 (its N0 counts the
                            triangle's zero eigenvalues).  Shape {1, 0} is the
                            triangle itself. */
    int32_t window_points;
    int32_t precision;   /* FIF_PREC_MIXED (default): transforms and stored
                            spectra in FP64, the residual whose extrema are
                            counted FP64 -- the form whose decisions match the
                            FP64 oracle.  FIF_PREC_FP32: transforms, stored
                            spectra and the four-step intermediate in FP32
                            (half the traffic); lambda, (1 - lambda)^m and the
                            stop-test sums stay FP64.  No parity claim: the
                            FP32 residual's rounding can add or remove extrema
                            and so change k, L, m or the IMF count.  Not with
                            a window shape or a proposal network. */
} fif_options;

/* fif_options.precision */
#define FIF_PREC_MIXED 0
#define FIF_PREC_FP32 1

typedef struct {
    int64_t k;           /* extrema count of the residual the IMF came from */
    int64_t L;           /* half-support of the triangle */
    int64_t m;           /* inner step count */
    double sd;           /* SD_m (FP64, Parseval); stop modes 1 and 2:
                            ||s_{m+1} - s_m||_2 */
    double sd_prev;      /* SD_{m-1}, +inf when m == 1; stop modes 1 and 2:
                            ||s_m - s_{m-1}||_2 */
    uint32_t flags;      /* FIF_IMF_* */
    uint32_t evals;      /* low 16 bits: FP32 passes over the spectrum in the
                            search for m; high 16 bits: FP64 evaluations */
} fif_imf_info;

typedef struct fif_plan fif_plan;

/* Fill *opt with the defaults listed above. */
void fif_options_default(fif_options* opt);

/* Message of the last failing call on this host thread ("" if none). */
const char* fif_last_error(void);
const char* fif_status_string(fif_status s);

/*
 * Create a plan for a batch of B signals with the given lengths (HOST array
 * of B int64) and at most max_imfs IMFs each.  The plan owns device tables
 * (twiddles, sine tables, work lists) allocated on the current device; it
 * does not depend on delta.  opt may be NULL (defaults).
 */
fif_status fif_plan_create(fif_plan** plan, const int64_t* lengths, int32_t B, int32_t max_imfs,
                           const fif_options* opt);
/*
 * How one signal length is transformed: one LDS pass (N <= 8192: N1 = 1,
 * N2 = N, TC = TR = 1), or the four-step split N = N1 * N2 whose pass 1
 * transforms TC columns of length N2 per workgroup and pass 2 TR rows of
 * length N1 (TC * N2 and TR * N1 at most 4096 elements; 8192 where a
 * factor exceeds 2048, so that a tile still holds two columns or rows),
 * each length-n transform a sequence of radix passes (2, 3, 4, 5, 7 or 8,
 * first pass first).  The FFT is what Section 4 makes the cost of each IMF; which
 * split, tiles and radix order run fastest is a property of the device.
 */
typedef struct {
    int64_t N;
    int32_t N1, N2;        /* four-step split (N1 = 1 for one LDS pass) */
    int32_t TC, TR;        /* columns per pass-1 tile, rows per pass-2 tile */
    int32_t n_rad1, n_rad2;
    int8_t rad1[24];       /* radices of the length-N2 transforms */
    int8_t rad2[24];       /* radices of the length-N1 transforms (none: n_rad2 = 0) */
    double us;             /* tuned plans: measured time of this choice (us), else 0 */
    double us_default;     /* tuned plans: measured time of the built-in choice, else 0 */
} fif_length_plan;

/*
 * fif_plan_create with plans picked by measurement.  For every distinct
 * length above 8192 the library times candidate choices -- the three most
 * balanced splits N1 * N2 (and the most balanced one with both factors even,
 * which mirror-paired pass-1 tiles need), the widest pass-1 and pass-2 tiles
 * and half of each (and the widest even pass-1 tile), the built-in radix
 * order and its reverse; the built-in choice is one of them -- by decomposing a synthetic batch of that length (two IMFs)
 * with each, and keeps the fastest.  Results are cached in the text file
 * tune_cache (NULL: the file named by the environment variable
 * FIF_TUNE_CACHE; NULL and unset: no cache) under a key made of the
 * device's architecture name and the HIP runtime version (and "/fp32" for
 * the FP32 lane, whose choices are kept apart); cached lengths are
 * not timed again.  Shorter lengths take the built-in choice.  Tuning
 * allocates and runs kernels on the current device and synchronises it.
 */
fif_status fif_plan_create_tuned(fif_plan** plan, const int64_t* lengths, int32_t B, int32_t max_imfs,
                                 const fif_options* opt, const char* tune_cache);
/* The choice the plan uses for length N (FIF_ERR_NOT_FOUND if the plan has
   no signal of that length). */
fif_status fif_plan_length_plan(const fif_plan* plan, int64_t N, fif_length_plan* out);
/* Host-only access to a tune cache file: the last valid entry for
   (device_key, N), or FIF_ERR_NOT_FOUND; and storing one (entries of
   other keys or lengths are kept, lines that are not valid entries are
   dropped; FIF_ERR_INVALID_ARG for an invalid choice or an unwritable
   file).  fif_device_tune_key writes the current device's key (at most
   `cap` bytes with the terminating zero). */
fif_status fif_tune_cache_lookup(const char* path, const char* device_key, int64_t N, fif_length_plan* out);
fif_status fif_tune_cache_store(const char* path, const char* device_key, const fif_length_plan* choice);
fif_status fif_device_tune_key(char* key, int32_t cap);

/* Bytes of device workspace fif_decompose_batched needs for this plan. */
fif_status fif_plan_workspace_size(const fif_plan* plan, size_t* bytes);
fif_status fif_plan_destroy(fif_plan* plan);

/*
 * Decompose the packed batch described by the plan (Algorithm 2 with the
 * one-step formula per IMF).  signals: FP32 [sum N_b]; imfs: FP32
 * [max_imfs * sum N_b]; remainders: FP32 [sum N_b]; n_imfs: int32 [B];
 * info: fif_imf_info [B * max_imfs] (row-major by signal), may be NULL;
 * sig_status: int32 [B] (FIF_OK or FIF_ERR_NONFINITE), may be NULL;
 * workspace: >= fif_plan_workspace_size bytes, 256-byte aligned.
 * delta > 0.  Enqueued on `stream` (a hipStream_t, NULL = null stream).
 */
fif_status fif_decompose_batched(fif_plan* plan, const float* signals, double delta,
                                 float* imfs, float* remainders, int32_t* n_imfs,
                                 fif_imf_info* info, int32_t* sig_status,
                                 void* workspace, void* stream);
/* Same with FP64 signals, IMFs and remainders. */
fif_status fif_decompose_batched_f64(fif_plan* plan, const double* signals, double delta,
                                     double* imfs, double* remainders, int32_t* n_imfs,
                                     fif_imf_info* info, int32_t* sig_status,
                                     void* workspace, void* stream);

/*
 * fif_decompose_batched replayed from a HIP graph: the first call captures
 * every launch of the batched decomposition on `stream` (which must not be
 * the null stream) into a graph and instantiates it; later calls with the
 * same arguments, the same proposal model and the same feature buffer
 * launch that graph with one hipGraphLaunch.  Different arguments replace
 * the cached graph.  Results equal fif_decompose_batched's.  Not available
 * while profiling is enabled.
 */
fif_status fif_decompose_batched_graph(fif_plan* plan, const float* signals, double delta,
                                       float* imfs, float* remainders, int32_t* n_imfs,
                                       fif_imf_info* info, int32_t* sig_status,
                                       void* workspace, void* stream);
/* Same with FP64 signals, IMFs and remainders (its own cached graph: a call
   of the other precision replaces it). */
fif_status fif_decompose_batched_graph_f64(fif_plan* plan, const double* signals, double delta,
                                           double* imfs, double* remainders, int32_t* n_imfs,
                                           fif_imf_info* info, int32_t* sig_status,
                                           void* workspace, void* stream);

/*
 * fif_decompose_batched without a workspace argument and without any
 * allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it).  The
 * workspace is a fixed array of FIF_STATIC_WORKSPACE_BYTES inside the
 * library, one copy per device, held from the library's load until the
 * process ends.  The call allocates nothing, creates no stream or event,
 * and issues every kernel on `stream` (the signal groups of the batched
 * call run one after another there).  Plans whose workspace
 * (fif_plan_workspace_size) exceeds FIF_STATIC_WORKSPACE_BYTES are
 * refused with FIF_ERR_CAPACITY; a plan with profiling enabled is refused
 * with FIF_ERR_INVALID_ARG.  Every call on one device shares that device's
 * array: calls that overlap in time on one device (two streams, two host
 * threads) race and give wrong results.  Each call writes every workspace
 * word before reading it, so nothing has to be cleared between calls.
 * Results equal fif_decompose_batched's.
 */
#define FIF_STATIC_WORKSPACE_BYTES (64u << 20)
fif_status fif_decompose_batched_static(fif_plan* plan, const float* signals, double delta,
                                        float* imfs, float* remainders, int32_t* n_imfs,
                                        fif_imf_info* info, int32_t* sig_status, void* stream);

/*
 * Plain single-signal form: one signal of length N, one IMF per host
 * iteration, the host reads the signal's state after every outer step and
 * stops launching once it has finished.  The library allocates and caches
 * its own plan and workspace for N on the current device.  Device pointers:
 * signal [N], imfs [max_imfs*N], remainder [N], n_imfs [1], info
 * [max_imfs] (may be NULL).  Returns FIF_ERR_NONFINITE if the signal holds
 * NaN or Inf (imfs zero, remainder = signal).  Synchronises `stream`.
 */
fif_status fif_decompose(const float* signal, int64_t N, fif_window window, double delta,
                         int32_t max_imfs, float* imfs, float* remainder, int32_t* n_imfs,
                         fif_imf_info* info, const fif_options* opt, void* stream);
fif_status fif_decompose_f64(const double* signal, int64_t N, fif_window window, double delta,
                             int32_t max_imfs, double* imfs, double* remainder, int32_t* n_imfs,
                             fif_imf_info* info, const fif_options* opt, void* stream);

/* Release the cached single-signal plans and workspaces of this process. */
void fif_release_cache(void);

/*
 * Kernel timing.  While enabled, every later fif_decompose_batched* call on
 * this plan brackets each kernel launch with a pair of HIP events recorded
 * on the call's stream.  fif_plan_profile_read waits for those events,
 * accumulates elapsed time per kernel kind since the last read into out
 * (HOST array of cap entries, one per kind seen, in first-launch order),
 * stores the number of kinds in *n and forgets the events.  Enabling adds
 * two event records per launch and nothing else.
 */
typedef struct {
    char name[40];       /* kernel kind, e.g. "pass1_step" */
    int64_t launches;
    double total_ms;
} fif_kernel_time;

fif_status fif_plan_profile(fif_plan* plan, int32_t enable);
fif_status fif_plan_profile_read(fif_plan* plan, fif_kernel_time* out, int32_t cap, int32_t* n);

/*
 * Learned proposal of the inner step count (an addition to the paper's
 * method).  A small network reads, for every outer step, the residual's
 * power spectrum in 1024 contiguous bin groups and the mask length L, and
 * proposes m; the Section 4 scan then starts from the proposal instead of
 * its fixed geometric probes and still accepts only the count whose FP64
 * stop test (equation "SD") gives SD_m <= delta < SD_{m-1}.  Decompositions
 * with and without a proposal are therefore the same.
 *
 * Network: input rows [1024 positions][8 channels] of bfloat16 (channel 0:
 * log2(mean group power / total power + 2^-60)/16 over groups of bins
 * 1..N/2, channel 1: log2(L)/16, channels 2..7: 0); six convolutions of
 * kernel 7, stride 2, zero padding 3, 64 channels and ReLU; mean over the
 * last 16 positions; linear 64 -> 2 giving (log2(m)/16, log2(L)/16).  The
 * FP32 parameter array (FIF_NET_PARAMS floats) holds, per layer l = 0..5,
 * W_l[7][C_in][64] then bias_l[64] (C_in = 8 for l = 0, 64 after), then
 * Wh[2][64], bh[2].  Convolutions run on bfloat16 operands with FP32
 * accumulation; activations and backpropagated gradients are stored in
 * bfloat16; the head, the loss and the Adam update are FP32.  Training loss:
 * sum (y - target)^2 / (2 B).
 *
 * A model owns its device memory (parameters, Adam moments, activation and
 * gradient buffers for up to max_batch rows), allocated on the current
 * device by fif_model_create/fif_model_load.  Calls that take a stream are
 * asynchronous; one model must not be used by two streams at once.
 */
#define FIF_NET_FEATURES 1024
#define FIF_NET_CHANNELS 8
#define FIF_NET_PARAMS 147458

typedef struct fif_model fif_model;

/* params: HOST [FIF_NET_PARAMS] (NULL: all zero).  max_batch >= 1. */
fif_status fif_model_create(fif_model** model, const float* params, int32_t max_batch);
fif_status fif_model_free(fif_model* model);
/* Copy the FP32 parameters to / from HOST memory (set also clears the Adam
   state).  Synchronous. */
fif_status fif_model_get_params(const fif_model* model, float* params);
fif_status fif_model_set_params(fif_model* model, const float* params);
/* File: 8-byte magic "FIFNET01", int32 parameter count, int32 zero, then
   the FP32 parameters (little endian). */
fif_status fif_model_save(const fif_model* model, const char* path);
fif_status fif_model_load(fif_model** model, const char* path, int32_t max_batch);
/* feats: DEVICE bfloat16 bits [B][1024][8]; out: DEVICE FP32 [B][2];
   1 <= B <= max_batch. */
fif_status fif_model_forward(fif_model* model, const uint16_t* feats, int32_t B, float* out, void* stream);
/* Loss and gradient without an update.  targets: DEVICE FP32 [B][2];
   grad: DEVICE FP32 [FIF_NET_PARAMS] or NULL; loss: DEVICE FP32 [1] or NULL. */
fif_status fif_model_grad(fif_model* model, const uint16_t* feats, const float* targets, int32_t B,
                          float* grad, float* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias corrected) on the
   gradient of one batch; loss (DEVICE FP32 [1]) may be NULL. */
fif_status fif_model_train_step(fif_model* model, const uint16_t* feats, const float* targets, int32_t B,
                                float lr, float* loss, void* stream);

/* Use `model` (NULL: none) to propose m in every later decomposition with
   this plan.  The model must live on the plan's device and outlive its use. */
fif_status fif_plan_set_proposal(fif_plan* plan, fif_model* model);
/* Record the network input rows of every outer step of later
   decompositions with this plan: DEVICE bfloat16 bits
   [B][max_imfs][1024][8] (row (b, j) = the residual that IMF j of signal b
   came from; rows of steps that did not run are left as they were), or
   NULL to stop recording. */
fif_status fif_plan_record_features(fif_plan* plan, uint16_t* feats);

#ifdef __cplusplus
}
#endif
#endif /* FIF_H */
