/*
 * sfft.h -- C ABI of an MI355X (gfx950) sparse FFT.
 *
 * The library recovers the k largest Fourier coefficients of an n-point
 * complex signal with the method of Hassanieh, Indyk, Katabi and Price,
 * "Nearly Optimal Sparse Fourier Transform":
 *   problem     given sample access to x in C^n (n = 2^m) and k, output a
 *               k-sparse xhat' with ||xhat - xhat'||_2 <= C * Err(xhat, k),
 *               exactly xhat when xhat is k-sparse, with constant success
 *               probability (Section 1, eq. (1); Section 2 Assumptions).
 *   convention  xhat_f = n^{-1/2} sum_j omega^{f j} x_j, omega = e^{-2 pi i/n}
 *               (Section 2, Notation).  Values are returned in this unitary
 *               convention unless SFFT_FLAG_NUMPY_NORM is set (then * sqrt(n)).
 *   hot path    HashToBins (Algorithm 1; computed as in the proof of the
 *               HashToBins lemma of Section 3): permuted gather
 *               x[sigma (t - a) mod n], flat-window multiply and modulation,
 *               fold into B buckets, B-point FFT; then exact phase decoding
 *               (Algorithm 1) or LocateInner voting and EstimateValues medians
 *               (Algorithms 2 and 3), and a final FP64 median re-estimation.
 *
 * Conventions of every entry point:
 *   * Pointers named *_dev are device pointers on the current HIP device;
 *     pointers named *_host are host pointers.  `stream` is a hipStream_t
 *     passed as void* (NULL = the default stream).
 *   * Nothing throws across the ABI.  On error a status code is returned,
 *     outputs are left untouched (asynchronous entry points: the status
 *     covers the launch), and sfft_last_error() describes the failure.
 *   * Input signals are contiguous, interleaved (re, im) complex64
 *     (SFFT_C64) or complex128 (SFFT_C128) arrays of n elements; a batch is
 *     [count][n] with signal stride n.  The caller owns them and must keep
 *     them alive until the stream has passed the call.
 *   * Output values are complex128, interleaved (re, im), i.e. double[2].
 *   * A plan is immutable after creation and may be shared by threads;
 *     calls that use the same plan on different streams at the same time
 *     race on the plan's workspace (one execute in flight per plan).
 */
#ifndef SFFT_H
#define SFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SFFT_OK = 0,
    SFFT_EINVAL = 1,     /* an argument is out of range or inconsistent      */
    SFFT_ENOTPOW2 = 2,   /* n or B is not a power of two                     */
    SFFT_ENOMEM = 3,     /* device or host allocation failed                 */
    SFFT_EBUDGET = 4,    /* the request does not fit the memory budget       */
    SFFT_EHIP = 5,       /* a HIP runtime call failed                        */
    SFFT_ETRUNC = 6,     /* more coefficients than cap; the top cap returned  */
    SFFT_EUNSUPPORTED = 7,/* parameters valid but not supported by a kernel  */
    SFFT_EAGAIN = 8,     /* a served request has not finished yet            */
    SFFT_ECANCELED = 9   /* a served request was cancelled before it ran     */
} sfft_status_t;

typedef enum { SFFT_MODE_EXACT = 0, SFFT_MODE_GENERAL = 1 } sfft_mode_t;
typedef enum { SFFT_C64 = 0, SFFT_C128 = 1 } sfft_dtype_t;
typedef enum { SFFT_F32 = 0, SFFT_F64 = 1 } sfft_prec_t;

/* flags */
#define SFFT_FLAG_NUMPY_NORM 0x1u   /* return values scaled by sqrt(n)                  */
#define SFFT_FLAG_TIMING 0x2u       /* record HIP events around each batched phase     */

/* per-signal info words written by the batched entry point (4 x uint32)     */
#define SFFT_INFO_ROUNDS 0          /* rounds whose bins were decoded                 */
#define SFFT_INFO_FLAGS 1           /* bit 0: output truncated to cap; bit 1: zhat full */
#define SFFT_INFO_ZHAT 2            /* number of zhat entries before the output filter */
#define SFFT_INFO_LOCATED 3         /* general mode: candidates located (last round)   */

/*
 * Plan description.  sfft_desc_init fills every field with its default;
 * change fields, then call sfft_plan_ex.  Parameter readings (the paper only
 * fixes Theta(.) constants):
 *   n, k      signal length (2^m, 2 <= m <= 40) and sparsity (1 <= k < n)
 *   B         bins of the first hashing round (power of two, 2 <= B <= n)
 *   w         window length, a multiple of B, B <= w <= n; 0 = the window's
 *             default (sfft_window_w): Gaussian, the smallest multiple of B
 *             whose window tail sum_{|t| >= w/2} |G*(t)| <= delta;
 *             Kaiser-Bessel, Kaiser's length rule
 *   seed      seed of the counter-based draws (SplitMix64; see below)
 *   mode      SFFT_MODE_EXACT (Algorithm 1) or SFFT_MODE_GENERAL (Algs 2, 3)
 *   in_dtype  storage type of the input signal
 *   loc_prec  arithmetic of the location hashings (exact pairs, LocateInner
 *             pairs): at large n the phase step 2 pi / n is below FP32
 *             resolution, so the default is SFFT_F64 for n >= 2^20
 *   est_prec  arithmetic of the EstimateValues hashings (general mode)
 *   alpha     flat-window transition fraction (Section 2 definition)
 *   delta     window accuracy ||Ghat - G'||_inf < delta; sets the Gaussian
 *             width sigma_g = (4B/alpha) sqrt(2 ln(3/delta)) (Section 7
 *             construction without its delta -> delta/n normalisation step),
 *             or the Kaiser-Bessel window's shape beta and length (window)
 *   theta     bin threshold of the exact decode (the paper's 1/2 for
 *             integer spectra, Algorithm 1)
 *   g_min     smallest window value G'_{-o(i)} a bin value is divided by
 *   rounds    exact: most NoiselessSparseFFTInner rounds (0 = 16); general:
 *             SparseFFT rounds (0 = max(7, ceil(log4 k) + 2))
 *   b_min     exact: round r uses B_r = max(B >> r, b_min) bins and a window
 *             of w B_r / B samples (Algorithm 1 shrinks B with k_t = k/2^t);
 *             0 = B/16 (at least 2); b_min = B keeps B fixed.  general:
 *             a further floor on B_r = max(B >> r, 4 k_r, b_min) (0 = none;
 *             b_min = B keeps B and w fixed in every round)
 *   patience  exact: stop after this many consecutive rounds whose bins are
 *             all below theta
 *   t, s      LocateInner regions per level and vote tolerance (Algorithm 3)
 *   R_loc     LocateInner measurements per level (Algorithm 3), 1..8
 *   R_est     EstimateValues measurements per round (Algorithm 2), 1..32
 *   cap       output capacity (0 = k)
 *   flags     SFFT_FLAG_*
 *   max_batch largest count accepted by sfft_execute_batch (workspace size)
 *   hash_threads  workgroup size of the batched HashToBins pair launches:
 *             256, 512 or 1024 (0 = 256); an exact-mode launch halves it
 *             (not below 256) while it exceeds the largest B_r of its
 *             rounds.  Launch shape only: results are the same up to the
 *             summation order of a bin's partial sums when B_r < threads
 *   chunks    sfft_execute_batch splits the batch into this many chunks whose
 *             decode overlaps the next chunk's HashToBins, 1..8 (0 = the
 *             SFFT_BATCH_CHUNKS environment variable, else 1).  Launch
 *             shape only: results do not depend on it
 *   stop_count  exact mode: also stop after stop_patience consecutive
 *             rounds whose bins are all below theta once at least this many
 *             zhat entries exceed theta/2 in magnitude (0 = off; k for
 *             exactly k-sparse input: with k such entries empty bins leave
 *             nothing to find unless a wrong entry stands in for a
 *             coefficient that stays invisible).  Ignored in general mode
 *   stop_patience  empty rounds in a row that end a signal under stop_count
 *             (>= 1; default 2: one empty round can hide a coefficient
 *             placed one location off, whose residual pair cancels in a bin)
 *   ratio_tol exact mode: decode only bins whose squared magnitudes at the
 *             two shifts agree within this fraction, ||u1|^2 - |u0|^2| <=
 *             ratio_tol |u0|^2 (0 = off): an isolated coefficient gives equal
 *             magnitudes (exact-estimation lemma), a collision rarely does.
 *             Such bins still count as nonempty
 *   group0    exact mode, batched: rounds hashed for every signal in the
 *             first HashToBins launch (0 = up to the first round at b_min
 *             bins plus patience + 1, the earliest the patience rule can stop
 *             a signal; capped at rounds).  Later launches hash 2, 2, 4, 8,
 *             ... rounds for the signals still decoding.  Launch shape only:
 *             results do not depend on it
 *   group_step  exact mode, batched: rounds of the second round group, each
 *             later group twice the previous (0 = 2, 2, 4, 8, ...).  Launch
 *             shape only
 *   hash_order  exact mode, batched: order of the (signal, round)
 *             workgroups of a HashToBins pair launch.  0: round-major (all
 *             signals' round r, then round r + 1, ...: the largest rounds
 *             first); 1: signal-major (all rounds of signal 0, then of
 *             signal 1, ...: fewer signals' samples in flight at once);
 *             2: signal-major per XCD (workgroups are handed to the 8 XCDs
 *             in turn, so workgroup j runs on XCD j mod 8: the signals
 *             s = x (mod 8) go to XCD x, each signal's rounds in a row, so
 *             they share that XCD's L2; batches whose size is not a
 *             multiple of 8 take order 1).  Launch shape only: results do
 *             not depend on it
 *   alpha_decay  exact mode: 0 (or 1) keeps alpha in every round; a value
 *             in (0, 1) shrinks it as the bin count shrinks (Section 3's
 *             alpha_t schedule): round r uses alpha * alpha_decay^m, m = r
 *             up to the first round at the smallest bin count and fixed
 *             after it, with a window w * (B_r / B) / alpha_decay^m rounded
 *             up to a multiple of B_r (the same tail mass) and its own
 *             window table.  Every round's window must stay within n.
 *   hash_split  exact mode, batched path: 0 or 1 hashes each (signal,
 *             round) in one workgroup; 2..64 splits its window over that
 *             many workgroups (partial folds summed in a fixed order, then
 *             the FFT), for small batches whose few hashings would each walk
 *             a long window on one CU.  Launch shape only: results equal the
 *             unsplit ones up to the order of floating-point additions, and
 *             do not depend on the batch.  Needs chunks <= 1.
 *   hash_mode exact mode, batched path (at most one chunk): 0 gathers every
 *             round's window (w_r + 1 random samples, a memory line each);
 *             1 reads the whole signal contiguously instead (stream mode:
 *             each sample is kept where its permuted position falls in the
 *             window) for the rounds whose window covers at least n/8
 *             samples, where n contiguous samples cost no more bytes than
 *             the gathered lines; 2 streams every round.  The raw bins are
 *             the same up to the order of floating-point additions.  The
 *             plain path and general mode always gather
 *   refine_shift  exact mode, batched path: 0 (off) or A, the shift of a
 *             third hashing per round (the multi-shift idea of LocateInner,
 *             Algorithm 3, used to estimate the phase with a few more
 *             samples).  The pair's phase gives a coarse permuted position
 *             p0; the position c in [p0 - E, p0 + E] whose angle
 *             2 pi (A c mod n) / n is nearest the phase of u / u_A (ties: the
 *             smaller c) replaces it, so FP32 bins (loc_prec SFFT_F32) locate
 *             at n where the pair's FP32 phase alone cannot.  The same pair
 *             workgroup accumulates the third hashing: A <= w_r reads
 *             A more samples per round, A > w_r another w_r.  Needs
 *             2 <= A < n, A (2E + 1) < n, hash_split <= 1 and hash_mode 0
 *   refine_window  E, the half-width of the refinement's candidate window
 *             (1..1024; default 16 when refine_shift is set)
 *   window    the flat window (G, G') of the Section 2 definition: 0 the
 *             Gaussian construction of the Section 7 lemma; 1 the ideal
 *             low-pass with cut-off C = (1 - alpha/2)/(2B) tapered by a
 *             Kaiser-Bessel window I0(beta sqrt(1 - (2t/w)^2)) / I0(beta),
 *             beta and the default w from Kaiser's rules for a ripple of
 *             delta/2 over the transition band (about half the Gaussian's
 *             support at the same alpha and delta), G' in the transition
 *             band the window's own response (tabulated at plan time)
 */
typedef struct {
    uint64_t n;
    uint64_t w;
    uint64_t seed;
    uint32_t k;
    uint32_t B;
    int32_t mode;
    int32_t in_dtype;
    int32_t loc_prec;
    int32_t est_prec;
    double alpha;
    double delta;
    double theta;
    double g_min;
    double s;
    uint32_t rounds;
    uint32_t b_min;
    uint32_t patience;
    uint32_t t;
    uint32_t R_loc;
    uint32_t R_est;
    uint32_t cap;
    uint32_t flags;
    uint32_t max_batch;
    uint32_t hash_threads;
    uint32_t chunks;
    uint32_t stop_count;
    uint32_t stop_patience;
    uint32_t group0;
    double ratio_tol;
    uint32_t group_step;
    uint32_t hash_order;
    double alpha_decay;
    uint32_t hash_split;
    uint32_t hash_mode;
    uint64_t refine_shift;
    uint32_t refine_window;
    uint32_t window;
} sfft_plan_desc_t;

typedef struct sfft_plan_s* sfft_plan_t;

/* Device bytes a plan created from *d would allocate (window tables,
 * twiddles, the workspace for max_batch signals and the plain path's
 * buffers); 0 when *d does not validate.  Pure host function. */
uint64_t sfft_plan_device_bytes(const sfft_plan_desc_t* d);

/* Samples of x one signal's sparse transform under *d reads, counting
 * every hashing's window: exact mode, the pair of each round up to the
 * earliest stop (round group 0: w_r + 1 samples per round, or n for a round
 * in stream mode); general mode, all rounds, each with its LocateInner
 * pairs (2 w_r per pair) and EstimateValues hashings (w_r each).  Each
 * gathered sample is a random access that costs a whole memory line (a
 * streamed one an eighth of a 64-byte line), so this against n sizes the
 * sparse path against a dense FFT.  0 when *d does not validate.  Pure host
 * function. */
uint64_t sfft_plan_samples(const sfft_plan_desc_t* d);

/* Rounds of round group 0 that *d hashes in stream mode (hash_mode); 0 when
 * none or when *d does not validate.  Pure host function. */
uint32_t sfft_plan_stream_rounds(const sfft_plan_desc_t* d);

/* Fill *d with the defaults for (n, k, B, w, seed); exact mode, complex64.
 * Pure host function: no device is touched.  Errors: SFFT_EINVAL if d is NULL. */
sfft_status_t sfft_desc_init(sfft_plan_desc_t* d, uint64_t n, uint32_t k, uint32_t B,
                             uint64_t w, uint64_t seed);

/* Check a description against the limits listed above (and the kernels'
 * LDS limit B <= 4096).  Pure host function.  Returns SFFT_OK, SFFT_ENOTPOW2, SFFT_EINVAL or
 * SFFT_EUNSUPPORTED. */
sfft_status_t sfft_validate_params(const sfft_plan_desc_t* d);

/* Default window length for (n, B, alpha, delta), as described for w above;
 * returns n when no shorter window meets delta.  Pure host function. */
uint64_t sfft_default_w(uint64_t n, uint32_t B, double alpha, double delta);

/* The same for the flat window `window` (0 Gaussian, as sfft_default_w; 1
 * Kaiser-Bessel: Kaiser's length rule (A - 7.95) / (14.36 alpha / (2B)) + 1
 * with A = -20 log10(delta / 2), rounded up to a multiple of B, at most n);
 * 0 for an unknown window.  Pure host function. */
uint64_t sfft_window_w(uint64_t n, uint32_t B, double alpha, double delta, uint32_t window);

/* Create a plan: validates, builds the FP64 window tables G (Section 7
 * construction) and FFT twiddles on the host, copies them to the current
 * device and allocates the workspace for max_batch signals.  The plan owns
 * all of its device memory.  Errors: validation codes, SFFT_ENOMEM, SFFT_EHIP. */
sfft_status_t sfft_plan_ex(const sfft_plan_desc_t* d, sfft_plan_t* out);

/* sfft_plan_ex with the defaults of sfft_desc_init: plan(n, k, B, w, seed). */
sfft_status_t sfft_plan(uint64_t n, uint32_t k, uint32_t B, uint64_t w, uint64_t seed,
                        sfft_plan_t* out);

/* Copy of the plan's (resolved) description; w is the resolved window. */
sfft_status_t sfft_plan_get_desc(sfft_plan_t p, sfft_plan_desc_t* out);

/* Release every device and host resource of the plan.  NULL is allowed. */
sfft_status_t sfft_destroy(sfft_plan_t p);

/*
 * One signal, one request at a time ("plain" path).  Each hashing is
 * launched on its own, split over many workgroups with a fixed-order
 * two-level reduction; the host drives the rounds and stops early
 * (exact mode: `patience` empty rounds).  Synchronises `stream` before
 * returning.
 *   x_dev      n input samples (in_dtype)
 *   idx_host   [cap] output indices, ascending
 *   val_host   [2*cap] output values (complex128)
 *   cap        capacity of idx_host/val_host (>= 1)
 *   count_host number of coefficients written
 *   info_host  optional [4] info words (SFFT_INFO_*), may be NULL
 * Returns SFFT_ETRUNC (outputs valid) when more than cap coefficients were
 * recovered; then the cap largest by magnitude are returned.
 */
sfft_status_t sfft_execute(sfft_plan_t p, const void* x_dev, uint64_t* idx_host,
                           double* val_host, uint32_t cap, uint32_t* count_host,
                           uint32_t* info_host, void* stream);

/*
 * A batch of independent signals ("batched" path).  The batch runs as one
 * chunk (SFFT_BATCH_CHUNKS=c splits it into c).  For each chunk, one launch
 * hashes every signal (HashToBins): general mode every round; exact mode the
 * first round group (up to patience + 1 rounds past the first round at
 * b_min bins).  A decode workgroup per signal runs the rounds on the device
 * (exact: NoiselessSparseFFTInner; general: SparseFFT).  In exact mode each
 * later group of two rounds is hashed, then decoded, only for signals whose
 * decode has not stopped.  The FP64 re-estimation and the output follow.
 * Chunk c's
 * decode runs on the plan's auxiliary stream while chunk c+1's HashToBins
 * runs on `stream`; `stream` waits for the last decode before the call's
 * work is complete.  Each chunk's launch sequences are captured once into
 * hipGraphs and replayed (keyed by the argument pointers and count).
 * The capture (the first call with a new argument set) runs on a
 * plan-private stream in thread-local capture mode; other threads of the
 * process should not allocate, free or synchronise the device while it
 * runs (a capture on one thread beside such calls on others has failed
 * with a HIP error); replays carry no such condition.  With the
 * environment variable SFFT_NO_GRAPH=1 every call launches the kernels
 * directly, with the same results.  The serving runtime does not capture.
 * Asynchronous on `stream`; nothing is copied to the host.
 *   x_dev      [count][n] signals (in_dtype)
 *   count      1 <= count <= max_batch
 *   seeds_dev  [count] per-signal seeds (uint64) or NULL for the plan seed
 *   idx_dev    [count][cap] indices (ascending per signal; unused slots 0)
 *   val_dev    [count][cap][2] values (complex128)
 *   count_dev  [count] number of coefficients per signal
 *   info_dev   [count][4] info words (SFFT_INFO_*), may be NULL
 * Results of one signal depend only on (its samples, its seed, the plan),
 * never on the other signals of the batch or on the chunking.
 */
sfft_status_t sfft_execute_batch(sfft_plan_t p, const void* x_dev, uint32_t count,
                                 const uint64_t* seeds_dev, uint64_t* idx_dev, double* val_dev,
                                 uint32_t* count_dev, uint32_t* info_dev, void* stream);

/*
 * Raw HashToBins of one signal at two shifts of one permutation (steps 1-3
 * of the HashToBins computation in Section 3): bins of P_{sigma,a,b} x and of
 * P_{sigma,a+beta,b} x with B_r bins and a window of w * B_r / B samples
 * (plan alpha, delta), scaled by sqrt(n), in `prec` arithmetic.  Exposed for
 * parity tests of the gather/fold/FFT kernels.  out0_dev/out1_dev are
 * [B_r][2] doubles.  sigma must be odd; a, b, beta < n; B_r a power of two
 * dividing the plan's B schedule (B_r <= B).
 */
sfft_status_t sfft_hash_pair_raw(sfft_plan_t p, const void* x_dev, uint64_t sigma, uint64_t a,
                                 uint64_t beta, uint64_t b, uint32_t B_r, int32_t prec,
                                 double* out0_dev, double* out1_dev, void* stream);

/*
 * Phase durations of the last sfft_execute_batch on a plan created with
 * SFFT_FLAG_TIMING, from HIP events recorded between the replayed graphs on
 * the streams they run on.  The caller must have synchronised the launch
 * stream.  ms_host[0] = state reset + the first HashToBins launch summed over
 * the batch's chunks (exact mode: the first round group, hashed for every
 * signal; general mode: every round), [1] = the rest summed over the chunks:
 * decode, the HashToBins of later exact round groups (only for signals whose
 * decode has not stopped), re-estimation and output (these run on the plan's
 * auxiliary stream, overlapped with the next chunk's first HashToBins),
 * [2] = time from the end of the last first-launch HashToBins to the end of
 * the batch, [3] = whole batch (milliseconds); [4] (if n_out > 4) = number of
 * chunks.  Errors: SFFT_EINVAL when the flag is not set or nothing ran yet,
 * SFFT_EHIP.
 */
sfft_status_t sfft_plan_timings(sfft_plan_t p, double* ms_host, uint32_t n_out);

/*
 * Algorithmic HBM bytes of the first batched HashToBins launch for `count`
 * signals (exact mode: the rounds of the first round group, which every
 * signal hashes; general mode: every round): every distinct input sample
 * read once per hashing pair ((w_r + 1) samples of in_dtype per round) plus
 * the raw bins written (2 B_r complex128 per round).  Pure host function.
 */
uint64_t sfft_plan_h2b_bytes(sfft_plan_t p, uint32_t count);

/*
 * Round groups of the batched exact path: ends_host[g] = one past the last
 * round of group g (ascending, the last equals the plan's rounds).  Group 0
 * is hashed for every signal; each later group only for signals whose decode
 * has not stopped.  Writes min(*n_groups, max) ends and sets *n_groups to the
 * number of groups (general mode: one group of every round).  Pure host
 * function.  Errors: SFFT_EINVAL for NULL p or n_groups.
 */
sfft_status_t sfft_plan_round_groups(sfft_plan_t p, uint32_t* ends_host, uint32_t max, uint32_t* n_groups);

/*
 * Copy the raw bins of one hashing slot of one signal from the batched
 * workspace (after sfft_execute_batch has completed on `stream`), for parity
 * tests of the batched HashToBins jobs.  Slots: exact mode, slot = round;
 * general mode, slot = first slot of round r + (level - 1) * R_loc + rep for
 * LocateInner pairs, then the R_est EstimateValues hashings.  out_dev is
 * [2][B_r][2] doubles (the two hashings of the slot); *B_r_out receives B_r.
 * Errors: SFFT_EINVAL for a signal beyond max_batch or a slot out of range.
 */
sfft_status_t sfft_plan_raw_slot(sfft_plan_t p, uint32_t sig, uint32_t slot, double* out_dev, uint32_t* B_r_out,
                                 void* stream);

/*
 * Copy the raw bins of the refinement hashing (shift refine_shift) of exact
 * round `round` of one signal from the batched workspace, after
 * sfft_execute_batch has completed on `stream`.  out_dev is [B_r][2]
 * doubles; *B_r_out receives B_r.  Rounds after a signal stopped hold stale
 * bins.  Errors: SFFT_EINVAL for NULL arguments, a plan without
 * refine_shift, or a signal or round out of range.
 */
sfft_status_t sfft_plan_raw_refine(sfft_plan_t p, uint32_t sig, uint32_t round, double* out_dev, uint32_t* B_r_out,
                                   void* stream);

/* sizeof(sfft_plan_desc_t) as this library was built, so a binding can
 * check its copy of the struct. */
uint32_t sfft_plan_desc_bytes(void);

/* Human-readable name of a status code (static storage). */
const char* sfft_status_string(sfft_status_t s);

/* Message of the last failure on the calling thread ("" if none). */
const char* sfft_last_error(void);

/* SplitMix64 counter draw used for every random choice of the method:
 * the (c+1)-th output of SplitMix64 started at `seed` (Steele, Lea and Flood,
 * OOPSLA 2014).  Counter layout c = round<<32 | level<<20 | rep<<8 | purpose.
 * Pure host function, exported so that callers can reproduce a plan's draws. */
uint64_t sfft_splitmix64(uint64_t seed, uint64_t c);

/* ================================================================ serving ==
 *
 * A server runs sparse FFT requests of mixed n, k and mode on one GPU with
 * continuous batching (the serving pattern of the problem statement: requests
 * admitted as they arrive, against a device-memory budget, with plans and
 * window tables kept resident):
 *   * a request (n, k, mode) maps to a shape: k rounded up to a power of two
 *     (at least 8), B = 4k' (exact) or 16k' (general) within [64 or 256,
 *     min(4096, n/16)], the Kaiser-Bessel window (window = 1) at its default
 *     length for the mode's delta; exact shapes
 *     use b_min = max(32, B/32) (at most B), at most 24 rounds, patience 5,
 *     hash_split = B/256 (1 to 16 parts) and hash_mode 1 (stream mode for
 *     rounds whose window covers n/8 or more).  Where that window would
 *     cover the whole signal (w >= n), or where a request served alone is
 *     predicted to finish sooner on the dense path, the request takes the
 *     dense path: predicted milliseconds, fitted to solo service times
 *     measured on MI355X, sparse exact SFFT_SERVER_EXACT_MS +
 *     SFFT_SERVER_GATHER_NS x gathered samples + SFFT_SERVER_STREAM_NS x
 *     streamed samples, sparse general SFFT_SERVER_GENERAL_MS +
 *     SFFT_SERVER_GENERAL_NS x samples (sfft_plan_samples,
 *     sfft_plan_stream_rounds), dense SFFT_SERVER_DENSE_MS +
 *     SFFT_SERVER_DENSE_NS x n.  The dense path is a full-length
 *     FP32 FFT (hipFFT, loaded on first use) and the k bins of largest
 *     magnitude (exact mode: those above theta/2);
 *   * each shape gets up to `instances` resident plan instances (workspace
 *     for `slots` signals each), created when needed, each on a thread of
 *     its own; idle sparse-path instances of other shapes with no waiting
 *     request are evicted, least recently used first, when a new one would
 *     exceed `budget_bytes` (which counts the library's allocations, not the
 *     work areas hipFFT allocates for the dense path's plans); no eviction
 *     runs while an instance is being built; dense-path instances are not
 *     evicted (see SFFT_SERVER_EVICT_DENSE);
 *   * a scheduler thread batches the waiting requests of each shape (oldest
 *     shape first) onto idle instances, one stream per instance, so batches
 *     of different shapes overlap on the device.
 * A request's result depends only on its samples, its seed and its shape:
 * it is the same alone and in any mix.  Inputs are complex64.  Batches of
 * different shapes overlap only as far as the process's hardware queues
 * allow: run servers with GPU_MAX_HW_QUEUES=16 (HIP's default is 4), set
 * before the process first uses HIP.
 */
typedef struct sfft_server_s* sfft_server_t;

/* server flags */
#define SFFT_SERVER_FAKE_DEVICE 0x1u /* no device work: instances allocate nothing and
                                        every batch finishes after fake_service_ms on a
                                        host timer with no coefficients; admission,
                                        eviction, batching and statistics run as usual
                                        (for testing the scheduler without a GPU)      */
#define SFFT_SERVER_DENSE_ONLY 0x2u  /* every request takes the dense path            */
#define SFFT_SERVER_SPARSE_ONLY 0x4u /* every request whose sparse plan validates with
                                        w < n takes the sparse path, whatever the path
                                        model predicts                                  */
#define SFFT_SERVER_EVICT_DENSE 0x8u /* also evict idle dense-path instances (by default
                                        they stay resident until the server is destroyed,
                                        and a shape that cannot fit beside them fails with
                                        SFFT_EBUDGET).  Not exercised on the GPU: a run
                                        that evicted and rebuilt hipFFT-backed instances
                                        under a small budget once stopped making progress,
                                        cause not found                                 */
/* the path model (milliseconds and nanoseconds per sample) */
#define SFFT_SERVER_EXACT_MS 0.13
#define SFFT_SERVER_GATHER_NS 1.05
#define SFFT_SERVER_STREAM_NS 0.03
#define SFFT_SERVER_GENERAL_MS 0.75
#define SFFT_SERVER_GENERAL_NS 0.13
#define SFFT_SERVER_DENSE_MS 0.09
#define SFFT_SERVER_DENSE_NS 0.027

typedef struct {
    uint64_t budget_bytes;   /* device memory the server may hold (instances)   */
    uint32_t slots;          /* signals per batch of one instance, 1..1024      */
    uint32_t instances;      /* instances per shape (batches in flight), 1..16  */
    int32_t device;          /* HIP device the server runs on                  */
    uint32_t flags;          /* SFFT_SERVER_*                                   */
    double delta_exact;      /* window accuracy of exact-mode shapes            */
    double delta_general;    /* window accuracy of general-mode shapes          */
    double theta;            /* exact-mode bin threshold                        */
    double fake_service_ms;  /* batch duration under SFFT_SERVER_FAKE_DEVICE    */
} sfft_server_desc_t;

typedef struct {
    const void* x_dev;       /* n complex64 samples on the server's device;
                                caller-owned until the request has finished  */
    uint64_t n;              /* 2^10 .. 2^30                                    */
    uint64_t seed;           /* the request's draws                             */
    uint32_t k;              /* 1 .. 1024                                       */
    int32_t mode;            /* SFFT_MODE_EXACT or SFFT_MODE_GENERAL            */
    uint64_t* idx_host;      /* [k] indices, ascending (caller-owned, or NULL)  */
    double* val_host;        /* [k][2] values, unitary convention (or NULL)     */
} sfft_request_t;

typedef struct {
    int32_t status;          /* SFFT_OK or the failure                          */
    uint32_t count;          /* coefficients written (<= k)                     */
    uint32_t flags;          /* SFFT_INFO_FLAGS word (sparse path)              */
    uint32_t rounds;         /* rounds decoded (sparse path)                    */
    int32_t path;            /* 0 sparse, 1 dense                               */
    uint32_t reserved;
    double queue_ms;         /* submit -> launch                                */
    double service_ms;       /* launch -> results on the host                   */
    double latency_ms;       /* submit -> results on the host                   */
    char message[128];       /* why it failed, NUL-terminated (empty on success):
                                the failing build or launch call and its HIP
                                error, or the budget reason                     */
} sfft_request_result_t;

typedef struct {
    uint64_t completed, dense, failed, batches, evictions;
    uint64_t bytes_in_use;   /* device bytes held by instances now              */
    uint64_t peak_bytes;     /* largest bytes_in_use since the last reset       */
    uint32_t pending, inflight, instances, reserved;
    double mean_batch;       /* requests per launched batch                     */
    double p50_ms, p99_ms;   /* latency percentiles (completed since reset)     */
    double queue_p50_ms, service_p50_ms;
    double rate;             /* completed per second, first submit -> last completion */
} sfft_server_stats_t;

/* The serving runtime's dense-path selection, for callers that run their
 * own full-length FFT (and for tests): of each of `count` spectra spec_dev
 * [count][n] complex64 (unnormalised FFT outputs), the `cap` bins of
 * largest magnitude, ties to the smaller index, in ascending index order,
 * values times `scale` as complex128.  Magnitudes are ranked by the FP32
 * key fma(re, re, im*im); with keep_above >= 0 only bins whose key exceeds
 * the FP32 value of (keep_above / scale)^2 are kept (exact mode: theta/2).
 * n a power of two in [2^10, 2^30], cap in [1, 8192], count >= 1.  Outputs
 * as in sfft_execute_batch: idx_dev [count][cap], val_dev [count][cap][2],
 * count_dev [count]; unused slots are zero.  scratch_dev:
 * sfft_dense_topk_scratch_bytes(count) bytes of device memory, overwritten.
 * Asynchronous on `stream` (a hipStream_t, NULL = the null stream).
 * Errors: SFFT_EINVAL, SFFT_ENOTPOW2, SFFT_EHIP. */
uint64_t sfft_dense_topk_scratch_bytes(uint32_t count);
sfft_status_t sfft_dense_topk(const void* spec_dev, uint64_t n, uint32_t count, uint32_t cap, double scale,
                              double keep_above, uint64_t* idx_dev, double* val_dev, uint32_t* count_dev,
                              void* scratch_dev, void* stream);

/* sfft_dense_topk without the scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same selection and results, with
 * the scratch taken from a static device array that the library holds on
 * each device from load to process end (about 1.3 MB, room for
 * sfft_dense_topk_noalloc_max_count() = 64 spectra).  It calls no
 * allocating routine; its first call on a device looks up that device's
 * address of the array.  Every call on one device shares that array, which
 * keeps the last call's contents (each call clears what it needs with a
 * kernel, no memset): calls that overlap on one device, on different
 * streams or threads, race and must be serialised by the caller.
 * Errors: as sfft_dense_topk, and SFFT_EINVAL for count above the maximum
 * (nothing is launched). */
uint32_t sfft_dense_topk_noalloc_max_count(void);
sfft_status_t sfft_dense_topk_noalloc(const void* spec_dev, uint64_t n, uint32_t count, uint32_t cap, double scale,
                                      double keep_above, uint64_t* idx_dev, double* val_dev, uint32_t* count_dev,
                                      void* stream);

/* Defaults: 16 GiB budget, 32 slots, 2 instances per shape, device 0,
 * delta 1e-9 (exact) / 1e-6 (general), theta 0.25.  Errors: SFFT_EINVAL. */
sfft_status_t sfft_server_desc_init(sfft_server_desc_t* d);

/* The shape a request (n, k, mode) maps to: its plan description, whether it
 * takes the dense path, and the device bytes of one instance.  Pure host
 * function.  Errors: SFFT_ENOTPOW2, SFFT_EINVAL. */
sfft_status_t sfft_server_shape(const sfft_server_desc_t* d, uint64_t n, uint32_t k, int32_t mode,
                                sfft_plan_desc_t* plan_out, int32_t* dense_out, uint64_t* bytes_out);

/* Start a server (its scheduler thread).  Errors: SFFT_EINVAL, SFFT_ENOMEM. */
sfft_status_t sfft_server_create(const sfft_server_desc_t* d, sfft_server_t* out);

/* Queue one request; *ticket names it.  The output buffers are written when
 * it finishes.  Errors: SFFT_EINVAL, SFFT_ENOTPOW2 (bad request), SFFT_EBUDGET
 * (one instance of its shape exceeds the budget). */
sfft_status_t sfft_server_submit(sfft_server_t s, const sfft_request_t* req, uint64_t* ticket);

/* SFFT_EAGAIN while the request runs; otherwise its status, with *res filled
 * (may be NULL) and the ticket released. */
sfft_status_t sfft_server_poll(sfft_server_t s, uint64_t ticket, sfft_request_result_t* res);

/* Block until the request finishes (timeout_ms < 0: no limit; SFFT_EAGAIN on
 * timeout), then as sfft_server_poll. */
sfft_status_t sfft_server_wait(sfft_server_t s, uint64_t ticket, double timeout_ms, sfft_request_result_t* res);

/* Withdraw a request that has not been launched yet: it finishes at once with
 * status SFFT_ECANCELED (collected by poll/wait as usual).  Returns SFFT_OK,
 * SFFT_EAGAIN when it is already running or finished (its result will come),
 * SFFT_EINVAL for an unknown ticket. */
sfft_status_t sfft_server_cancel(sfft_server_t s, uint64_t ticket);

/* Counters and latency percentiles since the last reset. */
sfft_status_t sfft_server_stats(sfft_server_t s, sfft_server_stats_t* st);
sfft_status_t sfft_server_reset_stats(sfft_server_t s);

/* Finish every queued request, stop the scheduler and free all instances. */
sfft_status_t sfft_server_destroy(sfft_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* SFFT_H */
