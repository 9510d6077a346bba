/*
 * pusch.h -- C ABI of the MI355X (gfx950) PUSCH lower-PHY receive chain.
 *
 * The chain follows Sec. II of "Efficient Parallelization of 5G-PUSCH on a
 * Scalable RISC-V Many-core Processor": OFDM demodulation (one FFT per antenna
 * and OFDM symbol), beamforming (a matrix product with known coefficients),
 * least-squares channel estimation on block-type pilot symbols, and the MIMO
 * stage of Eq. 2, x = (H^H H + sigma^2 I)^{-1} H^H y, evaluated through a
 * Cholesky decomposition of the Gram matrix and two triangular solves.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Numbers     complex values are interleaved FP32 pairs (pusch_c32, the same
 *             bytes as torch.complex64); arithmetic on the GPU is FP32 except
 *             where an entry point states a narrower form (pusch_slot_mixed,
 *             pusch_slot_bf16, the denoiser's bfloat16 layers).
 * Pointers    every data pointer is a caller-owned DEVICE buffer on the
 *             current HIP device.  The library never frees, retains or
 *             reallocates one after the call returns.  Buffers must be 8-byte
 *             aligned (16-byte alignment gives faster loads).
 * Streams     `stream` is a hipStream_t passed as void* (NULL = the legacy
 *             default stream).  Calls only enqueue work and return; outputs
 *             and status arrays are valid once the stream has been
 *             synchronised.  No call synchronises the device or allocates in
 *             steady state.  The first call on a device builds small
 *             immutable tables (FFT twiddles, DFT beamformers) once, and the
 *             first call with a slot geometry builds that geometry's
 *             estimation tables (channel interpolation taps, noise-estimation
 *             neighbours) once, on a stream of the library's own that it
 *             waits for (never on the caller's stream).
 * Errors      arguments are checked on the host before any device work; a
 *             rejected call returns a negative code and enqueues nothing.
 *             Launch failures return PUSCH_EHIP.  Numerical failure of one
 *             subcarrier (non-positive Cholesky pivot) is reported in the
 *             per-subcarrier status array, not in the return code.
 * Layouts     row-major; the innermost index is listed last.  "RE-major"
 *             beam-domain grids store, for every resource element (RE), its
 *             N_B beam values contiguously -- the per-subcarrier vector y of
 *             Eq. 1.
 * Subcarriers active subcarrier k (0 <= k < n_sc) sits on FFT bin
 *             (k - n_sc/2) mod n_fft (centred band, DC used, integer halving).
 * Pilots      block-type pilot symbols (whole OFDM symbols).  The n_ue UEs
 *             share each pilot symbol as a frequency comb: on pilot symbol j
 *             (0-based among the pilot symbols) subcarrier k carries the pilot
 *             of UE (k + j * (n_ue / n_pilot)) mod n_ue (staggered), or of UE
 *             k mod n_ue on every pilot symbol when a slot descriptor asks for
 *             the aligned comb.  Pilot values must be non-zero.
 */
#ifndef PUSCH_H_
#define PUSCH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float re, im;
} pusch_c32;

enum {
  PUSCH_OK = 0,
  PUSCH_EINVAL = -1,       /* bad argument (null pointer, size out of range, overlap) */
  PUSCH_EUNSUPPORTED = -2, /* valid request outside what this library implements */
  PUSCH_EHIP = -3,         /* HIP runtime / launch failure */
  PUSCH_ENOMEM = -4        /* workspace too small, or device table allocation failed */
};

/* Limits of this library. */
#define PUSCH_MAX_BEAMS 64
#define PUSCH_MAX_UES 32
#define PUSCH_MAX_PILOTS 4
#define PUSCH_MAX_SYMBOLS 16

/* Human-readable text for a return code (static storage). */
const char* pusch_strerror(int code);

/* Build the per-device immutable tables for the current device now instead
 * of on first use, and look up the device address of the scratch array of
 * pusch_noise_est_static.  Returns PUSCH_OK or PUSCH_EHIP. */
int pusch_init(void);

/*
 * OFDM demodulation (Sec. II; Table 1, row "OFDM dem.").
 * For each of `batch` time-domain vectors x_i of n_fft samples computes the
 * unscaled forward DFT X_i[f] = sum_n x_i[n] exp(-2 pi i f n / n_fft).
 *   n_fft  in {64, 256, 1024, 2048, 4096}, else PUSCH_EUNSUPPORTED.
 *   n_sc   0: write all n_fft bins in natural order, X is [batch][n_fft];
 *          1..n_fft: write only the n_sc active subcarriers in subcarrier
 *          order (bin (k - n_sc/2) mod n_fft), X is [batch][n_sc].
 *   x      [batch][n_fft].  x == X is allowed when n_sc is 0 or n_fft; any
 *          other overlap of x and X is PUSCH_EINVAL.
 *   batch  >= 0 (0 is a no-op).
 */
int pusch_fft(const pusch_c32* x, pusch_c32* X, int n_fft, int n_sc, long long batch, void* stream);

/*
 * Beamforming (Sec. II; Table 1, row "BF"): for every batch item i and RE n,
 *   Y_i[n][b] = sum_a W[b][a] X_i[a][n],   b < n_beams, a < n_ant, n < n_re.
 *   W      [n_beams][n_ant] known coefficients, or NULL for the built-in
 *          beamformer W[b][a] = exp(-2 pi i b a / n_ant) / sqrt(n_ant) (rows
 *          of the unitary DFT; requires n_beams <= n_ant).
 *   X      [batch][n_ant][ld_x] antenna-domain grid (antenna-major, as
 *          pusch_fft writes it), ld_x >= n_re.
 *   Y      [batch][n_re][n_beams] RE-major beam-domain grid.  Must not
 *          overlap X or W.
 *   1 <= n_beams <= PUSCH_MAX_BEAMS, 1 <= n_ant <= 1024, n_re >= 0, batch >= 0.
 */
int pusch_beamform(const pusch_c32* W, const pusch_c32* X, pusch_c32* Y, int n_beams, int n_ant, int n_re,
                   long long ld_x, long long batch, void* stream);

/*
 * Least-squares channel estimation (Sec. II, CHE; Table 1, row "CHE").
 * On pilot symbol j, subcarrier k (owned by UE l, see "Pilots") the LS value
 * of UE l's beam-domain channel is Yp_j[k][:] * conj(p_j[k]) / |p_j[k]|^2.
 * Per UE the values of all pilot symbols are merged by subcarrier (averaged
 * where two pilot symbols hit the same subcarrier) and interpolated linearly
 * along k, holding the first / last value beyond the outermost pilots.
 *   Yp     [batch][n_pilot][n_sc][n_beams] RE-major beam-domain pilot symbols.
 *   pilots [batch][n_pilot][n_sc] pilot value on each pilot RE (non-zero).
 *   H      [batch][n_sc][n_ue][n_beams]: per subcarrier, row l is UE l's
 *          channel across the beams (column l of H in Eq. 1).
 *   1 <= n_pilot <= PUSCH_MAX_PILOTS, 1 <= n_ue <= min(PUSCH_MAX_UES, n_beams),
 *   n_ue <= n_sc, 1 <= n_beams <= PUSCH_MAX_BEAMS, batch >= 0.
 */
int pusch_chest(const pusch_c32* Yp, const pusch_c32* pilots, pusch_c32* H, int n_beams, int n_ue, int n_sc,
                int n_pilot, long long batch, void* stream);

/*
 * Noise-variance estimation (Sec. II, NE; Table 1, row "NE"): the variance of
 * the difference between the received pilot REs and the values that the
 * estimated channel and the known pilots predict there, per batch item.
 * The LS estimate of pusch_chest passes through every pilot position, so
 * the prediction for pilot RE (j, k) of UE l is p_j[k] times UE l's channel
 * interpolated (as pusch_chest) from its OTHER pilot positions: the nearest
 * one below k and the nearest one above, or the nearest one on the only side
 * there is.  With weights w_i on positions holding c_i averaged LS values of
 * pilots p_s, the difference r = y - p h has noise variance sigma^2 kappa
 * per beam, kappa = 1 + |p|^2 sum_i (w_i / c_i)^2 sum_{s at i} 1 / |p_s|^2, and
 *   sigma2[i] = sum |r|^2 / (n_beams * sum kappa)
 * over all pilot REs of item i: unbiased for white noise of equal variance
 * on every beam (unitary beamformer rows) when the channel is linear in k
 * between the positions used; channel variation beyond that adds to it.
 *   Yp, pilots  as pusch_chest.
 *   sigma2 [batch] FP32 estimates (device).
 *   ws     device scratch of at least pusch_noise_est_workspace_bytes(batch)
 *          bytes, 8-byte aligned; its contents are not needed afterwards.
 *   2 n_ue <= n_sc <= 4096 (every UE has two pilot positions), other limits
 *   as pusch_chest.  sigma2, ws, Yp and pilots must not overlap.
 */
size_t pusch_noise_est_workspace_bytes(long long batch);
int pusch_noise_est(const pusch_c32* Yp, const pusch_c32* pilots, float* sigma2, int n_beams, int n_ue, int n_sc,
                    int n_pilot, long long batch, void* ws, size_t ws_bytes, void* stream);

/*
 * The same noise-variance estimate as pusch_noise_est, for callers that
 * cannot allocate device memory or pass a workspace (code captured into a
 * HIP graph, tight serving loops, harnesses that forbid hipMalloc).  It
 * allocates nothing and calls no allocating routine: its scratch (the
 * geometry's neighbour table and the per-item partial sums, 2.25 MiB) is a
 * device array inside the library, one copy per GPU, whose address is looked
 * up once per device (by pusch_init, or by the first call on that device).
 * Every call on a GPU shares that GPU's array and leaves its contents there;
 * each call rebuilds what it reads before reading it, so nothing needs
 * clearing, but two calls whose work overlaps on one GPU (different streams,
 * or a graph replayed while another call runs) race on the array and give
 * undefined estimates: serialise them.  Results are bit-identical to
 * pusch_noise_est on the same inputs.
 *   Yp, pilots, sigma2 and the limits as pusch_noise_est, plus
 *   batch <= PUSCH_NOISE_EST_STATIC_MAX_BATCH (PUSCH_EUNSUPPORTED beyond it).
 */
#define PUSCH_NOISE_EST_STATIC_MAX_BATCH 1024
int pusch_noise_est_static(const pusch_c32* Yp, const pusch_c32* pilots, float* sigma2, int n_beams, int n_ue,
                           int n_sc, int n_pilot, long long batch, void* stream);

/*
 * MMSE MIMO detection (Eq. 2) per subcarrier: G = H^H H + sigma2 I, the
 * Cholesky factor G = L L^H (Crout order, Sec. V-C), then for every data
 * symbol the matched filter b = H^H y, forward substitution L z = b and back
 * substitution L^H x = z.  One factorisation per subcarrier serves all data
 * symbols of the call.  With more than 16 UEs and n_ue > n_beams / 2 (Gram
 * matrices of condition numbers 1e3..1e5 at high SNR) one step of iterative
 * refinement follows, as the slot option refine describes.
 *   H      [batch][n_sc][n_ue][n_beams] as written by pusch_chest.
 *   Yd     [batch][n_data][n_sc][n_beams] RE-major data symbols.
 *   Xhat   [batch][n_data][n_sc][n_ue] detected symbols (0 where status = 1).
 *   status [batch][n_sc] int32 or NULL: 0 ok, 1 when a Cholesky pivot is not
 *          positive and finite.
 *   sigma2 >= 0 and finite.  1 <= n_ue <= min(PUSCH_MAX_UES, n_beams),
 *   1 <= n_beams <= PUSCH_MAX_BEAMS, n_sc >= 0, n_data >= 1, batch >= 0.
 */
int pusch_mmse_solve(const pusch_c32* H, const pusch_c32* Yd, float sigma2, pusch_c32* Xhat, int n_beams,
                     int n_ue, int n_sc, int n_data, long long batch, int32_t* status, void* stream);

/* One slot's geometry for pusch_slot (Sec. II use-case parameters). */
typedef struct {
  int n_ant;                        /* N_R receive antennas, 1..1024 */
  int n_fft;                        /* FFT size, as pusch_fft */
  int n_sc;                         /* active subcarriers, n_ue..n_fft */
  int n_symb;                       /* OFDM symbols per slot, 2..PUSCH_MAX_SYMBOLS */
  int n_beams;                      /* N_B, 1..PUSCH_MAX_BEAMS */
  int n_ue;                         /* N_L, 1..min(PUSCH_MAX_UES, n_beams) */
  int n_pilot;                      /* pilot symbols, 1..min(PUSCH_MAX_PILOTS, n_symb - 1) */
  int pilot_symb[PUSCH_MAX_PILOTS]; /* 0-based pilot symbol indices, strictly ascending */
  float sigma2;                     /* noise variance per RE after beamforming, >= 0 (unless noise_est) */
  const pusch_c32* W;               /* device [n_beams][n_ant], or NULL = built-in DFT rows */
  const pusch_c32* pilots;          /* device [n_slot][n_pilot][n_sc] */
  int noise_est;                    /* nonzero: estimate each slot's noise variance from its pilot
                                       symbols (as pusch_noise_est) and use it instead of sigma2;
                                       needs n_sc >= 2 n_ue */
  float* sigma2_est;                /* device [n_slot]: receives the estimates when noise_est is set,
                                       or NULL; must not overlap any other buffer of the call */
  int refine;                       /* nonzero: one step of iterative refinement of the MIMO solve
                                       (residual H^H (y - H x) - sigma2 x from the channel estimate
                                       and the data symbols, solved with the same Cholesky factor;
                                       the residual in FP64 for a subcarrier whose condition
                                       estimate ||G||_F ||G^-1||_F (the latter from +-1 probe
                                       vectors) exceeds 1e4, FP32 otherwise);
                                       for ill-conditioned Gram matrices (n_ue close to n_beams), where
                                       the 32-bit arithmetic of Sec. VI alone loses accuracy.
                                       Uses a stored channel estimate (larger workspace).  With more
                                       than 16 UEs and n_ue > n_beams / 2 the detection refines even
                                       when this is 0 */
  int time_varying;                 /* nonzero: a channel that changes over the slot -- each pilot
                                       symbol gives its own estimate (from its own comb positions),
                                       data symbol s uses their linear interpolation in s between the
                                       pilot symbols around it (held before the first and after the
                                       last), and the MIMO stage factors one Gram matrix per data
                                       symbol (the paper counts the Cholesky decomposition per data
                                       symbol, Sec. II).  Needs n_ue <= 16, an even n_beams and no
                                       refine (PUSCH_EUNSUPPORTED otherwise) */
  int comb_aligned;                 /* nonzero: the pilot comb without stagger -- every pilot symbol
                                       puts UE l's pilots on the subcarriers k = l mod n_ue (instead
                                       of k + j * (n_ue / n_pilot) = l mod n_ue).  The channel
                                       estimate then averages the pilot symbols at each position
                                       (half the positions of the staggered comb for two pilot
                                       symbols), and the noise estimate compares each pilot RE with
                                       the mean at its own subcarrier, so it holds noise only on any
                                       channel that is static over the slot; with the staggered comb
                                       the noise estimate predicts from neighbouring positions and
                                       counts the channel's variation between them as noise.
                                       pusch_slot_denoised: 0 only (PUSCH_EUNSUPPORTED otherwise) */
  int fft_mfma;                     /* nonzero: OFDM demodulation with every radix-16 butterfly on the
                                       matrix cores -- each pass of the 4096-point Stockham FFT is
                                       the 16 x 16 DFT matrix times the butterflies' inputs, with
                                       FP16 (pusch_slot_mixed) or BF16 (pusch_slot_bf16) operands
                                       rounded as they enter each pass and FP32 accumulation.  Only
                                       for those two entry points with n_fft = 4096
                                       (PUSCH_EUNSUPPORTED otherwise, and in pusch_cells and
                                       pusch_slot_denoised) */
} pusch_slot_desc;

/* Bytes of device workspace pusch_slot needs for n_slot slots (0 on bad input). */
size_t pusch_slot_workspace_bytes(const pusch_slot_desc* d, long long n_slot);
/* (Depends on the geometry fields and refine; W, pilots, sigma2, noise_est and sigma2_est are not read.) */

/*
 * The fused receive chain (Sec. II, Fig. "PUSCH processing chain") for n_slot
 * independent slots, enqueued on one stream: OFDM demodulation of every
 * antenna and symbol to the n_sc active subcarriers, beamforming, LS channel
 * estimation on the pilot symbols, optionally noise estimation (noise_est),
 * MMSE detection of every other ("data") symbol in ascending symbol order.  With n_ue <= 16 and an even n_beams the
 * channel estimate is computed inside the detection kernel and never stored.
 *   x_td   [n_slot][n_symb][n_ant][n_fft] time-domain samples.
 *   x_hat  [n_slot][n_data][n_sc][n_ue], n_data = n_symb - n_pilot.
 *   status [n_slot][n_sc] int32 or NULL, as pusch_mmse_solve.
 *   ws     device workspace of at least pusch_slot_workspace_bytes(d, n_slot)
 *          bytes, 256-byte aligned, not overlapping any other argument.
 */
int pusch_slot(const pusch_slot_desc* d, long long n_slot, const pusch_c32* x_td, pusch_c32* x_hat, int32_t* status,
               void* ws, size_t ws_bytes, void* stream);

/*
 * The same chain with the active-bin grids between OFDM demodulation and
 * beamforming stored in FP16 instead of FP32 (the paper's chain works on
 * 32-bit words, Sec. VI; this is a reduced-precision form of it): every
 * antenna row of every symbol is scaled by a power of two chosen from its
 * time-domain L1 norm, which bounds every output bin, so nothing overflows;
 * beamforming runs on FP16 matrix cores with FP32 accumulation (W rounded
 * to FP16, the rows rebased to each symbol's smallest exponent, the common
 * scale undone in FP32).  Channel estimation and detection stay FP32.  The
 * extra error is the FP16 rounding of the grids and of W (relative 2^-11 per
 * value).  It halves the bytes those grids move through HBM and takes the
 * beamforming product off the FP32 pipes.  Arguments and results as
 * pusch_slot; n_ant <= 64 (PUSCH_EUNSUPPORTED otherwise).
 */
size_t pusch_slot_mixed_workspace_bytes(const pusch_slot_desc* d, long long n_slot);
int pusch_slot_mixed(const pusch_slot_desc* d, long long n_slot, const pusch_c32* x_td, pusch_c32* x_hat,
                     int32_t* status, void* ws, size_t ws_bytes, void* stream);

/*
 * The same reduced-precision form with bfloat16 in place of FP16 (Sec. VI's
 * 32-bit words narrowed the other way: 8 significant bits, FP32's exponent
 * range): the active-bin grids are stored as bfloat16 pairs rounded to
 * nearest even, with no row scaling, and beamforming runs on BF16 matrix
 * cores with FP32 accumulation (W rounded to BF16).  The extra error is
 * relative 2^-9 per grid value and W entry.  Arguments, results, workspace
 * size and limits as pusch_slot_mixed.
 */
size_t pusch_slot_bf16_workspace_bytes(const pusch_slot_desc* d, long long n_slot);
int pusch_slot_bf16(const pusch_slot_desc* d, long long n_slot, const pusch_c32* x_td, pusch_c32* x_hat,
                    int32_t* status, void* ws, size_t ws_bytes, void* stream);

/*
 * Many independent cells of different geometries in one call (the paper runs
 * many independent small problems side by side, each on its own group of
 * cores between barriers: Sec. V, Sec. VI).  Cell c is a pusch_slot call
 * (pusch_slot_mixed with PUSCH_CELLS_MIXED) with descriptor d[c], n_slot[c]
 * slots and buffers x_td[c], x_hat[c], status[c] (status may be NULL, or any
 * status[c] may be NULL); results are those of that call, bit for bit.
 *
 * Launches.  The cells that detect with the channel interpolated inside the
 * detection kernel (up to 16 UEs, an even number of beams, no refinement, one
 * estimate per slot) and have up to 64 antennas run grouped: one launch per
 * stage for all such cells of one kernel shape (transform size; beamforming
 * tile class; detection class), on `stream`.  Every other cell (and every
 * cell with PUSCH_CELLS_STREAMS) runs as its own launches on
 * PUSCH_CELL_STREAMS library-owned side streams of default priority, the i-th
 * such cell on side stream i mod PUSCH_CELL_STREAMS, forked from and joined
 * back to `stream` with events.  The whole call is ordered on `stream` and can
 * be captured into a HIP graph (after one uncaptured call with the same cells
 * has built the device tables).
 *   ws     device workspace of at least pusch_cells_workspace_bytes bytes,
 *          256-byte aligned: one slice per cell, in cell order, each that
 *          cell's pusch_slot (or pusch_slot_mixed) workspace rounded up to
 *          256 bytes.
 *   flags  PUSCH_CELLS_MIXED: every cell runs as pusch_slot_mixed (each cell
 *          n_ant <= 64, else PUSCH_EUNSUPPORTED; workspace size 0);
 *          PUSCH_CELLS_STREAMS: no grouped launches;
 *          PUSCH_CELLS_WITH_PLAN(p): the grouped cells run launch plan p
 *          (below) instead of the one recorded for the cell set.
 *          Other bits: PUSCH_EINVAL.
 * Every cell's arguments are checked as for pusch_slot, and no cell's output
 * may overlap any other cell's buffers or the workspace.  1 <= n_cells <=
 * PUSCH_MAX_CELLS.  Calls on one device are serialised on the host while
 * they enqueue; a capture that includes a call holds the side streams until
 * it ends.
 */
#define PUSCH_CELL_STREAMS 4
#define PUSCH_MAX_CELLS 4096
#define PUSCH_CELLS_MIXED 1
#define PUSCH_CELLS_STREAMS 2
#define PUSCH_CELLS_WITH_PLAN(p) (4 | ((p) << 3)) /* 0 <= p < PUSCH_CELLS_PLANS */
size_t pusch_cells_workspace_bytes(const pusch_slot_desc* d, int n_cells, const long long* n_slot, int flags);
int pusch_cells(const pusch_slot_desc* d, int n_cells, const long long* n_slot, const pusch_c32* const* x_td,
                pusch_c32* const* x_hat, int32_t* const* status, void* ws, size_t ws_bytes, int flags,
                void* stream);

/*
 * Launch plan of the grouped cells: per stage, one launch for all kernel
 * shapes of the call (a kernel that runs each workgroup's shape: one ramp
 * and one tail, but the largest shape's registers and LDS for every
 * workgroup) or one launch per shape (each shape's own kernel, launched one
 * after another).  Plan p of PUSCH_CELLS_PLANS has fft_merged = p & 1,
 * bf_merged = (p >> 1) & 1, mmse_merged = (p >> 2) & 1.  Results do not
 * depend on the plan (every tile runs the same arithmetic).  A cell set that
 * pusch_cells_tune has not timed runs {1, 0, 1}.
 */
typedef struct pusch_cells_plan {
  int fft_merged;   /* one FFT launch for every transform size */
  int bf_merged;    /* one beamforming launch for every tile class (n_beams, n_ant) */
  int mmse_merged;  /* one detection launch for every class (n_beams, taps) */
} pusch_cells_plan;
#define PUSCH_CELLS_PLANS 8

/*
 * Autotuner of pusch_cells: runs the call (same arguments) once and then
 * `reps` times under every plan, timing each call with events on `stream`
 * (the host waits for each), and records the plan with the smallest median
 * time for this cell set (the geometries, slot counts, options and flags of
 * every cell) on the current device; later pusch_cells calls with the same
 * cell set use it.  Writes the plan to *chosen (if not NULL) and the median
 * time of plan p in microseconds to us[p] for p < n_us.  x_hat and status
 * hold the results of the last call.  1 <= reps <= 1000.  Not for capture
 * into a graph (it synchronises); creates and destroys two events.
 */
int pusch_cells_tune(const pusch_slot_desc* d, int n_cells, const long long* n_slot, const pusch_c32* const* x_td,
                     pusch_c32* const* x_hat, int32_t* const* status, void* ws, size_t ws_bytes, int flags, int reps,
                     pusch_cells_plan* chosen, float* us, int n_us, void* stream);
/* The plan pusch_cells would use for this cell set: returns 1 if tuned, 0 for
 * the default plan, or a negative code. */
int pusch_cells_plan_get(const pusch_slot_desc* d, int n_cells, const long long* n_slot, int flags,
                         pusch_cells_plan* plan);

/*
 * Learned refinement of the LS channel estimate (the paper's estimator is LS
 * on the pilot symbols, Sec. II, CHE; Table 1, row "CHE").  For every (UE,
 * beam) pair the LS estimate over the n_symb x n_sc grid (a complex grid: real
 * and imaginary parts are two channels) passes four 3x3 convolution layers,
 * 2 -> 32 -> 32 -> 32 -> 2 channels with ReLU after the first three, and the
 * result is added to the LS estimate.  Convolutions are cross-correlations
 * over (symbol, subcarrier) with zero padding.  The kernels run on bfloat16
 * matrix cores with FP32 accumulation: weights, the network input, the hidden
 * activations and the gradients entering the transposed convolutions are
 * rounded to bfloat16 (nearest, ties to even); biases, the residual addition,
 * weight gradients and the optimiser are FP32.
 *
 * Parameters: PUSCH_DN_PARAMS FP32 values (device), layer by layer
 * W[c_out][3][3][c_in] (c_in fastest) then b[c_out].
 * Grids: complex [n_grid][n_symb][n_sc] (subcarrier fastest).
 *   1 <= n_symb <= PUSCH_MAX_SYMBOLS, 1 <= n_sc <= 4096, n_grid >= 0.
 * ws: device workspace of at least pusch_dn_workspace_bytes(n_symb, n_sc,
 * n_grid) bytes, 256-byte aligned; pusch_dn_forward needs only its first part
 * (the hidden activations) but a smaller buffer is accepted only when it is
 * at least that part; pusch_dn_backward reads the activations the last
 * forward pass over the same grids left there.
 */
#define PUSCH_DN_PARAMS 19682
size_t pusch_dn_workspace_bytes(int n_symb, int n_sc, long long n_grid);
/* LS estimate on every symbol of every (UE, beam) pair: per pilot symbol from
 * that symbol's comb positions of the UE, linear along the subcarriers with
 * the end values held, then linear in time between the pilot symbols around
 * each symbol (held before the first and after the last).
 *   Yp [batch][n_pilot][n_sc][n_beams] RE-major received pilot symbols,
 *   pilots [batch][n_pilot][n_sc], pilot_symb: n_pilot host ints (the pilot
 *   symbols' indices among the n_symb, ascending),
 *   grid [batch][n_ue][n_beams][n_symb][n_sc]. */
int pusch_dn_ls_grid(const pusch_c32* Yp, const pusch_c32* pilots, pusch_c32* grid, int n_beams, int n_ue, int n_sc,
                     int n_symb, int n_pilot, const int* pilot_symb, long long batch, void* stream);
/* out = grid + sigma net(grid / sigma): the network on the grid in units of
 * sigma > 0 (the noise standard deviation of the LS values, as the network is
 * trained), its correction scaled back; sigma = 1 is the plain network.  out
 * must not overlap grid. */
int pusch_dn_forward(const float* params, const pusch_c32* grid, pusch_c32* out, float sigma, int n_symb, int n_sc,
                     long long n_grid, void* ws, size_t ws_bytes, void* stream);
/* grads[PUSCH_DN_PARAMS] = dL/dparams from dout = dL/d(out) (real part: the
 * derivative with respect to the output's real part, imaginary: imaginary),
 * after pusch_dn_forward(params, grid, ...) on the same ws.  Weight gradients
 * are summed in a fixed order (bit-reproducible).  The gradients are those of
 * the plain network (sigma = 1 in the forward pass).  n_grid >= 1. */
int pusch_dn_backward(const float* params, const pusch_c32* grid, const pusch_c32* dout, float* grads, int n_symb,
                      int n_sc, long long n_grid, void* ws, size_t ws_bytes, void* stream);
/* loss[0] = mean over all complex entries of w_g |out - target|^2, and
 * dout = 2 w_g (out - target) / (n_grid n_symb n_sc), with w_g = weights[g]
 * for the entries of grid g (weights: n_grid FP32 on the device, or NULL for
 * all 1).  n_grid >= 1. */
int pusch_dn_loss(const pusch_c32* out, const pusch_c32* target, const float* weights, pusch_c32* dout, float* loss,
                  int n_symb, int n_sc, long long n_grid, void* ws, size_t ws_bytes, void* stream);
/* One Adam step (Kingma and Ba) on the FP32 parameters, in place: m and v
 * (PUSCH_DN_PARAMS each, zero before step 1) are the moment estimates, step
 * >= 1 the step number (for the bias correction 1 - beta^step). */
int pusch_dn_adam(float* params, const float* grads, float* m, float* v, int step, float lr, float beta1, float beta2,
                  float eps, void* stream);

/*
 * The receive chain with the denoised channel estimate and the LS fallback.
 * OFDM demodulation and beamforming as pusch_slot; the LS estimate on every
 * symbol (as pusch_dn_ls_grid) and its denoised form (params, run as
 * pusch_dn_forward with sigma = sqrt(sigma2): the LS values' noise standard
 * deviation after a unitary beamformer and unit-power pilots); every data
 * symbol detected (Eq. 2) with each estimate of that symbol; then, per slot,
 * the fallback test: the post-MMSE residual sum |y - H_hat x_hat|^2 over the
 * slot's data REs and beams is formed for both estimates (neither has seen
 * those REs, so it grows with the estimation error), and the denoised
 * result is kept unless its residual exceeds the LS one, in which case the
 * slot falls back to plain LS.
 *   Arguments as pusch_slot; dn_params: PUSCH_DN_PARAMS FP32 (device);
 *   used_dn [n_slot] int32 (device) or NULL: 1 where the denoised estimate was
 *   used, 0 where the slot fell back to LS; status: the flags of the result
 *   kept.  sigma2 > 0 given (noise_est 0; PUSCH_EINVAL for sigma2 = 0),
 *   refine 0 and time_varying 0, else PUSCH_EUNSUPPORTED.
 */
size_t pusch_slot_denoised_workspace_bytes(const pusch_slot_desc* d, long long n_slot);
int pusch_slot_denoised(const pusch_slot_desc* d, long long n_slot, const pusch_c32* x_td, const float* dn_params,
                        pusch_c32* x_hat, int32_t* status, int32_t* used_dn, void* ws, size_t ws_bytes, void* stream);

/*
 * Stage timing for measurement.  pusch_profile_begin(max_calls) creates
 * HIP events (allocation happens here, not in pusch_slot); while active, each
 * pusch_slot call (not the cells of pusch_cells) records an event before and after each of its
 * PUSCH_SLOT_STAGES launches on its stream, for up to max_calls calls.
 * pusch_profile_end(stage_ms, n) synchronises on the last event, writes the
 * summed device time of each stage (ms; order: fft, beamform, chest = channel
 * and noise estimation, mmse) into stage_ms[0..n-1], releases the events and
 * returns the number of calls recorded (or a negative code).
 */
#define PUSCH_SLOT_STAGES 4
int pusch_profile_begin(int max_calls);
int pusch_profile_end(float* stage_ms, int n);

#ifdef __cplusplus
}
#endif

#endif /* PUSCH_H_ */
