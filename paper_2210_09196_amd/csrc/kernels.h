// Internal interface between the C-ABI host code (api.hip) and the gfx950
// kernels of the PUSCH receive chain.  Not installed; include/pusch.h is the
// public boundary.
#pragma once

#include <hip/hip_runtime.h>

namespace pusch {

// Interleaved FP32 complex, byte-compatible with pusch_c32 / torch.complex64.
struct cf {
  float r, i;
};

constexpr int kMaxSymbols = 16;
constexpr int kMaxPilots = 4;

// ---------------------------------------------------------------- FFT
// Offsets (in cf elements) of each FFT size's twiddle block inside the
// per-device table, and the table length.  Filled by fft_twiddle_layout().
struct TwiddleLayout {
  int offset[5];  // for n_fft = 64, 256, 1024, 2048, 4096
  int total;
};
TwiddleLayout fft_twiddle_layout();
// Writes the FP32 twiddle table (computed in FP64 on the host) into `host`
// (length fft_twiddle_layout().total).
void fft_fill_twiddles(cf* host);
int fft_size_index(int n_fft);  // 0..4, or -1 if unsupported

// X_i[(f + shift) mod n_fft] = DFT(x_i)[f] for the targets below out_len;
// output rows ldo elements apart (>= out_len).  With Xh set, the rows are
// written as FP16 pairs (half2 words, re low) scaled by 2^e per row instead
// (X unused): transform i = g * rows + a (rows <= 64) stores e in
// ex[g * 64 + (a % 4) * 16 + a / 4].  With Xh set and ex null, the rows are
// bfloat16 pairs (re low), rounded to nearest even and not scaled.
hipError_t launch_fft(const cf* x, cf* X, int n_fft, long long batch, int out_len, int shift, long long ldo,
                      const cf* twiddles, int n_cu, hipStream_t s, unsigned* Xh = nullptr,
                      signed char* ex = nullptr, int rows = 0);
// The same outputs in the 4-byte forms (Xh required: FP16 with ex, bfloat16
// without) with every radix-16 butterfly on the matrix cores (FP16 or BF16
// operands, FP32 accumulation); n_fft = 4096 only.
hipError_t launch_fft_mfma(const cf* x, int n_fft, long long batch, int out_len, int shift, long long ldo,
                           const cf* twiddles, int n_cu, hipStream_t s, unsigned* Xh, signed char* ex, int rows);

// Workgroups of a grouped persistent launch.  Cell c needs rounds(c)
// workgroup-rounds of work (its items over what one workgroup takes per
// round), each lasting about cost(c).  The launch lasts as long as its slowest
// cell, so the counts are chosen for the smallest time T with
// sum_c ceil(rounds(c) / floor(T / cost(c))) <= cap (the resident
// workgroups): no workgroup waits for a second wave, and every cell finishes
// within T.  (Shares rounded up from a proportional split can exceed cap by a
// few workgroups, which then run after everything else and double the launch
// time.)  Fills start[0..n] and returns start[n] (n when n > cap).
template <class Rounds, class Cost>
inline int share_work(int n, Rounds rounds, Cost cost, long long cap, int* start) {
  auto blocks_at = [&](long long T, int c) {
    const long long per = T / cost(c);  // rounds one workgroup of cell c fits in T
    if (per < 1) return rounds(c) + cap + 1;  // does not fit
    const long long k = (rounds(c) + per - 1) / per;
    return k < 1 ? 1ll : k;
  };
  auto total_at = [&](long long T) {
    long long b = 0;
    for (int c = 0; c < n; ++c) b += blocks_at(T, c);
    return b;
  };
  long long hi = 1, work = 0;
  for (int c = 0; c < n; ++c) {
    const long long w = rounds(c) * cost(c);
    hi = w > hi ? w : hi;  // one workgroup per cell
    work += w;
  }
  long long lo = work / (cap > 0 ? cap : 1);
  lo = lo < 1 ? 1 : (lo > hi ? hi : lo);
  while (lo < hi) {  // smallest T in [lo, hi] that fits (T = hi: one workgroup per cell)
    const long long mid = lo + (hi - lo) / 2;
    if (total_at(mid) <= cap) hi = mid;
    else lo = mid + 1;
  }
  int at = 0;
  for (int c = 0; c < n; ++c) {
    start[c] = at;
    const long long k = blocks_at(lo, c);
    at += (int)(k > rounds(c) ? (rounds(c) < 1 ? 1 : rounds(c)) : k);
  }
  start[n] = at;
  return at;
}

// Many cells of any FFT sizes in one launch (the grouped form of
// pusch_cells): the per-cell arguments of launch_fft (with X or Xh/ex/rows),
// up to kFftCellsPerLaunch cells; tw and start[] are filled by the launcher.
constexpr int kFftCellsPerLaunch = 48;
struct FftCell {
  const cf* x;
  cf* X;
  unsigned* Xh;
  signed char* ex;
  const cf* tw;  // filled by the launcher
  long long batch, ldo;
  int n_fft, rows, out_len, shift;
};
struct FftCells {
  FftCell cell[kFftCellsPerLaunch];
  int start[kFftCellsPerLaunch + 1];
  int n;
};
hipError_t launch_fft_cells(FftCells& t, bool h16, const cf* twiddles, int n_cu, hipStream_t s);

// ---------------------------------------------------------------- beamforming
// Optional beamforming epilogue of the fused slot: the outputs of pilot
// symbols are multiplied by conj(p)/|p|^2 (the LS division), batch item
// i = slot * n_symb + symbol.
struct PilotScale {
  const cf* pilots;                 // [n_slot][n_pilot][n_re], nullptr = no epilogue
  long long p_slot;                 // pilots elements between slots
  int n_symb;
  signed char pilot_of[kMaxSymbols];  // pilot index of each symbol, or -1
};
// Y_i[n][b] = sum_a W[b][a] X_i[a][n]; X_i = X + i*sx (row pitch ldx),
// Y_i = Y + i*sy (RE-major, n_beams values per RE).  With Xh set, X is read
// instead as FP16 pairs (half2 words, pitches in words) with row a of batch
// item i scaled by 2^e, e from launch_fft's exponent table (rows = n_ant),
// and the product runs on FP16 matrix cores with FP32 accumulation (W
// rounded to FP16); up to 64 antennas.  With Xh set and ex null, X is read
// as bfloat16 pairs (no scales) and the product runs on BF16 matrix cores (W
// rounded to BF16).
hipError_t launch_beamform(const cf* W, const cf* X, cf* Y, int n_beams, int n_ant, int n_re, long long ldx,
                           long long sx, long long sy, long long batch, int n_cu, hipStream_t s,
                           const PilotScale* pilot_scale = nullptr, const unsigned* Xh = nullptr,
                           const signed char* ex = nullptr);
// Many cells of one beamforming tile shape in one launch (the grouped form of
// pusch_cells): per cell the arguments of launch_beamform with up to 64
// antennas (the register-tile kernels); W must be a device table; the FP16
// form reads Xh/ex.  cls >= 0: every cell of the launch has that
// bf_cell_class(n_beams, n_ant) (the class's own kernel); cls = -1: any
// classes, one kernel that runs each workgroup's class.  ntn, ntiles, cls
// and start[] are filled by the launcher.
constexpr int kBfCellsPerLaunch = 24;
struct BfCell {
  const cf* W;
  const cf* X;
  const unsigned* Xh;
  const signed char* ex;
  cf* Y;
  long long ldx, sx, sy, batch;
  int nb, na, nre, ntiles, ntn, cls;
  PilotScale ps;
};
struct BfCells {
  BfCell cell[kBfCellsPerLaunch];
  int start[kBfCellsPerLaunch + 1];
  int n;
};
int bf_cell_class(int n_beams, int n_ant);  // -1 when the register-tile kernels do not apply
hipError_t launch_beamform_cells(BfCells& t, int cls, bool h16, int n_cu, hipStream_t s);


// ---------------------------------------------------------------- LS channel estimation
// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// id.  xcd_block(b, n) renumbers them so that XCD x gets one contiguous run of
// the n logical blocks: neighbouring blocks, which share input lines, then
// share an L2.  A bijection of [0, n) for any n.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int n) {
  const int per = n / kXcds, rem = n % kXcds;
  const int x = b % kXcds, local = b / kXcds;
  return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

struct ChestGeom {
  long long y_batch;              // Y elements between batch items
  long long y_sym;                // Y elements between the RE-major symbol grids [n_sc][n_beams]
  long long p_batch;              // pilots elements between batch items ([n_pilot][n_sc] each)
  long long h_batch;              // H elements between batch items ([n_sc][n_ue][n_beams] each)
  int pilot_sym[kMaxPilots];      // grid index of pilot symbol j (grid at pilot_sym[j] * y_sym)
  int n_beams, n_ue, n_sc, n_pilot;
  int comb_aligned;               // nonzero: the comb without stagger (comb_step 0)
};
// Pilot comb: on pilot symbol j, subcarrier k carries UE (k + j * step) mod
// n_ue's pilot, step = n_ue / n_pilot (staggered) or 0 (aligned).
__host__ __device__ inline int comb_step(const ChestGeom& g) { return g.comb_aligned ? 0 : g.n_ue / g.n_pilot; }
hipError_t launch_chest(const cf* Y, const cf* pilots, cf* H, const ChestGeom& g, long long batch, hipStream_t s);
// Channel interpolation of the fused detection as taps: the estimate of UE l
// at subcarrier k, beam b, is sum_t w_t * LS[off_t + b] over the n_tap taps
// of (k, l), LS being one batch item of the RE-major grids that hold per-RE
// LS values, off_t an element offset into it (pilot grid of the pilot symbol
// plus position * n_beams).  tab[(k * n_ue + l) * n_tap + t] = {off_t, bits
// of w_t}; unused taps repeat the first offset with weight 0.  Depends on the
// geometry only (n_sc, n_ue, n_pilot, n_beams, the pilot grid offsets).
int comb_taps(int n_ue, int n_pilot, bool aligned = false);  // taps per (k, l) the geometry needs: 2 or 8
hipError_t launch_comb_taps(int2* tab, const ChestGeom& g, int n_tap, hipStream_t s);
// Time-varying channel: 4 taps per (data symbol, k, l) (two frequency
// neighbours on each of two pilot symbols; unused taps weight 0),
// tab[((d * n_sc + k) * n_ue + l) * kTimeTaps + t]: UE l's estimate from each of the
// two pilot symbols around data symbol d (from that symbol's own positions),
// weighted linearly in time; held before the first and after the last pilot
// symbol.  data_sym: the symbol index of each data symbol.
struct TimeTapGeom {
  int data_sym[kMaxSymbols];
  int n_data;
};
constexpr int kTimeTaps = 4;
hipError_t launch_time_taps(int2* tab, const ChestGeom& g, const TimeTapGeom& t, hipStream_t s);
// Two pilot symbols: per (k, l) the 2 + 2 frequency taps of each pilot
// symbol's own estimate, tab[(k * n_ue + l) * 4 + 2 j + {0, 1}] (offset as
// for launch_comb_taps, weight), for launch_mmse_tv.
hipError_t launch_pair_taps(int2* tab, const ChestGeom& g, hipStream_t s);

// ---------------------------------------------------------------- noise estimation
// Noise variance of every batch item from its pilot symbols (grids at
// pilot_sym[j] * y_sym as for launch_chest): each pilot RE against the
// prediction of its UE's channel interpolated from the UE's other pilot
// positions, normalised by the noise gain of that prediction.  ls: the pilot
// grids already hold LS values y*conj(p)/|p|^2 (PilotScale epilogue) instead
// of received values.  tab: the geometry's neighbour table from
// launch_noise_table (noise_table_bytes(n_pilot, n_sc) bytes, 16-byte
// aligned; depends on n_sc, n_ue and n_pilot only); part: kNeParts float2 per
// batch item (scratch); sigma2: [batch].  Requires n_sc >= 2 * n_ue and
// n_sc <= 4096.
constexpr int kNeParts = 256;
size_t noise_table_bytes(int n_pilot, int n_sc);
hipError_t launch_noise_table(int4* tab, const ChestGeom& g, hipStream_t s);
hipError_t launch_noise_est(const cf* Y, const cf* pilots, bool ls, const int4* tab, float2* part, float* sigma2,
                            const ChestGeom& g, long long batch, hipStream_t s);

// ---------------------------------------------------------------- MMSE detection
struct MmseGeom {
  long long h_batch;          // H elements between batch items
  long long y_batch;          // Y elements between batch items
  long long y_sym;            // Y elements between the RE-major symbol grids [n_sc][n_beams]
  long long x_batch;          // Xhat elements between batch items ([n_data][n_sc][n_ue] block)
  long long st_batch;         // status elements between batch items
  int d_first;                // grid index of the call's first data symbol before skipping
  int n_skip;                 // grids that hold pilot symbols, ascending (skipped when
  int skip[kMaxPilots];       //   counting data symbols)
  int n_beams, n_ue, n_sc, n_data;
  float sigma2;
  const float* sigma2_item;   // device [batch] noise variance per batch item, or nullptr = sigma2
  int refine;                 // nonzero: one step of iterative refinement (stored-estimate path only;
                              //   launch_mmse also refines when mmse_auto_refine)
  int st_or;                  // nonzero: OR the status flags into st instead of writing them
};
hipError_t launch_mmse(const cf* H, const cf* Y, cf* Xhat, int* status, const MmseGeom& g, long long batch,
                       hipStream_t s);
// Same detection, with the channel interpolated on the fly from pilot
// symbols of Y that already hold LS values y*conj(p)/|p|^2 (PilotScale
// epilogue; grid offsets in cg as for launch_chest), using the taps of
// launch_comb_taps, instead of read from a stored estimate.  Requires
// mmse_fusable(n_ue, n_beams, y_batch).
bool mmse_fusable(int n_ue, int n_beams, long long y_batch);
// Beyond 16 UEs with more than half as many UEs as beams the detection
// refines its solve without being asked (the Gram matrices are ill-conditioned).
bool mmse_auto_refine(int n_ue, int n_beams);
hipError_t launch_mmse_fused(const cf* Y, const int2* taps, int n_tap, const ChestGeom& cg, cf* Xhat, int* status,
                             const MmseGeom& g, long long batch, hipStream_t s);
// Many cells' fused detections in one launch (the grouped form of
// pusch_cells): per cell the arguments of launch_mmse_fused (a batch of
// `batch` items, n_tap interpolation taps).  cls >= 0: every cell has that
// mmse_cell_class(n_beams, n_tap) (the class's own kernel; -1 from
// mmse_cell_class: no grouped kernel); cls = -1: any classes, one kernel.
// nblk_batch, cls and start[] are filled by the launcher.
// Time-varying channel with two pilot symbols in one launch: data symbol d's
// estimate is (1 - a_d) H_0 + a_d H_1, a_d = (s_d - p_0) / (p_1 - p_0)
// clamped to [0, 1] (s_d its symbol index, p_j the pilot symbols' indices;
// H_j from pilot symbol j alone, taps of launch_pair_taps), its Gram matrix is formed from H_0^H H_0,
// H_1^H H_1 and (H_0 + H_1)^H (H_0 + H_1), and each data symbol is factored
// and solved on its own; status flags OR over the data symbols (st_or as for
// launch_mmse).  Needs two pilot symbols, 1 <= g.n_data <= 16 and
// mmse_fusable(n_ue, n_beams, cg.y_batch); grids as for launch_mmse_fused.
hipError_t launch_mmse_tv(const cf* Y, const int2* taps, const ChestGeom& cg, cf* Xhat, int* status,
                          const MmseGeom& g, long long batch, hipStream_t s);

constexpr int kMmseCellsPerLaunch = 16;
struct MmseCell {
  const cf* Y;
  const int2* taps;
  cf* Xh;
  int* st;
  long long batch;
  MmseGeom g;
  ChestGeom cg;
  int n_tap, nblk_batch, cls;
};
struct MmseCells {
  MmseCell cell[kMmseCellsPerLaunch];
  int start[kMmseCellsPerLaunch + 1];
  int n;
};
int mmse_cell_class(int n_beams, int n_tap);
hipError_t launch_mmse_cells(MmseCells& t, int cls, hipStream_t s);
// kernel arguments stay within 4 KB
static_assert(sizeof(MmseCells) <= 4096, "grouped detection arguments");
static_assert(sizeof(BfCells) <= 4096, "grouped beamforming arguments");
static_assert(sizeof(FftCells) <= 4096, "grouped FFT arguments");

// ---------------------------------------------------------------- LS-estimate denoiser
// Four 3x3 convolution layers 2 -> 32 -> 32 -> 32 -> 2 over every [S][K] grid
// (complex values = two channels), ReLU after the first three, output added
// to the input.  Parameters: one FP32 vector, per layer W[c_out][3][3][c_in]
// then b[c_out].  Hidden activations are bfloat16 [position][32].
constexpr int kDnW1 = 32 * 9 * 2, kDnW2 = 32 * 9 * 32, kDnW4 = 2 * 9 * 32;
constexpr int kDnParams = (kDnW1 + 32) + 2 * (kDnW2 + 32) + (kDnW4 + 2);
constexpr int kDnWgradBlocks = 1024;  // workgroups (and partial sums) of one weight-gradient pass
int dn_wgrad_blocks(int n_cu);
// Workspace of n_grid grids: the three hidden activations (written by the
// forward pass, read by the backward pass), two FP32 gradient buffers, the
// weight-gradient partial sums and the loss partial sums (byte offsets).
struct DnLayout {
  long long off_act[3], off_dz[2], off_part, off_loss, total, fwd_total;
};
DnLayout dn_layout(int n_symb, int n_sc, long long n_grid, int n_cu);
// out = grid + sigma f(grid / sigma): the network on the grid in units of sigma
// (the noise standard deviation when the network was trained so), its
// correction scaled back; sigma = 1 is the plain network.
hipError_t launch_dn_forward(const float* params, const cf* grid, cf* out, int S, int K, long long n_grid, char* ws,
                             const DnLayout& lay, int n_cu, hipStream_t s, float sigma = 1.f);
// Gradients of a loss with respect to the parameters, from dL/d(out) and the
// activations the last forward pass (with sigma = 1) over the same grids left in ws.
hipError_t launch_dn_backward(const float* params, const cf* grid, const cf* dout, float* grads, int S, int K,
                              long long n_grid, char* ws, const DnLayout& lay, int n_cu, hipStream_t s);
// weights: one per grid of per_grid entries (nullptr: all 1).
hipError_t launch_dn_loss(const cf* out, const cf* target, const float* weights, long long per_grid, cf* dout,
                          float* loss, long long n, char* ws, const DnLayout& lay, hipStream_t s);
hipError_t launch_dn_adam(float* params, const float* grads, float* m, float* v, int n, float lr, float b1, float b2,
                          float eps, float c1, float c2, hipStream_t s);
// LS estimate on every symbol of every (UE, beam) pair: grid [item][n_ue][n_beams][n_symb][n_sc].
// Pilot symbol j of item i is RE-major at Y + i * y_batch + y_off[j]; pilots at
// P + i * p_batch + j * n_sc.
struct DnGridGeom {
  int n_beams, n_ue, n_sc, n_symb, n_pilot;
  int pilot_sym[kMaxPilots];
  long long y_off[kMaxPilots];
  long long y_batch, p_batch;
};
hipError_t launch_dn_ls_grid(const cf* Y, const cf* pilots, cf* grid, const DnGridGeom& g, long long batch,
                             hipStream_t s);
// Detection input from grids: H[item][n_sc][n_ue][n_beams] = symbol s of
// (use_b && use_b[item / per_use] ? b : a) [item][n_ue][n_beams][n_symb][n_sc].
hipError_t launch_dn_grid_to_h(const cf* a, const cf* b, const int* use_b, long long per_use, cf* H, int s_idx,
                               int n_ue, int n_beams, int n_symb, int n_sc, long long n_item, hipStream_t s);
// Fallback test: res[slot][e] = post-MMSE residual of estimate e (0: LS, 1:
// denoised) over the slot's data REs; H_e: [data symbol][slot][n_sc][n_ue][n_beams],
// X_e: [slot][data symbol][n_sc][n_ue], Y: [slot][n_symb][n_sc][n_beams] (y_slot apart).
struct DnSymbols {
  int n_data;
  int sym[kMaxSymbols];
};
hipError_t launch_dn_residual(const cf* H0, const cf* H1, const cf* X0, const cf* X1, const cf* Y, float* res,
                              const DnSymbols& ds, int n_ue, int n_beams, int n_sc, long long n_slot,
                              long long y_slot, hipStream_t s);
// X[slot] = res DN <= res LS ? X1 : X0 (per_slot entries each), the same for the
// status flags (st: [slot][n_sc], or nullptr), used[slot] (or nullptr) = the choice.
hipError_t launch_dn_select(const float* res, const cf* X0, const cf* X1, const int* st0, const int* st1, cf* X,
                            int* st, int* used, long long per_slot, int n_sc, long long n_slot, hipStream_t s);

}  // namespace pusch
