// OFDM-demodulation FFT (Sec. II; Table 1, row "OFDM dem.") for gfx950.
//
// N = R0 * 16^P with R0 in {4, 8, 16}: one radix-R0 pass followed by P
// radix-16 passes of the Stockham autosort formulation, so the result comes
// out in natural order without a digit-reversal step.  The paper's kernel is
// a radix-4 decimation-in-frequency FFT whose operands are folded into each
// core's local banks (Sec. V-A); here each 16-point butterfly is done in a
// thread's registers (a 4x4 split), and the data exchange between passes goes
// through LDS with one padding slot per 16 elements, which spreads the
// strided accesses of a pass over the banks.  It does not remove every
// conflict: the hardware counter (SQ_LDS_BANK_CONFLICT) still reports about
// 1,800 conflict cycles per wave at N = 4096, about 2 % of the wave's time.
//
// One workgroup of 256 threads owns 4096/N transforms at a time (N/16 threads
// per transform, 16 values per thread) and loops over the batch, so each
// thread loads its pass twiddles once, into registers.  Twiddles come from an
// FP32 table computed in FP64 on the host.  The final pass writes straight
// from registers to global memory, optionally keeping only the active
// subcarriers (fused gather), as FP32, FP16 with a per-row power of two, or
// bfloat16.  k_fft_mfma runs the same 4096-point passes with the butterflies
// on the matrix cores (reduced-precision outputs only).
#include <hip/hip_fp16.h>

#include <cmath>
#include <vector>

#include "kernels.h"

namespace pusch {
namespace {

__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cf cmul(cf a, cf b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cf mul_mi(cf a) { return {a.i, -a.r}; }  // * (-i)

// exp(-2 pi i m / 16) for the factors that occur inside a 16-point DFT.
constexpr float kC1 = 0.92387953251128675613f;  // cos(pi/8)
constexpr float kS1 = 0.38268343236508977173f;  // sin(pi/8)
constexpr float kR2 = 0.70710678118654752440f;  // sqrt(2)/2

__device__ __forceinline__ cf w16_1(cf a) { return {kC1 * a.r + kS1 * a.i, kC1 * a.i - kS1 * a.r}; }
__device__ __forceinline__ cf w16_2(cf a) { return {kR2 * (a.r + a.i), kR2 * (a.i - a.r)}; }
__device__ __forceinline__ cf w16_3(cf a) { return {kS1 * a.r + kC1 * a.i, kS1 * a.i - kC1 * a.r}; }
__device__ __forceinline__ cf w16_6(cf a) { return {kR2 * (a.i - a.r), -kR2 * (a.r + a.i)}; }
__device__ __forceinline__ cf w16_9(cf a) { return {-kC1 * a.r - kS1 * a.i, kS1 * a.r - kC1 * a.i}; }

// 4-point DFT of v[0], v[S], v[2S], v[3S], in place, natural order.
template <int S>
__device__ __forceinline__ void dft4s(cf* v) {
  const cf a = v[0], b = v[S], c = v[2 * S], d = v[3 * S];
  const cf t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = mul_mi(csub(b, d));
  v[0] = cadd(t0, t2);
  v[2 * S] = csub(t0, t2);
  v[S] = cadd(t1, t3);
  v[3 * S] = csub(t1, t3);
}

template <int R>
__device__ __forceinline__ void dft(cf* v);

template <>
__device__ __forceinline__ void dft<4>(cf* v) {
  dft4s<1>(v);
}

// 8 = 4 x 2: q = 2 q1 + q2, k = k1 + 4 k2.
template <>
__device__ __forceinline__ void dft<8>(cf* v) {
  dft4s<2>(v);
  dft4s<2>(v + 1);
  v[3] = w16_2(v[3]);   // w8^1
  v[5] = mul_mi(v[5]);  // w8^2
  v[7] = w16_6(v[7]);   // w8^3
  cf o[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    o[k1] = cadd(v[2 * k1], v[2 * k1 + 1]);
    o[k1 + 4] = csub(v[2 * k1], v[2 * k1 + 1]);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = o[i];
}

// 16 = 4 x 4: q = 4 q1 + q2, k = k1 + 4 k2.
template <>
__device__ __forceinline__ void dft<16>(cf* v) {
  dft4s<4>(v);
  dft4s<4>(v + 1);
  dft4s<4>(v + 2);
  dft4s<4>(v + 3);
  // position q2 + 4 k1 holds the inner DFT value; scale by w16^(k1 q2)
  v[5] = w16_1(v[5]);
  v[6] = w16_2(v[6]);
  v[7] = w16_3(v[7]);
  v[9] = w16_2(v[9]);
  v[10] = mul_mi(v[10]);
  v[11] = w16_6(v[11]);
  v[13] = w16_3(v[13]);
  v[14] = w16_6(v[14]);
  v[15] = w16_9(v[15]);
  dft4s<1>(v);
  dft4s<1>(v + 4);
  dft4s<1>(v + 8);
  dft4s<1>(v + 12);
  cf o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = o[i];
}

template <int N>
struct Shape;
template <>
struct Shape<64> {
  static constexpr int R0 = 4, P = 1;
};
template <>
struct Shape<256> {
  static constexpr int R0 = 16, P = 1;
};
template <>
struct Shape<1024> {
  static constexpr int R0 = 4, P = 2;
};
template <>
struct Shape<2048> {
  static constexpr int R0 = 8, P = 2;
};
template <>
struct Shape<4096> {
  static constexpr int R0 = 16, P = 2;
};

__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }

typedef float v2f __attribute__((ext_vector_type(2)));  // one complex value, for the non-temporal builtins

constexpr int kThreads = 256;

// FP16 output (H16): each transform's output row is stored as half2 words
// (re in the low half) scaled by 2^e, e = 14 - k where the row's input L1
// norm sum |re| + |im| = m * 2^k, m in [0.5, 1).  Every output bin is bounded
// by that norm, so |scaled| < 2^14 (no overflow); FP16 keeps 11 significant
// bits of every value.  The exponents go to an int8 table with 64 entries per
// group of `rows` transforms (one slot symbol: the antennas): transform
// i = g * rows + a stores e at g * 64 + (a % 4) * 16 + a / 4, so the 16
// antennas a = 4 j + q (j = 0..15) of one group are 16 consecutive bytes.
__device__ __forceinline__ unsigned pack_h2(float re, float im) {
  return (unsigned)__half_as_ushort(__float2half_rn(re)) | ((unsigned)__half_as_ushort(__float2half_rn(im)) << 16);
}

// BF16 output: the same words as bfloat16 pairs (re in the low half), rounded
// to nearest even (one v_cvt_pk_bf16_f32) and not scaled (bfloat16 has FP32's
// exponent range); no exponent table.
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_bf2(float re, float im) {
  const bf2v v = {(__bf16)re, (__bf16)im};
  return __builtin_bit_cast(unsigned, v);
}

// LDS of a workgroup: FPB = kThreads / (N / 16) padded transforms, the same
// 4352 complex values at every size (so one buffer serves every size of a
// grouped launch).
constexpr int kLdsCf = 4352;

// The transform loop of one launch (or of one cell's share of a grouped
// launch): workgroup vb of vg walks transforms vb*FPB, (vb + vg)*FPB, ...
// lds: kLdsCf values; red: kThreads / 64 floats (per-wave partial norms, FP16).
// FMT: 0 FP32 output, 1 FP16 (scaled rows, exponent table), 2 BF16.
template <int N, int FMT>
__device__ __forceinline__ void fft_body(cf* __restrict__ lds, float* __restrict__ red, int vb, int vg,
                                         const cf* __restrict__ x, cf* __restrict__ X, unsigned* __restrict__ Xh,
                                         signed char* __restrict__ ex, int rows, const cf* __restrict__ tw,
                                         long long batch, int out_len, int shift, long long ldo) {
  constexpr int T = N / 16;         // threads per transform
  constexpr int FPB = kThreads / T;  // transforms per workgroup
  constexpr int R0 = Shape<N>::R0;
  constexpr int P = Shape<N>::P;
  constexpr int LSTR = lds_pad(N);
  static_assert(FPB * LSTR == kLdsCf, "one LDS size for every transform size");
  constexpr bool HW = FMT != 0;   // 4-byte words out
  constexpr bool H16 = FMT == 1;  // FP16 with a power-of-two row scale

  const int fl = threadIdx.x / T;
  const int t = threadIdx.x % T;
  cf* L = lds + fl * LSTR;

  // Pass p (1..P) has stride Ns = R0 * 16^(p-1); this thread's twiddles are
  // exp(-2 pi i (t mod Ns) r / (16 Ns)), r = 1..15, table block [(r-1)*Ns + k].
  cf w[P][15];
  {
    int off = 0, ns = R0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int k = t % ns;
#pragma unroll
      for (int r = 1; r < 16; ++r) w[p][r - 1] = tw[off + (r - 1) * ns + k];
      off += 15 * ns;
      ns *= 16;
    }
  }

  // With FP16 or BF16 output the kernel no longer saturates HBM, so the input of the
  // workgroup's next transform is loaded during the current one's passes (a
  // transform past the batch re-reads the last one and is never stored).
  // With FP32 output the traffic is already at the bandwidth limit and the
  // registers are kept for occupancy.  Its time samples (read once) and its
  // output rows go through the caches as non-temporal accesses: measured on
  // the paper-scale slot, the FFT then takes ~4 us longer and the
  // beamforming that reads its output ~10 us less.
  const long long fstep = (long long)vg * FPB;
  cf vn[HW ? 16 : 1];
  auto prefetch = [&](long long f) {
    const cf* src = x + (f < batch ? f : batch - 1) * N;
#pragma unroll
    for (int m = 0; m < 16; ++m) vn[m] = src[t + m * T];
  };
  if constexpr (HW) prefetch((long long)vb * FPB + fl);
  for (long long f0 = (long long)vb * FPB; f0 < batch; f0 += fstep) {
    const long long fft = f0 + fl;
    const bool act = fft < batch;
    cf v[16];
    if constexpr (HW) {
#pragma unroll
      for (int m = 0; m < 16; ++m) v[m] = act ? vn[m] : cf{0.f, 0.f};
      prefetch(fft + fstep);
    } else if (act) {
      const v2f* src = reinterpret_cast<const v2f*>(x + fft * N);
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const v2f q = __builtin_nontemporal_load(src + t + m * T);
        v[m] = cf{q.x, q.y};
      }
    } else {
#pragma unroll
      for (int m = 0; m < 16; ++m) v[m] = cf{0.f, 0.f};
    }

    // FP16: the row's scale, from its L1 norm; it is applied only to the
    // output, so a transform wider than a wave leaves its per-wave partial
    // norms in LDS and adds them after pass 0's barrier (no barrier of its own)
    float scale = 1.f;
    float s1 = 0.f;
    auto set_scale = [&]() {
      int k = 0;
      (void)frexpf(s1, &k);
      int e = s1 > 0.f ? 14 - k : 0;
      e = e < -100 ? -100 : (e > 100 ? 100 : e);
      scale = ldexpf(1.f, e);
      if (t == 0 && act) {
        const long long grp = fft / rows;
        const int a = (int)(fft - grp * rows);
        ex[grp * 64 + (a & 3) * 16 + (a >> 2)] = (signed char)e;
      }
    };
    if constexpr (H16) {
#pragma unroll
      for (int m = 0; m < 16; ++m) s1 += fabsf(v[m].r) + fabsf(v[m].i);
      constexpr int WL = T < 64 ? T : 64;  // lanes of this transform in one wave
#pragma unroll
      for (int o = 1; o < WL; o <<= 1) s1 += __shfl_xor(s1, o);
      if constexpr (T > 64) {
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s1;
      } else {
        set_scale();
      }
    }

    // Pass 0: radix R0, Ns = 1 (no twiddles).  Butterfly j = t + u*T reads
    // x[j + r*N/R0] = v[u + r*16/R0] and writes element j*R0 + r.
#pragma unroll
    for (int u = 0; u < 16 / R0; ++u) {
      cf b[R0];
#pragma unroll
      for (int r = 0; r < R0; ++r) b[r] = v[u + r * (16 / R0)];
      dft<R0>(b);
      const int j = t + u * T;
#pragma unroll
      for (int r = 0; r < R0; ++r) L[lds_pad(j * R0 + r)] = b[r];
    }
    __syncthreads();
    if constexpr (H16 && T > 64) {
      s1 = 0.f;
#pragma unroll
      for (int w = 0; w < T / 64; ++w) s1 += red[fl * (T / 64) + w];
      set_scale();
    }

#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int ns = R0 << (4 * p);
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = L[lds_pad(t + r * T)];
      __syncthreads();
#pragma unroll
      for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], w[p][r - 1]);
      dft<16>(v);
      if (p < P - 1) {
        const int base = (t / ns) * 16 * ns + (t % ns);
#pragma unroll
        for (int r = 0; r < 16; ++r) L[lds_pad(base + r * ns)] = v[r];
        __syncthreads();
      } else if (act) {
        // last pass: Ns = N/16 = T, so bin f = t + r*T
        if constexpr (HW) {
          unsigned* dst = Xh + fft * ldo;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            int k = t + r * T + shift;
            if (k >= N) k -= N;
            if (k < out_len) dst[k] = H16 ? pack_h2(v[r].r * scale, v[r].i * scale) : pack_bf2(v[r].r, v[r].i);
          }
        } else {
          cf* dst = X + fft * ldo;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            int k = t + r * T + shift;
            if (k >= N) k -= N;
            if (k < out_len) __builtin_nontemporal_store(v2f{v[r].r, v[r].i}, reinterpret_cast<v2f*>(dst + k));
          }
        }
      }
    }
  }
}

template <int N, int FMT>
__global__ __launch_bounds__(kThreads) void k_fft(const cf* __restrict__ x, cf* __restrict__ X,
                                                  unsigned* __restrict__ Xh, signed char* __restrict__ ex, int rows,
                                                  const cf* __restrict__ tw, long long batch, int out_len,
                                                  int shift, long long ldo) {
  __shared__ cf lds[kLdsCf];
  __shared__ float red[kThreads / 64];
  fft_body<N, FMT>(lds, red, blockIdx.x, gridDim.x, x, X, Xh, ex, rows, tw, batch, out_len, shift, ldo);
}

// Many cells of any transform sizes in one launch: cell c owns workgroups
// [start[c], start[c + 1]) and runs the single-call loop of its size on its
// share (the size is uniform over a workgroup).
template <bool H16>
__global__ __launch_bounds__(kThreads) void k_fft_cells(FftCells t) {
  __shared__ cf lds[kLdsCf];
  __shared__ float red[kThreads / 64];
  int c = 0;
  while (c + 1 < t.n && (int)blockIdx.x >= t.start[c + 1]) ++c;
  const FftCell& e = t.cell[c];
  const int vb = blockIdx.x - t.start[c], vg = t.start[c + 1] - t.start[c];
  switch (e.n_fft) {
    case 64:
      fft_body<64, H16 ? 1 : 0>(lds, red, vb, vg, e.x, e.X, e.Xh, e.ex, e.rows, e.tw, e.batch, e.out_len, e.shift, e.ldo);
      break;
    case 256:
      fft_body<256, H16 ? 1 : 0>(lds, red, vb, vg, e.x, e.X, e.Xh, e.ex, e.rows, e.tw, e.batch, e.out_len, e.shift, e.ldo);
      break;
    case 1024:
      fft_body<1024, H16 ? 1 : 0>(lds, red, vb, vg, e.x, e.X, e.Xh, e.ex, e.rows, e.tw, e.batch, e.out_len, e.shift, e.ldo);
      break;
    case 2048:
      fft_body<2048, H16 ? 1 : 0>(lds, red, vb, vg, e.x, e.X, e.Xh, e.ex, e.rows, e.tw, e.batch, e.out_len, e.shift, e.ldo);
      break;
    default:
      fft_body<4096, H16 ? 1 : 0>(lds, red, vb, vg, e.x, e.X, e.Xh, e.ex, e.rows, e.tw, e.batch, e.out_len, e.shift, e.ldo);
      break;
  }
}

constexpr int kSizes[5] = {64, 256, 1024, 2048, 4096};
constexpr int kR0[5] = {4, 16, 4, 8, 16};
constexpr int kP[5] = {1, 1, 2, 2, 2};

}  // namespace

int fft_size_index(int n_fft) {
  for (int i = 0; i < 5; ++i)
    if (kSizes[i] == n_fft) return i;
  return -1;
}

TwiddleLayout fft_twiddle_layout() {
  TwiddleLayout t{};
  int off = 0;
  for (int s = 0; s < 5; ++s) {
    t.offset[s] = off;
    int ns = kR0[s];
    for (int p = 0; p < kP[s]; ++p) {
      off += 15 * ns;
      ns *= 16;
    }
  }
  t.total = off;
  return t;
}

void fft_fill_twiddles(cf* host) {
  const TwiddleLayout lay = fft_twiddle_layout();
  const double two_pi = 6.283185307179586476925286766559;
  for (int s = 0; s < 5; ++s) {
    int off = lay.offset[s];
    int ns = kR0[s];
    for (int p = 0; p < kP[s]; ++p) {
      const long m = 16L * ns;
      for (int r = 1; r < 16; ++r)
        for (int k = 0; k < ns; ++k) {
          const long e = ((long)k * r) % m;
          const double ang = -two_pi * (double)e / (double)m;
          host[off + (r - 1) * ns + k] = cf{(float)std::cos(ang), (float)std::sin(ang)};
        }
      off += 15 * ns;
      ns *= 16;
    }
  }
}

namespace {
// Persistent grid of exactly the resident workgroups (no second round of
// workgroups and its tail).
template <int N, int FMT>
hipError_t launch_nh(const cf* x, cf* X, unsigned* Xh, signed char* ex, int rows, const cf* tw, long long batch,
                     int out_len, int shift, long long ldo, long long blocks, int n_cu, hipStream_t s) {
  static const int per_cu = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fft<N, FMT>, kThreads, 0) != hipSuccess || n < 1) n = 1;
    return n;
  }();
  const long long cap = (long long)n_cu * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL((k_fft<N, FMT>), dim3((unsigned)blocks), dim3(kThreads), 0, s, x, X, Xh, ex, rows, tw, batch,
                     out_len, shift, ldo);
  return hipGetLastError();
}

// FP32 output (Xh null), FP16 (Xh and ex), BF16 (Xh, ex null)
template <int N>
hipError_t launch_n(const cf* x, cf* X, unsigned* Xh, signed char* ex, int rows, const cf* tw, long long batch,
                    int out_len, int shift, long long ldo, long long blocks, int n_cu, hipStream_t s) {
  if (!Xh) return launch_nh<N, 0>(x, X, Xh, ex, rows, tw, batch, out_len, shift, ldo, blocks, n_cu, s);
  if (ex) return launch_nh<N, 1>(x, X, Xh, ex, rows, tw, batch, out_len, shift, ldo, blocks, n_cu, s);
  return launch_nh<N, 2>(x, X, Xh, ex, rows, tw, batch, out_len, shift, ldo, blocks, n_cu, s);
}
}  // namespace

namespace {
template <bool H16>
hipError_t launch_cells_h(FftCells& t, int n_cu, hipStream_t s) {
  static const int per_cu = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fft_cells<H16>, kThreads, 0) != hipSuccess || n < 1) n = 1;
    return n;
  }();
  // work in workgroup rounds: a workgroup takes kThreads / (N / 16) transforms of
  // its cell per round (the same bytes and about the same time at every size)
  const int start = share_work(
      t.n, [&](int c) { const long long f = kThreads / (t.cell[c].n_fft / 16); return (t.cell[c].batch + f - 1) / f; },
      [](int) { return 1ll; }, (long long)n_cu * per_cu, t.start);
  hipLaunchKernelGGL((k_fft_cells<H16>), dim3((unsigned)start), dim3(kThreads), 0, s, t);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_fft_cells(FftCells& t, bool h16, const cf* twiddles, int n_cu, hipStream_t s) {
  if (t.n < 1 || t.n > kFftCellsPerLaunch) return hipErrorInvalidValue;
  const TwiddleLayout lay = fft_twiddle_layout();
  for (int c = 0; c < t.n; ++c) {
    FftCell& e = t.cell[c];
    const int si = fft_size_index(e.n_fft);
    if (si < 0 || e.batch <= 0) return hipErrorInvalidValue;
    if (h16 && (e.rows < 1 || e.rows > 64 || !e.Xh || !e.ex)) return hipErrorInvalidValue;
    e.tw = twiddles + lay.offset[si];
  }
  return h16 ? launch_cells_h<true>(t, n_cu, s) : launch_cells_h<false>(t, n_cu, s);
}

namespace {
// ---------------------------------------------------------------- radix-16 passes on matrix cores
// The reduced-precision chains' FFT with every radix-16 butterfly on the
// matrix cores: for N = 4096 = 16^3 each of the three Stockham passes is, per
// transform, the 16 x 16 DFT matrix F[m][r] = exp(-2 pi i m r / 16) times the
// 16 x 256 matrix of the butterflies' (twiddled) inputs, computed as four
// real 16x16x16 products (FP16 or BF16 operands, FP32 accumulation):
// Re = Fr Br - Fi Bi, Im = Fr Bi + Fi Br.  A workgroup of four waves takes
// one transform at a time; wave w owns butterflies 64 w .. 64 w + 63 as four
// 16-column blocks, and lane (q, c16) supplies inputs r = 4q .. 4q + 3 of
// butterfly 16 b + c16 (the B operand) and receives outputs m = 4q .. 4q + 3
// (the D operand), so the LDS exchange between passes, the twiddles and the
// output are those of the VALU kernel's Stockham formulation (k_fft):
// butterfly c of a pass with stride ns reads elements c + 256 r and writes
// (c / ns) 16 ns + c % ns + m ns.  Values are rounded to the operand format
// only as they enter a pass; LDS and the accumulators stay FP32.  FMT 1: FP16
// operands, every row scaled by a power of two from its L1 norm before the
// first pass (the partial sums of every pass are bounded by that norm, so no
// value leaves FP16's range) and stored as FP16 pairs with that exponent, as
// k_fft<N, 1>; FMT 2: BF16 operands and output, no scaling.
typedef _Float16 mh4 __attribute__((ext_vector_type(4)));
typedef short mb4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int FMT>
struct MmaOp;
template <>
struct MmaOp<1> {
  using T = mh4;
  static __device__ __forceinline__ T pack(float a, float b, float c, float d) {
    return T{(_Float16)a, (_Float16)b, (_Float16)c, (_Float16)d};
  }
  static __device__ __forceinline__ f32x4 mma(T a, T b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct MmaOp<2> {
  using T = mb4;
  static __device__ __forceinline__ T pack(float a, float b, float c, float d) {
    return __builtin_bit_cast(T, make_uint2(pack_bf2(a, b), pack_bf2(c, d)));
  }
  static __device__ __forceinline__ f32x4 mma(T a, T b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};

// cos(2 pi k / 16) from the three constants of the 16-point DFT
__device__ __forceinline__ float cos_16th(int k) {
  switch (k & 15) {
    case 0: return 1.f;
    case 1: return kC1;
    case 2: return kR2;
    case 3: return kS1;
    case 4: return 0.f;
    case 5: return -kS1;
    case 6: return -kR2;
    case 7: return -kC1;
    case 8: return -1.f;
    case 9: return -kC1;
    case 10: return -kR2;
    case 11: return -kS1;
    case 12: return 0.f;
    case 13: return kS1;
    case 14: return kR2;
    default: return kC1;
  }
}

template <int FMT>
__global__ __launch_bounds__(kThreads) void k_fft_mfma(const cf* __restrict__ x, unsigned* __restrict__ Xh,
                                                       signed char* __restrict__ ex, int rows,
                                                       const cf* __restrict__ tw, long long batch, int out_len,
                                                       int shift, long long ldo) {
  constexpr int N = 4096, T = N / 16;
  using O = MmaOp<FMT>;
  static_assert(kThreads == 256 && lds_pad(N - 1) < kLdsCf, "four waves, one transform in LDS");
  __shared__ cf lds[kLdsCf];
  __shared__ float red[kThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane >> 4, c16 = lane & 15;
  // A operand: F[c16][4q + i] as (re, im, -im)
  typename O::T Ar, Ai, An;
  {
    float fr[4], fi[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = c16 * (4 * q + i);
      fr[i] = cos_16th(k);
      fi[i] = -cos_16th(k - 4);  // -sin(2 pi k / 16)
    }
    Ar = O::pack(fr[0], fr[1], fr[2], fr[3]);
    Ai = O::pack(fi[0], fi[1], fi[2], fi[3]);
    An = O::pack(-fi[0], -fi[1], -fi[2], -fi[3]);
  }
  // twiddles of this lane's inputs r = 4q + i: the pass with stride 16 needs
  // exp(-2 pi i (c % 16) r / 256), the same for the lane's four butterflies;
  // the pass with stride 256 exp(-2 pi i c r / 4096) (table blocks as k_fft)
  cf w1[4], w2[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 4 * q + i;
    w1[i] = r ? tw[(r - 1) * 16 + c16] : cf{1.f, 0.f};
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int c = (wv * 4 + bb) * 16 + c16;
      w2[bb][i] = r ? tw[15 * 16 + (r - 1) * T + c] : cf{1.f, 0.f};
    }
  }
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  // one 16-column block: D = F B for the lane's four inputs (FP32 values)
  auto dft_block = [&](const cf (&v)[4], f32x4& dr, f32x4& di) {
    const typename O::T br = O::pack(v[0].r, v[1].r, v[2].r, v[3].r);
    const typename O::T bi = O::pack(v[0].i, v[1].i, v[2].i, v[3].i);
    dr = O::mma(An, bi, O::mma(Ar, br, z4));
    di = O::mma(Ai, br, O::mma(Ar, bi, z4));
  };

  // the next transform's input is loaded during the current one's passes (as
  // k_fft with 4-byte output; a transform past the batch re-reads the last)
  cf vn[4][4];
  auto load = [&](long long ff) {
    const cf* src = x + (ff < batch ? ff : batch - 1) * N;
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int i = 0; i < 4; ++i) vn[bb][i] = src[(wv * 4 + bb) * 16 + c16 + (4 * q + i) * T];
  };
  load(blockIdx.x);
  for (long long f = blockIdx.x; f < batch; f += gridDim.x) {
    cf v[4][4];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[bb][i] = vn[bb][i];
    load(f + gridDim.x);
    if constexpr (FMT == 1) {
      float s1 = 0.f;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int i = 0; i < 4; ++i) s1 += fabsf(v[bb][i].r) + fabsf(v[bb][i].i);
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) s1 += __shfl_xor(s1, o);
      if (lane == 0) red[wv] = s1;
      __syncthreads();
      s1 = red[0] + red[1] + red[2] + red[3];
      int k = 0;
      (void)frexpf(s1, &k);
      int e = s1 > 0.f ? 14 - k : 0;
      e = e < -100 ? -100 : (e > 100 ? 100 : e);
      const float scale = ldexpf(1.f, e);
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[bb][i] = cf{v[bb][i].r * scale, v[bb][i].i * scale};
      if (threadIdx.x == 0) {
        const long long grp = f / rows;
        const int a = (int)(f - grp * rows);
        ex[grp * 64 + (a & 3) * 16 + (a >> 2)] = (signed char)e;
      }
    }
    // pass 1 of 3 (stride 1, no twiddles): output m of butterfly c to c * 16 + m
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      f32x4 dr, di;
      dft_block(v[bb], dr, di);
      const int c = (wv * 4 + bb) * 16 + c16;
#pragma unroll
      for (int u = 0; u < 4; ++u) lds[lds_pad(c * 16 + 4 * q + u)] = cf{dr[u], di[u]};
    }
    __syncthreads();
    // pass 2 (stride 16)
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[bb][i] = lds[lds_pad((wv * 4 + bb) * 16 + c16 + (4 * q + i) * T)];
    __syncthreads();
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[bb][i] = cmul(v[bb][i], w1[i]);
      f32x4 dr, di;
      dft_block(v[bb], dr, di);
      const int cb = wv * 4 + bb;  // c / 16; c % 16 = c16
#pragma unroll
      for (int u = 0; u < 4; ++u) lds[lds_pad(cb * 256 + c16 + (4 * q + u) * 16)] = cf{dr[u], di[u]};
    }
    __syncthreads();
    // pass 3 (stride 256): output m of butterfly c is bin c + 256 m
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[bb][i] = lds[lds_pad((wv * 4 + bb) * 16 + c16 + (4 * q + i) * T)];
    __syncthreads();  // the next transform's first pass writes LDS
    unsigned* dst = Xh + f * ldo;
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[bb][i] = cmul(v[bb][i], w2[bb][i]);
      f32x4 dr, di;
      dft_block(v[bb], dr, di);
      const int c = (wv * 4 + bb) * 16 + c16;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        int k = c + (4 * q + u) * T + shift;
        if (k >= N) k -= N;
        if (k < out_len) dst[k] = FMT == 1 ? pack_h2(dr[u], di[u]) : pack_bf2(dr[u], di[u]);
      }
    }
  }
}
// Persistent grid of exactly the resident workgroups, as k_fft.
template <int FMT>
hipError_t launch_mfma_fmt(const cf* x, unsigned* Xh, signed char* ex, int rows, const cf* tw, long long batch,
                           int out_len, int shift, long long ldo, int n_cu, hipStream_t s) {
  static const int per_cu = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_fft_mfma<FMT>, kThreads, 0) != hipSuccess || n < 1) n = 1;
    return n;
  }();
  long long blocks = batch;
  const long long cap = (long long)n_cu * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL((k_fft_mfma<FMT>), dim3((unsigned)blocks), dim3(kThreads), 0, s, x, Xh, ex, rows, tw, batch,
                     out_len, shift, ldo);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_fft_mfma(const cf* x, int n_fft, long long batch, int out_len, int shift, long long ldo,
                           const cf* twiddles, int n_cu, hipStream_t s, unsigned* Xh, signed char* ex, int rows) {
  if (n_fft != 4096 || !Xh || (ex && (rows < 1 || rows > 64)) || out_len > n_fft || shift < 0 || shift >= n_fft ||
      ldo < out_len)
    return hipErrorInvalidValue;
  if (batch <= 0) return hipSuccess;
  const TwiddleLayout lay = fft_twiddle_layout();
  const cf* tw = twiddles + lay.offset[fft_size_index(n_fft)];
  return ex ? launch_mfma_fmt<1>(x, Xh, ex, rows, tw, batch, out_len, shift, ldo, n_cu, s)
            : launch_mfma_fmt<2>(x, Xh, ex, rows, tw, batch, out_len, shift, ldo, n_cu, s);
}

hipError_t launch_fft(const cf* x, cf* X, int n_fft, long long batch, int out_len, int shift, long long ldo,
                      const cf* twiddles, int n_cu, hipStream_t s, unsigned* Xh, signed char* ex, int rows) {
  if (Xh && ex && (rows < 1 || rows > 64)) return hipErrorInvalidValue;
  if (batch <= 0) return hipSuccess;
  const int si = fft_size_index(n_fft);
  const TwiddleLayout lay = fft_twiddle_layout();
  const cf* tw = twiddles + lay.offset[si];
  const long long fpb = kThreads / (n_fft / 16);
  const long long blocks = (batch + fpb - 1) / fpb;
  switch (n_fft) {
    case 64: return launch_n<64>(x, X, Xh, ex, rows, tw, batch, out_len, shift, ldo, blocks, n_cu, s);
    case 256: return launch_n<256>(x, X, Xh, ex, rows, tw, batch, out_len, shift, ldo, blocks, n_cu, s);
    case 1024: return launch_n<1024>(x, X, Xh, ex, rows, tw, batch, out_len, shift, ldo, blocks, n_cu, s);
    case 2048: return launch_n<2048>(x, X, Xh, ex, rows, tw, batch, out_len, shift, ldo, blocks, n_cu, s);
    case 4096: return launch_n<4096>(x, X, Xh, ex, rows, tw, batch, out_len, shift, ldo, blocks, n_cu, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pusch
