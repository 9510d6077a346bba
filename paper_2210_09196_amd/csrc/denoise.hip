// Learned refinement of the LS channel estimate (the paper's estimator is
// least squares on the pilot symbols, Sec. II, CHE): a four-layer 3x3
// convolutional network, 2 -> 32 -> 32 -> 32 -> 2 channels with ReLU after
// the first three, run on every (UE, beam) pair's LS estimate over the
// subcarrier x symbol grid (real and imaginary parts as the two channels),
// its output added to the LS estimate.  Training and inference kernels:
//
// k_dn_conv      one 3x3 convolution as an implicit GEMM on bfloat16 matrix
//                cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation).  A wave
//                computes 16 consecutive subcarriers of one symbol for all
//                output channels; the weights of the whole layer sit in its
//                registers as A fragments (rows = output channels, K = the
//                9 offsets x input channels, input channel fastest), the
//                activations are the B fragments, read from the layer input
//                ([position][channel], bfloat16 or FP32 rounded on load, zero
//                outside the grid).  Epilogues: hidden layers add the bias,
//                apply ReLU and store bfloat16; the last adds the bias and the
//                LS estimate (FP32); the input-gradient pass of backprop is
//                the same kernel with the layer's weights flipped and
//                transposed, its output masked by the ReLU of the layer below
//                and stored FP32.
// k_dn_wgrad     weight and bias gradients, dW[o][off][i] = sum_p dz[p][o]
//                x[p + off][i], in FP32 on the vector units: a workgroup stages
//                a row segment of the layer input (with its halo) and of dz in
//                LDS and accumulates over every segment it owns; the partial
//                sums per workgroup are reduced in a fixed order (k_dn_reduce),
//                so gradients do not depend on scheduling.
// k_dn_loss*     mean squared error against a target grid (optionally
//                weighted per grid) and its gradient.
// k_dn_adam      Adam update of the FP32 master parameters (the kernels round
//                the weights to bfloat16 when they load them).
// k_dn_ls_grid   the LS estimate on every symbol of every (UE, beam) pair,
//                linear along the subcarriers and in time between pilot
//                symbols.
// k_dn_data_residual, k_dn_select   the fallback test of the chain: the
//                post-MMSE residual |y - H x|^2 over a slot's data REs with
//                each estimate, and the pick of the denoised result unless
//                its residual exceeds the LS one.
#include "kernels.h"

namespace pusch {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kCh = 32;  // hidden channels

// FP32 -> bfloat16 bit pattern, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ f32x4 mfma_bf16(s4 a, s4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

enum { kEpiHidden = 0, kEpiLast = 1, kEpiDgrad = 2 };

// One 3x3 'same' convolution over a batch of [S][K] grids.  Input: CIN
// channels per position, bfloat16 (IN_BF16) or FP32 ([p][CIN]; CIN = 2 is a
// complex grid).  W: the layer's FP32 weights [co][off][ci] (off = 3 dy + dx);
// with EPI == kEpiDgrad they belong to the layer whose input gradient this is
// (its c_out = CIN, its c_in = COUT) and are used flipped and transposed.
// scale: multiplies a complex-grid input (CIN = 2) before rounding, and the
// correction of the last layer (out = resid + scale (acc + bias)); 1 elsewhere.
template <int CIN, int COUT, bool IN_BF16, int EPI>
__global__ __launch_bounds__(256) void k_dn_conv(const float* __restrict__ W, const float* __restrict__ bias,
                                                 const void* __restrict__ in, const cf* __restrict__ resid,
                                                 const unsigned short* __restrict__ mask, void* __restrict__ out, int S,
                                                 int K, long long ntiles, int ktiles, float scale) {
  constexpr int KSTEPS = (9 * CIN + 15) / 16;
  constexpr int MT = (COUT + 15) / 16;
  constexpr bool DG = EPI == kEpiDgrad;
  static_assert(CIN == 2 || CIN == kCh, "input channels");
  static_assert((COUT == 2 && EPI == kEpiLast) || (COUT == kCh && EPI != kEpiLast), "output channels");
  const int lane = threadIdx.x & 63, q = lane >> 4, col = lane & 15;

  // A fragments: lane (q, col) holds W'[16 m + col][16 t + 4 q + i], i = 0..3
  s4 wa[MT][KSTEPS];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < KSTEPS; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kk = 16 * t + 4 * q + i, off = kk / CIN, ci = kk % CIN, co = 16 * m + col;
        float w = 0.f;
        if (off < 9 && co < COUT) w = DG ? W[(ci * 9 + (8 - off)) * COUT + co] : W[(co * 9 + off) * CIN + ci];
        wa[m][t][i] = (short)bf16_bits(w);
      }

  const long long wave = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  for (long long tile = wave; tile < ntiles; tile += (long long)gridDim.x * 4) {
    const long long row = tile / ktiles;  // grid * S + symbol
    const int k0 = (int)(tile - row * ktiles) * 16;
    const int s = (int)(row % S);
    const long long gbase = (row - s) * K;  // position index of (grid, 0, 0)
    const int kc = k0 + col;
    f32x4 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < KSTEPS; ++t) {
      s4 b;
      if constexpr (CIN == kCh) {
        // K-step t: offset t / 2, channels 16 (t % 2) + 4 q .. + 3
        const int off = t >> 1, dy = off / 3, dx = off - 3 * dy;
        const int ss = s + dy - 1, kx = kc + dx - 1;
        const int c0 = (t & 1) * 16 + 4 * q;
        const bool ok = ss >= 0 && ss < S && kx >= 0 && kx < K;
        const long long p = gbase + (long long)ss * K + kx;
        if constexpr (IN_BF16) {
          uint2 u = make_uint2(0u, 0u);
          if (ok) u = *reinterpret_cast<const uint2*>(static_cast<const unsigned short*>(in) + p * kCh + c0);
          b = s4{(short)(u.x & 0xffffu), (short)(u.x >> 16), (short)(u.y & 0xffffu), (short)(u.y >> 16)};
        } else {
          float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
          if (ok) f = *reinterpret_cast<const float4*>(static_cast<const float*>(in) + p * kCh + c0);
          b = s4{(short)bf16_bits(f.x), (short)bf16_bits(f.y), (short)bf16_bits(f.z), (short)bf16_bits(f.w)};
        }
      } else {
        // two channels (a complex grid): K-step t covers offsets 8 t + 2 q and 8 t + 2 q + 1
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int off = 8 * t + 2 * q + h, dy = off / 3, dx = off - 3 * dy;
          const int ss = s + dy - 1, kx = kc + dx - 1;
          cf v = cf{0.f, 0.f};
          if (off < 9 && ss >= 0 && ss < S && kx >= 0 && kx < K)
            v = static_cast<const cf*>(in)[gbase + (long long)ss * K + kx];
          b[2 * h] = (short)bf16_bits(v.r * scale);
          b[2 * h + 1] = (short)bf16_bits(v.i * scale);
        }
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m] = mfma_bf16(wa[m][t], b, acc[m]);
    }
    if (kc >= K) continue;
    // lane (q, col) holds output channels 16 m + 4 q + v of position kc
    const long long p = gbase + (long long)s * K + kc;
    if constexpr (EPI == kEpiHidden) {
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        unsigned short h[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) h[v] = bf16_bits(fmaxf(acc[m][v] + bias[16 * m + 4 * q + v], 0.f));
        *reinterpret_cast<uint2*>(static_cast<unsigned short*>(out) + p * kCh + 16 * m + 4 * q) =
            make_uint2(h[0] | (unsigned)h[1] << 16, h[2] | (unsigned)h[3] << 16);
      }
    } else if constexpr (EPI == kEpiLast) {
      if (q == 0) {
        const cf r = resid[p];
        static_cast<cf*>(out)[p] = cf{r.r + scale * (acc[0][0] + bias[0]), r.i + scale * (acc[0][1] + bias[1])};
      }
    } else {
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const uint2 mk = *reinterpret_cast<const uint2*>(mask + p * kCh + 16 * m + 4 * q);
        float4 o;
        o.x = (mk.x & 0xffffu) ? acc[m][0] : 0.f;
        o.y = (mk.x >> 16) ? acc[m][1] : 0.f;
        o.z = (mk.y & 0xffffu) ? acc[m][2] : 0.f;
        o.w = (mk.y >> 16) ? acc[m][3] : 0.f;
        *reinterpret_cast<float4*>(static_cast<float*>(out) + p * kCh + 16 * m + 4 * q) = o;
      }
    }
  }
}

// Weight and bias gradients of one layer (CIN -> COUT) over row segments of
// kWgSeg positions: part[block][co * 9 CIN + off * CIN + ci], then the COUT
// bias sums.  x: the layer input as the forward pass read it (bfloat16
// [p][32], or a complex grid rounded to bfloat16); dz: FP32 [p][COUT] (COUT =
// 2: a complex grid).
constexpr int kWgSeg = 64;

template <int CIN, int COUT, bool IN_BF16>
__global__ __launch_bounds__(256) void k_dn_wgrad(const void* __restrict__ x, const float* __restrict__ dz,
                                                  float* __restrict__ part, int S, int K, long long nseg, int kseg) {
  constexpr int TPC = 256 / COUT;                 // threads per output channel
  constexpr int PER = (9 * CIN + TPC - 1) / TPC;  // (offset, input channel) pairs per thread
  constexpr int NW = COUT * 9 * CIN;
  __shared__ float sx[3][kWgSeg + 2][CIN];
  __shared__ float sd[kWgSeg][COUT];
  const int t = threadIdx.x, co = t / TPC, j = t - co * TPC;
  float acc[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) acc[r] = 0.f;
  float accb = 0.f;
  for (long long seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
    const long long row = seg / kseg;
    const int k0 = (int)(seg - row * kseg) * kWgSeg;
    const int s = (int)(row % S);
    const long long gbase = (row - s) * K;
    __syncthreads();
    for (int e = t; e < 3 * (kWgSeg + 2) * CIN; e += 256) {
      const int r = e / ((kWgSeg + 2) * CIN), rem = e - r * (kWgSeg + 2) * CIN;
      const int xx = rem / CIN, c = rem - xx * CIN;
      const int ss = s + r - 1, kx = k0 + xx - 1;
      float v = 0.f;
      if (ss >= 0 && ss < S && kx >= 0 && kx < K) {
        const long long p = gbase + (long long)ss * K + kx;
        if constexpr (IN_BF16) {
          v = bf16_val(static_cast<const unsigned short*>(x)[p * CIN + c]);
        } else {
          const float f = static_cast<const float*>(x)[p * CIN + c];
          v = bf16_val(bf16_bits(f));
        }
      }
      sx[r][xx][c] = v;
    }
    for (int e = t; e < kWgSeg * COUT; e += 256) {
      const int xx = e / COUT, c = e - xx * COUT;
      const int kx = k0 + xx;
      sd[xx][c] = kx < K ? dz[(gbase + (long long)s * K + kx) * COUT + c] : 0.f;
    }
    __syncthreads();
    for (int xx = 0; xx < kWgSeg; ++xx) {
      const float g = sd[xx][co];
      accb += g;
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const int f = j * PER + r;
        if (f < 9 * CIN) {
          const int off = f / CIN, ci = f - off * CIN, dy = off / 3, dx = off - 3 * dy;
          acc[r] += g * sx[dy][xx + dx][ci];
        }
      }
    }
  }
  float* pb = part + (long long)blockIdx.x * (NW + COUT);
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int f = j * PER + r;
    if (f < 9 * CIN) pb[co * 9 * CIN + f] = acc[r];
  }
  if (j == 0) pb[NW + co] = accb;
}

// out[w] = sum over blocks b (in order) of part[b][w].
__global__ __launch_bounds__(256) void k_dn_reduce(const float* __restrict__ part, float* __restrict__ out, int n,
                                                   int nblocks) {
  const int w = blockIdx.x * 256 + threadIdx.x;
  if (w >= n) return;
  float a = 0.f;
  for (int b = 0; b < nblocks; ++b) a += part[(long long)b * n + w];
  out[w] = a;
}

// Mean squared error over n complex entries and its gradient 2 (out - tgt) / n.
constexpr int kLossBlocks = 256;

__global__ __launch_bounds__(256) void k_dn_loss(const cf* __restrict__ o, const cf* __restrict__ tg,
                                                 const float* __restrict__ wg, long long per_grid, cf* __restrict__ d,
                                                 float* __restrict__ part, long long n, float two_over_n) {
  __shared__ float red[256];
  float a = 0.f;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const cf x = o[i], y = tg[i];
    const float w = wg ? wg[i / per_grid] : 1.f;
    const float er = x.r - y.r, ei = x.i - y.i;
    a += w * (er * er + ei * ei);
    d[i] = cf{two_over_n * w * er, two_over_n * w * ei};
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_dn_loss_final(const float* __restrict__ part, float* __restrict__ loss,
                                                       int nparts, float inv_n) {
  __shared__ float red[256];
  float a = 0.f;
  for (int i = threadIdx.x; i < nparts; i += 256) a += part[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] * inv_n;
}

// Adam (first and second moment, bias-corrected by c1 = 1 - beta1^t and c2 = 1 - beta2^t).
__global__ __launch_bounds__(256) void k_dn_adam(float* __restrict__ p, const float* __restrict__ g,
                                                 float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                 float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// LS estimate on every symbol: one thread per (item, UE, beam, subcarrier).
__global__ __launch_bounds__(256) void k_dn_ls_grid(const cf* __restrict__ Y, const cf* __restrict__ P,
                                                    cf* __restrict__ G, DnGridGeom g, long long total) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int K = g.n_sc, B = g.n_beams, L = g.n_ue;
  const int k = (int)(idx % K);
  long long r = idx / K;
  const int b = (int)(r % B);
  r /= B;
  const int l = (int)(r % L);
  const long long item = r / L;
  cf h[kMaxPilots];
  for (int j = 0; j < g.n_pilot; ++j) {
    // UE l's positions on pilot symbol j: first + step i
    const int o = j * (L / g.n_pilot);
    const int first = ((l - o) % L + L) % L, step = L;
    const int last = first + ((K - 1 - first) / step) * step;
    int lo = first, hi = first;
    float w = 0.f;
    if (k >= last) {
      lo = hi = last;
    } else if (k > first) {
      lo = first + ((k - first) / step) * step;
      hi = lo + step;
      w = (float)(k - lo) / (float)step;
    }
    const cf* yj = Y + item * g.y_batch + g.y_off[j];
    const cf* pj = P + item * g.p_batch + (long long)j * K;
    auto ls = [&](int pos) {
      const cf y = yj[(long long)pos * B + b], p = pj[pos];
      const float inv = 1.f / (p.r * p.r + p.i * p.i);
      return cf{(y.r * p.r + y.i * p.i) * inv, (y.i * p.r - y.r * p.i) * inv};
    };
    const cf a = ls(lo), c = ls(hi);
    h[j] = cf{a.r + w * (c.r - a.r), a.i + w * (c.i - a.i)};
  }
  cf* out = G + ((item * L + l) * B + b) * (long long)g.n_symb * K + k;
  for (int s = 0; s < g.n_symb; ++s) {
    cf v;
    if (s <= g.pilot_sym[0]) {
      v = h[0];
    } else if (s >= g.pilot_sym[g.n_pilot - 1]) {
      v = h[g.n_pilot - 1];
    } else {
      int jb = 1;
      while (g.pilot_sym[jb] <= s) ++jb;
      const int ja = jb - 1;
      const float den = (float)(g.pilot_sym[jb] - g.pilot_sym[ja]);
      const float wa = (float)(g.pilot_sym[jb] - s) / den, wb = (float)(s - g.pilot_sym[ja]) / den;
      v = cf{wa * h[ja].r + wb * h[jb].r, wa * h[ja].i + wb * h[jb].i};
    }
    out[(long long)s * K] = v;
  }
}

// H[item][k][l][b] = symbol s of the chosen grid; one thread per (item, k, l, b).
__global__ __launch_bounds__(256) void k_dn_grid_to_h(const cf* __restrict__ a, const cf* __restrict__ b,
                                                      const int* __restrict__ use_b, long long per_use,
                                                      cf* __restrict__ H, int s_idx, int L, int B, int S, int K,
                                                      long long total) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int bb = (int)(idx % B);
  long long r = idx / B;
  const int l = (int)(r % L);
  r /= L;
  const int k = (int)(r % K);
  const long long item = r / K;
  const cf* src = (use_b && use_b[item / per_use]) ? b : a;
  H[idx] = src[((item * L + l) * B + bb) * (long long)S * K + (long long)s_idx * K + k];
}

// One workgroup per (slot, estimate e): the post-MMSE residual sum over the
// slot's data REs and beams of |y - H x|^2, in a fixed order.  H of data
// symbol d: H_e + (d * n_slot + slot) * K * L * B ([K][L][B]); x: X_e [slot][d][K][L];
// y: the RE-major symbol grid of data symbol d.
__global__ __launch_bounds__(256) void k_dn_data_residual(const cf* __restrict__ H0, const cf* __restrict__ H1,
                                                          const cf* __restrict__ X0, const cf* __restrict__ X1,
                                                          const cf* __restrict__ Y, float* __restrict__ res,
                                                          DnSymbols ds, int L, int B, int K, long long n_slot,
                                                          long long y_slot) {
  __shared__ float red[256];
  const long long slot = blockIdx.x >> 1;
  const int e = blockIdx.x & 1;
  const cf* Hs = e ? H1 : H0;
  const cf* Xs = e ? X1 : X0;
  float acc = 0.f;
  for (int d = 0; d < ds.n_data; ++d) {
    const cf* Hd = Hs + ((long long)d * n_slot + slot) * K * L * B;
    const cf* Xd = Xs + ((slot * ds.n_data + d) * K) * L;
    const cf* Yd = Y + slot * y_slot + (long long)ds.sym[d] * K * B;
    for (int k = threadIdx.x; k < K; k += 256) {
      for (int b = 0; b < B; ++b) {
        cf r = Yd[(long long)k * B + b];
        for (int l = 0; l < L; ++l) {
          const cf h = Hd[((long long)k * L + l) * B + b], x = Xd[(long long)k * L + l];
          r.r -= h.r * x.r - h.i * x.i;
          r.i -= h.r * x.i + h.i * x.r;
        }
        acc += r.r * r.r + r.i * r.i;
      }
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) res[slot * 2 + e] = red[0];
}

// The pick per slot: the denoised result (estimate 1) unless its residual
// exceeds the LS one (estimate 0); one thread per detected symbol entry.
__global__ __launch_bounds__(256) void k_dn_select(const float* __restrict__ res, const cf* __restrict__ X0,
                                                   const cf* __restrict__ X1, const int* __restrict__ st0,
                                                   const int* __restrict__ st1, cf* __restrict__ X,
                                                   int* __restrict__ st, int* __restrict__ used, long long per_slot,
                                                   int K, long long total) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const long long slot = i / per_slot;
  const bool dn = res[slot * 2 + 1] <= res[slot * 2];
  X[i] = dn ? X1[i] : X0[i];
  const long long r = i - slot * per_slot;
  if (st && r < K) st[slot * K + r] = dn ? st1[slot * K + r] : st0[slot * K + r];
  if (used && r == 0) used[slot] = dn ? 1 : 0;
}

int conv_grid(long long ntiles, int n_cu) {
  const long long want = (ntiles + 3) / 4;
  const long long cap = (long long)n_cu * 8;
  return (int)(want < cap ? (want < 1 ? 1 : want) : cap);
}

template <int CIN, int COUT, bool IN_BF16, int EPI>
hipError_t conv(const float* W, const float* bias, const void* in, const cf* resid, const unsigned short* mask, void* out,
                int S, int K, long long n_grid, int n_cu, hipStream_t s, float scale = 1.f) {
  const int ktiles = (K + 15) / 16;
  const long long ntiles = n_grid * S * ktiles;
  hipLaunchKernelGGL((k_dn_conv<CIN, COUT, IN_BF16, EPI>), dim3(conv_grid(ntiles, n_cu)), dim3(256), 0, s, W, bias, in,
                     resid, mask, out, S, K, ntiles, ktiles, scale);
  return hipGetLastError();
}

template <int CIN, int COUT, bool IN_BF16>
hipError_t wgrad(const void* x, const float* dz, float* part, float* grad, int S, int K, long long n_grid, int n_cu,
                 hipStream_t s) {
  const int kseg = (K + kWgSeg - 1) / kWgSeg;
  const long long nseg = n_grid * S * kseg;
  const int nb = dn_wgrad_blocks(n_cu);
  const int blocks = (int)(nseg < nb ? nseg : nb);
  hipLaunchKernelGGL((k_dn_wgrad<CIN, COUT, IN_BF16>), dim3(blocks), dim3(256), 0, s, x, dz, part, S, K, nseg, kseg);
  if (hipError_t e = hipGetLastError()) return e;
  const int n = COUT * 9 * CIN + COUT;
  hipLaunchKernelGGL(k_dn_reduce, dim3((n + 255) / 256), dim3(256), 0, s, part, grad, n, blocks);
  return hipGetLastError();
}

}  // namespace

// A fixed count (not derived from the device) so that workspace sizes are
// known without a device and gradients sum in the same order on every part.
int dn_wgrad_blocks(int) { return kDnWgradBlocks; }

DnLayout dn_layout(int n_symb, int n_sc, long long n_grid, int n_cu) {
  DnLayout d;
  const long long P = n_grid * n_symb * (long long)n_sc;
  auto a256 = [](long long v) { return (v + 255) & ~255ll; };
  d.off_act[0] = 0;
  d.off_act[1] = a256(P * kCh * 2);
  d.off_act[2] = d.off_act[1] + a256(P * kCh * 2);
  d.off_dz[0] = d.off_act[2] + a256(P * kCh * 2);
  d.off_dz[1] = d.off_dz[0] + a256(P * kCh * 4);
  d.off_part = d.off_dz[1] + a256(P * kCh * 4);
  const long long nmax = kCh * 9 * kCh + kCh;
  d.off_loss = d.off_part + a256((long long)dn_wgrad_blocks(n_cu) * nmax * 4);
  d.total = d.off_loss + a256(kLossBlocks * 4);
  d.fwd_total = d.off_dz[0];
  return d;
}

hipError_t launch_dn_forward(const float* params, const cf* grid, cf* out, int S, int K, long long n_grid, char* ws,
                             const DnLayout& lay, int n_cu, hipStream_t s, float sigma) {
  unsigned short* a[3];
  for (int i = 0; i < 3; ++i) a[i] = reinterpret_cast<unsigned short*>(ws + lay.off_act[i]);
  const float* p = params;
  if (hipError_t e = conv<2, kCh, false, kEpiHidden>(p, p + kDnW1, grid, nullptr, nullptr, a[0], S, K, n_grid, n_cu, s,
                                                     1.f / sigma))
    return e;
  p += kDnW1 + kCh;
  if (hipError_t e = conv<kCh, kCh, true, kEpiHidden>(p, p + kDnW2, a[0], nullptr, nullptr, a[1], S, K, n_grid, n_cu, s))
    return e;
  p += kDnW2 + kCh;
  if (hipError_t e = conv<kCh, kCh, true, kEpiHidden>(p, p + kDnW2, a[1], nullptr, nullptr, a[2], S, K, n_grid, n_cu, s))
    return e;
  p += kDnW2 + kCh;
  return conv<kCh, 2, true, kEpiLast>(p, p + kDnW4, a[2], grid, nullptr, out, S, K, n_grid, n_cu, s, sigma);
}

hipError_t launch_dn_backward(const float* params, const cf* grid, const cf* dout, float* grads, int S, int K,
                              long long n_grid, char* ws, const DnLayout& lay, int n_cu, hipStream_t s) {
  const unsigned short* a[3];
  for (int i = 0; i < 3; ++i) a[i] = reinterpret_cast<const unsigned short*>(ws + lay.off_act[i]);
  float* dz[2] = {reinterpret_cast<float*>(ws + lay.off_dz[0]), reinterpret_cast<float*>(ws + lay.off_dz[1])};
  float* part = reinterpret_cast<float*>(ws + lay.off_part);
  const float* W1 = params;
  const float* W2 = W1 + kDnW1 + kCh;
  const float* W3 = W2 + kDnW2 + kCh;
  const float* W4 = W3 + kDnW2 + kCh;
  float* g1 = grads;
  float* g2 = g1 + kDnW1 + kCh;
  float* g3 = g2 + kDnW2 + kCh;
  float* g4 = g3 + kDnW2 + kCh;
  const float* d4 = reinterpret_cast<const float*>(dout);
  // layer 4 (32 -> 2): its gradients, then the gradient at its input through the ReLU of layer 3
  if (hipError_t e = wgrad<kCh, 2, true>(a[2], d4, part, g4, S, K, n_grid, n_cu, s)) return e;
  if (hipError_t e = conv<2, kCh, false, kEpiDgrad>(W4, nullptr, dout, nullptr, a[2], dz[0], S, K, n_grid, n_cu, s))
    return e;
  // layer 3
  if (hipError_t e = wgrad<kCh, kCh, true>(a[1], dz[0], part, g3, S, K, n_grid, n_cu, s)) return e;
  if (hipError_t e = conv<kCh, kCh, false, kEpiDgrad>(W3, nullptr, dz[0], nullptr, a[1], dz[1], S, K, n_grid, n_cu, s))
    return e;
  // layer 2
  if (hipError_t e = wgrad<kCh, kCh, true>(a[0], dz[1], part, g2, S, K, n_grid, n_cu, s)) return e;
  if (hipError_t e = conv<kCh, kCh, false, kEpiDgrad>(W2, nullptr, dz[1], nullptr, a[0], dz[0], S, K, n_grid, n_cu, s))
    return e;
  // layer 1 (2 -> 32): its input is the LS grid
  return wgrad<2, kCh, false>(grid, dz[0], part, g1, S, K, n_grid, n_cu, s);
}

hipError_t launch_dn_loss(const cf* out, const cf* target, const float* weights, long long per_grid, cf* dout,
                          float* loss, long long n, char* ws, const DnLayout& lay, hipStream_t s) {
  float* part = reinterpret_cast<float*>(ws + lay.off_loss);
  const float two_over_n = (float)(2.0 / (double)n), inv_n = (float)(1.0 / (double)n);
  hipLaunchKernelGGL(k_dn_loss, dim3(kLossBlocks), dim3(256), 0, s, out, target, weights, per_grid, dout, part, n,
                     two_over_n);
  if (hipError_t e = hipGetLastError()) return e;
  hipLaunchKernelGGL(k_dn_loss_final, dim3(1), dim3(256), 0, s, part, loss, kLossBlocks, inv_n);
  return hipGetLastError();
}

hipError_t launch_dn_adam(float* params, const float* grads, float* m, float* v, int n, float lr, float b1, float b2,
                          float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_dn_adam, dim3((n + 255) / 256), dim3(256), 0, s, params, grads, m, v, n, lr, b1, b2, eps, c1,
                     c2);
  return hipGetLastError();
}

hipError_t launch_dn_ls_grid(const cf* Y, const cf* pilots, cf* grid, const DnGridGeom& g, long long batch,
                             hipStream_t s) {
  const long long total = batch * g.n_ue * g.n_beams * (long long)g.n_sc;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dn_ls_grid, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Y, pilots, grid, g, total);
  return hipGetLastError();
}

hipError_t launch_dn_grid_to_h(const cf* a, const cf* b, const int* use_b, long long per_use, cf* H, int s_idx,
                               int n_ue, int n_beams, int n_symb, int n_sc, long long n_item, hipStream_t s) {
  const long long total = n_item * n_sc * (long long)n_ue * n_beams;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dn_grid_to_h, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, b, use_b, per_use, H,
                     s_idx, n_ue, n_beams, n_symb, n_sc, total);
  return hipGetLastError();
}

hipError_t launch_dn_residual(const cf* H0, const cf* H1, const cf* X0, const cf* X1, const cf* Y, float* res,
                              const DnSymbols& ds, int n_ue, int n_beams, int n_sc, long long n_slot,
                              long long y_slot, hipStream_t s) {
  if (n_slot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dn_data_residual, dim3((unsigned)(2 * n_slot)), dim3(256), 0, s, H0, H1, X0, X1, Y, res, ds,
                     n_ue, n_beams, n_sc, n_slot, y_slot);
  return hipGetLastError();
}

hipError_t launch_dn_select(const float* res, const cf* X0, const cf* X1, const int* st0, const int* st1, cf* X,
                            int* st, int* used, long long per_slot, int n_sc, long long n_slot, hipStream_t s) {
  const long long total = n_slot * per_slot;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dn_select, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, res, X0, X1, st0, st1, X, st,
                     used, per_slot, n_sc, total);
  return hipGetLastError();
}

}  // namespace pusch
