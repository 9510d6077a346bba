// Noise-variance estimation (Sec. II, NE; Table 1, row "NE"): the variance
// of the difference between each received pilot RE and the value that the
// estimated channel and the known pilot predict for it.
//
// The interpolated LS estimate passes through every pilot position, so the
// prediction at pilot RE (j, k) of UE l uses UE l's merged LS values at its
// other positions only: the nearest one below k and the nearest one above
// (weights linear in k), or the nearest one on the only side there is.  With
// weights w_i on positions holding c_i averaged LS values from pilots p_s,
// the difference r = y - p h has noise variance sigma^2 kappa per beam,
//   kappa = 1 + |p|^2 sum_i (w_i / c_i)^2 sum_{s at i} 1 / |p_s|^2,
// and the estimate is sum |r|^2 / (N_B sum kappa) over the pilot REs of a
// batch item.  Since y = p * LS(y), |r|^2 = |p|^2 |LS(y) - h|^2.
// Where c >= 2 pilot symbols carry UE l's pilot at k itself, the prediction
// is the mean of those c LS values at k (the same channel in every term, so
// the residual holds noise only, however selective the channel is); the RE's
// own noise is 1/c of that mean, so kappa = 1 - 2/c + |p|^2 / c^2 sum_s 1/|p_s|^2.
//
// k_noise_table finds every pilot RE's neighbours and weights (they depend
// on the geometry only: closed form per pilot symbol, the comb of residue
// classes mod n_ue), once per geometry.  Per call, k_noise_partial sums
// |r|^2 and N_B kappa over kNeParts fixed slices of an item's pilot REs and
// k_noise_final adds an item's slices and divides.  Every sum runs in a
// fixed order (no atomics), so the result does not depend on timing.
//
// Layout: BW lanes (a power of two) share one pilot RE, each taking NBV
// consecutive beams of its RE-major row, so a group reads whole rows.  Pilot
// REs are ordered subcarrier-major (s = k * n_pilot + j), so an RE's
// neighbours on other pilot symbols are a few REs away, and consecutive
// slices of an item run on one XCD (xcd_block): they share its L2 instead of
// fetching the same rows from HBM again.
#include "comb_ls.h"
#include "kernels.h"

namespace pusch {
namespace {

constexpr int kNeThreads = 256;

__device__ __forceinline__ int pos_mod(int a, int m) {
  const int r = a % m;
  return r < 0 ? r + m : r;
}

struct NeNeighbours {
  int lo, hi;          // nearest pilot subcarriers of the UE strictly below / above k (-1 / n_sc: none)
  unsigned mlo, mhi;   // pilot symbols whose pilot for the UE sits there
  float wlo, whi;      // prediction weights
};

__device__ __forceinline__ NeNeighbours ne_neighbours(int k, int l, int nue, int npil, int nsc, int step) {
  NeNeighbours n;
  n.lo = -1;
  n.hi = nsc;
  n.mlo = n.mhi = 0;
  for (int j = 0; j < npil; ++j) {
    const int rj = pos_mod(l - j * step, nue);            // UE l's residue class on pilot symbol j
    const int plo = (k - 1) - pos_mod(k - 1 - rj, nue);  // largest position < k in that class
    const int phi = (k + 1) + pos_mod(rj - k - 1, nue);  // smallest position > k
    if (plo >= 0) {
      if (plo > n.lo) {
        n.lo = plo;
        n.mlo = 1u << j;
      } else if (plo == n.lo) {
        n.mlo |= 1u << j;
      }
    }
    if (phi < nsc) {
      if (phi < n.hi) {
        n.hi = phi;
        n.mhi = 1u << j;
      } else if (phi == n.hi) {
        n.mhi |= 1u << j;
      }
    }
  }
  if (n.lo >= 0 && n.hi < nsc) {
    const float inv = 1.f / (float)(n.hi - n.lo);
    n.wlo = (float)(n.hi - k) * inv;
    n.whi = (float)(k - n.lo) * inv;
  } else {  // one side only: hold (the host guarantees at least one side)
    n.wlo = n.lo >= 0 ? 1.f : 0.f;
    n.whi = n.lo >= 0 ? 0.f : 1.f;
  }
  return n;
}

// LS value of pilot RE (j, p) for NBV consecutive beams: the grid value itself
// when the pilot symbols already hold LS values, else y conj(p) / |p|^2.
template <int NBV, bool LS>
__device__ __forceinline__ void ls_value(float (&vr)[NBV], float (&vi)[NBV], const cf* __restrict__ Yb,
                                         const ChestGeom& g, cf pv, int j, int p, int b0) {
  const cf* y = Yb + pilot_grid(g, j) + ((long long)p * g.n_beams + b0);
  const float inv = LS ? 1.f : 1.f / (pv.r * pv.r + pv.i * pv.i);
#pragma unroll
  for (int e = 0; e < NBV; ++e) {
    const cf v = y[e];
    vr[e] = LS ? v.r : (v.r * pv.r + v.i * pv.i) * inv;
    vi[e] = LS ? v.i : (v.i * pv.r - v.r * pv.i) * inv;
  }
}

// Mean LS value at position p over the pilot symbols in mask, accumulated
// with weight w into (hr, hi); returns sum_{s in mask} 1 / |p_s|^2.
template <int NBV, bool LS>
__device__ __forceinline__ float add_mean(float (&hr)[NBV], float (&hi)[NBV], const cf* __restrict__ Yb,
                                          const cf* __restrict__ Pb, const ChestGeom& g, unsigned mask, int p,
                                          float w, int b0) {
  const float wc = w / (float)__popc(mask);
  float q = 0.f;
  for (unsigned m = mask; m; m &= m - 1) {
    const int j = __ffs(m) - 1;
    const cf pv = Pb[(long long)j * g.n_sc + p];
    q += 1.f / (pv.r * pv.r + pv.i * pv.i);
    float vr[NBV], vi[NBV];
    ls_value<NBV, LS>(vr, vi, Yb, g, pv, j, p, b0);
#pragma unroll
    for (int e = 0; e < NBV; ++e) {
      hr[e] += wc * vr[e];
      hi[e] += wc * vi[e];
    }
  }
  return q;
}

__device__ __forceinline__ float2 wave_sum(float2 v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  return v;
}

// One table entry per pilot RE s = k * n_pilot + j: {lo | hi << 12 | mlo << 24 |
// mhi << 28, bits of wlo, bits of whi, k | j << 16 | self << 20}; a mask of 0
// marks a missing side (positions < 4096); self: the prediction is the mean
// at k itself (lo = k, mlo its pilot symbols, wlo = 1, no hi side).
__global__ __launch_bounds__(256) void k_noise_table(int4* __restrict__ tab, ChestGeom g) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.n_pilot * g.n_sc) return;
  const int k = s / g.n_pilot, j = s - k * g.n_pilot;
  const int step = comb_step(g);
  const int l = pos_mod(k + j * step, g.n_ue);
  unsigned here = 0;  // pilot symbols that put UE l's pilot at k
  for (int jj = 0; jj < g.n_pilot; ++jj)
    if (pos_mod(k + jj * step, g.n_ue) == l) here |= 1u << jj;
  if (__popc(here) >= 2) {
    tab[s] = make_int4(k | (int)(here << 24), __float_as_int(1.f), __float_as_int(0.f), k | j << 16 | 1 << 20);
    return;
  }
  const NeNeighbours n = ne_neighbours(k, l, g.n_ue, g.n_pilot, g.n_sc, step);
  const int lo = n.mlo ? n.lo : 0, hi = n.mhi ? n.hi : 0;
  tab[s] = make_int4(lo | hi << 12 | (int)(n.mlo << 24) | (int)(n.mhi << 28), __float_as_int(n.wlo),
                     __float_as_int(n.whi), k | j << 16);
}

// One workgroup per (item, slice): logical block id = (item - item0) * n_parts +
// slice, renumbered by xcd_block; part[item * kNeParts + slice] = (sum |r|^2,
// sum N_B kappa).
template <int NBV, bool LS>
__global__ __launch_bounds__(kNeThreads) void k_noise_partial(const cf* __restrict__ Y, const cf* __restrict__ P,
                                                              const int4* __restrict__ tab,
                                                              float2* __restrict__ part, ChestGeom g, int bw,
                                                              int n_parts, long long item0) {
  __shared__ float2 red[kNeThreads / 64];
  const int logical = xcd_block(blockIdx.x, gridDim.x);
  const int slice = logical % n_parts;
  const long long bi = item0 + logical / n_parts;
  const int nb = g.n_beams, nsc = g.n_sc;
  const int gl = threadIdx.x & (bw - 1);          // lane within the RE's group
  const int b0 = gl * NBV;                         // first beam of this lane
  const bool mine = b0 < nb;
  const int bb = mine ? b0 : 0;                    // lanes past the last beam read beam 0 and add nothing
  const int per_it = kNeThreads / bw;              // pilot REs per block per iteration
  const int n_re = g.n_pilot * nsc;
  const int stride = n_parts * per_it;
  const cf* Yb = Y + bi * g.y_batch;
  const cf* Pb = P + bi * g.p_batch;
  float num = 0.f, den = 0.f;
  for (int s = slice * per_it + (int)(threadIdx.x / bw); s < n_re; s += stride) {
    const int4 t = tab[s];
    const unsigned mlo = ((unsigned)t.x >> 24) & 15u, mhi = (unsigned)t.x >> 28;
    const int lo = t.x & 4095, hi = (t.x >> 12) & 4095;
    const int k = t.w & 0xffff, j = (t.w >> 16) & 15;
    const bool self = (t.w >> 20) & 1;
    float hr[NBV], hi_[NBV];
#pragma unroll
    for (int e = 0; e < NBV; ++e) hr[e] = hi_[e] = 0.f;
    float gain = 0.f, base = 1.f;  // kappa = base + |p|^2 gain
    if (self) base = 1.f - 2.f / (float)__popc(mlo);
    if (mlo) {
      const float wlo = __int_as_float(t.y);
      const float q = add_mean<NBV, LS>(hr, hi_, Yb, Pb, g, mlo, lo, wlo, bb);
      const float c = wlo / (float)__popc(mlo);
      gain += c * c * q;
    }
    if (mhi) {
      const float whi = __int_as_float(t.z);
      const float q = add_mean<NBV, LS>(hr, hi_, Yb, Pb, g, mhi, hi, whi, bb);
      const float c = whi / (float)__popc(mhi);
      gain += c * c * q;
    }
    const cf pv = Pb[(long long)j * nsc + k];
    const float pp = pv.r * pv.r + pv.i * pv.i;
    float vr[NBV], vi[NBV];
    ls_value<NBV, LS>(vr, vi, Yb, g, pv, j, k, bb);
    float e2 = 0.f;
#pragma unroll
    for (int e = 0; e < NBV; ++e) {
      const float dr = vr[e] - hr[e], di = vi[e] - hi_[e];
      e2 += dr * dr + di * di;
    }
    num += mine ? pp * e2 : 0.f;
    den += gl == 0 ? (float)nb * (base + pp * gain) : 0.f;
  }
  float2 v = wave_sum(make_float2(num, den));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float2 t = red[0];
#pragma unroll
    for (int w = 1; w < kNeThreads / 64; ++w) {
      t.x += red[w].x;
      t.y += red[w].y;
    }
    part[bi * kNeParts + slice] = t;
  }
}

// One wavefront per batch item: sigma2[item] = sum of its parts' |r|^2 / sum of N_B kappa
// (lane i adds parts i, i + 64, ... in order, then a fixed butterfly).
__global__ __launch_bounds__(256) void k_noise_final(const float2* __restrict__ part, float* __restrict__ sigma2,
                                                      int n_parts, long long batch) {
  const long long bi = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (bi >= batch) return;
  const int lane = threadIdx.x & 63;
  float2 v = make_float2(0.f, 0.f);
  for (int i = lane; i < n_parts; i += 64) {
    const float2 w = part[bi * kNeParts + i];
    v.x += w.x;
    v.y += w.y;
  }
  v = wave_sum(v);
  if (lane == 0) sigma2[bi] = v.x / v.y;
}

// Beams per lane and lanes per pilot RE (a power of two).
void ne_shape(int n_beams, int* nbv, int* bw) {
  *nbv = n_beams % 4 == 0 ? 4 : (n_beams % 2 == 0 ? 2 : 1);
  *bw = 1;
  while (*bw * *nbv < n_beams) *bw *= 2;
}

// One launch per run of at most 2^22 items (n_parts * items < 2^31 blocks).
template <int NBV, bool LS>
void launch_partial(const cf* Y, const cf* P, const int4* tab, float2* part, const ChestGeom& g, int bw, int n_parts,
                    long long batch, hipStream_t s) {
  constexpr long long kChunk = 1ll << 22;
  for (long long b0 = 0; b0 < batch; b0 += kChunk) {
    const long long items = batch - b0 < kChunk ? batch - b0 : kChunk;
    hipLaunchKernelGGL((k_noise_partial<NBV, LS>), dim3((unsigned)(items * n_parts)), dim3(kNeThreads), 0, s, Y, P,
                       tab, part, g, bw, n_parts, b0);
  }
}

template <bool LS>
void launch_partial_ls(int nbv, const cf* Y, const cf* P, const int4* tab, float2* part, const ChestGeom& g, int bw,
                       int n_parts, long long batch, hipStream_t s) {
  if (nbv == 4)
    launch_partial<4, LS>(Y, P, tab, part, g, bw, n_parts, batch, s);
  else if (nbv == 2)
    launch_partial<2, LS>(Y, P, tab, part, g, bw, n_parts, batch, s);
  else
    launch_partial<1, LS>(Y, P, tab, part, g, bw, n_parts, batch, s);
}

// Slices per batch item: one per block-iteration's worth of pilot REs, at most kNeParts.
int noise_parts(const ChestGeom& g) {
  int nbv, bw;
  ne_shape(g.n_beams, &nbv, &bw);
  const int per_it = kNeThreads / bw;
  const int want = (g.n_pilot * g.n_sc + per_it - 1) / per_it;
  return want < 1 ? 1 : (want > kNeParts ? kNeParts : want);
}

}  // namespace

size_t noise_table_bytes(int n_pilot, int n_sc) { return (size_t)n_pilot * n_sc * sizeof(int4); }

hipError_t launch_noise_table(int4* tab, const ChestGeom& g, hipStream_t s) {
  const int n_re = g.n_pilot * g.n_sc;
  if (n_re <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_noise_table, dim3((unsigned)((n_re + 255) / 256)), dim3(256), 0, s, tab, g);
  return hipGetLastError();
}

hipError_t launch_noise_est(const cf* Y, const cf* pilots, bool ls, const int4* tab, float2* part, float* sigma2,
                            const ChestGeom& g, long long batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  int nbv, bw;
  ne_shape(g.n_beams, &nbv, &bw);
  const int n_parts = noise_parts(g);
  if (ls)
    launch_partial_ls<true>(nbv, Y, pilots, tab, part, g, bw, n_parts, batch, s);
  else
    launch_partial_ls<false>(nbv, Y, pilots, tab, part, g, bw, n_parts, batch, s);
  if (hipError_t e = hipGetLastError()) return e;
  const long long blocks = (batch + 3) / 4;
  hipLaunchKernelGGL(k_noise_final, dim3((unsigned)blocks), dim3(256), 0, s, part, sigma2, n_parts, batch);
  return hipGetLastError();
}

}  // namespace pusch
