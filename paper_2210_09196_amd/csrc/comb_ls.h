// Device-side LS channel estimate of one UE at one subcarrier from comb
// pilots (Sec. II, CHE), shared by the stand-alone estimation kernel and the
// detection kernel that estimates on the fly inside the fused slot.
//
// On pilot symbol j, subcarrier k carries UE (k + j*step) mod n_ue's pilot,
// step = n_ue / n_pilot, so UE l's pilot subcarriers on symbol j are the
// residue class r_j = (l - j*step) mod n_ue.  The nearest pilot positions
// around k follow in closed form, together with the set of pilot symbols
// that put UE l's pilot there.  The LS value at a position is
// y * conj(p) / |p|^2, averaged over those pilot symbols; between the two
// nearest positions the estimate is linear in k, beyond the outermost
// positions it is held.
#pragma once

#include "kernels.h"

namespace pusch {

__device__ __forceinline__ int pmod(int a, int m) {
  const int r = a % m;
  return r < 0 ? r + m : r;
}

// Hardware reciprocal (v_rcp_f32, within 1 ulp).
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

struct CombBracket {
  int lo, hi;          // nearest pilot subcarriers of the UE at or below / at or above k
  unsigned mlo, mhi;   // pilot symbols whose pilot for the UE sits at lo / hi
  float w;             // interpolation weight of hi: (k - lo) / (hi - lo), 0 when lo == hi
};

__device__ __forceinline__ CombBracket comb_bracket(int k, int l, int nue, int npil, int nsc) {
  const int step = nue / npil;
  int lo = -1, hi = 0x7fffffff;
  unsigned mlo = 0, mhi = 0;
  for (int j = 0; j < npil; ++j) {
    const int rj = pmod(l - j * step, nue);
    const int plo = k - pmod(k - rj, nue);
    const int phi = k + pmod(rj - k, nue);
    if (plo >= 0) {
      if (plo > lo) {
        lo = plo;
        mlo = 1u << j;
      } else if (plo == lo) {
        mlo |= 1u << j;
      }
    }
    if (phi < nsc) {
      if (phi < hi) {
        hi = phi;
        mhi = 1u << j;
      } else if (phi == hi) {
        mhi |= 1u << j;
      }
    }
  }
  if (lo < 0) {  // left of the first pilot: hold
    lo = hi;
    mlo = mhi;
  }
  if (hi == 0x7fffffff) {  // right of the last pilot: hold
    hi = lo;
    mhi = mlo;
  }
  CombBracket c;
  c.lo = lo;
  c.hi = hi;
  c.mlo = mlo;
  c.mhi = mhi;
  c.w = hi != lo ? (float)(k - lo) * fast_rcp((float)(hi - lo)) : 0.f;
  return c;
}

__device__ __forceinline__ float inv_count(unsigned mask) {
  const int n = __popc(mask);
  return n == 1 ? 1.f : (n == 2 ? 0.5f : (n == 3 ? (1.f / 3.f) : 0.25f));
}

// LS value at pilot subcarrier p for NBV consecutive beams b0.. of an
// RE-major grid holding the received pilot symbols (y_pilot[j] = element
// offset of pilot symbol j's grid), P = [n_pilot][n_sc] pilot values.
template <int NBV>
__device__ __forceinline__ void ls_at(cf (&out)[NBV], const cf* __restrict__ Y, const long long* y_pilot,
                                      const cf* __restrict__ P, unsigned mask, int p, int b0, int nb, int nsc) {
  float sr[NBV], si[NBV];
#pragma unroll
  for (int e = 0; e < NBV; ++e) sr[e] = si[e] = 0.f;
  for (unsigned m = mask; m; m &= m - 1) {
    const int j = __ffs(m) - 1;
    const cf pv = P[(long long)j * nsc + p];
    const float inv = fast_rcp(pv.r * pv.r + pv.i * pv.i);
    const cf* y = Y + y_pilot[j] + (long long)p * nb + b0;
#pragma unroll
    for (int e = 0; e < NBV; ++e) {
      const cf v = y[e];
      sr[e] += __builtin_fmaf(v.r, pv.r, v.i * pv.i) * inv;  // y * conj(p) / |p|^2
      si[e] += __builtin_fmaf(v.i, pv.r, -v.r * pv.i) * inv;
    }
  }
  const float ic = inv_count(mask);
#pragma unroll
  for (int e = 0; e < NBV; ++e) out[e] = cf{sr[e] * ic, si[e] * ic};
}

// The same value from grids that already hold y * conj(p) / |p|^2 per RE
// (the fused slot divides in the beamforming epilogue).
template <int NBV>
__device__ __forceinline__ void merged_at(cf (&out)[NBV], const cf* __restrict__ LS, const long long* off,
                                          unsigned mask, int p, int b0, int nb) {
  float sr[NBV], si[NBV];
#pragma unroll
  for (int e = 0; e < NBV; ++e) sr[e] = si[e] = 0.f;
  for (unsigned m = mask; m; m &= m - 1) {
    const int j = __ffs(m) - 1;
    const cf* v = LS + off[j] + (long long)p * nb + b0;
#pragma unroll
    for (int e = 0; e < NBV; ++e) {
      sr[e] += v[e].r;
      si[e] += v[e].i;
    }
  }
  const float ic = inv_count(mask);
#pragma unroll
  for (int e = 0; e < NBV; ++e) out[e] = cf{sr[e] * ic, si[e] * ic};
}

template <int NBV>
__device__ __forceinline__ void lerp(cf (&lo)[NBV], const cf (&hi)[NBV], float w) {
#pragma unroll
  for (int e = 0; e < NBV; ++e)
    lo[e] = cf{__builtin_fmaf(w, hi[e].r - lo[e].r, lo[e].r), __builtin_fmaf(w, hi[e].i - lo[e].i, lo[e].i)};
}

// Interpolated LS estimate at subcarrier k for NBV consecutive beams.
template <int NBV>
__device__ __forceinline__ void ls_estimate(cf (&out)[NBV], const cf* __restrict__ Y, const long long* y_pilot,
                                            const cf* __restrict__ P, int k, int l, int b0, int nb, int nue,
                                            int npil, int nsc) {
  const CombBracket c = comb_bracket(k, l, nue, npil, nsc);
  ls_at<NBV>(out, Y, y_pilot, P, c.mlo, c.lo, b0, nb, nsc);
  if (c.hi != c.lo) {
    cf vhi[NBV];
    ls_at<NBV>(vhi, Y, y_pilot, P, c.mhi, c.hi, b0, nb, nsc);
    lerp<NBV>(out, vhi, c.w);
  }
}

}  // namespace pusch
