// Device-side LS channel estimate of one UE at one subcarrier from comb
// pilots (Sec. II, CHE): the stand-alone estimation kernel evaluates it
// directly, and the kernel that builds the interpolation taps of the fused
// slot uses the same brackets.
//
// On pilot symbol j, subcarrier k carries UE (k + j*step) mod n_ue's pilot,
// step = comb_step(g) (n_ue / n_pilot, or 0 for the aligned comb), so UE l's
// pilot subcarriers on symbol j are the
// residue class r_j = (l - j*step) mod n_ue.  The nearest pilot positions
// around k follow in closed form, together with the set of pilot symbols
// that put UE l's pilot there.  The LS value at a position is
// y * conj(p) / |p|^2, averaged over those pilot symbols; between the two
// nearest positions the estimate is linear in k, beyond the outermost
// positions it is held.
#pragma once

#include "kernels.h"

namespace pusch {

// a mod m in [0, m) for |a| < 2^20, with inv_m = 1/m: a float quotient
// corrected by one step (avoids the integer division sequence).
__device__ __forceinline__ int fmod_pos(int a, int m, float inv_m) {
  int r = a - (int)floorf((float)a * inv_m) * m;
  r = r < 0 ? r + m : r;
  return r >= m ? r - m : r;
}

// Hardware reciprocal (v_rcp_f32, within 1 ulp).
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

struct CombBracket {
  int lo, hi;          // nearest pilot subcarriers of the UE at or below / at or above k
  unsigned mlo, mhi;   // pilot symbols whose pilot for the UE sits at lo / hi
  float w;             // interpolation weight of hi: (k - lo) / (hi - lo), 0 when lo == hi
};

__device__ __forceinline__ CombBracket comb_bracket(int k, int l, int nue, int npil, int nsc, int step) {
  const float inv = fast_rcp((float)nue);
  int lo = -1, hi = 0x7fffffff;
  unsigned mlo = 0, mhi = 0;
  for (int j = 0; j < npil; ++j) {
    const int rj = fmod_pos(l - j * step, nue, inv);
    const int plo = k - fmod_pos(k - rj, nue, inv);
    const int phi = k + fmod_pos(rj - k, nue, inv);
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

// Element offset of pilot symbol j's grid, j taken per lane (selects, not a
// dynamically indexed kernel argument).
__device__ __forceinline__ long long pilot_grid(const ChestGeom& g, int j) {
  const int s = j == 0 ? g.pilot_sym[0] : (j == 1 ? g.pilot_sym[1] : (j == 2 ? g.pilot_sym[2] : g.pilot_sym[3]));
  return (long long)s * g.y_sym;
}

// LS value at pilot subcarrier p for NBV consecutive beams b0.. of an
// RE-major grid holding the received pilot symbols, P = [n_pilot][n_sc]
// pilot values.
template <int NBV>
__device__ __forceinline__ void ls_at(cf (&out)[NBV], const cf* __restrict__ Y, const ChestGeom& g,
                                      const cf* __restrict__ P, unsigned mask, int p, int b0) {
  const int nb = g.n_beams, nsc = g.n_sc;
  float sr[NBV], si[NBV];
#pragma unroll
  for (int e = 0; e < NBV; ++e) sr[e] = si[e] = 0.f;
  for (unsigned m = mask; m; m &= m - 1) {
    const int j = __ffs(m) - 1;
    const cf pv = P[j * nsc + p];
    const float inv = fast_rcp(pv.r * pv.r + pv.i * pv.i);
    const cf* y = Y + pilot_grid(g, j) + (p * nb + b0);
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

template <int NBV>
__device__ __forceinline__ void lerp(cf (&lo)[NBV], const cf (&hi)[NBV], float w) {
#pragma unroll
  for (int e = 0; e < NBV; ++e)
    lo[e] = cf{__builtin_fmaf(w, hi[e].r - lo[e].r, lo[e].r), __builtin_fmaf(w, hi[e].i - lo[e].i, lo[e].i)};
}

// Interpolated LS estimate at subcarrier k for NBV consecutive beams.
template <int NBV>
__device__ __forceinline__ void ls_estimate(cf (&out)[NBV], const cf* __restrict__ Y, const ChestGeom& g,
                                            const cf* __restrict__ P, int k, int l, int b0) {
  const CombBracket c = comb_bracket(k, l, g.n_ue, g.n_pilot, g.n_sc, comb_step(g));
  ls_at<NBV>(out, Y, g, P, c.mlo, c.lo, b0);
  if (c.hi != c.lo) {
    cf vhi[NBV];
    ls_at<NBV>(vhi, Y, g, P, c.mhi, c.hi, b0);
    lerp<NBV>(out, vhi, c.w);
  }
}

}  // namespace pusch
