// MMSE MIMO detection (Eq. 2) per subcarrier: G = H^H H + sigma^2 I,
// Cholesky G = L L^H in Crout order (column by column, Sec. V-C), then for
// every data symbol the matched filter b = H^H y, forward substitution
// L z = b and back substitution L^H x = z.
//
// The paper runs many independent small decompositions per core between
// barriers (Sec. VI).  Here one wavefront handles 64/LPS subcarriers at once;
// each subcarrier owns LPS = pow2 >= n_ue lanes and lane i holds row i of G,
// later of L, in registers.  The subcarriers' H blocks and data-symbol beam
// vectors are staged in LDS (rows padded so the broadcast and strided reads
// of a wavefront stay conflict-free), the Crout column step broadcasts row j
// of L inside the lane group with cross-lane shuffles, and the substitutions
// run column-oriented over all data symbols at once, so the factor is
// computed once per subcarrier and reused for every symbol.
#include <cmath>

#include "kernels.h"

namespace pusch {
namespace {

constexpr int kMaxD = 16;  // data symbols per kernel call (host splits larger requests)
constexpr int kDCh = 4;    // data symbols staged in LDS at a time

struct LdsGeom {
  int hrow, hgrp;  // H rows (beams) and per-subcarrier stride, in cf
  int lrow, lgrp;  // L rows / per-subcarrier stride (aliases the H region)
  int region;      // cf size of the H / L region
  int yg, ydd;     // Y per-subcarrier stride and per-symbol stride
  int total;       // cf size of the whole LDS buffer
};

template <int LPS>
__global__ __launch_bounds__(64) void k_mmse(const cf* __restrict__ H, const cf* __restrict__ Y, cf* __restrict__ Xh,
                                             int* __restrict__ st, MmseGeom g, LdsGeom lg, long long nblk,
                                             int nblk_batch) {
  extern __shared__ cf sm[];
  constexpr int SPW = 64 / LPS;
  const int lane = threadIdx.x;
  const int grp = lane / LPS, i = lane % LPS, gbase = grp * LPS;
  const int nb = g.n_beams, nue = g.n_ue, nsc = g.n_sc, nd = g.n_data;
  cf* Hs = sm;
  cf* Ls = sm;
  cf* Ys = sm + lg.region;
  const int irow = i < nue ? i : nue - 1;

  for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const long long bi = blk / nblk_batch;
    const int k0 = (int)(blk - bi * nblk_batch) * SPW;
    const int cnt = min(SPW, nsc - k0);
    const int k = k0 + grp;
    const bool valid = grp < cnt;

    __syncthreads();
    {
      const cf* src = H + bi * g.h_batch + (long long)k0 * nue * nb;
      const int n = cnt * nue * nb;
      for (int e = lane; e < n; e += 64) {
        const int b = e % nb, r = e / nb;
        Hs[(r / nue) * lg.hgrp + (r % nue) * lg.hrow + b] = src[e];
      }
    }
    __syncthreads();

    const cf* hi_row = Hs + grp * lg.hgrp + irow * lg.hrow;
    const cf* hg = Hs + grp * lg.hgrp;

    // Gram row i: G_ij = sum_b conj(H_bi) H_bj (+ sigma^2 on the diagonal)
    cf G[LPS];
#pragma unroll
    for (int j = 0; j < LPS; ++j) G[j] = cf{0.f, 0.f};
    for (int b = 0; b < nb; ++b) {
      const cf a = hi_row[b];
#pragma unroll
      for (int j = 0; j < LPS; ++j) {
        if (j < nue) {
          const cf c = hg[j * lg.hrow + b];
          G[j].r += a.r * c.r + a.i * c.i;
          G[j].i += a.r * c.i - a.i * c.r;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < LPS; ++j)
      if (j == i) G[j].r += g.sigma2;

    // matched filter r_d = H^H y_d for every data symbol
    cf rr[kMaxD];
#pragma unroll
    for (int d = 0; d < kMaxD; ++d) rr[d] = cf{0.f, 0.f};
#pragma unroll
    for (int c = 0; c < kMaxD / kDCh; ++c) {
      if (c * kDCh >= nd) continue;
      __syncthreads();
      for (int dd = 0; dd < kDCh; ++dd) {
        const int d = c * kDCh + dd;
        if (d >= nd) break;
        const cf* src = Y + bi * g.y_batch + g.y_sym[d] + (long long)k0 * nb;
        const int n = cnt * nb;
        for (int e = lane; e < n; e += 64) Ys[dd * lg.ydd + (e / nb) * lg.yg + (e % nb)] = src[e];
      }
      __syncthreads();
      const cf* yg = Ys + grp * lg.yg;
      for (int b = 0; b < nb; ++b) {
        const cf a = hi_row[b];
#pragma unroll
        for (int dd = 0; dd < kDCh; ++dd) {
          const cf y = yg[dd * lg.ydd + b];
          cf& o = rr[c * kDCh + dd];
          o.r += a.r * y.r + a.i * y.i;
          o.i += a.r * y.i - a.i * y.r;
        }
      }
    }

    // Cholesky-Crout: column j uses row j of L (lane j of the group)
    bool fail = false;
    float invd = 0.f;
    cf L[LPS];
#pragma unroll
    for (int j = 0; j < LPS; ++j) L[j] = G[j];
#pragma unroll
    for (int j = 0; j < LPS; ++j) {
      if (j >= nue) continue;
      cf t = L[j];
#pragma unroll
      for (int m = 0; m < j; ++m) {
        const float cr = __shfl(L[m].r, gbase + j);
        const float ci = __shfl(L[m].i, gbase + j);
        t.r -= L[m].r * cr + L[m].i * ci;  // L_im * conj(L_jm)
        t.i -= L[m].i * cr - L[m].r * ci;
      }
      const float dpiv = __shfl(t.r, gbase + j);
      fail = fail || !(dpiv > 0.f) || !(dpiv <= 3.402823466e38f);
      const float ljj = sqrtf(dpiv);
      const float inv = 1.0f / ljj;
      if (i == j) {
        L[j] = cf{ljj, 0.f};
        invd = inv;
      } else if (i > j) {
        L[j] = cf{t.r * inv, t.i * inv};
      } else {
        L[j] = cf{0.f, 0.f};
      }
    }

    // rows of L to LDS (reusing the H region) for the transposed reads of
    // the back substitution
    __syncthreads();
#pragma unroll
    for (int m = 0; m < LPS; ++m) Ls[grp * lg.lgrp + i * lg.lrow + m] = L[m];
    __syncthreads();

    // forward substitution L z = r, column-oriented
#pragma unroll
    for (int m = 0; m < LPS; ++m) {
      if (m >= nue) continue;
#pragma unroll
      for (int d = 0; d < kMaxD; ++d) {
        if (d >= nd) continue;
        const float zr = __shfl(rr[d].r * invd, gbase + m);
        const float zi = __shfl(rr[d].i * invd, gbase + m);
        if (i == m) {
          rr[d] = cf{zr, zi};
        } else if (i > m) {
          rr[d].r -= L[m].r * zr - L[m].i * zi;
          rr[d].i -= L[m].r * zi + L[m].i * zr;
        }
      }
    }
    // back substitution L^H x = z: x_m = (z_m - sum_{n>m} conj(L_nm) x_n) / L_mm
#pragma unroll
    for (int m = LPS - 1; m >= 0; --m) {
      if (m >= nue) continue;
      const cf lmi = Ls[grp * lg.lgrp + m * lg.lrow + i];
#pragma unroll
      for (int d = 0; d < kMaxD; ++d) {
        if (d >= nd) continue;
        const float xr = __shfl(rr[d].r * invd, gbase + m);
        const float xi = __shfl(rr[d].i * invd, gbase + m);
        if (i == m) {
          rr[d] = cf{xr, xi};
        } else if (i < m) {
          rr[d].r -= lmi.r * xr + lmi.i * xi;  // conj(L_mi) * x_m
          rr[d].i -= lmi.r * xi - lmi.i * xr;
        }
      }
    }

    if (valid && i < nue) {
      cf* dst = Xh + bi * g.x_batch + (long long)k * nue + i;
#pragma unroll
      for (int d = 0; d < kMaxD; ++d) {
        if (d >= nd) continue;
        dst[(long long)d * nsc * nue] = fail ? cf{0.f, 0.f} : rr[d];
      }
    }
    if (valid && i == 0 && st) st[bi * g.st_batch + k] = fail ? 1 : 0;
  }
}

LdsGeom lds_geom(int lps, int nb, int nue) {
  const int spw = 64 / lps;
  LdsGeom lg;
  lg.hrow = nb | 1;
  lg.hgrp = nue * lg.hrow + 1;
  lg.lrow = lps + 1;
  lg.lgrp = lps * lg.lrow + 1;
  lg.region = spw * (lg.hgrp > lg.lgrp ? lg.hgrp : lg.lgrp);
  lg.yg = nb | 1;
  lg.ydd = spw * lg.yg + 1;
  lg.total = lg.region + kDCh * lg.ydd;
  return lg;
}

template <int LPS>
hipError_t launch_lps(const cf* H, const cf* Y, cf* Xh, int* st, const MmseGeom& g, long long batch, hipStream_t s) {
  constexpr int SPW = 64 / LPS;
  const LdsGeom lg = lds_geom(LPS, g.n_beams, g.n_ue);
  const int nblk_batch = (g.n_sc + SPW - 1) / SPW;
  const long long nblk = batch * nblk_batch;
  if (nblk <= 0) return hipSuccess;
  long long blocks = nblk;
  if (blocks > (1LL << 30)) blocks = 1LL << 30;
  hipLaunchKernelGGL(k_mmse<LPS>, dim3((unsigned)blocks), dim3(64), (size_t)lg.total * sizeof(cf), s, H, Y, Xh, st, g,
                     lg, nblk, nblk_batch);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mmse(const cf* H, const cf* Y, cf* Xhat, int* status, const MmseGeom& g, long long batch,
                       hipStream_t s) {
  if (g.n_data > kMaxD) return hipErrorInvalidValue;
  if (g.n_ue <= 1) return launch_lps<1>(H, Y, Xhat, status, g, batch, s);
  if (g.n_ue <= 2) return launch_lps<2>(H, Y, Xhat, status, g, batch, s);
  if (g.n_ue <= 4) return launch_lps<4>(H, Y, Xhat, status, g, batch, s);
  if (g.n_ue <= 8) return launch_lps<8>(H, Y, Xhat, status, g, batch, s);
  if (g.n_ue <= 16) return launch_lps<16>(H, Y, Xhat, status, g, batch, s);
  if (g.n_ue <= 32) return launch_lps<32>(H, Y, Xhat, status, g, batch, s);
  return hipErrorInvalidValue;
}

}  // namespace pusch
