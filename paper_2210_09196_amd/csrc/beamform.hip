// Beamforming (Sec. II; Table 1, row "BF"): a complex matrix product with
// known coefficients, Y_i[n][b] = sum_a W[b][a] X_i[a][n], on gfx950 FP32
// matrix cores.
//
// The paper computes 4x4 output windows per core in registers (Sec. V-B).
// Here one wavefront owns an output tile of (16*MT beams) x 32 REs and walks
// the antenna axis four at a time with v_mfma_f32_16x16x4_f32.  The complex
// product is split into four real products on the interleaved operands,
//   Yr += Wr Xr - Wi Xi,  Yi += Wr Xi + Wi Xr,
// so a lane's single 8-byte load of X[a][n] feeds both the real and the
// imaginary MFMA without any de-interleaving pass.  Operand layouts of the
// 16x16x4 instruction: lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// receives D[4*(l/16)+v][l%16], v = 0..3.
#include "kernels.h"

namespace pusch {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kNT = 2;  // 16-column MFMA tiles per wavefront tile

template <int MT>
__global__ __launch_bounds__(64 * kWaves) void k_beamform(const cf* __restrict__ W, const cf* __restrict__ X,
                                                          cf* __restrict__ Y, int nb, int na, int nre,
                                                          long long ldx, long long sx, long long sy,
                                                          long long batch, long long ntn) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;  // A row / B column / D column inside a 16x16 tile
  const int kq = lane >> 4;   // A column / B row (antenna within the step of 4)
  const long long nwave = (long long)gridDim.x * kWaves;
  const int ksteps = (na + 3) >> 2;

  for (long long tile = (long long)blockIdx.x * kWaves + (threadIdx.x >> 6); tile < batch * ntn; tile += nwave) {
    const long long bi = tile / ntn;
    const int n0 = (int)(tile - bi * ntn) * (16 * kNT);
    const cf* Xb = X + bi * sx;
    f32x4 yr[MT][kNT], yi[MT][kNT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int t = 0; t < kNT; ++t) yr[m][t] = yi[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int ks = 0; ks < ksteps; ++ks) {
      const int a = ks * 4 + kq;
      const bool a_ok = a < na;
      cf xv[kNT];
#pragma unroll
      for (int t = 0; t < kNT; ++t) {
        const int n = n0 + t * 16 + col;
        xv[t] = (a_ok && n < nre) ? Xb[(long long)a * ldx + n] : cf{0.f, 0.f};
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int b = m * 16 + col;
        const cf wv = (a_ok && b < nb) ? W[b * na + a] : cf{0.f, 0.f};
        const float nwi = -wv.i;
#pragma unroll
        for (int t = 0; t < kNT; ++t) {
          yr[m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.r, xv[t].r, yr[m][t], 0, 0, 0);
          yr[m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(nwi, xv[t].i, yr[m][t], 0, 0, 0);
          yi[m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.r, xv[t].i, yi[m][t], 0, 0, 0);
          yi[m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.i, xv[t].r, yi[m][t], 0, 0, 0);
        }
      }
    }

    cf* Yb = Y + bi * sy;
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
      const int n = n0 + t * 16 + col;
      if (n >= nre) continue;
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int b = m * 16 + kq * 4 + v;
          if (b < nb) Yb[(long long)n * nb + b] = cf{yr[m][t][v], yi[m][t][v]};
        }
    }
  }
}

}  // namespace

hipError_t launch_beamform(const cf* W, const cf* X, cf* Y, int n_beams, int n_ant, int n_re, long long ldx,
                           long long sx, long long sy, long long batch, int n_cu, hipStream_t s) {
  if (batch <= 0 || n_re <= 0) return hipSuccess;
  const long long ntn = (n_re + 16 * kNT - 1) / (16 * kNT);
  const long long tiles = batch * ntn;
  long long blocks = (tiles + kWaves - 1) / kWaves;
  const long long cap = (long long)n_cu * 8;
  if (blocks > cap) blocks = cap;
  const dim3 grid((unsigned)blocks), block(64 * kWaves);
  const int mt = (n_beams + 15) / 16;
  switch (mt) {
    case 1: hipLaunchKernelGGL(k_beamform<1>, grid, block, 0, s, W, X, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ntn); break;
    case 2: hipLaunchKernelGGL(k_beamform<2>, grid, block, 0, s, W, X, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ntn); break;
    case 3: hipLaunchKernelGGL(k_beamform<3>, grid, block, 0, s, W, X, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ntn); break;
    case 4: hipLaunchKernelGGL(k_beamform<4>, grid, block, 0, s, W, X, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ntn); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pusch
