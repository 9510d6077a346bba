// Least-squares channel estimation on block-type pilot symbols (Sec. II,
// CHE; Table 1, row "CHE": an element-wise division per beam and UE), as a
// stand-alone kernel writing H[k][l][b].  The estimate itself (comb pilot
// positions in closed form, LS division, merge and linear interpolation)
// lives in comb_ls.h, shared with the detection kernel that estimates on the
// fly inside the fused slot.
//
// One thread per (subcarrier, UE, pair of beams): consecutive threads write
// consecutive 16-byte chunks of H and read the beams of one pilot RE
// contiguously from the RE-major grid.  grid.y walks the batch, so the index
// arithmetic inside a batch item stays 32-bit.
#include "comb_ls.h"
#include "kernels.h"

namespace pusch {
namespace {

template <int NBV>
__global__ __launch_bounds__(256) void k_chest(const cf* __restrict__ Y, const cf* __restrict__ P, cf* __restrict__ H,
                                               ChestGeom g, long long batch, int per_item) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= per_item) return;
  const int nb = g.n_beams, nue = g.n_ue, nsc = g.n_sc;
  const int nbc = nb / NBV;
  const int bc = idx % nbc;
  const int r = idx / nbc;
  const int l = r % nue;
  const int k = r / nue;
  for (long long bi = blockIdx.y; bi < batch; bi += gridDim.y) {
    cf h[NBV];
    ls_estimate<NBV>(h, Y + bi * g.y_batch, g, P + bi * g.p_batch, k, l, bc * NBV);
    cf* dst = H + bi * g.h_batch + ((long long)k * nue + l) * nb + bc * NBV;
#pragma unroll
    for (int e = 0; e < NBV; ++e) dst[e] = h[e];
  }
}

__global__ __launch_bounds__(256) void k_comb_table(int4* __restrict__ tab, int nsc, int nue, int npil) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nsc * nue) return;
  const int l = idx % nue, k = idx / nue;
  const CombBracket c = comb_bracket(k, l, nue, npil, nsc);
  tab[idx] = make_int4(c.lo, c.hi, (int)(c.mlo | (c.mhi << 8)), __float_as_int(c.w));
}

}  // namespace

hipError_t launch_comb_table(int4* tab, int n_sc, int n_ue, int n_pilot, hipStream_t s) {
  const int n = n_sc * n_ue;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_comb_table, dim3((n + 255) / 256), dim3(256), 0, s, tab, n_sc, n_ue, n_pilot);
  return hipGetLastError();
}

hipError_t launch_chest(const cf* Y, const cf* pilots, cf* H, const ChestGeom& g, long long batch, hipStream_t s) {
  if (batch <= 0 || g.n_sc <= 0) return hipSuccess;
  const bool pair = (g.n_beams % 2) == 0;
  const int per_item = g.n_sc * g.n_ue * (pair ? g.n_beams / 2 : g.n_beams);
  const dim3 grid((unsigned)((per_item + 255) / 256), (unsigned)(batch < 65535 ? batch : 65535));
  if (pair)
    hipLaunchKernelGGL(k_chest<2>, grid, dim3(256), 0, s, Y, pilots, H, g, batch, per_item);
  else
    hipLaunchKernelGGL(k_chest<1>, grid, dim3(256), 0, s, Y, pilots, H, g, batch, per_item);
  return hipGetLastError();
}

}  // namespace pusch
