// Least-squares channel estimation on block-type pilot symbols (Sec. II,
// CHE; Table 1, row "CHE": an element-wise division per beam and UE).
//
// The UEs share each pilot symbol as a frequency comb: on pilot symbol j,
// subcarrier k carries UE (k + j*step) mod n_ue's pilot, step = n_ue/n_pilot.
// UE l's pilot subcarriers are therefore the residues r_j = (l - j*step) mod
// n_ue of every pilot symbol, and the nearest pilot positions on either side
// of any k follow in closed form -- no sorted position list is built.  The LS
// value at a pilot position is y * conj(p) / |p|^2, averaged over the pilot
// symbols that hit the same subcarrier; between the two nearest positions the
// estimate is interpolated linearly, beyond the outermost ones it is held.
//
// One thread per output element H[k][l][b] (b fastest, so stores coalesce and
// the beams of one pilot RE are read contiguously from the RE-major grid).
#include "kernels.h"

namespace pusch {
namespace {

__device__ __forceinline__ int pmod(int a, int m) {
  const int r = a % m;
  return r < 0 ? r + m : r;
}

__global__ __launch_bounds__(256) void k_chest(const cf* __restrict__ Y, const cf* __restrict__ P, cf* __restrict__ H,
                                               ChestGeom g, long long total) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int nb = g.n_beams, nue = g.n_ue, nsc = g.n_sc, np = g.n_pilot;
  const int b = (int)(idx % nb);
  const long long q = idx / nb;
  const int l = (int)(q % nue);
  const long long q2 = q / nue;
  const int k = (int)(q2 % nsc);
  const long long bi = q2 / nsc;
  const int step = nue / np;

  int lo = -1, hi = 0x7fffffff;
  for (int j = 0; j < np; ++j) {
    const int rj = pmod(l - j * step, nue);
    const int plo = k - pmod(k - rj, nue);
    const int phi = k + pmod(rj - k, nue);
    if (plo >= 0 && plo > lo) lo = plo;
    if (phi < nsc && phi < hi) hi = phi;
  }
  if (lo < 0) lo = hi;            // left of the first pilot: hold
  if (hi == 0x7fffffff) hi = lo;  // right of the last pilot: hold

  const cf* Yb = Y + bi * g.y_batch;
  const cf* Pb = P + bi * g.p_batch;
  cf v[2];
  const int pos[2] = {lo, hi};
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int p = pos[e];
    float sr = 0.f, si = 0.f;
    int cnt = 0;
    for (int j = 0; j < np; ++j) {
      if (pmod(p + j * step, nue) != l) continue;
      const cf y = Yb[g.y_pilot[j] + (long long)p * nb + b];
      const cf pv = Pb[(long long)j * nsc + p];
      const float inv = 1.0f / (pv.r * pv.r + pv.i * pv.i);
      sr += (y.r * pv.r + y.i * pv.i) * inv;  // y * conj(p) / |p|^2
      si += (y.i * pv.r - y.r * pv.i) * inv;
      ++cnt;
    }
    const float ic = 1.0f / (float)cnt;
    v[e] = cf{sr * ic, si * ic};
  }
  cf h = v[0];
  if (hi != lo) {
    const float w = (float)(k - lo) / (float)(hi - lo);
    h = cf{v[0].r + w * (v[1].r - v[0].r), v[0].i + w * (v[1].i - v[0].i)};
  }
  H[bi * g.h_batch + ((long long)k * nue + l) * nb + b] = h;
}

}  // namespace

hipError_t launch_chest(const cf* Y, const cf* pilots, cf* H, const ChestGeom& g, long long batch, hipStream_t s) {
  const long long total = batch * g.n_sc * (long long)g.n_ue * g.n_beams;
  if (total <= 0) return hipSuccess;
  const long long blocks = (total + 255) / 256;
  hipLaunchKernelGGL(k_chest, dim3((unsigned)blocks), dim3(256), 0, s, Y, pilots, H, g, total);
  return hipGetLastError();
}

}  // namespace pusch
