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
  const int nb = g.n_beams, nue = g.n_ue;
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

__global__ __launch_bounds__(256) void k_comb_taps(int2* __restrict__ tab, ChestGeom g, int ntap) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.n_sc * g.n_ue) return;
  const int l = idx % g.n_ue, k = idx / g.n_ue;
  const CombBracket c = comb_bracket(k, l, g.n_ue, g.n_pilot, g.n_sc, comb_step(g));
  // lo end: average over the pilot symbols in mlo, times (1 - w); hi end
  // likewise with w (absent when the estimate is held, lo == hi)
  const bool two = c.hi != c.lo;
  const float wlo = (two ? 1.f - c.w : 1.f) * inv_count(c.mlo);
  const float whi = c.w * inv_count(c.mhi);
  int2* dst = tab + (long long)idx * ntap;
  int t = 0, first = -1;
  for (unsigned m = c.mlo; m; m &= m - 1) {
    const int off = (int)pilot_grid(g, __ffs(m) - 1) + c.lo * g.n_beams;
    first = first < 0 ? off : first;
    dst[t++] = make_int2(off, __float_as_int(wlo));
  }
  if (two)
    for (unsigned m = c.mhi; m; m &= m - 1)
      dst[t++] = make_int2((int)pilot_grid(g, __ffs(m) - 1) + c.hi * g.n_beams, __float_as_int(whi));
  for (; t < ntap; ++t) dst[t] = make_int2(first, 0);
}

// Time-varying channel: taps of data symbol d (symbol index t.data_sym[d])
// for (k, l), laid out tab[((d * n_sc + k) * n_ue + l) * kTimeTaps + t].  Between the
// pilot symbols a < s < b around it the estimate is ((b - s) H_a + (s - a) H_b)
// / (b - a), before the first pilot symbol H_0, after the last H_{n_pilot-1};
// H_j is UE l's estimate from pilot symbol j alone: linear between the
// nearest positions of its residue class on that symbol, held at the ends.
__global__ __launch_bounds__(256) void k_time_taps(int2* __restrict__ tab, ChestGeom g, TimeTapGeom t) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= t.n_data * g.n_sc * g.n_ue) return;
  const int l = idx % g.n_ue, k = (idx / g.n_ue) % g.n_sc, d = idx / (g.n_ue * g.n_sc);
  const int s = t.data_sym[d];
  // pilot symbols used and their time weights
  // (pilot symbol indices taken by selects: no dynamically indexed argument)
  auto psym = [&](int j) {
    return j == 0 ? g.pilot_sym[0] : (j == 1 ? g.pilot_sym[1] : (j == 2 ? g.pilot_sym[2] : g.pilot_sym[3]));
  };
  int jb = g.n_pilot - 1;  // the first pilot symbol after s, or the last one
#pragma unroll
  for (int j = kMaxPilots - 1; j >= 0; --j)
    if (j < g.n_pilot && psym(j) > s) jb = j;
  int ja = jb;
  float wb = 0.f;
  if (s > psym(g.n_pilot - 1)) {
    ja = jb = g.n_pilot - 1;  // after the last: hold
  } else if (jb > 0) {
    ja = jb - 1;  // between ja and jb
    wb = (float)(s - psym(ja)) / (float)(psym(jb) - psym(ja));
  }
  const int step = comb_step(g);
  const float inv = fast_rcp((float)g.n_ue);
  int2* dst = tab + (long long)idx * kTimeTaps;
  int n = 0;
  auto add = [&](int j, float wt) {
    const int rj = fmod_pos(l - j * step, g.n_ue, inv);  // UE l's residue class on pilot symbol j
    int lo = k - fmod_pos(k - rj, g.n_ue, inv);
    int hi = k + fmod_pos(rj - k, g.n_ue, inv);
    if (lo < 0) lo = hi;
    if (hi >= g.n_sc) hi = lo;
    const long long base = pilot_grid(g, j);
    if (hi == lo) {
      dst[n++] = make_int2((int)(base + (long long)lo * g.n_beams), __float_as_int(wt));
    } else {
      const float w = (float)(k - lo) / (float)(hi - lo);
      dst[n++] = make_int2((int)(base + (long long)lo * g.n_beams), __float_as_int(wt * (1.f - w)));
      dst[n++] = make_int2((int)(base + (long long)hi * g.n_beams), __float_as_int(wt * w));
    }
  };
  add(ja, 1.f - wb);
  if (jb != ja) add(jb, wb);
  const int first = dst[0].x;
  for (; n < kTimeTaps; ++n) dst[n] = make_int2(first, 0);
}

}  // namespace

hipError_t launch_time_taps(int2* tab, const ChestGeom& g, const TimeTapGeom& t, hipStream_t s) {
  const long long n = (long long)t.n_data * g.n_sc * g.n_ue;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_time_taps, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, g, t);
  return hipGetLastError();
}

namespace {
// Two pilot symbols, each UE's estimate from each alone (as for k_time_taps):
// tab[(k * n_ue + l) * 4 + 2 j + {0, 1}] = the (offset, weight) taps of pilot
// symbol j (the nearest positions below and above k of UE l's residue class
// on symbol j, linear in k; a hold gives (offset, 1) and (offset, 0)).
__global__ __launch_bounds__(256) void k_pair_taps(int2* __restrict__ tab, ChestGeom g) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.n_sc * g.n_ue) return;
  const int l = idx % g.n_ue, k = idx / g.n_ue;
  const int step = comb_step(g);
  const float inv = fast_rcp((float)g.n_ue);
  int2* dst = tab + (long long)idx * 4;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int rj = fmod_pos(l - j * step, g.n_ue, inv);  // UE l's residue class on pilot symbol j
    int lo = k - fmod_pos(k - rj, g.n_ue, inv);
    int hi = k + fmod_pos(rj - k, g.n_ue, inv);
    if (lo < 0) lo = hi;
    if (hi >= g.n_sc) hi = lo;
    const long long base = pilot_grid(g, j);
    const float w = hi == lo ? 0.f : (float)(k - lo) / (float)(hi - lo);
    dst[2 * j] = make_int2((int)(base + (long long)lo * g.n_beams), __float_as_int(1.f - w));
    dst[2 * j + 1] = make_int2((int)(base + (long long)hi * g.n_beams), __float_as_int(w));
  }
}
}  // namespace

hipError_t launch_pair_taps(int2* tab, const ChestGeom& g, hipStream_t s) {
  const long long n = (long long)g.n_sc * g.n_ue;
  if (n <= 0) return hipSuccess;
  if (g.n_pilot != 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pair_taps, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, g);
  return hipGetLastError();
}

int comb_taps(int n_ue, int n_pilot, bool aligned) {
  // pilot symbols j, j' put UE l's pilot on the same subcarriers when
  // (j - j') * step = 0 mod n_ue (step = n_ue / n_pilot, or 0 when aligned):
  // then a bracket end averages several of them
  const int step = aligned ? 0 : n_ue / n_pilot;
  for (int j = 1; j < n_pilot; ++j)
    if ((j * step) % n_ue == 0) return 2 * kMaxPilots;
  return 2;
}

hipError_t launch_comb_taps(int2* tab, const ChestGeom& g, int n_tap, hipStream_t s) {
  const int n = g.n_sc * g.n_ue;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_comb_taps, dim3((n + 255) / 256), dim3(256), 0, s, tab, g, n_tap);
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
