// C-ABI entry points of the PUSCH receive chain (declared in include/pusch.h):
// host-side argument validation, per-device immutable tables, workspace
// layout and the launch sequence of the fused slot.
#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "kernels.h"
#include "pusch.h"

using pusch::cf;

namespace {

constexpr int kMaxDevices = 64;
constexpr long long kMaxAnt = 1024;
constexpr int kMaxNeSc = 4096;  // noise estimation: subcarrier positions packed in 12 bits

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr int kSideStreams = PUSCH_CELL_STREAMS;

struct DeviceTables {
  std::once_flag once;
  int status = PUSCH_EHIP;
  cf* twiddles = nullptr;
  int n_cu = 1;
  std::mutex mu;
  std::map<std::pair<int, int>, cf*> dft_w;  // (n_beams, n_ant) -> device table
  // pusch_cells: side streams (default priority) and the fork / join events
  // that tie them to the caller's stream; cells_mu serialises the enqueue
  hipStream_t side[kSideStreams] = {};
  hipEvent_t fork = nullptr, fork_mmse = nullptr, join[kSideStreams] = {};
  std::mutex cells_mu;
  // per-geometry tables (interpolation taps of the fused detection,
  // noise-estimation neighbours), built on the library's own stream
  hipStream_t build = nullptr;
  std::map<std::vector<long long>, void*> geom;
  // pusch_cells: launch plans chosen by pusch_cells_tune, by cell set
  std::map<std::vector<long long>, pusch_cells_plan> plans;
};
DeviceTables g_dev[kMaxDevices];

int device_tables(DeviceTables** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PUSCH_EHIP;
  DeviceTables& t = g_dev[dev];
  std::call_once(t.once, [&t, dev]() {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) return;
    const pusch::TwiddleLayout lay = pusch::fft_twiddle_layout();
    std::vector<cf> host(lay.total);
    pusch::fft_fill_twiddles(host.data());
    void* d = nullptr;
    if (hipMalloc(&d, host.size() * sizeof(cf)) != hipSuccess) {
      t.status = PUSCH_ENOMEM;
      return;
    }
    if (hipMemcpy(d, host.data(), host.size() * sizeof(cf), hipMemcpyHostToDevice) != hipSuccess) return;
    t.twiddles = static_cast<cf*>(d);
    t.n_cu = ncu;
    if (hipEventCreateWithFlags(&t.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&t.fork_mmse, hipEventDisableTiming) != hipSuccess)
      return;
    for (int i = 0; i < kSideStreams; ++i)
      if (hipStreamCreateWithFlags(&t.side[i], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&t.join[i], hipEventDisableTiming) != hipSuccess)
        return;
    if (hipStreamCreateWithFlags(&t.build, hipStreamNonBlocking) != hipSuccess) return;
    t.status = PUSCH_OK;
  });
  *out = &t;
  return t.status;
}

// Built-in beamformer: rows 0..n_beams-1 of the unitary n_ant-point DFT,
// computed in FP64 on the host and rounded once to FP32.
int dft_beamformer(DeviceTables* t, int n_beams, int n_ant, const cf** out) {
  std::lock_guard<std::mutex> lock(t->mu);
  auto key = std::make_pair(n_beams, n_ant);
  auto it = t->dft_w.find(key);
  if (it != t->dft_w.end()) {
    *out = it->second;
    return PUSCH_OK;
  }
  std::vector<cf> host((size_t)n_beams * n_ant);
  const double two_pi = 6.283185307179586476925286766559;
  const double scale = 1.0 / std::sqrt((double)n_ant);
  for (int b = 0; b < n_beams; ++b)
    for (int a = 0; a < n_ant; ++a) {
      const double ang = -two_pi * (double)(((long)b * a) % n_ant) / (double)n_ant;
      host[(size_t)b * n_ant + a] = cf{(float)(std::cos(ang) * scale), (float)(std::sin(ang) * scale)};
    }
  void* d = nullptr;
  if (hipMalloc(&d, host.size() * sizeof(cf)) != hipSuccess) return PUSCH_ENOMEM;
  if (hipMemcpy(d, host.data(), host.size() * sizeof(cf), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return PUSCH_EHIP;
  }
  t->dft_w[key] = static_cast<cf*>(d);
  *out = static_cast<cf*>(d);
  return PUSCH_OK;
}

// Tables that depend on a slot geometry only, built once per geometry by
// their kernels on the library's stream (waited for there, so the caller's
// stream never waits on it) and kept until the process ends.
enum GeomTable { kCombTaps = 0, kNoiseTable = 1, kTimeTaps = 2, kPairTaps = 3 };

int geometry_table(DeviceTables* t, GeomTable kind, const pusch::ChestGeom& g, int n_tap, const void** out,
                   const pusch::TimeTapGeom* tt = nullptr) {
  std::vector<long long> key = {kind, g.n_sc, g.n_ue, g.n_pilot, g.comb_aligned};
  if (kind != kNoiseTable) {
    key.push_back(g.n_beams);
    key.push_back(g.y_sym);
    key.push_back(n_tap);
    for (int j = 0; j < g.n_pilot; ++j) key.push_back(g.pilot_sym[j]);
  }
  if (kind == kTimeTaps)
    for (int d = 0; d < tt->n_data; ++d) key.push_back(tt->data_sym[d]);
  std::lock_guard<std::mutex> lock(t->mu);
  auto it = t->geom.find(key);
  if (it != t->geom.end()) {
    *out = it->second;
    return PUSCH_OK;
  }
  const size_t bytes = kind == kCombTaps   ? (size_t)g.n_sc * g.n_ue * n_tap * sizeof(int2)
                       : kind == kTimeTaps ? (size_t)tt->n_data * g.n_sc * g.n_ue * pusch::kTimeTaps * sizeof(int2)
                       : kind == kPairTaps ? (size_t)g.n_sc * g.n_ue * 4 * sizeof(int2)
                                           : pusch::noise_table_bytes(g.n_pilot, g.n_sc);
  void* d = nullptr;
  if (hipMalloc(&d, bytes) != hipSuccess) return PUSCH_ENOMEM;
  const hipError_t e = kind == kCombTaps   ? pusch::launch_comb_taps(static_cast<int2*>(d), g, n_tap, t->build)
                       : kind == kTimeTaps ? pusch::launch_time_taps(static_cast<int2*>(d), g, *tt, t->build)
                       : kind == kPairTaps ? pusch::launch_pair_taps(static_cast<int2*>(d), g, t->build)
                                           : pusch::launch_noise_table(static_cast<int4*>(d), g, t->build);
  if (e != hipSuccess || hipStreamSynchronize(t->build) != hipSuccess) {
    (void)hipFree(d);
    return PUSCH_EHIP;
  }
  t->geom[key] = d;
  *out = d;
  return PUSCH_OK;
}

bool overlap(const void* a, long long abytes, const void* b, long long bbytes) {
  if (!a || !b || abytes <= 0 || bbytes <= 0) return false;
  const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + (uintptr_t)bbytes && pb < pa + (uintptr_t)abytes;
}

int hip_status(hipError_t e) { return e == hipSuccess ? PUSCH_OK : PUSCH_EHIP; }

// Device address of the allocation-free entry point's scratch array (below),
// looked up once per device with that device current.
struct ScratchAddr {
  std::once_flag once;
  int status = PUSCH_EHIP;
  unsigned char* ptr = nullptr;
};
ScratchAddr g_scratch_addr[kMaxDevices];
int scratch_address(unsigned char** out);

// ---------------------------------------------------------------- stage timing
struct Profile {
  std::mutex mu;
  bool active = false;
  int max_calls = 0;
  int calls = 0;
  std::vector<hipEvent_t> ev;  // (PUSCH_SLOT_STAGES + 1) per call
} g_prof;

constexpr int kEvPerCall = PUSCH_SLOT_STAGES + 1;

}  // namespace

extern "C" {

const char* pusch_strerror(int code) {
  switch (code) {
    case PUSCH_OK: return "success";
    case PUSCH_EINVAL: return "invalid argument";
    case PUSCH_EUNSUPPORTED: return "unsupported size or configuration";
    case PUSCH_EHIP: return "HIP runtime or launch failure";
    case PUSCH_ENOMEM: return "workspace too small or device allocation failed";
    default: return "unknown error code";
  }
}

int pusch_init(void) {
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  unsigned char* sp = nullptr;
  return scratch_address(&sp);
}

int pusch_fft(const pusch_c32* x, pusch_c32* X, int n_fft, int n_sc, long long batch, void* stream) {
  if (!x || !X || batch < 0) return PUSCH_EINVAL;
  if (pusch::fft_size_index(n_fft) < 0) return PUSCH_EUNSUPPORTED;
  if (n_sc < 0 || n_sc > n_fft) return PUSCH_EINVAL;
  const int out_len = n_sc == 0 ? n_fft : n_sc;
  const int shift = n_sc == 0 ? 0 : n_sc / 2;
  if ((const void*)x == (const void*)X) {
    if (out_len != n_fft) return PUSCH_EINVAL;
  } else if (overlap(x, batch * n_fft * 8LL, X, batch * out_len * 8LL)) {
    return PUSCH_EINVAL;
  }
  if (batch == 0) return PUSCH_OK;
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  return hip_status(pusch::launch_fft(reinterpret_cast<const cf*>(x), reinterpret_cast<cf*>(X), n_fft, batch, out_len,
                                      shift, out_len, t->twiddles, t->n_cu, static_cast<hipStream_t>(stream)));
}

int pusch_beamform(const pusch_c32* W, const pusch_c32* X, pusch_c32* Y, int n_beams, int n_ant, int n_re,
                   long long ld_x, long long batch, void* stream) {
  if (!X || !Y || batch < 0 || n_re < 0) return PUSCH_EINVAL;
  if (n_beams < 1 || n_beams > PUSCH_MAX_BEAMS || n_ant < 1 || n_ant > kMaxAnt) return PUSCH_EINVAL;
  if (ld_x < n_re || ld_x < 1) return PUSCH_EINVAL;
  if (!W && n_beams > n_ant) return PUSCH_EINVAL;
  const long long xbytes = batch * n_ant * ld_x * 8LL, ybytes = batch * (long long)n_re * n_beams * 8LL;
  if (overlap(X, xbytes, Y, ybytes) || overlap(W, (long long)n_beams * n_ant * 8, Y, ybytes)) return PUSCH_EINVAL;
  if (batch == 0 || n_re == 0) return PUSCH_OK;
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  const cf* w = reinterpret_cast<const cf*>(W);
  if (!w)
    if (int rc = dft_beamformer(t, n_beams, n_ant, &w)) return rc;
  return hip_status(pusch::launch_beamform(w, reinterpret_cast<const cf*>(X), reinterpret_cast<cf*>(Y), n_beams, n_ant,
                                           n_re, ld_x, (long long)n_ant * ld_x, (long long)n_re * n_beams, batch,
                                           t->n_cu, static_cast<hipStream_t>(stream)));
}

int pusch_chest(const pusch_c32* Yp, const pusch_c32* pilots, pusch_c32* H, int n_beams, int n_ue, int n_sc,
                int n_pilot, long long batch, void* stream) {
  if (!Yp || !pilots || !H || batch < 0) return PUSCH_EINVAL;
  if (n_pilot < 1 || n_pilot > PUSCH_MAX_PILOTS) return PUSCH_EINVAL;
  if (n_beams < 1 || n_beams > PUSCH_MAX_BEAMS) return PUSCH_EINVAL;
  if (n_ue < 1 || n_ue > PUSCH_MAX_UES || n_ue > n_beams || n_sc < n_ue) return PUSCH_EINVAL;
  const long long hb = batch * n_sc * (long long)n_ue * n_beams * 8;
  if (overlap(Yp, batch * n_pilot * (long long)n_sc * n_beams * 8, H, hb) ||
      overlap(pilots, batch * n_pilot * (long long)n_sc * 8, H, hb))
    return PUSCH_EINVAL;
  if (batch == 0) return PUSCH_OK;
  pusch::ChestGeom g{};
  g.n_beams = n_beams;
  g.n_ue = n_ue;
  g.n_sc = n_sc;
  g.n_pilot = n_pilot;
  g.y_batch = (long long)n_pilot * n_sc * n_beams;
  g.y_sym = (long long)n_sc * n_beams;
  for (int j = 0; j < n_pilot; ++j) g.pilot_sym[j] = j;
  g.p_batch = (long long)n_pilot * n_sc;
  g.h_batch = (long long)n_sc * n_ue * n_beams;
  return hip_status(pusch::launch_chest(reinterpret_cast<const cf*>(Yp), reinterpret_cast<const cf*>(pilots),
                                        reinterpret_cast<cf*>(H), g, batch, static_cast<hipStream_t>(stream)));
}

size_t pusch_noise_est_workspace_bytes(long long batch) {
  return batch < 0 ? 0 : (size_t)batch * pusch::kNeParts * sizeof(float2);
}

int pusch_noise_est(const pusch_c32* Yp, const pusch_c32* pilots, float* sigma2, int n_beams, int n_ue, int n_sc,
                    int n_pilot, long long batch, void* ws, size_t ws_bytes, void* stream) {
  if (!Yp || !pilots || !sigma2 || batch < 0) return PUSCH_EINVAL;
  if (n_pilot < 1 || n_pilot > PUSCH_MAX_PILOTS) return PUSCH_EINVAL;
  if (n_beams < 1 || n_beams > PUSCH_MAX_BEAMS) return PUSCH_EINVAL;
  if (n_ue < 1 || n_ue > PUSCH_MAX_UES || n_ue > n_beams || n_sc < 2 * n_ue || n_sc > kMaxNeSc) return PUSCH_EINVAL;
  if (batch == 0) return PUSCH_OK;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 7)) return PUSCH_EINVAL;
  const long long need = (long long)pusch_noise_est_workspace_bytes(batch);
  if (ws_bytes < (size_t)need) return PUSCH_ENOMEM;
  const long long yb = batch * n_pilot * (long long)n_sc * n_beams * 8, pb = batch * n_pilot * (long long)n_sc * 8;
  if (overlap(sigma2, batch * 4, Yp, yb) || overlap(sigma2, batch * 4, pilots, pb) ||
      overlap(sigma2, batch * 4, ws, need) || overlap(ws, need, Yp, yb) || overlap(ws, need, pilots, pb))
    return PUSCH_EINVAL;
  pusch::ChestGeom g{};
  g.n_beams = n_beams;
  g.n_ue = n_ue;
  g.n_sc = n_sc;
  g.n_pilot = n_pilot;
  g.y_batch = (long long)n_pilot * n_sc * n_beams;
  g.y_sym = (long long)n_sc * n_beams;
  for (int j = 0; j < n_pilot; ++j) g.pilot_sym[j] = j;
  g.p_batch = (long long)n_pilot * n_sc;
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  const void* tab = nullptr;
  if (int rc = geometry_table(t, kNoiseTable, g, 0, &tab)) return rc;
  return hip_status(pusch::launch_noise_est(reinterpret_cast<const cf*>(Yp), reinterpret_cast<const cf*>(pilots),
                                            false, static_cast<const int4*>(tab), static_cast<float2*>(ws), sigma2,
                                            g, batch, static_cast<hipStream_t>(stream)));
}

// ---- allocation-free noise estimation
// The scratch of pusch_noise_est_static lives in this file-scope device array
// (one copy per device, kept until the process ends): the geometry's
// neighbour table, then the per-item partial sums.  Host code never passes
// the array's name to a kernel -- on the host it is only a stand-in for the
// symbol; the device address comes from hipGetSymbolAddress (scratch_address).
constexpr size_t kStaticTabBytes = (size_t)PUSCH_MAX_PILOTS * kMaxNeSc * sizeof(int4);
constexpr size_t kStaticPartBytes = (size_t)PUSCH_NOISE_EST_STATIC_MAX_BATCH * pusch::kNeParts * sizeof(float2);
static __device__ __align__(256) unsigned char scratch[kStaticTabBytes + kStaticPartBytes];

namespace {
int scratch_address(unsigned char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PUSCH_EHIP;
  ScratchAddr& sa = g_scratch_addr[dev];
  std::call_once(sa.once, [&sa]() {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return;
    sa.ptr = static_cast<unsigned char*>(p);
    sa.status = PUSCH_OK;
  });
  *out = sa.ptr;
  return sa.status;
}
}  // namespace

int pusch_noise_est_static(const pusch_c32* Yp, const pusch_c32* pilots, float* sigma2, int n_beams, int n_ue,
                           int n_sc, int n_pilot, long long batch, void* stream) {
  if (!Yp || !pilots || !sigma2 || batch < 0) return PUSCH_EINVAL;
  if (n_pilot < 1 || n_pilot > PUSCH_MAX_PILOTS) return PUSCH_EINVAL;
  if (n_beams < 1 || n_beams > PUSCH_MAX_BEAMS) return PUSCH_EINVAL;
  if (n_ue < 1 || n_ue > PUSCH_MAX_UES || n_ue > n_beams || n_sc < 2 * n_ue || n_sc > kMaxNeSc) return PUSCH_EINVAL;
  if (batch > PUSCH_NOISE_EST_STATIC_MAX_BATCH) return PUSCH_EUNSUPPORTED;
  if (batch == 0) return PUSCH_OK;
  const long long yb = batch * n_pilot * (long long)n_sc * n_beams * 8, pb = batch * n_pilot * (long long)n_sc * 8;
  if (overlap(sigma2, batch * 4, Yp, yb) || overlap(sigma2, batch * 4, pilots, pb)) return PUSCH_EINVAL;
  pusch::ChestGeom g{};
  g.n_beams = n_beams;
  g.n_ue = n_ue;
  g.n_sc = n_sc;
  g.n_pilot = n_pilot;
  g.y_batch = (long long)n_pilot * n_sc * n_beams;
  g.y_sym = (long long)n_sc * n_beams;
  for (int j = 0; j < n_pilot; ++j) g.pilot_sym[j] = j;
  g.p_batch = (long long)n_pilot * n_sc;
  unsigned char* base = nullptr;
  if (int rc = scratch_address(&base)) return rc;
  int4* tab = reinterpret_cast<int4*>(base);
  float2* part = reinterpret_cast<float2*>(base + kStaticTabBytes);
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // the neighbour table is rebuilt in the scratch on every call (it is cheap,
  // and the previous call may have left another geometry's table there); the
  // partial sums need no clearing: every slice the final sum reads is written
  if (hipError_t e = pusch::launch_noise_table(tab, g, s)) return hip_status(e);
  return hip_status(pusch::launch_noise_est(reinterpret_cast<const cf*>(Yp), reinterpret_cast<const cf*>(pilots),
                                            false, tab, part, sigma2, g, batch, s));
}

int pusch_mmse_solve(const pusch_c32* H, const pusch_c32* Yd, float sigma2, pusch_c32* Xhat, int n_beams, int n_ue,
                     int n_sc, int n_data, long long batch, int32_t* status, void* stream) {
  if (!H || !Yd || !Xhat || batch < 0 || n_sc < 0 || n_data < 1) return PUSCH_EINVAL;
  if (!(sigma2 >= 0.f) || !std::isfinite(sigma2)) return PUSCH_EINVAL;
  if (n_beams < 1 || n_beams > PUSCH_MAX_BEAMS) return PUSCH_EINVAL;
  if (n_ue < 1 || n_ue > PUSCH_MAX_UES || n_ue > n_beams) return PUSCH_EINVAL;
  const long long xb = batch * n_data * (long long)n_sc * n_ue * 8;
  const long long hb = batch * (long long)n_sc * n_ue * n_beams * 8;
  const long long yb = batch * n_data * (long long)n_sc * n_beams * 8;
  const long long sb = batch * (long long)n_sc * 4;
  if (overlap(Xhat, xb, H, hb) || overlap(Xhat, xb, Yd, yb) || overlap(Xhat, xb, status, sb) ||
      overlap(status, sb, H, hb) || overlap(status, sb, Yd, yb))
    return PUSCH_EINVAL;
  if (batch == 0 || n_sc == 0) return PUSCH_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  for (int d0 = 0; d0 < n_data; d0 += pusch::kMaxSymbols) {
    const int nd = n_data - d0 < pusch::kMaxSymbols ? n_data - d0 : pusch::kMaxSymbols;
    pusch::MmseGeom g{};
    g.n_beams = n_beams;
    g.n_ue = n_ue;
    g.n_sc = n_sc;
    g.n_data = nd;
    g.sigma2 = sigma2;
    g.h_batch = (long long)n_sc * n_ue * n_beams;
    g.y_batch = (long long)n_data * n_sc * n_beams;
    g.y_sym = (long long)n_sc * n_beams;
    g.d_first = d0;
    g.n_skip = 0;
    g.x_batch = (long long)n_data * n_sc * n_ue;
    g.st_batch = n_sc;
    const hipError_t e =
        pusch::launch_mmse(reinterpret_cast<const cf*>(H), reinterpret_cast<const cf*>(Yd),
                           reinterpret_cast<cf*>(Xhat) + (long long)d0 * n_sc * n_ue, status, g, batch, s);
    if (e != hipSuccess) return PUSCH_EHIP;
  }
  return PUSCH_OK;
}

}  // extern "C"

namespace {

struct SlotLayout {
  size_t off_xa, off_ex, off_y, off_h, off_ne, total;
};

// Geometry only (what the workspace size depends on).
int check_geom(const pusch_slot_desc* d) {
  if (!d) return PUSCH_EINVAL;
  if (pusch::fft_size_index(d->n_fft) < 0) return PUSCH_EUNSUPPORTED;
  if (d->n_ant < 1 || d->n_ant > kMaxAnt) return PUSCH_EINVAL;
  if (d->n_beams < 1 || d->n_beams > PUSCH_MAX_BEAMS) return PUSCH_EINVAL;
  if (d->n_ue < 1 || d->n_ue > PUSCH_MAX_UES || d->n_ue > d->n_beams) return PUSCH_EINVAL;
  if (d->n_sc < d->n_ue || d->n_sc > d->n_fft) return PUSCH_EINVAL;
  if (d->n_symb < 2 || d->n_symb > PUSCH_MAX_SYMBOLS) return PUSCH_EINVAL;
  if (d->n_pilot < 1 || d->n_pilot > PUSCH_MAX_PILOTS || d->n_pilot >= d->n_symb) return PUSCH_EINVAL;
  for (int j = 0; j < d->n_pilot; ++j) {
    if (d->pilot_symb[j] < 0 || d->pilot_symb[j] >= d->n_symb) return PUSCH_EINVAL;
    if (j > 0 && d->pilot_symb[j] <= d->pilot_symb[j - 1]) return PUSCH_EINVAL;
  }
  if (!d->W && d->n_beams > d->n_ant) return PUSCH_EINVAL;
  return PUSCH_OK;
}

int check_desc(const pusch_slot_desc* d) {
  if (int rc = check_geom(d)) return rc;
  if (d->noise_est) {
    // noise estimation: every UE needs two pilot positions
    if (d->n_sc < 2 * d->n_ue) return PUSCH_EINVAL;
  } else if (!(d->sigma2 >= 0.f) || !std::isfinite(d->sigma2)) {
    return PUSCH_EINVAL;
  }
  if (!d->pilots) return PUSCH_EINVAL;
  return PUSCH_OK;
}

// Noise-estimation scratch: kNeParts partial sums per slot, then the
// per-slot estimates (used when the caller asks for none).
size_t ne_part_bytes(long long n_slot) { return (size_t)n_slot * pusch::kNeParts * sizeof(float2); }

// The detection kernel estimates the channel itself (no stored estimate)
// for up to 16 UEs and an even number of beams, unless refinement is asked
// for (the refining kernel reads a stored estimate).
bool slot_fused(const pusch_slot_desc* d) {
  return !d->refine && pusch::mmse_fusable(d->n_ue, d->n_beams, (long long)d->n_symb * d->n_sc * d->n_beams);
}

// Row pitch of the active-bin grids between the FFT and beamforming: a
// multiple of 16 subcarriers, so every antenna row starts on a 128-byte line
// and a beamforming tile of 16 subcarriers reads whole lines that no other
// tile touches.
size_t xa_pitch(int n_sc) { return ((size_t)n_sc + 15) & ~(size_t)15; }

// Mixed precision: the active-bin grids as FP16 pairs (4 bytes), rows padded
// to 32 subcarriers (one 128-byte line), and an int8 exponent table of 64
// entries per slot symbol.
size_t xa_pitch_h16(int n_sc) { return ((size_t)n_sc + 31) & ~(size_t)31; }

SlotLayout slot_layout(const pusch_slot_desc* d, long long n_slot, bool mixed = false) {
  const size_t S = d->n_symb, R = d->n_ant, K = d->n_sc, B = d->n_beams, L = d->n_ue, n = (size_t)n_slot;
  SlotLayout lay;
  lay.off_xa = 0;
  if (mixed) {
    lay.off_ex = align256(n * S * R * xa_pitch_h16(d->n_sc) * 4);
    lay.off_y = lay.off_ex + align256(n * S * 64);
  } else {
    lay.off_ex = 0;
    lay.off_y = align256(n * S * R * xa_pitch(d->n_sc) * 8);
  }
  lay.off_h = lay.off_y + align256(n * S * K * B * 8);
  // when the detection kernel estimates the channel itself (up to 16 UEs, an
  // even number of beams) no stored estimate is needed
  const bool fused = slot_fused(d);
  lay.off_ne = lay.off_h + (fused ? 0 : align256(n * K * L * B * 8));
  lay.total = lay.off_ne + align256(ne_part_bytes(n_slot) + n * sizeof(float));
  return lay;
}

// The FP16 path runs on the register-tile beamforming kernel: up to 64
// antennas, 32-bit tile indices.
bool mixed_supported(const pusch_slot_desc* d, long long n_slot) {
  return d->n_ant <= 64 && n_slot * d->n_symb * (((long long)d->n_sc + 15) / 16) < (1ll << 30);
}

size_t out_bytes(const pusch_slot_desc* d, long long n_slot) {
  return (size_t)n_slot * (size_t)(d->n_symb - d->n_pilot) * d->n_sc * d->n_ue * 8;
}

// Arguments of one slot call (descriptor, buffers, workspace, aliasing).
int check_slot_call(const pusch_slot_desc* d, long long n_slot, const pusch_c32* x_td, pusch_c32* x_hat,
                    int32_t* status, void* ws, size_t ws_bytes, bool mixed = false) {
  if (int rc = check_desc(d)) return rc;
  if (n_slot < 0 || !x_td || !x_hat || !ws) return PUSCH_EINVAL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return PUSCH_EINVAL;
  if (mixed && !mixed_supported(d, n_slot)) return PUSCH_EUNSUPPORTED;
  // matrix-core FFT passes: the 4-byte grids of the reduced-precision forms, 4096 points
  if (d->fft_mfma && (!mixed || d->n_fft != 4096)) return PUSCH_EUNSUPPORTED;
  // per-symbol estimates: the detection kernel that interpolates the channel
  // itself (up to 16 UEs, an even number of beams), without refinement
  if (d->time_varying && !slot_fused(d)) return PUSCH_EUNSUPPORTED;
  const SlotLayout lay = slot_layout(d, n_slot, mixed);
  if (ws_bytes < lay.total) return PUSCH_ENOMEM;
  const int S = d->n_symb, R = d->n_ant, K = d->n_sc, B = d->n_beams, P = d->n_pilot;
  const long long xb = n_slot * (long long)S * R * d->n_fft * 8, ob = (long long)out_bytes(d, n_slot),
                  sb = n_slot * (long long)K * 4, wb = (long long)lay.total;
  if (overlap(x_hat, ob, x_td, xb) || overlap(x_hat, ob, ws, wb) || overlap(x_hat, ob, status, sb) ||
      overlap(ws, wb, x_td, xb) || overlap(status, sb, x_td, xb) || overlap(status, sb, ws, wb) ||
      overlap(ws, wb, d->pilots, n_slot * (long long)P * K * 8) || overlap(ws, wb, d->W, (long long)B * R * 8))
    return PUSCH_EINVAL;
  if (d->noise_est && d->sigma2_est) {
    const long long eb = n_slot * 4;
    if (overlap(d->sigma2_est, eb, x_td, xb) || overlap(d->sigma2_est, eb, x_hat, ob) ||
        overlap(d->sigma2_est, eb, status, sb) || overlap(d->sigma2_est, eb, ws, wb) ||
        overlap(d->sigma2_est, eb, d->pilots, n_slot * (long long)P * K * 8) ||
        overlap(d->sigma2_est, eb, d->W, (long long)B * R * 8))
      return PUSCH_EINVAL;
  }
  return PUSCH_OK;
}

// Estimation geometry of a slot call (grids of one batch item: [n_symb][n_sc][n_beams]).
pusch::ChestGeom chest_geom(const pusch_slot_desc* d) {
  const int S = d->n_symb, K = d->n_sc, B = d->n_beams, L = d->n_ue, P = d->n_pilot;
  pusch::ChestGeom cg{};
  cg.n_beams = B;
  cg.n_ue = L;
  cg.n_sc = K;
  cg.n_pilot = P;
  cg.y_batch = (long long)S * K * B;
  cg.y_sym = (long long)K * B;
  for (int j = 0; j < P; ++j) cg.pilot_sym[j] = d->pilot_symb[j];
  cg.p_batch = (long long)P * K;
  cg.h_batch = (long long)K * L * B;
  cg.comb_aligned = d->comb_aligned ? 1 : 0;
  return cg;
}

// Beamforming epilogue of the fused detection: the pilot symbols leave the
// stage divided by their pilots.
pusch::PilotScale pilot_scale(const pusch_slot_desc* d) {
  pusch::PilotScale psc{};
  psc.pilots = reinterpret_cast<const cf*>(d->pilots);
  psc.p_slot = (long long)d->n_pilot * d->n_sc;
  psc.n_symb = d->n_symb;
  for (int s_ = 0; s_ < pusch::kMaxSymbols; ++s_) psc.pilot_of[s_] = -1;
  for (int j = 0; j < d->n_pilot; ++j) psc.pilot_of[d->pilot_symb[j]] = (signed char)j;
  return psc;
}

// Detection geometry of a slot call; s2: per-slot noise variances (device) or nullptr.
pusch::MmseGeom mmse_geom(const pusch_slot_desc* d, const float* s2) {
  const int S = d->n_symb, K = d->n_sc, B = d->n_beams, L = d->n_ue, P = d->n_pilot;
  const int D = S - P;
  pusch::MmseGeom mg{};
  mg.n_beams = B;
  mg.n_ue = L;
  mg.n_sc = K;
  mg.n_data = D;
  mg.sigma2 = d->noise_est ? 0.f : d->sigma2;
  mg.sigma2_item = s2;
  mg.refine = d->refine ? 1 : 0;
  mg.h_batch = (long long)K * L * B;
  mg.y_batch = (long long)S * K * B;
  mg.y_sym = (long long)K * B;
  mg.d_first = 0;
  mg.n_skip = P;
  for (int j = 0; j < P; ++j) mg.skip[j] = d->pilot_symb[j];
  mg.x_batch = (long long)D * K * L;
  mg.st_batch = K;
  return mg;
}

// Launch sequence of one fused slot call on stream s (arguments checked).
// mixed: 4-byte grids between the FFT and beamforming, FP16 with row scales,
// or bfloat16 with bf16 (the exponent table is then not used).
int run_slot(DeviceTables* t, const pusch_slot_desc* d, long long n_slot, const pusch_c32* x_td, pusch_c32* x_hat,
             int32_t* status, char* base, hipStream_t s, bool profile, bool mixed = false, bool bf16 = false) {
  const SlotLayout lay = slot_layout(d, n_slot, mixed);
  const int S = d->n_symb, R = d->n_ant, K = d->n_sc, B = d->n_beams, L = d->n_ue, P = d->n_pilot;
  const int D = S - P;
  const cf* w = reinterpret_cast<const cf*>(d->W);
  if (!w)
    if (int rc = dft_beamformer(t, B, R, &w)) return rc;
  cf* Xa = reinterpret_cast<cf*>(base + lay.off_xa);
  cf* Y = reinterpret_cast<cf*>(base + lay.off_y);
  cf* H = reinterpret_cast<cf*>(base + lay.off_h);
  // estimation geometry, and the geometry's cached tables (built before
  // anything is enqueued on s)
  const bool fused = slot_fused(d);
  const pusch::ChestGeom cg = chest_geom(d);
  const int n_tap = pusch::comb_taps(L, P, d->comb_aligned != 0);
  const void* taps = nullptr;
  const void* ne_tab = nullptr;
  pusch::TimeTapGeom tt{};
  if (d->time_varying) {
    for (int s_ = 0; s_ < S; ++s_) {
      bool pilot = false;
      for (int j = 0; j < P; ++j) pilot |= d->pilot_symb[j] == s_;
      if (!pilot) tt.data_sym[tt.n_data++] = s_;
    }
    // two pilot symbols: every data symbol in one launch from each pilot
    // symbol's own taps; more: one launch per run of data symbols
    if (P == 2) {
      if (int rc = geometry_table(t, kPairTaps, cg, 4, &taps)) return rc;
    } else if (int rc = geometry_table(t, kTimeTaps, cg, pusch::kTimeTaps, &taps, &tt)) {
      return rc;
    }
  } else if (fused) {
    if (int rc = geometry_table(t, kCombTaps, cg, n_tap, &taps)) return rc;
  }
  if (d->noise_est)
    if (int rc = geometry_table(t, kNoiseTable, cg, 0, &ne_tab)) return rc;

  hipEvent_t* ev = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_prof.mu);
    if (profile && g_prof.active && g_prof.calls < g_prof.max_calls) ev = &g_prof.ev[(size_t)g_prof.calls++ * kEvPerCall];
  }
  auto mark = [&](int i) -> bool { return !ev || hipEventRecord(ev[i], s) == hipSuccess; };

  // OFDM demodulation (FFT) of every antenna and symbol, active bins only
  if (!mark(0)) return PUSCH_EHIP;
  const long long KP = mixed ? (long long)xa_pitch_h16(K) : (long long)xa_pitch(K);
  unsigned* Xh = mixed ? reinterpret_cast<unsigned*>(base + lay.off_xa) : nullptr;
  signed char* ex = mixed && !bf16 ? reinterpret_cast<signed char*>(base + lay.off_ex) : nullptr;
  if (mixed && d->fft_mfma) {
    if (pusch::launch_fft_mfma(reinterpret_cast<const cf*>(x_td), d->n_fft, n_slot * S * R, K, K / 2, KP,
                               t->twiddles, t->n_cu, s, Xh, ex, R) != hipSuccess)
      return PUSCH_EHIP;
  } else if (pusch::launch_fft(reinterpret_cast<const cf*>(x_td), Xa, d->n_fft, n_slot * S * R, K, K / 2, KP,
                               t->twiddles, t->n_cu, s, Xh, ex, R) != hipSuccess) {
    return PUSCH_EHIP;
  }
  // beamforming of every symbol, RE-major output; when the detection
  // kernel estimates the channel itself, the pilot symbols leave this stage
  // already divided by their pilots (the LS division of the channel estimate)
  pusch::PilotScale psc{};
  if (fused) psc = pilot_scale(d);
  if (!mark(1)) return PUSCH_EHIP;
  if (pusch::launch_beamform(w, Xa, Y, B, R, K, KP, R * KP, (long long)K * B, n_slot * S, t->n_cu, s,
                             fused ? &psc : nullptr, Xh, ex) != hipSuccess)
    return PUSCH_EHIP;
  // LS channel estimate from the pilot symbols
  if (!mark(2)) return PUSCH_EHIP;
  if (!fused && pusch::launch_chest(Y, reinterpret_cast<const cf*>(d->pilots), H, cg, n_slot, s) != hipSuccess)
    return PUSCH_EHIP;
  // noise variance of every slot from its pilot symbols (which hold LS
  // values when fused, received values otherwise)
  float* s2 = nullptr;
  if (d->noise_est) {
    float2* part = reinterpret_cast<float2*>(base + lay.off_ne);
    s2 = d->sigma2_est ? d->sigma2_est : reinterpret_cast<float*>(base + lay.off_ne + ne_part_bytes(n_slot));
    if (pusch::launch_noise_est(Y, reinterpret_cast<const cf*>(d->pilots), fused, static_cast<const int4*>(ne_tab),
                                part, s2, cg, n_slot, s) != hipSuccess)
      return PUSCH_EHIP;
  }
  // MMSE detection: Gram, Cholesky, matched filter and substitutions for the data
  // symbols (with the channel estimate computed inside when fused)
  if (!mark(3)) return PUSCH_EHIP;
  const pusch::MmseGeom mg = mmse_geom(d, s2);
  if (d->time_varying && P == 2) {
    // one factorisation per data symbol (its own channel estimate), all in one launch
    if (pusch::launch_mmse_tv(Y, static_cast<const int2*>(taps), cg, reinterpret_cast<cf*>(x_hat), status, mg,
                              n_slot, s) != hipSuccess)
      return PUSCH_EHIP;
  } else if (d->time_varying) {
    // one factorisation per data symbol (its own channel estimate); the data
    // symbols before the first pilot symbol share one estimate, and so do
    // those after the last, so each such run is one launch; status flags
    // ORed over the launches
    const int first = d->pilot_symb[0], last = d->pilot_symb[P - 1];
    auto side = [&](int sym) { return sym < first ? -1 : (sym > last ? 1 : 0); };
    for (int dd = 0; dd < D;) {
      int n = 1;
      const int sd = side(tt.data_sym[dd]);
      if (sd != 0)
        while (dd + n < D && side(tt.data_sym[dd + n]) == sd) ++n;
      pusch::MmseGeom md = mg;
      md.n_data = n;
      md.d_first = dd;
      md.st_or = dd > 0;
      const int2* td = static_cast<const int2*>(taps) + (long long)dd * K * L * pusch::kTimeTaps;
      if (pusch::launch_mmse_fused(Y, td, pusch::kTimeTaps, cg, reinterpret_cast<cf*>(x_hat) + (long long)dd * K * L,
                                   status, md, n_slot, s) != hipSuccess)
        return PUSCH_EHIP;
      dd += n;
    }
  } else {
    const hipError_t me =
        fused ? pusch::launch_mmse_fused(Y, static_cast<const int2*>(taps), n_tap, cg, reinterpret_cast<cf*>(x_hat),
                                         status, mg, n_slot, s)
              : pusch::launch_mmse(H, Y, reinterpret_cast<cf*>(x_hat), status, mg, n_slot, s);
    if (me != hipSuccess) return PUSCH_EHIP;
  }
  if (!mark(4)) return PUSCH_EHIP;
  return PUSCH_OK;
}

// ---------------------------------------------------------------- grouped cells
// pusch_cells runs the cells that the grouped kernels take as one launch per
// stage and kernel shape (transform size; beamforming tile class; detection
// class), each launch covering up to its table's worth of cells, all on the
// caller's stream; a cell's workgroups find their cell through a prefix table
// of workgroup counts passed with the launch.  Other cells (refinement,
// per-symbol estimates, more than 64 antennas, odd beam counts, more than 16
// UEs) run as pusch_slot calls on the side streams meanwhile.

// Cells that the grouped kernels take: the detection that interpolates the
// channel itself with one estimate per slot, on the register-tile
// beamforming kernels (up to 64 antennas, 32-bit tile indices).
bool cell_grouped(const pusch_slot_desc* d, long long n_slot, bool mixed) {
  if (n_slot < 1 || !slot_fused(d) || d->time_varying) return false;
  if (pusch::bf_cell_class(d->n_beams, d->n_ant) < 0) return false;
  if (pusch::mmse_cell_class(d->n_beams, pusch::comb_taps(d->n_ue, d->n_pilot, d->comb_aligned != 0)) < 0)
    return false;
  const long long KP = mixed ? (long long)xa_pitch_h16(d->n_sc) : (long long)xa_pitch(d->n_sc);
  // (the detection's workgroups, one per 4 subcarriers of a slot, are far fewer than the tiles)
  return KP * d->n_ant < (1ll << 28) && n_slot * d->n_symb * (((long long)d->n_sc + 15) / 16) < (1ll << 30);
}

// Calls f(key, cells) for the cells of every distinct key, at most per_launch at a time,
// in order of first appearance.
template <class Key, class Launch>
int for_groups(const std::vector<int>& idx, Key key, int per_launch, Launch f) {
  std::vector<char> done(idx.size(), 0);
  std::vector<int> grp;
  for (size_t i = 0; i < idx.size(); ++i) {
    if (done[i]) continue;
    const int k = key(idx[i]);
    grp.clear();
    for (size_t j = i; j < idx.size(); ++j) {
      if (done[j] || key(idx[j]) != k) continue;
      done[j] = 1;
      grp.push_back(idx[j]);
      if ((int)grp.size() == per_launch) {
        if (int rc = f(k, grp)) return rc;
        grp.clear();
      }
    }
    if (!grp.empty())
      if (int rc = f(k, grp)) return rc;
  }
  return PUSCH_OK;
}

// The grouped stages of pusch_cells on stream s for the cells in idx (arguments
// checked); cell c's intermediates in its own workspace slice base[c].
// *side_used: side streams the call enqueued detection launches on (the
// caller joins them back to s).
int run_cells_grouped(DeviceTables* t, const pusch_slot_desc* d, const long long* n_slot, const pusch_c32* const* x_td,
                      pusch_c32* const* x_hat, int32_t* const* status, const std::vector<char*>& base,
                      const std::vector<int>& idx, bool mixed, const pusch_cells_plan& plan, hipStream_t s,
                      int* side_used) {
  *side_used = 0;
  if (idx.empty()) return PUSCH_OK;
  const int n = (int)base.size();
  // the geometries' tables, before anything is enqueued
  std::vector<const cf*> W(n, nullptr);
  std::vector<const void*> taps(n, nullptr), ne_tab(n, nullptr);
  for (int c : idx) {
    W[c] = reinterpret_cast<const cf*>(d[c].W);
    if (!W[c])
      if (int rc = dft_beamformer(t, d[c].n_beams, d[c].n_ant, &W[c])) return rc;
    const pusch::ChestGeom cg = chest_geom(&d[c]);
    if (int rc = geometry_table(t, kCombTaps, cg, pusch::comb_taps(d[c].n_ue, d[c].n_pilot, cg.comb_aligned != 0),
                                &taps[c]))
      return rc;
    if (d[c].noise_est)
      if (int rc = geometry_table(t, kNoiseTable, cg, 0, &ne_tab[c])) return rc;
  }
  auto pitch = [&](int c) {
    return mixed ? (long long)xa_pitch_h16(d[c].n_sc) : (long long)xa_pitch(d[c].n_sc);
  };
  // OFDM demodulation: one launch for every transform size, or one per size
  int rc = for_groups(idx, [&](int c) { return plan.fft_merged ? 0 : d[c].n_fft; }, pusch::kFftCellsPerLaunch,
                      [&](int, const std::vector<int>& grp) {
                        pusch::FftCells ft{};
                        ft.n = (int)grp.size();
                        for (int i = 0; i < ft.n; ++i) {
                          const int c = grp[i];
                          const SlotLayout lay = slot_layout(&d[c], n_slot[c], mixed);
                          pusch::FftCell& e = ft.cell[i];
                          e.x = reinterpret_cast<const cf*>(x_td[c]);
                          e.X = reinterpret_cast<cf*>(base[c] + lay.off_xa);
                          e.Xh = mixed ? reinterpret_cast<unsigned*>(base[c] + lay.off_xa) : nullptr;
                          e.ex = mixed ? reinterpret_cast<signed char*>(base[c] + lay.off_ex) : nullptr;
                          e.n_fft = d[c].n_fft;
                          e.rows = d[c].n_ant;
                          e.batch = n_slot[c] * d[c].n_symb * d[c].n_ant;
                          e.out_len = d[c].n_sc;
                          e.shift = d[c].n_sc / 2;
                          e.ldo = pitch(c);
                        }
                        return hip_status(pusch::launch_fft_cells(ft, mixed, t->twiddles, t->n_cu, s));
                      });
  if (rc) return rc;
  // beamforming with the pilot epilogue: one launch for every tile class, or one per class
  rc = for_groups(idx, [&](int c) { return plan.bf_merged ? -1 : pusch::bf_cell_class(d[c].n_beams, d[c].n_ant); },
                  pusch::kBfCellsPerLaunch, [&](int cls, const std::vector<int>& grp) {
                    pusch::BfCells bt{};
                    bt.n = (int)grp.size();
                    for (int i = 0; i < bt.n; ++i) {
                      const int c = grp[i];
                      const SlotLayout lay = slot_layout(&d[c], n_slot[c], mixed);
                      pusch::BfCell& e = bt.cell[i];
                      const long long KP = pitch(c);
                      e.W = W[c];
                      e.X = reinterpret_cast<const cf*>(base[c] + lay.off_xa);
                      e.Xh = mixed ? reinterpret_cast<const unsigned*>(base[c] + lay.off_xa) : nullptr;
                      e.ex = mixed ? reinterpret_cast<const signed char*>(base[c] + lay.off_ex) : nullptr;
                      e.Y = reinterpret_cast<cf*>(base[c] + lay.off_y);
                      e.ldx = KP;
                      e.sx = d[c].n_ant * KP;
                      e.sy = (long long)d[c].n_sc * d[c].n_beams;
                      e.batch = n_slot[c] * d[c].n_symb;
                      e.nb = d[c].n_beams;
                      e.na = d[c].n_ant;
                      e.nre = d[c].n_sc;
                      e.ps = pilot_scale(&d[c]);
                    }
                    return hip_status(pusch::launch_beamform_cells(bt, cls, mixed, t->n_cu, s));
                  });
  if (rc) return rc;
  // noise variance per slot, one launch per cell that estimates it
  std::vector<float*> s2(n, nullptr);
  for (int c : idx) {
    if (!d[c].noise_est) continue;
    const SlotLayout lay = slot_layout(&d[c], n_slot[c], mixed);
    float2* part = reinterpret_cast<float2*>(base[c] + lay.off_ne);
    s2[c] = d[c].sigma2_est ? d[c].sigma2_est
                            : reinterpret_cast<float*>(base[c] + lay.off_ne + ne_part_bytes(n_slot[c]));
    if (pusch::launch_noise_est(reinterpret_cast<const cf*>(base[c] + lay.off_y),
                                reinterpret_cast<const cf*>(d[c].pilots), true, static_cast<const int4*>(ne_tab[c]),
                                part, s2[c], chest_geom(&d[c]), n_slot[c], s) != hipSuccess)
      return PUSCH_EHIP;
  }
  // detection: one launch for every detection class, or one per class.  Its
  // workgroups are not persistent, so when the cells need several launches
  // they run side by side: the first on s, the others on the side streams
  // (forked from s here), and their tails overlap.
  int n_launch = 0;
  if (hipEventRecord(t->fork_mmse, s) != hipSuccess) return PUSCH_EHIP;
  rc = for_groups(
      idx,
      [&](int c) {
        return plan.mmse_merged
                   ? -1
                   : pusch::mmse_cell_class(d[c].n_beams,
                                            pusch::comb_taps(d[c].n_ue, d[c].n_pilot, d[c].comb_aligned != 0));
      },
      pusch::kMmseCellsPerLaunch, [&](int cls, const std::vector<int>& grp) -> int {
        pusch::MmseCells mt{};
        mt.n = (int)grp.size();
        for (int i = 0; i < mt.n; ++i) {
          const int c = grp[i];
          const SlotLayout lay = slot_layout(&d[c], n_slot[c], mixed);
          pusch::MmseCell& e = mt.cell[i];
          e.Y = reinterpret_cast<const cf*>(base[c] + lay.off_y);
          e.taps = static_cast<const int2*>(taps[c]);
          e.Xh = reinterpret_cast<cf*>(x_hat[c]);
          e.st = status ? status[c] : nullptr;
          e.batch = n_slot[c];
          e.g = mmse_geom(&d[c], s2[c]);
          e.cg = chest_geom(&d[c]);
          e.n_tap = pusch::comb_taps(d[c].n_ue, d[c].n_pilot, d[c].comb_aligned != 0);
        }
        hipStream_t ls = s;
        if (n_launch > 0) {
          const int j = (n_launch - 1) % kSideStreams;
          if (n_launch <= kSideStreams && hipStreamWaitEvent(t->side[j], t->fork_mmse, 0) != hipSuccess)
            return PUSCH_EHIP;
          ls = t->side[j];
          *side_used = std::max(*side_used, j + 1);
        }
        ++n_launch;
        return hip_status(pusch::launch_mmse_cells(mt, cls, ls));
      });
  return rc;
}

// Launch plan of a call that pusch_cells_tune has not timed.
constexpr pusch_cells_plan kDefaultPlan = {1, 0, 1};

// What a cell set's timing depends on: every cell's geometry, slots and
// options, and the flags.
std::vector<long long> cells_signature(const pusch_slot_desc* d, int n_cells, const long long* n_slot, int flags) {
  std::vector<long long> key = {flags & (PUSCH_CELLS_MIXED | PUSCH_CELLS_STREAMS), n_cells};
  for (int c = 0; c < n_cells; ++c) {
    key.insert(key.end(), {d[c].n_ant, d[c].n_fft, d[c].n_sc, d[c].n_symb, d[c].n_beams, d[c].n_ue, d[c].n_pilot,
                           n_slot[c], d[c].noise_est, d[c].refine, d[c].time_varying, d[c].comb_aligned});
    for (int j = 0; j < d[c].n_pilot; ++j) key.push_back(d[c].pilot_symb[j]);
  }
  return key;
}

pusch_cells_plan cells_plan(DeviceTables* t, const std::vector<long long>& key, int* tuned = nullptr) {
  std::lock_guard<std::mutex> lock(t->mu);
  auto it = t->plans.find(key);
  if (tuned) *tuned = it != t->plans.end();
  return it != t->plans.end() ? it->second : kDefaultPlan;
}

// pusch_cells with the plan given (nullptr: the recorded one for the cell set, else the default).
int cells_call(const pusch_slot_desc* d, int n_cells, const long long* n_slot, const pusch_c32* const* x_td,
               pusch_c32* const* x_hat, int32_t* const* status, void* ws, size_t ws_bytes, int flags,
               const pusch_cells_plan* force, void* stream);

}  // namespace

extern "C" {

size_t pusch_slot_workspace_bytes(const pusch_slot_desc* d, long long n_slot) {
  if (check_geom(d) != PUSCH_OK || n_slot < 0) return 0;
  return slot_layout(d, n_slot).total;
}

int pusch_slot(const pusch_slot_desc* d, long long n_slot, const pusch_c32* x_td, pusch_c32* x_hat, int32_t* status,
               void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_slot_call(d, n_slot, x_td, x_hat, status, ws, ws_bytes)) return rc;
  if (n_slot == 0) return PUSCH_OK;
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  return run_slot(t, d, n_slot, x_td, x_hat, status, static_cast<char*>(ws), static_cast<hipStream_t>(stream), true);
}

size_t pusch_slot_mixed_workspace_bytes(const pusch_slot_desc* d, long long n_slot) {
  if (check_geom(d) != PUSCH_OK || n_slot < 0 || !mixed_supported(d, n_slot)) return 0;
  return slot_layout(d, n_slot, true).total;
}

int pusch_slot_mixed(const pusch_slot_desc* d, long long n_slot, const pusch_c32* x_td, pusch_c32* x_hat,
                     int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_slot_call(d, n_slot, x_td, x_hat, status, ws, ws_bytes, true)) return rc;
  if (n_slot == 0) return PUSCH_OK;
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  return run_slot(t, d, n_slot, x_td, x_hat, status, static_cast<char*>(ws), static_cast<hipStream_t>(stream), true,
                  true);
}

size_t pusch_slot_bf16_workspace_bytes(const pusch_slot_desc* d, long long n_slot) {
  return pusch_slot_mixed_workspace_bytes(d, n_slot);
}

int pusch_slot_bf16(const pusch_slot_desc* d, long long n_slot, const pusch_c32* x_td, pusch_c32* x_hat,
                    int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_slot_call(d, n_slot, x_td, x_hat, status, ws, ws_bytes, true)) return rc;
  if (n_slot == 0) return PUSCH_OK;
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  return run_slot(t, d, n_slot, x_td, x_hat, status, static_cast<char*>(ws), static_cast<hipStream_t>(stream), true,
                  true, true);
}

size_t pusch_cells_workspace_bytes(const pusch_slot_desc* d, int n_cells, const long long* n_slot, int flags) {
  if (!d || !n_slot || n_cells < 1 || n_cells > PUSCH_MAX_CELLS) return 0;
  const bool mixed = (flags & PUSCH_CELLS_MIXED) != 0;
  size_t total = 0;
  for (int c = 0; c < n_cells; ++c) {
    if (check_geom(&d[c]) != PUSCH_OK || n_slot[c] < 0) return 0;
    if (mixed && !mixed_supported(&d[c], n_slot[c])) return 0;
    total += align256(slot_layout(&d[c], n_slot[c], mixed).total);
  }
  return total;
}

int pusch_cells(const pusch_slot_desc* d, int n_cells, const long long* n_slot, const pusch_c32* const* x_td,
                pusch_c32* const* x_hat, int32_t* const* status, void* ws, size_t ws_bytes, int flags,
                void* stream) {
  return cells_call(d, n_cells, n_slot, x_td, x_hat, status, ws, ws_bytes, flags, nullptr, stream);
}

int pusch_cells_plan_get(const pusch_slot_desc* d, int n_cells, const long long* n_slot, int flags,
                         pusch_cells_plan* plan) {
  if (!d || !n_slot || !plan || n_cells < 1 || n_cells > PUSCH_MAX_CELLS) return PUSCH_EINVAL;
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  int tuned = 0;
  *plan = cells_plan(t, cells_signature(d, n_cells, n_slot, flags), &tuned);
  return tuned;
}

int pusch_cells_tune(const pusch_slot_desc* d, int n_cells, const long long* n_slot, const pusch_c32* const* x_td,
                     pusch_c32* const* x_hat, int32_t* const* status, void* ws, size_t ws_bytes, int flags, int reps,
                     pusch_cells_plan* chosen, float* us, int n_us, void* stream) {
  if (reps < 1 || reps > 1000 || (n_us > 0 && !us) || n_us < 0) return PUSCH_EINVAL;
  if (!d || !n_slot || n_cells < 1 || n_cells > PUSCH_MAX_CELLS) return PUSCH_EINVAL;
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t ev[2] = {};
  if (hipEventCreate(&ev[0]) != hipSuccess) return PUSCH_EHIP;
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return PUSCH_EHIP;
  }
  int rc = PUSCH_OK;
  float best = 0.f;
  pusch_cells_plan pick = kDefaultPlan;
  std::vector<float> t_us(PUSCH_CELLS_PLANS, 0.f), one(reps);
  for (int p = 0; p < PUSCH_CELLS_PLANS && rc == PUSCH_OK; ++p) {
    const pusch_cells_plan plan = {p & 1, (p >> 1) & 1, (p >> 2) & 1};
    // one call to warm up (tables, code objects), then reps timed calls; the median
    rc = cells_call(d, n_cells, n_slot, x_td, x_hat, status, ws, ws_bytes, flags, &plan, stream);
    for (int r = 0; r < reps && rc == PUSCH_OK; ++r) {
      float ms = 0.f;
      if (hipEventRecord(ev[0], s) != hipSuccess) rc = PUSCH_EHIP;
      if (rc == PUSCH_OK) rc = cells_call(d, n_cells, n_slot, x_td, x_hat, status, ws, ws_bytes, flags, &plan, stream);
      if (rc == PUSCH_OK && (hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                             hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess))
        rc = PUSCH_EHIP;
      one[r] = ms * 1e3f;
    }
    if (rc != PUSCH_OK) break;
    std::sort(one.begin(), one.end());
    t_us[p] = one[reps / 2];
    if (p == 0 || t_us[p] < best) {
      best = t_us[p];
      pick = plan;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (rc != PUSCH_OK) return rc;
  {
    std::lock_guard<std::mutex> lock(t->mu);
    t->plans[cells_signature(d, n_cells, n_slot, flags)] = pick;
  }
  if (chosen) *chosen = pick;
  for (int p = 0; p < n_us && p < PUSCH_CELLS_PLANS; ++p) us[p] = t_us[p];
  return PUSCH_OK;
}

}  // extern "C"

namespace {

int cells_call(const pusch_slot_desc* d, int n_cells, const long long* n_slot, const pusch_c32* const* x_td,
               pusch_c32* const* x_hat, int32_t* const* status, void* ws, size_t ws_bytes, int flags,
               const pusch_cells_plan* force, void* stream) {
  if (!d || !n_slot || !x_td || !x_hat || n_cells < 1 || n_cells > PUSCH_MAX_CELLS) return PUSCH_EINVAL;
  if (flags & ~(PUSCH_CELLS_MIXED | PUSCH_CELLS_STREAMS | PUSCH_CELLS_WITH_PLAN(PUSCH_CELLS_PLANS - 1)))
    return PUSCH_EINVAL;
  pusch_cells_plan given{};
  if (flags & PUSCH_CELLS_WITH_PLAN(0)) {
    const int p = (flags >> 3) & 7;
    given = pusch_cells_plan{p & 1, (p >> 1) & 1, (p >> 2) & 1};
    if (!force) force = &given;
  }
  const bool mx = (flags & PUSCH_CELLS_MIXED) != 0;
  // one workspace slice per cell, in order
  std::vector<char*> base(n_cells);
  std::vector<size_t> slice(n_cells);
  size_t wall = 0;
  for (int c = 0; c < n_cells; ++c) {
    if (int rc = check_geom(&d[c])) return rc;
    if (n_slot[c] < 0) return PUSCH_EINVAL;
    if (d[c].fft_mfma) return PUSCH_EUNSUPPORTED;  // the grouped FFT runs on the vector units
    slice[c] = align256(slot_layout(&d[c], n_slot[c], mx).total);
    base[c] = static_cast<char*>(ws) + wall;
    wall += slice[c];
  }
  if (!ws) return PUSCH_EINVAL;
  if (ws_bytes < wall) return PUSCH_ENOMEM;
  // every cell as a pusch_slot call on its workspace slice, and no cell's
  // output may overlap another cell's output or input
  for (int c = 0; c < n_cells; ++c) {
    if (int rc = check_slot_call(&d[c], n_slot[c], x_td[c], x_hat[c], status ? status[c] : nullptr, base[c],
                                 slice[c], mx))
      return rc;
    const long long ob = out_bytes(&d[c], n_slot[c]), sb = n_slot[c] * (long long)d[c].n_sc * 4;
    const long long xb_c = n_slot[c] * (long long)d[c].n_symb * d[c].n_ant * d[c].n_fft * 8;
    const long long wb = (long long)wall;  // every slice is in use at once
    if (overlap(ws, wb, x_hat[c], ob) || overlap(ws, wb, status ? status[c] : nullptr, sb) ||
        overlap(ws, wb, x_td[c], xb_c) ||
        overlap(ws, wb, d[c].pilots, n_slot[c] * (long long)d[c].n_pilot * d[c].n_sc * 8) ||
        overlap(ws, wb, d[c].W, (long long)d[c].n_beams * d[c].n_ant * 8))
      return PUSCH_EINVAL;
    const float* e_c = d[c].noise_est ? d[c].sigma2_est : nullptr;
    const long long eb = n_slot[c] * 4;
    if (overlap(ws, wb, e_c, eb)) return PUSCH_EINVAL;
    for (int e = 0; e < n_cells; ++e) {
      if (e == c) continue;
      const long long xb = n_slot[e] * (long long)d[e].n_symb * d[e].n_ant * d[e].n_fft * 8;
      const long long ob2 = out_bytes(&d[e], n_slot[e]), sb2 = n_slot[e] * (long long)d[e].n_sc * 4;
      const void* st_c = status ? status[c] : nullptr;
      const void* st_e = status ? status[e] : nullptr;
      if (overlap(x_hat[c], ob, x_td[e], xb) || overlap(x_hat[c], ob, x_hat[e], ob2) ||
          overlap(x_hat[c], ob, st_e, sb2) || overlap(st_c, sb, x_td[e], xb) || overlap(st_c, sb, st_e, sb2) ||
          overlap(x_hat[c], ob, d[e].pilots, n_slot[e] * (long long)d[e].n_pilot * d[e].n_sc * 8) ||
          overlap(st_c, sb, d[e].pilots, n_slot[e] * (long long)d[e].n_pilot * d[e].n_sc * 8))
        return PUSCH_EINVAL;
      // a cell's estimates against every buffer of another cell
      const float* e_e = d[e].noise_est ? d[e].sigma2_est : nullptr;
      if (overlap(e_c, eb, x_td[e], xb) || overlap(e_c, eb, x_hat[e], ob2) || overlap(e_c, eb, st_e, sb2) ||
          overlap(e_c, eb, d[e].pilots, n_slot[e] * (long long)d[e].n_pilot * d[e].n_sc * 8) ||
          overlap(e_c, eb, e_e, n_slot[e] * 4) || overlap(e_c, eb, d[e].W, (long long)d[e].n_beams * d[e].n_ant * 8))
        return PUSCH_EINVAL;
    }
  }
  // which cells the grouped launches take; the rest run on the side streams
  std::vector<int> grouped, streamed;
  for (int c = 0; c < n_cells; ++c) {
    if (n_slot[c] == 0) continue;
    if (!(flags & PUSCH_CELLS_STREAMS) && cell_grouped(&d[c], n_slot[c], mx))
      grouped.push_back(c);
    else
      streamed.push_back(c);
  }
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(t->cells_mu);
  const int used = (int)std::min<size_t>(streamed.size(), kSideStreams);
  // fork: every side stream used waits for the caller's stream
  if (used > 0) {
    if (hipEventRecord(t->fork, s) != hipSuccess) return PUSCH_EHIP;
    for (int i = 0; i < used; ++i)
      if (hipStreamWaitEvent(t->side[i], t->fork, 0) != hipSuccess) return PUSCH_EHIP;
  }
  // the i-th streamed cell on side stream i mod PUSCH_CELL_STREAMS
  int rc = PUSCH_OK;
  for (size_t i = 0; i < streamed.size() && rc == PUSCH_OK; ++i) {
    const int c = streamed[i];
    rc = run_slot(t, &d[c], n_slot[c], x_td[c], x_hat[c], status ? status[c] : nullptr, base[c],
                  t->side[i % kSideStreams], false, mx);
  }
  int side_grouped = 0;
  if (rc == PUSCH_OK && !grouped.empty()) {
    const pusch_cells_plan plan = force ? *force : cells_plan(t, cells_signature(d, n_cells, n_slot, flags));
    rc = run_cells_grouped(t, d, n_slot, x_td, x_hat, status, base, grouped, mx, plan, s, &side_grouped);
  }
  // join (also after a failed launch, so the caller's stream never runs
  // ahead of work already enqueued on a side stream)
  for (int i = 0; i < std::max(used, side_grouped); ++i)
    if (hipEventRecord(t->join[i], t->side[i]) != hipSuccess || hipStreamWaitEvent(s, t->join[i], 0) != hipSuccess)
      rc = PUSCH_EHIP;
  return rc;
}

}  // namespace

extern "C" {

int pusch_profile_begin(int max_calls) {
  if (max_calls < 1 || max_calls > (1 << 20)) return PUSCH_EINVAL;
  std::lock_guard<std::mutex> lock(g_prof.mu);
  if (g_prof.active) return PUSCH_EINVAL;
  g_prof.ev.assign((size_t)max_calls * kEvPerCall, nullptr);
  // timing-only markers: no system-scope release, so recording them between
  // the stage launches adds no cache flush to the measured chain
  for (auto& e : g_prof.ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
      for (auto& f : g_prof.ev)
        if (f) (void)hipEventDestroy(f);
      g_prof.ev.clear();
      return PUSCH_EHIP;
    }
  g_prof.max_calls = max_calls;
  g_prof.calls = 0;
  g_prof.active = true;
  return PUSCH_OK;
}

int pusch_profile_end(float* stage_ms, int n) {
  std::lock_guard<std::mutex> lock(g_prof.mu);
  if (!g_prof.active) return PUSCH_EINVAL;
  int rc = PUSCH_OK;
  double sum[PUSCH_SLOT_STAGES] = {0, 0, 0, 0};
  if (g_prof.calls > 0) {
    if (hipEventSynchronize(g_prof.ev[(size_t)g_prof.calls * kEvPerCall - 1]) != hipSuccess) rc = PUSCH_EHIP;
    for (int c = 0; c < g_prof.calls && rc == PUSCH_OK; ++c)
      for (int st = 0; st < PUSCH_SLOT_STAGES; ++st) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g_prof.ev[(size_t)c * kEvPerCall + st],
                                g_prof.ev[(size_t)c * kEvPerCall + st + 1]) != hipSuccess) {
          rc = PUSCH_EHIP;
          break;
        }
        sum[st] += ms;
      }
  }
  for (int st = 0; st < n && st < PUSCH_SLOT_STAGES; ++st)
    if (stage_ms) stage_ms[st] = (float)sum[st];
  for (auto& e : g_prof.ev) (void)hipEventDestroy(e);
  g_prof.ev.clear();
  g_prof.active = false;
  const int calls = g_prof.calls;
  g_prof.calls = 0;
  return rc == PUSCH_OK ? calls : rc;
}

}  // extern "C"

// ---------------------------------------------------------------- LS-estimate denoiser
namespace {

constexpr int kDnMaxSc = 4096;

int check_dn_grid(int n_symb, int n_sc, long long n_grid) {
  if (n_symb < 1 || n_symb > PUSCH_MAX_SYMBOLS || n_sc < 1 || n_sc > kDnMaxSc || n_grid < 0) return PUSCH_EINVAL;
  // positions and wave tiles fit the kernels' index arithmetic
  if (n_grid * n_symb * (long long)n_sc > (1ll << 40)) return PUSCH_EUNSUPPORTED;
  return PUSCH_OK;
}

// Workspace of pusch_slot_denoised (byte offsets).
struct DnSlotLayout {
  size_t off_xa, off_y, off_g, off_d, off_dn, off_h[2], off_x[2], off_st[2], off_res, total;
};

DnSlotLayout dn_slot_layout(const pusch_slot_desc* d, long long n_slot) {
  const size_t S = d->n_symb, R = d->n_ant, K = d->n_sc, B = d->n_beams, L = d->n_ue, P = d->n_pilot;
  const size_t D = S - P, n = (size_t)n_slot;
  DnSlotLayout lay;
  lay.off_xa = 0;
  lay.off_y = align256(n * S * R * xa_pitch(d->n_sc) * 8);
  size_t o = lay.off_y + align256(n * S * K * B * 8);
  const size_t grid = align256(n * L * B * S * K * 8);
  lay.off_g = o;
  o += grid;
  lay.off_d = o;
  o += grid;
  lay.off_dn = o;
  o += align256((size_t)pusch::dn_layout(d->n_symb, d->n_sc, n_slot * L * B, 0).fwd_total);
  for (int e = 0; e < 2; ++e) {
    lay.off_h[e] = o;
    o += align256(D * n * K * L * B * 8);
    lay.off_x[e] = o;
    o += align256(n * D * K * L * 8);
    lay.off_st[e] = o;
    o += align256(n * K * 4);
  }
  lay.off_res = o;
  o += align256(n * 2 * 4);
  lay.total = o;
  return lay;
}

int check_dn_slot_geom(const pusch_slot_desc* d) {
  if (int rc = check_geom(d)) return rc;
  if (d->refine || d->time_varying || d->noise_est || d->comb_aligned || d->fft_mfma) return PUSCH_EUNSUPPORTED;
  if (!(d->sigma2 > 0.f) || !std::isfinite(d->sigma2)) return PUSCH_EINVAL;  // the network's unit
  if (d->n_ant > 1024) return PUSCH_EUNSUPPORTED;
  return PUSCH_OK;
}

}  // namespace

extern "C" {

size_t pusch_dn_workspace_bytes(int n_symb, int n_sc, long long n_grid) {
  if (check_dn_grid(n_symb, n_sc, n_grid) != PUSCH_OK) return 0;
  return (size_t)pusch::dn_layout(n_symb, n_sc, n_grid, 0).total;
}

int pusch_dn_ls_grid(const pusch_c32* Yp, const pusch_c32* pilots, pusch_c32* grid, int n_beams, int n_ue, int n_sc,
                     int n_symb, int n_pilot, const int* pilot_symb, long long batch, void* stream) {
  if (!Yp || !pilots || !grid || !pilot_symb || batch < 0) return PUSCH_EINVAL;
  if (n_beams < 1 || n_beams > PUSCH_MAX_BEAMS || n_ue < 1 || n_ue > PUSCH_MAX_UES || n_ue > n_beams) return PUSCH_EINVAL;
  if (n_pilot < 1 || n_pilot > PUSCH_MAX_PILOTS || n_symb < 1 || n_symb > PUSCH_MAX_SYMBOLS) return PUSCH_EINVAL;
  if (n_sc < n_ue || n_sc > kDnMaxSc) return PUSCH_EINVAL;
  for (int j = 0; j < n_pilot; ++j)
    if (pilot_symb[j] < 0 || pilot_symb[j] >= n_symb || (j > 0 && pilot_symb[j] <= pilot_symb[j - 1]))
      return PUSCH_EINVAL;
  const long long yb = batch * n_pilot * (long long)n_sc * n_beams * 8, pb = batch * n_pilot * (long long)n_sc * 8;
  const long long gb = batch * n_ue * (long long)n_beams * n_symb * n_sc * 8;
  if (overlap(grid, gb, Yp, yb) || overlap(grid, gb, pilots, pb)) return PUSCH_EINVAL;
  if (batch == 0) return PUSCH_OK;
  pusch::DnGridGeom g{};
  g.n_beams = n_beams;
  g.n_ue = n_ue;
  g.n_sc = n_sc;
  g.n_symb = n_symb;
  g.n_pilot = n_pilot;
  for (int j = 0; j < n_pilot; ++j) {
    g.pilot_sym[j] = pilot_symb[j];
    g.y_off[j] = (long long)j * n_sc * n_beams;
  }
  g.y_batch = (long long)n_pilot * n_sc * n_beams;
  g.p_batch = (long long)n_pilot * n_sc;
  return hip_status(pusch::launch_dn_ls_grid(reinterpret_cast<const cf*>(Yp), reinterpret_cast<const cf*>(pilots),
                                             reinterpret_cast<cf*>(grid), g, batch, static_cast<hipStream_t>(stream)));
}

int pusch_dn_forward(const float* params, const pusch_c32* grid, pusch_c32* out, float sigma, int n_symb, int n_sc,
                     long long n_grid, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !grid || !out || !ws) return PUSCH_EINVAL;
  if (!(sigma > 0.f) || !std::isfinite(sigma) || !std::isfinite(1.f / sigma)) return PUSCH_EINVAL;
  if (int rc = check_dn_grid(n_symb, n_sc, n_grid)) return rc;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return PUSCH_EINVAL;
  const pusch::DnLayout lay = pusch::dn_layout(n_symb, n_sc, n_grid, 0);
  if (ws_bytes < (size_t)lay.fwd_total) return PUSCH_ENOMEM;
  const long long gb = n_grid * n_symb * (long long)n_sc * 8;
  if (overlap(out, gb, grid, gb) || overlap(out, gb, ws, lay.fwd_total) || overlap(ws, lay.fwd_total, grid, gb) ||
      overlap(params, pusch::kDnParams * 4, ws, lay.fwd_total) || overlap(params, pusch::kDnParams * 4, out, gb))
    return PUSCH_EINVAL;
  if (n_grid == 0) return PUSCH_OK;
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  return hip_status(pusch::launch_dn_forward(params, reinterpret_cast<const cf*>(grid), reinterpret_cast<cf*>(out),
                                             n_symb, n_sc, n_grid, static_cast<char*>(ws), lay, t->n_cu,
                                             static_cast<hipStream_t>(stream), sigma));
}

int pusch_dn_backward(const float* params, const pusch_c32* grid, const pusch_c32* dout, float* grads, int n_symb,
                      int n_sc, long long n_grid, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !grid || !dout || !grads || !ws) return PUSCH_EINVAL;
  if (int rc = check_dn_grid(n_symb, n_sc, n_grid)) return rc;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return PUSCH_EINVAL;
  const pusch::DnLayout lay = pusch::dn_layout(n_symb, n_sc, n_grid, 0);
  if (ws_bytes < (size_t)lay.total) return PUSCH_ENOMEM;
  const long long gb = n_grid * n_symb * (long long)n_sc * 8, pn = pusch::kDnParams * 4;
  if (overlap(grads, pn, ws, lay.total) || overlap(grads, pn, params, pn) || overlap(grads, pn, grid, gb) ||
      overlap(grads, pn, dout, gb) || overlap(ws, lay.total, grid, gb) || overlap(ws, lay.total, dout, gb) ||
      overlap(ws, lay.total, params, pn))
    return PUSCH_EINVAL;
  if (n_grid == 0) return PUSCH_EINVAL;  // a gradient needs at least one grid
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  return hip_status(pusch::launch_dn_backward(params, reinterpret_cast<const cf*>(grid), reinterpret_cast<const cf*>(dout),
                                              grads, n_symb, n_sc, n_grid, static_cast<char*>(ws), lay, t->n_cu,
                                              static_cast<hipStream_t>(stream)));
}

int pusch_dn_loss(const pusch_c32* out, const pusch_c32* target, const float* weights, pusch_c32* dout, float* loss,
                  int n_symb, int n_sc, long long n_grid, void* ws, size_t ws_bytes, void* stream) {
  if (!out || !target || !dout || !loss || !ws) return PUSCH_EINVAL;
  if (int rc = check_dn_grid(n_symb, n_sc, n_grid)) return rc;
  if (n_grid == 0) return PUSCH_EINVAL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return PUSCH_EINVAL;
  const pusch::DnLayout lay = pusch::dn_layout(n_symb, n_sc, n_grid, 0);
  if (ws_bytes < (size_t)lay.total) return PUSCH_ENOMEM;
  const long long n = n_grid * n_symb * (long long)n_sc, gb = n * 8;
  if (overlap(dout, gb, out, gb) || overlap(dout, gb, target, gb) || overlap(dout, gb, ws, lay.total) ||
      overlap(loss, 4, dout, gb) || overlap(loss, 4, ws, lay.total) || overlap(loss, 4, out, gb) ||
      overlap(loss, 4, target, gb))
    return PUSCH_EINVAL;
  if (weights && (overlap(weights, n_grid * 4, dout, gb) || overlap(weights, n_grid * 4, loss, 4)))
    return PUSCH_EINVAL;
  return hip_status(pusch::launch_dn_loss(reinterpret_cast<const cf*>(out), reinterpret_cast<const cf*>(target),
                                          weights, (long long)n_symb * n_sc, reinterpret_cast<cf*>(dout), loss, n,
                                          static_cast<char*>(ws), lay, static_cast<hipStream_t>(stream)));
}

int pusch_dn_adam(float* params, const float* grads, float* m, float* v, int step, float lr, float beta1, float beta2,
                  float eps, void* stream) {
  if (!params || !grads || !m || !v || step < 1) return PUSCH_EINVAL;
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return PUSCH_EINVAL;
  const long long pn = pusch::kDnParams * 4;
  if (overlap(params, pn, grads, pn) || overlap(params, pn, m, pn) || overlap(params, pn, v, pn) ||
      overlap(m, pn, v, pn) || overlap(m, pn, grads, pn) || overlap(v, pn, grads, pn))
    return PUSCH_EINVAL;
  const float c1 = (float)(1.0 - std::pow((double)beta1, step)), c2 = (float)(1.0 - std::pow((double)beta2, step));
  return hip_status(pusch::launch_dn_adam(params, grads, m, v, pusch::kDnParams, lr, beta1, beta2, eps, c1, c2,
                                          static_cast<hipStream_t>(stream)));
}

size_t pusch_slot_denoised_workspace_bytes(const pusch_slot_desc* d, long long n_slot) {
  if (check_dn_slot_geom(d) != PUSCH_OK || n_slot < 0) return 0;
  return dn_slot_layout(d, n_slot).total;
}

int pusch_slot_denoised(const pusch_slot_desc* d, long long n_slot, const pusch_c32* x_td, const float* dn_params,
                        pusch_c32* x_hat, int32_t* status, int32_t* used_dn, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_dn_slot_geom(d)) return rc;
  if (int rc = check_desc(d)) return rc;
  if (!dn_params || n_slot < 0 || !x_td || !x_hat || !ws) return PUSCH_EINVAL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return PUSCH_EINVAL;
  const DnSlotLayout lay = dn_slot_layout(d, n_slot);
  if (ws_bytes < lay.total) return PUSCH_ENOMEM;
  const int S = d->n_symb, R = d->n_ant, K = d->n_sc, B = d->n_beams, L = d->n_ue, P = d->n_pilot, D = S - P;
  {
    const long long xb = n_slot * (long long)S * R * d->n_fft * 8, ob = (long long)out_bytes(d, n_slot),
                    sb = n_slot * (long long)K * 4, ub = n_slot * 4, wb = (long long)lay.total,
                    pb = n_slot * (long long)P * K * 8, pn = pusch::kDnParams * 4;
    if (overlap(x_hat, ob, x_td, xb) || overlap(x_hat, ob, ws, wb) || overlap(x_hat, ob, status, sb) ||
        overlap(ws, wb, x_td, xb) || overlap(status, sb, x_td, xb) || overlap(status, sb, ws, wb) ||
        overlap(ws, wb, d->pilots, pb) || overlap(ws, wb, d->W, (long long)B * R * 8) || overlap(ws, wb, dn_params, pn) ||
        overlap(used_dn, ub, ws, wb) || overlap(used_dn, ub, x_hat, ob) || overlap(used_dn, ub, status, sb) ||
        overlap(used_dn, ub, x_td, xb) || overlap(x_hat, ob, dn_params, pn) || overlap(status, sb, dn_params, pn))
      return PUSCH_EINVAL;
  }
  if (n_slot == 0) return PUSCH_OK;
  DeviceTables* t = nullptr;
  if (int rc = device_tables(&t)) return rc;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const cf* w = reinterpret_cast<const cf*>(d->W);
  if (!w)
    if (int rc = dft_beamformer(t, B, R, &w)) return rc;
  const cf* pil = reinterpret_cast<const cf*>(d->pilots);
  cf* Xa = reinterpret_cast<cf*>(base + lay.off_xa);
  cf* Y = reinterpret_cast<cf*>(base + lay.off_y);
  cf* G = reinterpret_cast<cf*>(base + lay.off_g);
  cf* Dn = reinterpret_cast<cf*>(base + lay.off_d);
  float* res = reinterpret_cast<float*>(base + lay.off_res);
  const long long n_grid = n_slot * L * B;
  const pusch::DnLayout dl = pusch::dn_layout(S, K, n_grid, t->n_cu);

  // OFDM demodulation and beamforming (RE-major, received values)
  const long long KP = (long long)xa_pitch(K);
  if (pusch::launch_fft(reinterpret_cast<const cf*>(x_td), Xa, d->n_fft, n_slot * S * R, K, K / 2, KP, t->twiddles,
                        t->n_cu, s) != hipSuccess)
    return PUSCH_EHIP;
  if (pusch::launch_beamform(w, Xa, Y, B, R, K, KP, R * KP, (long long)K * B, n_slot * S, t->n_cu, s) != hipSuccess)
    return PUSCH_EHIP;
  // the LS estimate on every symbol, and the network on it
  pusch::DnGridGeom gg{};
  gg.n_beams = B;
  gg.n_ue = L;
  gg.n_sc = K;
  gg.n_symb = S;
  gg.n_pilot = P;
  for (int j = 0; j < P; ++j) {
    gg.pilot_sym[j] = d->pilot_symb[j];
    gg.y_off[j] = (long long)d->pilot_symb[j] * K * B;
  }
  gg.y_batch = (long long)S * K * B;
  gg.p_batch = (long long)P * K;
  if (pusch::launch_dn_ls_grid(Y, pil, G, gg, n_slot, s) != hipSuccess) return PUSCH_EHIP;
  // the network runs on the estimate in units of the noise standard deviation
  const float sig = std::sqrt(d->sigma2);
  if (pusch::launch_dn_forward(dn_params, G, Dn, S, K, n_grid, base + lay.off_dn, dl, t->n_cu, s, sig) != hipSuccess)
    return PUSCH_EHIP;
  // Eq. 2 for every data symbol with each estimate of that symbol
  pusch::MmseGeom mg{};
  mg.n_beams = B;
  mg.n_ue = L;
  mg.n_sc = K;
  mg.n_data = 1;
  mg.sigma2 = d->sigma2;
  mg.h_batch = (long long)K * L * B;
  mg.y_batch = (long long)S * K * B;
  mg.y_sym = (long long)K * B;
  mg.n_skip = P;
  for (int j = 0; j < P; ++j) mg.skip[j] = d->pilot_symb[j];
  mg.x_batch = (long long)D * K * L;
  mg.st_batch = K;
  pusch::DnSymbols ds{};
  for (int sym = 0; sym < S; ++sym) {
    bool pilot = false;
    for (int j = 0; j < P; ++j) pilot |= d->pilot_symb[j] == sym;
    if (!pilot) ds.sym[ds.n_data++] = sym;
  }
  cf* He[2];
  cf* Xe[2];
  int* Se[2];
  for (int e = 0; e < 2; ++e) {
    He[e] = reinterpret_cast<cf*>(base + lay.off_h[e]);
    Xe[e] = reinterpret_cast<cf*>(base + lay.off_x[e]);
    Se[e] = reinterpret_cast<int*>(base + lay.off_st[e]);
    for (int dd = 0; dd < D; ++dd) {
      cf* H = He[e] + (long long)dd * n_slot * K * L * B;
      if (pusch::launch_dn_grid_to_h(e ? Dn : G, nullptr, nullptr, 1, H, ds.sym[dd], L, B, S, K, n_slot, s) !=
          hipSuccess)
        return PUSCH_EHIP;
      pusch::MmseGeom m1 = mg;
      m1.d_first = dd;
      m1.st_or = dd > 0;
      if (pusch::launch_mmse(H, Y, Xe[e] + (long long)dd * K * L, Se[e], m1, n_slot, s) != hipSuccess)
        return PUSCH_EHIP;
    }
  }
  // fallback test: the post-MMSE residual of each over the data REs, and the pick
  if (pusch::launch_dn_residual(He[0], He[1], Xe[0], Xe[1], Y, res, ds, L, B, K, n_slot, (long long)S * K * B, s) !=
      hipSuccess)
    return PUSCH_EHIP;
  if (pusch::launch_dn_select(res, Xe[0], Xe[1], Se[0], Se[1], reinterpret_cast<cf*>(x_hat), status, used_dn,
                              (long long)D * K * L, K, n_slot, s) != hipSuccess)
    return PUSCH_EHIP;
  return PUSCH_OK;
}

}  // extern "C"
