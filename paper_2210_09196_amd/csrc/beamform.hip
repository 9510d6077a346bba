// Beamforming (Sec. II; Table 1, row "BF"): a complex matrix product with
// known coefficients, Y_i[n][b] = sum_a W[b][a] X_i[a][n], on gfx950 matrix
// cores.
//
// The paper computes 4x4 output windows per core in registers (Sec. V-B);
// here the matrix cores take that role.  Every complex step takes three real
// products (Gauss/Karatsuba):
//   T1 = Wr Xr,  T2 = Wi Xi,  T3 = (Wr + Wi)(Xr + Xi),
//   Yr = T1 - T2,  Yi = T3 - T1 - T2,
// 25% fewer matrix-core operations than the four-product form, with W staged
// once per workgroup in LDS in operand order (Wr, Wi, Wr + Wi per lane).
// Three kernels:
//   k_beamform_k (up to 64 antennas): a wavefront owns 16 REs x (16*MT
//     beams), keeps its tile's whole antenna axis in registers and prefetches
//     the next tile during the current one's v_mfma_f32_16x16x4_f32s;
//   k_beamform_h16 (mixed-precision slot): the same tiles from FP16 grids
//     with per-row power-of-two scales, on v_mfma_f32_16x16x16_f16;
//     k_beamform_b16 from bfloat16 grids on v_mfma_f32_16x16x16_bf16;
//   k_beamform (any antenna count): 32-RE tiles walking the antenna axis in
//     double-buffered chunks of 16.
// Operand layouts of the 16x16x4 instruction: lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and receives D[4*(l/16)+v][l%16].
//
// Optional epilogue for the fused slot: outputs of pilot symbols are turned
// into LS channel values y * conj(p) / |p|^2 before they are stored (the
// element-wise division of the paper's channel-estimation step).
#include <hip/hip_fp16.h>

#include "comb_ls.h"
#include "kernels.h"

namespace pusch {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kTileN = 32;  // REs per wavefront tile (two interleaved 16-column MFMA tiles)

__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// X operand of K-step ks for this lane: antenna ks*4 + kq, columns nc and
// nc+1.  load_x_raw reads from a clamped in-bounds address with no branch;
// mask_x zeroes the out-of-range entries when the operand is consumed, so a
// prefetched load has no consumer until the next chunk.  VEC: one 16-byte
// load (even row pitch, batch stride and RE count).
template <bool VEC>
__device__ __forceinline__ int4 load_x_raw(const cf* __restrict__ Xb, long long ldx, int ks, int kq, int na, int nc,
                                           int nre) {
  const int a = ks * 4 + kq;
  const cf* row = Xb + (long long)(a < na ? a : na - 1) * ldx;
  if (VEC) return *reinterpret_cast<const int4*>(row + (nc < nre ? nc : nre - 2));
  const int2 v0 = *reinterpret_cast<const int2*>(row + (nc < nre ? nc : nre - 1));
  const int2 v1 = *reinterpret_cast<const int2*>(row + (nc + 1 < nre ? nc + 1 : nre - 1));
  return make_int4(v0.x, v0.y, v1.x, v1.y);
}

__device__ __forceinline__ float4 mask_x(int4 v, int ks, int kq, int na, int nc, int nre) {
  const bool ok = ks * 4 + kq < na;
  const int m0 = -(int)(ok && nc < nre), m1 = -(int)(ok && nc + 1 < nre);
  return make_float4(__int_as_float(v.x & m0), __int_as_float(v.y & m0), __int_as_float(v.z & m1),
                     __int_as_float(v.w & m1));
}

// Any antenna count: a wavefront owns (16*MT beams) x 32 REs.  Its two
// 16-column MFMA tiles take interleaved columns (lane c owns columns 2c and
// 2c+1), so one 16-byte load of the interleaved complex grid feeds both; the
// antenna axis goes in double-buffered chunks of 4 K-steps; W is read from
// LDS when it fits (64 KB), else from global memory.
template <int MT, bool W_LDS, bool VEC>
__global__ __launch_bounds__(64 * kWaves) void k_beamform(const cf* __restrict__ W, const cf* __restrict__ X,
                                                          cf* __restrict__ Y, int nb, int na, int nre, long long ldx,
                                                          long long sx, long long sy, long long batch, long long ntn,
                                                          PilotScale ps) {
  extern __shared__ float4 wl[];  // [ks][m][lane] = (Wr, Wi, Wr + Wi, 0)
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;  // A row / B column / D column inside a 16x16 tile
  const int kq = lane >> 4;   // A column / B row (antenna within the step of 4)
  const int ksteps = (na + 3) >> 2;
  const int kspad = (ksteps + 3) & ~3;  // whole chunks of 4 steps

  if (W_LDS) {
    for (int e = threadIdx.x; e < kspad * MT * 64; e += blockDim.x) {
      const int l = e & 63, m = (e >> 6) % MT, ks = (e >> 6) / MT;
      const int b = m * 16 + (l & 15), a = ks * 4 + (l >> 4);
      const cf w = (a < na && b < nb) ? W[b * na + a] : cf{0.f, 0.f};
      wl[e] = make_float4(w.r, w.i, w.r + w.i, 0.f);
    }
    __syncthreads();
  }

  const long long nwave = (long long)gridDim.x * kWaves;
  for (long long tile = (long long)blockIdx.x * kWaves + (threadIdx.x >> 6); tile < batch * ntn; tile += nwave) {
    const long long bi = tile / ntn;
    const int n0 = (int)(tile - bi * ntn) * kTileN;
    const int nc = n0 + 2 * col;  // this lane's two columns: nc, nc + 1
    const cf* Xb = X + bi * sx;
    f32x4 t1[MT][2], t2[MT][2], t3[MT][2];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int t = 0; t < 2; ++t) t1[m][t] = t2[m][t] = t3[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    // K loop in chunks of 4 steps (16 antennas): the next chunk's loads are
    // issued before the current chunk's 48 MFMAs (double buffering)
    constexpr int CH = 4;
    int4 xa[CH], xb[CH];
    // one chunk of CH K-steps: 12*MT MFMAs per step
    auto chunk = [&](const int4 (&xr)[CH], int kc) {
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int ks = kc + u;
        const float4 xv = mask_x(xr[u], ks, kq, na, nc, nre);
        const cf x0 = cf{xv.x, xv.y}, x1 = cf{xv.z, xv.w};
        const float s0 = x0.r + x0.i, s1 = x1.r + x1.i;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          float4 w;
          if (W_LDS) {
            w = wl[(ks * MT + m) * 64 + lane];
          } else {
            const int b = m * 16 + col, a = ks * 4 + kq;
            const cf c = (a < na && b < nb) ? W[b * na + a] : cf{0.f, 0.f};
            w = make_float4(c.r, c.i, c.r + c.i, 0.f);
          }
          t1[m][0] = mfma(w.x, x0.r, t1[m][0]);
          t2[m][0] = mfma(w.y, x0.i, t2[m][0]);
          t3[m][0] = mfma(w.z, s0, t3[m][0]);
          t1[m][1] = mfma(w.x, x1.r, t1[m][1]);
          t2[m][1] = mfma(w.y, x1.i, t2[m][1]);
          t3[m][1] = mfma(w.z, s1, t3[m][1]);
        }
      }
    };
    // ping-pong double buffering: the next chunk's loads are issued before
    // the current chunk's MFMAs and are never copied while in flight (the
    // last prefetches re-read a clamped step and are dropped)
    const int klast = (ksteps - 1) & ~(CH - 1);  // first step of the last chunk
#pragma unroll
    for (int u = 0; u < CH; ++u) xa[u] = load_x_raw<VEC>(Xb, ldx, u, kq, na, nc, nre);
    for (int kc = 0; kc < ksteps; kc += 2 * CH) {
      const int k1 = kc + CH <= klast ? kc + CH : klast;
#pragma unroll
      for (int u = 0; u < CH; ++u) xb[u] = load_x_raw<VEC>(Xb, ldx, k1 + u, kq, na, nc, nre);
      __builtin_amdgcn_sched_barrier(0);
      chunk(xa, kc);
      const int k2 = kc + 2 * CH <= klast ? kc + 2 * CH : klast;
#pragma unroll
      for (int u = 0; u < CH; ++u) xa[u] = load_x_raw<VEC>(Xb, ldx, k2 + u, kq, na, nc, nre);
      __builtin_amdgcn_sched_barrier(0);
      if (kc + CH < ksteps) chunk(xb, kc + CH);
    }

    // optional LS epilogue for pilot symbols
    cf sc[2] = {cf{1.f, 0.f}, cf{1.f, 0.f}};
    bool scaled = false;
    if (ps.pilots) {
      const long long slot = bi / ps.n_symb;
      const int j = ps.pilot_of[bi - slot * ps.n_symb];
      if (j >= 0) {
        scaled = true;
        const cf* pv = ps.pilots + slot * ps.p_slot + (long long)j * nre;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if (nc + t < nre) {
            const cf p = pv[nc + t];
            const float inv = fast_rcp(p.r * p.r + p.i * p.i);
            sc[t] = cf{p.r * inv, -p.i * inv};
          }
        }
      }
    }

    cf* Yb = Y + bi * sy;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int n = nc + t;
      if (n >= nre) continue;
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int b0 = m * 16 + kq * 4;
        cf o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float re = t1[m][t][v] - t2[m][t][v];
          const float im = t3[m][t][v] - t1[m][t][v] - t2[m][t][v];
          o[v] = scaled ? cf{re * sc[t].r - im * sc[t].i, re * sc[t].i + im * sc[t].r} : cf{re, im};
        }
        cf* dst = Yb + (long long)n * nb + b0;
        if (b0 + 3 < nb && (nb & 1) == 0) {
          reinterpret_cast<float4*>(dst)[0] = make_float4(o[0].r, o[0].i, o[1].r, o[1].i);
          reinterpret_cast<float4*>(dst)[1] = make_float4(o[2].r, o[2].i, o[3].r, o[3].i);
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (b0 + v < nb) dst[v] = o[v];
        }
      }
    }
  }
}

// Up to 64 antennas: a wavefront owns 16 REs x (16*MT beams) and holds the
// whole antenna axis of its tile in registers (KS K-steps of one 8-byte X
// value per lane); the next tile's loads are in flight while the current
// tile's MFMAs run (ping-pong over a tile loop unrolled by two).  Half the
// accumulators of the 32-RE tile, so two tiles of X fit next to them.
template <int MT, int KS>
__device__ __forceinline__ void bf_k_body(int vb, int vg, const cf* __restrict__ W, const cf* __restrict__ X,
                                          cf* __restrict__ Y, int nb, int na, int nre, long long ldx, long long sx,
                                          long long sy, int ntiles, int ntn, const PilotScale& ps) {
  extern __shared__ float4 wl[];  // [ks][m][lane] = (Wr, Wi, Wr + Wi, 0); zero for padded antennas / beams
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;  // A row / B column / D column inside a 16x16 tile
  const int kq = lane >> 4;   // A column / B row (antenna within the step of 4)
  for (int e = threadIdx.x; e < KS * MT * 64; e += blockDim.x) {
    const int l = e & 63, m = (e >> 6) % MT, ks = (e >> 6) / MT;
    const int b = m * 16 + (l & 15), a = ks * 4 + (l >> 4);
    const cf w = (a < na && b < nb) ? W[b * na + a] : cf{0.f, 0.f};
    wl[e] = make_float4(w.r, w.i, w.r + w.i, 0.f);
  }
  __syncthreads();

  const int nwave = vg * kWaves;
  const int t0 = vb * kWaves + (threadIdx.x >> 6);
  // X operand of every K-step of a tile, from a wave-uniform base with
  // 32-bit lane offsets (the host guarantees n_ant * ldx < 2^28).  Loads are
  // clamped in bounds: padded antennas meet zero W entries, REs past n_re are
  // not stored, and a tile index past the end re-reads the last tile (such a
  // prefetch is dropped).
  auto load = [&](cf (&x)[KS], int tile) {
    tile = tile < ntiles ? tile : ntiles - 1;
    const int bi = tile / ntn;
    const int n = (tile - bi * ntn) * 16 + col;
    const unsigned nn = (unsigned)(n < nre ? n : nre - 1);
    const cf* base = X + bi * sx;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int a = ks * 4 + kq;
      x[ks] = base[(unsigned)(a < na ? a : na - 1) * (unsigned)ldx + nn];
    }
  };
  // X is the A operand and W the B operand, so the result tile is
  // D[RE][beam]: lane (kq, col) receives REs n0 + 4 kq + v of beam col, and
  // sixteen consecutive lanes hold one RE's sixteen consecutive beams (each
  // store instruction writes whole 128-byte lines).
  auto compute = [&](const cf (&x)[KS], int tile) {
    const int bi = tile / ntn;
    const int n0 = (tile - bi * ntn) * 16;
    f32x4 t1[MT], t2[MT], t3[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) t1[m] = t2[m] = t3[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float xr = x[ks].r, xi = x[ks].i, xs = xr + xi;
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const float4 w = wl[(ks * MT + m) * 64 + lane];
        t1[m] = mfma(xr, w.x, t1[m]);
        t2[m] = mfma(xi, w.y, t2[m]);
        t3[m] = mfma(xs, w.z, t3[m]);
      }
    }
    // optional LS epilogue for pilot symbols: y * conj(p) / |p|^2 per RE
    cf sc[4] = {cf{1.f, 0.f}, cf{1.f, 0.f}, cf{1.f, 0.f}, cf{1.f, 0.f}};
    bool scaled = false;
    if (ps.pilots) {
      const long long slot = bi / ps.n_symb;
      const int j = ps.pilot_of[bi - slot * ps.n_symb];
      if (j >= 0) {
        scaled = true;
        const cf* pv = ps.pilots + slot * ps.p_slot + (long long)j * nre;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = n0 + 4 * kq + v;
          const cf p = pv[n < nre ? n : nre - 1];
          const float inv = fast_rcp(p.r * p.r + p.i * p.i);
          sc[v] = cf{p.r * inv, -p.i * inv};
        }
      }
    }
    cf o[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float re = t1[m][v] - t2[m][v];
        const float im = t3[m][v] - t1[m][v] - t2[m][v];
        o[m][v] = scaled ? cf{re * sc[v].r - im * sc[v].i, re * sc[v].i + im * sc[v].r} : cf{re, im};
      }
    cf* yb = Y + bi * sy + (long long)n0 * nb;  // wave-uniform
    if (n0 + 16 <= nre && nb == 16 * MT) {
      // whole tile: 32-bit lane offsets, no per-store checks
      const unsigned lo = (unsigned)(4 * kq * nb + col);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) yb[lo + (unsigned)(v * nb + m * 16)] = o[m][v];
    } else {
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = n0 + 4 * kq + v, b = m * 16 + col;
          if (n < nre && b < nb) yb[(long long)(4 * kq + v) * nb + b] = o[m][v];
        }
    }
  };
  if (t0 >= ntiles) return;
  cf xa[KS], xb[KS];
  load(xa, t0);
  for (int t = t0; t < ntiles; t += 2 * nwave) {
    load(xb, t + nwave);
    __builtin_amdgcn_sched_barrier(0);
    compute(xa, t);
    load(xa, t + 2 * nwave);
    __builtin_amdgcn_sched_barrier(0);
    if (t + nwave < ntiles) compute(xb, t + nwave);
  }
}

template <int MT, int KS>
__global__ __launch_bounds__(64 * kWaves) void k_beamform_k(const cf* __restrict__ W, const cf* __restrict__ X,
                                                            cf* __restrict__ Y, int nb, int na, int nre,
                                                            long long ldx, long long sx, long long sy, int ntiles,
                                                            int ntn, PilotScale ps) {
  bf_k_body<MT, KS>(blockIdx.x, gridDim.x, W, X, Y, nb, na, nre, ldx, sx, sy, ntiles, ntn, ps);
}

// Many cells of one tile shape in one launch: cell c owns workgroups
// [start[c], start[c + 1]) (its W staged once in each) and walks its tiles.
template <int MT, int KS>
__global__ __launch_bounds__(64 * kWaves) void k_beamform_k_cells(BfCells t) {
  int c = 0;
  while (c + 1 < t.n && (int)blockIdx.x >= t.start[c + 1]) ++c;
  const BfCell& e = t.cell[c];
  bf_k_body<MT, KS>(blockIdx.x - t.start[c], t.start[c + 1] - t.start[c], e.W, e.X, e.Y, e.nb, e.na, e.nre, e.ldx,
                    e.sx, e.sy, e.ntiles, e.ntn, e.ps);
}

template <int MT, int KS>
hipError_t launch_k(const cf* W, const cf* X, cf* Y, int nb, int na, int nre,
                    long long ldx, long long sx, long long sy, long long batch, const PilotScale& ps, int n_cu,
                    hipStream_t s) {
  const int ntn = (nre + 15) / 16;
  const long long tiles = batch * ntn;  // < 2^30 (checked by the caller)
  const size_t lds = (size_t)KS * MT * 64 * sizeof(float4);
  // persistent grid of exactly the resident workgroups: every wave walks its
  // tiles from the start, no second round of workgroups and its tail
  static const int per_cu = [&] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_beamform_k<MT, KS>, 64 * kWaves, lds) != hipSuccess ||
        n < 1)
      n = 1;
    return n;
  }();
  long long blocks = (tiles + kWaves - 1) / kWaves;
  const long long cap = (long long)n_cu * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL((k_beamform_k<MT, KS>), dim3((unsigned)blocks), dim3(64 * kWaves), lds, s, W, X, Y, nb, na,
                     nre, ldx, sx, sy, (int)tiles, ntn, ps);
  return hipGetLastError();
}

// FP16 input on FP16 matrix cores (v_mfma_f32_16x16x16_f16, FP32
// accumulation), up to 64 antennas in J blocks of 16.  Lane (kq, col) loads,
// for K-step ks, antenna 4 ks + kq of RE col (as k_beamform_k); the four
// K-steps 4j..4j+3 are the four A-operand halves of block j, i.e. block j
// slot (kq, i) holds antenna 4 (4j + i) + kq.  The contraction over antennas
// does not depend on the order, and W is staged in the same order.  Rows
// carry their own power of two; they are rebased to the symbol's smallest
// exponent (each value scaled down by 2^(e_a - e_min), exact unless it
// drops below the FP16 range, where it is negligible next to the row with
// e_min), and 2^-e_min is applied to the FP32 accumulators.  W is rounded to
// FP16 (entries of a beamformer are O(1); |W| must lie inside FP16's range).
//
// BF (bfloat16 input, Xh written by the FFT's BF16 form): no exponents, the
// words are bfloat16 pairs whose halves are the MFMA operands as they stand;
// only the sum xr + xi of the three-product form is rounded again (to
// nearest even), and the product runs on v_mfma_f32_16x16x16_bf16 (W
// rounded to BF16).
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef short b4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(h4 a, h4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfmab16(b4 a, b4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// FP32 to bfloat16 bits, round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ short bf16_bits(float f) { return __builtin_bit_cast(short, (__bf16)f); }

template <int MT, int J, bool BF = false>
__device__ __forceinline__ void bf_h16_body(int vb, int vg, const cf* __restrict__ W, const unsigned* __restrict__ Xh,
                                            const signed char* __restrict__ ex, cf* __restrict__ Y, int nb, int na,
                                            int nre, long long ldx, long long sx, long long sy, int ntiles, int ntn,
                                            const PilotScale& ps) {
  constexpr int KS = 4 * J;
  // [j][m][lane] = (Wr, Wi, Wr + Wi) as three half4, lane (q, col): beam
  // m*16 + col, antennas 4 (4j + i) + q, i = 0..3; zero past n_ant / n_beams
  extern __shared__ h4 wh[];
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;
  const int kq = lane >> 4;
  for (int e = threadIdx.x; e < J * MT * 64; e += blockDim.x) {
    const int l = e & 63, m = (e >> 6) % MT, j = (e >> 6) / MT;
    const int b = m * 16 + (l & 15), q = l >> 4;
    h4 wr, wi, ws;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int a = 4 * (4 * j + i) + q;
      const cf w = (a < na && b < nb) ? W[b * na + a] : cf{0.f, 0.f};
      if constexpr (BF) {
        wr[i] = __builtin_bit_cast(_Float16, bf16_bits(w.r));
        wi[i] = __builtin_bit_cast(_Float16, bf16_bits(w.i));
        ws[i] = __builtin_bit_cast(_Float16, bf16_bits(w.r + w.i));
      } else {
        wr[i] = (_Float16)w.r;
        wi[i] = (_Float16)w.i;
        ws[i] = (_Float16)(w.r + w.i);
      }
    }
    wh[3 * e] = wr;
    wh[3 * e + 1] = wi;
    wh[3 * e + 2] = ws;
  }
  __syncthreads();

  const int nwave = vg * kWaves;
  const int t0 = vb * kWaves + (threadIdx.x >> 6);
  struct Buf {
    unsigned w[KS];
    int4 e;
  };
  auto load = [&](Buf& xb, int tile) {
    tile = tile < ntiles ? tile : ntiles - 1;
    const int bi = tile / ntn;
    const int n = (tile - bi * ntn) * 16 + col;
    const unsigned nn = (unsigned)(n < nre ? n : nre - 1);
    const unsigned* base = Xh + bi * sx;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int a = ks * 4 + kq;
      xb.w[ks] = base[(unsigned)(a < na ? a : na - 1) * (unsigned)ldx + nn];
    }
    if constexpr (!BF) xb.e = *reinterpret_cast<const int4*>(ex + (long long)bi * 64 + kq * 16);
  };
  auto compute = [&](const Buf& xb, int tile) {
    const int bi = tile / ntn;
    const int n0 = (tile - bi * ntn) * 16;
    // this lane's exponents (antennas past n_ant: never written, ignored)
    int ev[KS];
    int emin = 127;
    if constexpr (!BF) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int word = (ks >> 2) == 0 ? xb.e.x : ((ks >> 2) == 1 ? xb.e.y : ((ks >> 2) == 2 ? xb.e.z : xb.e.w));
        const bool ok = ks * 4 + kq < na;
        ev[ks] = ok ? (int)__builtin_amdgcn_sbfe((unsigned)word, 8 * (ks & 3), 8) : 127;
        emin = ev[ks] < emin ? ev[ks] : emin;
      }
      // symbol-wide minimum: the four antenna groups kq sit 16 lanes apart
      emin = min(emin, __shfl_xor(emin, 16));
      emin = min(emin, __shfl_xor(emin, 32));
    }
    f32x4 t1[MT], t2[MT], t3[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) t1[m] = t2[m] = t3[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if constexpr (BF) {
        b4 ar, ai, as;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const unsigned u = xb.w[4 * j + i];
          ar[i] = (short)(u & 0xffffu);
          ai[i] = (short)(u >> 16);
          as[i] = bf16_bits(__uint_as_float(u << 16) + __uint_as_float(u & 0xffff0000u));
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const h4* w = wh + 3 * ((j * MT + m) * 64 + lane);
          t1[m] = mfmab16(ar, __builtin_bit_cast(b4, w[0]), t1[m]);
          t2[m] = mfmab16(ai, __builtin_bit_cast(b4, w[1]), t2[m]);
          t3[m] = mfmab16(as, __builtin_bit_cast(b4, w[2]), t3[m]);
        }
      } else {
        h4 ar, ai, as;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int ks = 4 * j + i;
          const unsigned u = xb.w[ks];
          const int d = ev[ks] == 127 ? 0 : emin - ev[ks];  // <= 0: scale down to the common exponent
          const float xr = ldexpf(__half2float(__ushort_as_half((unsigned short)(u & 0xffffu))), d);
          const float xi = ldexpf(__half2float(__ushort_as_half((unsigned short)(u >> 16))), d);
          ar[i] = (_Float16)xr;
          ai[i] = (_Float16)xi;
          as[i] = (_Float16)(xr + xi);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const h4* w = wh + 3 * ((j * MT + m) * 64 + lane);
          t1[m] = mfma16(ar, w[0], t1[m]);
          t2[m] = mfma16(ai, w[1], t2[m]);
          t3[m] = mfma16(as, w[2], t3[m]);
        }
      }
    }
    const float escale = BF ? 1.f : ldexpf(1.f, emin == 127 ? 0 : -emin);
    // optional LS epilogue for pilot symbols: y * conj(p) / |p|^2 per RE
    cf sc[4] = {cf{escale, 0.f}, cf{escale, 0.f}, cf{escale, 0.f}, cf{escale, 0.f}};
    if (ps.pilots) {
      const long long slot = bi / ps.n_symb;
      const int jp = ps.pilot_of[bi - slot * ps.n_symb];
      if (jp >= 0) {
        const cf* pv = ps.pilots + slot * ps.p_slot + (long long)jp * nre;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = n0 + 4 * kq + v;
          const cf p = pv[n < nre ? n : nre - 1];
          const float inv = fast_rcp(p.r * p.r + p.i * p.i) * escale;
          sc[v] = cf{p.r * inv, -p.i * inv};
        }
      }
    }
    cf o[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float re = t1[m][v] - t2[m][v];
        const float im = t3[m][v] - t1[m][v] - t2[m][v];
        o[m][v] = cf{re * sc[v].r - im * sc[v].i, re * sc[v].i + im * sc[v].r};
      }
    cf* yb = Y + bi * sy + (long long)n0 * nb;
    if (n0 + 16 <= nre && nb == 16 * MT) {
      const unsigned lo = (unsigned)(4 * kq * nb + col);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) yb[lo + (unsigned)(v * nb + m * 16)] = o[m][v];
    } else {
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = n0 + 4 * kq + v, b = m * 16 + col;
          if (n < nre && b < nb) yb[(long long)(4 * kq + v) * nb + b] = o[m][v];
        }
    }
  };
  if (t0 >= ntiles) return;
  Buf xa, xb;
  load(xa, t0);
  for (int t = t0; t < ntiles; t += 2 * nwave) {
    load(xb, t + nwave);
    __builtin_amdgcn_sched_barrier(0);
    compute(xa, t);
    load(xa, t + 2 * nwave);
    __builtin_amdgcn_sched_barrier(0);
    if (t + nwave < ntiles) compute(xb, t + nwave);
  }
}

template <int MT, int J>
__global__ __launch_bounds__(64 * kWaves) void k_beamform_h16(const cf* __restrict__ W,
                                                              const unsigned* __restrict__ Xh,
                                                              const signed char* __restrict__ ex,
                                                              cf* __restrict__ Y, int nb, int na, int nre,
                                                              long long ldx, long long sx, long long sy, int ntiles,
                                                              int ntn, PilotScale ps) {
  // neighbouring workgroups take neighbouring 16-RE tiles, whose 64-byte row
  // segments share 128-byte lines: keep them on one XCD's L2
  bf_h16_body<MT, J>(xcd_block(blockIdx.x, gridDim.x), gridDim.x, W, Xh, ex, Y, nb, na, nre, ldx, sx, sy, ntiles,
                     ntn, ps);
}

// The same on bfloat16 grids (ex unused).
template <int MT, int J>
__global__ __launch_bounds__(64 * kWaves) void k_beamform_b16(const cf* __restrict__ W,
                                                              const unsigned* __restrict__ Xh,
                                                              cf* __restrict__ Y, int nb, int na, int nre,
                                                              long long ldx, long long sx, long long sy, int ntiles,
                                                              int ntn, PilotScale ps) {
  bf_h16_body<MT, J, true>(xcd_block(blockIdx.x, gridDim.x), gridDim.x, W, Xh, nullptr, Y, nb, na, nre, ldx, sx, sy,
                           ntiles, ntn, ps);
}

template <int MT, int J>
__global__ __launch_bounds__(64 * kWaves) void k_beamform_h16_cells(BfCells t) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);  // as k_beamform_h16
  int c = 0;
  while (c + 1 < t.n && blk >= t.start[c + 1]) ++c;
  const BfCell& e = t.cell[c];
  bf_h16_body<MT, J>(blk - t.start[c], t.start[c + 1] - t.start[c], e.W, e.Xh, e.ex, e.Y, e.nb, e.na, e.nre, e.ldx,
                     e.sx, e.sy, e.ntiles, e.ntn, e.ps);
}

template <int MT, int J>
hipError_t launch_h16(const cf* W, const unsigned* Xh, const signed char* ex, cf* Y, int nb, int na, int nre,
                      long long ldx, long long sx, long long sy, long long batch, const PilotScale& ps, int n_cu,
                      hipStream_t s) {
  const int ntn = (nre + 15) / 16;
  const long long tiles = batch * ntn;  // < 2^30 (checked by the caller)
  const size_t lds = (size_t)J * MT * 64 * 3 * sizeof(h4);
  static const int per_cu = [&] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_beamform_h16<MT, J>, 64 * kWaves, lds) != hipSuccess ||
        n < 1)
      n = 1;
    return n;
  }();
  long long blocks = (tiles + kWaves - 1) / kWaves;
  const long long cap = (long long)n_cu * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL((k_beamform_h16<MT, J>), dim3((unsigned)blocks), dim3(64 * kWaves), lds, s, W, Xh, ex, Y, nb, na,
                     nre, ldx, sx, sy, (int)tiles, ntn, ps);
  return hipGetLastError();
}

template <int MT, int J>
hipError_t launch_b16(const cf* W, const unsigned* Xh, cf* Y, int nb, int na, int nre, long long ldx, long long sx,
                      long long sy, long long batch, const PilotScale& ps, int n_cu, hipStream_t s) {
  const int ntn = (nre + 15) / 16;
  const long long tiles = batch * ntn;  // < 2^30 (checked by the caller)
  const size_t lds = (size_t)J * MT * 64 * 3 * sizeof(h4);
  static const int per_cu = [&] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_beamform_b16<MT, J>, 64 * kWaves, lds) != hipSuccess ||
        n < 1)
      n = 1;
    return n;
  }();
  long long blocks = (tiles + kWaves - 1) / kWaves;
  const long long cap = (long long)n_cu * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL((k_beamform_b16<MT, J>), dim3((unsigned)blocks), dim3(64 * kWaves), lds, s, W, Xh, Y, nb, na,
                     nre, ldx, sx, sy, (int)tiles, ntn, ps);
  return hipGetLastError();
}

template <int MT>
hipError_t launch_k_mt(const cf* W, const cf* X, const unsigned* Xh, const signed char* ex, cf* Y, int nb, int na,
                       int nre, long long ldx, long long sx, long long sy, long long batch, const PilotScale& ps,
                       int n_cu, hipStream_t s) {
  if (Xh && !ex) {
    if (na <= 16) return launch_b16<MT, 1>(W, Xh, Y, nb, na, nre, ldx, sx, sy, batch, ps, n_cu, s);
    if (na <= 32) return launch_b16<MT, 2>(W, Xh, Y, nb, na, nre, ldx, sx, sy, batch, ps, n_cu, s);
    return launch_b16<MT, 4>(W, Xh, Y, nb, na, nre, ldx, sx, sy, batch, ps, n_cu, s);
  }
  if (Xh) {
    if (na <= 16) return launch_h16<MT, 1>(W, Xh, ex, Y, nb, na, nre, ldx, sx, sy, batch, ps, n_cu, s);
    if (na <= 32) return launch_h16<MT, 2>(W, Xh, ex, Y, nb, na, nre, ldx, sx, sy, batch, ps, n_cu, s);
    return launch_h16<MT, 4>(W, Xh, ex, Y, nb, na, nre, ldx, sx, sy, batch, ps, n_cu, s);
  }
  if (na <= 16) return launch_k<MT, 4>(W, X, Y, nb, na, nre, ldx, sx, sy, batch, ps, n_cu, s);
  if (na <= 32) return launch_k<MT, 8>(W, X, Y, nb, na, nre, ldx, sx, sy, batch, ps, n_cu, s);
  return launch_k<MT, 16>(W, X, Y, nb, na, nre, ldx, sx, sy, batch, ps, n_cu, s);
}

// Relative time of one workgroup round (kWaves tiles of 16 REs): the tile's
// padded antennas read plus beams written.
long long bf_round_cost(int cls) { return (long long)(4 << (cls % 3)) * 4 + (cls / 3 + 1) * 16; }

int share_blocks(BfCells& t, long long cap) {
  return share_work(
      t.n, [&](int c) { return (long long)(t.cell[c].ntiles + kWaves - 1) / kWaves; },
      [&](int c) { return bf_round_cost(t.cell[c].cls); }, cap, t.start);
}

// Any tile classes in one launch: each workgroup runs its cell's class (the
// W stage in dynamic LDS is sized for the launch's largest class).
__global__ __launch_bounds__(64 * kWaves) void k_beamform_k_any(BfCells t) {
  int c = 0;
  while (c + 1 < t.n && (int)blockIdx.x >= t.start[c + 1]) ++c;
  const BfCell& e = t.cell[c];
  const int vb = blockIdx.x - t.start[c], vg = t.start[c + 1] - t.start[c];
#define BF_K_CASE(CLS, MT, KS)                                                                                    \
  case CLS:                                                                                                      \
    bf_k_body<MT, KS>(vb, vg, e.W, e.X, e.Y, e.nb, e.na, e.nre, e.ldx, e.sx, e.sy, e.ntiles, e.ntn, e.ps); \
    break;
  switch (e.cls) {
    BF_K_CASE(0, 1, 4)
    BF_K_CASE(1, 1, 8)
    BF_K_CASE(2, 1, 16)
    BF_K_CASE(3, 2, 4)
    BF_K_CASE(4, 2, 8)
    BF_K_CASE(5, 2, 16)
    BF_K_CASE(6, 3, 4)
    BF_K_CASE(7, 3, 8)
    BF_K_CASE(8, 3, 16)
    BF_K_CASE(9, 4, 4)
    BF_K_CASE(10, 4, 8)
    default: BF_K_CASE(11, 4, 16)
  }
#undef BF_K_CASE
}

__global__ __launch_bounds__(64 * kWaves) void k_beamform_h16_any(BfCells t) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);  // as k_beamform_h16
  int c = 0;
  while (c + 1 < t.n && blk >= t.start[c + 1]) ++c;
  const BfCell& e = t.cell[c];
  const int vb = blk - t.start[c], vg = t.start[c + 1] - t.start[c];
#define BF_H_CASE(CLS, MT, J)                                                                                     \
  case CLS:                                                                                                      \
    bf_h16_body<MT, J>(vb, vg, e.W, e.Xh, e.ex, e.Y, e.nb, e.na, e.nre, e.ldx, e.sx, e.sy, e.ntiles, e.ntn, e.ps); \
    break;
  switch (e.cls) {
    BF_H_CASE(0, 1, 1)
    BF_H_CASE(1, 1, 2)
    BF_H_CASE(2, 1, 4)
    BF_H_CASE(3, 2, 1)
    BF_H_CASE(4, 2, 2)
    BF_H_CASE(5, 2, 4)
    BF_H_CASE(6, 3, 1)
    BF_H_CASE(7, 3, 2)
    BF_H_CASE(8, 3, 4)
    BF_H_CASE(9, 4, 1)
    BF_H_CASE(10, 4, 2)
    default: BF_H_CASE(11, 4, 4)
  }
#undef BF_H_CASE
}

// W stage of a class (bytes of dynamic LDS).
size_t bf_class_lds(int cls, bool h16) {
  const int mt = cls / 3 + 1, k = cls % 3;
  return h16 ? (size_t)(1 << k) * mt * 64 * 3 * sizeof(h4) : (size_t)(4 << k) * mt * 64 * sizeof(float4);
}

hipError_t launch_any_cells(BfCells& t, bool h16, int n_cu, hipStream_t s) {
  int top = 0;  // the class with the largest W stage
  for (int c = 0; c < t.n; ++c)
    if (bf_class_lds(t.cell[c].cls, h16) > bf_class_lds(top, h16)) top = t.cell[c].cls;
  const size_t lds = bf_class_lds(top, h16);
  static int per_cu[2][12] = {};  // occupancy by W stage size, looked up once
  int& pc = per_cu[h16][top];
  if (pc == 0) {
    int n = 0;
    const hipError_t e = h16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_beamform_h16_any, 64 * kWaves, lds)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_beamform_k_any, 64 * kWaves, lds);
    pc = (e != hipSuccess || n < 1) ? 1 : n;
  }
  const int blocks = share_blocks(t, (long long)n_cu * pc);
  if (h16)
    hipLaunchKernelGGL(k_beamform_h16_any, dim3((unsigned)blocks), dim3(64 * kWaves), lds, s, t);
  else
    hipLaunchKernelGGL(k_beamform_k_any, dim3((unsigned)blocks), dim3(64 * kWaves), lds, s, t);
  return hipGetLastError();
}

template <int MT, int KS>
hipError_t launch_k_cells(BfCells& t, int n_cu, hipStream_t s) {
  const size_t lds = (size_t)KS * MT * 64 * sizeof(float4);
  static const int per_cu = [&] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_beamform_k_cells<MT, KS>, 64 * kWaves, lds) !=
            hipSuccess ||
        n < 1)
      n = 1;
    return n;
  }();
  const int blocks = share_blocks(t, (long long)n_cu * per_cu);
  hipLaunchKernelGGL((k_beamform_k_cells<MT, KS>), dim3((unsigned)blocks), dim3(64 * kWaves), lds, s, t);
  return hipGetLastError();
}

template <int MT, int J>
hipError_t launch_h16_cells(BfCells& t, int n_cu, hipStream_t s) {
  const size_t lds = (size_t)J * MT * 64 * 3 * sizeof(h4);
  static const int per_cu = [&] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_beamform_h16_cells<MT, J>, 64 * kWaves, lds) !=
            hipSuccess ||
        n < 1)
      n = 1;
    return n;
  }();
  const int blocks = share_blocks(t, (long long)n_cu * per_cu);
  hipLaunchKernelGGL((k_beamform_h16_cells<MT, J>), dim3((unsigned)blocks), dim3(64 * kWaves), lds, s, t);
  return hipGetLastError();
}

template <int MT>
hipError_t launch_cells_mt(BfCells& t, int ks_class, bool h16, int n_cu, hipStream_t s) {
  if (h16) {
    if (ks_class == 0) return launch_h16_cells<MT, 1>(t, n_cu, s);
    if (ks_class == 1) return launch_h16_cells<MT, 2>(t, n_cu, s);
    return launch_h16_cells<MT, 4>(t, n_cu, s);
  }
  if (ks_class == 0) return launch_k_cells<MT, 4>(t, n_cu, s);
  if (ks_class == 1) return launch_k_cells<MT, 8>(t, n_cu, s);
  return launch_k_cells<MT, 16>(t, n_cu, s);
}

constexpr size_t kWLdsMax = 64 * 1024;

template <int MT, bool VEC>
hipError_t launch_mtv(const cf* W, const cf* X, cf* Y, int nb, int na, int nre, long long ldx, long long sx,
                      long long sy, long long batch, long long ntn, const PilotScale& ps, dim3 grid, hipStream_t s) {
  const size_t lds = (size_t)((((na + 3) / 4) + 3) & ~3) * MT * 64 * sizeof(float4);
  if (lds <= kWLdsMax)
    hipLaunchKernelGGL((k_beamform<MT, true, VEC>), grid, dim3(64 * kWaves), lds, s, W, X, Y, nb, na, nre, ldx, sx,
                       sy, batch, ntn, ps);
  else
    hipLaunchKernelGGL((k_beamform<MT, false, VEC>), grid, dim3(64 * kWaves), 0, s, W, X, Y, nb, na, nre, ldx, sx,
                       sy, batch, ntn, ps);
  return hipGetLastError();
}

template <int MT>
hipError_t launch_mt(const cf* W, const cf* X, cf* Y, int nb, int na, int nre, long long ldx, long long sx,
                     long long sy, long long batch, long long ntn, const PilotScale& ps, dim3 grid, hipStream_t s) {
  const bool vec = ((ldx | sx | nre) & 1) == 0 && nre >= 2;
  return vec ? launch_mtv<MT, true>(W, X, Y, nb, na, nre, ldx, sx, sy, batch, ntn, ps, grid, s)
             : launch_mtv<MT, false>(W, X, Y, nb, na, nre, ldx, sx, sy, batch, ntn, ps, grid, s);
}

}  // namespace

int bf_cell_class(int n_beams, int n_ant) {
  if (n_beams < 1 || n_beams > 64 || n_ant < 1 || n_ant > 64) return -1;
  const int mt = (n_beams + 15) / 16, ks = n_ant <= 16 ? 0 : (n_ant <= 32 ? 1 : 2);
  return (mt - 1) * 3 + ks;
}

hipError_t launch_beamform_cells(BfCells& t, int cls, bool h16, int n_cu, hipStream_t s) {
  if (t.n < 1 || t.n > kBfCellsPerLaunch || cls < -1 || cls >= 12) return hipErrorInvalidValue;
  for (int c = 0; c < t.n; ++c) {
    BfCell& e = t.cell[c];
    e.cls = bf_cell_class(e.nb, e.na);
    if (e.cls < 0 || (cls >= 0 && e.cls != cls) || e.nre <= 0 || e.batch <= 0) return hipErrorInvalidValue;
    if (e.ldx * e.na >= (1ll << 28) || e.batch * ((e.nre + 15) / 16) >= (1ll << 30)) return hipErrorInvalidValue;
    e.ntn = (e.nre + 15) / 16;
    e.ntiles = (int)(e.batch * e.ntn);
  }
  if (cls < 0) return launch_any_cells(t, h16, n_cu, s);
  switch (cls / 3) {
    case 0: return launch_cells_mt<1>(t, cls % 3, h16, n_cu, s);
    case 1: return launch_cells_mt<2>(t, cls % 3, h16, n_cu, s);
    case 2: return launch_cells_mt<3>(t, cls % 3, h16, n_cu, s);
    default: return launch_cells_mt<4>(t, cls % 3, h16, n_cu, s);
  }
}

hipError_t launch_beamform(const cf* W, const cf* X, cf* Y, int n_beams, int n_ant, int n_re, long long ldx,
                           long long sx, long long sy, long long batch, int n_cu, hipStream_t s,
                           const PilotScale* pilot_scale, const unsigned* Xh, const signed char* ex) {
  if (batch <= 0 || n_re <= 0) return hipSuccess;
  PilotScale ps{};
  if (pilot_scale) ps = *pilot_scale;
  // 32-bit lane offsets and tile indices (with room for the prefetch index)
  if (n_ant <= 64 && ldx * n_ant < (1ll << 28) && batch * ((n_re + 15) / 16) < (1ll << 30)) {
    switch ((n_beams + 15) / 16) {
      case 1: return launch_k_mt<1>(W, X, Xh, ex, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ps, n_cu, s);
      case 2: return launch_k_mt<2>(W, X, Xh, ex, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ps, n_cu, s);
      case 3: return launch_k_mt<3>(W, X, Xh, ex, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ps, n_cu, s);
      case 4: return launch_k_mt<4>(W, X, Xh, ex, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ps, n_cu, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (Xh) return hipErrorInvalidValue;  // FP16 input: register-tile kernel only (up to 64 antennas)
  const long long ntn = (n_re + kTileN - 1) / kTileN;
  const long long tiles = batch * ntn;
  long long blocks = (tiles + kWaves - 1) / kWaves;
  const long long cap = (long long)n_cu * 8;
  if (blocks > cap) blocks = cap;
  const dim3 grid((unsigned)blocks);
  switch ((n_beams + 15) / 16) {
    case 1: return launch_mt<1>(W, X, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ntn, ps, grid, s);
    case 2: return launch_mt<2>(W, X, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ntn, ps, grid, s);
    case 3: return launch_mt<3>(W, X, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ntn, ps, grid, s);
    case 4: return launch_mt<4>(W, X, Y, n_beams, n_ant, n_re, ldx, sx, sy, batch, ntn, ps, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pusch
