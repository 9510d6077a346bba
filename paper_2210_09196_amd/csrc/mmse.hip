// MMSE MIMO detection (Eq. 2) per subcarrier: G = H^H H + sigma^2 I,
// Cholesky G = L L^H in Crout order (column by column, Sec. V-C), then for
// every data symbol the matched filter b = H^H y, forward substitution
// L z = b and back substitution L^H x = z.  The factor is computed once per
// subcarrier and reused for every data symbol.
//
// The paper runs many independent small decompositions per core between
// barriers (Sec. VI).  Three gfx950 kernels:
//
// k_mmse_mfma (n_ue <= 16): one wavefront takes 4 subcarriers per pass.
//   Phase A runs the two dense products of each subcarrier -- the Gram
//   matrix H^H H and the matched filter H^H [y_1 .. y_D] -- as 16x16x4 FP32
//   MFMAs, each complex product taking three real ones (Gauss/Karatsuba); a
//   lane's single fragment of H feeds both operands of the Gram product.  Phase B does the
//   Crout factorisation with one lane per row of L (16 lanes per subcarrier,
//   row j broadcast by cross-lane shuffles).  Phase C runs both
//   substitutions with one lane per data symbol, reading L from LDS by
//   broadcast.  With FUSED the kernel interpolates H itself, from the LS
//   values that the beamforming epilogue leaves in the pilot symbols and a
//   table of interpolation taps (launch_comb_taps), so the fused slot never
//   writes or re-reads a channel estimate.
//
// k_mmse_rows (n_ue <= 32, and iterative refinement): two subcarriers per
//   wavefront.  The Gram matrix (three 16x16 blocks of its lower triangle)
//   and the matched filter run on 16x16x4 FP32 MFMAs as above, through LDS;
//   then lane i of a group of 32 holds row i of G and L for the Crout
//   factorisation and the substitutions (rows broadcast by lane permutes).
//   With refinement (asked for, or beyond 16 UEs with N_L > N_B / 2), one step
//   of iterative refinement: the residual H^H (y - H x0) - sigma^2 x0 from the
//   stored estimate and the data symbols, on FP32 MFMA, or in FP64 for a
//   subcarrier whose condition estimate exceeds 1e4 (||G||_F times a
//   Hutchinson estimate of ||G^-1||_F from +-1 probe vectors solved in the
//   spare right-hand-side slots), solved with the same factor.
//
// k_mmse_tv (time-varying channel, two pilot symbols, n_ue <= 16): every
//   data symbol d has its own estimate (1 - a_d) H_0 + a_d H_1 and its own
//   Gram matrix, formed from three Hermitian products per subcarrier; one
//   workgroup takes 4 subcarriers one at a time, its four lane groups four
//   data symbols at a time (details at the kernel).
#include <cmath>

#include "kernels.h"

namespace pusch {
namespace {

constexpr int kMaxD = 16;  // data symbols per kernel call (host splits larger requests)
// Subcarriers whose condition estimate exceeds this get their refinement
// residual in FP64.
constexpr float kFp64Cond = 1e4f;
constexpr int kProbes = 4;  // probe vectors of the condition estimate

// ---- shared by both detection kernels: MFMA operands and cross-lane moves

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kSPW = 4;              // subcarriers per wavefront pass
// P of one subcarrier in LDS: 16 UE rows of NDP data symbols (NDP = 12 or
// 16, the call's count rounded up), padded to an odd row length so the 4
// groups' broadcasts hit distinct banks.
template <int NDP>
constexpr int kRowP = NDP + 1;
template <int NDP>
constexpr int kMatP = 16 * kRowP<NDP> + 1;
constexpr int kTri = 16 * 17 / 2 + 1;  // packed lower triangle (row i at i(i+1)/2), odd stride
constexpr int kDinv = 17;
// staged solutions: rows of 16 cf, pair p of row (grp, d) at pair p ^ (d & 7)
// (spreads the 16-byte accesses of one instruction over the banks)
static_assert(kSPW * 12 * 16 <= kSPW * kMatP<12> && kSPW * 16 * 16 <= kSPW * kMatP<16>,
              "solution staging must fit in the P buffer");

__device__ __forceinline__ int tri(int i) { return (i * (i + 1)) >> 1; }

__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Value of v in lane j of this lane's row of 16 (DPP row_newbcast; j must
// fold to a constant after unrolling).
__device__ __forceinline__ float row_bcast(float v, int j) {
  int x = __float_as_int(v), r;
  switch (j) {
    case 0: r = __builtin_amdgcn_update_dpp(0, x, 0x150, 0xF, 0xF, true); break;
    case 1: r = __builtin_amdgcn_update_dpp(0, x, 0x151, 0xF, 0xF, true); break;
    case 2: r = __builtin_amdgcn_update_dpp(0, x, 0x152, 0xF, 0xF, true); break;
    case 3: r = __builtin_amdgcn_update_dpp(0, x, 0x153, 0xF, 0xF, true); break;
    case 4: r = __builtin_amdgcn_update_dpp(0, x, 0x154, 0xF, 0xF, true); break;
    case 5: r = __builtin_amdgcn_update_dpp(0, x, 0x155, 0xF, 0xF, true); break;
    case 6: r = __builtin_amdgcn_update_dpp(0, x, 0x156, 0xF, 0xF, true); break;
    case 7: r = __builtin_amdgcn_update_dpp(0, x, 0x157, 0xF, 0xF, true); break;
    case 8: r = __builtin_amdgcn_update_dpp(0, x, 0x158, 0xF, 0xF, true); break;
    case 9: r = __builtin_amdgcn_update_dpp(0, x, 0x159, 0xF, 0xF, true); break;
    case 10: r = __builtin_amdgcn_update_dpp(0, x, 0x15A, 0xF, 0xF, true); break;
    case 11: r = __builtin_amdgcn_update_dpp(0, x, 0x15B, 0xF, 0xF, true); break;
    case 12: r = __builtin_amdgcn_update_dpp(0, x, 0x15C, 0xF, 0xF, true); break;
    case 13: r = __builtin_amdgcn_update_dpp(0, x, 0x15D, 0xF, 0xF, true); break;
    case 14: r = __builtin_amdgcn_update_dpp(0, x, 0x15E, 0xF, 0xF, true); break;
    default: r = __builtin_amdgcn_update_dpp(0, x, 0x15F, 0xF, 0xF, true); break;
  }
  return __int_as_float(r);
}

// Complex value of lane j of this lane's row of 16: one 64-bit DPP
// broadcast (v_mov_b64 with row_newbcast; j must fold to a constant).
__device__ __forceinline__ cf row_bcast_c(cf v, int j) {
  long long x = (long long)(unsigned)__float_as_int(v.r) | ((long long)__float_as_int(v.i) << 32), r;
  switch (j) {
    case 0: r = __builtin_amdgcn_update_dpp(x, x, 0x150, 0xF, 0xF, true); break;
    case 1: r = __builtin_amdgcn_update_dpp(x, x, 0x151, 0xF, 0xF, true); break;
    case 2: r = __builtin_amdgcn_update_dpp(x, x, 0x152, 0xF, 0xF, true); break;
    case 3: r = __builtin_amdgcn_update_dpp(x, x, 0x153, 0xF, 0xF, true); break;
    case 4: r = __builtin_amdgcn_update_dpp(x, x, 0x154, 0xF, 0xF, true); break;
    case 5: r = __builtin_amdgcn_update_dpp(x, x, 0x155, 0xF, 0xF, true); break;
    case 6: r = __builtin_amdgcn_update_dpp(x, x, 0x156, 0xF, 0xF, true); break;
    case 7: r = __builtin_amdgcn_update_dpp(x, x, 0x157, 0xF, 0xF, true); break;
    case 8: r = __builtin_amdgcn_update_dpp(x, x, 0x158, 0xF, 0xF, true); break;
    case 9: r = __builtin_amdgcn_update_dpp(x, x, 0x159, 0xF, 0xF, true); break;
    case 10: r = __builtin_amdgcn_update_dpp(x, x, 0x15A, 0xF, 0xF, true); break;
    case 11: r = __builtin_amdgcn_update_dpp(x, x, 0x15B, 0xF, 0xF, true); break;
    case 12: r = __builtin_amdgcn_update_dpp(x, x, 0x15C, 0xF, 0xF, true); break;
    case 13: r = __builtin_amdgcn_update_dpp(x, x, 0x15D, 0xF, 0xF, true); break;
    case 14: r = __builtin_amdgcn_update_dpp(x, x, 0x15E, 0xF, 0xF, true); break;
    default: r = __builtin_amdgcn_update_dpp(x, x, 0x15F, 0xF, 0xF, true); break;
  }
  return cf{__int_as_float((int)(r & 0xffffffffll)), __int_as_float((int)(r >> 32))};
}

// acc -= a * b and acc -= conj(a) * b, as explicit FMAs
__device__ __forceinline__ void csub_mul(cf& acc, cf a, cf b) {
  acc.r = __builtin_fmaf(-a.r, b.r, __builtin_fmaf(a.i, b.i, acc.r));
  acc.i = __builtin_fmaf(-a.r, b.i, __builtin_fmaf(-a.i, b.r, acc.i));
}
__device__ __forceinline__ void csub_conj_mul(cf& acc, cf a, cf b) {
  acc.r = __builtin_fmaf(-a.r, b.r, __builtin_fmaf(-a.i, b.i, acc.r));
  acc.i = __builtin_fmaf(-a.r, b.i, __builtin_fmaf(a.i, b.r, acc.i));
}

// Fragment slot s of the lane with A-column / B-row index q holds beam
// 8*(s/2) + 2*q + s%2: each lane owns pairs of adjacent beams (16-byte loads)
// and every K-step still sees four distinct beams.
__device__ __forceinline__ int frag_beam(int s, int q) { return 8 * (s >> 1) + 2 * q + (s & 1); }

// Beams b, b+1 of an RE-major row (zero beyond nb or when !ok).
__device__ __forceinline__ void load_pair(cf& v0, cf& v1, const cf* __restrict__ row, int b, int nb, bool ok,
                                          bool vec) {
  v0 = v1 = cf{0.f, 0.f};
  if (!ok) return;
  if (vec && b + 1 < nb) {
    const float4 t = *reinterpret_cast<const float4*>(row + b);
    v0 = cf{t.x, t.y};
    v1 = cf{t.z, t.w};
  } else {
    if (b < nb) v0 = row[b];
    if (b + 1 < nb) v1 = row[b + 1];
  }
}

// Beams b, b+1 of an RE-major row with an even number of beams, one 16-byte
// load; past the last beam the load reads beams 0, 1 instead (valid memory;
// the caller discards or zeroes what it gets there).
__device__ __forceinline__ float4 load_pair_even(const cf* __restrict__ row, int b, int nb) {
  return *reinterpret_cast<const float4*>(row + (b < nb ? b : 0));
}



// Value of v in the lane whose byte address (4 * lane) is src_byte.
__device__ __forceinline__ float lane_bcast(float v, int src_byte) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_byte, __float_as_int(v)));
}

// Element offset of data symbol d's grid: the d-th grid from d_first that
// is not one of the (ascending) skipped pilot grids.
__device__ __forceinline__ long long data_grid(const MmseGeom& g, int d) {
  int s = g.d_first + d;
#pragma unroll
  for (int j = 0; j < kMaxPilots; ++j)
    if (j < g.n_skip && g.skip[j] <= s) ++s;
  return (long long)s * g.y_sym;
}

struct LdsGeom {
  int gt;            // packed lower triangle of G per subcarrier (row i at i(i+1)/2), cf
  int poff, prow, pg;  // matched filter [grp][UE][symbol]: offset, row and subcarrier strides
  int lrow, lgrp;    // rows of L [grp][row][col] (reuse the G and P space once both are read)
  int xoff, xd, xg;  // refinement: first solution [grp][d][i] (offset, symbol and subcarrier strides)
  int eoff, ed, eg;  // refinement: residual of the data symbols [grp][d][b]
  int total;         // cf size of the whole LDS buffer
};

// L L^H v = v for every data symbol (v[d], lane i of the group holding
// component i): lane i holds row i of L in registers (L[m] = L_im) and
// 1/L_ii in invd; Lg holds the rows of the group's L (row stride lrow) for
// the transposed reads of the back substitution.
template <int LPS>
__device__ __forceinline__ void row_solve(cf (&v)[kMaxD], const cf (&L)[LPS], float invd, const cf* Lg, int lrow, int i,
                                          int gbase, int nue, int nd) {
  // forward substitution L z = v, column-oriented
#pragma unroll
  for (int m = 0; m < LPS; ++m) {
    if (m >= nue) continue;
#pragma unroll
    for (int d = 0; d < kMaxD; ++d) {
      if (d >= nd) continue;
      const float zr = lane_bcast(v[d].r * invd, (gbase + m) << 2);
      const float zi = lane_bcast(v[d].i * invd, (gbase + m) << 2);
      if (i == m) {
        v[d] = cf{zr, zi};
      } else if (i > m) {
        v[d].r -= L[m].r * zr - L[m].i * zi;
        v[d].i -= L[m].r * zi + L[m].i * zr;
      }
    }
  }
  // back substitution L^H x = z: x_m = (z_m - sum_{n>m} conj(L_nm) x_n) / L_mm
#pragma unroll
  for (int m = LPS - 1; m >= 0; --m) {
    if (m >= nue) continue;
    const cf lmi = Lg[m * lrow + i];
#pragma unroll
    for (int d = 0; d < kMaxD; ++d) {
      if (d >= nd) continue;
      const float xr = lane_bcast(v[d].r * invd, (gbase + m) << 2);
      const float xi = lane_bcast(v[d].i * invd, (gbase + m) << 2);
      if (i == m) {
        v[d] = cf{xr, xi};
      } else if (i < m) {
        v[d].r -= lmi.r * xr + lmi.i * xi;  // conj(L_mi) * x_m
        v[d].i -= lmi.r * xi - lmi.i * xr;
      }
    }
  }
}

// REFINE: after the first solve, one step of iterative refinement (a separate
// instance, so the plain path keeps its registers and LDS); the residual is
// FP32 on MFMA, or FP64 for a subcarrier whose condition estimate exceeds
// kFp64Cond.
template <int LPS, bool REFINE>
__global__ __launch_bounds__(64, 2) void k_mmse_rows(const cf* __restrict__ H, const cf* __restrict__ Y, cf* __restrict__ Xh,
                                             int* __restrict__ st, MmseGeom g, LdsGeom lg, long long nblk,
                                             int nblk_batch) {
  extern __shared__ cf sm[];
  constexpr int SPW = 64 / LPS;
  static_assert(LPS == 32, "two UE blocks of 16 per subcarrier");
  const int lane = threadIdx.x;
  const int grp = lane / LPS, i = lane % LPS, gbase = grp * LPS;
  const int q = lane >> 4, c16 = lane & 15;  // MFMA operand row / column inside a 16x16 block
  const int nb = g.n_beams, nue = g.n_ue, nsc = g.n_sc, nd = g.n_data;
  const bool vec = (nb & 1) == 0;
  const int ksteps = ((nb + 7) >> 3) << 1;  // k-steps of 4 beams, in pairs (a lane loads two adjacent beams)
  cf* Ls = sm;

  for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const long long bi = blk / nblk_batch;
    const int k0 = (int)(blk - bi * nblk_batch) * SPW;
    const int cnt = min(SPW, nsc - k0);
    const int k = k0 + grp;
    const bool valid = grp < cnt;

    // ---- Gram matrix and matched filter of each subcarrier on MFMA
    // (16x16x4 FP32, three real products per complex step as in the <= 16-UE
    // kernel): blocks G00, G10, G11 of the lower triangle (UE blocks of 16)
    // and P0, P1 (UE block x data symbol), then to LDS.
    __syncthreads();
    for (int sc = 0; sc < cnt; ++sc) {
      const cf* Hb = H + bi * g.h_batch + (long long)(k0 + sc) * nue * nb;
      const cf* hrow0 = Hb + (long long)(c16 < nue ? c16 : 0) * nb;
      const cf* hrow1 = Hb + (long long)(16 + c16 < nue ? 16 + c16 : 0) * nb;
      const cf* yrow = Y + bi * g.y_batch + data_grid(g, c16 < nd ? c16 : 0) + (long long)(k0 + sc) * nb;
      f32x4 acc[15];
#pragma unroll
      for (int t = 0; t < 15; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      // conj(a) b as T1 = ar br, T2 = ai bi, T3 = (ar - ai)(br + bi)
      auto prod = [&](int t, cf a, cf b) {
        acc[t] = mfma(a.r, b.r, acc[t]);
        acc[t + 1] = mfma(a.i, b.i, acc[t + 1]);
        acc[t + 2] = mfma(a.r - a.i, b.r + b.i, acc[t + 2]);
      };
      for (int s = 0; s < ksteps; s += 2) {
        cf h0[2], h1[2], y[2];
        load_pair(h0[0], h0[1], hrow0, frag_beam(s, q), nb, c16 < nue, vec);
        load_pair(h1[0], h1[1], hrow1, frag_beam(s, q), nb, 16 + c16 < nue, vec);
        load_pair(y[0], y[1], yrow, frag_beam(s, q), nb, c16 < nd, vec);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          prod(0, h0[u], h0[u]);   // G00
          prod(3, h1[u], h0[u]);   // G10
          prod(6, h1[u], h1[u]);   // G11
          prod(9, h0[u], y[u]);    // P0
          prod(12, h1[u], y[u]);   // P1
        }
      }
      // lane holds rows 4q..4q+3 of column c16 of every block
      cf* Gp = sm + sc * lg.gt;
      cf* Pp = sm + lg.poff + sc * lg.pg;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * q + v;
        auto val = [&](int t) {
          return cf{acc[t][v] + acc[t + 1][v], acc[t + 2][v] - acc[t][v] + acc[t + 1][v]};
        };
        if (c16 <= r) Gp[tri(r) + c16] = val(0);
        Gp[tri(16 + r) + c16] = val(3);
        if (c16 <= r) Gp[tri(16 + r) + 16 + c16] = val(6);
        Pp[r * lg.prow + c16] = val(9);
        Pp[(16 + r) * lg.prow + c16] = val(12);
      }
    }
    __syncthreads();

    // Gram row i (lower part; sigma^2 on the diagonal) and matched filter
    // outputs of this lane's subcarrier
    const float s2 = g.sigma2_item ? g.sigma2_item[bi] : g.sigma2;
    cf G[LPS];
    {
      const cf* Gr = sm + grp * lg.gt + tri(i);
#pragma unroll
      for (int j = 0; j < LPS; ++j) G[j] = j <= i ? Gr[j] : cf{0.f, 0.f};
    }
    float gii = 0.f;  // this row's regularised diagonal entry
#pragma unroll
    for (int j = 0; j < LPS; ++j)
      if (j == i) {
        G[j].r += s2;
        gii = G[j].r;
      }
    cf rr[kMaxD];
    {
      const cf* Pr = sm + lg.poff + grp * lg.pg + i * lg.prow;
#pragma unroll
      for (int d = 0; d < kMaxD; ++d) rr[d] = (d < nd && i < nue) ? Pr[d] : cf{0.f, 0.f};
    }
    // With refinement, the right-hand sides past the data symbols carry probe
    // vectors of +-1 entries (a fixed sign pattern per slot), so the same
    // substitutions give z = G^-1 v for the condition estimate below.
    const int nprobe = REFINE ? min(kProbes, kMaxD - nd) : 0;
#pragma unroll
    for (int d = 0; d < kMaxD; ++d)
      if (d >= nd && d < nd + nprobe && i < nue) rr[d] = cf{(((i * (2 * d + 3) + d) >> 1) & 1) ? -1.f : 1.f, 0.f};
    float gfro = 0.f;  // sum of |G_ij|^2 over this row's lower triangle
#pragma unroll
    for (int j = 0; j < LPS; ++j) gfro += G[j].r * G[j].r + G[j].i * G[j].i;

    // Cholesky-Crout: column j uses row j of L (lane j of the group)
    int fail = 0;
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
        const float cr = lane_bcast(L[m].r, (gbase + j) << 2);
        const float ci = lane_bcast(L[m].i, (gbase + j) << 2);
        t.r -= L[m].r * cr + L[m].i * ci;  // L_im * conj(L_jm)
        t.i -= L[m].i * cr - L[m].r * ci;
      }
      const float dpiv = lane_bcast(t.r, (gbase + j) << 2);
      fail |= (dpiv > 0.f && dpiv <= 3.402823466e38f) ? 0 : 1;
      const float ljj = sqrtf(dpiv);
      const float inv = 1.0f / ljj;
      const cf lij = cf{t.r * inv, t.i * inv};
      L[j] = i == j ? cf{ljj, 0.f} : (i > j ? lij : cf{0.f, 0.f});
      invd = i == j ? inv : invd;
    }

    // rows of L to LDS (reusing the G and P space) for the transposed reads
    // of the back substitution
    __syncthreads();
#pragma unroll
    for (int m = 0; m < LPS; ++m) Ls[grp * lg.lgrp + i * lg.lrow + m] = L[m];
    __syncthreads();

    row_solve<LPS>(rr, L, invd, Ls + grp * lg.lgrp, lg.lrow, i, gbase, nue, nd + nprobe);

    if constexpr (REFINE) {
      // Condition estimate of each subcarrier's G: ||G||_F ||G^-1||_F, with
      // ||G^-1||_F^2 the mean of |G^-1 v|^2 over the probes (E[v v^H] = I for
      // independent +-1 entries); ||G||_F^2 from the lower triangles.  It is
      // at least the 2-norm condition number up to the probes' sampling error.
      // Without a spare right-hand side (16 data symbols): max_i G_ii /
      // min_i L_ii^2, a lower bound.
      float zsq = 0.f;
#pragma unroll
      for (int d = 0; d < kMaxD; ++d)
        if (d >= nd && d < nd + nprobe) zsq += rr[d].r * rr[d].r + rr[d].i * rr[d].i;
      float fro = (i < nue) ? 2.f * gfro - gii * gii : 0.f;  // off-diagonal entries count twice
      float gmax = (i < nue) ? gii : 0.f, dmax = (i < nue) ? invd : 0.f;  // invd = 1 / L_ii
#pragma unroll
      for (int o = 16; o >= 1; o >>= 1) {
        zsq += __shfl_xor(zsq, o);
        fro += __shfl_xor(fro, o);
        gmax = fmaxf(gmax, __shfl_xor(gmax, o));
        dmax = fmaxf(dmax, __shfl_xor(dmax, o));
      }
      const float kap_own = nprobe > 0 ? sqrtf(fro * zsq / (float)nprobe) : gmax * dmax * dmax;
      float kap[SPW];
#pragma unroll
      for (int sc = 0; sc < SPW; ++sc) kap[sc] = __shfl(kap_own, sc * LPS);
      // One step of iterative refinement.  The residual of the normal
      // equations, r = H^H (y - H x0) - sigma^2 x0, is formed from the stored
      // estimate and the data symbols themselves (not from the rounded G);
      // L L^H dx = r with the same factor; x1 = x0 + dx.  Both products run
      // on MFMA per subcarrier: e = y - H x0 (beam blocks of 16 x the data
      // symbols, UEs as K) and H^H e (as the matched filter, e for y).
      __syncthreads();
      {
        cf* Xg = sm + lg.xoff + grp * lg.xg;
#pragma unroll
        for (int d = 0; d < kMaxD; ++d)
          if (d < nd) Xg[d * lg.xd + i] = (i < nue) ? rr[d] : cf{0.f, 0.f};
      }
      __syncthreads();
      for (int sc = 0; sc < cnt; ++sc) {
        cf* Xsc = sm + lg.xoff + sc * lg.xg;  // x0 [d][UE]; then H^H e in its place
        cf* Esc = sm + lg.eoff + sc * lg.eg;  // e [d][beam]
        const cf* Hb = H + bi * g.h_batch + (long long)(k0 + sc) * nue * nb;
        if (kap[sc] > kFp64Cond) {
          // Ill-conditioned: the whole residual r = H^H (y - H x0) - sigma^2 x0 in
          // FP64 (products of FP32 values are exact there), rounded once to FP32
          // into x0's place.  e [d][beam] in FP64 spans the E region of both
          // subcarriers (used one subcarrier at a time).
          double* E = reinterpret_cast<double*>(sm + lg.eoff);
          const cf* yb = Y + bi * g.y_batch + (long long)(k0 + sc) * nb;
          for (int t = lane; t < nd * nb; t += 64) {
            const int d = t / nb, b = t - d * nb;
            const cf y = yb[data_grid(g, d) + b];
            double er = y.r, ei = y.i;
            for (int l = 0; l < nue; ++l) {
              const cf h = Hb[(long long)l * nb + b], x = Xsc[d * lg.xd + l];
              er -= (double)h.r * x.r - (double)h.i * x.i;
              ei -= (double)h.r * x.i + (double)h.i * x.r;
            }
            E[2 * t] = er;
            E[2 * t + 1] = ei;
          }
          __syncthreads();
          // r[d][l]: each entry reads only its own x0[d][l] (and E), so it can
          // replace it at once
          for (int t = lane; t < nd * nue; t += 64) {
            const int d = t / nue, l = t - d * nue;
            const cf x = Xsc[d * lg.xd + l];
            double ar = -(double)s2 * x.r, ai = -(double)s2 * x.i;
            for (int b = 0; b < nb; ++b) {
              const cf h = Hb[(long long)l * nb + b];
              const double er = E[2 * (d * nb + b)], ei = E[2 * (d * nb + b) + 1];
              ar += (double)h.r * er + (double)h.i * ei;  // conj(h) e
              ai += (double)h.r * ei - (double)h.i * er;
            }
            Xsc[d * lg.xd + l] = cf{(float)ar, (float)ai};
          }
          __syncthreads();
          continue;
        }
        const cf* ysrc = Y + bi * g.y_batch + data_grid(g, c16 < nd ? c16 : 0) + (long long)(k0 + sc) * nb;
        // e = y - H x0: A[m][k] = H[beam 16 bb + m][UE k], B[k][n] = x0[UE k][symbol n];
        // a b as T1 = ar br, T2 = ai bi, T3 = (ar + ai)(br + bi)
        for (int bb = 0; bb * 16 < nb; ++bb) {
          f32x4 t1 = {0.f, 0.f, 0.f, 0.f}, t2 = t1, t3 = t1;
          const int beam = 16 * bb + c16;
          for (int s = 0; s < LPS / 4; ++s) {
            const int ue = 4 * s + q;
            const cf a = (ue < nue && beam < nb) ? Hb[(long long)ue * nb + beam] : cf{0.f, 0.f};
            const cf x = Xsc[c16 * lg.xd + ue];
            t1 = mfma(a.r, x.r, t1);
            t2 = mfma(a.i, x.i, t2);
            t3 = mfma(a.r + a.i, x.r + x.i, t3);
          }
          // lane holds rows (beams) 16 bb + 4q + v of column (symbol) c16
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int b = 16 * bb + 4 * q + v;
            if (b < nb && c16 < nd) {
              const cf y = ysrc[b];
              Esc[c16 * lg.ed + b] = cf{y.r - (t1[v] - t2[v]), y.i - (t3[v] - t1[v] - t2[v])};
            }
          }
        }
        __syncthreads();
        // H^H e: the matched filter's products with e from LDS
        f32x4 acc[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        auto prod = [&](int t, cf a, cf b) {
          acc[t] = mfma(a.r, b.r, acc[t]);
          acc[t + 1] = mfma(a.i, b.i, acc[t + 1]);
          acc[t + 2] = mfma(a.r - a.i, b.r + b.i, acc[t + 2]);
        };
        const cf* hrow0 = Hb + (long long)(c16 < nue ? c16 : 0) * nb;
        const cf* hrow1 = Hb + (long long)(16 + c16 < nue ? 16 + c16 : 0) * nb;
        for (int s = 0; s < ksteps; s += 2) {
          cf h0[2], h1[2], e[2];
          const int fb = frag_beam(s, q);
          load_pair(h0[0], h0[1], hrow0, fb, nb, c16 < nue, vec);
          load_pair(h1[0], h1[1], hrow1, fb, nb, 16 + c16 < nue, vec);
          e[0] = (c16 < nd && fb < nb) ? Esc[c16 * lg.ed + fb] : cf{0.f, 0.f};
          e[1] = (c16 < nd && fb + 1 < nb) ? Esc[c16 * lg.ed + fb + 1] : cf{0.f, 0.f};
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            prod(0, h0[u], e[u]);
            prod(3, h1[u], e[u]);
          }
        }
        __syncthreads();  // H^H e goes into x0's space (read above)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 4 * q + v;
          if (c16 < nd) {
            Xsc[c16 * lg.xd + r] = cf{acc[0][v] + acc[1][v], acc[2][v] - acc[0][v] + acc[1][v]};
            Xsc[c16 * lg.xd + 16 + r] = cf{acc[3][v] + acc[4][v], acc[5][v] - acc[3][v] + acc[4][v]};
          }
        }
      }
      __syncthreads();
      // r_i = (H^H e)_i - sigma^2 x0_i (x0 is still in rr); an FP64 subcarrier's
      // slot already holds the whole residual
      cf r[kMaxD];
      {
        const cf* Rg = sm + lg.xoff + grp * lg.xg;
        const float s2r = kap_own > kFp64Cond ? 0.f : s2;
#pragma unroll
        for (int d = 0; d < kMaxD; ++d) {
          const cf he = (d < nd && i < nue) ? Rg[d * lg.xd + i] : cf{0.f, 0.f};
          r[d] = cf{he.r - s2r * rr[d].r, he.i - s2r * rr[d].i};
        }
      }
      row_solve<LPS>(r, L, invd, Ls + grp * lg.lgrp, lg.lrow, i, gbase, nue, nd);
#pragma unroll
      for (int d = 0; d < kMaxD; ++d) rr[d] = cf{rr[d].r + r[d].r, rr[d].i + r[d].i};
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

LdsGeom lds_geom(int lps, int nb, bool refine) {
  const int spw = 64 / lps;
  LdsGeom lg;
  lg.gt = lps * (lps + 1) / 2 + 1;
  lg.prow = kMaxD + 1;
  lg.pg = lps * lg.prow + 1;
  lg.poff = spw * lg.gt;
  lg.lrow = lps + 1;
  lg.lgrp = lps * lg.lrow + 1;
  const int gp = lg.poff + spw * lg.pg, l = spw * lg.lgrp;
  lg.total = gp > l ? gp : l;
  lg.xd = lps + 1;
  lg.xg = kMaxD * lg.xd + 1;
  lg.ed = nb | 1;
  lg.eg = kMaxD * lg.ed + 1;
  lg.xoff = lg.eoff = 0;
  if (refine) {
    lg.xoff = lg.total;
    lg.eoff = lg.xoff + spw * lg.xg;
    lg.total = lg.eoff + spw * lg.eg;
  }
  return lg;
}

template <int LPS>
hipError_t launch_lps(const cf* H, const cf* Y, cf* Xh, int* st, const MmseGeom& g, long long batch, hipStream_t s) {
  constexpr int SPW = 64 / LPS;
  const LdsGeom lg = lds_geom(LPS, g.n_beams, g.refine != 0);
  const int nblk_batch = (g.n_sc + SPW - 1) / SPW;
  const long long nblk = batch * nblk_batch;
  if (nblk <= 0) return hipSuccess;
  long long blocks = nblk;
  if (blocks > (1LL << 30)) blocks = 1LL << 30;
  if (g.refine)
    hipLaunchKernelGGL((k_mmse_rows<LPS, true>), dim3((unsigned)blocks), dim3(64), (size_t)lg.total * sizeof(cf), s, H,
                       Y, Xh, st, g, lg, nblk, nblk_batch);
  else
    hipLaunchKernelGGL((k_mmse_rows<LPS, false>), dim3((unsigned)blocks), dim3(64), (size_t)lg.total * sizeof(cf), s,
                       H, Y, Xh, st, g, lg, nblk, nblk_batch);
  return hipGetLastError();
}

}  // namespace


// ---------------------------------------------------------------- MFMA path (n_ue <= 16)
namespace {

// FUSED: NT interpolation taps per (subcarrier, UE), 0 when H is read.
// LDS of a workgroup: the lower triangles of G (then of L in place), the
// matched filters P[i][d] = (H^H y_d)_i (then the staged solutions; 16-byte
// aligned) and the reciprocal diagonals of L.
template <int NDP>
struct MfmaLds {
  cf G[kSPW * kTri];
  cf P[kSPW * kMatP<NDP>];
  float Dinv[kSPW * kDinv];
};

// Crout factorisation of a 16 x 16 block per group of 16 lanes (Sec. V-C):
// on entry lane i holds row i of the regularised Gram matrix in L[0..i]
// (zeros beyond); rows and columns from nue on must be the identity.  On exit
// L[j] = L_ij for j < i and L[i] = L_ii (the lane keeps t / L_jj in the
// columns above its diagonal, which are never read), 1 / L_jj goes to
// dinv[j] (LDS, if given) and the lane's own 1 / L_ii to dvi.  Row j of L
// reaches every lane of the group by a DPP row broadcast.  Returns 1 when a
// pivot is not positive and finite (the same value in all 16 lanes).
__device__ __forceinline__ int crout_rows(cf (&L)[16], const int i, const int nue, float* __restrict__ dinv,
                                          float& dvi) {
  int fail = 0;
  dvi = 1.f;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    // padded rows / columns beyond n_ue stay the identity: G is zero off
    // the diagonal there (zero rows of H) and 1 on it, so is L, and the
    // substitutions never read that part (a uniform branch)
    if (j < nue) {
      // t = G_ij - sum_m L_im conj(L_jm), row j's entries broadcast
      float tr = L[j].r, ti = L[j].i;
#pragma unroll
      for (int m = 0; m < j; ++m) {
        const cf c = row_bcast_c(L[m], j);
        tr = __builtin_fmaf(-c.r, L[m].r, tr);
        tr = __builtin_fmaf(-c.i, L[m].i, tr);
        ti = __builtin_fmaf(-c.r, L[m].i, ti);
        ti = __builtin_fmaf(c.i, L[m].r, ti);
      }
      const cf t = cf{tr, ti};
      const float dpiv = row_bcast(t.r, j);
      fail |= (dpiv > 0.f && dpiv <= 3.402823466e38f) ? 0 : 1;
      const float inv = rsqrtf(dpiv);  // 1 / L_jj
      L[j] = cf{t.r * inv, t.i * inv};
      if (dinv) dinv[j] = inv;
      if (j == i) dvi = inv;
    }
  }
  return fail;
}

// Phases B and C of one block (G and P of its kSPW subcarriers in LDS):
// Crout factorisation, then the substitutions and the stores of x_hat and
// the status flags.
template <int NDP>
__device__ __forceinline__ void mmse_factor_solve(MfmaLds<NDP>& lds, const int bi, const int k0, cf* __restrict__ Xh,
                                                  int* __restrict__ st, const MmseGeom& g) {
  cf* __restrict__ Gs = lds.G;
  cf* __restrict__ Ps = lds.P;
  float* __restrict__ Dinv = lds.Dinv;
  const int lane = threadIdx.x;
  const int c16 = lane & 15, q = lane >> 4;
  const int nue = g.n_ue, nsc = g.n_sc, nd = g.n_data;
  {
    // ---- phase B: Crout factorisation, lane (q, c16) holds row c16 of
    // subcarrier q; the 16 lanes of a subcarrier are one DPP row, so row j of
    // L reaches every lane by a row broadcast
    const int grp = q, i = c16;
    cf* Gm = Gs + grp * kTri;
    cf* Grow = Gm + tri(i);
    // regularise the own diagonal entry (padding rows beyond n_ue get 1 so
    // their part of L is the identity; so do the rows of a subcarrier past n_sc)
    const float s2 = g.sigma2_item ? g.sigma2_item[bi] : g.sigma2;
    Grow[i].r += (i < nue && k0 + grp < nsc) ? s2 : 1.0f;
    cf L[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) L[j] = j <= i ? Grow[j] : cf{0.f, 0.f};
    float dvi;
    const int fail = crout_rows(L, i, nue, Dinv + grp * kDinv, dvi);
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (j <= i) Grow[j] = L[j];
    __syncthreads();

    // ---- phase C: forward and back substitution, lane (q, c16) solves data symbol c16
    const int d = c16;
    const float* dv = Dinv + grp * kDinv;
    cf z[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = Ps[grp * kMatP<NDP> + r * kRowP<NDP> + (d < NDP ? d : NDP - 1)];
#pragma unroll
    for (int r = 0; r < 16; ++r) {  // L z = b, row by row
      if (r >= nue) continue;
#pragma unroll
      for (int m = 0; m < r; ++m) csub_mul(z[r], Gm[tri(r) + m], z[m]);
      const float s = dv[r];
      z[r] = cf{z[r].r * s, z[r].i * s};
    }
#pragma unroll
    for (int m = 15; m >= 0; --m) {  // L^H x = z, column by column: x_m is final, remove it from rows r < m
      if (m >= nue) continue;
      const float s = dv[m];
      z[m] = cf{z[m].r * s, z[m].i * s};
#pragma unroll
      for (int r = 0; r < m; ++r) csub_conj_mul(z[r], Gm[tri(m) + r], z[m]);  // z_r -= conj(L_mr) x_m
    }
    const int k = k0 + grp;
    if (nue == 16 && k0 + kSPW <= nsc) {
      // x_hat[d][k0 .. k0+3][0..15] is one contiguous 512-byte run per data
      // symbol: stage the solutions in LDS (P is consumed) and write each run
      // with 16-byte stores, consecutive lanes on consecutive bytes.
      cf* Xs = Ps;  // [grp][d] rows of 16 (swizzled pairs)
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; r += 2)
        if (d < NDP)
          *reinterpret_cast<float4*>(Xs + (grp * NDP + d) * 16 + 2 * ((r >> 1) ^ (d & 7))) =
              fail ? float4{0.f, 0.f, 0.f, 0.f} : float4{z[r].r, z[r].i, z[r + 1].r, z[r + 1].i};
      __syncthreads();
      cf* xb = Xh + bi * g.x_batch + (long long)k0 * 16;
#pragma unroll
      for (int it = 0; it < NDP * kSPW * 16 / 2 / 64; ++it) {
        const int c = it * 64 + lane;  // 16-byte chunk: data symbol, subcarrier, UE pair
        const int dd = c >> 5, gg = (c >> 3) & 3, rp = c & 7;
        if (dd < nd)
          *reinterpret_cast<float4*>(xb + (long long)dd * nsc * 16 + gg * 16 + 2 * rp) =
              *reinterpret_cast<const float4*>(Xs + (gg * NDP + dd) * 16 + 2 * (rp ^ (dd & 7)));
      }
    } else if (k < nsc && d < nd) {
      cf* dst = Xh + bi * g.x_batch + ((long long)d * nsc + k) * nue;
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (r < nue) dst[r] = fail ? cf{0.f, 0.f} : z[r];
    }
    if (k < nsc && d == 0 && st) {
      int* sp = st + bi * g.st_batch + k;
      *sp = g.st_or ? (*sp | fail) : fail;
    }
  }
}

// Phase A accumulators of one subcarrier: the Gram matrix and the matched
// filter, each as three real products (Gauss/Karatsuba): with T1 = ar br,
// T2 = ai bi, T3 = (ar - ai)(br + bi), conj(a) b = (T1 + T2) + i (T3 - T1 + T2).
struct GpAcc {
  f32x4 g1, g2, g3, p1, p2, p3;
};

// One K-step (4 beams): 6 MFMAs.  The lane's fragment of H is both the A row
// (UE c16) and the B column (UE c16) of the Gram product.
__device__ __forceinline__ void gp_kstep(GpAcc& c, cf h, cf y) {
  const float hm = h.r - h.i, hp = h.r + h.i, ys = y.r + y.i;
  c.g1 = mfma(h.r, h.r, c.g1);
  c.g2 = mfma(h.i, h.i, c.g2);
  c.g3 = mfma(hm, hp, c.g3);
  c.p1 = mfma(h.r, y.r, c.p1);
  c.p2 = mfma(h.i, y.i, c.p2);
  c.p3 = mfma(hm, ys, c.p3);
}

// Subcarrier sc's G (lower triangle) and P to LDS: the lane holds rows
// 4q..4q+3 of column c16.
template <int NDP>
__device__ __forceinline__ void gp_store(MfmaLds<NDP>& lds, int sc, const GpAcc& c, int q, int c16) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * q + v;
    const float g12 = c.g1[v] + c.g2[v], p12 = c.p1[v] + c.p2[v];
    if (i >= c16) lds.G[sc * kTri + tri(i) + c16] = cf{g12, c.g3[v] - c.g1[v] + c.g2[v]};
    if (c16 < kRowP<NDP>) lds.P[sc * kMatP<NDP> + i * kRowP<NDP> + c16] = cf{p12, c.p3[v] - c.p1[v] + c.p2[v]};
  }
}

// blk: the workgroup's logical block (kSPW subcarriers of one batch item).
template <int KS, bool FUSED, int NT, int NDP>
__device__ __forceinline__ void mmse_mfma_body(MfmaLds<NDP>& lds, const int blk, const cf* __restrict__ H,
                                               const cf* __restrict__ Y, const int2* __restrict__ taps,
                                               cf* __restrict__ Xh, int* __restrict__ st, const MmseGeom& g,
                                               const ChestGeom& cg, int nblk_batch) {
  const int lane = threadIdx.x;
  const int c16 = lane & 15, q = lane >> 4;
  const int nb = g.n_beams, nue = g.n_ue, nsc = g.n_sc, nd = g.n_data;
  const bool vec = (nb & 1) == 0;
  // offset of this lane's data symbol (B operand of the matched filter)
  const long long ysym = data_grid(g, c16 < nd ? c16 : 0);

  {
    // one workgroup = one block of kSPW subcarriers (no enclosing loop, so no
    // lane predicates are hoisted and kept alive across blocks)
    const int bi = blk / nblk_batch;
    const int k0 = (blk - bi * nblk_batch) * kSPW;

    // ---- phase A: Gram and matched filter of each subcarrier on MFMA
    // 8 MFMAs of one K-step: G += h^H h, P += h^H y (complex as real parts)
    // 6 MFMAs of one K-step.  Both products take three real products
    // (Gauss/Karatsuba): with T1 = ar br, T2 = ai bi, T3 = (ar - ai)(br + bi),
    // conj(a) b = (T1 + T2) + i (T3 - T1 + T2).  The lane's fragment of H is
    // both the A row (UE c16) and the B column (UE c16) of the Gram product.
    using Acc = GpAcc;
    auto kstep = [](Acc& c, cf h, cf y) { gp_kstep(c, h, y); };
    auto store_gp = [&](int sc, const Acc& c) { gp_store(lds, sc, c, q, c16); };
    const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
    // Two taps and up to 8 K-steps (the common fused case): all kSPW
    // subcarriers unrolled, the loads of subcarrier sc + 1 in flight during
    // the MFMAs of sc (double-buffered registers).
    constexpr bool PIPE = FUSED && NT == 2 && KS <= 8;
    if constexpr (PIPE) {
      const int ue = c16 < nue ? c16 : 0;  // lanes past n_ue: UE 0's taps, result discarded
      int4 tq[kSPW];
#pragma unroll
      for (int sc = 0; sc < kSPW; ++sc) {
        const int kk = k0 + sc < nsc ? k0 + sc : nsc - 1;
        tq[sc] = reinterpret_cast<const int4*>(taps)[(long long)kk * nue + ue];
      }
      const cf* LSb = Y + bi * cg.y_batch;
      float4 lv[2][KS / 2][2], yv[2][KS / 2];
      auto issue = [&](int sc, int buf) {
        const int kk = k0 + sc < nsc ? k0 + sc : nsc - 1;
        const cf* yrow = Y + bi * g.y_batch + ysym + (long long)kk * nb;
#pragma unroll
        for (int u = 0; u < KS / 2; ++u) {
          const int b = frag_beam(2 * u, q);
          lv[buf][u][0] = load_pair_even(LSb + tq[sc].x, b, nb);
          lv[buf][u][1] = load_pair_even(LSb + tq[sc].z, b, nb);
          yv[buf][u] = load_pair_even(yrow, b, nb);
        }
      };
      issue(0, 0);
#pragma unroll
      for (int sc = 0; sc < kSPW; ++sc) {
        const int buf = sc & 1;
        if (sc + 1 < kSPW) issue(sc + 1, buf ^ 1);
        __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of this subcarrier's arithmetic
        Acc ac{z4, z4, z4, z4, z4, z4};
        const float w0 = __int_as_float(tq[sc].y), w1 = __int_as_float(tq[sc].w);
        const bool live = c16 < nue && k0 + sc < nsc;  // else zero rows of H (G = 0, P = 0)
#pragma unroll
        for (int u = 0; u < KS / 2; ++u) {
          const int b = frag_beam(2 * u, q);
          const float4 l0 = lv[buf][u][0], l1 = lv[buf][u][1], yy = yv[buf][u];
          const bool keep = live && b < nb;
          const float4 a = {__builtin_fmaf(w1, l1.x, w0 * l0.x), __builtin_fmaf(w1, l1.y, w0 * l0.y),
                            __builtin_fmaf(w1, l1.z, w0 * l0.z), __builtin_fmaf(w1, l1.w, w0 * l0.w)};
          kstep(ac, cf{keep ? a.x : 0.f, keep ? a.y : 0.f}, cf{yy.x, yy.y});
          kstep(ac, cf{keep ? a.z : 0.f, keep ? a.w : 0.f}, cf{yy.z, yy.w});
        }
        store_gp(sc, ac);
      }
    }
    // fused: this lane's taps (UE c16; lanes past n_ue read UE 0's and
    // discard the result), prefetched one subcarrier ahead
    constexpr int NQ = NT > 0 ? NT / 2 : 1;
    int4 tnext[NQ];
    auto load_taps = [&](int kk) {
      kk = kk < nsc ? kk : nsc - 1;
      const int4* tp = reinterpret_cast<const int4*>(taps + ((long long)kk * nue + (c16 < nue ? c16 : 0)) * NT);
#pragma unroll
      for (int u = 0; u < NQ; ++u) tnext[u] = tp[u];
    };
    if constexpr (FUSED && !PIPE) load_taps(k0);
#pragma unroll 1
    for (int sc = 0; sc < (PIPE ? 0 : kSPW); ++sc) {
      const int k = k0 + sc;
      Acc ac{z4, z4, z4, z4, z4, z4};
      if constexpr (FUSED) {
        int off[NT];
        float w[NT];
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
          off[2 * u] = tnext[u].x;
          w[2 * u] = __int_as_float(tnext[u].y);
          off[2 * u + 1] = tnext[u].z;
          w[2 * u + 1] = __int_as_float(tnext[u].w);
        }
        if (sc + 1 < kSPW) load_taps(k + 1);
        if (k < nsc) {
          // H interpolated from the LS values the beamforming epilogue left in
          // the pilot symbols.  The loads of CH beam pairs go out together
          // (one wait), then their arithmetic.  Even n_beams: one 16-byte load
          // per pair; y columns of lanes past n_data only feed columns of P
          // that are never read, beams past n_beams meet zero columns of H.
          const cf* LSb = Y + bi * cg.y_batch;
          const cf* yrow = Y + bi * g.y_batch + ysym + (long long)k * nb;
          constexpr int CH = NT <= 2 ? 4 : (NT <= 4 ? 2 : 1);
#pragma unroll
          for (int c0 = 0; c0 < KS / 2; c0 += CH) {
            float4 lv[CH][NT], yv[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
              if (c0 + u >= KS / 2) continue;
              const int b = frag_beam(2 * (c0 + u), q);
#pragma unroll
              for (int t = 0; t < NT; ++t) lv[u][t] = load_pair_even(LSb + off[t], b, nb);
              yv[u] = load_pair_even(yrow, b, nb);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < CH; ++u) {
              if (c0 + u >= KS / 2) continue;
              const int b = frag_beam(2 * (c0 + u), q);
              float4 a = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
              for (int t = 0; t < NT; ++t) {
                a.x = __builtin_fmaf(w[t], lv[u][t].x, a.x);
                a.y = __builtin_fmaf(w[t], lv[u][t].y, a.y);
                a.z = __builtin_fmaf(w[t], lv[u][t].z, a.z);
                a.w = __builtin_fmaf(w[t], lv[u][t].w, a.w);
              }
              const bool keep = c16 < nue && b < nb;  // zero rows / columns of H
              kstep(ac, cf{keep ? a.x : 0.f, keep ? a.y : 0.f}, cf{yv[u].x, yv[u].y});
              kstep(ac, cf{keep ? a.z : 0.f, keep ? a.w : 0.f}, cf{yv[u].z, yv[u].w});
            }
          }
        }
      } else if (k < nsc) {
        cf h[KS], y[KS];
        const cf* hrow = H + bi * g.h_batch + ((long long)k * nue + (c16 < nue ? c16 : 0)) * nb;
#pragma unroll
        for (int s = 0; s < KS; s += 2) load_pair(h[s], h[s + 1], hrow, frag_beam(s, q), nb, c16 < nue, vec);
        const cf* yrow = Y + bi * g.y_batch + ysym + (long long)k * nb;
#pragma unroll
        for (int s = 0; s < KS; s += 2) load_pair(y[s], y[s + 1], yrow, frag_beam(s, q), nb, c16 < nd, vec);
#pragma unroll
        for (int s = 0; s < KS; ++s) kstep(ac, h[s], y[s]);
      }
      store_gp(sc, ac);
    }
    __syncthreads();
    mmse_factor_solve(lds, bi, k0, Xh, st, g);
  }
}

template <int KS, bool FUSED, int NT, int NDP>
__global__ __launch_bounds__(64) void k_mmse_mfma(const cf* __restrict__ H, const cf* __restrict__ Y,
                                                  const int2* __restrict__ taps, cf* __restrict__ Xh,
                                                  int* __restrict__ st, MmseGeom g, ChestGeom cg, int nblk_batch) {
  __shared__ __align__(16) MfmaLds<NDP> lds;
  // neighbouring subcarriers on one XCD (shared pilot rows)
  mmse_mfma_body<KS, FUSED, NT, NDP>(lds, xcd_block(blockIdx.x, gridDim.x), H, Y, taps, Xh, st, g, cg, nblk_batch);
}

// Many cells in one launch: logical block b (after the XCD renumbering, so a
// cell's neighbouring subcarriers still share an L2) belongs to the cell c
// with start[c] <= b < start[c + 1].
template <int KS, int NT>
__global__ __launch_bounds__(64) void k_mmse_mfma_cells(MmseCells t) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  int c = 0;
  while (c + 1 < t.n && blk >= t.start[c + 1]) ++c;
  const MmseCell& e = t.cell[c];
  __shared__ __align__(16) MfmaLds<kMaxD> lds;
  mmse_mfma_body<KS, true, NT, kMaxD>(lds, blk - t.start[c], nullptr, e.Y, e.taps, e.Xh, e.st, e.g, e.cg,
                                      e.nblk_batch);
}

template <int KS, bool FUSED, int NT>
hipError_t launch_mfma(const cf* H, const cf* Y, const int2* taps, const ChestGeom& cg, cf* Xh, int* st,
                       const MmseGeom& g, long long batch, hipStream_t s) {
  const int nblk_batch = (g.n_sc + kSPW - 1) / kSPW;
  const long long nblk = batch * nblk_batch;
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  // P for 12 data symbols when the call has at most 12 (less LDS per wave)
  if (g.n_data <= 12)
    hipLaunchKernelGGL((k_mmse_mfma<KS, FUSED, NT, 12>), dim3((unsigned)nblk), dim3(64), 0, s, H, Y, taps, Xh, st, g,
                       cg, nblk_batch);
  else
    hipLaunchKernelGGL((k_mmse_mfma<KS, FUSED, NT, kMaxD>), dim3((unsigned)nblk), dim3(64), 0, s, H, Y, taps, Xh, st,
                       g, cg, nblk_batch);
  return hipGetLastError();
}

template <bool FUSED, int NT>
hipError_t dispatch_mfma(const cf* H, const cf* Y, const int2* taps, const ChestGeom& cg, cf* Xh, int* st,
                         const MmseGeom& g, long long batch, hipStream_t s) {
  const int nb = g.n_beams;
  if (nb <= 8) return launch_mfma<2, FUSED, NT>(H, Y, taps, cg, Xh, st, g, batch, s);
  if (nb <= 16) return launch_mfma<4, FUSED, NT>(H, Y, taps, cg, Xh, st, g, batch, s);
  if (nb <= 32) return launch_mfma<8, FUSED, NT>(H, Y, taps, cg, Xh, st, g, batch, s);
  if (nb <= 64) return launch_mfma<16, FUSED, NT>(H, Y, taps, cg, Xh, st, g, batch, s);
  return hipErrorInvalidValue;
}

// Any detection classes in one launch: each workgroup runs its cell's class.
__global__ __launch_bounds__(64) void k_mmse_mfma_any(MmseCells t) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  int c = 0;
  while (c + 1 < t.n && blk >= t.start[c + 1]) ++c;
  const MmseCell& e = t.cell[c];
  const int b = blk - t.start[c];
  __shared__ __align__(16) MfmaLds<kMaxD> lds;
#define MM_CASE(CLS, KS, NT)                                                                              \
  case CLS:                                                                                              \
    mmse_mfma_body<KS, true, NT, kMaxD>(lds, b, nullptr, e.Y, e.taps, e.Xh, e.st, e.g, e.cg, e.nblk_batch); \
    break;
  switch (e.cls) {
    MM_CASE(0, 2, 2)
    MM_CASE(1, 2, 2 * kMaxPilots)
    MM_CASE(2, 4, 2)
    MM_CASE(3, 4, 2 * kMaxPilots)
    MM_CASE(4, 8, 2)
    MM_CASE(5, 8, 2 * kMaxPilots)
    MM_CASE(6, 16, 2)
    default: MM_CASE(7, 16, 2 * kMaxPilots)
  }
#undef MM_CASE
}

// ---------------------------------------------------------------- time-varying channel, two pilot symbols
// Data symbol d's estimate is H_d = (1 - a) H_0 + a H_1, so
//   H_d^H H_d = (1 - a)(1 - 2a) H_0^H H_0 + a(2a - 1) H_1^H H_1 + a(1 - a) H_u^H H_u,  H_u = H_0 + H_1,
//   H_d^H y_d = (1 - a) H_0^H y_d + a H_1^H y_d:
// one pass of MFMAs per subcarrier (9 + 6 per K-step) gives every data
// symbol's Gram matrix and matched filter.  Written as a polynomial in a,
//   H_d^H H_d = A + a (B + a C),  A = H_0^H H_0,  B = H_u^H H_u - 3 A - H_1^H H_1,
//   C = 2 A + 2 H_1^H H_1 - H_u^H H_u,
// it costs two multiply-adds per entry and data symbol.  Each data symbol is
// then factored (Crout, as the static kernel) and solved with one lane per
// row: forward and back substitution step through the rows, each final
// component reaching the other rows by a DPP row broadcast.

// Grid index of data symbol d: the d-th from d_first that is not a pilot grid.
__device__ __forceinline__ int data_symbol(const MmseGeom& g, int d) {
  int s = g.d_first + d;
#pragma unroll
  for (int j = 0; j < kMaxPilots; ++j)
    if (j < g.n_skip && g.skip[j] <= s) ++s;
  return s;
}

// LDS of a workgroup: the lower triangles of A (with the regularisation on
// its diagonal), B and C of the subcarrier in work, its matched filters
// H_d^H y_d = (1 - a_d) H_0^H y_d + a_d H_1^H y_d (rows of NDP data symbols,
// as MfmaLds), and per lane group the factor of the data symbol it is
// solving (strictly lower part, each row divided by its diagonal entry,
// packed by rows as the triangles: row i at tri(i), so a row written by 16
// lanes and a column read by them each spread over the banks).
template <int NDP>
struct TvLds {
  cf GA[kTri];
  cf GB[kTri];
  cf GC[kTri];
  cf P[kMatP<NDP>];
  cf Lt[kSPW * kTri];
};

// dreg: the regularisation of row c16, on the diagonal of A.  g*: the three
// Hermitian products as three real products each (GpAcc's g1, g2, g3).
__device__ __forceinline__ void tv_store_g(cf* __restrict__ GA, cf* __restrict__ GB, cf* __restrict__ GC,
                                           const f32x4 (&g0)[3], const f32x4 (&g1)[3], const f32x4 (&gu)[3],
                                           float dreg, int q, int c16) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * q + v;
    if (i >= c16) {
      const int e = tri(i) + c16;
      const cf a0 = cf{g0[0][v] + g0[1][v], g0[2][v] - g0[0][v] + g0[1][v]};
      const cf a1 = cf{g1[0][v] + g1[1][v], g1[2][v] - g1[0][v] + g1[1][v]};
      const cf au = cf{gu[0][v] + gu[1][v], gu[2][v] - gu[0][v] + gu[1][v]};
      GA[e] = cf{a0.r + (i == c16 ? dreg : 0.f), a0.i};
      GB[e] = cf{au.r - 3.f * a0.r - a1.r, au.i - 3.f * a0.i - a1.i};
      GC[e] = cf{2.f * (a0.r + a1.r) - au.r, 2.f * (a0.i + a1.i) - au.i};
    }
  }
}

// The time-weighted matched filter of column c16 (data symbol c16, weight al)
// from both pilot symbols' products p0, p1 (three real products each).
template <int NDP>
__device__ __forceinline__ void tv_store_p(cf* __restrict__ P, const f32x4 (&p0)[3], const f32x4 (&p1)[3], float al,
                                           int q, int c16) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * q + v;
    if (c16 < kRowP<NDP>) {
      const cf b0 = cf{p0[0][v] + p0[1][v], p0[2][v] - p0[0][v] + p0[1][v]};
      const cf b1 = cf{p1[0][v] + p1[1][v], p1[2][v] - p1[0][v] + p1[1][v]};
      P[i * kRowP<NDP> + c16] = cf{(1.f - al) * b0.r + al * b1.r, (1.f - al) * b0.i + al * b1.i};
    }
  }
}

// One workgroup takes kSPW subcarriers, one at a time: phase A puts the
// subcarrier's three Gram products and its matched filters in LDS, then the
// four lane groups take four of its data symbols at a time (group q the
// data symbols q, q + 4, ...), each lane holding row c16 of that data
// symbol's Gram matrix.  Holding one subcarrier's products, not four, keeps
// the workgroup's LDS small enough for several waves per SIMD.
// FULL (16 UEs): the row and column guards fold away, so the scalar unit
// holds no per-row conditions.
template <int KS, int NDP, bool FULL>
__global__ __launch_bounds__(64, 3) void k_mmse_tv(const cf* __restrict__ Y, const int2* __restrict__ taps,
                                                   cf* __restrict__ Xh, int* __restrict__ st, MmseGeom g, ChestGeom cg,
                                                   int nblk_batch) {
  __shared__ __align__(16) TvLds<NDP> lds;
  const int lane = threadIdx.x;
  const int c16 = lane & 15, q = lane >> 4;
  const int nb = g.n_beams, nue = FULL ? 16 : g.n_ue, nsc = g.n_sc, nd = g.n_data;
  const long long ysym = data_grid(g, c16 < nd ? c16 : 0);  // this lane's data symbol (B operand)
  const int blk = xcd_block(blockIdx.x, gridDim.x);  // neighbouring subcarriers on one XCD
  const int bi = blk / nblk_batch;
  const int k0 = (blk - bi * nblk_batch) * kSPW;
  const int ue = c16 < nue ? c16 : 0;  // lanes past n_ue: UE 0's taps, result discarded
  const cf* LSb = Y + bi * cg.y_batch;
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  const float pa = (float)cg.pilot_sym[0], pspan = (float)(cg.pilot_sym[1] - cg.pilot_sym[0]);
  auto weight = [&](int d) {  // time weight of pilot symbol 1 for data symbol d
    const float a = ((float)data_symbol(g, d) - pa) / pspan;
    return a < 0.f ? 0.f : (a > 1.f ? 1.f : a);
  };
  const float al_lane = weight(c16 < nd ? c16 : 0);  // this lane's matched-filter column
  const float s2 = g.sigma2_item ? g.sigma2_item[bi] : g.sigma2;
  const int grp = q, i = c16;
  const cf* GAr = lds.GA + tri(i);
  const cf* GBr = lds.GB + tri(i);
  const cf* GCr = lds.GC + tri(i);
  cf* Ltg = lds.Lt + grp * kTri;

#pragma unroll 1
  for (int sc = 0; sc < kSPW; ++sc) {
    // ---- phase A: both pilot symbols' estimates of this lane's UE and
    // beams, then the three Gram matrices and the two matched filters
    const int k = k0 + sc;
    {
      const int kk = k < nsc ? k : nsc - 1;
      const int4* tp = reinterpret_cast<const int4*>(taps + ((long long)kk * nue + ue) * 4);
      const int4 ta = tp[0], tb = tp[1];  // pilot symbol 0: two (offset, weight) taps; pilot symbol 1
      const float wa0 = __int_as_float(ta.y), wa1 = __int_as_float(ta.w);
      const float wb0 = __int_as_float(tb.y), wb1 = __int_as_float(tb.w);
      const cf* yrow = Y + bi * g.y_batch + ysym + (long long)kk * nb;
      const bool live = c16 < nue && k < nsc;  // else zero rows of H
      // both pilot symbols' estimates of K-step pair u (beams of fragment
      // slots 2u, 2u + 1), zero on rows past n_ue and beams past n_beams
      auto est = [&](int u, float4& h0, float4& h1) {
        const int b = frag_beam(2 * u, q);
        const float4 p = load_pair_even(LSb + ta.x, b, nb), r = load_pair_even(LSb + ta.z, b, nb);
        const float4 s_ = load_pair_even(LSb + tb.x, b, nb), t = load_pair_even(LSb + tb.z, b, nb);
        const bool keep = live && b < nb;
        h0 = float4{__builtin_fmaf(wa1, r.x, wa0 * p.x), __builtin_fmaf(wa1, r.y, wa0 * p.y),
                    __builtin_fmaf(wa1, r.z, wa0 * p.z), __builtin_fmaf(wa1, r.w, wa0 * p.w)};
        h1 = float4{__builtin_fmaf(wb1, t.x, wb0 * s_.x), __builtin_fmaf(wb1, t.y, wb0 * s_.y),
                    __builtin_fmaf(wb1, t.z, wb0 * s_.z), __builtin_fmaf(wb1, t.w, wb0 * s_.w)};
        if (!keep) h0 = h1 = float4{0.f, 0.f, 0.f, 0.f};
      };
      // pass 1: the three Hermitian products (9 MFMAs per K-step), to LDS
      {
        f32x4 g0[3] = {z4, z4, z4}, g1[3] = {z4, z4, z4}, gu[3] = {z4, z4, z4};
#pragma unroll
        for (int u = 0; u < KS / 2; ++u) {
          float4 h0, h1;
          est(u, h0, h1);
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const cf x0 = e ? cf{h0.z, h0.w} : cf{h0.x, h0.y};
            const cf x1 = e ? cf{h1.z, h1.w} : cf{h1.x, h1.y};
            const cf xu = cf{x0.r + x1.r, x0.i + x1.i};
            g0[0] = mfma(x0.r, x0.r, g0[0]);
            g0[1] = mfma(x0.i, x0.i, g0[1]);
            g0[2] = mfma(x0.r - x0.i, x0.r + x0.i, g0[2]);
            g1[0] = mfma(x1.r, x1.r, g1[0]);
            g1[1] = mfma(x1.i, x1.i, g1[1]);
            g1[2] = mfma(x1.r - x1.i, x1.r + x1.i, g1[2]);
            gu[0] = mfma(xu.r, xu.r, gu[0]);
            gu[1] = mfma(xu.i, xu.i, gu[1]);
            gu[2] = mfma(xu.r - xu.i, xu.r + xu.i, gu[2]);
          }
        }
        // padding rows beyond n_ue (and a subcarrier past n_sc) get 1, so
        // their part of every factor is the identity
        tv_store_g(lds.GA, lds.GB, lds.GC, g0, g1, gu, (c16 < nue && k < nsc) ? s2 : 1.0f, q, c16);
      }
      // pass 2: both matched filters (6 MFMAs per K-step; the estimates are
      // formed again from the same LS values, L2 hits), to LDS
      {
        f32x4 p0[3] = {z4, z4, z4}, p1[3] = {z4, z4, z4};
#pragma unroll
        for (int u = 0; u < KS / 2; ++u) {
          float4 h0, h1;
          est(u, h0, h1);
          const float4 yy = load_pair_even(yrow, frag_beam(2 * u, q), nb);
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const cf x0 = e ? cf{h0.z, h0.w} : cf{h0.x, h0.y};
            const cf x1 = e ? cf{h1.z, h1.w} : cf{h1.x, h1.y};
            const cf y = e ? cf{yy.z, yy.w} : cf{yy.x, yy.y};
            const float ys = y.r + y.i;
            p0[0] = mfma(x0.r, y.r, p0[0]);
            p0[1] = mfma(x0.i, y.i, p0[1]);
            p0[2] = mfma(x0.r - x0.i, ys, p0[2]);
            p1[0] = mfma(x1.r, y.r, p1[0]);
            p1[1] = mfma(x1.i, y.i, p1[1]);
            p1[2] = mfma(x1.r - x1.i, ys, p1[2]);
          }
        }
        tv_store_p<NDP>(lds.P, p0, p1, al_lane, q, c16);
      }
    }
    __syncthreads();

    // ---- per data symbol: Gram matrix, Crout factorisation and both
    // substitutions, lane (q, c16) holding row c16; group q takes data
    // symbols q, q + 4, ... (a group past n_data repeats the last one and
    // stores nothing, so every lane reaches the barriers)
    int fail_any = 0;
#pragma unroll 1
    for (int d0 = 0; d0 < nd; d0 += kSPW) {
      const bool act = d0 + grp < nd;
      const int d = act ? d0 + grp : nd - 1;
      const float al = weight(d);
      // row i of the Gram matrix A + a (B + a C) (every lane reads 16
      // entries, in bounds of the triangles: no divergent loads; the entries
      // past its diagonal are other rows' and only feed columns above the
      // diagonal, which the factorisation computes but never reads)
      cf L[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const cf a = GAr[j], b = GBr[j], c = GCr[j];
        L[j] = cf{__builtin_fmaf(al, __builtin_fmaf(al, c.r, b.r), a.r),
                  __builtin_fmaf(al, __builtin_fmaf(al, c.i, b.i), a.i)};
      }
      float dvi;
      const int fail = crout_rows(L, i, nue, nullptr, dvi);
      // L = D L' with D = diag(L_ii): row i of the unit lower triangle L'
      // (L_ij / L_ii below the diagonal, zero elsewhere, so the forward
      // substitution needs no per-lane branch), and the rows to LDS for the
      // column reads.  G x = b is then L' z = D^-1 b, L'^H w = z, x = D^-1 w,
      // with no division inside either substitution.
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        L[j] = j < i ? cf{L[j].r * dvi, L[j].i * dvi} : cf{0.f, 0.f};
        if (j < i) Ltg[tri(i) + j] = L[j];
      }
      __syncthreads();
      // right-hand side H_d^H y_d, component i, divided by L_ii
      const cf bi_ = lds.P[i * kRowP<NDP> + d];
      cf zi = cf{bi_.r * dvi, bi_.i * dvi};
      // L' z = D^-1 b: lane m's value is final once the rows above it are
      // removed; it is broadcast and removed from the rows below (L'[m] is
      // zero on the lanes at or above row m, so a lane's own value stays put
      // after its turn)
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        if (m < nue) {
          const cf zm = row_bcast_c(zi, m);
          csub_mul(zi, L[m], zm);
        }
      }
      // L'^H w = z: column i of L' (entries of rows m > i; the reads of rows
      // m <= i stay inside the group's triangle and are replaced by zero);
      // w_m final on lane m, broadcast, and removed from the rows above;
      // then x_i = w_i / L_ii
      cf Lc[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const cf v = Ltg[tri(m) + i];
        Lc[m] = m > i ? v : cf{0.f, 0.f};
      }
#pragma unroll
      for (int m = 15; m >= 0; --m) {
        if (m < nue) {
          const cf wm = row_bcast_c(zi, m);
          csub_conj_mul(zi, Lc[m], wm);
        }
      }
      zi = cf{zi.r * dvi, zi.i * dvi};
      if (act && k < nsc && i < nue) Xh[bi * g.x_batch + ((long long)d * nsc + k) * nue + i] = fail ? cf{0.f, 0.f} : zi;
      fail_any |= act ? fail : 0;
      __syncthreads();  // the next data symbols write their factors over these
    }
    // the subcarrier's flag: any of its data symbols, over the four groups
    fail_any |= __shfl_xor(fail_any, 16);
    fail_any |= __shfl_xor(fail_any, 32);
    if (k < nsc && lane == 0 && st) {
      int* sp = st + bi * g.st_batch + k;
      *sp = g.st_or ? (*sp | fail_any) : fail_any;
    }
  }
}

template <int KS>
hipError_t launch_tv_ks(const cf* Y, const int2* taps, const ChestGeom& cg, cf* Xh, int* st, const MmseGeom& g,
                        long long nblk, int nblk_batch, hipStream_t s) {
  const bool full = g.n_ue == 16;
  if (g.n_data <= 12 && full)
    hipLaunchKernelGGL((k_mmse_tv<KS, 12, true>), dim3((unsigned)nblk), dim3(64), 0, s, Y, taps, Xh, st, g, cg,
                       nblk_batch);
  else if (g.n_data <= 12)
    hipLaunchKernelGGL((k_mmse_tv<KS, 12, false>), dim3((unsigned)nblk), dim3(64), 0, s, Y, taps, Xh, st, g, cg,
                       nblk_batch);
  else if (full)
    hipLaunchKernelGGL((k_mmse_tv<KS, kMaxD, true>), dim3((unsigned)nblk), dim3(64), 0, s, Y, taps, Xh, st, g, cg,
                       nblk_batch);
  else
    hipLaunchKernelGGL((k_mmse_tv<KS, kMaxD, false>), dim3((unsigned)nblk), dim3(64), 0, s, Y, taps, Xh, st, g, cg,
                       nblk_batch);
  return hipGetLastError();
}

template <int KS>
hipError_t launch_cells_ks(MmseCells& t, int n_tap, unsigned blocks, hipStream_t s) {
  if (n_tap == 2) hipLaunchKernelGGL((k_mmse_mfma_cells<KS, 2>), dim3(blocks), dim3(64), 0, s, t);
  else hipLaunchKernelGGL((k_mmse_mfma_cells<KS, 2 * kMaxPilots>), dim3(blocks), dim3(64), 0, s, t);
  return hipGetLastError();
}

}  // namespace

int mmse_cell_class(int n_beams, int n_tap) {
  if (n_tap != 2 && n_tap != 2 * kMaxPilots) return -1;
  const int ks = n_beams <= 8 ? 0 : (n_beams <= 16 ? 1 : (n_beams <= 32 ? 2 : (n_beams <= 64 ? 3 : -1)));
  return ks < 0 ? -1 : ks * 2 + (n_tap == 2 ? 0 : 1);
}

hipError_t launch_mmse_cells(MmseCells& t, int cls, hipStream_t s) {
  if (t.n < 1 || t.n > kMmseCellsPerLaunch || cls < -1 || cls >= 8) return hipErrorInvalidValue;
  long long start = 0;
  for (int c = 0; c < t.n; ++c) {
    MmseCell& e = t.cell[c];
    e.cls = mmse_cell_class(e.g.n_beams, e.n_tap);
    if (e.batch <= 0 || e.g.n_data > kMaxD || e.g.n_data < 1 || e.g.n_beams != e.cg.n_beams ||
        !mmse_fusable(e.g.n_ue, e.g.n_beams, e.cg.y_batch) || e.cls < 0 || (cls >= 0 && e.cls != cls))
      return hipErrorInvalidValue;
    e.nblk_batch = (e.g.n_sc + kSPW - 1) / kSPW;
    t.start[c] = (int)start;
    start += e.batch * e.nblk_batch;
    if (start > 0x7fffffffLL) return hipErrorInvalidValue;
  }
  t.start[t.n] = (int)start;
  if (cls < 0) {
    hipLaunchKernelGGL(k_mmse_mfma_any, dim3((unsigned)start), dim3(64), 0, s, t);
    return hipGetLastError();
  }
  const int n_tap = cls % 2 ? 2 * kMaxPilots : 2;
  switch (cls / 2) {
    case 0: return launch_cells_ks<2>(t, n_tap, (unsigned)start, s);
    case 1: return launch_cells_ks<4>(t, n_tap, (unsigned)start, s);
    case 2: return launch_cells_ks<8>(t, n_tap, (unsigned)start, s);
    default: return launch_cells_ks<16>(t, n_tap, (unsigned)start, s);
  }
}

hipError_t launch_mmse_tv(const cf* Y, const int2* taps, const ChestGeom& cg, cf* Xhat, int* status,
                          const MmseGeom& g, long long batch, hipStream_t s) {
  if (g.n_data > kMaxD || g.n_data < 1 || cg.n_pilot != 2 || cg.pilot_sym[1] <= cg.pilot_sym[0] ||
      !mmse_fusable(g.n_ue, g.n_beams, cg.y_batch))
    return hipErrorInvalidValue;
  const int nblk_batch = (g.n_sc + kSPW - 1) / kSPW;
  const long long nblk = batch * nblk_batch;
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  const int nb = g.n_beams;
  if (nb <= 8) return launch_tv_ks<2>(Y, taps, cg, Xhat, status, g, nblk, nblk_batch, s);
  if (nb <= 16) return launch_tv_ks<4>(Y, taps, cg, Xhat, status, g, nblk, nblk_batch, s);
  if (nb <= 32) return launch_tv_ks<8>(Y, taps, cg, Xhat, status, g, nblk, nblk_batch, s);
  return launch_tv_ks<16>(Y, taps, cg, Xhat, status, g, nblk, nblk_batch, s);
}

bool mmse_auto_refine(int n_ue, int n_beams) { return n_ue > 16 && 2 * n_ue > n_beams; }

bool mmse_fusable(int n_ue, int n_beams, long long y_batch) {
  // MFMA tile of 16 UEs; paired 16-byte beam loads; 32-bit tap offsets
  return n_ue >= 1 && n_ue <= 16 && n_beams >= 2 && n_beams <= 64 && n_beams % 2 == 0 && y_batch < (1ll << 31);
}

hipError_t launch_mmse(const cf* H, const cf* Y, cf* Xhat, int* status, const MmseGeom& g, long long batch,
                       hipStream_t s) {
  if (g.n_data > kMaxD || g.n_data < 1) return hipErrorInvalidValue;
  // refinement: the row kernel (any n_ue up to 32).  Beyond 16 UEs with more
  // than half as many UEs as beams it refines without being asked: the
  // smallest eigenvalue of H^H H shrinks like (1 - sqrt(N_L / N_B))^2 relative
  // to the largest (for channels with independent entries), so the
  // regularised Gram matrices reach condition numbers of 1e3..1e5 at high SNR,
  // where the FP32 solve alone misses 1e-4; at N_B >= 2 N_L they stay near
  // 1e1..1e2.
  if (g.n_ue <= 16 && !g.refine) return dispatch_mfma<false, 0>(H, Y, nullptr, ChestGeom{}, Xhat, status, g, batch, s);
  if (g.n_ue <= 32) {
    MmseGeom gr = g;
    gr.refine = g.refine || mmse_auto_refine(g.n_ue, g.n_beams);
    return launch_lps<32>(H, Y, Xhat, status, gr, batch, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mmse_fused(const cf* Y, const int2* taps, int n_tap, const ChestGeom& cg, cf* Xhat, int* status,
                             const MmseGeom& g, long long batch, hipStream_t s) {
  if (g.n_data > kMaxD || g.n_data < 1 || !mmse_fusable(g.n_ue, g.n_beams, cg.y_batch)) return hipErrorInvalidValue;
  if (n_tap == 2) return dispatch_mfma<true, 2>(nullptr, Y, taps, cg, Xhat, status, g, batch, s);
  if (n_tap == 4) return dispatch_mfma<true, 4>(nullptr, Y, taps, cg, Xhat, status, g, batch, s);
  if (n_tap == 2 * kMaxPilots) return dispatch_mfma<true, 2 * kMaxPilots>(nullptr, Y, taps, cg, Xhat, status, g, batch, s);
  return hipErrorInvalidValue;
}

}  // namespace pusch
