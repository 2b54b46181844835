// Legendre stage of the spherical harmonic transforms on gfx950.
//
// Synthesis (first half of Y, Sect. 2.1):
//     F^{c|s}_m(r) = sum_{l=m..L} lambda_lm(z_r) u^{c|s}_lm
// Adjoint (second half of Y^T, Sect. 3.2):
//     v^{c|s}_lm   = sum_r lambda_lm(z_r) H^{c|s}_m(r)
// The normalised Legendre functions are generated in registers by the
// mu-recurrence mu_l = g_lm z mu_{l-1} - mu_{l-2} (lambda = f_lm mu, see
// grid.hip), so the harmonic vectors handed to these kernels are "hat"
// vectors u^ = c_m f_lm u (c_0 = 1, c_m = sqrt 2) and the adjoint returns
// v^ with v = c_m f_lm v^.  North/south ring pairs share the recurrence:
// lambda_lm(-z) = (-1)^(l+m) lambda_lm(z), so even and odd l-m terms are
// accumulated separately (E, O) and F_N = E + O, F_S = E - O.
//
// Each (ring pair, m) starts at the first l where |lambda_lm| reaches 2^-100
// (start table from grid.hip); smaller terms are not evaluated.  Lanes of a
// wave start at different l: the wave runs one recurrence step per l for
// all lanes and, at the (wave-uniform) l where some lane starts, injects
// that lane's start values.
#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <tuple>
#include <cstdio>
#include <cstdlib>

#include "internal.h"

namespace crs {

namespace {

// Read-only tables and harmonic inputs are read through the constant
// address space so that wave-uniform loads become scalar (SMEM) loads.
typedef __attribute__((address_space(4))) const double cdouble;
__device__ __forceinline__ cdouble* as_const(const double* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (cdouble*)(((uint64_t)hi << 32) | lo);
}
// wave-uniform element (scalar load)
__device__ __forceinline__ double uld(cdouble* p, int i) { return p[__builtin_amdgcn_readfirstlane(i)]; }

// minimum over the wave's active lanes (DPP reduction, no LDS round trips)
__device__ __forceinline__ int wave_min(int v) {
  return __builtin_amdgcn_readfirstlane(__ockl_wfred_min_i32(v));
}

// v + v of lane t ^ 32 and v + v of lane t ^ 16, with the gfx950 lane-swap
// instructions (v_permlane32_swap exchanges the upper half of its first
// operand with the lower half of its second; v_permlane16_swap the odd rows of
// the first with the even rows of the second): swapping v with itself leaves
// the lane's own value in one result and the partner's in the other.
__device__ __forceinline__ double add_xor32(double v) {
  const uint64_t u = __double_as_longlong(v);
  const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double x = __longlong_as_double((long long)(((uint64_t)b[0] << 32) | a[0]));
  const double y = __longlong_as_double((long long)(((uint64_t)b[1] << 32) | a[1]));
  return x + y;
}
// Transposing form: lanes t < 32 get A(t) + A(t + 32), lanes t >= 32 get
// B(t - 32) + B(t) (both lanes of a pair add in the same order).
__device__ __forceinline__ double fold32(double A, double B) {
  const uint64_t ua = __double_as_longlong(A), ub = __double_as_longlong(B);
  const auto a = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  const double x = __longlong_as_double((long long)(((uint64_t)b[0] << 32) | a[0]));
  const double y = __longlong_as_double((long long)(((uint64_t)b[1] << 32) | a[1]));
  return x + y;
}
__device__ __forceinline__ double add_xor16(double v) {
  const uint64_t u = __double_as_longlong(v);
  const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double x = __longlong_as_double((long long)(((uint64_t)b[0] << 32) | a[0]));
  const double y = __longlong_as_double((long long)(((uint64_t)b[1] << 32) | a[1]));
  return x + y;
}

__device__ __forceinline__ int64_t moff(int L, int m) {
  return (m == 0) ? 0 : (int64_t)(L + 1) + 2 * ((int64_t)(m - 1) * (L + 1) - (int64_t)(m - 1) * m / 2);
}
__device__ __forceinline__ int64_t tri(int L, int m) {
  return (int64_t)m * (L + 1) - (int64_t)m * (m - 1) / 2;
}

// ------------------------------------------------------- per-wave stepper
// A wave owns R groups of 64 ring pairs: pair of group j on lane t is
// base + 64 j + t (j = 0 most polar).  Per group the wave keeps the lanes'
// recurrence state and two wave-uniform numbers: lw (first l any lane of
// groups j..R-1 evaluates; lw[R-1] is where the wave starts stepping) and nx
// (next l where some lane of the group starts).  Between start events all
// groups step in lockstep; a lane before its start carries zero state.
template <int R>
struct Grp {
  double z[R], a0[R], a1[R];
  double2 st[R];  // the lane's start values (mu_{ls-1}, mu_ls), loaded up front
  int ls[R];
  int lw[R];
  int nx[R];
};

template <int R>
__device__ __forceinline__ void grp_init(Grp<R>& G, const LegArgs& a, int m, int base, int lane) {
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int p = base + 64 * j + lane;
    const bool valid = p < a.npairs;
    G.z[j] = a.zpair[valid ? p : a.npairs - 1];
    G.ls[j] = valid ? a.ls[(size_t)m * a.npairs + p] : INT_MAX;
    G.st[j] = valid ? a.ms[(size_t)m * a.npairs + p] : make_double2(0.0, 0.0);
    G.a0[j] = 0.0;
    G.a1[j] = 0.0;
    const int w = wave_min(G.ls[j]);
    G.nx[j] = w;
    G.lw[j] = (j == 0) ? w : min(w, G.lw[j - 1]);
  }
}

// One step of group j at l with start injection (event step).
template <int R>
__device__ __forceinline__ double grp_event_step(Grp<R>& G, int j, const LegArgs& a, int m, int base,
                                                 int lane, int l, double gl) {
  double c = fma(gl * G.z[j], G.a1[j], -G.a0[j]);
  double pv = G.a1[j];
  if (l == G.nx[j]) {
    if (G.ls[j] == l) {
      c = G.st[j].y;
      pv = G.st[j].x;
    }
    G.nx[j] = wave_min(G.ls[j] > l ? G.ls[j] : INT_MAX);
  }
  G.a0[j] = pv;
  G.a1[j] = c;
  return c;
}

// ------------------------------------------------------------- synthesis
// Accumulators X (parity of the next step) and Y (the other parity): every
// step adds into X and then swaps X and Y, so consecutive steps need no
// parity test (the swap is free inside unrolled pairs).  At the end X holds
// the sum over l with l - m of the parity of L + 1 - m.
template <int NM, int R>
struct SynAcc {
  double X[R][NM][2], Y[R][NM][2];  // [group][map][cos, sin]
};

template <int NM, int R>
__device__ __forceinline__ void syn_swap(SynAcc<NM, R>& A) {
#pragma unroll
  for (int j = 0; j < R; ++j)
#pragma unroll
    for (int k = 0; k < NM; ++k)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double t = A.X[j][k][c];
        A.X[j][k][c] = A.Y[j][k][c];
        A.Y[j][k][c] = t;
      }
}

// one step of every group into X (no swap)
template <int NM, int R, bool HAS_S>
__device__ __forceinline__ void syn_acc(SynAcc<NM, R>& A, Grp<R>& G, double gl, const double* uc,
                                        const double* us) {
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const double c = fma(gl * G.z[j], G.a1[j], -G.a0[j]);
    G.a0[j] = G.a1[j];
    G.a1[j] = c;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      A.X[j][k][0] = fma(c, uc[k], A.X[j][k][0]);
      if (HAS_S) A.X[j][k][1] = fma(c, us[k], A.X[j][k][1]);
    }
  }
}

// One chunk of B steps from l (B even, so the even / odd accumulators keep
// their roles).  EV: some lane may start inside the chunk; every step then
// checks for start events (wave-uniform test per group, start values and
// the next event only at an event).
template <int NM, int R, bool HAS_S, bool EV>
__device__ __forceinline__ void syn_chunk(SynAcc<NM, R>& A, Grp<R>& G, const LegArgs& a, int m, int base,
                                          int lane, cdouble* gb, cdouble* const* ub, int nsl, int l) {
  constexpr int B = (NM == 1) ? 8 : ((NM == 2) ? 4 : 2);
  l = __builtin_amdgcn_readfirstlane(l);
  cdouble* gp = gb + l;
  double gv[B], uc[B][NM], us[B][NM];
#pragma unroll
  for (int i = 0; i < B; ++i) gv[i] = gp[i];
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    cdouble* up = ub[k] + l;
#pragma unroll
    for (int i = 0; i < B; ++i) {
      uc[i][k] = up[i];
      us[i][k] = HAS_S ? up[i + nsl] : 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i < B; ++i) {
    if (EV) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const double c = grp_event_step<R>(G, j, a, m, base, lane, l + i, gv[i]);
#pragma unroll
        for (int k = 0; k < NM; ++k) {
          A.X[j][k][0] = fma(c, uc[i][k], A.X[j][k][0]);
          if (HAS_S) A.X[j][k][1] = fma(c, us[i][k], A.X[j][k][1]);
        }
      }
    } else {
      syn_acc<NM, R, HAS_S>(A, G, gv[i], uc[i], us[i]);
    }
    syn_swap<NM, R>(A);
  }
}

// one event-checked step at l (the last steps of a wave, fewer than a chunk)
template <int NM, int R, bool HAS_S>
__device__ __forceinline__ void syn_step(SynAcc<NM, R>& A, Grp<R>& G, const LegArgs& a, int m, int base,
                                         int lane, cdouble* gb, cdouble* const* ub, int nsl, int l) {
  const double gl = uld(gb, l);
  double uc[NM], us[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    uc[k] = uld(ub[k], l);
    us[k] = HAS_S ? uld(ub[k], l + nsl) : 0.0;
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const double c = grp_event_step<R>(G, j, a, m, base, lane, l, gl);
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      A.X[j][k][0] = fma(c, uc[k], A.X[j][k][0]);
      if (HAS_S) A.X[j][k][1] = fma(c, us[k], A.X[j][k][1]);
    }
  }
  syn_swap<NM, R>(A);
}

// map slots of a launch (see LegArgs::mlist)
__device__ __forceinline__ int leg_nslots(const LegArgs& a, int nmaps) {
  return a.mcount ? __builtin_amdgcn_readfirstlane(*a.mcount) : nmaps;
}
__device__ __forceinline__ int leg_map(const LegArgs& a, int slot) { return a.mlist ? a.mlist[slot] : slot; }
// some slot of [s0, s0 + n) holds a map to process
__device__ __forceinline__ bool leg_any(const LegArgs& a, int s0, int n, int ns) {
  if (!a.skip.act) return s0 < ns;
  bool any = false;
  for (int k = 0; k < n && s0 + k < ns; ++k) any = any || !a.skip.off(leg_map(a, s0 + k));
  return any;
}

template <int NM, int R, bool HAS_S>
__device__ __forceinline__ void synth_wave(const LegArgs& a, int m, int base, int lane, int nmaps, int map0,
                                           const double* __restrict__ uhat, int64_t ustride,
                                           double2* __restrict__ phase, int64_t pstride) {
  const int L = a.lmax;
  cdouble* gb = as_const(a.g + tri(L, m) - m);
  const int nsl = L - m + 1;
  cdouble* ub[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k)
    ub[k] = as_const(uhat + (int64_t)leg_map(a, min(map0 + k, nmaps - 1)) * ustride + moff(L, m) - m);
  Grp<R> G;
  grp_init<R>(G, a, m, base, lane);
  SynAcc<NM, R> A;
#pragma unroll
  for (int j = 0; j < R; ++j)
#pragma unroll
    for (int k = 0; k < NM; ++k) A.X[j][k][0] = A.X[j][k][1] = A.Y[j][k][0] = A.Y[j][k][1] = 0.0;
  // all R groups step from the first start of any of them (groups that have
  // not started carry zero state and add zeros), in chunks of B steps; a
  // chunk takes the event-checked path only if a start falls inside it
  constexpr int B = (NM == 1) ? 8 : ((NM == 2) ? 4 : 2);
  int l = G.lw[R - 1];
  for (; l + B <= L + 1; l += B) {
    int ne = G.nx[0];
#pragma unroll
    for (int j = 1; j < R; ++j) ne = min(ne, G.nx[j]);
    if (ne >= l + B)
      syn_chunk<NM, R, HAS_S, false>(A, G, a, m, base, lane, gb, ub, nsl, l);
    else
      syn_chunk<NM, R, HAS_S, true>(A, G, a, m, base, lane, gb, ub, nsl, l);
  }
  for (; l <= L; ++l) syn_step<NM, R, HAS_S>(A, G, a, m, base, lane, gb, ub, nsl, l);
  // X holds parity (L + 1 - m) & 1 (the loop always ends at l = L + 1, or
  // never ran, in which case X = Y = 0)
  const bool x_is_odd = ((L + 1 - m) & 1) != 0;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int p = base + 64 * j + lane;
    const int rs = a.nring - 1 - p;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const double ec = x_is_odd ? A.Y[j][k][0] : A.X[j][k][0];
      const double es = x_is_odd ? A.Y[j][k][1] : A.X[j][k][1];
      const double oc = x_is_odd ? A.X[j][k][0] : A.Y[j][k][0];
      const double os = x_is_odd ? A.X[j][k][1] : A.Y[j][k][1];
      if (p < a.npairs && map0 + k < nmaps) {
        double2* ph = phase + (int64_t)leg_map(a, map0 + k) * pstride;
        ph[(int64_t)p * (L + 1) + m] = make_double2(ec + oc, es + os);
        if (rs != p) ph[(int64_t)rs * (L + 1) + m] = make_double2(ec - oc, es - os);
      }
    }
  }
}

// XCD-aware order: the 8 XCDs take blocks round-robin; consecutive blocks on
// one XCD share an m-block (same harmonic coefficients, one L2) and small m
// (the longest recurrences) are dispatched first.  Wave w of a block takes
// m = 4 mb + w.
__device__ __forceinline__ void block_coords(int ntiles, int& mb, int& tile) {
  const int b = blockIdx.x;
  const int xcd = b & 7, q = b >> 3;
  tile = q % ntiles;
  mb = (q / ntiles) * 8 + xcd;
}

template <int NM, int R>
__global__ __launch_bounds__(256) void k_leg_synth(LegArgs a, int nmaps, const double* __restrict__ uhat,
                                                   int64_t ustride, double2* __restrict__ phase,
                                                   int64_t pstride, int ntiles) {
  int mb, tile;
  block_coords(ntiles, mb, tile);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = mb * 4 + wave;
  if (m > a.lmax) return;
  const int lane = threadIdx.x & 63;
  const int base = tile * 64 * R;
  const int map0 = blockIdx.y * NM;
  const int ns = leg_nslots(a, nmaps);
  if (!leg_any(a, map0, NM, ns)) return;
  if (m == 0)
    synth_wave<NM, R, false>(a, m, base, lane, ns, map0, uhat, ustride, phase, pstride);
  else
    synth_wave<NM, R, true>(a, m, base, lane, ns, map0, uhat, ustride, phase, pstride);
}

// ------------------------------------------------------ synthesis, MFMA
// For many maps the l-contraction F_par[p][col] = sum_{l of parity par}
// lambda_lm(p) u[l][col] is a dense product: rows = ring pairs, K = values of
// l of one parity (l - m even: E, odd: O), N = 16 columns = 8 maps x (cos,
// sin).  Operand layouts of v_mfma_f64_16x16x4 on gfx950 (measured): A lane t
// = A[t % 16][t / 16], B lane t = B[t / 16][t % 16], D lane t register r =
// D[t / 16 + 4 r][t % 16].
// One wave owns (m, 64 ring pairs, 8 maps); lane t runs the recurrence of
// pair t.  Each block of 8 steps [lb, lb + 8) (lb - m even) goes through a
// wave-private LDS tile lam[8][64] so that row block rb (pairs 16 rb ..
// 16 rb + 15) can be handed to the MFMA as A (lane (i, k) takes lam[2k][16 rb
// + i] for E, lam[2k + 1][...] for O); B is u at l = lb + 2k (+1) for the 16
// columns.  8 MFMAs per block, start indices injected at wave-uniform event
// blocks as in the vector kernels.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void lds_wave_sync() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS traffic done
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(256) void k_leg_synth_mfma(LegArgs a, int nmaps, const double* __restrict__ uhat,
                                                        int64_t ustride, double2* __restrict__ phase,
                                                        int64_t pstride, int ntiles) {
  __shared__ double lamsh[4][8 * 64];
  int mb, tile;
  block_coords(ntiles, mb, tile);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = mb * 4 + wave;
  const int L = a.lmax;
  if (m > L) return;
  const int mg = blockIdx.y;
  const int ns = leg_nslots(a, nmaps);
  if (!leg_any(a, mg * 8, 8, ns)) return;
  double* lam = lamsh[wave];
  const int lane = threadIdx.x & 63;
  const int i16 = lane & 15, kq = lane >> 4;
  const int p = tile * 64 + lane;
  const bool valid = p < a.npairs;
  const double z = valid ? a.zpair[p] : 0.0;
  const int ls = valid ? a.ls[(size_t)m * a.npairs + p] : INT_MAX;
  const double2 st = valid ? a.ms[(size_t)m * a.npairs + p] : make_double2(0.0, 0.0);
  // B column of this lane: map mg * 8 + j / 2, part j & 1 (cos, sin)
  const int j = i16;
  const int slot = mg * 8 + (j >> 1), cs = j & 1;
  const bool sok = slot < ns;
  const int map = sok ? leg_map(a, slot) : 0;
  const double* __restrict__ ub =
      (sok && !(m == 0 && cs == 1)) ? uhat + (int64_t)map * ustride + moff(L, m) + cs * (L - m + 1) - m : nullptr;
  cdouble* gb = as_const(a.g + tri(L, m) - m);  // 8 zeros follow the table
  // B loads are unconditional (clamped index, then masked) so that the
  // in-order vector-memory counter lets the next block's loads stay in flight
  const double* __restrict__ ubase = ub ? ub : uhat + m;
  const double bmask = ub ? 1.0 : 0.0;
  auto loadB = [&](int l) {
    const double v = ubase[l <= L ? l : L];
    return v * (l <= L ? bmask : 0.0);  // the value is always used: the load stays unconditional
  };
  const int lfirst = wave_min(ls);
  v4d DE[4], DO[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    DE[rb] = v4d{0.0, 0.0, 0.0, 0.0};
    DO[rb] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  if (lfirst <= L) {
    int lb = lfirst - ((lfirst - m) & 1);
    int nx = lfirst;  // next l at which some lane starts
    double a0 = 0.0, a1 = 0.0;
    double bE = loadB(lb + 2 * kq);
    double bO = loadB(lb + 2 * kq + 1);
    for (; lb <= L; lb += 8) {
      lb = __builtin_amdgcn_readfirstlane(lb);
      const double nE = loadB(lb + 8 + 2 * kq);
      const double nO = loadB(lb + 9 + 2 * kq);
      double gv[8];
      cdouble* gp = gb + lb;
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) gv[s2] = gp[s2];
      if (nx >= lb + 8) {
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) {
          const double cc = fma(gv[s2] * z, a1, -a0);
          a0 = a1;
          a1 = cc;
          lam[s2 * 64 + lane] = cc;
        }
      } else {
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) {
          double cc = fma(gv[s2] * z, a1, -a0);
          double pv = a1;
          if (ls == lb + s2) {
            cc = st.y;
            pv = st.x;
          }
          a0 = pv;
          a1 = cc;
          lam[s2 * 64 + lane] = cc;
        }
        nx = wave_min(ls >= lb + 8 ? ls : INT_MAX);
      }
      lds_wave_sync();
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const double aE = lam[(2 * kq) * 64 + 16 * rb + i16];
        const double aO = lam[(2 * kq + 1) * 64 + 16 * rb + i16];
        DE[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aE, bE, DE[rb], 0, 0, 0);
        DO[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aO, bO, DO[rb], 0, 0, 0);
      }
      // the next block's LDS writes follow these reads in this wave's program
      // order, which the LDS preserves; only keep the compiler from hoisting them
      __builtin_amdgcn_wave_barrier();
      bE = nE;
      bO = nO;
    }
  }
  // D[rb][row = kq + 4 r][col = j]: ring pair tile*64 + 16 rb + kq + 4 r
  if (!sok) return;
  double* ph = reinterpret_cast<double*>(phase + (int64_t)map * pstride);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pp = tile * 64 + 16 * rb + kq + 4 * r;
      if (pp >= a.npairs) continue;
      const int rs = a.nring - 1 - pp;
      ph[2 * ((int64_t)pp * (L + 1) + m) + cs] = DE[rb][r] + DO[rb][r];
      if (rs != pp) ph[2 * ((int64_t)rs * (L + 1) + m) + cs] = DE[rb][r] - DO[rb][r];
    }
}

// --------------------------------------------------------------- adjoint
// Same wave decomposition.  Per l every lane sums its groups' products into
// P[s]; each chunk of CH steps is reduced over the wave's 64 lanes through a
// wave-private LDS block (no block barrier) in a fixed order and written as
// the wave's partial v^ (one partial per ring tile of 64 R pairs).
constexpr int kRedStride = 33;  // row stride (doubles) of the reduction block
template <int NM>
struct AdjCfg {
  static constexpr int CH = (8 / NM) < 1 ? 1 : (8 / NM);
  static constexpr int NOUT = CH * NM * 2;
};

// One chunk of CH steps [lc, lc + CH) for all R groups (lc - m even: even
// steps use E, odd steps O).  Groups that have not started yet carry zero
// state and contribute zeros.  FAST: no start event inside the chunk and all
// CH steps <= L, so there are no per-step checks and P is initialised by the
// first group's products.  Otherwise every step checks for start events and
// the band-limit, and P must be zeroed by the caller.
template <int NM, int R, bool FAST, bool SQ, bool HAS_S>
__device__ __forceinline__ void adj_chunk(Grp<R>& G, const double (&E)[R][NM][2], const double (&O)[R][NM][2],
                                          const double (&gv)[AdjCfg<NM>::CH], const LegArgs& a, int m,
                                          int base, int lane, int lc, int L,
                                          double (&P)[AdjCfg<NM>::CH][NM][2]) {
  constexpr int CH = AdjCfg<NM>::CH;
#pragma unroll
  for (int s = 0; s < CH; ++s) {
    const int l = lc + s;
    if (!FAST && l > L) break;
    const bool odd = (s & 1) != 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      double c;
      if (FAST) {
        c = fma(gv[s] * G.z[j], G.a1[j], -G.a0[j]);
        G.a0[j] = G.a1[j];
        G.a1[j] = c;
      } else {
        c = grp_event_step<R>(G, j, a, m, base, lane, l, gv[s]);
      }
      const double w = SQ ? c * c : c;
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        const double hc = (SQ || !odd) ? E[j][k][0] : O[j][k][0];
        const double hs = (SQ || !odd) ? E[j][k][1] : O[j][k][1];
        if (FAST && j == 0) {
          P[s][k][0] = w * hc;
          P[s][k][1] = HAS_S ? w * hs : 0.0;
        } else {
          P[s][k][0] = fma(w, hc, P[s][k][0]);
          if (HAS_S) P[s][k][1] = fma(w, hs, P[s][k][1]);
        }
      }
    }
  }
}

template <int NM, int R, bool SQ, bool HAS_S>
__device__ __forceinline__ void adjoint_wave(const LegArgs& a, int m, int tile, int lane, int nmaps, int map0,
                                             const double2* __restrict__ phase, int64_t pstride,
                                             double* __restrict__ vpart, int64_t vstride, int64_t tstride,
                                             double* __restrict__ wb) {
  constexpr int CH = AdjCfg<NM>::CH;
  constexpr int NOUT = AdjCfg<NM>::NOUT;
  static_assert(NOUT == 16, "wave reduction assumes 16 outputs per chunk");
  static_assert(CH % 2 == 0, "chunks keep the parity of their first step");
  const int L = a.lmax;
  const int base = tile * 64 * R;
  cdouble* gb = as_const(a.g + tri(L, m) - m);
  Grp<R> G;
  grp_init<R>(G, a, m, base, lane);
  double E[R][NM][2], O[R][NM][2];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int p = base + 64 * j + lane;
    const bool valid = p < a.npairs;
    const int pc = valid ? p : a.npairs - 1;
    const int rs = a.nring - 1 - pc;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const double2* ph = phase + (int64_t)leg_map(a, min(map0 + k, nmaps - 1)) * pstride;
      const double2 hn = valid ? ph[(int64_t)pc * (L + 1) + m] : make_double2(0.0, 0.0);
      const double2 hs = (valid && rs != pc) ? ph[(int64_t)rs * (L + 1) + m] : make_double2(0.0, 0.0);
      if (valid && rs == pc) {
        // equator ring: its own pair, lambda(z) H for both parities
        E[j][k][0] = hn.x; E[j][k][1] = hn.y;
        O[j][k][0] = SQ ? 0.0 : hn.x; O[j][k][1] = SQ ? 0.0 : hn.y;
      } else {
        E[j][k][0] = hn.x + hs.x; E[j][k][1] = hn.y + hs.y;
        O[j][k][0] = hn.x - hs.x; O[j][k][1] = hn.y - hs.y;
      }
    }
  }
  const int nsl = L - m + 1;
  double* const vbase = vpart + (int64_t)tile * tstride + moff(L, m);
  // first evaluated l of any group, moved down to the parity of m (the step
  // before a start produces zeros)
  int l0 = G.lw[R - 1];
  if (l0 < m) l0 = m;
  if (l0 > L + 1) l0 = L + 1;
  l0 -= (l0 - m) & 1;
  // zero-fill this tile's output below the first evaluated l
  for (int i = lane; i < (l0 - m) * NM * 2; i += 64) {
    const int nl = l0 - m;
    const int ll = i % nl, rest = i / nl, cs = rest & 1, k = rest >> 1;
    if ((cs == 1 && !HAS_S) || map0 + k >= nmaps) continue;
    vbase[(int64_t)leg_map(a, map0 + k) * vstride + cs * nsl + ll] = 0.0;
  }
  for (int lc = l0; lc <= L; lc += CH) {
    const int lend = lc + CH - 1;
    int ne = G.nx[0];
#pragma unroll
    for (int j = 1; j < R; ++j) ne = min(ne, G.nx[j]);
    const bool fast = ne > lend && lend <= L;
    // g of m is followed by g of m + 1 (and the table by 8 zeros), so the CH
    // values from lc are always in bounds; those past L go unused
    double gv[CH];
    cdouble* gp = gb + __builtin_amdgcn_readfirstlane(lc);
#pragma unroll
    for (int s = 0; s < CH; ++s) gv[s] = gp[s];
    double P[CH][NM][2];
    if (fast) {
      adj_chunk<NM, R, true, SQ, HAS_S>(G, E, O, gv, a, m, base, lane, lc, L, P);
    } else {
#pragma unroll
      for (int s = 0; s < CH; ++s)
#pragma unroll
        for (int k = 0; k < NM; ++k) P[s][k][0] = P[s][k][1] = 0.0;
      adj_chunk<NM, R, false, SQ, HAS_S>(G, E, O, gv, a, m, base, lane, lc, L, P);
    }
    // wave-private reduction of the 16 outputs u = (s NM + k) 2 + cs.  A
    // lane-swap step first sums lanes t and t + 32 (outputs u < 8 stay in the
    // lower half, u + 8 in the upper), so the LDS block wb[16][kRedStride]
    // holds 32 partials per output; four lanes then sum 8 columns each (the
    // column groups of lanes t and t ^ 16 are 16 apart: no bank conflicts)
    // and two more swap steps finish.
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int v = u + 8;
      const double h = fold32(P[u / (NM * 2)][(u >> 1) % NM][u & 1], P[v / (NM * 2)][(v >> 1) % NM][v & 1]);
      wb[(u + 8 * (lane >> 5)) * kRedStride + (lane & 31)] = h;
    }
    __builtin_amdgcn_wave_barrier();
    const int o = lane & 15, sub = lane >> 4;
    const double* wr = wb + o * kRedStride + 8 * (((sub & 1) << 1) | (sub >> 1));
    double acc = wr[0];
#pragma unroll
    for (int i = 1; i < 8; ++i) acc += wr[i];
    acc = add_xor16(acc);
    acc = add_xor32(acc);
    __builtin_amdgcn_wave_barrier();
    if (sub == 0) {
      const int s = o / (NM * 2), k = (o >> 1) % NM, cs = o & 1;
      const int l = lc + s;
      if (l <= L && map0 + k < nmaps && (HAS_S || cs == 0))
        vbase[(int64_t)leg_map(a, map0 + k) * vstride + cs * nsl + (l - m)] = acc;
    }
  }
}

template <int NM, int R, bool SQ>
__global__ __launch_bounds__(256) void k_leg_adjoint(LegArgs a, int nmaps, const double2* __restrict__ phase,
                                                     int64_t pstride, double* __restrict__ vpart,
                                                     int64_t vstride, int64_t tstride, int ntiles) {
  __shared__ double wbuf[4][AdjCfg<NM>::NOUT * kRedStride];
  int mb, tile;
  block_coords(ntiles, mb, tile);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = mb * 4 + wave;
  if (m > a.lmax) return;
  const int lane = threadIdx.x & 63;
  const int map0 = blockIdx.y * NM;
  const int ns = leg_nslots(a, nmaps);
  if (!leg_any(a, map0, NM, ns)) return;
  if (m == 0)
    adjoint_wave<NM, R, SQ, false>(a, m, tile, lane, ns, map0, phase, pstride, vpart, vstride, tstride, wbuf[wave]);
  else
    adjoint_wave<NM, R, SQ, true>(a, m, tile, lane, ns, map0, phase, pstride, vpart, vstride, tstride, wbuf[wave]);
}

// -------------------------------------------------------- adjoint, MFMA
// v_par[l][col] = sum_p lambda_lm(p) H_par(p)[col] as a dense product: rows =
// 16 values of l of one parity, K = ring pairs, N = 16 columns (8 maps x cos,
// sin).  One wave owns (m, T tiles of 64 ring pairs, 8 maps); lane t runs the
// recurrences of pair t of each tile and, tile after tile, writes each chunk
// of 32 steps [lb, lb + 32) (lb - m even) to wave-private LDS tiles lamE /
// lamO [64 pairs][16 steps of one parity]; K-block kb (pairs 4 kb .. 4 kb + 3)
// then feeds the MFMA with A lane (i, k) = lam_par[4 kb + k][i] and B lane
// (j, k) = H_par(4 kb + k)[j] (held in registers: T tiles x 16 K-blocks x
// E/O).  The T tiles accumulate into the same 16 x 16 results, the wave's
// partial v for 32 values of l: one partial per T tiles, T times less
// partial-sum traffic to and from HBM than one per tile.
template <int T>
__global__ __launch_bounds__(256) void k_leg_adjoint_mfma(LegArgs a, int nmaps, const double2* __restrict__ phase,
                                                          int64_t pstride, double* __restrict__ vpart,
                                                          int64_t vstride, int64_t tstride, int ntg) {
  // pair-major tiles per parity, lamE[pair][i] = lambda at l = lb + 2 i (O:
  // + 1), rows of 17 doubles: a lane group's A reads (16 consecutive i) and
  // the per-step writes (consecutive pairs, stride 17) are both conflict-free
  constexpr int RS = 17;
  __shared__ double lamsh[4][2 * 64 * RS];
  int mb, tg;
  block_coords(ntg, mb, tg);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = mb * 4 + wave;
  const int L = a.lmax;
  if (m > L) return;
  const int mg = blockIdx.y;
  const int ns = leg_nslots(a, nmaps);
  if (!leg_any(a, mg * 8, 8, ns)) return;
  double* lamE = lamsh[wave];
  double* lamO = lamE + 64 * RS;
  const int lane = threadIdx.x & 63;
  const int i16 = lane & 15, kq = lane >> 4;
  // this lane's column: map mg * 8 + j / 2, part j & 1
  const int j = i16;
  const int slot = mg * 8 + (j >> 1), cs = j & 1;
  const bool sok = slot < ns;
  const int map = sok ? leg_map(a, slot) : 0;
  const bool colok = sok && !(m == 0 && cs == 1);
  double z[T], a0[T], a1[T];
  double2 st[T];
  int ls[T], nx[T];
  // B operands: H_E, H_O of pair (tg T + t) 64 + 4 kb + kq in column j
  double HE[T][16], HO[T][16];
  int lfirst = INT_MAX;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int tile = tg * T + t;
    const int p = tile * 64 + lane;
    const bool valid = p < a.npairs;
    z[t] = valid ? a.zpair[p] : 0.0;
    ls[t] = valid ? a.ls[(size_t)m * a.npairs + p] : INT_MAX;
    st[t] = valid ? a.ms[(size_t)m * a.npairs + p] : make_double2(0.0, 0.0);
    a0[t] = a1[t] = 0.0;
    nx[t] = wave_min(ls[t]);
    lfirst = min(lfirst, nx[t]);
    const double* ph = reinterpret_cast<const double*>(phase + (int64_t)(colok ? map : 0) * pstride);
#pragma unroll
    for (int kb = 0; kb < 16; ++kb) {
      const int pp = tile * 64 + 4 * kb + kq;
      double hn = 0.0, hs = 0.0;
      const bool ok = colok && pp < a.npairs;
      const int rs = a.nring - 1 - pp;
      if (ok) {
        hn = ph[2 * ((int64_t)pp * (L + 1) + m) + cs];
        if (rs != pp) hs = ph[2 * ((int64_t)rs * (L + 1) + m) + cs];
      }
      // the equator ring is its own pair: lambda(z) H for both parities
      HE[t][kb] = (ok && rs == pp) ? hn : hn + hs;
      HO[t][kb] = (ok && rs == pp) ? hn : hn - hs;
    }
  }
  const int nsl = L - m + 1;
  double* const vb = vpart + (int64_t)tg * tstride + (int64_t)(colok ? map : 0) * vstride + moff(L, m) + cs * nsl - m;
  const int l0 = lfirst <= L ? lfirst - ((lfirst - m) & 1) : L + 1;
  // zero partial below the first evaluated l
  if (colok)
    for (int l = m + kq; l < l0; l += 4) vb[l] = 0.0;
  cdouble* gb = as_const(a.g + tri(L, m) - m);  // 8 zeros follow the table
  for (int lb = l0; lb <= L; lb += 32) {
    lb = __builtin_amdgcn_readfirstlane(lb);
    // two independent accumulator pairs (even / odd K-blocks)
    v4d DE2[2], DO2[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      DE2[v] = v4d{0.0, 0.0, 0.0, 0.0};
      DO2[v] = v4d{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const bool fast = nx[t] >= lb + 32;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // groups of 8 steps that start past L are not loaded (their rows are
        // never stored)
        double gv[8];
        cdouble* gp = gb + lb + 8 * q;
        const bool in = lb + 8 * q <= L;
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) gv[s2] = in ? gp[s2] : 0.0;
        if (fast) {
#pragma unroll
          for (int s2 = 0; s2 < 8; ++s2) {
            const double cc = fma(gv[s2] * z[t], a1[t], -a0[t]);
            a0[t] = a1[t];
            a1[t] = cc;
            ((s2 & 1) ? lamO : lamE)[lane * RS + 4 * q + (s2 >> 1)] = cc;
          }
        } else {
#pragma unroll
          for (int s2 = 0; s2 < 8; ++s2) {
            double cc = fma(gv[s2] * z[t], a1[t], -a0[t]);
            double pv = a1[t];
            if (ls[t] == lb + 8 * q + s2) {
              cc = st[t].y;
              pv = st[t].x;
            }
            a0[t] = pv;
            a1[t] = cc;
            ((s2 & 1) ? lamO : lamE)[lane * RS + 4 * q + (s2 >> 1)] = cc;
          }
        }
      }
      if (!fast) nx[t] = wave_min(ls[t] >= lb + 32 ? ls[t] : INT_MAX);
      lds_wave_sync();
#pragma unroll
      for (int kb = 0; kb < 16; ++kb) {
        const double aE = lamE[(4 * kb + kq) * RS + i16];
        const double aO = lamO[(4 * kb + kq) * RS + i16];
        DE2[kb & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aE, HE[t][kb], DE2[kb & 1], 0, 0, 0);
        DO2[kb & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aO, HO[t][kb], DO2[kb & 1], 0, 0, 0);
      }
      // the next tile's (or chunk's) steps overwrite lam only after these reads
      lds_wave_sync();
    }
    const v4d DE = DE2[0] + DE2[1];
    const v4d DO = DO2[0] + DO2[1];
    // D[row = kq + 4 r][col = j]: l = lb + 2 row (E), lb + 2 row + 1 (O)
    if (colok) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lE = lb + 2 * (kq + 4 * r);
        if (lE <= L) vb[lE] = DE[r];
        if (lE + 1 <= L) vb[lE + 1] = DO[r];
      }
    }
  }
}

// -------------------------------------------------------- hat scaling
// out[map][i] = c_m f_lm (or f_lm^2) * sum_t in[t][map][i]
__global__ void k_hat_scale(const double* __restrict__ f, int L, int nmaps,
                            const double* __restrict__ in, int64_t istride, int ntiles,
                            int64_t tstride, double* __restrict__ out, int64_t ostride, int square) {
  const int m = blockIdx.y;
  const int map = blockIdx.z;
  const int nsl = L - m + 1;
  const int np = (m == 0) ? 1 : 2;
  const int64_t mo = moff(L, m);
  const double cm = (m == 0 || square) ? 1.0 : 1.4142135623730951;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nsl * np; i += gridDim.x * blockDim.x) {
    const int ll = i % nsl;
    const double fv = f[tri(L, m) + ll];
    const double sc = square ? fv * fv : cm * fv;
    double acc = 0.0;
    for (int t = 0; t < ntiles; ++t) acc += in[(int64_t)t * tstride + (int64_t)map * istride + mo + i];
    out[(int64_t)map * ostride + mo + i] = sc * acc;
  }
}

}  // namespace

// ------------------------------------------------------------ launchers
// Default kernel choice (measured on MI355X, HEALPix Nside 64..1024):
// matrix-core kernels from 4 maps on; vector ring-pair groups per lane R as
// large as still leaves >= 4096 waves, up to 2 for synthesis (Nside 1024 /
// L 2000 / 1 map: 0.68 ms vs 0.75 ms at R = 1 and R = 4) and 4 for the adjoint
// (0.94 ms vs 1.28 ms at R = 2); two 64-pair tiles per matrix-core adjoint
// wave under the same wave count rule.
static int largest_r(int npairs, int L, int rmax, long want) {
  for (int R : {4, 2, 1}) {
    if (R > rmax) continue;
    const long tiles = (npairs + 64L * R - 1) / (64L * R);
    if ((long)(L + 1) * tiles >= want) return R;
  }
  return 1;
}

// Maps per wave of the vector synthesis: all of them up to 8, else the
// group size in {8, 6, 4} that leaves the fewest empty slots.
static int syn_nm(int nmaps) {
  if (nmaps <= 8) return nmaps;
  int best = 8, waste = 1 << 30;
  for (int c : {8, 6, 4}) {
    const int w = ((nmaps + c - 1) / c) * c - nmaps;
    if (w < waste) {
      waste = w;
      best = c;
    }
  }
  return best;
}

static int syn_rmax(int nmaps) { return std::max(1, 4 / syn_nm(nmaps)); }

static LegChoice default_choice(int npairs, int L, int nmaps) {
  LegChoice c;
  c.syn_mfma = c.adj_mfma = nmaps >= 4;
  c.syn_r = largest_r(npairs, L, std::min(2, syn_rmax(nmaps)), 4096);
  // the adjoint's per-chunk lane reduction wants more waves in flight: four
  // pairs per lane only from 8192 waves (Nside 512 / L 1024, one map: two
  // pairs per lane 0.169 ms, four 0.185 ms; Nside 1024 / L 2000: four 0.97,
  // two 1.03 ms)
  c.adj_r = largest_r(npairs, L, 4, 8192);
  const long nt = (npairs + 63) / 64;
  c.adj_t = (long)(L + 1) * ((nt + 1) / 2) * ((nmaps + 7) / 8) >= 4096 ? 2 : 1;
  return c;
}

static int env_int(const char* name) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : 0;
}

static void apply_env(LegChoice& c, int nmaps) {
  if (const int v = env_int("CRS_LEG_MFMA_MIN")) c.syn_mfma = c.adj_mfma = nmaps >= std::max(1, v);
  if (const int v = env_int("CRS_LEG_RS"))
    if (v == 1 || v == 2 || v == 4) c.syn_r = std::min(v, syn_rmax(nmaps));
  if (const int v = env_int("CRS_LEG_RA"))
    if (v == 1 || v == 2 || v == 4) c.adj_r = v;
  if (const int v = env_int("CRS_LEG_TA")) c.adj_t = v == 2 ? 2 : 1;
}

static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, LegChoice> g_tuned;  // (npairs, L, nmaps)

LegChoice leg_choice(int npairs, int L, int nmaps) {
  LegChoice c;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(npairs, L, nmaps));
    c = it != g_tuned.end() ? it->second : default_choice(npairs, L, nmaps);
  }
  apply_env(c, nmaps);
  return c;
}

void launch_leg_synth(const LegChoice& c, const LegArgs& a, int nmaps, const double* uhat, int64_t ustride,
                      double2* phase, int64_t pstride, hipStream_t s) {
  const int L = a.lmax;
  if (c.syn_mfma) {
    const int ntiles = (a.npairs + 63) / 64;
    const int nmb = (L + 1 + 3) / 4;
    const int nmb8 = (nmb + 7) / 8 * 8;
    dim3 grid(nmb8 * ntiles, (nmaps + 7) / 8);
    hipLaunchKernelGGL(k_leg_synth_mfma, grid, dim3(256), 0, s, a, nmaps, uhat, ustride, phase, pstride, ntiles);
    CRS_HIP(hipGetLastError());
    return;
  }
  const int nm = syn_nm(nmaps);
  const int R = std::min(c.syn_r, syn_rmax(nmaps));
  const int ntiles = (a.npairs + 64 * R - 1) / (64 * R);
  const int nmb = (L + 1 + 3) / 4;
  const int nmb8 = (nmb + 7) / 8 * 8;
  dim3 grid(nmb8 * ntiles, (nmaps + nm - 1) / nm);
  dim3 block(256);
#define CRS_SYN(N, RR) \
  if (nm == N && R == RR) { hipLaunchKernelGGL((k_leg_synth<N, RR>), grid, block, 0, s, a, nmaps, uhat, ustride, phase, pstride, ntiles); CRS_HIP(hipGetLastError()); return; }
  CRS_SYN(1, 1) CRS_SYN(1, 2) CRS_SYN(1, 4)
  CRS_SYN(2, 1) CRS_SYN(2, 2)
  CRS_SYN(3, 1) CRS_SYN(4, 1) CRS_SYN(5, 1) CRS_SYN(6, 1) CRS_SYN(7, 1) CRS_SYN(8, 1)
#undef CRS_SYN
  throw Error{CRS_EINVAL, "no synthesis kernel variant"};
}

// Vector adjoint: R is chosen first and the maps per wave follow (R * NM <= 8).
static int adj_nm(int nmaps, int R) {
  const int cap = 8 / R;
  const int nm = nmaps >= 4 ? 4 : (nmaps >= 2 ? 2 : 1);
  return std::min(nm, cap);
}

int leg_adjoint_tiles(const LegChoice& c, int npairs, bool square) {
  if (c.adj_mfma && !square) return ((npairs + 63) / 64 + c.adj_t - 1) / c.adj_t;
  return (npairs + 64 * c.adj_r - 1) / (64 * c.adj_r);
}

void launch_leg_adjoint(const LegChoice& c, const LegArgs& a, int nmaps, const double2* phase, int64_t pstride,
                        double* vpart, int64_t vstride, int64_t tstride, bool square,
                        hipStream_t s) {
  const int L = a.lmax;
  const int ntg = leg_adjoint_tiles(c, a.npairs, square);
  const int nmb = (L + 1 + 3) / 4;
  const int nmb8 = (nmb + 7) / 8 * 8;
  if (c.adj_mfma && !square) {
    dim3 grid(nmb8 * ntg, (nmaps + 7) / 8);
    if (c.adj_t == 2)
      hipLaunchKernelGGL(k_leg_adjoint_mfma<2>, grid, dim3(256), 0, s, a, nmaps, phase, pstride, vpart, vstride,
                         tstride, ntg);
    else
      hipLaunchKernelGGL(k_leg_adjoint_mfma<1>, grid, dim3(256), 0, s, a, nmaps, phase, pstride, vpart, vstride,
                         tstride, ntg);
    CRS_HIP(hipGetLastError());
    return;
  }
  const int R = c.adj_r;
  const int nm = adj_nm(nmaps, R);
  dim3 grid(nmb8 * ntg, (nmaps + nm - 1) / nm);
#define CRS_ADJ(N, RR)                                                                            \
  if (nm == N && R == RR) {                                                                       \
    if (square)                                                                                   \
      hipLaunchKernelGGL((k_leg_adjoint<N, RR, true>), grid, dim3(256), 0, s, a, nmaps, phase,    \
                         pstride, vpart, vstride, tstride, ntg);                                  \
    else                                                                                          \
      hipLaunchKernelGGL((k_leg_adjoint<N, RR, false>), grid, dim3(256), 0, s, a, nmaps, phase,   \
                         pstride, vpart, vstride, tstride, ntg);                                  \
    CRS_HIP(hipGetLastError());                                                                   \
    return;                                                                                       \
  }
  CRS_ADJ(1, 1) CRS_ADJ(1, 2) CRS_ADJ(1, 4)
  CRS_ADJ(2, 1) CRS_ADJ(2, 2) CRS_ADJ(2, 4)
  CRS_ADJ(4, 1) CRS_ADJ(4, 2)
#undef CRS_ADJ
  throw Error{CRS_EINVAL, "no adjoint kernel variant"};
}

// ------------------------------------------------------------ autotuner
// Average time of `reps` launches after one warm-up, with HIP events on s.
template <class F>
static float time_launches(F&& launch, int reps, hipStream_t s) {
  launch();
  hipEvent_t e0, e1;
  CRS_HIP(hipEventCreate(&e0));
  CRS_HIP(hipEventCreate(&e1));
  CRS_HIP(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i) launch();
  CRS_HIP(hipEventRecord(e1, s));
  CRS_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  CRS_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

LegChoice leg_autotune(const LegArgs& a0, int nmaps, double* uhat, double2* phase, hipStream_t s) {
  LegArgs a = a0;
  a.skip = MapSkip{};
  const int L = a.lmax;
  const int64_t nalm = (int64_t)(L + 1) * (L + 1);
  const int64_t pst = (int64_t)a.nring * (L + 1);
  const LegChoice base = default_choice(a.npairs, L, nmaps);
  // the largest tile count of any candidate (one 64-pair tile per wave)
  DevBuf<double> vpart;
  vpart.alloc((size_t)((a.npairs + 63) / 64) * nmaps * nalm);
  CRS_HIP(hipMemsetAsync(uhat, 0, (size_t)nmaps * nalm * sizeof(double), s));
  CRS_HIP(hipMemsetAsync(phase, 0, (size_t)nmaps * pst * sizeof(double2), s));
  const int reps = 3;
  LegChoice best = base;
  float tbest = 1e30f;
  auto try_syn = [&](LegChoice c) {
    const float t = time_launches([&] { launch_leg_synth(c, a, nmaps, uhat, nalm, phase, pst, s); }, reps, s);
    if (t < tbest) {
      tbest = t;
      best.syn_mfma = c.syn_mfma;
      best.syn_r = c.syn_r;
    }
  };
  for (int r : {1, 2, 4}) {
    if (r > syn_rmax(nmaps)) continue;
    LegChoice c = base;
    c.syn_mfma = 0;
    c.syn_r = r;
    try_syn(c);
  }
  if (nmaps >= 2) {
    LegChoice c = base;
    c.syn_mfma = 1;
    try_syn(c);
  }
  tbest = 1e30f;
  auto try_adj = [&](LegChoice c) {
    const float t = time_launches([&] {
      launch_leg_adjoint(c, a, nmaps, phase, pst, vpart.p, nalm, (int64_t)nmaps * nalm, false, s);
    }, reps, s);
    if (t < tbest) {
      tbest = t;
      best.adj_mfma = c.adj_mfma;
      best.adj_r = c.adj_r;
      best.adj_t = c.adj_t;
    }
  };
  for (int r : {1, 2, 4}) {
    LegChoice c = base;
    c.adj_mfma = 0;
    c.adj_r = r;
    try_adj(c);
  }
  if (nmaps >= 2)
    for (int t : {1, 2}) {
      LegChoice c = base;
      c.adj_mfma = 1;
      c.adj_t = t;
      try_adj(c);
    }
  CRS_HIP(hipStreamSynchronize(s));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(a.npairs, L, nmaps)] = best;
  }
  // the environment overrides apply to a tuned choice as to the default one
  apply_env(best, nmaps);
  return best;
}

namespace {
__global__ void k_tile_sum(const double* __restrict__ hs, int64_t nalm, const double* __restrict__ in,
                           int64_t istride, int ntiles, int64_t tstride, double* __restrict__ out,
                           int64_t ostride) {
  const int map = blockIdx.y;
  const double* __restrict__ src = in + (int64_t)map * istride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nalm; i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int t = 0; t < ntiles; ++t) acc += src[(int64_t)t * tstride + i];
    out[(int64_t)map * ostride + i] = hs[i] * acc;
  }
}
}  // namespace

void launch_tile_sum(const double* hs, int64_t nalm, int nmaps, const double* in, int64_t istride,
                     int ntiles, int64_t tstride, double* out, int64_t ostride, hipStream_t s) {
  const int64_t nb = std::min<int64_t>((nalm + 255) / 256, 4096);
  hipLaunchKernelGGL(k_tile_sum, dim3((unsigned)nb, nmaps), dim3(256), 0, s, hs, nalm, in, istride, ntiles, tstride,
                     out, ostride);
  CRS_HIP(hipGetLastError());
}

void launch_hat_scale(const double* f, int lmax, int nmaps, const double* in, int64_t istride,
                      int ntiles, int64_t tstride, double* out, int64_t ostride, bool square,
                      hipStream_t s) {
  dim3 grid((2 * (lmax + 1) + 255) / 256, lmax + 1, nmaps);
  hipLaunchKernelGGL(k_hat_scale, grid, dim3(256), 0, s, f, lmax, nmaps, in, istride, ntiles,
                     tstride, out, ostride, square ? 1 : 0);
  CRS_HIP(hipGetLastError());
}

}  // namespace crs
