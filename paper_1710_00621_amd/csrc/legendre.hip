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

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return __builtin_amdgcn_readfirstlane(v);
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
// recurrence state and two wave-uniform numbers: lw (first l any lane of the
// group evaluates, forced non-increasing in j so that the groups running at
// a given l are a suffix j >= q) and nx (next l where some lane of the group
// starts).  Between start events all running groups step in lockstep.
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

// first running group at l (lw[R-1] <= l is required)
template <int R>
__device__ __forceinline__ int grp_first(const Grp<R>& G, int l) {
  int q = R - 1;
#pragma unroll
  for (int j = R - 1; j >= 0; --j)
    if (G.lw[j] <= l) q = j;
  return q;
}

template <int R>
__device__ __forceinline__ int grp_next_event(const Grp<R>& G, int q) {
  int ne = INT_MAX;
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (j >= q) ne = min(ne, G.nx[j]);
  return ne;
}

template <int R>
__device__ __forceinline__ int grp_next_start(const Grp<R>& G, int q, int L) {
  int pe = L + 1;
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (j == q - 1) pe = G.lw[j];
  return pe;
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

// one step for groups J0..R-1 into X (no swap)
template <int NM, int R, int J0, bool HAS_S>
__device__ __forceinline__ void syn_acc(SynAcc<NM, R>& A, Grp<R>& G, double gl, const double* uc,
                                        const double* us) {
#pragma unroll
  for (int j = J0; j < R; ++j) {
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

template <int NM, int R, int NA, bool HAS_S>
__device__ __forceinline__ void syn_plain(SynAcc<NM, R>& A, Grp<R>& G, cdouble* gb, cdouble* const* ub,
                                          int nsl, int l, int stop) {
  constexpr int J0 = R - NA;
  constexpr int B = (NM == 1) ? 8 : ((NM == 2) ? 4 : 2);
  for (; l + B <= stop; l += B) {
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
      syn_acc<NM, R, J0, HAS_S>(A, G, gv[i], uc[i], us[i]);
      syn_swap<NM, R>(A);
    }
  }
  for (; l < stop; ++l) {
    double uc[NM], us[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      uc[k] = uld(ub[k], l);
      us[k] = HAS_S ? uld(ub[k], l + nsl) : 0.0;
    }
    syn_acc<NM, R, J0, HAS_S>(A, G, uld(gb, l), uc, us);
    syn_swap<NM, R>(A);
  }
}

template <int NM, int R, int NA, bool HAS_S>
__device__ __forceinline__ void syn_event(SynAcc<NM, R>& A, Grp<R>& G, const LegArgs& a, int m, int base,
                                          int lane, cdouble* gb, cdouble* const* ub, int nsl, int l) {
  constexpr int J0 = R - NA;
  const double gl = uld(gb, l);
  double uc[NM], us[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    uc[k] = uld(ub[k], l);
    us[k] = HAS_S ? uld(ub[k], l + nsl) : 0.0;
  }
#pragma unroll
  for (int j = J0; j < R; ++j) {
    const double c = grp_event_step<R>(G, j, a, m, base, lane, l, gl);
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      A.X[j][k][0] = fma(c, uc[k], A.X[j][k][0]);
      if (HAS_S) A.X[j][k][1] = fma(c, us[k], A.X[j][k][1]);
    }
  }
  syn_swap<NM, R>(A);
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
    ub[k] = as_const(uhat + (int64_t)min(map0 + k, nmaps - 1) * ustride + moff(L, m) - m);
  Grp<R> G;
  grp_init<R>(G, a, m, base, lane);
  SynAcc<NM, R> A;
#pragma unroll
  for (int j = 0; j < R; ++j)
#pragma unroll
    for (int k = 0; k < NM; ++k) A.X[j][k][0] = A.X[j][k][1] = A.Y[j][k][0] = A.Y[j][k][1] = 0.0;
  int l = G.lw[R - 1];
  while (l <= L) {
    const int q = grp_first<R>(G, l);
    const int ne = grp_next_event<R>(G, q);
    if (ne == l) {
      switch (R - q) {
#define SYN_EV(NA) case NA: if (NA <= R) syn_event<NM, R, (NA <= R ? NA : R), HAS_S>(A, G, a, m, base, lane, gb, ub, nsl, l); break;
        SYN_EV(1) SYN_EV(2) SYN_EV(3) SYN_EV(4)
#undef SYN_EV
      }
      ++l;
      continue;
    }
    const int stop = min(min(grp_next_start<R>(G, q, L), ne), L + 1);
    switch (R - q) {
#define SYN_PL(NA) case NA: if (NA <= R) syn_plain<NM, R, (NA <= R ? NA : R), HAS_S>(A, G, gb, ub, nsl, l, stop); break;
      SYN_PL(1) SYN_PL(2) SYN_PL(3) SYN_PL(4)
#undef SYN_PL
    }
    l = stop;
  }
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
        double2* ph = phase + (int64_t)(map0 + k) * pstride;
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
  if (a.skip.act) {
    bool any = false;
    for (int k = 0; k < NM && map0 + k < nmaps; ++k) any = any || !a.skip.off(map0 + k);
    if (!any) return;
  }
  if (m == 0)
    synth_wave<NM, R, false>(a, m, base, lane, nmaps, map0, uhat, ustride, phase, pstride);
  else
    synth_wave<NM, R, true>(a, m, base, lane, nmaps, map0, uhat, ustride, phase, pstride);
}

// --------------------------------------------------------------- adjoint
// Same wave decomposition.  Per l every lane sums its groups' products into
// P[s]; each chunk of CH steps is reduced over the wave's 64 lanes through a
// wave-private LDS block (no block barrier) in a fixed order and written as
// the wave's partial v^ (one partial per ring tile of 64 R pairs).
template <int NM>
struct AdjCfg {
  static constexpr int CH = (8 / NM) < 1 ? 1 : (8 / NM);
  static constexpr int NOUT = CH * NM * 2;
};

template <int NM, int R, int NA, bool FAST, bool ODD0, bool SQ, bool HAS_S>
__device__ __forceinline__ void adj_chunk(Grp<R>& G, const double (&E)[R][NM][2], const double (&O)[R][NM][2],
                                          const double (&gv)[AdjCfg<NM>::CH], const LegArgs& a, int m,
                                          int base, int lane, int lc, int L,
                                          double (&P)[AdjCfg<NM>::CH][NM][2]) {
  constexpr int CH = AdjCfg<NM>::CH;
  constexpr int J0 = R - NA;
#pragma unroll
  for (int s = 0; s < CH; ++s) {
    const int l = lc + s;
    if (l > L) break;
    const bool odd = ODD0 ^ ((s & 1) != 0);
#pragma unroll
    for (int j = J0; j < R; ++j) {
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
        P[s][k][0] = fma(w, (SQ || !odd) ? E[j][k][0] : O[j][k][0], P[s][k][0]);
        if (HAS_S) P[s][k][1] = fma(w, (SQ || !odd) ? E[j][k][1] : O[j][k][1], P[s][k][1]);
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
      const double2* ph = phase + (int64_t)min(map0 + k, nmaps - 1) * pstride;
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
  int l0 = G.lw[R - 1];
  if (l0 < m) l0 = m;
  if (l0 > L + 1) l0 = L + 1;
  // zero-fill this tile's output below the first evaluated l
  for (int i = lane; i < (l0 - m) * NM * 2; i += 64) {
    const int nl = l0 - m;
    const int ll = i % nl, rest = i / nl, cs = rest & 1, k = rest >> 1;
    if ((cs == 1 && !HAS_S) || map0 + k >= nmaps) continue;
    vbase[(int64_t)(map0 + k) * vstride + cs * nsl + ll] = 0.0;
  }
  for (int lc = l0; lc <= L; lc += CH) {
    const int lend = min(lc + CH - 1, L);
    const int q = grp_first<R>(G, lend);
    const bool fast = grp_next_event<R>(G, q) > lend;
    const bool odd0 = ((lc - m) & 1) != 0;
    double gv[CH];
    cdouble* gp = gb + __builtin_amdgcn_readfirstlane(lc);
#pragma unroll
    for (int s = 0; s < CH; ++s) gv[s] = (lc + s <= L) ? gp[s] : 0.0;
    double P[CH][NM][2];
#pragma unroll
    for (int s = 0; s < CH; ++s)
#pragma unroll
      for (int k = 0; k < NM; ++k) P[s][k][0] = P[s][k][1] = 0.0;
#define ADJ_CASE(NA)                                                                                  \
  case NA:                                                                                            \
    if (NA <= R) {                                                                                    \
      constexpr int NAc = NA <= R ? NA : R;                                                           \
      if (fast) {                                                                                     \
        if (odd0) adj_chunk<NM, R, NAc, true, true, SQ, HAS_S>(G, E, O, gv, a, m, base, lane, lc, L, P);   \
        else adj_chunk<NM, R, NAc, true, false, SQ, HAS_S>(G, E, O, gv, a, m, base, lane, lc, L, P);       \
      } else {                                                                                        \
        if (odd0) adj_chunk<NM, R, NAc, false, true, SQ, HAS_S>(G, E, O, gv, a, m, base, lane, lc, L, P);  \
        else adj_chunk<NM, R, NAc, false, false, SQ, HAS_S>(G, E, O, gv, a, m, base, lane, lc, L, P);      \
      }                                                                                               \
    }                                                                                                 \
    break;
    switch (R - q) { ADJ_CASE(1) ADJ_CASE(2) ADJ_CASE(3) ADJ_CASE(4) }
#undef ADJ_CASE
    // wave-private reduction: wb is [NOUT][65]
#pragma unroll
    for (int s = 0; s < CH; ++s)
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        wb[((s * NM + k) * 2 + 0) * 65 + lane] = P[s][k][0];
        wb[((s * NM + k) * 2 + 1) * 65 + lane] = P[s][k][1];
      }
    __builtin_amdgcn_wave_barrier();
    const int o = lane & 15, sub = lane >> 4;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc += wb[o * 65 + sub + 4 * i];
    acc += __shfl_xor(acc, 16, 64);
    acc += __shfl_xor(acc, 32, 64);
    __builtin_amdgcn_wave_barrier();
    if (sub == 0) {
      const int s = o / (NM * 2), k = (o >> 1) % NM, cs = o & 1;
      const int l = lc + s;
      if (l <= L && map0 + k < nmaps && (HAS_S || cs == 0))
        vbase[(int64_t)(map0 + k) * vstride + cs * nsl + (l - m)] = acc;
    }
  }
}

template <int NM, int R, bool SQ>
__global__ __launch_bounds__(256) void k_leg_adjoint(LegArgs a, int nmaps, const double2* __restrict__ phase,
                                                     int64_t pstride, double* __restrict__ vpart,
                                                     int64_t vstride, int64_t tstride, int ntiles) {
  __shared__ double wbuf[4][AdjCfg<NM>::NOUT * 65];
  int mb, tile;
  block_coords(ntiles, mb, tile);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = mb * 4 + wave;
  if (m > a.lmax) return;
  const int lane = threadIdx.x & 63;
  const int map0 = blockIdx.y * NM;
  if (a.skip.act) {
    bool any = false;
    for (int k = 0; k < NM && map0 + k < nmaps; ++k) any = any || !a.skip.off(map0 + k);
    if (!any) return;
  }
  if (m == 0)
    adjoint_wave<NM, R, SQ, false>(a, m, tile, lane, nmaps, map0, phase, pstride, vpart, vstride, tstride, wbuf[wave]);
  else
    adjoint_wave<NM, R, SQ, true>(a, m, tile, lane, nmaps, map0, phase, pstride, vpart, vstride, tstride, wbuf[wave]);
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
// Ring-pair groups per lane: larger R amortises the scalar coefficient
// loads and the adjoint's cross-lane reduction over more pairs, smaller R
// gives more waves.  Take the largest R (up to rmax) that still leaves
// `want` waves in the launch.  Measured on MI355X (HEALPix Nside 64..1024):
// synthesis is fastest at R = 1 throughout, the adjoint at R = 2 once that
// leaves >= 4096 waves.  The environment variables CRS_LEG_RS and
// CRS_LEG_RA fix R for synthesis and adjoint (tuning).
static int pick_r(int npairs, int L, int rmax, long want, const char* env) {
  if (const char* e = std::getenv(env)) {
    const int r = std::atoi(e);
    if (r == 1 || r == 2 || r == 4) return std::min(r, rmax);
  }
  for (int R : {4, 2, 1}) {
    if (R > rmax) continue;
    const long tiles = (npairs + 64L * R - 1) / (64L * R);
    const long waves = (long)(L + 1) * tiles;
    if (waves >= want) return R;
  }
  return 1;
}

static int syn_nm(int nmaps) {
  if (nmaps <= 8) return nmaps;
  int best = 8, waste = 1 << 30;
  for (int c : {8, 6, 4}) {
    const int w = ((nmaps + c - 1) / c) * c - nmaps;
    if (w < waste) { waste = w; best = c; }
  }
  return best;
}

void launch_leg_synth(const LegArgs& a, int nmaps, const double* uhat, int64_t ustride,
                      double2* phase, int64_t pstride, hipStream_t s) {
  const int L = a.lmax;
  const int nm = syn_nm(nmaps);
  const int R = pick_r(a.npairs, L, std::max(1, 4 / nm), 1L << 40, "CRS_LEG_RS");
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

// The adjoint's ring tile count depends on (npairs, L) only, so that the
// partial-sum buffers and their consumers do not depend on the map count:
// R is chosen first and the maps per wave follow (R * NM <= 8).
static int adj_r(int npairs, int L) { return pick_r(npairs, L, 2, 4096, "CRS_LEG_RA"); }

static int adj_nm(int nmaps, int R) {
  const int cap = 8 / R;
  const int nm = nmaps >= 4 ? 4 : (nmaps >= 2 ? 2 : 1);
  return std::min(nm, cap);
}

int leg_adjoint_tiles(int npairs, int L) {
  const int R = adj_r(npairs, L);
  return (npairs + 64 * R - 1) / (64 * R);
}

void launch_leg_adjoint(const LegArgs& a, int nmaps, const double2* phase, int64_t pstride,
                        double* vpart, int64_t vstride, int64_t tstride, bool square,
                        hipStream_t s) {
  const int L = a.lmax;
  const int R = adj_r(a.npairs, L);
  const int nm = adj_nm(nmaps, R);
  const int ntiles = (a.npairs + 64 * R - 1) / (64 * R);
  const int nmb = (L + 1 + 3) / 4;
  const int nmb8 = (nmb + 7) / 8 * 8;
  dim3 grid(nmb8 * ntiles, (nmaps + nm - 1) / nm);
#define CRS_ADJ(N, RR)                                                                            \
  if (nm == N && R == RR) {                                                                       \
    if (square)                                                                                   \
      hipLaunchKernelGGL((k_leg_adjoint<N, RR, true>), grid, dim3(256), 0, s, a, nmaps, phase,    \
                         pstride, vpart, vstride, tstride, ntiles);                               \
    else                                                                                          \
      hipLaunchKernelGGL((k_leg_adjoint<N, RR, false>), grid, dim3(256), 0, s, a, nmaps, phase,   \
                         pstride, vpart, vstride, tstride, ntiles);                               \
    CRS_HIP(hipGetLastError());                                                                   \
    return;                                                                                       \
  }
  CRS_ADJ(1, 1) CRS_ADJ(1, 2) CRS_ADJ(1, 4)
  CRS_ADJ(2, 1) CRS_ADJ(2, 2) CRS_ADJ(2, 4)
  CRS_ADJ(4, 1) CRS_ADJ(4, 2)
#undef CRS_ADJ
  throw Error{CRS_EINVAL, "no adjoint kernel variant"};
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
