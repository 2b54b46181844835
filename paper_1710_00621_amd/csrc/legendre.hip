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
#include <climits>

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

// ------------------------------------------------------------- synthesis
template <int NM, bool HAS_S>
__device__ __forceinline__ void synth_body(const LegArgs& a, int m, int p, bool valid, int nmaps,
                                           int map0, const double* __restrict__ uhat,
                                           int64_t ustride, double2* __restrict__ phase,
                                           int64_t pstride) {
  const int L = a.lmax;
  const int pc = valid ? p : a.npairs - 1;
  const double z = a.zpair[pc];
  const int ls = valid ? a.ls[(size_t)m * a.npairs + p] : INT_MAX;
  const double2 ms = valid ? a.ms[(size_t)m * a.npairs + p] : make_double2(0.0, 0.0);
  cdouble* gb = as_const(a.g + tri(L, m) - m);
  const int nsl = L - m + 1;
  cdouble* ub[NM];
#pragma unroll
  for (int j = 0; j < NM; ++j) {
    int mj = min(map0 + j, nmaps - 1);
    ub[j] = as_const(uhat + (int64_t)mj * ustride + moff(L, m) - m);
  }
  double Ec[NM], Es[NM], Oc[NM], Os[NM];
#pragma unroll
  for (int j = 0; j < NM; ++j) Ec[j] = Es[j] = Oc[j] = Os[j] = 0.0;

  int l = wave_min(ls);
  if (l <= L) {
    double a0 = 0.0, a1 = 0.0;  // mu_{l-2}, mu_{l-1}
    int next = l;
    auto accE = [&](double c, int ll) {
#pragma unroll
      for (int j = 0; j < NM; ++j) {
        Ec[j] = fma(c, uld(ub[j], ll), Ec[j]);
        if (HAS_S) Es[j] = fma(c, uld(ub[j], ll + nsl), Es[j]);
      }
    };
    auto accO = [&](double c, int ll) {
#pragma unroll
      for (int j = 0; j < NM; ++j) {
        Oc[j] = fma(c, uld(ub[j], ll), Oc[j]);
        if (HAS_S) Os[j] = fma(c, uld(ub[j], ll + nsl), Os[j]);
      }
    };
    while (l <= L) {
      if (l == next) {
        double c = fma(uld(gb, l) * z, a1, -a0);
        const bool inj = (ls == l);
        c = inj ? ms.y : c;
        const double pv = inj ? ms.x : a1;
        if ((l - m) & 1) accO(c, l); else accE(c, l);
        a0 = pv;
        a1 = c;
        ++l;
        next = wave_min(ls >= l ? ls : INT_MAX);
        continue;
      }
      const int stop = min(next, L + 1);
      if (((l - m) & 1) && l < stop) {
        double c = fma(uld(gb, l) * z, a1, -a0);
        accO(c, l);
        a0 = a1;
        a1 = c;
        ++l;
      }
      // blocks of B steps starting at even l - m; coefficients of a block are
      // fetched with a few wide scalar loads before the block's arithmetic
      constexpr int B = (NM == 1) ? 8 : ((NM == 2) ? 4 : 2);
      for (; l + B <= stop; l += B) {
        l = __builtin_amdgcn_readfirstlane(l);
        cdouble* gp = gb + l;
        double gv[B], uc[NM][B], us[NM][B];
#pragma unroll
        for (int i = 0; i < B; ++i) gv[i] = gp[i];
#pragma unroll
        for (int j = 0; j < NM; ++j) {
          cdouble* up = ub[j] + l;
#pragma unroll
          for (int i = 0; i < B; ++i) {
            uc[j][i] = up[i];
            us[j][i] = HAS_S ? up[i + nsl] : 0.0;
          }
        }
#pragma unroll
        for (int i = 0; i < B; ++i) {
          const double c = fma(gv[i] * z, a1, -a0);
          a0 = a1;
          a1 = c;
#pragma unroll
          for (int j = 0; j < NM; ++j) {
            if (i & 1) {
              Oc[j] = fma(c, uc[j][i], Oc[j]);
              if (HAS_S) Os[j] = fma(c, us[j][i], Os[j]);
            } else {
              Ec[j] = fma(c, uc[j][i], Ec[j]);
              if (HAS_S) Es[j] = fma(c, us[j][i], Es[j]);
            }
          }
        }
      }
      for (; l < stop; ++l) {
        double c = fma(uld(gb, l) * z, a1, -a0);
        if ((l - m) & 1) accO(c, l); else accE(c, l);
        a0 = a1;
        a1 = c;
      }
    }
  }
  if (!valid) return;
  const int rs = a.nring - 1 - p;
#pragma unroll
  for (int j = 0; j < NM; ++j) {
    if (map0 + j >= nmaps) break;
    double2* ph = phase + (int64_t)(map0 + j) * pstride;
    ph[(int64_t)p * (L + 1) + m] = make_double2(Ec[j] + Oc[j], Es[j] + Os[j]);
    if (rs != p) ph[(int64_t)rs * (L + 1) + m] = make_double2(Ec[j] - Oc[j], Es[j] - Os[j]);
  }
}

template <int NM>
__global__ __launch_bounds__(256) void k_leg_synth(LegArgs a, int nmaps, const double* __restrict__ uhat,
                                                   int64_t ustride, double2* __restrict__ phase,
                                                   int64_t pstride, int ntiles) {
  // XCD-aware order: the 8 XCDs take blocks round-robin; consecutive blocks
  // on one XCD share an m-block (same harmonic coefficients, one L2), and
  // small m (the longest recurrences) are dispatched first.
  const int b = blockIdx.x;
  const int xcd = b & 7, q = b >> 3;
  const int tile = q % ntiles;
  const int mb = (q / ntiles) * 8 + xcd;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = mb * 4 + wave;
  if (m > a.lmax) return;
  const int p = tile * 64 + (threadIdx.x & 63);
  const bool valid = p < a.npairs;
  const int map0 = blockIdx.y * NM;
  if (m == 0)
    synth_body<NM, false>(a, m, p, valid, nmaps, map0, uhat, ustride, phase, pstride);
  else
    synth_body<NM, true>(a, m, p, valid, nmaps, map0, uhat, ustride, phase, pstride);
}

// --------------------------------------------------------------- adjoint
// Block: one m, 256 lanes, R adjacent ring pairs per lane (pair = tile*256R + tid*R + j).
// Per l each lane sums its R products; the 256 lane sums are reduced through
// LDS every CH steps (fixed order, deterministic) and written as the tile's
// partial v^.
template <int NM, int R, int CH, bool SQ, bool HAS_S, bool ODD0>
__device__ __forceinline__ void adj_chunk_fast(cdouble* gb, int lc, int L,
                                               const double (&z)[R], double (&a0)[R], double (&a1)[R],
                                               const double (&E)[R][NM][2], const double (&O)[R][NM][2],
                                               double (&P)[CH][NM][2]) {
  double gv[CH];
  cdouble* gp = gb + __builtin_amdgcn_readfirstlane(lc);
#pragma unroll
  for (int s = 0; s < CH; ++s) gv[s] = (lc + s <= L) ? gp[s] : 0.0;
#pragma unroll
  for (int s = 0; s < CH; ++s) {
    const int l = lc + s;
    if (l > L) break;
    const double gl = gv[s];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      double c = fma(gl * z[j], a1[j], -a0[j]);
      a0[j] = a1[j];
      a1[j] = c;
      const bool odd = ODD0 ^ (s & 1);
      const double w = SQ ? c * c : c;
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        const double hc = (SQ || !odd) ? E[j][k][0] : O[j][k][0];
        P[s][k][0] = fma(w, hc, P[s][k][0]);
        if (HAS_S) {
          const double hs = (SQ || !odd) ? E[j][k][1] : O[j][k][1];
          P[s][k][1] = fma(w, hs, P[s][k][1]);
        }
      }
    }
  }
}

template <int NM>
struct AdjShared {
  static constexpr int CH = (8 / NM) < 1 ? 1 : (8 / NM);
  static constexpr int NOUT = CH * NM * 2;
  double buf[NOUT][257];
  double red[4][NOUT];
  int smin[4];
};

template <int NM, int R, bool SQ, bool HAS_S>
__device__ __forceinline__ void adjoint_body(const LegArgs& a, int m, int tile, int map0, int nmaps,
                                             const double2* __restrict__ phase, int64_t pstride,
                                             double* __restrict__ vpart, int64_t vstride,
                                             int64_t tstride, AdjShared<NM>& sh) {
  constexpr int CH = AdjShared<NM>::CH;
  constexpr int NOUT = AdjShared<NM>::NOUT;
  static_assert(NOUT <= 64 && (NOUT & (NOUT - 1)) == 0, "NOUT must be a power of two <= 64");
  auto& buf = sh.buf;
  auto& red = sh.red;
  auto& smin = sh.smin;
  const int L = a.lmax;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  cdouble* gb = as_const(a.g + tri(L, m) - m);

  double z[R], a0[R], a1[R];
  double E[R][NM][2], O[R][NM][2];
  int lw[R], nx[R];
  const int pbase = tile * 256 * R + tid * R;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int p = pbase + j;
    const bool valid = p < a.npairs;
    const int pc = valid ? p : a.npairs - 1;
    z[j] = a.zpair[pc];
    const int lsj = valid ? a.ls[(size_t)m * a.npairs + p] : INT_MAX;
    const int rs = a.nring - 1 - pc;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int mk = min(map0 + k, nmaps - 1);
      const double2* ph = phase + (int64_t)mk * pstride;
      double2 hn = valid ? ph[(int64_t)pc * (L + 1) + m] : make_double2(0.0, 0.0);
      double2 hs = (valid && rs != pc) ? ph[(int64_t)rs * (L + 1) + m] : make_double2(0.0, 0.0);
      if (valid && rs == pc) {
        // equator ring: its own pair, lambda(z) H for both parities
        E[j][k][0] = hn.x; E[j][k][1] = hn.y;
        O[j][k][0] = SQ ? 0.0 : hn.x; O[j][k][1] = SQ ? 0.0 : hn.y;
      } else {
        E[j][k][0] = hn.x + hs.x; E[j][k][1] = hn.y + hs.y;
        O[j][k][0] = hn.x - hs.x; O[j][k][1] = hn.y - hs.y;
      }
    }
    a0[j] = 0.0;
    a1[j] = 0.0;
    lw[j] = wave_min(lsj);
    nx[j] = lw[j];
  }
  int lwm = INT_MAX;
#pragma unroll
  for (int j = 0; j < R; ++j) lwm = min(lwm, lw[j]);
  if ((tid & 63) == 0) smin[wave] = lwm;
  __syncthreads();
  int l0 = min(min(smin[0], smin[1]), min(smin[2], smin[3]));
  l0 = max(l0, m);
  if (l0 > L + 1) l0 = L + 1;
  // zero-fill the part of this tile's output that no ring reaches
  {
    const int nl = l0 - m;
    const int nsl = L - m + 1;
    for (int i = tid; i < nl * NM * 2; i += 256) {
      const int ll = i % nl, rest = i / nl, cs = rest & 1, k = rest >> 1;
      if (cs == 1 && !HAS_S) continue;
      if (map0 + k >= nmaps) continue;
      vpart[(int64_t)tile * tstride + (int64_t)(map0 + k) * vstride + moff(L, m) + cs * nsl + ll] = 0.0;
    }
  }
  const int nsl = L - m + 1;
  for (int lc = l0; lc <= L; lc += CH) {
    double P[CH][NM][2];
#pragma unroll
    for (int s = 0; s < CH; ++s)
#pragma unroll
      for (int k = 0; k < NM; ++k) P[s][k][0] = P[s][k][1] = 0.0;
    bool fast = true;
#pragma unroll
    for (int j = 0; j < R; ++j) fast = fast && (lw[j] <= lc) && (nx[j] >= lc + CH);
    const bool odd0 = ((lc - m) & 1) != 0;
    if (fast) {
      if (odd0)
        adj_chunk_fast<NM, R, CH, SQ, HAS_S, true>(gb, lc, L, z, a0, a1, E, O, P);
      else
        adj_chunk_fast<NM, R, CH, SQ, HAS_S, false>(gb, lc, L, z, a0, a1, E, O, P);
    } else {
#pragma unroll
      for (int s = 0; s < CH; ++s) {
        const int l = lc + s;
        if (l > L) break;
        const double gl = uld(gb, l);
        const bool odd = ((l - m) & 1) != 0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          if (l < lw[j]) continue;
          double c = fma(gl * z[j], a1[j], -a0[j]);
          double pv = a1[j];
          if (l == nx[j]) {
            // start values are re-read at these (rare) events to keep them
            // out of registers
            const int p = pbase + j;
            const bool valid = p < a.npairs;
            const int lsj = valid ? a.ls[(size_t)m * a.npairs + p] : INT_MAX;
            const bool inj = (lsj == l);
            if (inj) {
              const double2 msj = a.ms[(size_t)m * a.npairs + p];
              c = msj.y;
              pv = msj.x;
            }
            nx[j] = wave_min(lsj > l ? lsj : INT_MAX);
          }
          a0[j] = pv;
          a1[j] = c;
          const double w = SQ ? c * c : c;
#pragma unroll
          for (int k = 0; k < NM; ++k) {
            const double hc = (SQ || !odd) ? E[j][k][0] : O[j][k][0];
            P[s][k][0] = fma(w, hc, P[s][k][0]);
            if (HAS_S) {
              const double hs = (SQ || !odd) ? E[j][k][1] : O[j][k][1];
              P[s][k][1] = fma(w, hs, P[s][k][1]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int s = 0; s < CH; ++s)
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        buf[(s * NM + k) * 2 + 0][tid] = P[s][k][0];
        buf[(s * NM + k) * 2 + 1][tid] = P[s][k][1];
      }
    __syncthreads();
    {
      // NOUT outputs, NPER = 256 / NOUT threads each: every thread sums NOUT
      // lane values, lanes of a wave combine by xor-shuffles, the 4 wave
      // partials are added in a fixed order.
      constexpr int NPER = 256 / NOUT;
      const int o = tid % NOUT;
      const int sub = tid / NOUT;
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < NOUT; ++i) acc += buf[o][sub + NPER * i];
#pragma unroll
      for (int off = NOUT; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
      if ((tid & 63) < NOUT) red[wave][o] = acc;
    }
    __syncthreads();
    if (tid < NOUT) {
      const int o = tid;
      const double acc = (red[0][o] + red[1][o]) + (red[2][o] + red[3][o]);
      const int s = o / (NM * 2);
      const int k = (o / 2) % NM;
      const int cs = o & 1;
      const int l = lc + s;
      if (l <= L && map0 + k < nmaps && (HAS_S || cs == 0))
        vpart[(int64_t)tile * tstride + (int64_t)(map0 + k) * vstride + moff(L, m) + cs * nsl + (l - m)] = acc;
    }
  }
}

template <int NM, int R, bool SQ>
__global__ __launch_bounds__(256) void k_leg_adjoint(LegArgs a, int nmaps, const double2* __restrict__ phase,
                                                     int64_t pstride, double* __restrict__ vpart,
                                                     int64_t vstride, int64_t tstride) {
  __shared__ AdjShared<NM> sh;
  const int m = blockIdx.x;
  const int tile = blockIdx.y;
  const int map0 = blockIdx.z * NM;
  if (m == 0)
    adjoint_body<NM, R, SQ, false>(a, m, tile, map0, nmaps, phase, pstride, vpart, vstride, tstride, sh);
  else
    adjoint_body<NM, R, SQ, true>(a, m, tile, map0, nmaps, phase, pstride, vpart, vstride, tstride, sh);
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
void launch_leg_synth(const LegArgs& a, int nmaps, const double* uhat, int64_t ustride,
                      double2* phase, int64_t pstride, hipStream_t s) {
  const int L = a.lmax;
  const int ntiles = (a.npairs + 63) / 64;
  const int nmb = (L + 1 + 3) / 4;
  const int nmb8 = (nmb + 7) / 8 * 8;
  int nm = nmaps <= 8 ? nmaps : 8;
  if (nmaps > 8) {
    // pick the chunk size with the least padding
    int best = 8, waste = 1 << 30;
    for (int c : {8, 6, 4}) {
      int w = ((nmaps + c - 1) / c) * c - nmaps;
      if (w < waste) { waste = w; best = c; }
    }
    nm = best;
  }
  dim3 grid(nmb8 * ntiles, (nmaps + nm - 1) / nm);
  dim3 block(256);
#define CRS_SYN(N) \
  case N: hipLaunchKernelGGL(k_leg_synth<N>, grid, block, 0, s, a, nmaps, uhat, ustride, phase, pstride, ntiles); break;
  switch (nm) {
    CRS_SYN(1) CRS_SYN(2) CRS_SYN(3) CRS_SYN(4) CRS_SYN(5) CRS_SYN(6) CRS_SYN(7) CRS_SYN(8)
    default: throw Error{CRS_EINVAL, "bad map chunk"};
  }
#undef CRS_SYN
  CRS_HIP(hipGetLastError());
}

static int adj_r(int npairs) {
  int need = (npairs + 255) / 256;
  if (need <= 1) return 1;
  if (need <= 2) return 2;
  return 4;
}

int leg_adjoint_tiles(int npairs) {
  int r = adj_r(npairs);
  return (npairs + 256 * r - 1) / (256 * r);
}

void launch_leg_adjoint(const LegArgs& a, int nmaps, const double2* phase, int64_t pstride,
                        double* vpart, int64_t vstride, int64_t tstride, bool square,
                        hipStream_t s) {
  const int L = a.lmax;
  const int r = adj_r(a.npairs);
  const int ntiles = leg_adjoint_tiles(a.npairs);
  int nm = nmaps >= 4 ? 4 : (nmaps >= 2 ? 2 : 1);
  dim3 grid(L + 1, ntiles, (nmaps + nm - 1) / nm);
  dim3 block(256);
#define CRS_ADJ(N, RR)                                                                          \
  if (nm == N && r == RR) {                                                                     \
    if (square)                                                                                 \
      hipLaunchKernelGGL((k_leg_adjoint<N, RR, true>), grid, block, 0, s, a, nmaps, phase,      \
                         pstride, vpart, vstride, tstride);                                     \
    else                                                                                        \
      hipLaunchKernelGGL((k_leg_adjoint<N, RR, false>), grid, block, 0, s, a, nmaps, phase,     \
                         pstride, vpart, vstride, tstride);                                     \
    CRS_HIP(hipGetLastError());                                                                 \
    return;                                                                                     \
  }
  CRS_ADJ(1, 1) CRS_ADJ(1, 2) CRS_ADJ(1, 4)
  CRS_ADJ(2, 1) CRS_ADJ(2, 2) CRS_ADJ(2, 4)
  CRS_ADJ(4, 1) CRS_ADJ(4, 2) CRS_ADJ(4, 4)
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
