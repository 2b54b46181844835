// Operators, right-hand side and PCG on a set of independent systems.
//
//   A   = S^-1 + sum_nu P_nu^T N_nu^-1 P_nu       (Sect. 2.3, eq:A)
//   P_nu = Y_nu B_nu q_{nu,k}                       (eq:P; Q~ = q I, Sect. 3.3)
//   M_PI = U^+ T^+ (U^+)^T                          (eq:fullmodel-preconditioner)
//   M_diag = (U^T diag(T) U)^-1                     (Sect. 5)
//   b = sum_nu P_nu^T (tau d + tau^1/2 w1) + S^-1/2 w2
//
// A and M_PI share one shape: a per-l component -> band mix (k_mix_fwd),
// one SHT round trip per band with a pixel weight (Legendre synthesis, ring
// FFTs with the weight, Legendre adjoint), and a per-l band -> component mix
// plus a per-l component -> component term (k_mix_back).  Every (system,
// band) pair whose band shares (grid, L) with others is one map of a group,
// so a group's Legendre and ring launches carry all of them at once.
//
// PCG (Sect. 2.3; Hestenes-Stiefel form): per system the scalars live on the
// device (alpha, beta, rho, |r|^2, flags); the host reads them once per
// iteration.  Each system stops when its recursive residual |r|/|b| <= rtol,
// its true residual b - A x is then formed once, and it restarts from its
// iterate (beta = 0) if that fails rtol.  With use_graph the iteration body
// (M r, r.z, p update, A p, p.Ap, x/r update) is one captured hipGraph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>

#include "model.h"

namespace crs {

namespace {

constexpr int kDotBlocks = 256;   // fixed partition of every dot product
constexpr int kScal = 8;          // scalars per system
enum { S_RHO = 0, S_ALPHA = 1, S_BETA = 2, S_RR = 3, S_ACTIVE = 4, S_BREAK = 5, S_RESTART = 6, S_TMP = 7 };

// ---------------------------------------------------------------- kernels
__device__ __forceinline__ double block_sum256(double acc, double* red) {
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// uhat[map][i] = c_m f_lm sum_k coef[l][band][k] x[sys][coff_k + idx_k]
// for the packed indices of block xb of map `map` (kWorkBlock indices)
__device__ __forceinline__ void mix_fwd_block(const double* __restrict__ x, const SysDev* __restrict__ sys,
                                              const ProbDev* __restrict__ probs, const SlotDev* __restrict__ slots,
                                              int usep, int Lb, double* __restrict__ uhat, int64_t nalm,
                                              const double* __restrict__ act, int map, int xb) {
  const SlotDev sl = slots[map];
  if (act && act[kScal * sl.sys] == 0.0) return;
  const SysDev S = sys[sl.sys];
  const ProbDev P = probs[S.prob];
  const double* __restrict__ coef = usep ? P.cP : P.cA;
  const double* __restrict__ xs = x + S.off;
  const int64_t i0 = (int64_t)xb * kWorkBlock;
  const int64_t i1 = min(nalm, i0 + kWorkBlock);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    int m, part, ll;
    unpack_lm(Lb, i, m, part, ll);
    const int l = m + ll;
    double acc = 0.0;
    for (int k = 0; k < P.nc; ++k) {
      const int L = P.lk[k];
      if (l > L) continue;
      const double c = coef[((int64_t)l * P.nb + sl.band) * P.nc + k];
      const int64_t loc = moff_h(L, m) + (int64_t)part * (L - m + 1) + ll;
      // a spatially varying pair reads y = Q~ x_k instead of x_k (eq:Q)
      const int v = (!usep && P.vidx) ? P.vidx[sl.band * P.nc + k] : -1;
      const double xv = v >= 0 ? P.ybuf[P.yoff[v] + (int64_t)S.rhs * (int64_t)(L + 1) * (L + 1) + loc]
                               : xs[P.coff[k] + loc];
      acc = fma(c, xv, acc);
    }
    const double cm = (m == 0) ? 1.0 : 1.4142135623730951;
    uhat[(int64_t)map * nalm + i] = cm * P.ftab[tri_h(P.Lf, m) + ll] * acc;
  }
}

// one group (grid: packed-index blocks of kWorkBlock x maps)
__global__ void k_mix_fwd(const double* __restrict__ x, const SysDev* __restrict__ sys,
                          const ProbDev* __restrict__ probs, const SlotDev* __restrict__ slots, int usep,
                          int Lb, double* __restrict__ uhat, int64_t nalm, const double* __restrict__ act) {
  mix_fwd_block(x, sys, probs, slots, usep, Lb, uhat, nalm, act, blockIdx.y, blockIdx.x);
}

// Several groups in one launch (an operator application then launches one
// mixing kernel instead of one per group): group t owns the blocks
// [first, first + nbx * nmaps) of the one-dimensional grid.
constexpr int kFuseGroups = 16;
struct MixFwdGroup {
  const SlotDev* slots;
  double* uhat;
  int64_t nalm;
  int Lb, nbx, first;
};
struct MixFwdAll {
  MixFwdGroup g[kFuseGroups];
  int ng;
};
__global__ void k_mix_fwd_all(const double* __restrict__ x, const SysDev* __restrict__ sys,
                              const ProbDev* __restrict__ probs, int usep, const double* __restrict__ act,
                              const MixFwdAll a) {
  const int b = blockIdx.x;
  int t = 0;
  while (t + 1 < a.ng && b >= a.g[t + 1].first) ++t;
  const int loc = b - a.g[t].first;
  const int map = loc / a.g[t].nbx;
  mix_fwd_block(x, sys, probs, a.g[t].slots, usep, a.g[t].Lb, a.g[t].uhat, a.g[t].nalm, act, map,
                loc - map * a.g[t].nbx);
}

// y[sys][coff_k + idx] = diag term + sum_nu coef[l][nu][k] c_m f_lm sum_t vpart_nu[t][map][idx_nu]
// dmode 0: no diag term; 1: (dsqrt ? C^-1/2 : C^-1) din; 2: Pi_l din.
// (grid: one block per work-list entry over the systems, packed index u of
// P.Lc; each thread forms all components of its (l, m), so the band partials
// of an index are read once, not once per component)
// wpart (optional): this block's part of din . y at wpart[blockIdx.x]
__global__ __launch_bounds__(256) void k_mix_back(double* __restrict__ y, const double* __restrict__ din,
                                                  const SysDev* __restrict__ sys, const ProbDev* __restrict__ probs,
                                                  const int4* __restrict__ wl, int dmode, int dsqrt, int usep,
                                                  const double* __restrict__ act, double* __restrict__ wpart) {
  __shared__ double red[4];
  const int4 w = wl[blockIdx.x];
  if (act && act[kScal * w.x] == 0.0) {
    if (wpart && threadIdx.x == 0) wpart[blockIdx.x] = 0.0;
    return;
  }
  double dacc = 0.0;
  const SysDev S = sys[w.x];
  const ProbDev P = probs[S.prob];
  const int Lc = P.Lc, nc = P.nc;
  const double* __restrict__ coef = usep ? P.cP : P.cA;
  const double* __restrict__ ds = din ? din + S.off : nullptr;
  for (int u = w.y + threadIdx.x; u < w.z; u += blockDim.x) {
    int m, part, ll;
    unpack_lm(Lc, u, m, part, ll);
    const int l = m + ll;
    // index of (l, m, part) in each component's layout (-1: above its band-limit)
    int64_t ix[8];
    double acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      ix[k] = -1;
      acc[k] = 0.0;
      if (k < nc) {
        const int L = P.lk[k];
        if (l <= L) ix[k] = P.coff[k] + moff_h(L, m) + (int64_t)part * (L - m + 1) + ll;
      }
    }
    if (dmode == 1) {
      const double* dt = dsqrt ? P.dSqrt : P.dInv;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < nc && ix[k] >= 0) acc[k] = dt[(int64_t)l * nc + k] * ds[ix[k]];
    } else if (dmode == 2) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (k >= nc || ix[k] < 0) continue;
        double a = 0.0;
#pragma unroll
        for (int kp = 0; kp < 8; ++kp)
          if (kp < nc && ix[kp] >= 0) a = fma(P.dPi[((int64_t)l * nc + k) * nc + kp], ds[ix[kp]], a);
        acc[k] = a;
      }
    }
    const double cm = (m == 0) ? 1.0 : 1.4142135623730951;
    const double fs = cm * P.ftab[tri_h(P.Lf, m) + ll];
    for (int nu = 0; nu < P.nb; ++nu) {
      const int* bi = P.binfo + kBinfo * nu;
      const int L = bi[0];
      if (l > L || (usep && bi[5])) continue;  // bands merged into another drop out of M_PI
      const int gmaps = bi[1], map = bi[2] + S.rhs * bi[4], nt = bi[3];
      const int64_t nalm = (int64_t)(L + 1) * (L + 1);
      const int64_t tstride = (int64_t)gmaps * nalm;
      const double* v = P.vptr[nu] + (int64_t)map * nalm + moff_h(L, m) + (int64_t)part * (L - m + 1) + ll;
      // tile partials, four loads in flight, summed in tile order
      double sv = 0.0;
      int t = 0;
      for (; t + 4 <= nt; t += 4) {
        const double v0 = v[t * tstride], v1 = v[(t + 1) * tstride];
        const double v2 = v[(t + 2) * tstride], v3 = v[(t + 3) * tstride];
        sv += v0;
        sv += v1;
        sv += v2;
        sv += v3;
      }
      for (; t < nt; ++t) sv += v[t * tstride];
      const double* cn = coef + ((int64_t)l * P.nb + nu) * nc;
      const int* vb = (!usep && P.vidx) ? P.vidx + nu * nc : nullptr;  // varying pairs: added afterwards
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < nc && ix[k] >= 0 && !(vb && vb[k] >= 0)) acc[k] = fma(cn[k] * fs, sv, acc[k]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k >= nc || ix[k] < 0) continue;
      y[S.off + ix[k]] = acc[k];
      if (wpart) dacc = fma(ds[ix[k]], acc[k], dacc);
    }
  }
  if (wpart) {
    const double t = block_sum256(dacc, red);
    if (threadIdx.x == 0) wpart[blockIdx.x] = t;
  }
}

// z[sys][coff_k + idx] = sum_k' Dinv[u][k][k'] r[sys][coff_k' + idx'] over active k'
// (grid: one block per work-list entry over the systems, packed index u of P.Lc)
// wpart (optional): this block's part of r . z at wpart[blockIdx.x]
__global__ __launch_bounds__(256) void k_diag_apply(const double* __restrict__ r, double* __restrict__ z,
                                                    const SysDev* __restrict__ sys, const ProbDev* __restrict__ probs,
                                                    const int4* __restrict__ wl, const double* __restrict__ act,
                                                    double* __restrict__ wpart) {
  __shared__ double red[4];
  const int4 w = wl[blockIdx.x];
  if (act && act[kScal * w.x] == 0.0) {
    if (wpart && threadIdx.x == 0) wpart[blockIdx.x] = 0.0;
    return;
  }
  double dacc = 0.0;
  const SysDev S = sys[w.x];
  const ProbDev P = probs[S.prob];
  const int Lc = P.Lc, nc = P.nc;
  const double* rs = r + S.off;
  double* zs = z + S.off;
  for (int u = w.y + threadIdx.x; u < w.z; u += blockDim.x) {
    int m, part, ll;
    unpack_lm(Lc, u, m, part, ll);
    const int l = m + ll;
    double rv[8];
    for (int k = 0; k < nc; ++k) {
      const int L = P.lk[k];
      rv[k] = (l <= L) ? rs[P.coff[k] + moff_h(L, m) + (int64_t)part * (L - m + 1) + ll] : 0.0;
    }
    for (int k = 0; k < nc; ++k) {
      const int L = P.lk[k];
      if (l > L) continue;
      double acc = 0.0;
      for (int kp = 0; kp < nc; ++kp) acc = fma(P.Dinv[((int64_t)u * nc + k) * nc + kp], rv[kp], acc);
      zs[P.coff[k] + moff_h(L, m) + (int64_t)part * (L - m + 1) + ll] = acc;
      dacc = fma(rv[k], acc, dacc);
    }
  }
  if (wpart) {
    const double t = block_sum256(dacc, red);
    if (threadIdx.x == 0) wpart[blockIdx.x] = t;
  }
}

// wpart[b] = this work-list block's part of a . b over its packed indices of
// every component (the partition k_mix_back uses for its fused dot)
__global__ __launch_bounds__(256) void k_wl_dot(const double* __restrict__ a, const double* __restrict__ b,
                                                const SysDev* __restrict__ sys, const ProbDev* __restrict__ probs,
                                                const int4* __restrict__ wl, const double* __restrict__ act,
                                                double* __restrict__ wpart) {
  __shared__ double red[4];
  const int4 w = wl[blockIdx.x];
  if (act && act[kScal * w.x] == 0.0) {
    if (threadIdx.x == 0) wpart[blockIdx.x] = 0.0;
    return;
  }
  const SysDev S = sys[w.x];
  const ProbDev P = probs[S.prob];
  double acc = 0.0;
  for (int u = w.y + threadIdx.x; u < w.z; u += blockDim.x) {
    int m, part, ll;
    unpack_lm(P.Lc, u, m, part, ll);
    const int l = m + ll;
    for (int k = 0; k < P.nc; ++k) {
      const int L = P.lk[k];
      if (l > L) continue;
      const int64_t i = S.off + P.coff[k] + moff_h(L, m) + (int64_t)part * (L - m + 1) + ll;
      acc = fma(a[i], b[i], acc);
    }
  }
  const double t = block_sum256(acc, red);
  if (threadIdx.x == 0) wpart[blockIdx.x] = t;
}

// y[sys][coff_k + idx] = C^-1_{k,l} x[sys][coff_k + idx] (work list over rows)
__global__ void k_prior(double* __restrict__ y, const double* __restrict__ x, const SysDev* __restrict__ sys,
                        const ProbDev* __restrict__ probs, const int2* __restrict__ rows,
                        const int4* __restrict__ wl) {
  const int4 w = wl[blockIdx.x];
  const int2 row = rows[w.x];
  const SysDev S = sys[row.x];
  const ProbDev P = probs[S.prob];
  const int k = row.y;
  const int Lk = P.lk[k];
  const int64_t o = S.off + P.coff[k];
  for (int i = w.y + threadIdx.x; i < w.z; i += blockDim.x) {
    int m, part, ll;
    unpack_lm(Lk, i, m, part, ll);
    y[o + i] = P.dInv[(int64_t)(m + ll) * P.nc + k] * x[o + i];
  }
}

// One block per (r, nu, k) of a single-problem Exec (see exec_mix_grad).
__global__ __launch_bounds__(256) void k_dq(const double* __restrict__ va, int sa0, const double* __restrict__ vb,
                                            int sb0, double sign, const SysDev* __restrict__ sys,
                                            const ProbDev* __restrict__ probs, const double* __restrict__ beamtab,
                                            double* __restrict__ dq) {
  __shared__ double red[4];
  const ProbDev P = probs[0];
  const int nb = P.nb, nc = P.nc;
  const int k = blockIdx.x % nc;
  const int nu = (blockIdx.x / nc) % nb;
  const int r = blockIdx.x / (nc * nb);
  const int Lk = P.lk[k];
  const int* bi = P.binfo + kBinfo * nu;
  const int Lb = bi[0];
  const int Lm = min(Lk, Lb);
  const int64_t nalm = (int64_t)(Lb + 1) * (Lb + 1);
  const int64_t tstride = (int64_t)bi[1] * nalm;
  const SysDev SA = sys[sa0 + r];
  const double* VA = P.vptr[nu] + (int64_t)(bi[2] + SA.rhs * bi[4]) * nalm;
  const double* VB = nullptr;
  const double* xb = nullptr;
  if (vb) {
    const SysDev SB = sys[sb0 + r];
    VB = P.vptr[nu] + (int64_t)(bi[2] + SB.rhs * bi[4]) * nalm;
    xb = vb + SA.off;
  }
  const double* xa = va + SA.off;
  double acc = 0.0;
  for (int m = 0; m <= Lm; ++m) {
    const int np = (m == 0) ? 1 : 2;
    const int ns = Lm - m + 1;
    const double cm = (m == 0) ? 1.0 : 1.4142135623730951;
    for (int i = threadIdx.x; i < np * ns; i += 256) {
      const int part = i / ns, ll = i % ns, l = m + ll;
      const int64_t ik = P.coff[k] + moff_h(Lk, m) + (int64_t)part * (Lk - m + 1) + ll;
      const int64_t ib = moff_h(Lb, m) + (int64_t)part * (Lb - m + 1) + ll;
      const double fs = beamtab[(int64_t)l * nb + nu] * cm * P.ftab[tri_h(P.Lf, m) + ll];
      double sa = 0.0, sb = 0.0;
      for (int t = 0; t < bi[3]; ++t) {
        sa += VA[t * tstride + ib];
        if (VB) sb += VB[t * tstride + ib];
      }
      acc = fma(xa[ik], fs * sa, acc);
      if (VB) acc = fma(xb[ik], fs * sb, acc);
    }
  }
  const double t = block_sum256(acc, red);
  if (threadIdx.x == 0) dq[blockIdx.x] = sign * t;
}

// partial[sys][blk] = this block's slice of a . b (grid: kDotBlocks x nsys)
__global__ __launch_bounds__(256) void k_dot(const double* __restrict__ a, const double* __restrict__ b,
                                             const SysDev* __restrict__ sys, double* __restrict__ partial,
                                             const double* __restrict__ act) {
  __shared__ double red[4];
  if (act && act[kScal * blockIdx.y] == 0.0) {  // finished system: its scalars are not used
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const SysDev S = sys[blockIdx.y];
  const double* pa = a + S.off;
  const double* pb = b + S.off;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < S.n; i += (int64_t)gridDim.x * 256)
    acc = fma(pa[i], pb[i], acc);
  const double t = block_sum256(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// op 0: alpha = rho / p.q ; op 1: beta = r.z / rho, rho = r.z ; op 2: rr = sum ;
// op 3: rho = r.z (start) ; op 4: tmp = sum.   One block per system, fixed-order sum.
__device__ void scalar_op(int op, double s, double* st);

// the fixed-order sum of partial[first .. first + n) (one block)
__device__ __forceinline__ double sum_partials(const double* __restrict__ partial, int64_t first, int n) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += partial[first + i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

__global__ __launch_bounds__(256) void k_scalar(int op, const double* __restrict__ partial, int nblk,
                                                double* __restrict__ scal) {
  const int sy = blockIdx.x;
  const double s = sum_partials(partial, (int64_t)sy * nblk, nblk);
  if (threadIdx.x == 0) scalar_op(op, s, scal + sy * kScal);
}

// the same with each system's partials a range (first, count) of one array
// (the per-block partials of a work-list kernel)
__global__ __launch_bounds__(256) void k_scalar_ranges(int op, const double* __restrict__ partial,
                                                       const int2* __restrict__ rng, double* __restrict__ scal) {
  const int sy = blockIdx.x;
  const int2 r = rng[sy];
  const double s = sum_partials(partial, r.x, r.y);
  if (threadIdx.x == 0) scalar_op(op, s, scal + sy * kScal);
}

__device__ void scalar_op(int op, double s, double* st) {
  const bool active = st[S_ACTIVE] != 0.0;
  if (op == 0) {
    if (!active) { st[S_ALPHA] = 0.0; return; }
    if (!(s > 0.0) || !isfinite(s)) {
      st[S_ALPHA] = 0.0;
      st[S_BREAK] = 1.0;
      st[S_ACTIVE] = 0.0;
      return;
    }
    st[S_ALPHA] = st[S_RHO] / s;
  } else if (op == 1) {
    if (!active) { st[S_BETA] = 0.0; return; }
    if (!(s > 0.0) || !isfinite(s)) {
      st[S_BETA] = 0.0;
      st[S_BREAK] = 1.0;
      st[S_ACTIVE] = 0.0;
      return;
    }
    st[S_BETA] = (st[S_RESTART] != 0.0) ? 0.0 : s / st[S_RHO];
    st[S_RESTART] = 0.0;
    st[S_RHO] = s;
  } else if (op == 2) {
    st[S_RR] = s;
  } else if (op == 3) {
    if (!(s > 0.0) || !isfinite(s)) {
      st[S_BREAK] = (s == 0.0) ? 0.0 : 1.0;  // r = 0: already solved
      st[S_ACTIVE] = 0.0;
    }
    st[S_RHO] = s;
  } else {
    st[S_TMP] = s;
  }
}

// x += alpha p ; r -= alpha q ; partial r.r
__global__ __launch_bounds__(256) void k_update_xr(double* __restrict__ x, double* __restrict__ r,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   const SysDev* __restrict__ sys, const double* __restrict__ scal,
                                                   double* __restrict__ partial) {
  __shared__ double red[4];
  if (scal[blockIdx.y * kScal + S_ACTIVE] == 0.0) {  // finished system: x and r stay, |r|^2 unused
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const SysDev S = sys[blockIdx.y];
  const double al = scal[blockIdx.y * kScal + S_ALPHA];
  double* px = x + S.off;
  double* pr = r + S.off;
  const double* pp = p + S.off;
  const double* pq = q + S.off;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < S.n; i += (int64_t)gridDim.x * 256) {
    if (al != 0.0) {
      px[i] = fma(al, pp[i], px[i]);
      pr[i] = fma(-al, pq[i], pr[i]);
    }
    const double v = pr[i];
    acc = fma(v, v, acc);
  }
  const double t = block_sum256(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// p = z + beta p (active systems only)
__global__ void k_update_p(double* __restrict__ p, const double* __restrict__ z, const SysDev* __restrict__ sys,
                           const double* __restrict__ scal) {
  const double* st = scal + blockIdx.y * kScal;
  if (st[S_ACTIVE] == 0.0) return;
  const SysDev S = sys[blockIdx.y];
  const double be = st[S_BETA];
  double* pp = p + S.off;
  const double* pz = z + S.off;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < S.n; i += (int64_t)gridDim.x * 256)
    pp[i] = fma(be, pp[i], pz[i]);
}

// out = a - b, or out = a (b == NULL), on the systems sel selects (sel == NULL: all)
__global__ void k_sub_sel(double* __restrict__ out, const double* __restrict__ a, const double* __restrict__ b,
                          const SysDev* __restrict__ sys, const int* __restrict__ sel) {
  if (sel && !sel[blockIdx.y]) return;
  const SysDev S = sys[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < S.n; i += (int64_t)gridDim.x * 256)
    out[S.off + i] = b ? a[S.off + i] - b[S.off + i] : a[S.off + i];
}

// f[map] = tau d + sqrt(tau) w1 (per-map pointer tables; NULL = zero)
__global__ void k_pix_rhs(double* __restrict__ f, const double* const* __restrict__ tau,
                          const double* const* __restrict__ d, const double* const* __restrict__ w1,
                          int64_t npix) {
  const int map = blockIdx.y;
  const double* t = tau[map];
  const double* dv = d[map];
  const double* wv = w1[map];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)gridDim.x * 256) {
    const double tv = t[i];
    double v = 0.0;
    if (dv) v = tv * dv[i];
    if (wv) v = fma(sqrt(tv), wv[i], v);
    f[(int64_t)map * npix + i] = v;
  }
}

// res[map] = d[map] - res[map] (res holds P x on entry; d NULL = zero) and
// partial[map][blk] = this block's part of res^T tau res
__global__ __launch_bounds__(256) void k_resid_chi2(double* const* __restrict__ res, const double* const* __restrict__ d,
                                                    const double* const* __restrict__ tau, int64_t npix,
                                                    double* __restrict__ partial) {
  __shared__ double red[4];
  const int map = blockIdx.y;
  double* r = res[map];
  const double* dv = d[map];
  const double* t = tau[map];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)gridDim.x * 256) {
    const double v = (dv ? dv[i] : 0.0) - r[i];
    r[i] = v;
    acc = fma(t[i] * v, v, acc);
  }
  const double sum = block_sum256(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)map * gridDim.x + blockIdx.x] = sum;
}

// out[map] = scale tau[map] in[map]
__global__ void k_noise_weight(double* const* __restrict__ out, const double* const* __restrict__ in,
                               const double* const* __restrict__ tau, double scale, int64_t npix) {
  const int map = blockIdx.y;
  double* o = out[map];
  const double* v = in[map];
  const double* t = tau[map];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)gridDim.x * 256)
    o[i] = scale * t[i] * (v ? v[i] : 0.0);
}

// out[sys] = scale * sum of the partials of the system's maps: per system,
// the ranges rng[j] (first, count) for j in [rofs[sys], rofs[sys + 1]), in order
__global__ __launch_bounds__(256) void k_sum_ranges(const double* __restrict__ partial, const int2* __restrict__ rng,
                                                    const int* __restrict__ rofs, double scale,
                                                    double* __restrict__ out) {
  const int sy = blockIdx.x;
  double tot = 0.0;
  for (int j = rofs[sy]; j < rofs[sy + 1]; ++j) {
    const int2 r = rng[j];
    tot += sum_partials(partial, r.x, r.y);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[sy] = scale * tot;
}

// out[sys] = scale * scal[sys][S_TMP]
__global__ void k_scal_out(const double* __restrict__ scal, int nsys, double scale, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsys) out[i] = scale * scal[i * kScal + S_TMP];
}

// per map of a group: flag[8 j] = keep[j] and (act == NULL or the map's system is active)
__global__ void k_pi_flags(double* __restrict__ flag, const int* __restrict__ keep, const int* __restrict__ mapsys,
                           const double* __restrict__ act, int nmaps) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nmaps) return;
  const bool on = keep[j] != 0 && (act == nullptr || act[kScal * mapsys[j]] != 0.0);
  flag[kActStride * j] = on ? 1.0 : 0.0;
}

// The maps of a group that a launch processes (not skipped), ascending, and
// their count: the Legendre kernels then run dense groups of active maps
// (one block; a thread takes a contiguous run of maps).
__device__ __forceinline__ void compact_block(const MapSkip& skip, int nmaps, int* __restrict__ mlist,
                                              int* __restrict__ mcount) {
  __shared__ int cnt[256];
  const int t = threadIdx.x;
  const int per = (nmaps + 255) / 256;
  const int b0 = min(nmaps, t * per), b1 = min(nmaps, b0 + per);
  int c = 0;
  for (int j = b0; j < b1; ++j) c += skip.off(j) ? 0 : 1;
  cnt[t] = c;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {  // inclusive prefix sum
    const int v = t >= o ? cnt[t - o] : 0;
    __syncthreads();
    cnt[t] += v;
    __syncthreads();
  }
  int pos = cnt[t] - c;
  for (int j = b0; j < b1; ++j)
    if (!skip.off(j)) mlist[pos++] = j;
  if (t == 255) mcount[0] = cnt[255];
}

__global__ __launch_bounds__(256) void k_compact(MapSkip skip, int nmaps, int* __restrict__ mlist,
                                                 int* __restrict__ mcount) {
  compact_block(skip, nmaps, mlist, mcount);
}

// the lists of several groups in one launch (block t: group t)
struct CompactGroup {
  MapSkip skip;
  int nmaps;
  int* mlist;
  int* mcount;
};
struct CompactAll {
  CompactGroup g[kFuseGroups];
};
__global__ __launch_bounds__(256) void k_compact_all(const CompactAll a) {
  const CompactGroup& g = a.g[blockIdx.x];
  compact_block(g.skip, g.nmaps, g.mlist, g.mcount);
}

inline dim3 vgrid(int nsys) { return dim3(kDotBlocks, nsys); }

void mix_back(Exec& e, double* out, const double* din, int dmode, int dsqrt, int usep, hipStream_t s,
              const double* act = nullptr, double* wpart = nullptr) {
  hipLaunchKernelGGL(k_mix_back, dim3(e.nwl_sys), dim3(256), 0, s, out, din, e.dsys.p, e.dprobs.p, e.wl_sys.p,
                     dmode, dsqrt, usep, act, wpart);
  CRS_HIP(hipGetLastError());
}

// act: skip systems whose flag is 0 (inside the iteration); NULL: all systems
void dot_to(Exec& e, const double* a, const double* b, int op, hipStream_t s, const double* act = nullptr) {
  hipLaunchKernelGGL(k_dot, vgrid(e.nsys), dim3(256), 0, s, a, b, e.dsys.p, e.partial.p, act);
  hipLaunchKernelGGL(k_scalar, dim3(e.nsys), dim3(256), 0, s, op, e.partial.p, kDotBlocks, e.scal.p);
  CRS_HIP(hipGetLastError());
}

}  // namespace

Exec::~Exec() {
  graphs.clear();
  if (hscal) (void)hipHostFree(hscal);
  if (hsel) (void)hipHostFree(hsel);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  for (hipStream_t t : side) (void)hipStreamDestroy(t);
  for (hipEvent_t ev : join) (void)hipEventDestroy(ev);
  if (fork) (void)hipEventDestroy(fork);
}

int64_t exec_plan_bytes(const std::vector<crs_model>& models, int nrhs) {
  // the buffers make_exec allocates (the right-hand side's pixel maps are
  // allocated on the first build_rhs / project and counted here too)
  std::map<std::pair<crs_grid, int>, int> maps;
  int64_t ntot = 0, nsys = 0;
  for (const crs_model m : models) {
    ntot += m->n * nrhs;
    nsys += nrhs;
    for (const Band& b : m->bands) maps[std::make_pair(b.grid, b.lmax)] += nrhs;
  }
  int64_t bytes = 0;
  for (const auto& kv : maps) {
    const crs_grid g = kv.first.first;
    const int L = kv.first.second, nm = kv.second;
    const int64_t nalm = (int64_t)(L + 1) * (L + 1);
    const int npairs = (g->nring + 1) / 2;
    const LegChoice c = leg_choice(npairs, L, nm);
    bytes += (int64_t)nm * nalm * 8;                          // uhat
    bytes += (int64_t)nm * g->nring * (L + 1) * 16;           // phase
    bytes += (int64_t)leg_adjoint_tiles(c, npairs, false) * nm * nalm * 8;  // adjoint partial sums
    bytes += (int64_t)nm * g->npix * 8;                       // pixel maps (right-hand side)
  }
  bytes += 7 * ntot * 8;                                      // r, z, p, q, t, x and the caller's b
  bytes += nsys * (kDotBlocks + 4 * kScal) * 8;
  return bytes;
}

std::unique_ptr<Exec> make_exec(const std::vector<crs_model>& models, int nrhs, hipStream_t s, bool autotune) {
  CRS_CHECK(!models.empty() && nrhs >= 1, CRS_EINVAL, "no systems");
  {
    // memory plan: refuse up front rather than fail part-way through the allocations
    size_t freeb = 0, totb = 0;
    if (hipMemGetInfo(&freeb, &totb) == hipSuccess) {
      const int64_t need = exec_plan_bytes(models, nrhs);
      CRS_CHECK(need <= (int64_t)freeb, CRS_ENOMEM,
                "the operator state needs " + std::to_string(need >> 20) + " MiB of device memory, " +
                    std::to_string(freeb >> 20) + " MiB are free");
    }
  }
  auto e = std::make_unique<Exec>();
  e->probs = models;
  const int np = (int)models.size();
  int64_t off = 0;
  for (int p = 0; p < np; ++p) {
    const crs_model m = models[p];
    e->Lc = std::max(e->Lc, m->Lc);
    e->has_diag = e->has_diag && m->has_diag;
    for (int r = 0; r < nrhs; ++r) {
      e->hsys.push_back(SysDev{p, r, off, m->n});
      off += m->n;
    }
  }
  e->nsys = (int)e->hsys.size();
  e->ntot = off;
  e->hact.assign(e->nsys, 1);
  {
    std::vector<int> id(e->nsys);
    for (int i = 0; i < e->nsys; ++i) id[i] = i;
    e->sys_ident.upload(id, s);
  }
  // groups: maps (problem, band) x rhs, map = base + rhs
  std::map<std::pair<crs_grid, int>, int> gid;
  std::vector<std::vector<int>> bmap(np);  // per problem per band: map base
  std::vector<std::vector<int>> bgrp(np);
  for (int p = 0; p < np; ++p) {
    const crs_model m = models[p];
    bmap[p].resize(m->nbands);
    bgrp[p].resize(m->nbands);
    for (int nu = 0; nu < m->nbands; ++nu) {
      const Band& b = m->bands[nu];
      auto key = std::make_pair(b.grid, b.lmax);
      auto it = gid.find(key);
      if (it == gid.end()) {
        gid[key] = (int)e->groups.size();
        e->groups.emplace_back();
        ExecGroup& g = e->groups.back();
        g.grid = b.grid;
        g.lmax = b.lmax;
        it = gid.find(key);
      }
      ExecGroup& g = e->groups[it->second];
      bgrp[p][nu] = it->second;
      bmap[p][nu] = g.nmaps;
      g.nmaps += nrhs;
      for (int r = 0; r < nrhs; ++r) g.hslots.push_back(SlotDev{p * nrhs + r, nu});
    }
  }
  for (auto& g : e->groups) {
    g.plan = &get_plan(g.grid, g.lmax, s);
    g.nalm = (int64_t)(g.lmax + 1) * (g.lmax + 1);
    g.pst = (int64_t)g.grid->nring * (g.lmax + 1);
    g.uhat.alloc((size_t)g.nmaps * g.nalm);
    g.mlist.alloc((size_t)g.nmaps);
    g.mcount.alloc(1);
    g.phase.alloc((size_t)g.nmaps * g.pst);
    g.leg = autotune ? leg_autotune(leg_args(g.grid, *g.plan), g.nmaps, g.uhat.p, g.phase.p, s)
                     : leg_choice(g.plan->npairs, g.lmax, g.nmaps);
    g.ntiles = leg_adjoint_tiles(g.leg, g.plan->npairs, false);
    std::vector<const double*> wa, wp, ta;
    for (const SlotDev& sl : g.hslots) {
      const Band& b = models[e->hsys[sl.sys].prob]->bands[sl.band];
      wa.push_back(b.tau.p);
      wp.push_back(b.tplus.p);
      ta.push_back(b.tau.p);
    }
    g.slots.upload(g.hslots, s);
    std::vector<int> ms, ident, keep;
    g.pi_maps = 0;
    for (const SlotDev& sl : g.hslots) {
      ms.push_back(sl.sys);
      ident.push_back((int)ident.size());
      const crs_model pm = models[e->hsys[sl.sys].prob];
      const int k = pm->pi_drop.empty() ? 1 : !pm->pi_drop[sl.band];
      keep.push_back(k);
      g.pi_maps += k;
    }
    g.mapsys.upload(ms, s);
    g.ident.upload(ident, s);
    g.pikeep.upload(keep, s);
    g.hkeep = keep;
    g.piflag.alloc((size_t)kActStride * g.nmaps);
    g.wA.upload(wa, s);
    g.wP.upload(wp, s);
    g.tau.upload(ta, s);
    g.vpart.alloc((size_t)g.ntiles * g.nmaps * g.nalm);
  }
  // per-problem device views
  std::vector<ProbDev> pd(np);
  e->vptr.resize(np);
  e->binfo.resize(np);
  for (int p = 0; p < np; ++p) {
    const crs_model m = models[p];
    std::vector<const double*> vp(m->nbands);
    std::vector<int> bi(kBinfo * m->nbands);
    for (int nu = 0; nu < m->nbands; ++nu) {
      const ExecGroup& g = e->groups[bgrp[p][nu]];
      vp[nu] = g.vpart.p;
      bi[kBinfo * nu + 0] = g.lmax;
      bi[kBinfo * nu + 1] = g.nmaps;
      bi[kBinfo * nu + 2] = bmap[p][nu];
      bi[kBinfo * nu + 3] = g.ntiles;
      bi[kBinfo * nu + 4] = 1;
      bi[kBinfo * nu + 5] = m->pi_drop.empty() ? 0 : m->pi_drop[nu];
    }
    e->vptr[p].upload(vp, s);
    e->binfo[p].upload(bi, s);
    ProbDev& d = pd[p];
    d.nc = m->ncomp;
    d.nb = m->nbands;
    d.Lf = m->Lmax;
    d.Lc = m->Lc;
    d.lk = m->d_lk.p;
    d.coff = m->d_coff.p;
    d.cA = m->cA.p;
    d.cP = m->cP.p;
    d.dInv = m->dInv.p;
    d.dSqrt = m->dSqrt.p;
    d.dPi = m->dPi.p;
    d.ftab = m->ftab.p;
    d.Dinv = m->has_diag ? m->Dinv.p : nullptr;
    d.vptr = e->vptr[p].p;
    d.binfo = e->binfo[p].p;
    d.vidx = nullptr;
    d.ybuf = nullptr;
    d.yoff = nullptr;
  }
  if (!models.empty()) {
    bool any = false;
    for (const crs_model m : models) any = any || !m->varmix.empty();
    CRS_CHECK(!any || models.size() == 1, CRS_EUNSUPPORTED,
              "spatially varying mixing maps are supported on single models, not in batches");
    if (any) exec_varmix_prepare(*e, s);  // sets the varying-pair fields of pd[0]
    if (any) {
      pd[0].vidx = e->vm_vidx;
      pd[0].ybuf = e->vm_ybuf;
      pd[0].yoff = e->vm_yoff;
    }
  }
  e->dprobs.upload(pd, s);
  e->dsys.upload(e->hsys, s);
  std::vector<int2> rows;
  for (int sy = 0; sy < e->nsys; ++sy)
    for (int k = 0; k < models[e->hsys[sy].prob]->ncomp; ++k) rows.push_back(make_int2(sy, k));
  e->nrows = (int)rows.size();
  e->rows.upload(rows, s);
  // work lists: contiguous packed-index ranges of kWorkBlock per block
  std::vector<int4> wlr, wls;
  for (int r = 0; r < e->nrows; ++r) {
    const crs_model m = models[e->hsys[rows[r].x].prob];
    const int64_t n = (int64_t)(m->lk[rows[r].y] + 1) * (m->lk[rows[r].y] + 1);
    for (int64_t a = 0; a < n; a += kWorkBlock) wlr.push_back(make_int4(r, (int)a, (int)std::min<int64_t>(n, a + kWorkBlock), 0));
  }
  for (int sy = 0; sy < e->nsys; ++sy) {
    const crs_model m = models[e->hsys[sy].prob];
    const int64_t n = (int64_t)(m->Lc + 1) * (m->Lc + 1);
    for (int64_t a = 0; a < n; a += kWorkBlock) wls.push_back(make_int4(sy, (int)a, (int)std::min<int64_t>(n, a + kWorkBlock), 0));
  }
  e->nwl_rows = (int)wlr.size();
  e->nwl_sys = (int)wls.size();
  e->wl_rows.upload(wlr, s);
  e->wl_sys.upload(wls, s);
  // per system: its blocks in the system work list (contiguous)
  std::vector<int2> rs(e->nsys, make_int2(0, 0));
  for (int b = (int)wls.size() - 1; b >= 0; --b) {
    int2& q = rs[wls[b].x];
    q.x = b;
    ++q.y;
  }
  e->rng_sys.upload(rs, s);
  e->wpart.alloc((size_t)e->nwl_sys);
  const size_t nn = (size_t)e->ntot;
  e->r.alloc(nn);
  e->z.alloc(nn);
  e->p.alloc(nn);
  e->q.alloc(nn);
  e->t.alloc(nn);
  e->xw.alloc(nn);
  e->partial.alloc((size_t)e->nsys * kDotBlocks);
  e->scal.alloc((size_t)e->nsys * kScal);
  e->cand.alloc((size_t)e->nsys * kScal);
  CRS_HIP(hipHostMalloc((void**)&e->hscal, (size_t)e->nsys * kScal * sizeof(double), hipHostMallocDefault));
  CRS_HIP(hipHostMalloc((void**)&e->hsel, (size_t)e->nsys * sizeof(int), hipHostMallocDefault));
  e->dsel.alloc(e->nsys);
  e->dcand.alloc(e->nsys);
  e->bbdev.alloc(e->nsys);
  e->hrows.alloc((size_t)kChunk * e->nsys);
  e->live.assign(e->groups.size(), 1);
  CRS_HIP(hipStreamSynchronize(s));
  if (const char* v = std::getenv("CRS_GROUP_STREAMS")) exec_set_streams(*e, std::atoi(v));
  return e;
}

namespace {
// maps of group g whose system is active (all of them when not masked), and
// for M_PI (pi) whose band is not merged into another band's row
int active_maps(const Exec& e, const ExecGroup& g, bool masked, bool pi = false) {
  int n = 0;
  for (int j = 0; j < g.nmaps; ++j)
    n += ((!masked || e.hact[g.hslots[j].sys]) && (!pi || g.hkeep[j])) ? 1 : 0;
  return n;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}
}  // namespace

// Algorithmic work of one operator launch of group gi over its active maps.
Work3 group_work(const Exec& e, int gi, int family, bool masked, bool pi) {
  const ExecGroup& g = e.groups[gi];
  const int na = active_maps(e, g, masked, pi);
  if (family == FAM_RING)
    return bytes_work(na * (ring_bytes(g.grid, g.lmax, 1, RING_ROUNDTRIP) + (double)g.grid->npix * 8.0));
  return leg_work(*g.plan, na);
}

void exec_set_streams(Exec& e, int n) {
  CRS_CHECK(n >= 1 && n <= kMaxGroupStreams, CRS_EINVAL, "stream count out of range");
  const int want = std::min<int>(n, (int)e.groups.size()) - 1;
  while ((int)e.side.size() < want) {
    hipStream_t t = nullptr;
    CRS_HIP(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
    e.side.push_back(t);
    hipEvent_t ev = nullptr;
    CRS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    e.join.push_back(ev);
  }
  if (!e.side.empty() && !e.fork) CRS_HIP(hipEventCreateWithFlags(&e.fork, hipEventDisableTiming));
  e.nstreams = n;
}

void exec_bands(Exec& e, OpKind kind, const double* in, hipStream_t s0, const double* act) {
  const bool pinv = kind == OP_PI;
  const bool skip_done = act != nullptr;
  const bool cap = capturing(s0);
  std::vector<int> run;
  for (int gi = 0; gi < (int)e.groups.size(); ++gi) {
    const ExecGroup& g = e.groups[gi];
    // groups whose systems have all finished launch nothing (their partial
    // sums are read only for active systems): outside a capture from the
    // host's activity mirror, inside one from the live-group set it was
    // captured for
    if (skip_done && !cap && active_maps(e, g, true) == 0) continue;
    if (skip_done && cap && !e.live[gi]) continue;
    // M_PI of merged observations: the bands merged into another band skip T^+
    if (pinv && g.pi_maps == 0) continue;
    run.push_back(gi);
  }
  // groups in order of work over the caller's stream and the side streams
  // (each to the least loaded one)
  const int nstr = std::min({e.nstreams, 1 + (int)e.side.size(), (int)run.size()});
  std::vector<int64_t> load(nstr, 0);
  std::vector<hipStream_t> gstream(e.groups.size(), s0);
  if (nstr > 1) {
    std::vector<int> order = run;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return e.groups[a].plan->fp64_triples * e.groups[a].nmaps > e.groups[b].plan->fp64_triples * e.groups[b].nmaps;
    });
    CRS_HIP(hipEventRecord(e.fork, s0));
    for (int i = 1; i < nstr; ++i) CRS_HIP(hipStreamWaitEvent(e.side[i - 1], e.fork, 0));
    for (int gi : order) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[k] += (int64_t)(e.groups[gi].plan->fp64_triples * e.groups[gi].nmaps);
      gstream[gi] = k == 0 ? s0 : e.side[k - 1];
    }
  }
  // the maps a group's launches skip: merged bands leave M_PI (flags formed
  // on the device), finished systems leave every operator
  auto group_skip = [&](ExecGroup& g, hipStream_t s) {
    MapSkip skip;
    if (pinv && g.pi_maps < g.nmaps) {
      hipLaunchKernelGGL(k_pi_flags, dim3((g.nmaps + 255) / 256), dim3(256), 0, s, g.piflag.p, g.pikeep.p,
                         g.mapsys.p, act, g.nmaps);
      CRS_HIP(hipGetLastError());
      skip.mapsys = g.ident.p;
      skip.act = g.piflag.p;
    } else if (skip_done) {
      skip.mapsys = g.mapsys.p;
      skip.act = act;
    }
    return skip;
  };
  // the Legendre launches take the active maps compacted (a launch late in a
  // solve then runs few dense groups instead of many sparse ones; a group of
  // at most 8 maps is one group of maps either way)
  auto compacted = [](const ExecGroup& g, const MapSkip& skip) { return skip.act != nullptr && g.nmaps > 8; };
  auto transforms = [&](int gi, const MapSkip& skip, hipStream_t s) {
    ExecGroup& g = e.groups[gi];
    const int tag = ((e.chunk_iter << 1) | (pinv ? 1 : 0)) * 1024 + gi;
    LegArgs la = leg_args(g.grid, *g.plan);
    la.skip = skip;
    if (compacted(g, skip)) {
      la.mlist = g.mlist.p;
      la.mcount = g.mcount.p;
      la.skip = MapSkip{};
    }
    {
      ProfScope ps(FAM_LEG_SYNTH, group_work(e, gi, FAM_LEG_SYNTH, skip_done, pinv), s, tag);
      launch_leg_synth(g.leg, la, g.nmaps, g.uhat.p, g.nalm, g.phase.p, g.pst, s);
    }
    {
      ProfScope ps(FAM_RING, group_work(e, gi, FAM_RING, skip_done, pinv), s, tag);
      launch_ring(g.grid, g.lmax, RING_ROUNDTRIP, g.nmaps, g.phase.p, g.pst, nullptr, nullptr, 0,
                  pinv ? g.wP.p : g.wA.p, 1, s, skip);
    }
    {
      ProfScope ps(FAM_LEG_ADJ, group_work(e, gi, FAM_LEG_ADJ, skip_done, pinv), s, tag);
      launch_leg_adjoint(g.leg, la, g.nmaps, g.phase.p, g.pst, g.vpart.p, g.nalm, (int64_t)g.nmaps * g.nalm, false,
                         s);
    }
  };
  // On one stream the groups' mixing and active-map kernels run as one
  // launch each (fewer launches per operator application; every block does
  // the same arithmetic as in the per-group launches).
  int64_t fwd_blocks = 0;
  for (int gi : run) fwd_blocks += (e.groups[gi].nalm + kWorkBlock - 1) / kWorkBlock * e.groups[gi].nmaps;
  const bool fuse = nstr <= 1 && run.size() > 1 && run.size() <= (size_t)kFuseGroups && fwd_blocks < (1ll << 31);
  if (fuse) {
    std::vector<MapSkip> sk(run.size());
    for (size_t t = 0; t < run.size(); ++t) sk[t] = group_skip(e.groups[run[t]], s0);
    CompactAll ca{};
    int nc = 0;
    for (size_t t = 0; t < run.size(); ++t) {
      ExecGroup& g = e.groups[run[t]];
      if (compacted(g, sk[t])) ca.g[nc++] = CompactGroup{sk[t], g.nmaps, g.mlist.p, g.mcount.p};
    }
    if (nc > 0) {
      hipLaunchKernelGGL(k_compact_all, dim3(nc), dim3(256), 0, s0, ca);
      CRS_HIP(hipGetLastError());
    }
    MixFwdAll ma{};
    int first = 0;
    for (size_t t = 0; t < run.size(); ++t) {
      ExecGroup& g = e.groups[run[t]];
      const int nbx = (int)((g.nalm + kWorkBlock - 1) / kWorkBlock);
      ma.g[t] = MixFwdGroup{g.slots.p, g.uhat.p, g.nalm, g.lmax, nbx, first};
      first += nbx * g.nmaps;
    }
    ma.ng = (int)run.size();
    hipLaunchKernelGGL(k_mix_fwd_all, dim3((unsigned)first), dim3(256), 0, s0, in, e.dsys.p, e.dprobs.p,
                       pinv ? 1 : 0, act, ma);
    CRS_HIP(hipGetLastError());
    for (size_t t = 0; t < run.size(); ++t) transforms(run[t], sk[t], s0);
  } else {
    for (int gi : run) {
      ExecGroup& g = e.groups[gi];
      hipStream_t s = gstream[gi];
      const MapSkip skip = group_skip(g, s);
      dim3 gr((unsigned)((g.nalm + kWorkBlock - 1) / kWorkBlock), g.nmaps);
      hipLaunchKernelGGL(k_mix_fwd, gr, dim3(256), 0, s, in, e.dsys.p, e.dprobs.p, g.slots.p, pinv ? 1 : 0,
                         g.lmax, g.uhat.p, g.nalm, act);
      CRS_HIP(hipGetLastError());
      if (compacted(g, skip)) {
        hipLaunchKernelGGL(k_compact, dim3(1), dim3(256), 0, s, skip, g.nmaps, g.mlist.p, g.mcount.p);
        CRS_HIP(hipGetLastError());
      }
      transforms(gi, skip, s);
    }
  }
  for (int i = 1; i < nstr; ++i) {
    CRS_HIP(hipEventRecord(e.join[i - 1], e.side[i - 1]));
    CRS_HIP(hipStreamWaitEvent(s0, e.join[i - 1], 0));
  }
}

void exec_apply(Exec& e, OpKind kind, const double* in, double* out, hipStream_t s, const double* act,
                double* wpart) {
  const bool vm = kind == OP_A && exec_has_varmix(e);
  if (vm) exec_varmix_fwd(e, in, s, act);
  exec_bands(e, kind, in, s, act);
  if (kind == OP_PI) {
    mix_back(e, out, in, 2, 0, 1, s, act, wpart);
  } else if (!vm) {
    mix_back(e, out, in, 1, 0, 0, s, act, wpart);
  } else {
    // the varying pairs add to out after the back-mix: the fused dot follows them
    mix_back(e, out, in, 1, 0, 0, s, act, nullptr);
    exec_varmix_back(e, out, s, act);
    if (wpart) {
      hipLaunchKernelGGL(k_wl_dot, dim3(e.nwl_sys), dim3(256), 0, s, in, out, e.dsys.p, e.dprobs.p, e.wl_sys.p, act,
                         wpart);
      CRS_HIP(hipGetLastError());
    }
  }
}

void exec_diag(Exec& e, const double* r, double* z, hipStream_t s, const double* act, double* wpart) {
  CRS_CHECK(e.has_diag, CRS_EINVAL, "model was created without CRS_MODEL_DIAG");
  hipLaunchKernelGGL(k_diag_apply, dim3(e.nwl_sys), dim3(256), 0, s, r, z, e.dsys.p, e.dprobs.p, e.wl_sys.p, act,
                     wpart);
  CRS_HIP(hipGetLastError());
}

void exec_rhs_bands(Exec& e, const std::vector<std::vector<const double*>>& d,
                    const std::vector<std::vector<const double*>>& w1, hipStream_t s) {
  std::vector<std::vector<const double*>> hold;  // alive until the sync below
  hold.reserve(2 * e.groups.size());             // (references into it stay valid)
  for (auto& g : e.groups) {
    const int64_t npix = g.grid->npix;
    hold.emplace_back(g.nmaps);
    std::vector<const double*>& dp = hold.back();
    hold.emplace_back(g.nmaps);
    std::vector<const double*>& wp = hold.back();
    for (int i = 0; i < g.nmaps; ++i) {
      const SlotDev& sl = g.hslots[i];
      dp[i] = d.empty() ? nullptr : d[sl.sys][sl.band];
      wp[i] = w1.empty() ? nullptr : w1[sl.sys][sl.band];
    }
    g.dptr.upload(dp, s);
    g.wptr.upload(wp, s);
    g.pix.alloc((size_t)g.nmaps * npix);
    hipLaunchKernelGGL(k_pix_rhs, dim3(kDotBlocks, g.nmaps), dim3(256), 0, s, g.pix.p, g.tau.p, g.dptr.p,
                       g.wptr.p, npix);
    CRS_HIP(hipGetLastError());
    launch_ring(g.grid, g.lmax, RING_ADJOINT, g.nmaps, g.phase.p, g.pst, g.pix.p, nullptr, npix, nullptr, 1, s);
    launch_leg_adjoint(g.leg, leg_args(g.grid, *g.plan), g.nmaps, g.phase.p, g.pst, g.vpart.p, g.nalm,
                       (int64_t)g.nmaps * g.nalm, false, s);
  }
  // the pointer tables were uploaded from host temporaries: finish before they go
  CRS_HIP(hipStreamSynchronize(s));
}

void exec_rhs(Exec& e, const std::vector<std::vector<const double*>>& d,
              const std::vector<std::vector<const double*>>& w1, const double* w2, double* b,
              hipStream_t s) {
  exec_rhs_bands(e, d, w1, s);
  mix_back(e, b, w2, w2 ? 1 : 0, 1, 0, s);
  exec_varmix_back(e, b, s, nullptr);
}

void exec_prior_inv(Exec& e, const double* x, double* y, hipStream_t s) {
  // the back-mix with no band terms: y = C^-1 x
  hipLaunchKernelGGL(k_prior, dim3(e.nwl_rows), dim3(256), 0, s, y, x, e.dsys.p, e.dprobs.p, e.rows.p,
                     e.wl_rows.p);
  CRS_HIP(hipGetLastError());
}

// dq[r][nu][k] = sign sum_lm ( va_r,k(lm) V(sa0 + r, nu)(lm) + vb_r,k(lm) V(sb0 + r, nu)(lm) ),
// V(s, nu) = b_{nu,l} c_m f_lm sum_t vpart_nu[t][map(s, nu)]: the band-nu adjoint of system s.
void exec_mix_grad(Exec& e, const double* va, int sa0, const double* vb, int sb0, int nrhs, double sign,
                   const double* beamtab, double* dq, hipStream_t s) {
  const crs_model m = e.probs[0];
  dim3 gr(nrhs * m->nbands * m->ncomp);
  hipLaunchKernelGGL(k_dq, gr, dim3(256), 0, s, va, sa0, vb, sb0, sign, e.dsys.p, e.dprobs.p, beamtab, dq);
  CRS_HIP(hipGetLastError());
}

void exec_project(Exec& e, const double* x, const std::vector<std::vector<double*>>& maps, hipStream_t s) {
  exec_varmix_fwd(e, x, s, nullptr);
  for (auto& g : e.groups) {
    const int64_t npix = g.grid->npix;
    g.pix.alloc((size_t)g.nmaps * npix);
    dim3 gr((unsigned)((g.nalm + kWorkBlock - 1) / kWorkBlock), g.nmaps);
    hipLaunchKernelGGL(k_mix_fwd, gr, dim3(256), 0, s, x, e.dsys.p, e.dprobs.p, g.slots.p, 0, g.lmax, g.uhat.p,
                       g.nalm, (const double*)nullptr);
    CRS_HIP(hipGetLastError());
    launch_leg_synth(g.leg, leg_args(g.grid, *g.plan), g.nmaps, g.uhat.p, g.nalm, g.phase.p, g.pst, s);
    launch_ring(g.grid, g.lmax, RING_SYNTH, g.nmaps, g.phase.p, g.pst, nullptr, g.pix.p, npix, nullptr, 1, s);
    for (int i = 0; i < g.nmaps; ++i) {
      const SlotDev& sl = g.hslots[i];
      CRS_HIP(hipMemcpyAsync(maps[sl.sys][sl.band], g.pix.p + (int64_t)i * npix, npix * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    }
  }
}

// val[sys] = 1/2 x^T S^-1 x, y = S^-1 x
void exec_prior_quad(Exec& e, const double* x, double* y, double* val, hipStream_t s) {
  exec_prior_inv(e, x, y, s);
  hipLaunchKernelGGL(k_dot, vgrid(e.nsys), dim3(256), 0, s, x, y, e.dsys.p, e.partial.p, (const double*)nullptr);
  hipLaunchKernelGGL(k_scalar, dim3(e.nsys), dim3(256), 0, s, 4, e.partial.p, kDotBlocks, e.scal.p);
  hipLaunchKernelGGL(k_scal_out, dim3((e.nsys + 255) / 256), dim3(256), 0, s, e.scal.p, e.nsys, 0.5, val);
  CRS_HIP(hipGetLastError());
}

// res[sys][band] = d - P x (maps of the caller), val[sys] = sum_band res^T tau res
void exec_chi2(Exec& e, const double* x, const std::vector<std::vector<const double*>>& d,
               const std::vector<std::vector<double*>>& res, double* val, hipStream_t s) {
  exec_project(e, x, res, s);
  // per (system, band) map: kDotBlocks partials, grouped by band group
  std::vector<int2> rng;
  std::vector<std::vector<int2>> per(e.nsys);
  int64_t base = 0;
  // host pointer tables stay alive until the stream sync below
  std::vector<std::vector<const double*>> hold;
  hold.reserve(2 * e.groups.size());  // (references into it stay valid)
  for (auto& g : e.groups) {
    hold.emplace_back(g.nmaps);
    std::vector<const double*>& dp = hold.back();
    hold.emplace_back(g.nmaps);
    std::vector<const double*>& rp = hold.back();
    for (int i = 0; i < g.nmaps; ++i) {
      const SlotDev& sl = g.hslots[i];
      dp[i] = d.empty() ? nullptr : d[sl.sys][sl.band];
      rp[i] = res[sl.sys][sl.band];
      per[sl.sys].push_back(make_int2((int)(base + (int64_t)i * kDotBlocks), kDotBlocks));
    }
    g.dptr.upload(dp, s);
    g.wptr.upload(rp, s);  // the residual maps (written in place)
    base += (int64_t)g.nmaps * kDotBlocks;
  }
  e.chi2part.alloc((size_t)base);
  std::vector<int> rofs(e.nsys + 1, 0);
  for (int sy = 0; sy < e.nsys; ++sy) {
    // bands in model order
    rofs[sy + 1] = rofs[sy] + (int)per[sy].size();
    for (auto& r : per[sy]) rng.push_back(r);
  }
  base = 0;
  for (auto& g : e.groups) {
    hipLaunchKernelGGL(k_resid_chi2, dim3(kDotBlocks, g.nmaps), dim3(256), 0, s, (double* const*)g.wptr.p,
                       g.dptr.p, g.tau.p, g.grid->npix, e.chi2part.p + base);
    CRS_HIP(hipGetLastError());
    base += (int64_t)g.nmaps * kDotBlocks;
  }
  DevBuf<int2> drng;
  DevBuf<int> drofs;
  drng.upload(rng, s);
  drofs.upload(rofs, s);
  hipLaunchKernelGGL(k_sum_ranges, dim3(e.nsys), dim3(256), 0, s, e.chi2part.p, drng.p, drofs.p, 1.0, val);
  CRS_HIP(hipGetLastError());
  // the pointer tables are handle buffers; the range tables are temporaries
  CRS_HIP(hipStreamSynchronize(s));
}

// out[sys][band] = scale tau_band in[sys][band] (in NULL = zero)
void exec_noise_weight(Exec& e, double scale, const std::vector<std::vector<const double*>>& in,
                       const std::vector<std::vector<double*>>& out, hipStream_t s) {
  std::vector<std::vector<const double*>> hold;  // alive until the sync below
  hold.reserve(2 * e.groups.size());             // (references into it stay valid)
  for (auto& g : e.groups) {
    hold.emplace_back(g.nmaps);
    std::vector<const double*>& ip = hold.back();
    hold.emplace_back(g.nmaps);
    std::vector<const double*>& op = hold.back();
    for (int i = 0; i < g.nmaps; ++i) {
      const SlotDev& sl = g.hslots[i];
      ip[i] = in.empty() ? nullptr : in[sl.sys][sl.band];
      op[i] = out[sl.sys][sl.band];
    }
    g.dptr.upload(ip, s);
    g.wptr.upload(op, s);
    hipLaunchKernelGGL(k_noise_weight, dim3(kDotBlocks, g.nmaps), dim3(256), 0, s, (double* const*)g.wptr.p,
                       g.dptr.p, g.tau.p, scale, g.grid->npix);
    CRS_HIP(hipGetLastError());
  }
  CRS_HIP(hipStreamSynchronize(s));
}

namespace {

void precond_apply(Exec& e, int precond, const double* r, double* z, hipStream_t s, const double* act = nullptr) {
  if (precond == CRS_PRECOND_PINV) {
    exec_apply(e, OP_PI, r, z, s, act);
  } else if (precond == CRS_PRECOND_ADD) {
    // M_add = M_PI + M_mask (Sect. 4.2)
    exec_apply(e, OP_PI, r, z, s, act);
    exec_mask(e, r, z, true, s, act);
  } else if (precond == CRS_PRECOND_DIAG) {
    exec_diag(e, r, z, s, act);
  } else {
    hipLaunchKernelGGL(k_sub_sel, vgrid(e.nsys), dim3(256), 0, s, z, r, (const double*)nullptr, e.dsys.p,
                       (const int*)nullptr);
    CRS_HIP(hipGetLastError());
  }
}

// second half of an iteration: z = M r, rho/beta, p = z + beta p (r . z
// summed inside the preconditioner's last kernel, per work-list block)
void iter_precond(Exec& e, int precond, hipStream_t s) {
  const double* act = e.scal.p + S_ACTIVE;
  if (precond == CRS_PRECOND_PINV) {
    exec_apply(e, OP_PI, e.r.p, e.z.p, s, act, e.wpart.p);
    hipLaunchKernelGGL(k_scalar_ranges, dim3(e.nsys), dim3(256), 0, s, 1, e.wpart.p, e.rng_sys.p, e.scal.p);
  } else if (precond == CRS_PRECOND_DIAG) {
    exec_diag(e, e.r.p, e.z.p, s, act, e.wpart.p);
    hipLaunchKernelGGL(k_scalar_ranges, dim3(e.nsys), dim3(256), 0, s, 1, e.wpart.p, e.rng_sys.p, e.scal.p);
  } else if (precond == CRS_PRECOND_ADD) {
    precond_apply(e, precond, e.r.p, e.z.p, s, act);
    dot_to(e, e.r.p, e.z.p, 1, s, act);
  } else {
    precond_apply(e, precond, e.r.p, e.z.p, s, act);
    dot_to(e, e.r.p, e.z.p, 1, s, act);
  }
  hipLaunchKernelGGL(k_update_p, vgrid(e.nsys), dim3(256), 0, s, e.p.p, e.z.p, e.dsys.p, e.scal.p);
  CRS_HIP(hipGetLastError());
}

// first half: q = A p, alpha, x += alpha p, r -= alpha q, |r|^2 (the sum of
// its partials left to the caller when rr is false)
void iter_apply(Exec& e, hipStream_t s, bool rr = true) {
  exec_apply(e, OP_A, e.p.p, e.q.p, s, e.scal.p + S_ACTIVE, e.wpart.p);
  hipLaunchKernelGGL(k_scalar_ranges, dim3(e.nsys), dim3(256), 0, s, 0, e.wpart.p, e.rng_sys.p, e.scal.p);
  hipLaunchKernelGGL(k_update_xr, vgrid(e.nsys), dim3(256), 0, s, e.xw.p, e.r.p, e.p.p, e.q.p, e.dsys.p, e.scal.p,
                     e.partial.p);
  if (rr) hipLaunchKernelGGL(k_scalar, dim3(e.nsys), dim3(256), 0, s, 2, e.partial.p, kDotBlocks, e.scal.p);
  CRS_HIP(hipGetLastError());
}

hipGraphExec_t capture(Exec& e, hipStream_t cs, const std::function<void()>& body,
                       std::vector<ProfRecord>& recs) {
  (void)prof_take_captured();
  CRS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  try {
    body();
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(cs, &g);
    if (g) (void)hipGraphDestroy(g);
    auto left = prof_take_captured();
    prof_release(left);
    throw;
  }
  hipGraph_t g = nullptr;
  CRS_HIP(hipStreamEndCapture(cs, &g));
  recs = prof_take_captured();
  hipGraphExec_t ge = nullptr;
  const hipError_t err = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (err != hipSuccess) {
    prof_release(recs);
    throw Error{CRS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(err)};
  }
  (void)e;
  return ge;
}

}  // namespace

namespace {

// Start of iteration j of a chunk: row[i] = 0 if system i is active, else -1.
__global__ void k_chunk_start(const double* __restrict__ scal, double* __restrict__ row, int nsys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsys) row[i] = scal[i * kScal + S_ACTIVE] != 0.0 ? 0.0 : -1.0;
}

// End of iteration j of a chunk for system i: row[i] = |r|^2 of a system
// that ran the iteration (-2 if it broke down in it); a system whose
// recursive residual passes rtol stops (inactive for the rest of the chunk)
// and becomes a candidate for the host's true-residual check.
__device__ __forceinline__ void chunk_check(double* __restrict__ st, double bbi, double rtol2,
                                            double* __restrict__ rowi, double* __restrict__ candi) {
  if (*rowi < 0.0) return;
  if (st[S_ACTIVE] == 0.0) {
    *rowi = -2.0;
    return;
  }
  const double rr = st[S_RR];
  if (!isfinite(rr)) {
    st[S_BREAK] = 1.0;
    st[S_ACTIVE] = 0.0;
    *rowi = -2.0;
    return;
  }
  *rowi = rr;
  if (rr <= rtol2 * bbi) {
    st[S_ACTIVE] = 0.0;
    *candi = 1.0;
  }
}

// The |r|^2 sum of k_scalar, the check above and, when next is given, the next
// iteration's k_chunk_start in one launch (one block per system).
__global__ __launch_bounds__(256) void k_iter_end(const double* __restrict__ partial, int nblk,
                                                  double* __restrict__ scal, const double* __restrict__ bb,
                                                  double rtol2, double* __restrict__ row,
                                                  double* __restrict__ next, double* __restrict__ cand) {
  const int sy = blockIdx.x;
  const double s = sum_partials(partial, (int64_t)sy * nblk, nblk);
  if (threadIdx.x == 0) {
    double* st = scal + sy * kScal;
    scalar_op(2, s, st);
    chunk_check(st, bb[sy], rtol2, row + sy, cand + sy);
    if (next) next[sy] = st[S_ACTIVE] != 0.0 ? 0.0 : -1.0;
  }
}

}  // namespace

Exec::GraphEntry::~GraphEntry() {
  if (exec) (void)hipGraphExecDestroy(exec);
  prof_release(prof);
}

int exec_pcg(Exec& e, int precond, const double* b, double* x, double rtol, int maxiter, int* iters,
             double* relres, double* history, bool use_graph, hipStream_t s) {
  CRS_CHECK(precond == CRS_PRECOND_NONE || precond == CRS_PRECOND_DIAG || precond == CRS_PRECOND_PINV ||
                precond == CRS_PRECOND_ADD,
            CRS_EINVAL, "unknown preconditioner");
  CRS_CHECK(precond != CRS_PRECOND_DIAG || e.has_diag, CRS_EINVAL, "model was created without CRS_MODEL_DIAG");
  CRS_CHECK(precond != CRS_PRECOND_ADD || exec_has_mask(e), CRS_EINVAL,
            "M_add needs a mask preconditioner on every model (crs_model_set_mask)");
  CRS_CHECK(rtol > 0.0 && maxiter >= 0, CRS_EINVAL, "rtol must be > 0 and maxiter >= 0");
  const int ns = e.nsys;
  const int ng = (int)e.groups.size();
  const size_t bytes = (size_t)e.ntot * sizeof(double);
  e.stats = ExecStats{};
  if (precond == CRS_PRECOND_ADD) exec_mask_prepare(e, s);
  // scalars and flags go through pinned host memory (plain DMA transfers)
  double* const hs = e.hscal;
  const size_t hsb = (size_t)ns * kScal * sizeof(double);
  std::vector<double> bb(ns);
  std::fill(hs, hs + (size_t)ns * kScal, 0.0);
  for (int i = 0; i < ns; ++i) hs[i * kScal + S_ACTIVE] = 1.0;
  CRS_HIP(hipMemcpyAsync(e.scal.p, hs, hsb, hipMemcpyHostToDevice, s));
  std::fill(e.live.begin(), e.live.end(), 1);
  // |b|^2
  dot_to(e, b, b, 4, s);
  CRS_HIP(hipMemcpyAsync(hs, e.scal.p, hsb, hipMemcpyDeviceToHost, s));
  CRS_HIP(hipStreamSynchronize(s));
  std::vector<int> active(ns, 1), status(ns, 0), it_used(ns, 0), sel(ns, 0);
  for (int i = 0; i < ns; ++i) {
    bb[i] = hs[i * kScal + S_TMP];
    if (!(bb[i] > 0.0)) active[i] = 0;  // b = 0: x = 0 is the solution
  }
  CRS_HIP(hipMemcpyAsync(e.xw.p, x, bytes, hipMemcpyDeviceToDevice, s));
  for (int i = 0; i < ns; ++i)
    if (!active[i]) CRS_HIP(hipMemsetAsync(e.xw.p + e.hsys[i].off, 0, e.hsys[i].n * sizeof(double), s));
  // r = b - A x, z = M r, p = z, rho = r.z
  exec_apply(e, OP_A, e.xw.p, e.q.p, s);
  hipLaunchKernelGGL(k_sub_sel, vgrid(ns), dim3(256), 0, s, e.r.p, b, e.q.p, e.dsys.p, (const int*)nullptr);
  precond_apply(e, precond, e.r.p, e.z.p, s);
  CRS_HIP(hipMemcpyAsync(e.p.p, e.z.p, bytes, hipMemcpyDeviceToDevice, s));
  for (int i = 0; i < ns; ++i) hs[i * kScal + S_ACTIVE] = active[i];
  CRS_HIP(hipMemcpyAsync(e.scal.p, hs, hsb, hipMemcpyHostToDevice, s));
  dot_to(e, e.r.p, e.z.p, 3, s);
  CRS_HIP(hipMemcpyAsync(hs, e.scal.p, hsb, hipMemcpyDeviceToHost, s));
  CRS_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < ns; ++i)
    if (active[i] && hs[i * kScal + S_ACTIVE] == 0.0) {
      active[i] = 0;
      status[i] = hs[i * kScal + S_BREAK] != 0.0 ? 2 : 0;  // r = 0 (x0 exact) counts as converged
    }
  const bool prof = prof_enabled();
  auto any_active = [&] {
    for (int i = 0; i < ns; ++i)
      if (active[i]) return true;
    return false;
  };
  auto mirror = [&](const std::vector<int>& flags) {
    for (int i = 0; i < ns; ++i) e.hact[i] = flags[i] ? 1 : 0;
  };
  // true residual of the systems sel marks: the ones within rtol finish, the
  // others restart from their iterate (r = b - A x, beta = 0)
  auto true_residual_check = [&] {
    std::vector<double> cflag((size_t)ns * kScal, 0.0);  // lives past the sync that ends this block
    for (int i = 0; i < ns; ++i) cflag[(size_t)i * kScal] = sel[i] ? 1.0 : 0.0;
    CRS_HIP(hipMemcpyAsync(e.cand.p, cflag.data(), hsb, hipMemcpyHostToDevice, s));
    mirror(sel);
    exec_apply(e, OP_A, e.xw.p, e.q.p, s, e.cand.p);
    hipLaunchKernelGGL(k_sub_sel, vgrid(ns), dim3(256), 0, s, e.t.p, b, e.q.p, e.dsys.p, (const int*)nullptr);
    dot_to(e, e.t.p, e.t.p, 4, s);
    CRS_HIP(hipMemcpyAsync(hs, e.scal.p, hsb, hipMemcpyDeviceToHost, s));
    CRS_HIP(hipStreamSynchronize(s));
    ++e.stats.host_syncs;
    bool restart = false;
    for (int i = 0; i < ns; ++i) {
      if (!sel[i]) continue;
      if (std::sqrt(hs[i * kScal + S_TMP] / bb[i]) <= rtol) {
        active[i] = 0;
        status[i] = 0;
        sel[i] = 0;
      } else {
        active[i] = 1;
        restart = true;  // keep sel[i] = 1: restart from the true residual
      }
    }
    for (int i = 0; i < ns; ++i) {
      hs[i * kScal + S_ACTIVE] = active[i];
      hs[i * kScal + S_RESTART] = sel[i];
    }
    CRS_HIP(hipMemcpyAsync(e.scal.p, hs, hsb, hipMemcpyHostToDevice, s));
    if (restart) {
      std::copy(sel.begin(), sel.end(), e.hsel);
      CRS_HIP(hipMemcpyAsync(e.dsel.p, e.hsel, ns * sizeof(int), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_sub_sel, vgrid(ns), dim3(256), 0, s, e.r.p, e.t.p, (const double*)nullptr, e.dsys.p,
                         e.dsel.p);
      CRS_HIP(hipGetLastError());
    }
    CRS_HIP(hipStreamSynchronize(s));
  };
  int it = 0;
  if (!use_graph) {
    // one iteration at a time, the host deciding after each
    while (any_active() && it < maxiter) {
      ++it;
      mirror(active);
      if (it > 1) iter_precond(e, precond, s);
      iter_apply(e, s);
      CRS_HIP(hipMemcpyAsync(hs, e.scal.p, hsb, hipMemcpyDeviceToHost, s));
      CRS_HIP(hipStreamSynchronize(s));
      ++e.stats.host_syncs;
      bool cand = false;
      for (int i = 0; i < ns; ++i) {
        sel[i] = 0;
        if (!active[i]) continue;
        if (hs[i * kScal + S_BREAK] != 0.0) {
          active[i] = 0;
          status[i] = 2;
          it_used[i] = it;
          continue;
        }
        const double rel = std::sqrt(hs[i * kScal + S_RR] / bb[i]);
        if (history) history[(size_t)(it - 1) * ns + i] = rel;
        it_used[i] = it;
        if (!std::isfinite(rel)) {
          active[i] = 0;
          status[i] = 2;
          continue;
        }
        if (rel <= rtol) {
          sel[i] = 1;
          cand = true;
        }
      }
      if (cand) true_residual_check();
    }
  } else {
    // chunks of up to kChunk iterations per graph launch: each iteration
    // records its residuals and stops converged systems on the device; the
    // host reads the flags between chunks, checks the candidates' true
    // residuals and restarts the ones that fail.  Groups whose systems have
    // all finished are left out of the captured chunk (a new graph is
    // captured when that set changes; graphs are kept per key for reuse).
    if (!e.cap_stream) CRS_HIP(hipStreamCreateWithFlags(&e.cap_stream, hipStreamNonBlocking));
    hipStream_t cs = e.cap_stream;
    e.bbdev.upload(bb, s);
    std::vector<double> hrow((size_t)kChunk * ns), hcand(ns);
    auto get_graph = [&](bool first, int k) -> Exec::GraphEntry& {
      uint64_t mask = 0;
      for (int gi = 0; gi < ng && gi < 64; ++gi)
        if (e.live[gi]) mask |= uint64_t(1) << gi;
      const auto key = std::make_tuple((precond * 2 + (prof ? 1 : 0)) * 16 + e.nstreams, first ? 1 : 0, k, mask);
      auto itg = e.graphs.find(key);
      if (itg != e.graphs.end() && itg->second->rtol == rtol) return *itg->second;
      auto ge = std::make_unique<Exec::GraphEntry>();
      ge->rtol = rtol;
      const double rtol2 = rtol * rtol;
      auto body = [&] {
        // each iteration ends with one kernel that sums |r|^2, checks the
        // systems and opens the next iteration's row
        hipLaunchKernelGGL(k_chunk_start, dim3((ns + 255) / 256), dim3(256), 0, cs, e.scal.p, e.hrows.p, ns);
        for (int j = 0; j < k; ++j) {
          double* row = e.hrows.p + (size_t)j * ns;
          e.chunk_iter = j;
          if (!(first && j == 0)) iter_precond(e, precond, cs);
          iter_apply(e, cs, false);
          hipLaunchKernelGGL(k_iter_end, dim3(ns), dim3(256), 0, cs, e.partial.p, kDotBlocks, e.scal.p, e.bbdev.p,
                             rtol2, row, j + 1 < k ? row + ns : nullptr, e.dcand.p);
          CRS_HIP(hipGetLastError());
        }
        e.chunk_iter = 0;
      };
      try {
        ge->exec = capture(e, cs, body, ge->prof);
      } catch (const Error&) {
        if (!prof) throw;
        // the runtime refused event records inside the capture: capture
        // without them (kernel timing is then unavailable inside graphs)
        (void)hipGetLastError();
        prof_disable_in_graphs();
        ge->exec = capture(e, cs, body, ge->prof);
      }
      ++e.stats.graph_captures;
      auto& ref = *ge;
      e.graphs[key] = std::move(ge);
      return ref;
    };
    while (any_active() && it < maxiter) {
      const int k = std::min(kChunk, maxiter - it);
      const bool first = it == 0;
      // live groups: those with an active system
      for (int gi = 0; gi < ng; ++gi) {
        e.live[gi] = 0;
        for (const SlotDev& sl : e.groups[gi].hslots)
          if (active[sl.sys]) {
            e.live[gi] = 1;
            break;
          }
      }
      Exec::GraphEntry& ge = get_graph(first, k);
      std::fill(hcand.begin(), hcand.end(), 0.0);
      CRS_HIP(hipMemcpyAsync(e.dcand.p, hcand.data(), ns * sizeof(double), hipMemcpyHostToDevice, s));
      CRS_HIP(hipGraphLaunch(ge.exec, s));
      ++e.stats.graph_launches;
      CRS_HIP(hipMemcpyAsync(hs, e.scal.p, hsb, hipMemcpyDeviceToHost, s));
      CRS_HIP(hipMemcpyAsync(hrow.data(), e.hrows.p, (size_t)k * ns * sizeof(double), hipMemcpyDeviceToHost, s));
      CRS_HIP(hipMemcpyAsync(hcand.data(), e.dcand.p, ns * sizeof(double), hipMemcpyDeviceToHost, s));
      CRS_HIP(hipStreamSynchronize(s));
      ++e.stats.host_syncs;
      if (prof)
        prof_account(ge.prof, [&](const ProfRecord& r) {
          if (r.tag < 0) return r.work;
          // tag = (chunk iteration, M_PI flag, group): the systems that ran that iteration
          const int j = r.tag / 2048, pi = (r.tag / 1024) & 1, gi = r.tag % 1024;
          for (int i = 0; i < ns; ++i) e.hact[i] = hrow[(size_t)j * ns + i] != -1.0 ? 1 : 0;
          return group_work(e, gi, r.family, true, pi != 0);
        });
      bool cand = false;
      for (int i = 0; i < ns; ++i) {
        sel[i] = 0;
        if (!active[i]) continue;
        for (int j = 0; j < k; ++j) {
          const double v = hrow[(size_t)j * ns + i];
          if (v == -1.0) break;
          it_used[i] = it + j + 1;
          if (v >= 0.0 && history) history[(size_t)(it + j) * ns + i] = std::sqrt(v / bb[i]);
        }
        if (hs[i * kScal + S_BREAK] != 0.0) {
          active[i] = 0;
          status[i] = 2;
          continue;
        }
        if (hcand[i] != 0.0) {
          active[i] = 0;
          sel[i] = 1;
          cand = true;
        }
      }
      it += k;
      if (cand) true_residual_check();
    }
    it = 0;
    for (int i = 0; i < ns; ++i) it = std::max(it, it_used[i]);
  }
  e.stats.iterations = it;
  for (int i = 0; i < ns; ++i)
    if (active[i]) status[i] = 1;  // maxiter
  // final true residuals
  exec_apply(e, OP_A, e.xw.p, e.q.p, s);
  hipLaunchKernelGGL(k_sub_sel, vgrid(ns), dim3(256), 0, s, e.t.p, b, e.q.p, e.dsys.p, (const int*)nullptr);
  dot_to(e, e.t.p, e.t.p, 4, s);
  CRS_HIP(hipMemcpyAsync(hs, e.scal.p, hsb, hipMemcpyDeviceToHost, s));
  CRS_HIP(hipMemcpyAsync(x, e.xw.p, bytes, hipMemcpyDeviceToDevice, s));
  CRS_HIP(hipStreamSynchronize(s));
  int ret = CRS_OK;
  for (int i = 0; i < ns; ++i) {
    if (iters) iters[i] = it_used[i];
    if (relres) relres[i] = bb[i] > 0 ? std::sqrt(hs[i * kScal + S_TMP] / bb[i]) : 0.0;
    if (status[i] == 2) ret = CRS_EBREAKDOWN;
    else if (status[i] == 1 && ret == CRS_OK) ret = CRS_ENOTCONV;
  }
  if (ret == CRS_EBREAKDOWN) set_error(ret, "PCG breakdown (p.Ap <= 0, r.z <= 0 or non-finite)");
  if (ret == CRS_ENOTCONV) set_error(ret, "PCG reached maxiter");
  return ret;
}

}  // namespace crs
