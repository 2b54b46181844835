// The constrained-realization system and its solver (gfx950, float64).
//
//   A = S^-1 + sum_nu P_nu^T N_nu^-1 P_nu           (Sect. 2.3, eq:A)
//   P_nu = Y_nu B_nu q_{nu,k}                        (eq:P, Q~ = q I, Sect. 3.3)
//   M_PI = U^+ T^+ (U^+)^T                            (eq:fullmodel-preconditioner)
//   M_diag = (U^T diag(T) U)^-1                       (Sect. 5)
//   PCG on A x = b                                    (Sect. 2.3)
//   b = sum_nu P_nu^T (tau d + tau^1/2 w1) + S^-1/2 w2 (Sect. 2.3)
//
// Both A and M_PI have the same shape: a per-l component->band mix, one SHT
// round trip per band with a pixel weight, and a per-l band->component mix
// plus a per-l component->component term.  Bands sharing (grid, L_nu) form
// a group whose Legendre launches carry all of the group's bands and
// right-hand sides as maps.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace crs {
LegArgs leg_args(crs_grid g, ShtPlan& p);
RingArgs ring_args(crs_grid g, int lmax);
double leg_flops(const ShtPlan& p, int nmaps);
double ring_bytes(crs_grid g, int lmax, int nmaps, int mode);
}  // namespace crs

namespace {
using namespace crs;

constexpr int kDotBlocks = 256;

struct Band {
  crs_grid grid = nullptr;
  int lmax = 0;
  int64_t npix = 0;
  std::vector<double> beam, q, tau_host, w_host;
  DevBuf<double> tau, tplus;
  double alpha2 = 0;
  int group = 0, gidx = 0;
};

struct Group {
  crs_grid grid = nullptr;
  int lmax = 0;
  std::vector<int> bands;
  ShtPlan* plan = nullptr;
  int ntiles = 1;
  int64_t nalm = 0, pst = 0;
  DevBuf<double> uhat, vpart, pix;
  DevBuf<double2> phase;
  DevBuf<const double*> wA, wP;  // per band in group: tau, alpha^2 w^2 tau^+
  DevBuf<int> bandids;
};

__host__ __device__ inline int64_t moff_h(int L, int m) {
  return (m == 0) ? 0 : (int64_t)(L + 1) + 2 * ((int64_t)(m - 1) * (L + 1) - (int64_t)(m - 1) * m / 2);
}
__host__ __device__ inline int64_t tri_h(int L, int m) { return (int64_t)m * (L + 1) - (int64_t)m * (m - 1) / 2; }

}  // namespace

struct crs_model_s {
  int ncomp = 0, nbands = 0;
  std::vector<int> lk;
  std::vector<std::vector<double>> invcl;
  std::vector<int64_t> coff;
  int64_t n = 0;
  int Lc = 0, Lmax = 0;
  std::vector<Band> bands;
  std::vector<Group> groups;
  bool has_diag = false;
  // per-l tables
  DevBuf<double> cA, cP;        // [Lmax+1][nb][nc]
  DevBuf<double> dInv, dSqrt;   // [Lmax+1][nc] diagonal prior terms
  DevBuf<double> dPi;           // [Lmax+1][nc][nc]
  DevBuf<double> ftab;          // f_lm triangle at Lmax
  DevBuf<double> Dinv;          // [(Lc+1)^2][nc][nc]
  DevBuf<int> d_lk;
  DevBuf<int64_t> d_coff;
  // band views for the back-mix
  DevBuf<const double*> d_vptr;
  DevBuf<int> d_binfo;  // per band: L, gsize, gidx, ntiles
  std::vector<double> upinv;  // host copy [Lmax+1][nc][nb+nc]
  // workspaces
  int nrhs_ws = 0;
  DevBuf<double> r, z, p, q, t;
  DevBuf<double> partial;
  DevBuf<double> scal;  // per rhs: rho, alpha, beta, rr, bb, flags...
  DevBuf<double> om1, om2, bcr;
  DevBuf<int> dsel;
  int device = 0;
};

namespace {

// ---------------------------------------------------------------- kernels
// out_hat[map][i] = c_m f_lm * sum_k coef[l][band][k] * x[rhs][coff_k + idx_k]
__global__ void k_mix_fwd(const double* __restrict__ x, int64_t n, int nrhs, int nc,
                          const int* __restrict__ lk, const int64_t* __restrict__ coff,
                          const double* __restrict__ coef, int nb, const int* __restrict__ bandids,
                          int Lb, const double* __restrict__ ftab, int Lf,
                          double* __restrict__ uhat, int64_t nalm) {
  const int m = blockIdx.y;
  const int map = blockIdx.z;  // = gidx * nrhs + rhs
  const int gidx = map / nrhs, rhs = map % nrhs;
  const int band = bandids[gidx];
  const int nsl = Lb - m + 1;
  const int np = (m == 0) ? 1 : 2;
  const double cm = (m == 0) ? 1.0 : 1.4142135623730951;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np * nsl; i += gridDim.x * blockDim.x) {
    const int part = i / nsl, ll = i % nsl, l = m + ll;
    double acc = 0.0;
    for (int k = 0; k < nc; ++k) {
      const int L = lk[k];
      if (l > L) continue;
      const double c = coef[((int64_t)l * nb + band) * nc + k];
      const int64_t idx = coff[k] + moff_h(L, m) + (int64_t)part * (L - m + 1) + ll;
      acc = fma(c, x[(int64_t)rhs * n + idx], acc);
    }
    uhat[(int64_t)map * nalm + moff_h(Lb, m) + i] = cm * ftab[tri_h(Lf, m) + ll] * acc;
  }
}

// y[rhs][coff_k + idx_k] = diag-term + sum_nu coef[l][nu][k] c_m f_lm sum_t vpart_nu[t][map][idx_nu]
// binfo per band: {L, gsize, gidx, ntiles}
__global__ void k_mix_back(double* __restrict__ y, const double* __restrict__ din, int64_t n, int nrhs,
                           int nc, const int* __restrict__ lk, const int64_t* __restrict__ coff,
                           const double* __restrict__ coef, int nb,
                           const double* const* __restrict__ vptr, const int* __restrict__ binfo,
                           int dmode, const double* __restrict__ dtab, const double* __restrict__ ftab,
                           int Lf, int Lc) {
  const int m = blockIdx.y;
  const int k = blockIdx.z % nc;
  const int rhs = blockIdx.z / nc;
  const int Lk = lk[k];
  if (m > Lk) return;
  const int nsl = Lk - m + 1;
  const int np = (m == 0) ? 1 : 2;
  const double cm = (m == 0) ? 1.0 : 1.4142135623730951;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np * nsl; i += gridDim.x * blockDim.x) {
    const int part = i / nsl, ll = i % nsl, l = m + ll;
    double acc = 0.0;
    if (dmode == 1) {
      acc = dtab[(int64_t)l * nc + k] * din[(int64_t)rhs * n + coff[k] + moff_h(Lk, m) + i];
    } else if (dmode == 2) {
      for (int kp = 0; kp < nc; ++kp) {
        const int Lp = lk[kp];
        if (l > Lp) continue;
        acc = fma(dtab[((int64_t)l * nc + k) * nc + kp],
                  din[(int64_t)rhs * n + coff[kp] + moff_h(Lp, m) + (int64_t)part * (Lp - m + 1) + ll], acc);
      }
    }
    const double fs = cm * ftab[tri_h(Lf, m) + ll];
    for (int nu = 0; nu < nb; ++nu) {
      const int L = binfo[4 * nu + 0];
      if (l > L) continue;
      const int gsize = binfo[4 * nu + 1], gidx = binfo[4 * nu + 2], nt = binfo[4 * nu + 3];
      const int64_t nalm = (int64_t)(L + 1) * (L + 1);
      const int64_t tstride = (int64_t)gsize * nrhs * nalm;
      const double* v = vptr[nu] + (int64_t)(gidx * nrhs + rhs) * nalm + moff_h(L, m) +
                        (int64_t)part * (L - m + 1) + ll;
      double s = 0.0;
      for (int t = 0; t < nt; ++t) s += v[t * tstride];
      acc = fma(coef[((int64_t)l * nb + nu) * nc + k] * fs, s, acc);
    }
    y[(int64_t)rhs * n + coff[k] + moff_h(Lk, m) + i] = acc;
  }
}

// z[rhs][coff_k + idx] = sum_k' Dinv[u][k][k'] r[rhs][coff_k' + idx'] over active k'
__global__ void k_diag_apply(const double* __restrict__ r, double* __restrict__ z, int64_t n, int nc,
                             const int* __restrict__ lk, const int64_t* __restrict__ coff,
                             const double* __restrict__ Dinv, int Lc) {
  const int m = blockIdx.y;
  const int rhs = blockIdx.z;
  const int nsl = Lc - m + 1;
  const int np = (m == 0) ? 1 : 2;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np * nsl; i += gridDim.x * blockDim.x) {
    const int part = i / nsl, ll = i % nsl, l = m + ll;
    const int64_t u = moff_h(Lc, m) + i;
    double rv[8];
    for (int k = 0; k < nc; ++k) {
      const int L = lk[k];
      rv[k] = (l <= L) ? r[(int64_t)rhs * n + coff[k] + moff_h(L, m) + (int64_t)part * (L - m + 1) + ll] : 0.0;
    }
    for (int k = 0; k < nc; ++k) {
      const int L = lk[k];
      if (l > L) continue;
      double acc = 0.0;
      for (int kp = 0; kp < nc; ++kp) acc = fma(Dinv[(u * nc + k) * nc + kp], rv[kp], acc);
      z[(int64_t)rhs * n + coff[k] + moff_h(L, m) + (int64_t)part * (L - m + 1) + ll] = acc;
    }
  }
}

// partial[rhs][blk] = sum over this block's slice of a[rhs][i] * b[rhs][i]
__global__ __launch_bounds__(256) void k_dot(const double* __restrict__ a, const double* __restrict__ b,
                                             int64_t n, double* __restrict__ partial) {
  __shared__ double red[4];
  const int rhs = blockIdx.y;
  const double* pa = a + (int64_t)rhs * n;
  const double* pb = b + (int64_t)rhs * n;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    acc = fma(pa[i], pb[i], acc);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[(int64_t)rhs * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Per-rhs scalar state, layout scal[rhs * 8 + field].
enum { S_RHO = 0, S_ALPHA = 1, S_BETA = 2, S_RR = 3, S_ACTIVE = 4, S_BREAK = 5, S_RESTART = 6, S_TMP = 7 };

// op 0: alpha = rho / p.q ; op 1: beta = r.z / rho, rho = r.z ; op 2: rr = sum ;
// op 3: rho = r.z (start) ; op 4: tmp = sum
__global__ __launch_bounds__(256) void k_scalar(int op, const double* __restrict__ partial, int nblk,
                                                int nrhs, double* __restrict__ scal) {
  // one block per rhs: fixed-order tree sum of the block partials
  __shared__ double red[256];
  const int rhs = blockIdx.x;
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) v += partial[(int64_t)rhs * nblk + i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double s = red[0];
  double* st = scal + rhs * 8;
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
                                                   int64_t n, const double* __restrict__ scal,
                                                   double* __restrict__ partial) {
  __shared__ double red[4];
  const int rhs = blockIdx.y;
  const double al = scal[rhs * 8 + S_ALPHA];
  double* px = x + (int64_t)rhs * n;
  double* pr = r + (int64_t)rhs * n;
  const double* pp = p + (int64_t)rhs * n;
  const double* pq = q + (int64_t)rhs * n;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (al != 0.0) {
      px[i] = fma(al, pp[i], px[i]);
      pr[i] = fma(-al, pq[i], pr[i]);
    }
    const double v = pr[i];
    acc = fma(v, v, acc);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[(int64_t)rhs * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// p = z + beta p (active rhs only)
__global__ void k_update_p(double* __restrict__ p, const double* __restrict__ z, int64_t n,
                           const double* __restrict__ scal) {
  const int rhs = blockIdx.y;
  const double* st = scal + rhs * 8;
  if (st[S_ACTIVE] == 0.0) return;
  const double be = st[S_BETA];
  double* pp = p + (int64_t)rhs * n;
  const double* pz = z + (int64_t)rhs * n;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    pp[i] = fma(be, pp[i], pz[i]);
}

// out = a - b (per rhs, only where mask rhs flag selects; mask == null: all)
__global__ void k_sub(double* __restrict__ out, const double* __restrict__ a, const double* __restrict__ b,
                      int64_t n, const int* __restrict__ sel) {
  const int rhs = blockIdx.y;
  if (sel && !sel[rhs]) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[(int64_t)rhs * n + i] = a[(int64_t)rhs * n + i] - b[(int64_t)rhs * n + i];
}

__global__ void k_copy_sel(double* __restrict__ out, const double* __restrict__ a, int64_t n,
                           const int* __restrict__ sel) {
  const int rhs = blockIdx.y;
  if (sel && !sel[rhs]) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[(int64_t)rhs * n + i] = a[(int64_t)rhs * n + i];
}

// f = tau d + sqrt(tau) w1 for one band's maps (rhs-major)
__global__ void k_pix_rhs(double* __restrict__ f, const double* __restrict__ tau,
                          const double* __restrict__ d, const double* __restrict__ w1, int64_t npix) {
  const int rhs = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npix; i += (int64_t)gridDim.x * 256) {
    const double t = tau[i];
    double v = 0.0;
    if (d) v = t * d[(int64_t)rhs * npix + i];
    if (w1) v = fma(sqrt(t), w1[(int64_t)rhs * npix + i], v);
    f[(int64_t)rhs * npix + i] = v;
  }
}

// Philox4x64-10 (Salmon et al. SC'11) and Box-Muller normals.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ void k_philox_normals(uint64_t seed, uint64_t stream, uint64_t rhs0, int64_t n,
                                 double* __restrict__ out) {
  const uint64_t rhs = rhs0 + blockIdx.y;
  double* o = out + (int64_t)blockIdx.y * n;
  const int64_t nblk = (n + 3) / 4;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblk; b += (int64_t)gridDim.x * blockDim.x) {
    uint64_t c[4] = {(uint64_t)b, rhs, 0ull, 0ull};
    philox4x64_10(c, seed, stream);
    double u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = ((double)(c[i] >> 11) + 0.5) * 0x1p-53;
    double v[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double rad = sqrt(-2.0 * log(u[2 * h]));
      double sv, cv;
      sincospi(2.0 * u[2 * h + 1], &sv, &cv);
      v[2 * h] = rad * cv;
      v[2 * h + 1] = rad * sv;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * b + i < n) o[4 * b + i] = v[i];
  }
}

inline dim3 vgrid(int64_t n, int nrhs) {
  int64_t nb = (n + 255) / 256;
  if (nb > kDotBlocks) nb = kDotBlocks;
  if (nb < 1) nb = 1;
  return dim3((unsigned)nb, nrhs);
}

// ------------------------------------------------------------ host helpers
// Pseudo-inverse of a small m x n matrix (row-major) by one-sided Jacobi SVD.
void small_pinv(const std::vector<double>& A, int m, int n, std::vector<double>& P) {
  std::vector<double> U(A), V((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double al = 0, be = 0, ga = 0;
        for (int i = 0; i < m; ++i) {
          al += U[i * n + p] * U[i * n + p];
          be += U[i * n + q] * U[i * n + q];
          ga += U[i * n + p] * U[i * n + q];
        }
        if (ga == 0.0 || std::fabs(ga) <= 1e-17 * std::sqrt(al * be)) continue;
        off = std::max(off, std::fabs(ga) / std::sqrt(al * be));
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < m; ++i) {
          double up = U[i * n + p], uq = U[i * n + q];
          U[i * n + p] = c * up - s * uq;
          U[i * n + q] = s * up + c * uq;
        }
        for (int i = 0; i < n; ++i) {
          double vp = V[i * n + p], vq = V[i * n + q];
          V[i * n + p] = c * vp - s * vq;
          V[i * n + q] = s * vp + c * vq;
        }
      }
    if (off < 1e-16) break;
  }
  std::vector<double> sig(n);
  double smax = 0;
  for (int j = 0; j < n; ++j) {
    double s2 = 0;
    for (int i = 0; i < m; ++i) s2 += U[i * n + j] * U[i * n + j];
    sig[j] = std::sqrt(s2);
    smax = std::max(smax, sig[j]);
  }
  P.assign((size_t)n * m, 0.0);
  const double tol = smax * 1e-13 * std::max(m, n);
  for (int l = 0; l < n; ++l) {
    if (sig[l] <= tol || sig[l] == 0.0) continue;
    const double inv2 = 1.0 / (sig[l] * sig[l]);  // u_l = U[:, l] / sig_l
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < m; ++i) P[(size_t)j * m + i] += V[j * n + l] * inv2 * U[i * n + l];
  }
}

void build_ftab(crs_model m, hipStream_t s) {
  const int L = m->Lmax;
  int64_t ntri = (int64_t)(L + 1) * (L + 2) / 2;
  std::vector<double> ft(ntri, 0.0);
  for (int mm = 0; mm <= L; ++mm) {
    int64_t o = tri_h(L, mm) - mm;
    ft[o + mm] = 1.0;
    if (mm + 1 <= L) ft[o + mm + 1] = 1.0;
    for (int l = mm + 2; l <= L; ++l) {
      double dl = l, dm = mm;
      double a = std::sqrt((4.0 * dl * dl - 1.0) / ((dl - dm) * (dl + dm)));
      double b = std::sqrt(((dl - 1.0 - dm) * (dl - 1.0 + dm)) / (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
      ft[o + l] = a * b * ft[o + l - 2];
    }
  }
  m->ftab.upload(ft, s);
}

// U_l^+ and the derived device tables (cP, dPi); alpha must be set.
void build_pinv_tables(crs_model m, hipStream_t s) {
  const int nb = m->nbands, nc = m->ncomp, L = m->Lmax;
  const int rows = nb + nc;
  m->upinv.assign((size_t)(L + 1) * nc * rows, 0.0);
  std::vector<double> cP((size_t)(L + 1) * nb * nc, 0.0), dPi((size_t)(L + 1) * nc * nc, 0.0);
  for (int l = 0; l <= L; ++l) {
    std::vector<int> act;
    for (int k = 0; k < nc; ++k)
      if (l <= m->lk[k]) act.push_back(k);
    if (act.empty()) continue;
    const int na = (int)act.size();
    std::vector<double> U((size_t)rows * na, 0.0), P;
    for (int ja = 0; ja < na; ++ja) {
      const int k = act[ja];
      for (int nu = 0; nu < nb; ++nu)
        if (l <= m->bands[nu].lmax)
          U[(size_t)nu * na + ja] = std::sqrt(m->bands[nu].alpha2) * m->bands[nu].beam[l] * m->bands[nu].q[k];
      U[(size_t)(nb + k) * na + ja] = std::sqrt(m->invcl[k][l]);
    }
    small_pinv(U, rows, na, P);  // P: na x rows
    for (int ja = 0; ja < na; ++ja)
      for (int i = 0; i < rows; ++i) m->upinv[((size_t)l * nc + act[ja]) * rows + i] = P[(size_t)ja * rows + i];
    for (int k = 0; k < nc; ++k)
      for (int nu = 0; nu < nb; ++nu)
        cP[((size_t)l * nb + nu) * nc + k] = m->upinv[((size_t)l * nc + k) * rows + nu];
    for (int k = 0; k < nc; ++k)
      for (int kp = 0; kp < nc; ++kp) {
        double acc = 0;
        for (int j = 0; j < nc; ++j)
          acc += m->upinv[((size_t)l * nc + k) * rows + nb + j] * m->upinv[((size_t)l * nc + kp) * rows + nb + j];
        dPi[((size_t)l * nc + k) * nc + kp] = acc;
      }
  }
  m->cP.upload(cP, s);
  m->dPi.upload(dPi, s);
}

void build_mix_tables(crs_model m, hipStream_t s) {
  const int nb = m->nbands, nc = m->ncomp, L = m->Lmax;
  std::vector<double> cA((size_t)(L + 1) * nb * nc, 0.0), di((size_t)(L + 1) * nc, 0.0), ds(di.size(), 0.0);
  for (int l = 0; l <= L; ++l) {
    for (int nu = 0; nu < nb; ++nu)
      if (l <= m->bands[nu].lmax)
        for (int k = 0; k < nc; ++k) cA[((size_t)l * nb + nu) * nc + k] = m->bands[nu].beam[l] * m->bands[nu].q[k];
    for (int k = 0; k < nc; ++k)
      if (l <= m->lk[k]) {
        di[(size_t)l * nc + k] = m->invcl[k][l];
        ds[(size_t)l * nc + k] = std::sqrt(m->invcl[k][l]);
      }
  }
  m->cA.upload(cA, s);
  m->dInv.upload(di, s);
  m->dSqrt.upload(ds, s);
}

void ensure_ws(crs_model m, int nrhs, hipStream_t s) {
  if (nrhs <= m->nrhs_ws) return;
  CRS_HIP(hipStreamSynchronize(s));
  for (auto& g : m->groups) {
    const int nmaps = (int)g.bands.size() * nrhs;
    g.uhat.alloc((size_t)nmaps * g.nalm);
    g.phase.alloc((size_t)nmaps * g.pst);
    g.vpart.alloc((size_t)g.ntiles * nmaps * g.nalm);
  }
  std::vector<const double*> vp(m->nbands);
  for (int nu = 0; nu < m->nbands; ++nu) vp[nu] = m->groups[m->bands[nu].group].vpart.p;
  m->d_vptr.upload(vp, s);
  const size_t nn = (size_t)nrhs * m->n;
  m->r.alloc(nn);
  m->z.alloc(nn);
  m->p.alloc(nn);
  m->q.alloc(nn);
  m->t.alloc(nn);
  m->partial.alloc((size_t)nrhs * kDotBlocks);
  m->scal.alloc((size_t)nrhs * 8);
  m->dsel.alloc(nrhs);
  CRS_HIP(hipStreamSynchronize(s));
  m->nrhs_ws = nrhs;
}

int model_nalm_union(crs_model m) { return (m->Lc + 1) * (m->Lc + 1); }

// coefficient table / diag choice for an operator
enum OpKind { OP_A = 0, OP_PI = 1 };

void run_band_ops(crs_model m, int nrhs, const double* in, const double* coef, bool pinv, hipStream_t s) {
  for (size_t gi = 0; gi < m->groups.size(); ++gi) {
    Group& g = m->groups[gi];
    const int nmaps = (int)g.bands.size() * nrhs;
    dim3 gr((2 * (g.lmax + 1) + 255) / 256, g.lmax + 1, nmaps);
    hipLaunchKernelGGL(k_mix_fwd, gr, dim3(256), 0, s, in, m->n, nrhs, m->ncomp, m->d_lk.p, m->d_coff.p,
                       coef, m->nbands, g.bandids.p, g.lmax, m->ftab.p, m->Lmax, g.uhat.p, g.nalm);
    CRS_HIP(hipGetLastError());
    {
      ProfScope ps(FAM_LEG_SYNTH, leg_flops(*g.plan, nmaps), s);
      launch_leg_synth(leg_args(g.grid, *g.plan), nmaps, g.uhat.p, g.nalm, g.phase.p, g.pst, s);
    }
    {
      ProfScope ps(FAM_RING, ring_bytes(g.grid, g.lmax, nmaps, RING_ROUNDTRIP) +
                                 (double)g.bands.size() * g.grid->npix * 8.0, s);
      launch_ring(g.grid, g.lmax, RING_ROUNDTRIP, nmaps, g.phase.p, g.pst, nullptr, nullptr, 0,
                  pinv ? g.wP.p : g.wA.p, nrhs, s);
    }
    {
      ProfScope ps(FAM_LEG_ADJ, leg_flops(*g.plan, nmaps), s);
      launch_leg_adjoint(leg_args(g.grid, *g.plan), nmaps, g.phase.p, g.pst, g.vpart.p, g.nalm,
                         (int64_t)nmaps * g.nalm, false, s);
    }
  }
}

void mix_back(crs_model m, int nrhs, double* out, const double* din, int dmode, const double* dtab,
              const double* coef, hipStream_t s) {
  dim3 gr((2 * (m->Lc + 1) + 255) / 256, m->Lc + 1, m->ncomp * nrhs);
  hipLaunchKernelGGL(k_mix_back, gr, dim3(256), 0, s, out, din, m->n, nrhs, m->ncomp, m->d_lk.p, m->d_coff.p,
                     coef, m->nbands, m->d_vptr.p, m->d_binfo.p, dmode, dtab, m->ftab.p, m->Lmax, m->Lc);
  CRS_HIP(hipGetLastError());
}

void op_apply(crs_model m, OpKind kind, int nrhs, const double* in, double* out, hipStream_t s) {
  ensure_ws(m, nrhs, s);
  const bool pinv = kind == OP_PI;
  const double* coef = pinv ? m->cP.p : m->cA.p;
  run_band_ops(m, nrhs, in, coef, pinv, s);
  if (pinv)
    mix_back(m, nrhs, out, in, 2, m->dPi.p, coef, s);
  else
    mix_back(m, nrhs, out, in, 1, m->dInv.p, coef, s);
}

void diag_apply(crs_model m, int nrhs, const double* r, double* z, hipStream_t s) {
  dim3 gr((2 * (m->Lc + 1) + 255) / 256, m->Lc + 1, nrhs);
  hipLaunchKernelGGL(k_diag_apply, gr, dim3(256), 0, s, r, z, m->n, m->ncomp, m->d_lk.p, m->d_coff.p,
                     m->Dinv.p, m->Lc);
  CRS_HIP(hipGetLastError());
}

void precond_apply(crs_model m, int precond, int nrhs, const double* r, double* z, hipStream_t s) {
  if (precond == CRS_PRECOND_PINV) {
    op_apply(m, OP_PI, nrhs, r, z, s);
  } else if (precond == CRS_PRECOND_DIAG) {
    diag_apply(m, nrhs, r, z, s);
  } else {
    CRS_HIP(hipMemcpyAsync(z, r, (size_t)nrhs * m->n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
}

// M_diag setup: diag(Y^T tau Y) per band via the squared Legendre adjoint of
// the ring spectrum of tau, then the N_comp x N_comp blocks on the host.
void build_diag(crs_model m, hipStream_t s) {
  const int nb = m->nbands, nc = m->ncomp, Lc = m->Lc;
  std::vector<std::vector<double>> dg(nb);
  for (int nu = 0; nu < nb; ++nu) {
    Band& b = m->bands[nu];
    Group& g = m->groups[b.group];
    ShtPlan& p = *g.plan;
    DevBuf<double2> ph;
    DevBuf<double> vp, out;
    ph.alloc((size_t)g.pst);
    vp.alloc((size_t)g.ntiles * g.nalm);
    out.alloc((size_t)g.nalm);
    launch_ring(g.grid, g.lmax, RING_DIAG, 1, ph.p, g.pst, b.tau.p, nullptr, g.grid->npix, nullptr, 1, s);
    launch_leg_adjoint(leg_args(g.grid, p), 1, ph.p, g.pst, vp.p, g.nalm, g.nalm, true, s);
    launch_hat_scale(p.f.p, g.lmax, 1, vp.p, g.nalm, g.ntiles, g.nalm, out.p, g.nalm, true, s);
    dg[nu].resize(g.nalm);
    CRS_HIP(hipMemcpyAsync(dg[nu].data(), out.p, g.nalm * sizeof(double), hipMemcpyDeviceToHost, s));
    CRS_HIP(hipStreamSynchronize(s));
  }
  const int64_t nu_ = (int64_t)(Lc + 1) * (Lc + 1);
  std::vector<double> Dinv((size_t)nu_ * nc * nc, 0.0);
  std::vector<double> D(nc * nc), P;
  for (int mm = 0; mm <= Lc; ++mm) {
    const int np = mm == 0 ? 1 : 2;
    for (int part = 0; part < np; ++part)
      for (int l = mm; l <= Lc; ++l) {
        const int64_t u = moff_h(Lc, mm) + (int64_t)part * (Lc - mm + 1) + (l - mm);
        std::vector<int> act;
        for (int k = 0; k < nc; ++k)
          if (l <= m->lk[k]) act.push_back(k);
        const int na = (int)act.size();
        if (!na) continue;
        std::vector<double> Da((size_t)na * na, 0.0);
        for (int nu = 0; nu < nb; ++nu) {
          const Band& b = m->bands[nu];
          if (l > b.lmax) continue;
          const double d = dg[nu][moff_h(b.lmax, mm) + (int64_t)part * (b.lmax - mm + 1) + (l - mm)] * b.beam[l] * b.beam[l];
          for (int i = 0; i < na; ++i)
            for (int j = 0; j < na; ++j) Da[i * na + j] += d * b.q[act[i]] * b.q[act[j]];
        }
        for (int i = 0; i < na; ++i) Da[i * na + i] += m->invcl[act[i]][l];
        // inverse of the symmetric block (pseudo-inverse if singular)
        small_pinv(Da, na, na, P);
        for (int i = 0; i < na; ++i)
          for (int j = 0; j < na; ++j) Dinv[((size_t)u * nc + act[i]) * nc + act[j]] = P[(size_t)i * na + j];
      }
  }
  m->Dinv.upload(Dinv, s);
  CRS_HIP(hipStreamSynchronize(s));
}

void validate_desc(const crs_model_desc* d) {
  CRS_CHECK(d != nullptr, CRS_EINVAL, "desc is NULL");
  CRS_CHECK(d->ncomp >= 1 && d->ncomp <= 8, CRS_EINVAL, "ncomp must be in 1..8");
  CRS_CHECK(d->nbands >= 1, CRS_EINVAL, "nbands must be >= 1");
  CRS_CHECK(d->lmax_comp != nullptr && d->inv_cl != nullptr && d->bands != nullptr, CRS_EINVAL,
            "lmax_comp, inv_cl or bands is NULL");
  for (int k = 0; k < d->ncomp; ++k) {
    CRS_CHECK(d->lmax_comp[k] >= 0, CRS_EINVAL, "component lmax must be >= 0");
    CRS_CHECK(d->inv_cl[k] != nullptr, CRS_EINVAL, "inv_cl entry is NULL");
    for (int l = 0; l <= d->lmax_comp[k]; ++l)
      CRS_CHECK(d->inv_cl[k][l] >= 0.0 && std::isfinite(d->inv_cl[k][l]), CRS_EINVAL,
                "inv_cl must be finite and >= 0");
  }
  for (int nu = 0; nu < d->nbands; ++nu) {
    const crs_band_desc& b = d->bands[nu];
    CRS_CHECK(b.grid != nullptr, CRS_EINVAL, "band grid is NULL");
    CRS_CHECK(b.lmax >= 0, CRS_EINVAL, "band lmax must be >= 0");
    CRS_CHECK(b.beam != nullptr && b.tau != nullptr && b.q != nullptr, CRS_EINVAL,
              "band beam, tau or q is NULL");
    for (int64_t i = 0; i < b.grid->npix; ++i)
      CRS_CHECK(b.tau[i] >= 0.0 && std::isfinite(b.tau[i]), CRS_EINVAL, "tau must be finite and >= 0");
    for (int k = 0; k < d->ncomp; ++k) CRS_CHECK(std::isfinite(b.q[k]), CRS_EINVAL, "q must be finite");
    for (int l = 0; l <= b.lmax; ++l) CRS_CHECK(std::isfinite(b.beam[l]), CRS_EINVAL, "beam must be finite");
  }
}

}  // namespace

using namespace crs;

extern "C" {

int crs_model_create(const crs_model_desc* d, crs_stream st, crs_model* out) {
  return guarded([&] {
    CRS_CHECK(out != nullptr, CRS_EINVAL, "out is NULL");
    validate_desc(d);
    hipStream_t s = (hipStream_t)st;
    auto m = std::make_unique<crs_model_s>();
    CRS_HIP(hipGetDevice(&m->device));
    m->ncomp = d->ncomp;
    m->nbands = d->nbands;
    m->lk.assign(d->lmax_comp, d->lmax_comp + d->ncomp);
    m->coff.resize(d->ncomp);
    int64_t off = 0;
    for (int k = 0; k < d->ncomp; ++k) {
      m->coff[k] = off;
      off += (int64_t)(m->lk[k] + 1) * (m->lk[k] + 1);
      m->invcl.emplace_back(d->inv_cl[k], d->inv_cl[k] + m->lk[k] + 1);
      m->Lc = std::max(m->Lc, m->lk[k]);
    }
    m->n = off;
    m->Lmax = m->Lc;
    m->bands.resize(d->nbands);
    for (int nu = 0; nu < d->nbands; ++nu) {
      const crs_band_desc& bd = d->bands[nu];
      Band& b = m->bands[nu];
      b.grid = bd.grid;
      b.lmax = bd.lmax;
      b.npix = bd.grid->npix;
      b.beam.assign(bd.beam, bd.beam + bd.lmax + 1);
      b.q.assign(bd.q, bd.q + d->ncomp);
      b.tau_host.assign(bd.tau, bd.tau + b.npix);
      m->Lmax = std::max(m->Lmax, b.lmax);
      // alpha^2 = sum t^2 / sum t, t = tau / w   (App. A.1, eq:optimal-alpha)
      b.w_host.resize(b.npix);
      double s1 = 0, s2 = 0;
      for (int r = 0; r < b.grid->nring; ++r)
        for (int j = 0; j < b.grid->nphi[r]; ++j) {
          const int64_t i = b.grid->offset[r] + j;
          const double w = b.grid->ringw[r];
          b.w_host[i] = w;
          const double t = b.tau_host[i] / w;
          s1 += t;
          s2 += t * t;
        }
      CRS_CHECK(s1 > 0.0, CRS_EINVAL, "a band has no unmasked pixel");
      b.alpha2 = s2 / s1;
      b.tau.upload(b.tau_host, s);
      std::vector<double> tp(b.npix);
      for (int64_t i = 0; i < b.npix; ++i)
        tp[i] = b.tau_host[i] > 0.0 ? b.alpha2 * b.w_host[i] * b.w_host[i] / b.tau_host[i] : 0.0;
      b.tplus.upload(tp, s);
      // group by (grid, lmax)
      int gi = -1;
      for (size_t k = 0; k < m->groups.size(); ++k)
        if (m->groups[k].grid == b.grid && m->groups[k].lmax == b.lmax) gi = (int)k;
      if (gi < 0) {
        m->groups.emplace_back();
        gi = (int)m->groups.size() - 1;
        m->groups[gi].grid = b.grid;
        m->groups[gi].lmax = b.lmax;
      }
      b.group = gi;
      b.gidx = (int)m->groups[gi].bands.size();
      m->groups[gi].bands.push_back(nu);
    }
    for (auto& g : m->groups) {
      g.plan = &get_plan(g.grid, g.lmax, s);
      g.ntiles = leg_adjoint_tiles(g.plan->npairs, g.lmax);
      g.nalm = (int64_t)(g.lmax + 1) * (g.lmax + 1);
      g.pst = (int64_t)g.grid->nring * (g.lmax + 1);
      std::vector<const double*> wa, wp;
      for (int nu : g.bands) {
        wa.push_back(m->bands[nu].tau.p);
        wp.push_back(m->bands[nu].tplus.p);
      }
      g.wA.upload(wa, s);
      g.wP.upload(wp, s);
      g.bandids.upload(g.bands, s);
    }
    std::vector<int> binfo(4 * d->nbands);
    for (int nu = 0; nu < d->nbands; ++nu) {
      const Band& b = m->bands[nu];
      binfo[4 * nu + 0] = b.lmax;
      binfo[4 * nu + 1] = (int)m->groups[b.group].bands.size();
      binfo[4 * nu + 2] = b.gidx;
      binfo[4 * nu + 3] = m->groups[b.group].ntiles;
    }
    m->d_binfo.upload(binfo, s);
    m->d_lk.upload(m->lk, s);
    m->d_coff.upload(m->coff, s);
    build_ftab(m.get(), s);
    build_mix_tables(m.get(), s);
    build_pinv_tables(m.get(), s);
    if (d->flags & CRS_MODEL_DIAG) {
      build_diag(m.get(), s);
      m->has_diag = true;
    }
    ensure_ws(m.get(), 1, s);
    CRS_HIP(hipStreamSynchronize(s));
    *out = m.release();
    return CRS_OK;
  });
}

int crs_model_destroy(crs_model m) {
  return guarded([&] {
    delete m;
    return CRS_OK;
  });
}

int crs_model_size(crs_model m, int64_t* n) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && n != nullptr, CRS_EINVAL, "model or n is NULL");
    *n = m->n;
    return CRS_OK;
  });
}

int crs_model_alpha2(crs_model m, double* a2) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && a2 != nullptr, CRS_EINVAL, "model or alpha2 is NULL");
    for (int nu = 0; nu < m->nbands; ++nu) a2[nu] = m->bands[nu].alpha2;
    return CRS_OK;
  });
}

int crs_model_set_mixing(crs_model m, const double* q, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && q != nullptr, CRS_EINVAL, "model or q is NULL");
    for (int i = 0; i < m->nbands * m->ncomp; ++i) CRS_CHECK(std::isfinite(q[i]), CRS_EINVAL, "q must be finite");
    hipStream_t s = (hipStream_t)st;
    for (int nu = 0; nu < m->nbands; ++nu) m->bands[nu].q.assign(q + nu * m->ncomp, q + (nu + 1) * m->ncomp);
    CRS_HIP(hipStreamSynchronize(s));
    build_mix_tables(m, s);
    build_pinv_tables(m, s);
    if (m->has_diag) build_diag(m, s);
    CRS_HIP(hipStreamSynchronize(s));
    return CRS_OK;
  });
}

static void check_vec(crs_model m, int nrhs, const void* a, const void* b) {
  CRS_CHECK(m != nullptr, CRS_EINVAL, "model is NULL");
  CRS_CHECK(nrhs >= 1, CRS_EINVAL, "nrhs must be >= 1");
  CRS_CHECK(a != nullptr && b != nullptr, CRS_EINVAL, "vector pointer is NULL");
}

int apply_A(crs_model m, int nrhs, const double* x, double* y, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, x, y);
    op_apply(m, OP_A, nrhs, x, y, (hipStream_t)st);
    return CRS_OK;
  });
}

int apply_pinv_precond(crs_model m, int nrhs, const double* r, double* z, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, r, z);
    op_apply(m, OP_PI, nrhs, r, z, (hipStream_t)st);
    return CRS_OK;
  });
}

int apply_diag_precond(crs_model m, int nrhs, const double* r, double* z, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, r, z);
    CRS_CHECK(m->has_diag, CRS_EINVAL, "model was created without CRS_MODEL_DIAG");
    ensure_ws(m, nrhs, (hipStream_t)st);
    diag_apply(m, nrhs, r, z, (hipStream_t)st);
    return CRS_OK;
  });
}

int pcg_solve(crs_model m, int precond, int nrhs, const double* b, double* x, double rtol, int maxiter,
              int* iters, double* relres, double* history, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, b, x);
    CRS_CHECK(precond == CRS_PRECOND_NONE || precond == CRS_PRECOND_DIAG || precond == CRS_PRECOND_PINV,
              CRS_EINVAL, "unknown preconditioner");
    CRS_CHECK(precond != CRS_PRECOND_DIAG || m->has_diag, CRS_EINVAL,
              "model was created without CRS_MODEL_DIAG");
    CRS_CHECK(rtol > 0.0 && maxiter >= 0, CRS_EINVAL, "rtol must be > 0 and maxiter >= 0");
    hipStream_t s = (hipStream_t)st;
    ensure_ws(m, nrhs, s);
    const int64_t n = m->n;
    const dim3 vg = vgrid(n, nrhs);
    const int nblk = (int)vg.x;
    double* scal = m->scal.p;
    auto dot_to = [&](const double* a, const double* bb, int op) {
      hipLaunchKernelGGL(k_dot, vg, dim3(256), 0, s, a, bb, n, m->partial.p);
      hipLaunchKernelGGL(k_scalar, dim3(nrhs), dim3(256), 0, s, op, m->partial.p, nblk, nrhs, scal);
    };
    std::vector<double> hs((size_t)nrhs * 8, 0.0), bb(nrhs);
    for (int i = 0; i < nrhs; ++i) hs[i * 8 + S_ACTIVE] = 1.0;
    CRS_HIP(hipMemcpyAsync(scal, hs.data(), hs.size() * sizeof(double), hipMemcpyHostToDevice, s));
    // |b|^2
    dot_to(b, b, 4);
    CRS_HIP(hipMemcpyAsync(hs.data(), scal, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    CRS_HIP(hipStreamSynchronize(s));
    std::vector<int> active(nrhs, 1), status(nrhs, 0), it_used(nrhs, 0);
    for (int i = 0; i < nrhs; ++i) {
      bb[i] = hs[i * 8 + S_TMP];
      if (!(bb[i] > 0.0)) {
        active[i] = 0;  // b = 0: x = 0 is the solution
      }
    }
    // zero x for b = 0 rhs
    for (int i = 0; i < nrhs; ++i)
      if (!active[i]) CRS_HIP(hipMemsetAsync(x + (int64_t)i * n, 0, n * sizeof(double), s));
    // r = b - A x
    op_apply(m, OP_A, nrhs, x, m->q.p, s);
    hipLaunchKernelGGL(k_sub, vg, dim3(256), 0, s, m->r.p, b, m->q.p, n, (const int*)nullptr);
    precond_apply(m, precond, nrhs, m->r.p, m->z.p, s);
    CRS_HIP(hipMemcpyAsync(m->p.p, m->z.p, (size_t)nrhs * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    for (int i = 0; i < nrhs; ++i) hs[i * 8 + S_ACTIVE] = active[i];
    CRS_HIP(hipMemcpyAsync(scal, hs.data(), hs.size() * sizeof(double), hipMemcpyHostToDevice, s));
    dot_to(m->r.p, m->z.p, 3);
    CRS_HIP(hipMemcpyAsync(hs.data(), scal, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    CRS_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nrhs; ++i) {
      if (active[i] && hs[i * 8 + S_ACTIVE] == 0.0) {
        active[i] = 0;
        status[i] = hs[i * 8 + S_BREAK] != 0.0 ? 2 : 0;  // r = 0 (x0 exact) counts as converged
      }
    }
    DevBuf<int>& dsel = m->dsel;
    std::vector<int> sel(nrhs);
    int it = 0;
    auto any_active = [&] {
      for (int i = 0; i < nrhs; ++i)
        if (active[i]) return true;
      return false;
    };
    while (any_active() && it < maxiter) {
      ++it;
      op_apply(m, OP_A, nrhs, m->p.p, m->q.p, s);
      dot_to(m->p.p, m->q.p, 0);
      hipLaunchKernelGGL(k_update_xr, vg, dim3(256), 0, s, x, m->r.p, m->p.p, m->q.p, n, scal, m->partial.p);
      hipLaunchKernelGGL(k_scalar, dim3(nrhs), dim3(256), 0, s, 2, m->partial.p, nblk, nrhs, scal);
      CRS_HIP(hipMemcpyAsync(hs.data(), scal, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      CRS_HIP(hipStreamSynchronize(s));
      bool cand = false;
      for (int i = 0; i < nrhs; ++i) {
        sel[i] = 0;
        if (!active[i]) continue;
        if (hs[i * 8 + S_BREAK] != 0.0) {
          active[i] = 0;
          status[i] = 2;
          it_used[i] = it;
          continue;
        }
        const double rel = std::sqrt(hs[i * 8 + S_RR] / bb[i]);
        if (history) history[(size_t)(it - 1) * nrhs + i] = rel;
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
      if (cand) {
        // true residual of the candidates: t = b - A x
        op_apply(m, OP_A, nrhs, x, m->q.p, s);
        hipLaunchKernelGGL(k_sub, vg, dim3(256), 0, s, m->t.p, b, m->q.p, n, (const int*)nullptr);
        dot_to(m->t.p, m->t.p, 4);
        CRS_HIP(hipMemcpyAsync(hs.data(), scal, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        CRS_HIP(hipStreamSynchronize(s));
        bool restart = false;
        for (int i = 0; i < nrhs; ++i) {
          if (!sel[i]) continue;
          if (std::sqrt(hs[i * 8 + S_TMP] / bb[i]) <= rtol) {
            active[i] = 0;
            status[i] = 0;
            sel[i] = 0;
          } else {
            restart = true;  // keep sel[i] = 1: restart from the true residual
          }
        }
        for (int i = 0; i < nrhs; ++i) {
          hs[i * 8 + S_ACTIVE] = active[i];
          hs[i * 8 + S_RESTART] = sel[i];
        }
        CRS_HIP(hipMemcpyAsync(scal, hs.data(), hs.size() * sizeof(double), hipMemcpyHostToDevice, s));
        if (restart) {
          CRS_HIP(hipMemcpyAsync(dsel.p, sel.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
          hipLaunchKernelGGL(k_copy_sel, vg, dim3(256), 0, s, m->r.p, m->t.p, n, dsel.p);
        }
        CRS_HIP(hipStreamSynchronize(s));
      }
      if (!any_active()) break;
      precond_apply(m, precond, nrhs, m->r.p, m->z.p, s);
      dot_to(m->r.p, m->z.p, 1);
      hipLaunchKernelGGL(k_update_p, vg, dim3(256), 0, s, m->p.p, m->z.p, n, scal);
    }
    for (int i = 0; i < nrhs; ++i)
      if (active[i]) status[i] = 1;  // maxiter
    // final true residuals
    op_apply(m, OP_A, nrhs, x, m->q.p, s);
    hipLaunchKernelGGL(k_sub, vg, dim3(256), 0, s, m->t.p, b, m->q.p, n, (const int*)nullptr);
    dot_to(m->t.p, m->t.p, 4);
    CRS_HIP(hipMemcpyAsync(hs.data(), scal, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    CRS_HIP(hipStreamSynchronize(s));
    int ret = CRS_OK;
    for (int i = 0; i < nrhs; ++i) {
      if (iters) iters[i] = it_used[i];
      if (relres) relres[i] = bb[i] > 0 ? std::sqrt(hs[i * 8 + S_TMP] / bb[i]) : 0.0;
      if (status[i] == 2) ret = CRS_EBREAKDOWN;
      else if (status[i] == 1 && ret == CRS_OK) ret = CRS_ENOTCONV;
    }
    if (ret == CRS_EBREAKDOWN) set_error(ret, "PCG breakdown (p.Ap <= 0, r.z <= 0 or non-finite)");
    if (ret == CRS_ENOTCONV) set_error(ret, "PCG reached maxiter");
    return ret;
  });
}

int build_rhs(crs_model m, int nrhs, const double* const* d, const double* const* omega1,
              const double* omega2, double* b, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && b != nullptr, CRS_EINVAL, "model or b is NULL");
    CRS_CHECK(nrhs >= 1, CRS_EINVAL, "nrhs must be >= 1");
    hipStream_t s = (hipStream_t)st;
    ensure_ws(m, nrhs, s);
    for (auto& g : m->groups) {
      const int nmaps = (int)g.bands.size() * nrhs;
      const int64_t npix = g.grid->npix;
      g.pix.alloc((size_t)nmaps * npix);
      for (size_t gi = 0; gi < g.bands.size(); ++gi) {
        const int nu = g.bands[gi];
        const double* dv = d ? d[nu] : nullptr;
        const double* wv = omega1 ? omega1[nu] : nullptr;
        hipLaunchKernelGGL(k_pix_rhs, vgrid(npix, nrhs), dim3(256), 0, s, g.pix.p + (int64_t)gi * nrhs * npix,
                           m->bands[nu].tau.p, dv, wv, npix);
      }
      CRS_HIP(hipGetLastError());
      launch_ring(g.grid, g.lmax, RING_ADJOINT, nmaps, g.phase.p, g.pst, g.pix.p, nullptr, npix,
                  nullptr, 1, s);
      launch_leg_adjoint(leg_args(g.grid, *g.plan), nmaps, g.phase.p, g.pst, g.vpart.p, g.nalm,
                         (int64_t)nmaps * g.nalm, false, s);
    }
    mix_back(m, nrhs, b, omega2, omega2 ? 1 : 0, m->dSqrt.p, m->cA.p, s);
    return CRS_OK;
  });
}

int crs_model_project(crs_model m, int nrhs, const double* x, double* const* maps, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && x != nullptr && maps != nullptr, CRS_EINVAL, "model, x or maps is NULL");
    CRS_CHECK(nrhs >= 1, CRS_EINVAL, "nrhs must be >= 1");
    for (int nu = 0; nu < m->nbands; ++nu) CRS_CHECK(maps[nu] != nullptr, CRS_EINVAL, "maps entry is NULL");
    hipStream_t s = (hipStream_t)st;
    ensure_ws(m, nrhs, s);
    for (auto& g : m->groups) {
      const int nmaps = (int)g.bands.size() * nrhs;
      const int64_t npix = g.grid->npix;
      g.pix.alloc((size_t)nmaps * npix);
      dim3 gr((2 * (g.lmax + 1) + 255) / 256, g.lmax + 1, nmaps);
      hipLaunchKernelGGL(k_mix_fwd, gr, dim3(256), 0, s, x, m->n, nrhs, m->ncomp, m->d_lk.p, m->d_coff.p,
                         m->cA.p, m->nbands, g.bandids.p, g.lmax, m->ftab.p, m->Lmax, g.uhat.p, g.nalm);
      CRS_HIP(hipGetLastError());
      launch_leg_synth(leg_args(g.grid, *g.plan), nmaps, g.uhat.p, g.nalm, g.phase.p, g.pst, s);
      launch_ring(g.grid, g.lmax, RING_SYNTH, nmaps, g.phase.p, g.pst, nullptr, g.pix.p, npix,
                  nullptr, 1, s);
      for (size_t gi = 0; gi < g.bands.size(); ++gi)
        CRS_HIP(hipMemcpyAsync(maps[g.bands[gi]], g.pix.p + (int64_t)gi * nrhs * npix,
                               (size_t)nrhs * npix * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    return CRS_OK;
  });
}

int crs_philox_normals(uint64_t seed, uint64_t stream, uint64_t rhs, int64_t n, double* out, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(out != nullptr && n >= 0, CRS_EINVAL, "out is NULL or n < 0");
    if (n == 0) return CRS_OK;
    int64_t nb = ((n + 3) / 4 + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_philox_normals, dim3((unsigned)nb, 1), dim3(256), 0, (hipStream_t)st, seed, stream, rhs, n, out);
    CRS_HIP(hipGetLastError());
    return CRS_OK;
  });
}

int constrained_realization(crs_model m, int nrhs, const double* const* d, uint64_t seed, int mode,
                            int precond, double rtol, int maxiter, double* x, int* iters, double* relres,
                            crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && x != nullptr, CRS_EINVAL, "model or x is NULL");
    CRS_CHECK(nrhs >= 1, CRS_EINVAL, "nrhs must be >= 1");
    CRS_CHECK(mode == CRS_MODE_WF || mode == CRS_MODE_CR, CRS_EINVAL, "mode must be WF or CR");
    hipStream_t s = (hipStream_t)st;
    ensure_ws(m, nrhs, s);
    std::vector<const double*> w1(m->nbands, nullptr);
    const double* w2 = nullptr;
    if (mode == CRS_MODE_CR) {
      int64_t tot = 0;
      for (auto& b : m->bands) tot += b.npix;
      m->om1.alloc((size_t)tot * nrhs);
      m->om2.alloc((size_t)m->n * nrhs);
      int64_t o = 0;
      for (int nu = 0; nu < m->nbands; ++nu) {
        const int64_t np = m->bands[nu].npix;
        int64_t nb = ((np + 3) / 4 + 255) / 256;
        if (nb > 4096) nb = 4096;
        hipLaunchKernelGGL(k_philox_normals, dim3((unsigned)nb, nrhs), dim3(256), 0, s, seed,
                           (uint64_t)(0x100 + nu), (uint64_t)0, np, m->om1.p + o);
        w1[nu] = m->om1.p + o;
        o += np * nrhs;
      }
      int64_t nb = ((m->n + 3) / 4 + 255) / 256;
      if (nb > 4096) nb = 4096;
      hipLaunchKernelGGL(k_philox_normals, dim3((unsigned)nb, nrhs), dim3(256), 0, s, seed, (uint64_t)0x200,
                         (uint64_t)0, m->n, m->om2.p);
      CRS_HIP(hipGetLastError());
      w2 = m->om2.p;
    }
    // the right-hand side is kept in a model-owned buffer
    m->bcr.alloc((size_t)m->n * nrhs);
    int rc = build_rhs(m, nrhs, d, mode == CRS_MODE_CR ? w1.data() : nullptr, w2, m->bcr.p, st);
    if (rc != CRS_OK) return rc;
    CRS_HIP(hipMemsetAsync(x, 0, (size_t)m->n * nrhs * sizeof(double), s));
    rc = pcg_solve(m, precond, nrhs, m->bcr.p, x, rtol, maxiter, iters, relres, nullptr, st);
    CRS_HIP(hipStreamSynchronize(s));
    return rc;
  });
}

}  // extern "C"
