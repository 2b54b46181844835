// The constrained-realization model: tables, setup and the per-model entry
// points (gfx950, float64).
//
//   A = S^-1 + sum_nu P_nu^T N_nu^-1 P_nu           (Sect. 2.3, eq:A)
//   P_nu = Y_nu B_nu q_{nu,k}                        (eq:P, Q~ = q I, Sect. 3.3)
//   M_PI = U^+ T^+ (U^+)^T                            (eq:fullmodel-preconditioner)
//   M_diag = (U^T diag(T) U)^-1                       (Sect. 5)
//   b = sum_nu P_nu^T (tau d + tau^1/2 w1) + S^-1/2 w2 (Sect. 2.3)
//
// A model owns the per-l tables of one problem: the component -> band mix
// b_{nu,l} q_{nu,k}, the pseudo-inverse blocks U_l^+ (Sect. 3.3), the prior
// terms and optionally the M_diag blocks.  Operators and the solver run
// through an Exec over the model's right-hand sides (exec.hip).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "model.h"

namespace {
using namespace crs;

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
          U[(size_t)nu * na + ja] = std::sqrt(m->bands[nu].alpha2) * m->bands[nu].beam[l] * mix_q_pre(m, nu, k);
      U[(size_t)(nb + k) * na + ja] = std::sqrt(m->invcl[k][l]);
    }
    // merged observations (App. A.3): per group the representative's row
    // scaled by sqrt(1 + sum gamma^2), gamma the least-squares scale of each
    // other member's row onto it; the members' rows are zeroed
    if (!m->merge_group.empty())
      for (int rep = 0; rep < nb; ++rep) {
        const int grp = m->merge_group[rep];
        if (grp < 0 || m->pi_drop[rep]) continue;
        double n0 = 0.0;
        for (int ja = 0; ja < na; ++ja) n0 += U[(size_t)rep * na + ja] * U[(size_t)rep * na + ja];
        double g2 = 0.0;
        for (int nu = rep + 1; nu < nb; ++nu) {
          if (m->merge_group[nu] != grp) continue;
          double dot = 0.0;
          for (int ja = 0; ja < na; ++ja) dot += U[(size_t)nu * na + ja] * U[(size_t)rep * na + ja];
          const double g = n0 > 0.0 ? dot / n0 : 0.0;
          g2 += g * g;
          for (int ja = 0; ja < na; ++ja) U[(size_t)nu * na + ja] = 0.0;
        }
        const double sc = std::sqrt(1.0 + g2);
        for (int ja = 0; ja < na; ++ja) U[(size_t)rep * na + ja] *= sc;
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
  std::vector<double> bt((size_t)(L + 1) * nb, 0.0);
  for (int l = 0; l <= L; ++l) {
    for (int nu = 0; nu < nb; ++nu)
      if (l <= m->bands[nu].lmax) {
        bt[(size_t)l * nb + nu] = m->bands[nu].beam[l];
        for (int k = 0; k < nc; ++k) cA[((size_t)l * nb + nu) * nc + k] = m->bands[nu].beam[l] * mix_q_a(m, nu, k);
      }
    for (int k = 0; k < nc; ++k)
      if (l <= m->lk[k]) {
        di[(size_t)l * nc + k] = m->invcl[k][l];
        ds[(size_t)l * nc + k] = std::sqrt(m->invcl[k][l]);
      }
  }
  m->cA.upload(cA, s);
  m->beamtab.upload(bt, s);
  m->dInv.upload(di, s);
  m->dSqrt.upload(ds, s);
}

// M_diag setup: diag(Y^T tau Y) per band via the squared Legendre adjoint of
// the ring spectrum of tau, then the N_comp x N_comp blocks on the host.
void build_diag(crs_model m, hipStream_t s) {
  const int nb = m->nbands, nc = m->ncomp, Lc = m->Lc;
  std::vector<std::vector<double>> dg(nb);
  for (int nu = 0; nu < nb; ++nu) {
    Band& b = m->bands[nu];
    ShtPlan& p = get_plan(b.grid, b.lmax, s);
    const LegChoice lc = leg_choice(p.npairs, b.lmax, 1);
    const int ntiles = leg_adjoint_tiles(lc, p.npairs, true);
    const int64_t nalm = (int64_t)(b.lmax + 1) * (b.lmax + 1);
    const int64_t pst = (int64_t)b.grid->nring * (b.lmax + 1);
    DevBuf<double2> ph;
    DevBuf<double> vp, out;
    ph.alloc((size_t)pst);
    vp.alloc((size_t)ntiles * nalm);
    out.alloc((size_t)nalm);
    launch_ring(b.grid, b.lmax, RING_DIAG, 1, ph.p, pst, b.tau.p, nullptr, b.grid->npix, nullptr, 1, s);
    launch_leg_adjoint(lc, leg_args(b.grid, p), 1, ph.p, pst, vp.p, nalm, nalm, true, s);
    launch_hat_scale(p.f.p, b.lmax, 1, vp.p, nalm, ntiles, nalm, out.p, nalm, true, s);
    dg[nu].resize(nalm);
    CRS_HIP(hipMemcpyAsync(dg[nu].data(), out.p, nalm * sizeof(double), hipMemcpyDeviceToHost, s));
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
            for (int j = 0; j < na; ++j) Da[i * na + j] += d * mix_q_pre(m, nu, act[i]) * mix_q_pre(m, nu, act[j]);
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


// The model's Exec for nrhs right-hand sides (kept per nrhs, built on first use).
Exec& model_exec(crs_model m, int nrhs, hipStream_t s) {
  auto it = m->execs.find(nrhs);
  if (it != m->execs.end()) return *it->second;
  auto e = make_exec({m}, nrhs, s);
  Exec& ref = *e;
  m->execs[nrhs] = std::move(e);
  return ref;
}

void check_vec(crs_model m, int nrhs, const void* a, const void* b) {
  CRS_CHECK(m != nullptr, CRS_EINVAL, "model is NULL");
  CRS_CHECK(nrhs >= 1, CRS_EINVAL, "nrhs must be >= 1");
  CRS_CHECK(a != nullptr && b != nullptr, CRS_EINVAL, "vector pointer is NULL");
}

// per (system, band) map pointers of a model's [nrhs][npix] band arrays
std::vector<std::vector<const double*>> sys_band_ptrs(crs_model m, int nrhs, const double* const* arr) {
  std::vector<std::vector<const double*>> out;
  if (!arr) return out;
  out.assign(nrhs, std::vector<const double*>(m->nbands, nullptr));
  for (int r = 0; r < nrhs; ++r)
    for (int nu = 0; nu < m->nbands; ++nu)
      out[r][nu] = arr[nu] ? arr[nu] + (int64_t)r * m->bands[nu].npix : nullptr;
  return out;
}

}  // namespace

namespace crs {
Exec& model_exec_ref(crs_model m, int nrhs, hipStream_t s) { return model_exec(m, nrhs, s); }

double mix_q_a(crs_model m, int nu, int k) {
  for (const VarMix& v : m->varmix)
    if (v.nu == nu && v.k == k) return 1.0;
  return m->bands[nu].q[k];
}

double mix_q_pre(crs_model m, int nu, int k) {
  for (const VarMix& v : m->varmix)
    if (v.nu == nu && v.k == k) return v.qeff;
  return m->bands[nu].q[k];
}

void model_rebuild_tables(crs_model m, hipStream_t s) {
  CRS_HIP(hipStreamSynchronize(s));
  build_mix_tables(m, s);
  build_pinv_tables(m, s);
  if (m->has_diag) build_diag(m, s);
  m->execs.clear();
  CRS_HIP(hipStreamSynchronize(s));
}

void launch_philox_normals(uint64_t seed, uint64_t stream, uint64_t rhs0, int nrhs, int64_t n, double* out,
                           hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  int64_t nb = ((n + 3) / 4 + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_philox_normals, dim3((unsigned)nb, nrhs), dim3(256), 0, s, seed, stream, rhs0, n, out);
  CRS_HIP(hipGetLastError());
}

// omega_1 (per band, streams 0x100 + nu) and omega_2 (stream 0x200) of the
// constrained-realization right-hand side into the model's buffers.
void model_draw_omegas(crs_model m, int nrhs, uint64_t seed, std::vector<const double*>& w1,
                       const double*& w2, hipStream_t s) {
  int64_t tot = 0;
  for (auto& b : m->bands) tot += b.npix;
  m->om1.alloc((size_t)tot * nrhs);
  m->om2.alloc((size_t)m->n * nrhs);
  w1.assign(m->nbands, nullptr);
  int64_t o = 0;
  for (int nu = 0; nu < m->nbands; ++nu) {
    const int64_t np = m->bands[nu].npix;
    launch_philox_normals(seed, (uint64_t)(0x100 + nu), 0, nrhs, np, m->om1.p + o, s);
    w1[nu] = m->om1.p + o;
    o += np * nrhs;
  }
  launch_philox_normals(seed, 0x200, 0, nrhs, m->n, m->om2.p, s);
  w2 = m->om2.p;
}
}  // namespace crs

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
    }
    m->d_lk.upload(m->lk, s);
    m->d_coff.upload(m->coff, s);
    build_ftab(m.get(), s);
    build_mix_tables(m.get(), s);
    build_pinv_tables(m.get(), s);
    if (d->flags & CRS_MODEL_DIAG) {
      build_diag(m.get(), s);
      m->has_diag = true;
    }
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

int crs_model_plan_bytes(crs_model m, int nrhs, int64_t* model_bytes, int64_t* exec_bytes) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && nrhs >= 1, CRS_EINVAL, "model is NULL or nrhs < 1");
    if (model_bytes) {
      int64_t b = 0;
      const int64_t nl = m->Lmax + 1;
      b += 4 * nl * m->nbands * m->ncomp * 8;                             // mixing and U^+ tables
      b += 3 * nl * m->ncomp * 8 + nl * m->ncomp * m->ncomp * 8;          // prior terms
      if (m->has_diag) b += (int64_t)(m->Lc + 1) * (m->Lc + 1) * m->ncomp * m->ncomp * 8;  // M_diag
      for (const Band& bd : m->bands) b += 2 * bd.npix * 8;               // tau and T^+ weights
      *model_bytes = b;
    }
    if (exec_bytes) *exec_bytes = exec_plan_bytes({m}, nrhs);
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

int crs_model_merge_observations(crs_model m, const int* group, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr, CRS_EINVAL, "model is NULL");
    hipStream_t s = (hipStream_t)st;
    std::vector<int> grp(m->nbands, -1);
    if (group)
      for (int nu = 0; nu < m->nbands; ++nu) grp[nu] = group[nu] < 0 ? -1 : group[nu];
    std::vector<char> drop(m->nbands, 0);
    for (int nu = 0; nu < m->nbands; ++nu) {
      if (grp[nu] < 0) continue;
      for (int r = 0; r < nu; ++r)
        if (grp[r] == grp[nu]) {
          CRS_CHECK(m->bands[r].grid == m->bands[nu].grid && m->bands[r].lmax == m->bands[nu].lmax, CRS_EINVAL,
                    "merged observations must share their grid and band-limit");
          drop[nu] = 1;  // the lowest band index of a group keeps the row
          break;
        }
    }
    CRS_HIP(hipStreamSynchronize(s));
    m->merge_group = grp;
    m->pi_drop = drop;
    build_pinv_tables(m, s);
    m->execs.clear();  // per-band merge flags are part of every Exec's tables
    CRS_HIP(hipStreamSynchronize(s));
    return CRS_OK;
  });
}

int apply_A(crs_model m, int nrhs, const double* x, double* y, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, x, y);
    exec_apply(model_exec(m, nrhs, (hipStream_t)st), OP_A, x, y, (hipStream_t)st);
    return CRS_OK;
  });
}

int apply_pinv_precond(crs_model m, int nrhs, const double* r, double* z, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, r, z);
    exec_apply(model_exec(m, nrhs, (hipStream_t)st), OP_PI, r, z, (hipStream_t)st);
    return CRS_OK;
  });
}

int apply_diag_precond(crs_model m, int nrhs, const double* r, double* z, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, r, z);
    CRS_CHECK(m->has_diag, CRS_EINVAL, "model was created without CRS_MODEL_DIAG");
    exec_diag(model_exec(m, nrhs, (hipStream_t)st), r, z, (hipStream_t)st);
    return CRS_OK;
  });
}

int pcg_solve(crs_model m, int precond, int nrhs, const double* b, double* x, double rtol, int maxiter,
              int* iters, double* relres, double* history, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, b, x);
    hipStream_t s = (hipStream_t)st;
    return exec_pcg(model_exec(m, nrhs, s), precond, b, x, rtol, maxiter, iters, relres, history, false, s);
  });
}

int build_rhs(crs_model m, int nrhs, const double* const* d, const double* const* omega1,
              const double* omega2, double* b, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && b != nullptr, CRS_EINVAL, "model or b is NULL");
    CRS_CHECK(nrhs >= 1, CRS_EINVAL, "nrhs must be >= 1");
    hipStream_t s = (hipStream_t)st;
    exec_rhs(model_exec(m, nrhs, s), sys_band_ptrs(m, nrhs, d), sys_band_ptrs(m, nrhs, omega1), omega2, b, s);
    return CRS_OK;
  });
}

int crs_model_project(crs_model m, int nrhs, const double* x, double* const* maps, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && x != nullptr && maps != nullptr, CRS_EINVAL, "model, x or maps is NULL");
    CRS_CHECK(nrhs >= 1, CRS_EINVAL, "nrhs must be >= 1");
    for (int nu = 0; nu < m->nbands; ++nu) CRS_CHECK(maps[nu] != nullptr, CRS_EINVAL, "maps entry is NULL");
    hipStream_t s = (hipStream_t)st;
    std::vector<std::vector<double*>> mp(nrhs, std::vector<double*>(m->nbands));
    for (int r = 0; r < nrhs; ++r)
      for (int nu = 0; nu < m->nbands; ++nu) mp[r][nu] = maps[nu] + (int64_t)r * m->bands[nu].npix;
    exec_project(model_exec(m, nrhs, s), x, mp, s);
    return CRS_OK;
  });
}

int apply_prior_inv(crs_model m, int nrhs, const double* x, double* y, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, x, y);
    exec_prior_inv(model_exec(m, nrhs, (hipStream_t)st), x, y, (hipStream_t)st);
    return CRS_OK;
  });
}

int apply_dA_dmix(crs_model m, int nrhs, const double* lam, const double* x, double* dq, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, lam, x);
    CRS_CHECK(m->varmix.empty(), CRS_EUNSUPPORTED, "mixing gradients with spatially varying mixing maps");
    CRS_CHECK(dq != nullptr, CRS_EINVAL, "dq is NULL");
    hipStream_t s = (hipStream_t)st;
    // systems [x_0 .. x_{nrhs-1}, lam_0 .. lam_{nrhs-1}] through the band round trips
    Exec& e = model_exec(m, 2 * nrhs, s);
    const size_t nn = (size_t)nrhs * m->n;
    m->gwork.alloc(2 * nn);
    CRS_HIP(hipMemcpyAsync(m->gwork.p, x, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
    CRS_HIP(hipMemcpyAsync(m->gwork.p + nn, lam, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
    exec_bands(e, OP_A, m->gwork.p, s);
    // -(lam_k . V(x) + x_k . V(lam)); lam_r sits at system nrhs + r of gwork
    exec_mix_grad(e, m->gwork.p + nn, 0, m->gwork.p, nrhs, nrhs, -1.0, m->beamtab.p, dq, s);
    return CRS_OK;
  });
}

int apply_db_dmix(crs_model m, int nrhs, const double* lam, const double* const* d, double* dq, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, lam, dq);
    CRS_CHECK(m->varmix.empty(), CRS_EUNSUPPORTED, "mixing gradients with spatially varying mixing maps");
    CRS_CHECK(d != nullptr, CRS_EINVAL, "d is NULL");
    hipStream_t s = (hipStream_t)st;
    Exec& e = model_exec(m, nrhs, s);
    exec_rhs_bands(e, sys_band_ptrs(m, nrhs, d), {}, s);
    exec_mix_grad(e, lam, 0, nullptr, 0, nrhs, 1.0, m->beamtab.p, dq, s);
    return CRS_OK;
  });
}

int crs_prior_quad(crs_model m, int nrhs, const double* x, double* y, double* val, crs_stream st) {
  return guarded([&] {
    check_vec(m, nrhs, x, y);
    CRS_CHECK(val != nullptr, CRS_EINVAL, "val is NULL");
    hipStream_t s = (hipStream_t)st;
    exec_prior_quad(model_exec(m, nrhs, s), x, y, val, s);
    return CRS_OK;
  });
}

int crs_chi2(crs_model m, int nrhs, const double* x, const double* const* d, double* const* res, double* val,
             crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && x != nullptr && res != nullptr && val != nullptr, CRS_EINVAL,
              "model, x, res or val is NULL");
    CRS_CHECK(nrhs >= 1, CRS_EINVAL, "nrhs must be >= 1");
    for (int nu = 0; nu < m->nbands; ++nu) CRS_CHECK(res[nu] != nullptr, CRS_EINVAL, "res entry is NULL");
    hipStream_t s = (hipStream_t)st;
    std::vector<std::vector<double*>> rp(nrhs, std::vector<double*>(m->nbands));
    for (int r = 0; r < nrhs; ++r)
      for (int nu = 0; nu < m->nbands; ++nu) rp[r][nu] = res[nu] + (int64_t)r * m->bands[nu].npix;
    exec_chi2(model_exec(m, nrhs, s), x, sys_band_ptrs(m, nrhs, d), rp, val, s);
    return CRS_OK;
  });
}

int crs_noise_weight(crs_model m, int nrhs, double scale, const double* const* in, double* const* out,
                     crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && out != nullptr, CRS_EINVAL, "model or out is NULL");
    CRS_CHECK(nrhs >= 1, CRS_EINVAL, "nrhs must be >= 1");
    for (int nu = 0; nu < m->nbands; ++nu) CRS_CHECK(out[nu] != nullptr, CRS_EINVAL, "out entry is NULL");
    hipStream_t s = (hipStream_t)st;
    std::vector<std::vector<double*>> op(nrhs, std::vector<double*>(m->nbands));
    for (int r = 0; r < nrhs; ++r)
      for (int nu = 0; nu < m->nbands; ++nu) op[r][nu] = out[nu] + (int64_t)r * m->bands[nu].npix;
    exec_noise_weight(model_exec(m, nrhs, s), scale, sys_band_ptrs(m, nrhs, in), op, s);
    return CRS_OK;
  });
}

int crs_philox_normals(uint64_t seed, uint64_t stream, uint64_t rhs, int64_t n, double* out, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(out != nullptr && n >= 0, CRS_EINVAL, "out is NULL or n < 0");
    launch_philox_normals(seed, stream, rhs, 1, n, out, (hipStream_t)st);
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
    Exec& e = model_exec(m, nrhs, s);
    std::vector<const double*> w1;
    const double* w2 = nullptr;
    if (mode == CRS_MODE_CR) model_draw_omegas(m, nrhs, seed, w1, w2, s);
    // the right-hand side is kept in a model-owned buffer
    m->bcr.alloc((size_t)m->n * nrhs);
    exec_rhs(e, sys_band_ptrs(m, nrhs, d), sys_band_ptrs(m, nrhs, mode == CRS_MODE_CR ? w1.data() : nullptr), w2,
             m->bcr.p, s);
    CRS_HIP(hipMemsetAsync(x, 0, (size_t)m->n * nrhs * sizeof(double), s));
    const int rc = exec_pcg(e, precond, m->bcr.p, x, rtol, maxiter, iters, relres, nullptr, false, s);
    CRS_HIP(hipStreamSynchronize(s));
    return rc;
  });
}

}  // extern "C"
