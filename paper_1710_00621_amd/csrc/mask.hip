// Mask-restricted preconditioner M_mask and M_add = M_PI + M_mask.
//
//   M_mask = Z^T (Z S^-1 Z^T)^-1 Z                  (Sect. 4.2, eq:M_mask)
//   Z = (masked pixels of) Y R,  r_l = exp(-beta l^2 (l+1)^2),  r_{L/2}^2 = 0.05
//                                                    (Sect. 4.3, eq:rl)
//   G = Z S^-1 Z^T = Y D Y^T,  d_l = r_l^2 / C_l     (Sect. 4.4, eq:W)
//
// (Z S^-1 Z^T)^-1 is approximated by the multigrid V-cycle of fig:code:mg on
// a hierarchy of HEALPix grids: Nside halves and the band-limit halves per
// level, a coarse pixel is in the level's mask when its four children are,
// the restriction I_h^H = Y_H R_H Y_h^T W_h uses a Gaussian R_H whose FWHM is
// the coarse pixel size, D_H = R_H^2 D_h, the smoother is omega / diag(G_h)
// (one constant per level: sum_l d_l (2l+1) / 4 pi), and the first level with
// fewer than nbottom masked pixels is solved with the pseudo-inverse of its
// dense G (addition theorem, eigenvalues below rcond * max dropped).  The
// cycle is the optimized form with J = Y_h^T W_h Y_h taken as I: six SHTs per
// level.  Each component with a prior runs its own cycle (S is block
// diagonal); all of them, for every right-hand side, share the launches.
//
// Vectors of a level are full maps that are zero outside the level's mask.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "model.h"

namespace crs {

namespace {

__host__ __device__ inline int64_t nalm_of(int L) { return (int64_t)(L + 1) * (L + 1); }

// HEALPix RING index of the point (z, phi) at nside (Gorski et al. 2005):
// equatorial zone by the two edge-line indices, polar caps by the distance
// to the pole.
int64_t ang2pix_ring(int nside, double z, double phi) {
  const double twopi = 2.0 * M_PI;
  phi = std::fmod(phi, twopi);
  if (phi < 0) phi += twopi;
  const int64_t ns = nside;
  const double tt = phi / (0.5 * M_PI);
  const double za = std::fabs(z);
  if (za <= 2.0 / 3.0) {
    const double t1 = ns * (0.5 + tt), t2 = ns * z * 0.75;
    const int64_t jp = (int64_t)std::floor(t1 - t2), jm = (int64_t)std::floor(t1 + t2);
    const int64_t ir = ns + 1 + jp - jm;
    const int64_t kshift = 1 - (ir & 1);
    int64_t ip = (jp + jm - ns + kshift + 1) / 2;
    ip = ((ip % (4 * ns)) + 4 * ns) % (4 * ns);
    return 2 * ns * (ns - 1) + (ir - 1) * 4 * ns + ip;
  }
  const double tp = tt - std::floor(tt);
  const double tmp = ns * std::sqrt(3.0 * (1.0 - za));
  const int64_t jp = (int64_t)std::floor(tp * tmp), jm = (int64_t)std::floor((1.0 - tp) * tmp);
  const int64_t ir = jp + jm + 1;
  int64_t ip = (int64_t)std::floor(tt * ir);
  ip = ((ip % (4 * ir)) + 4 * ir) % (4 * ir);
  return z > 0 ? 2 * ir * (ir - 1) + ip : 12 * ns * ns - 2 * ir * (ir + 1) + ip;
}

void pixel_centres(crs_grid g, std::vector<double>& z, std::vector<double>& phi) {
  z.resize(g->npix);
  phi.resize(g->npix);
  for (int r = 0; r < g->nring; ++r)
    for (int j = 0; j < g->nphi[r]; ++j) {
      const int64_t i = g->offset[r] + j;
      z[i] = g->z[r];
      phi[i] = M_PI * g->phi0_num[r] / g->phi0_den[r] + 2.0 * M_PI * j / g->nphi[r];
    }
}

// bottom level: x_j[idx[i]] = sum_k Gp_c[i][k] b_j[idx[k]] (x_j is zero elsewhere)
__global__ __launch_bounds__(256) void k_bottom(double* __restrict__ x, const double* __restrict__ b, int64_t npix,
                                                const int* __restrict__ idx, int n,
                                                const double* __restrict__ Gp, const int* __restrict__ mc,
                                                MapSkip skip) {
  extern __shared__ double bs[];
  const int j = blockIdx.y;
  if (skip.off(j)) return;
  const double* bj = b + (int64_t)j * npix;
  for (int k = threadIdx.x; k < n; k += blockDim.x) bs[k] = bj[idx[k]];
  __syncthreads();
  const double* G = Gp + (int64_t)mc[j] * n * n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* gi = G + (int64_t)i * n;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) acc = fma(gi[k], bs[k], acc);
  x[(int64_t)j * npix + idx[i]] = acc;
}

// Gp[i][j] = sum_k V[i][k] w[k] V[j][k]  (V column-major n x n)
__global__ void k_form_pinv(double* __restrict__ Gp, const double* __restrict__ V, const double* __restrict__ w,
                            int n) {
  const int i = blockIdx.y;
  const int jj = blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= n) return;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) {
    const double wk = w[k];
    if (wk != 0.0) acc = fma(V[(int64_t)k * n + i] * wk, V[(int64_t)k * n + jj], acc);
  }
  Gp[(int64_t)i * n + jj] = acc;
}

}  // namespace

// ------------------------------------------------------------ structures
struct MaskLevel {
  crs_grid grid = nullptr;
  bool owned = false;
  int nside = 0, lmax = 0;
  int nmasked = 0;
  double w = 0.0;                // quadrature weight 4 pi / Npix
  DevBuf<double> ind;            // 0/1 per pixel
  DevBuf<int> idx;               // masked pixels (bottom level)
  DevBuf<double> rH;             // restriction filter to the next level, L_{h+1} + 1 entries
  DevBuf<double> D;              // [ncm][L_h + 1]: d_l per masked component
  std::vector<double> smooth;    // per masked component: omega / diag(G_h)
};

struct MaskMG {
  std::vector<MaskLevel> levels;
  std::vector<int> comps;        // components with a prior
  int L0 = 0;
  double omega = 0.2, rcond = 1e-6, r2half = 0.05;
  int nbottom = 1000;
  bool exact_j = false;          // J = Y_h^T W_h Y_h applied exactly (else taken as I)
  DevBuf<double> ones;           // l-table of ones (unscaled subtraction in k_from_parts)
  DevBuf<double> rtop;           // r_l at L0 (the low-pass of Z)
  DevBuf<double> gplus;          // [ncm][n_b][n_b] bottom pseudo-inverses
  ~MaskMG() {
    for (auto& l : levels)
      if (l.owned) crs_grid_destroy(l.grid);
  }
};

void MaskMGDel::operator()(MaskMG* p) const { delete p; }

namespace {

// The per-Exec state of one problem's cycle: nm = (systems of the problem) x
// (masked components) maps, level buffers and the transform scratch.
struct MaskRunImpl {
  int prob = 0, nm = 0, ncm = 0;
  std::vector<int> sys_of;                   // per map: system
  DevBuf<int> mc, mapsys;                    // per map: masked component index, system
  DevBuf<int64_t> off_top;                   // per map: offset of its component vector in the stacked vectors
  std::vector<DevBuf<double>> b, x, y, u, rt, ct;  // per level
  std::vector<DevBuf<double>> jv;            // per level (exact J): J applied to a vector at L_h
  std::vector<DevBuf<double>> sm;            // per level: per-map smoother constant
  ShtScratch sc;                              // transform scratch of every level
};

}  // namespace

struct MaskRun : MaskRunImpl {};

void MaskRunDel::operator()(MaskRun* p) const { delete p; }

namespace {

void synth_ws(crs_grid g, int L, int nm, const double* hat, double* map, MaskRun& r, MapSkip skip, hipStream_t s) {
  scratch_synth(r.sc, g, L, nm, hat, map, skip, s);
}

int adjoint_ws(crs_grid g, int L, int nm, const double* map, MaskRun& r, MapSkip skip, hipStream_t s) {
  return scratch_adjoint(r.sc, g, L, nm, map, skip, s);
}

void map_op(int op, MaskRun& r, double* x, const double* b, const double* y, const double* ind, const double* sm,
            double alpha, int64_t npix, MapSkip skip, hipStream_t s) {
  launch_map_op(op, x, b, y, ind, sm, alpha, npix, r.nm, skip, s);
}

// out = J v = W_h Y_h^T (mask_h) Y_h v at band-limit L, v given as hat
// vectors in the scratch; map: a level map buffer for the synthesis
void apply_j(const MaskLevel& lv, int L, const ShtPlan& p, MaskRun& r, double* map, double* out, MapSkip skip,
             hipStream_t s) {
  const int nm = r.nm;
  synth_ws(lv.grid, L, nm, r.sc.hat.p, map, r, skip, s);
  map_op(MOP_MASK, r, map, nullptr, nullptr, lv.ind.p, nullptr, 0.0, lv.grid->npix, skip, s);
  const int nt = adjoint_ws(lv.grid, L, nm, map, r, skip, s);
  launch_from_parts(out, (const int64_t*)nullptr, L, 0, lv.w, p.hs.p, r.sc.parts.p, nt, (int64_t)nm * nalm_of(L),
                    (const double*)nullptr, 0, (const double*)nullptr, 0, (int64_t)0, (const double*)nullptr, 0,
                    r.mc.p, nm, skip, s);
}

void vcycle(const MaskMG& mg, MaskRun& r, int h, MapSkip skip, hipStream_t s) {
  const MaskLevel& lv = mg.levels[h];
  const int64_t np = lv.grid->npix;
  const int nm = r.nm;
  if (h + 1 == (int)mg.levels.size()) {
    map_op(MOP_ZERO, r, r.x[h].p, nullptr, nullptr, nullptr, nullptr, 0.0, np, skip, s);
    if (lv.nmasked > 0) {
      dim3 gr((lv.nmasked + 255) / 256, nm);
      hipLaunchKernelGGL(k_bottom, gr, dim3(256), (size_t)lv.nmasked * sizeof(double), s, r.x[h].p, r.b[h].p, np,
                         lv.idx.p, lv.nmasked, mg.gplus.p, r.mc.p, skip);
      CRS_HIP(hipGetLastError());
    }
    return;
  }
  const MaskLevel& cv = mg.levels[h + 1];
  const int Lh = lv.lmax, LH = cv.lmax;
  const ShtPlan& ph = get_plan(lv.grid, Lh, s);
  const ShtPlan& pH = get_plan(lv.grid, LH, s);
  // x = M_h b
  map_op(MOP_SCALE, r, r.x[h].p, r.b[h].p, nullptr, nullptr, r.sm[h].p, 0.0, np, skip, s);
  // u = Y_h^T x                                               (L_h, N_h)
  int nt = adjoint_ws(lv.grid, Lh, nm, r.x[h].p, r, skip, s);
  launch_from_parts(r.u[h].p, (const int64_t*)nullptr, Lh, 0, 1.0,
                     ph.hs.p, r.sc.parts.p, nt, (int64_t)nm * nalm_of(Lh), (const double*)nullptr, 0,
                     (const double*)nullptr, 0, (int64_t)0, (const double*)nullptr, 0, r.mc.p, nm, skip, s);
  // exact J: jv = J D_h u = W_h Y_h^T (mask_h) Y_h D_h u       (L_h, N_h)
  if (mg.exact_j) {
    launch_hat_from(r.sc.hat.p, Lh, ph.hs.p, (const double*)r.u[h].p, Lh, (const int64_t*)nullptr, nalm_of(Lh),
                    (const double*)nullptr, 0, (int64_t)0, lv.D.p, Lh + 1, r.mc.p, nm, skip, s);
    apply_j(lv, Lh, ph, r, r.y[h].p, r.jv[h].p, skip, s);
  }
  // r~ = W_h Y_h^T b - D_h u (J D_h u with exact J), at L_H  (L_H, N_h)
  nt = adjoint_ws(lv.grid, LH, nm, r.b[h].p, r, skip, s);
  if (mg.exact_j) {
    launch_from_parts(r.rt[h].p, (const int64_t*)nullptr, LH, 0, lv.w, pH.hs.p, r.sc.parts.p, nt,
                      (int64_t)nm * nalm_of(LH), (const double*)nullptr, 0, r.jv[h].p, Lh, nalm_of(Lh),
                      mg.ones.p, 0, r.mc.p, nm, skip, s);
  } else {
    launch_from_parts(r.rt[h].p, (const int64_t*)nullptr, LH, 0,
                       lv.w, pH.hs.p, r.sc.parts.p, nt, (int64_t)nm * nalm_of(LH), (const double*)nullptr, 0, r.u[h].p, Lh,
                       nalm_of(Lh), lv.D.p, Lh + 1, r.mc.p, nm, skip, s);
  }
  // r_H = (mask_H) Y_H R_H r~                                (L_H, N_H)
  launch_hat_from(r.sc.hat.p, LH, get_plan(cv.grid, LH, s).hs.p,
                     (const double*)r.rt[h].p, LH, (const int64_t*)nullptr, nalm_of(LH), (const double*)nullptr, 0,
                     (int64_t)0, lv.rH.p, 0, r.mc.p, nm, skip, s);
  CRS_HIP(hipGetLastError());
  synth_ws(cv.grid, LH, nm, r.sc.hat.p, r.b[h + 1].p, r, skip, s);
  map_op(MOP_MASK, r, r.b[h + 1].p, nullptr, nullptr, cv.ind.p, nullptr, 0.0, cv.grid->npix, skip, s);
  vcycle(mg, r, h + 1, skip, s);
  // c~ = R_H Y_H^T c_H                                       (L_H, N_H)
  nt = adjoint_ws(cv.grid, LH, nm, r.x[h + 1].p, r, skip, s);
  launch_from_parts(r.ct[h].p, (const int64_t*)nullptr, LH, 0,
                     1.0, get_plan(cv.grid, LH, s).hs.p, r.sc.parts.p, nt, (int64_t)nm * nalm_of(LH), lv.rH.p, 0,
                     (const double*)nullptr, 0, (int64_t)0, (const double*)nullptr, 0, r.mc.p, nm, skip, s);
  // x += (mask_h) W_h Y_h c~                                 (L_H, N_h)
  launch_hat_from(r.sc.hat.p, LH, pH.hs.p, (const double*)r.ct[h].p,
                     LH, (const int64_t*)nullptr, nalm_of(LH), (const double*)nullptr, 0, (int64_t)0,
                     (const double*)nullptr, 0, r.mc.p, nm, skip, s);
  CRS_HIP(hipGetLastError());
  synth_ws(lv.grid, LH, nm, r.sc.hat.p, r.y[h].p, r, skip, s);
  map_op(MOP_AXPY_MASK, r, r.x[h].p, nullptr, r.y[h].p, lv.ind.p, nullptr, lv.w, np, skip, s);
  // x += M_h (b - (mask_h) Y_h D_h (u + c~))                 (L_h, N_h)
  // (exact J: u + J c~, J c~ = W_h Y_h^T (mask_h) Y_h c~ at L_h)
  if (mg.exact_j) {
    launch_hat_from(r.sc.hat.p, Lh, ph.hs.p, (const double*)r.ct[h].p, LH, (const int64_t*)nullptr, nalm_of(LH),
                    (const double*)nullptr, 0, (int64_t)0, (const double*)nullptr, 0, r.mc.p, nm, skip, s);
    apply_j(lv, Lh, ph, r, r.y[h].p, r.jv[h].p, skip, s);
    launch_hat_from(r.sc.hat.p, Lh, ph.hs.p, (const double*)r.u[h].p, Lh, (const int64_t*)nullptr, nalm_of(Lh),
                    (const double*)r.jv[h].p, Lh, nalm_of(Lh), lv.D.p, Lh + 1, r.mc.p, nm, skip, s);
  } else {
    launch_hat_from(r.sc.hat.p, Lh, ph.hs.p, (const double*)r.u[h].p,
                       Lh, (const int64_t*)nullptr, nalm_of(Lh), (const double*)r.ct[h].p, LH, nalm_of(LH), lv.D.p,
                       Lh + 1, r.mc.p, nm, skip, s);
  }
  CRS_HIP(hipGetLastError());
  synth_ws(lv.grid, Lh, nm, r.sc.hat.p, r.y[h].p, r, skip, s);
  map_op(MOP_POST, r, r.x[h].p, r.b[h].p, r.y[h].p, lv.ind.p, r.sm[h].p, 0.0, np, skip, s);
}

}  // namespace

// ------------------------------------------------------------ setup
// d_l at level 0 = r_l^2 C_l^-1; at level h+1 d_{h+1} = rH_h^2 d_h (up to L_{h+1}).
void build_mask(crs_model m, crs_grid g, const uint8_t* mask, const crs_mask_opts* o, hipStream_t s) {
  std::unique_ptr<MaskMG, MaskMGDel> mg(new MaskMG);
  if (o) {
    if (o->lowpass_r2 > 0) mg->r2half = o->lowpass_r2;
    if (o->omega > 0) mg->omega = o->omega;
    if (o->nbottom > 0) mg->nbottom = o->nbottom;
    if (o->rcond > 0) mg->rcond = o->rcond;
    mg->exact_j = o->exact_j != 0;
  }
  CRS_CHECK(mg->r2half < 1.0, CRS_EINVAL, "lowpass_r2 must be in (0, 1)");
  for (int k = 0; k < m->ncomp; ++k) {
    bool any = false;
    for (double v : m->invcl[k]) any = any || v > 0.0;
    if (any) mg->comps.push_back(k);
  }
  CRS_CHECK(!mg->comps.empty(), CRS_EINVAL, "no component has a prior: the mask-restricted system is empty");
  mg->L0 = m->lk[mg->comps[0]];
  for (int k : mg->comps)
    CRS_CHECK(m->lk[k] == mg->L0, CRS_EUNSUPPORTED,
              "the components with a prior must share one band-limit for the mask preconditioner");
  const int ncm = (int)mg->comps.size();
  // levels
  std::vector<uint8_t> cur(mask, mask + g->npix);
  crs_grid gh = g;
  int L = mg->L0;
  std::vector<double> zc, pc;
  while (true) {
    MaskLevel lv;
    lv.grid = gh;
    lv.owned = gh != g;
    lv.nside = gh->nside;
    lv.lmax = L;
    lv.w = 4.0 * M_PI / (double)gh->npix;
    std::vector<double> ind(gh->npix);
    std::vector<int> idx;
    for (int64_t i = 0; i < gh->npix; ++i) {
      ind[i] = cur[i] ? 1.0 : 0.0;
      if (cur[i]) idx.push_back((int)i);
    }
    lv.nmasked = (int)idx.size();
    lv.ind.upload(ind, s);
    const bool bottom = lv.nmasked < mg->nbottom || lv.nside < 2 || (lv.nside % 2) != 0 || L < 2;
    if (bottom) lv.idx.upload(idx, s);
    mg->levels.push_back(std::move(lv));
    if (bottom) break;
    // the coarse mask: pixels whose four children are all masked
    const int nsc = gh->nside / 2;
    pixel_centres(gh, zc, pc);
    std::vector<int> cover((size_t)12 * nsc * nsc, 0);
    for (int i : idx) cover[ang2pix_ring(nsc, zc[i], pc[i])] += 1;
    crs_grid gc = nullptr;
    const int st = crs_grid_healpix(nsc, &gc);
    CRS_CHECK(st == CRS_OK, st, "could not create a coarse HEALPix grid");
    cur.assign(cover.size(), 0);
    for (size_t i = 0; i < cover.size(); ++i) cur[i] = cover[i] == 4 ? 1 : 0;
    gh = gc;
    L = L / 2;
  }
  const int nlev = (int)mg->levels.size();
  // filters: r_l (top), rH per level, d per level and component
  const int L0 = mg->L0;
  const double hh = 0.5 * L0;
  const double beta = L0 > 0 ? -std::log(mg->r2half) / (2.0 * hh * hh * (hh + 1.0) * (hh + 1.0)) : 0.0;
  std::vector<double> rl(L0 + 1);
  for (int l = 0; l <= L0; ++l) rl[l] = std::exp(-beta * (double)l * l * (l + 1.0) * (l + 1.0));
  mg->rtop.upload(rl, s);
  const std::vector<double> ones_h((size_t)L0 + 1, 1.0);  // alive until the stream sync below
  mg->ones.upload(ones_h, s);
  std::vector<std::vector<double>> d(ncm, std::vector<double>(L0 + 1, 0.0));
  for (int c = 0; c < ncm; ++c)
    for (int l = 0; l <= L0; ++l) d[c][l] = rl[l] * rl[l] * m->invcl[mg->comps[c]][l];
  for (int h = 0; h < nlev; ++h) {
    MaskLevel& lv = mg->levels[h];
    const int Lh = lv.lmax;
    std::vector<double> D((size_t)ncm * (Lh + 1));
    lv.smooth.assign(ncm, 0.0);
    for (int c = 0; c < ncm; ++c) {
      double diag = 0.0;
      for (int l = 0; l <= Lh; ++l) {
        D[(size_t)c * (Lh + 1) + l] = d[c][l];
        diag += d[c][l] * (2.0 * l + 1.0) / (4.0 * M_PI);
      }
      lv.smooth[c] = diag > 0 ? mg->omega / diag : 0.0;
    }
    lv.D.upload(D, s);
    if (h + 1 < nlev) {
      const int LH = mg->levels[h + 1].lmax;
      const int nsc = mg->levels[h + 1].nside;
      const double fwhm = std::sqrt(4.0 * M_PI / (12.0 * nsc * nsc));
      const double sig = fwhm / std::sqrt(8.0 * std::log(2.0));
      std::vector<double> rH(LH + 1);
      for (int l = 0; l <= LH; ++l) rH[l] = std::exp(-0.5 * l * (l + 1.0) * sig * sig);
      lv.rH.upload(rH, s);
      for (int c = 0; c < ncm; ++c) {
        d[c].resize(LH + 1);
        for (int l = 0; l <= LH; ++l) d[c][l] *= rH[l] * rH[l];
      }
    }
    // Legendre and ring tables of every transform the cycle runs (setup, not hot path)
    get_plan(lv.grid, Lh, s);
    if (h + 1 < nlev) get_plan(lv.grid, mg->levels[h + 1].lmax, s);
  }
  // bottom: dense G per component by the addition theorem, pseudo-inverse by
  // a symmetric eigendecomposition (rocSOLVER)
  MaskLevel& bt = mg->levels.back();
  const int n = bt.nmasked;
  CRS_CHECK(n <= 8192, CRS_EUNSUPPORTED,
            "the mask hierarchy ends (odd Nside or band-limit below 2) with more than 8192 masked pixels");
  if (n > 0) {
    std::vector<int> idx(n);
    CRS_HIP(hipMemcpyAsync(idx.data(), bt.idx.p, n * sizeof(int), hipMemcpyDeviceToHost, s));
    CRS_HIP(hipStreamSynchronize(s));
    pixel_centres(bt.grid, zc, pc);
    std::vector<double> vx(n), vy(n), vz(n);
    for (int i = 0; i < n; ++i) {
      const double z = zc[idx[i]], st = std::sqrt(std::max(0.0, (1.0 - z) * (1.0 + z)));
      vx[i] = st * std::cos(pc[idx[i]]);
      vy[i] = st * std::sin(pc[idx[i]]);
      vz[i] = z;
    }
    const int Lb = bt.lmax;
    mg->gplus.alloc((size_t)ncm * n * n);
    rocblas_handle hb = nullptr;
    CRS_CHECK(rocblas_create_handle(&hb) == rocblas_status_success, CRS_EHIP, "rocblas_create_handle failed");
    std::unique_ptr<_rocblas_handle, rocblas_status (*)(rocblas_handle)> hold(hb, rocblas_destroy_handle);
    CRS_CHECK(rocblas_set_stream(hb, s) == rocblas_status_success, CRS_EHIP, "rocblas_set_stream failed");
    DevBuf<double> A, ev, E, w;
    DevBuf<int> info;
    A.alloc((size_t)n * n);
    ev.alloc(n);
    E.alloc(n);
    w.alloc(n);
    info.alloc(1);
    std::vector<double> G((size_t)n * n), P(Lb + 1), evh(n), wh(n);
    for (int c = 0; c < ncm; ++c) {
      std::vector<double> coef(Lb + 1);
      for (int l = 0; l <= Lb; ++l) coef[l] = d[c][l] * (2.0 * l + 1.0) / (4.0 * M_PI);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
          const double x = std::max(-1.0, std::min(1.0, vx[i] * vx[j] + vy[i] * vy[j] + vz[i] * vz[j]));
          // Legendre polynomials by Bonnet's recurrence
          double p0 = 1.0, p1 = x, acc = coef[0];
          if (Lb >= 1) acc += coef[1] * x;
          for (int l = 2; l <= Lb; ++l) {
            const double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
            acc += coef[l] * p2;
            p0 = p1;
            p1 = p2;
          }
          G[(size_t)i * n + j] = G[(size_t)j * n + i] = acc;
        }
      A.upload(G, s);
      CRS_CHECK(rocsolver_dsyevd(hb, rocblas_evect_original, rocblas_fill_upper, n, A.p, n, ev.p, E.p, info.p) ==
                    rocblas_status_success,
                CRS_EHIP, "rocsolver_dsyevd failed");
      int ih = 0;
      CRS_HIP(hipMemcpyAsync(evh.data(), ev.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
      CRS_HIP(hipMemcpyAsync(&ih, info.p, sizeof(int), hipMemcpyDeviceToHost, s));
      CRS_HIP(hipStreamSynchronize(s));
      CRS_CHECK(ih == 0, CRS_EHIP, "rocsolver_dsyevd did not converge");
      double top = 0.0;
      for (double v : evh) top = std::max(top, std::fabs(v));
      for (int k = 0; k < n; ++k) wh[k] = std::fabs(evh[k]) > mg->rcond * top ? 1.0 / evh[k] : 0.0;
      w.upload(wh, s);
      hipLaunchKernelGGL(k_form_pinv, dim3((n + 255) / 256, n), dim3(256), 0, s, mg->gplus.p + (size_t)c * n * n, A.p,
                         w.p, n);
      CRS_HIP(hipGetLastError());
      CRS_HIP(hipStreamSynchronize(s));
    }
  }
  CRS_HIP(hipStreamSynchronize(s));
  m->mask = std::move(mg);
  // every Exec of the model rebuilds its cycle state on next use
  for (auto& kv : m->execs) kv.second->mask_runs.clear();
}

namespace {
MaskRun& mask_run(Exec& e, int p, hipStream_t s) {
  if (e.mask_runs.size() != e.probs.size()) e.mask_runs.resize(e.probs.size());
  auto& slot = e.mask_runs[p];
  if (slot) return *slot;
  const crs_model m = e.probs[p];
  const MaskMG& mg = *m->mask;
  std::unique_ptr<MaskRun, MaskRunDel> r(new MaskRun);
  r->prob = p;
  r->ncm = (int)mg.comps.size();
  std::vector<int> mc, ms;
  std::vector<int64_t> off;
  for (int sy = 0; sy < e.nsys; ++sy) {
    if (e.hsys[sy].prob != p) continue;
    for (int c = 0; c < r->ncm; ++c) {
      mc.push_back(c);
      ms.push_back(sy);
      off.push_back(e.hsys[sy].off + m->coff[mg.comps[c]]);
      r->sys_of.push_back(sy);
    }
  }
  r->nm = (int)mc.size();
  r->mc.upload(mc, s);
  r->mapsys.upload(ms, s);
  r->off_top.upload(off, s);
  const int nl = (int)mg.levels.size();
  r->b.resize(nl);
  r->x.resize(nl);
  r->y.resize(nl);
  r->u.resize(nl);
  r->rt.resize(nl);
  r->ct.resize(nl);
  r->sm.resize(nl);
  r->jv.resize(nl);
  for (int h = 0; h < nl; ++h) {
    const MaskLevel& lv = mg.levels[h];
    const size_t np = (size_t)lv.grid->npix * r->nm;
    r->b[h].alloc(np);
    r->x[h].alloc(np);
    r->y[h].alloc(np);
    std::vector<double> sm(r->nm);
    for (int j = 0; j < r->nm; ++j) sm[j] = lv.smooth[mc[j]];
    r->sm[h].upload(sm, s);
    std::vector<int> Ls = {lv.lmax};
    if (h + 1 < nl) Ls.push_back(mg.levels[h + 1].lmax);
    r->u[h].alloc((size_t)nalm_of(lv.lmax) * r->nm);
    if (mg.exact_j && h + 1 < nl) r->jv[h].alloc((size_t)nalm_of(lv.lmax) * r->nm);
    if (h + 1 < nl) {
      r->rt[h].alloc((size_t)nalm_of(Ls[1]) * r->nm);
      r->ct[h].alloc((size_t)nalm_of(Ls[1]) * r->nm);
    }
    for (int L : Ls) r->sc.reserve(lv.grid, L, r->nm, s);
  }
  CRS_HIP(hipStreamSynchronize(s));
  slot = std::move(r);
  return *slot;
}
}  // namespace

// z (+)= M_mask r for every system of e whose problem has a mask (act: skip
// finished systems; NULL: all).  Without accumulate, z is overwritten for the
// components the mask preconditioner acts on and left alone elsewhere.
void exec_mask(Exec& e, const double* r, double* z, bool accumulate, hipStream_t s, const double* act) {
  for (int p = 0; p < (int)e.probs.size(); ++p) {
    const crs_model m = e.probs[p];
    if (!m->mask) continue;
    const MaskMG& mg = *m->mask;
    MaskRun& run = mask_run(e, p, s);
    if (run.nm == 0) continue;
    MapSkip skip;
    if (act) {
      skip.mapsys = run.mapsys.p;
      skip.act = act;
    }
    const MaskLevel& l0 = mg.levels[0];
    const int L0 = mg.L0;
    const ShtPlan& p0 = get_plan(l0.grid, L0, s);
    // b_0 = (mask) Y R r_k
    launch_hat_from(run.sc.hat.p, L0, p0.hs.p, r, L0,
                       run.off_top.p, (int64_t)0, (const double*)nullptr, 0, (int64_t)0, mg.rtop.p, 0, run.mc.p, run.nm, skip, s);
    CRS_HIP(hipGetLastError());
    synth_ws(l0.grid, L0, run.nm, run.sc.hat.p, run.b[0].p, run, skip, s);
    map_op(MOP_MASK, run, run.b[0].p, nullptr, nullptr, l0.ind.p, nullptr, 0.0, l0.grid->npix, skip, s);
    vcycle(mg, run, 0, skip, s);
    // z_k (+)= R Y^T x_0
    const int nt = adjoint_ws(l0.grid, L0, run.nm, run.x[0].p, run, skip, s);
    launch_from_parts(z, run.off_top.p, L0, accumulate ? 1 : 0,
                       1.0, p0.hs.p, run.sc.parts.p, nt, (int64_t)run.nm * nalm_of(L0), mg.rtop.p, 0,
                       (const double*)nullptr, 0, (int64_t)0, (const double*)nullptr, 0, run.mc.p, run.nm, skip, s);
    CRS_HIP(hipGetLastError());
  }
}

void exec_mask_prepare(Exec& e, hipStream_t s) {
  for (int p = 0; p < (int)e.probs.size(); ++p)
    if (e.probs[p]->mask) mask_run(e, p, s);
}

bool exec_has_mask(const Exec& e) {
  for (const crs_model m : e.probs)
    if (!m->mask) return false;
  return !e.probs.empty();
}

}  // namespace crs

using namespace crs;

extern "C" {

int crs_model_set_mask(crs_model m, crs_grid g, const uint8_t* mask, const crs_mask_opts* opts, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && g != nullptr && mask != nullptr, CRS_EINVAL, "model, grid or mask is NULL");
    CRS_CHECK(g->kind == 0, CRS_EINVAL, "the mask grid must be a HEALPix grid");
    if (opts) {
      CRS_CHECK(opts->lowpass_r2 >= 0 && opts->omega >= 0 && opts->nbottom >= 0 && opts->rcond >= 0, CRS_EINVAL,
                "mask options must be >= 0 (0 selects the default)");
      CRS_CHECK(opts->nbottom <= 8192, CRS_EUNSUPPORTED, "nbottom above 8192 is not supported");
    }
    build_mask(m, g, mask, opts, (hipStream_t)st);
    return CRS_OK;
  });
}

int crs_model_mask_info(crs_model m, int* nlevels, int* out, int n) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && nlevels != nullptr, CRS_EINVAL, "model or nlevels is NULL");
    CRS_CHECK(m->mask != nullptr, CRS_EINVAL, "the model has no mask preconditioner (crs_model_set_mask)");
    const auto& lv = m->mask->levels;
    *nlevels = (int)lv.size();
    for (int h = 0; h < (int)lv.size() && out && 3 * h + 2 < n; ++h) {
      out[3 * h] = lv[h].nside;
      out[3 * h + 1] = lv[h].lmax;
      out[3 * h + 2] = lv[h].nmasked;
    }
    return CRS_OK;
  });
}

int apply_mask_precond(crs_model m, int nrhs, const double* r, double* z, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr && r != nullptr && z != nullptr, CRS_EINVAL, "model or vector pointer is NULL");
    CRS_CHECK(nrhs >= 1, CRS_EINVAL, "nrhs must be >= 1");
    CRS_CHECK(m->mask != nullptr, CRS_EINVAL, "the model has no mask preconditioner (crs_model_set_mask)");
    hipStream_t s = (hipStream_t)st;
    Exec& e = model_exec_ref(m, nrhs, s);
    // components the mask part does not act on are zero
    CRS_HIP(hipMemsetAsync(z, 0, (size_t)nrhs * m->n * sizeof(double), s));
    exec_mask(e, r, z, true, s, nullptr);
    return CRS_OK;
  });
}

}  // extern "C"
