// Spatially varying mixing maps (Sect. 2.2, eq:P and eq:Q):
//
//   P_{nu,k} = Y_nu B_nu Q~_{nu,k},   Q~_{nu,k} = Y^T W Q_{nu,k} Y
//
// on a grid specific to the pair (Gauss-Legendre or HEALPix), at the
// component band-limit L_k (the product's modes above L_k are truncated, the
// approximation the paper allows).  W and Q are diagonal, so Q~ is symmetric
// and the transpose applies the same operator.  A pair whose mixing is
// spatially constant keeps q_{nu,k} I; a varying pair costs four SHTs per
// application of A (two before the forward mix, two after the transpose).
// The preconditioners approximate the map by the scalar of eq:optimal-q
// (App. A.2).
#include <algorithm>
#include <cmath>

#include "model.h"

namespace crs {

// Per-Exec state: maps = the systems (right-hand sides of the one problem).
struct VarMixRun {
  int nm = 0;
  ShtScratch sc;
  DevBuf<double> map;        // nm x (largest grid npix)
  DevBuf<double> ybuf;       // per pair: nm x nalm(L_k), y = Q~ x_k
  std::vector<int64_t> hyoff;
  DevBuf<int64_t> yoff;      // per pair: start of its block in ybuf
  DevBuf<int> vidx;          // [nbands][ncomp]: pair index or -1
  std::vector<DevBuf<int64_t>> xoff;  // per pair, per map: offset of x_k of the map's system
};

void VarMixRunDel::operator()(VarMixRun* p) const { delete p; }

namespace {

// hat[j][i] = hs_i^2 b_{nu,l} sum_t parts_nu[t][map(j)][i_nu] at band-limit Lk:
// the synthesis input of Q~ applied to B_nu v_nu (v_nu the plain band
// adjoint), repacked from the band's layout at L_nu (zero above L_nu).
__global__ void k_band_hat(double* __restrict__ hat, int Lk, const SysDev* __restrict__ sys,
                           const ProbDev* __restrict__ probs, int nu, const double* __restrict__ beamtab, int nb,
                           MapSkip skip) {
  const int j = blockIdx.y;  // system
  if (skip.off(j)) return;
  const SysDev S = sys[j];
  const ProbDev P = probs[S.prob];
  const int* bi = P.binfo + kBinfo * nu;
  const int Lb = bi[0];
  const int map = bi[2] + S.rhs * bi[4], nt = bi[3];
  const int64_t nalm_b = (int64_t)(Lb + 1) * (Lb + 1);
  const int64_t tstride = (int64_t)bi[1] * nalm_b;
  const double* v = P.vptr[nu] + (int64_t)map * nalm_b;
  const int64_t n = (int64_t)(Lk + 1) * (Lk + 1);
  double* o = hat + (int64_t)j * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int m, part, ll;
    unpack_lm(Lk, i, m, part, ll);
    const int l = m + ll;
    double val = 0.0;
    if (l <= Lb) {
      const int64_t ib = moff_h(Lb, m) + (int64_t)part * (Lb - m + 1) + ll;
      double sv = 0.0;
      for (int t = 0; t < nt; ++t) sv += v[(int64_t)t * tstride + ib];
      const double cm = (m == 0) ? 1.0 : 1.4142135623730951;
      const double hs = cm * P.ftab[tri_h(P.Lf, m) + ll];
      val = hs * hs * beamtab[(int64_t)l * nb + nu] * sv;
    }
    o[i] = val;
  }
}

}  // namespace

bool exec_has_varmix(const Exec& e) { return e.varmix != nullptr; }

void exec_varmix_prepare(Exec& e, hipStream_t s) {
  const crs_model m = e.probs[0];
  if (m->varmix.empty()) return;
  std::unique_ptr<VarMixRun, VarMixRunDel> r(new VarMixRun);
  r->nm = e.nsys;
  int64_t maxpix = 0, tot = 0;
  std::vector<int> vidx((size_t)m->nbands * m->ncomp, -1);
  for (size_t v = 0; v < m->varmix.size(); ++v) {
    const VarMix& vm = m->varmix[v];
    const int Lk = m->lk[vm.k];
    vidx[(size_t)vm.nu * m->ncomp + vm.k] = (int)v;
    r->hyoff.push_back(tot);
    tot += (int64_t)r->nm * (Lk + 1) * (Lk + 1);
    maxpix = std::max(maxpix, vm.grid->npix);
    r->sc.reserve(vm.grid, Lk, r->nm, s);
    std::vector<int64_t> xo(r->nm);
    for (int j = 0; j < r->nm; ++j) xo[j] = e.hsys[j].off + m->coff[vm.k];
    r->xoff.emplace_back();
    r->xoff.back().upload(xo, s);
  }
  r->map.alloc((size_t)maxpix * r->nm);
  r->ybuf.alloc((size_t)std::max<int64_t>(tot, 1));
  r->yoff.upload(r->hyoff, s);
  r->vidx.upload(vidx, s);
  CRS_HIP(hipStreamSynchronize(s));
  e.vm_vidx = r->vidx.p;
  e.vm_ybuf = r->ybuf.p;
  e.vm_yoff = r->yoff.p;
  e.varmix = std::move(r);
}

void exec_varmix_fwd(Exec& e, const double* x, hipStream_t s, const double* act) {
  if (!e.varmix) return;
  VarMixRun& r = *e.varmix;
  const crs_model m = e.probs[0];
  MapSkip skip;
  if (act) {
    skip.mapsys = e.sys_ident.p;
    skip.act = act;
  }
  for (size_t v = 0; v < m->varmix.size(); ++v) {
    const VarMix& vm = m->varmix[v];
    const int Lk = m->lk[vm.k];
    const double* hs = get_plan(vm.grid, Lk, s).hs.p;
    // y = Y^T W Q Y x_k
    launch_hat_from(r.sc.hat.p, Lk, hs, x, Lk, r.xoff[v].p, 0, nullptr, 0, 0, nullptr, 0, nullptr, r.nm, skip, s);
    scratch_synth(r.sc, vm.grid, Lk, r.nm, r.sc.hat.p, r.map.p, skip, s);
    launch_map_op(MOP_MASK, r.map.p, nullptr, nullptr, vm.qw.p, nullptr, 0.0, vm.grid->npix, r.nm, skip, s);
    const int nt = scratch_adjoint(r.sc, vm.grid, Lk, r.nm, r.map.p, skip, s);
    const int64_t nalm = (int64_t)(Lk + 1) * (Lk + 1);
    launch_from_parts(r.ybuf.p + r.hyoff[v], nullptr, Lk, 0, 1.0, hs, r.sc.parts.p, nt, (int64_t)r.nm * nalm,
                      nullptr, 0, nullptr, 0, 0, nullptr, 0, nullptr, r.nm, skip, s);
  }
}

void exec_varmix_back(Exec& e, double* out, hipStream_t s, const double* act) {
  if (!e.varmix) return;
  VarMixRun& r = *e.varmix;
  const crs_model m = e.probs[0];
  MapSkip skip;
  if (act) {
    skip.mapsys = e.sys_ident.p;
    skip.act = act;
  }
  for (size_t v = 0; v < m->varmix.size(); ++v) {
    const VarMix& vm = m->varmix[v];
    const int Lk = m->lk[vm.k];
    const double* hs = get_plan(vm.grid, Lk, s).hs.p;
    const int64_t nalm = (int64_t)(Lk + 1) * (Lk + 1);
    // out_k += Y^T W Q Y (B_nu v_nu)
    dim3 gr((unsigned)std::min<int64_t>((nalm + 255) / 256, 2048), r.nm);
    hipLaunchKernelGGL(k_band_hat, gr, dim3(256), 0, s, r.sc.hat.p, Lk, e.dsys.p, e.dprobs.p, vm.nu, m->beamtab.p,
                       m->nbands, skip);
    CRS_HIP(hipGetLastError());
    scratch_synth(r.sc, vm.grid, Lk, r.nm, r.sc.hat.p, r.map.p, skip, s);
    launch_map_op(MOP_MASK, r.map.p, nullptr, nullptr, vm.qw.p, nullptr, 0.0, vm.grid->npix, r.nm, skip, s);
    const int nt = scratch_adjoint(r.sc, vm.grid, Lk, r.nm, r.map.p, skip, s);
    launch_from_parts(out, r.xoff[v].p, Lk, 1, 1.0, hs, r.sc.parts.p, nt, (int64_t)r.nm * nalm, nullptr, 0,
                      nullptr, 0, 0, nullptr, 0, nullptr, r.nm, skip, s);
  }
}

}  // namespace crs

using namespace crs;

extern "C" {

int crs_model_set_mixing_map(crs_model m, int band, int comp, crs_grid grid, const double* qmap, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(m != nullptr, CRS_EINVAL, "model is NULL");
    CRS_CHECK(band >= 0 && band < m->nbands && comp >= 0 && comp < m->ncomp, CRS_EINVAL,
              "band or component index out of range");
    hipStream_t s = (hipStream_t)st;
    auto it = std::find_if(m->varmix.begin(), m->varmix.end(),
                           [&](const VarMix& v) { return v.nu == band && v.k == comp; });
    if (qmap == nullptr) {
      if (it != m->varmix.end()) m->varmix.erase(it);
      model_rebuild_tables(m, s);
      return CRS_OK;
    }
    CRS_CHECK(grid != nullptr, CRS_EINVAL, "grid is NULL");
    double s1 = 0.0, s2 = 0.0;
    std::vector<double> qw(grid->npix);
    for (int r = 0; r < grid->nring; ++r)
      for (int j = 0; j < grid->nphi[r]; ++j) {
        const int64_t i = grid->offset[r] + j;
        CRS_CHECK(std::isfinite(qmap[i]), CRS_EINVAL, "the mixing map must be finite");
        s1 += qmap[i];
        s2 += qmap[i] * qmap[i];
        qw[i] = qmap[i] * grid->ringw[r];
      }
    CRS_CHECK(s1 > 0.0, CRS_EINVAL, "the mixing map must have a positive sum (eq:optimal-q)");
    // the Legendre tables of the pair's transforms (setup, not the hot path)
    get_plan(grid, m->lk[comp], s);
    VarMix v;
    v.nu = band;
    v.k = comp;
    v.grid = grid;
    v.qw.upload(qw, s);
    v.qeff = s2 / s1;
    CRS_HIP(hipStreamSynchronize(s));
    if (it != m->varmix.end())
      *it = std::move(v);
    else
      m->varmix.push_back(std::move(v));
    model_rebuild_tables(m, s);
    return CRS_OK;
  });
}

}  // extern "C"
