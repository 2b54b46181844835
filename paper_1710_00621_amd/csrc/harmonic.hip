// Generic operations on batches of harmonic vectors and pixel maps, and
// transforms on caller-sized scratch, shared by the mask-restricted
// preconditioner (Sect. 4.4) and the spatially varying mixing operators
// (Sect. 2.2, eq:Q).
//
// Harmonic vectors are packed m-major (unpack_lm / moff_h); "hat" vectors
// (the Legendre kernels' input) are c_m f_lm times the plain coefficients,
// and the adjoint's per-tile partial sums become plain coefficients after the
// same scaling (hs tables of a plan).
#include <algorithm>

#include "model.h"

namespace crs {

namespace {

__host__ __device__ inline int64_t nalm_of(int L) { return (int64_t)(L + 1) * (L + 1); }

// Harmonic vectors: packed m-major (unpack_lm / moff_h of model.h).  Maps of
// a batch of nm vectors; map j skipped when skip.off(j).
__device__ __forceinline__ int64_t repack_idx(int L, int m, int part, int ll) {
  return moff_h(L, m) + (int64_t)part * (L - m + 1) + ll;
}

// out_hat[j][i] = hs[i] f_j[l] (in1_j + in2_j)[l, m, part]  (inputs at their own
// band-limits, zero above them; in2 optional; f optional)
__global__ void k_hat_from(double* __restrict__ out, int LO, const double* __restrict__ hs,
                           const double* __restrict__ in1, int L1, const int64_t* __restrict__ off1, int64_t st1,
                           const double* __restrict__ in2, int L2, int64_t st2,
                           const double* __restrict__ F, int fst, const int* __restrict__ mc, MapSkip skip) {
  const int j = blockIdx.y;
  if (skip.off(j)) return;
  const int64_t n = nalm_of(LO);
  const double* a = in1 + (off1 ? off1[j] : (int64_t)j * st1);
  const double* b = in2 ? in2 + (int64_t)j * st2 : nullptr;
  const double* f = F ? F + (int64_t)mc[j] * fst : nullptr;
  double* o = out + (int64_t)j * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int m, part, ll;
    unpack_lm(LO, i, m, part, ll);
    const int l = m + ll;
    double v = (l <= L1) ? a[repack_idx(L1, m, part, l - m)] : 0.0;
    if (b && l <= L2) v += b[repack_idx(L2, m, part, l - m)];
    if (f) v *= f[l];
    o[i] = hs[i] * v;
  }
}

// out_j[i] = (acc ? out_j[i] : 0) + alpha f_j[l] hs[i] sum_t parts[t][j][i] - g_j[l] sub_j[l, m, part]
// (adjoint partial sums at band-limit LO to a plain vector; f, sub optional)
__global__ void k_from_parts(double* __restrict__ out, const int64_t* __restrict__ offo, int LO, int acc,
                             double alpha, const double* __restrict__ hs, const double* __restrict__ parts, int ntiles,
                             int64_t tstride, const double* __restrict__ F, int fst,
                             const double* __restrict__ sub, int Ls, int64_t sst, const double* __restrict__ Gs,
                             int gst, const int* __restrict__ mc, MapSkip skip) {
  const int j = blockIdx.y;
  if (skip.off(j)) return;
  const int64_t n = nalm_of(LO);
  double* o = out + (offo ? offo[j] : (int64_t)j * n);
  const double* pp = parts + (int64_t)j * n;
  const double* f = F ? F + (int64_t)mc[j] * fst : nullptr;
  const double* sb = sub ? sub + (int64_t)j * sst : nullptr;
  const double* g = Gs ? Gs + (int64_t)mc[j] * gst : nullptr;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double sv = 0.0;
    for (int t = 0; t < ntiles; ++t) sv += pp[(int64_t)t * tstride + i];
    int m, part, ll;
    unpack_lm(LO, i, m, part, ll);
    const int l = m + ll;
    double v = alpha * hs[i] * sv;
    if (f) v *= f[l];
    if (sb) v -= (l <= Ls ? g[l] * sb[repack_idx(Ls, m, part, ll)] : 0.0);
    o[i] = acc ? o[i] + v : v;
  }
}

// pointwise map operations on nm maps of npix pixels (ind: 0/1 mask of the level)
enum { MOP_MASK = 0, MOP_SCALE = 1, MOP_AXPY_MASK = 2, MOP_POST = 3, MOP_ZERO = 4 };
__global__ void k_map_op(int op, double* __restrict__ x, const double* __restrict__ b, const double* __restrict__ y,
                         const double* __restrict__ ind, const double* __restrict__ sm, double alpha, int64_t npix,
                         MapSkip skip) {
  const int j = blockIdx.y;
  if (skip.off(j)) return;
  double* xj = x + (int64_t)j * npix;
  const double* bj = b ? b + (int64_t)j * npix : nullptr;
  const double* yj = y ? y + (int64_t)j * npix : nullptr;
  const double s = sm ? sm[j] : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += (int64_t)gridDim.x * blockDim.x) {
    switch (op) {
      case MOP_MASK: xj[i] *= ind[i]; break;
      case MOP_SCALE: xj[i] = s * bj[i]; break;
      case MOP_AXPY_MASK: xj[i] = fma(alpha * ind[i], yj[i], xj[i]); break;
      case MOP_POST: xj[i] = fma(s, bj[i] - ind[i] * yj[i], xj[i]); break;
      default: xj[i] = 0.0; break;
    }
  }
}


dim3 alm_grid(int L, int nm) {
  const int64_t n = nalm_of(L);
  return dim3((unsigned)std::min<int64_t>((n + 255) / 256, 2048), nm);
}
dim3 map_grid(int64_t npix, int nm) { return dim3((unsigned)std::min<int64_t>((npix + 255) / 256, 2048), nm); }

}  // namespace

void launch_hat_from(double* out, int LO, const double* hs, const double* in1, int L1, const int64_t* off1,
                     int64_t st1, const double* in2, int L2, int64_t st2, const double* F, int fst, const int* mc,
                     int nm, MapSkip skip, hipStream_t s) {
  hipLaunchKernelGGL(k_hat_from, alm_grid(LO, nm), dim3(256), 0, s, out, LO, hs, in1, L1, off1, st1, in2, L2, st2, F,
                     fst, mc, skip);
  CRS_HIP(hipGetLastError());
}

void launch_from_parts(double* out, const int64_t* offo, int LO, int acc, double alpha, const double* hs,
                       const double* parts, int ntiles, int64_t tstride, const double* F, int fst, const double* sub,
                       int Ls, int64_t sst, const double* Gs, int gst, const int* mc, int nm, MapSkip skip,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_from_parts, alm_grid(LO, nm), dim3(256), 0, s, out, offo, LO, acc, alpha, hs, parts, ntiles,
                     tstride, F, fst, sub, Ls, sst, Gs, gst, mc, skip);
  CRS_HIP(hipGetLastError());
}

void launch_map_op(int op, double* x, const double* b, const double* y, const double* ind, const double* sm,
                   double alpha, int64_t npix, int nm, MapSkip skip, hipStream_t s) {
  hipLaunchKernelGGL(k_map_op, map_grid(npix, nm), dim3(256), 0, s, op, x, b, y, ind, sm, alpha, npix, skip);
  CRS_HIP(hipGetLastError());
}

// ------------------------------------------------------ transform scratch
void ShtScratch::reserve(crs_grid g, int L, int nm, hipStream_t s) {
  ShtPlan& p = get_plan(g, L, s);
  LegChoice c;
  auto it = choice.find(std::make_pair(g, L));
  if (it != choice.end() && it->second.first >= nm) {
    c = it->second.second;
  } else {
    c = leg_choice(p.npairs, L, nm);
    choice[std::make_pair(g, L)] = std::make_pair(nm, c);
  }
  hat.alloc((size_t)nalm_of(L) * nm);
  phase.alloc((size_t)g->nring * (L + 1) * nm);
  parts.alloc((size_t)leg_adjoint_tiles(c, p.npairs, false) * nalm_of(L) * nm);
}

void scratch_synth(ShtScratch& w, crs_grid g, int L, int nm, const double* hat, double* map, MapSkip skip,
                   hipStream_t s) {
  ShtPlan& p = get_plan(g, L, s);
  LegArgs la = leg_args(g, p);
  la.skip = skip;
  const LegChoice c = w.choice.at(std::make_pair(g, L)).second;
  const int64_t pst = (int64_t)g->nring * (L + 1);
  {
    ProfScope ps(FAM_LEG_SYNTH, leg_work(p, nm), s);
    launch_leg_synth(c, la, nm, hat, nalm_of(L), w.phase.p, pst, s);
  }
  {
    ProfScope ps(FAM_RING, bytes_work(ring_bytes(g, L, nm, RING_SYNTH)), s);
    launch_ring(g, L, RING_SYNTH, nm, w.phase.p, pst, nullptr, map, g->npix, nullptr, 1, s, skip);
  }
}

int scratch_adjoint(ShtScratch& w, crs_grid g, int L, int nm, const double* map, MapSkip skip, hipStream_t s) {
  ShtPlan& p = get_plan(g, L, s);
  LegArgs la = leg_args(g, p);
  la.skip = skip;
  const LegChoice c = w.choice.at(std::make_pair(g, L)).second;
  const int nt = leg_adjoint_tiles(c, p.npairs, false);
  const int64_t pst = (int64_t)g->nring * (L + 1);
  {
    ProfScope ps(FAM_RING, bytes_work(ring_bytes(g, L, nm, RING_ADJOINT)), s);
    launch_ring(g, L, RING_ADJOINT, nm, w.phase.p, pst, map, nullptr, g->npix, nullptr, 1, s, skip);
  }
  {
    ProfScope ps(FAM_LEG_ADJ, leg_work(p, nm), s);
    launch_leg_adjoint(c, la, nm, w.phase.p, pst, w.parts.p, nalm_of(L), (int64_t)nm * nalm_of(L), false, s);
  }
  return nt;
}

}  // namespace crs
