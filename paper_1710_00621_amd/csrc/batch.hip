// Many independent problems in one solve.
//
// A batch stacks the component vectors of its models and runs one Exec over
// them: bands of all problems that share (grid, L) become the maps of one
// group, so each Legendre / ring launch covers every problem at once, and the
// PCG iteration (Sect. 2.3) advances every problem with its own scalars.
// With use_graph the PCG runs in chunks of iterations, each chunk one captured
// hipGraph launch that tests convergence on the device (exec_pcg).  The
// constrained-realization right-hand side of problem p uses the Philox
// streams of constrained_realization with seed p, so a batched solve matches
// the per-model solves.
#include <algorithm>
#include <cstring>

#include "model.h"

struct crs_batch_s {
  std::vector<crs_model> models;
  std::unique_ptr<crs::Exec> ex;
  crs::DevBuf<double> b, x, om1, om2;
  std::vector<int64_t> om1_off;  // per (problem, band) offset into om1
};

using namespace crs;

extern "C" {

int crs_batch_create(const crs_model* models, int nprob, crs_stream st, crs_batch* out) {
  return guarded([&] {
    CRS_CHECK(out != nullptr && models != nullptr, CRS_EINVAL, "models or out is NULL");
    CRS_CHECK(nprob >= 1, CRS_EINVAL, "nprob must be >= 1");
    for (int p = 0; p < nprob; ++p) CRS_CHECK(models[p] != nullptr, CRS_EINVAL, "a model is NULL");
    hipStream_t s = (hipStream_t)st;
    auto b = std::make_unique<crs_batch_s>();
    b->models.assign(models, models + nprob);
    b->ex = make_exec(b->models, 1, s, /*autotune=*/true);
    const Exec& e = *b->ex;
    b->b.alloc((size_t)e.ntot);
    b->x.alloc((size_t)e.ntot);
    b->om2.alloc((size_t)e.ntot);
    int64_t tot = 0;
    for (const crs_model m : b->models)
      for (const auto& band : m->bands) {
        b->om1_off.push_back(tot);
        tot += band.npix;
      }
    b->om1.alloc((size_t)tot);
    CRS_HIP(hipStreamSynchronize(s));
    *out = b.release();
    return CRS_OK;
  });
}

int crs_batch_destroy(crs_batch b) {
  return guarded([&] {
    delete b;
    return CRS_OK;
  });
}

int crs_batch_info(crs_batch b, int* nprob, int64_t* ntot) {
  return guarded([&] {
    CRS_CHECK(b != nullptr, CRS_EINVAL, "batch is NULL");
    if (nprob) *nprob = (int)b->models.size();
    if (ntot) *ntot = b->ex->ntot;
    return CRS_OK;
  });
}

int crs_batch_solve(crs_batch b, int mode, const double* const* const* d, const uint64_t* seeds, int precond,
                    double rtol, int maxiter, double* const* x, int* iters, double* relres, int use_graph,
                    crs_stream st) {
  return guarded([&] {
    CRS_CHECK(b != nullptr && x != nullptr, CRS_EINVAL, "batch or x is NULL");
    CRS_CHECK(mode == CRS_MODE_WF || mode == CRS_MODE_CR, CRS_EINVAL, "mode must be WF or CR");
    CRS_CHECK(mode == CRS_MODE_WF || seeds != nullptr, CRS_EINVAL, "CR mode needs seeds");
    const int np = (int)b->models.size();
    for (int p = 0; p < np; ++p) CRS_CHECK(x[p] != nullptr, CRS_EINVAL, "an x entry is NULL");
    hipStream_t s = (hipStream_t)st;
    Exec& e = *b->ex;
    std::vector<std::vector<const double*>> dt(np), wt;
    size_t ob = 0;
    if (mode == CRS_MODE_CR) wt.resize(np);
    for (int p = 0; p < np; ++p) {
      const crs_model m = b->models[p];
      dt[p].assign(m->nbands, nullptr);
      if (d && d[p])
        for (int nu = 0; nu < m->nbands; ++nu) dt[p][nu] = d[p][nu];
      if (mode == CRS_MODE_CR) {
        wt[p].resize(m->nbands);
        for (int nu = 0; nu < m->nbands; ++nu) {
          double* w = b->om1.p + b->om1_off[ob + nu];
          launch_philox_normals(seeds[p], (uint64_t)(0x100 + nu), 0, 1, m->bands[nu].npix, w, s);
          wt[p][nu] = w;
        }
        launch_philox_normals(seeds[p], 0x200, 0, 1, m->n, b->om2.p + e.hsys[p].off, s);
      }
      ob += m->nbands;
    }
    exec_rhs(e, dt, wt, mode == CRS_MODE_CR ? b->om2.p : nullptr, b->b.p, s);
    CRS_HIP(hipMemsetAsync(b->x.p, 0, (size_t)e.ntot * sizeof(double), s));
    const int rc = exec_pcg(e, precond, b->b.p, b->x.p, rtol, maxiter, iters, relres, nullptr, use_graph != 0, s);
    for (int p = 0; p < np; ++p)
      CRS_HIP(hipMemcpyAsync(x[p], b->x.p + e.hsys[p].off, e.hsys[p].n * sizeof(double), hipMemcpyDeviceToDevice,
                             s));
    CRS_HIP(hipStreamSynchronize(s));
    return rc;
  });
}

int crs_batch_set_streams(crs_batch b, int nstreams) {
  return guarded([&] {
    CRS_CHECK(b != nullptr, CRS_EINVAL, "batch is NULL");
    exec_set_streams(*b->ex, nstreams);
    return CRS_OK;
  });
}

int crs_batch_stats(crs_batch b, int* out) {
  return guarded([&] {
    CRS_CHECK(b != nullptr && out != nullptr, CRS_EINVAL, "batch or out is NULL");
    const ExecStats& st = b->ex->stats;
    out[0] = st.iterations;
    out[1] = st.graph_launches;
    out[2] = st.graph_captures;
    out[3] = st.host_syncs;
    return CRS_OK;
  });
}

}  // extern "C"
