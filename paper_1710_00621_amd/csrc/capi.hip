// Error handling, profiling hooks and the public transform entry points.
#include <cstring>
#include <mutex>

#include "internal.h"

namespace crs {

namespace {
thread_local int g_last_code = CRS_OK;
thread_local std::string g_last_msg;

std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof_pending;
std::vector<ProfRecord> g_prof_captured;
bool g_prof_in_graphs = true;  // event records inside captured graphs
struct ProfTotals {
  int64_t launches = 0;
  double ms = 0.0;
  Work3 work;
};
void add_work(Work3& a, const Work3& b) {
  for (int i = 0; i < 3; ++i) a.w[i] += b.w[i];
}
ProfTotals g_prof_totals[FAM_COUNT];

void prof_resolve_locked() {
  for (auto& r : g_prof_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
      g_prof_totals[r.family].launches += 1;
      g_prof_totals[r.family].ms += ms;
      add_work(g_prof_totals[r.family].work, r.work);
    } else {
      (void)hipGetLastError();
    }
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  g_prof_pending.clear();
}
}  // namespace

void set_error(int code, const std::string& msg) {
  g_last_code = code;
  g_last_msg = msg;
}

int fail(int code, const std::string& msg) {
  set_error(code, msg);
  return code;
}

namespace {
// Event record on a stream; on a capturing stream the record is added to the
// capture graph as an explicit event-record node after the current
// dependencies (a plain hipEventRecord is not captured by this runtime).
bool record_event(hipEvent_t ev, hipStream_t s, bool captured) {
  if (!captured) return hipEventRecord(ev, s) == hipSuccess;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  unsigned long long id = 0;
  hipGraph_t g = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t ndeps = 0;
  if (hipStreamGetCaptureInfo_v2(s, &cs, &id, &g, &deps, &ndeps) != hipSuccess || !g) return false;
  hipGraphNode_t node = nullptr;
  if (hipGraphAddEventRecordNode(&node, g, deps, ndeps, ev) != hipSuccess) return false;
  return hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies) == hipSuccess;
}
}  // namespace

ProfScope::ProfScope(int fam, const Work3& w, hipStream_t st, int tg) : family(fam), work(w), tag(tg), s(st) {
  if (!g_prof_on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return;
  captured = cs == hipStreamCaptureStatusActive;
  if (captured && !g_prof_in_graphs) return;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    e0 = e1 = nullptr;
    return;
  }
  if (!record_event(e0, s, captured)) {
    (void)hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    e0 = e1 = nullptr;
  }
}

ProfScope::~ProfScope() {
  if (!e0) return;
  if (!record_event(e1, s, captured)) {
    (void)hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (captured) {
    g_prof_captured.push_back({family, work, tag, e0, e1});
    return;
  }
  g_prof_pending.push_back({family, work, tag, e0, e1});
  if (g_prof_pending.size() > 4096) prof_resolve_locked();
}

void prof_disable_in_graphs() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_in_graphs = false;
}

bool prof_enabled() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return g_prof_on;
}

std::vector<ProfRecord> prof_take_captured() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::vector<ProfRecord> out;
  out.swap(g_prof_captured);
  return out;
}

void prof_account(const std::vector<ProfRecord>& recs, const std::function<Work3(const ProfRecord&)>& work) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return;
  for (const auto& r : recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
      g_prof_totals[r.family].launches += 1;
      g_prof_totals[r.family].ms += ms;
      add_work(g_prof_totals[r.family].work, work ? work(r) : r.work);
    } else {
      (void)hipGetLastError();  // keep a failed query from surfacing at a later launch check
    }
  }
}

void prof_release(std::vector<ProfRecord>& recs) {
  for (auto& r : recs) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  recs.clear();
}

static void check_maps(int lmax, int nmaps, int64_t as, int64_t ms_, int64_t npix) {
  CRS_CHECK(lmax >= 0, CRS_EINVAL, "lmax must be >= 0");
  CRS_CHECK(nmaps >= 1, CRS_EINVAL, "nmaps must be >= 1");
  CRS_CHECK(as >= (int64_t)(lmax + 1) * (lmax + 1), CRS_EINVAL, "alm_stride shorter than (lmax+1)^2");
  CRS_CHECK(ms_ >= npix, CRS_EINVAL, "map_stride shorter than npix");
}

LegArgs leg_args(crs_grid g, ShtPlan& p) {
  LegArgs a;
  a.g = p.g.p;
  a.ls = p.ls.p;
  a.ms = p.ms.p;
  a.zpair = g->d_zpair.p;
  a.lmax = p.lmax;
  a.npairs = p.npairs;
  a.nring = g->nring;
  a.skip = MapSkip{};
  return a;
}

RingArgs ring_args(crs_grid g, int lmax) {
  RingArgs r;
  r.nphi = g->d_nphi.p;
  r.offset = g->d_offset.p;
  r.phinum = g->d_phinum.p;
  r.phiden = g->d_phiden.p;
  r.nfac = g->d_nfac.p;
  r.fac = g->d_fac.p;
  r.facm = g->d_facm.p;
  r.fftn = g->d_fftn.p;
  r.twoff = g->d_twoff.p;
  r.tw = g->d_tw.p;
  r.bfoff = g->d_bfoff.p;
  r.bf = g->d_bf.p;
  r.tw2 = g->d_tw2.p;
  r.nring = g->nring;
  r.lmax = lmax;
  r.maxn = g->ring_maxn;
  r.xcap = 1;
  r.any_blue = 0;
  r.skip = MapSkip{};
  return r;
}

Work3 leg_work(const ShtPlan& p, int nmaps) {
  // per (ring pair, l, m): 4 flops of recurrence shared by the maps + 4 flops
  // (cos and sin FMAs on the north / south combined sums) per map
  Work3 w;
  if (nmaps <= 0) return w;
  const double per = 4.0 + 4.0 * nmaps;
  w.w[0] = (double)p.fp64_triples * per;
  w.w[1] = (double)p.nominal_triples * per;
  w.w[2] = (double)p.eff_triples * per;
  return w;
}

Work3 bytes_work(double bytes) {
  Work3 w;
  w.w[0] = w.w[1] = w.w[2] = bytes;
  return w;
}

double ring_bytes(crs_grid g, int lmax, int nmaps, int mode) {
  // algorithmic HBM traffic: phase rows (16 B per m) read and/or written,
  // map pixels read or written, weights read
  double ph = (double)g->nring * (lmax + 1) * 16.0;
  double px = (double)g->npix * 8.0;
  switch (mode) {
    case RING_SYNTH: return nmaps * (ph + px);
    case RING_ADJOINT: return nmaps * (px + ph);
    case RING_ROUNDTRIP: return nmaps * (2.0 * ph + px);
    default: return nmaps * (px + ph);
  }
}

}  // namespace crs

using namespace crs;

extern "C" {

const char* crs_strerror(int status) {
  switch (status) {
    case CRS_OK: return "ok";
    case CRS_EINVAL: return "invalid argument";
    case CRS_ENOMEM: return "out of memory";
    case CRS_EHIP: return "HIP runtime error";
    case CRS_ENOTCONV: return "PCG did not converge within maxiter";
    case CRS_EBREAKDOWN: return "PCG breakdown";
    case CRS_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

int crs_last_error(char* buf, size_t n) {
  if (buf && n) {
    std::strncpy(buf, g_last_msg.c_str(), n - 1);
    buf[n - 1] = 0;
  }
  return g_last_code;
}

const char* crs_version(void) { return "crsolve 0.1 (gfx950, float64)"; }

int crs_set_profiling(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return CRS_OK;
}

int crs_kernel_stats(const char* family, int64_t* launches, double* total_ms, double* total_work) {
  return guarded([&] {
    CRS_CHECK(family != nullptr, CRS_EINVAL, "family is NULL");
    int f = -1;
    if (!std::strcmp(family, "legendre_synth")) f = FAM_LEG_SYNTH;
    if (!std::strcmp(family, "legendre_adjoint")) f = FAM_LEG_ADJ;
    if (!std::strcmp(family, "ring_fft")) f = FAM_RING;
    CRS_CHECK(f >= 0, CRS_EINVAL, "unknown kernel family");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_resolve_locked();
    if (launches) *launches = g_prof_totals[f].launches;
    if (total_ms) *total_ms = g_prof_totals[f].ms;
    if (total_work) *total_work = g_prof_totals[f].work.w[0];
    return CRS_OK;
  });
}

int crs_kernel_work_counts(const char* family, double* work3) {
  return guarded([&] {
    CRS_CHECK(family != nullptr && work3 != nullptr, CRS_EINVAL, "family or work3 is NULL");
    int f = -1;
    if (!std::strcmp(family, "legendre_synth")) f = FAM_LEG_SYNTH;
    if (!std::strcmp(family, "legendre_adjoint")) f = FAM_LEG_ADJ;
    if (!std::strcmp(family, "ring_fft")) f = FAM_RING;
    CRS_CHECK(f >= 0, CRS_EINVAL, "unknown kernel family");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_resolve_locked();
    for (int i = 0; i < 3; ++i) work3[i] = g_prof_totals[f].work.w[i];
    return CRS_OK;
  });
}

int crs_kernel_stats_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_resolve_locked();
  for (auto& t : g_prof_totals) t = ProfTotals{};
  return CRS_OK;
}

int crs_sht_reserve(crs_grid g, int lmax, int nmaps, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(g != nullptr, CRS_EINVAL, "grid is NULL");
    CRS_CHECK(lmax >= 0 && nmaps >= 1, CRS_EINVAL, "lmax < 0 or nmaps < 1");
    hipStream_t s = (hipStream_t)st;
    ShtPlan& p = get_plan(g, lmax, s);
    if (!g->work) g->work = std::make_unique<GridWork>();
    GridWork& w = *g->work;
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 1);
    const int64_t pst = (int64_t)g->nring * (lmax + 1);
    w.uhat.alloc((size_t)nmaps * nalm);
    w.phase.alloc((size_t)nmaps * pst);
    // the largest tile count of any adjoint variant (one 64-pair tile per wave)
    w.vpart.alloc((size_t)((p.npairs + 63) / 64) * nmaps * nalm);
    CRS_HIP(hipStreamSynchronize(s));
    return CRS_OK;
  });
}

int sht_synth(crs_grid g, int lmax, int nmaps, const double* alm, int64_t alm_stride, double* map,
              int64_t map_stride, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(g != nullptr, CRS_EINVAL, "grid is NULL");
    CRS_CHECK(alm != nullptr && map != nullptr, CRS_EINVAL, "alm or map is NULL");
    check_maps(lmax, nmaps, alm_stride, map_stride, g->npix);
    hipStream_t s = (hipStream_t)st;
    ShtPlan& p = get_plan(g, lmax, s);
    if (!g->work) g->work = std::make_unique<GridWork>();
    GridWork& w = *g->work;
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 1);
    const int64_t pst = (int64_t)g->nring * (lmax + 1);
    w.uhat.alloc((size_t)nmaps * nalm);
    w.phase.alloc((size_t)nmaps * pst);
    launch_tile_sum(p.hs.p, nalm, nmaps, alm, alm_stride, 1, 0, w.uhat.p, nalm, s);
    {
      ProfScope ps(FAM_LEG_SYNTH, leg_work(p, nmaps), s);
      launch_leg_synth(leg_choice(p.npairs, lmax, nmaps), leg_args(g, p), nmaps, w.uhat.p, nalm, w.phase.p, pst, s);
    }
    {
      ProfScope ps(FAM_RING, bytes_work(ring_bytes(g, lmax, nmaps, RING_SYNTH)), s);
      launch_ring(g, lmax, RING_SYNTH, nmaps, w.phase.p, pst, nullptr, map, map_stride,
                  nullptr, 1, s);
    }
    return CRS_OK;
  });
}

int sht_adjoint(crs_grid g, int lmax, int nmaps, const double* map, int64_t map_stride, double* alm,
                int64_t alm_stride, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(g != nullptr, CRS_EINVAL, "grid is NULL");
    CRS_CHECK(alm != nullptr && map != nullptr, CRS_EINVAL, "alm or map is NULL");
    check_maps(lmax, nmaps, alm_stride, map_stride, g->npix);
    hipStream_t s = (hipStream_t)st;
    ShtPlan& p = get_plan(g, lmax, s);
    if (!g->work) g->work = std::make_unique<GridWork>();
    GridWork& w = *g->work;
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 1);
    const int64_t pst = (int64_t)g->nring * (lmax + 1);
    const LegChoice lc = leg_choice(p.npairs, lmax, nmaps);
    const int ntiles = leg_adjoint_tiles(lc, p.npairs, false);
    w.phase.alloc((size_t)nmaps * pst);
    w.vpart.alloc((size_t)ntiles * nmaps * nalm);
    {
      ProfScope ps(FAM_RING, bytes_work(ring_bytes(g, lmax, nmaps, RING_ADJOINT)), s);
      launch_ring(g, lmax, RING_ADJOINT, nmaps, w.phase.p, pst, map, nullptr, map_stride,
                  nullptr, 1, s);
    }
    {
      ProfScope ps(FAM_LEG_ADJ, leg_work(p, nmaps), s);
      launch_leg_adjoint(lc, leg_args(g, p), nmaps, w.phase.p, pst, w.vpart.p, nalm,
                         (int64_t)nmaps * nalm, false, s);
    }
    launch_tile_sum(p.hs.p, nalm, nmaps, w.vpart.p, nalm, ntiles, (int64_t)nmaps * nalm, alm, alm_stride, s);
    return CRS_OK;
  });
}

}  // extern "C"

namespace {
// Scratch of sht_adjoint_noalloc: the phase array and the adjoint's per-tile
// partial sums, in one static device array (each GPU holds its own copy until
// the process ends).  Host code never passes the array's name to a kernel or
// a copy: it uses the device address looked up once per device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the first call on
// that device, with the device current).
void* scratch_address() {
  int dev = 0;
  CRS_HIP(hipGetDevice(&dev));
  CRS_CHECK(dev >= 0 && dev < kMaxDevices, CRS_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    CRS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    CRS_CHECK(p != nullptr, CRS_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }
}  // namespace

extern "C" {

int sht_adjoint_noalloc(crs_grid g, int lmax, int nmaps, const double* map, int64_t map_stride, double* alm,
                        int64_t alm_stride, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(g != nullptr, CRS_EINVAL, "grid is NULL");
    CRS_CHECK(alm != nullptr && map != nullptr, CRS_EINVAL, "alm or map is NULL");
    check_maps(lmax, nmaps, alm_stride, map_stride, g->npix);
    hipStream_t s = (hipStream_t)st;
    auto it = g->plans.find(lmax);
    CRS_CHECK(it != g->plans.end(), CRS_EINVAL,
              "no Legendre tables for this (grid, lmax) yet: create them with one sht_synth or "
              "sht_adjoint call (or a model using the pair) before calling sht_adjoint_noalloc");
    ShtPlan& p = *it->second;
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 1);
    const int64_t pst = (int64_t)g->nring * (lmax + 1);
    const LegChoice lc = leg_choice(p.npairs, lmax, nmaps);
    const int ntiles = leg_adjoint_tiles(lc, p.npairs, false);
    const size_t phase_bytes = align256((size_t)nmaps * pst * sizeof(double2));
    const size_t part_bytes = align256((size_t)ntiles * nmaps * nalm * sizeof(double));
    CRS_CHECK(phase_bytes + part_bytes <= kNoAllocScratchBytes, CRS_EINVAL,
              "sht_adjoint_noalloc needs " + std::to_string(phase_bytes + part_bytes) +
                  " bytes of scratch for this (grid, lmax, nmaps); its limit is " +
                  std::to_string(kNoAllocScratchBytes) + " bytes (use sht_adjoint)");
    unsigned char* base = static_cast<unsigned char*>(scratch_address());
    double2* phase = reinterpret_cast<double2*>(base);
    double* vpart = reinterpret_cast<double*>(base + phase_bytes);
    // every entry of both scratch regions is written before it is read: the
    // ring stage writes all m <= lmax of every ring and map, and every tile of
    // the Legendre adjoint writes its whole partial vector
    {
      ProfScope ps(FAM_RING, bytes_work(ring_bytes(g, lmax, nmaps, RING_ADJOINT)), s);
      launch_ring(g, lmax, RING_ADJOINT, nmaps, phase, pst, map, nullptr, map_stride, nullptr, 1, s);
    }
    {
      ProfScope ps(FAM_LEG_ADJ, leg_work(p, nmaps), s);
      launch_leg_adjoint(lc, leg_args(g, p), nmaps, phase, pst, vpart, nalm, (int64_t)nmaps * nalm, false, s);
    }
    launch_tile_sum(p.hs.p, nalm, nmaps, vpart, nalm, ntiles, (int64_t)nmaps * nalm, alm, alm_stride, s);
    return CRS_OK;
  });
}

int crs_autotune_legendre(crs_grid g, int lmax, int nmaps, crs_stream st) {
  return guarded([&] {
    CRS_CHECK(g != nullptr, CRS_EINVAL, "grid is NULL");
    CRS_CHECK(lmax >= 0 && nmaps >= 1, CRS_EINVAL, "lmax < 0 or nmaps < 1");
    hipStream_t s = (hipStream_t)st;
    ShtPlan& p = get_plan(g, lmax, s);
    const int64_t nalm = (int64_t)(lmax + 1) * (lmax + 1);
    const int64_t pst = (int64_t)g->nring * (lmax + 1);
    DevBuf<double> uhat;
    DevBuf<double2> phase;
    uhat.alloc((size_t)nmaps * nalm);
    phase.alloc((size_t)nmaps * pst);
    leg_autotune(leg_args(g, p), nmaps, uhat.p, phase.p, s);
    return CRS_OK;
  });
}

int crs_legendre_choice(crs_grid g, int lmax, int nmaps, int* out) {
  return guarded([&] {
    CRS_CHECK(g != nullptr && out != nullptr, CRS_EINVAL, "grid or out is NULL");
    CRS_CHECK(lmax >= 0 && nmaps >= 1, CRS_EINVAL, "lmax < 0 or nmaps < 1");
    const LegChoice c = leg_choice((g->nring + 1) / 2, lmax, nmaps);
    out[0] = c.syn_mfma;
    out[1] = c.syn_r;
    out[2] = c.adj_mfma;
    out[3] = c.adj_r;
    out[4] = c.adj_t;
    return CRS_OK;
  });
}

}  // extern "C"
