// Internal declarations of the crsolve HIP library (gfx950, float64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/crsolve.h"

namespace crs {

// ---------------------------------------------------------------- errors
struct Error {
  int code;
  std::string msg;
};
void set_error(int code, const std::string& msg);
int fail(int code, const std::string& msg);  // sets and returns code

#define CRS_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::crs::Error{CRS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define CRS_CHECK(cond, code, msg)                          \
  do {                                                      \
    if (!(cond)) throw ::crs::Error{(code), (msg)};         \
  } while (0)

// Runs f() and turns exceptions into status codes.
template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(CRS_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(CRS_EINVAL, e.what());
  }
}

// Device buffer owned by a handle.
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (count <= n && p) return;
    release();
    if (count == 0) return;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{CRS_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
    }
    n = count;
  }
  void upload(const T* host, size_t count, hipStream_t s) {
    alloc(count);
    if (count) CRS_HIP(hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void upload(const std::vector<T>& v, hipStream_t s) { upload(v.data(), v.size(), s); }
};

constexpr int kMaxRing = 8192;   // pixels per ring (the FFT stays LDS resident)
constexpr int kMaxFactors = 16;  // radices per ring length
constexpr int kBlueMax = 8192;   // longest Bluestein convolution (power of two)
constexpr size_t kMaxLds = 160 * 1024;  // LDS bytes one workgroup may use (gfx950)

// ---------------------------------------------------------------- grids
// Per-(grid, lmax) Legendre plan: start table and recurrence tables.
struct ShtPlan {
  int lmax = 0;
  int npairs = 0;
  int64_t eff_triples = 0;     // (ring pair, l, m) triples the kernels evaluate (|lambda| >= 2^-100)
  int64_t fp64_triples = 0;    // triples whose |lambda| reaches the float64 normal range
  int64_t nominal_triples = 0; // npairs * (L+1)(L+2)/2
  DevBuf<double> g;            // triangle: g_lm, mu recurrence coefficient
  DevBuf<double> f;            // triangle: f_lm, lambda = f * mu
  DevBuf<double> hs;           // packed alm layout: c_m f_lm (plain <-> hat vectors)
  DevBuf<int> ls;              // [L+1][npairs]: first l evaluated (L+1 = never)
  DevBuf<double2> ms;          // [L+1][npairs]: (mu_{ls-1}, mu_ls)
};

// Rings are launched in classes by FFT length tier (ring_tier_maxfft(t),
// ring_tier_threads(t) threads per block) and, from tier 2 up, by Bluestein
// or direct transform and whether the FFT has odd radices.
struct RingClass {
  std::vector<int> rings;
  bool blue = false;  // some ring of the class uses Bluestein's convolution
  bool odd = false;   // some FFT length of the class has radices 3, 5 or 7
  int tier = 0;
  int xcap = 1;       // complex LDS words for ring data / convolution
  int maxn = 1;       // longest ring in the class
  int gcap = 0;       // fold scratch words (rings shorter than the block)
};
// tiers: FFT length <= 512 / 1024 / 4096 / 8192 with 128 / 256 / 512 / 1024
// threads (the longest FFT is a Bluestein convolution of kBlueMax words)
constexpr int kMaxRingClasses = 16;  // at most 4 per tier
inline int ring_tier_threads(int tier) { return 128 << tier; }
inline int ring_tier_maxfft(int tier) {
  return tier == 0 ? 512 : tier == 1 ? 1024 : tier == 2 ? 4096 : kBlueMax;
}

// Workspace of the public transforms (sht_synth / sht_adjoint).
struct GridWork {
  DevBuf<double> uhat;
  DevBuf<double2> phase;
  DevBuf<double> vpart;
};

}  // namespace crs

struct crs_grid_s {
  int kind = 0;  // 0 HEALPix, 1 Gauss-Legendre
  int nside = 0, nring = 0, nphi_gl = 0;
  int64_t npix = 0;
  std::vector<double> z, sint, ringw;
  std::vector<int> nphi, phi0_num, phi0_den;  // phi0 = pi * num / den
  std::vector<int64_t> offset;
  // device ring tables
  crs::DevBuf<int> d_nphi, d_phinum, d_phiden, d_nfac, d_fac, d_fftn;
  crs::DevBuf<unsigned> d_facm;
  crs::DevBuf<int64_t> d_offset, d_twoff, d_bfoff;
  crs::DevBuf<double2> d_bf;      // Bluestein filter spectra per distinct length
  crs::DevBuf<double2> d_tw2;     // exp(-2 pi i t / kBlueMax), t < kBlueMax
  crs::DevBuf<double> d_zpair;    // z of the north ring of each pair
  crs::DevBuf<double> d_spair;    // sin(theta) of the north ring of each pair
  crs::DevBuf<double2> d_tw;      // twiddles exp(-2 pi i t / N) per distinct N
  int ring_maxn = 1;
  std::vector<crs::RingClass> ring_classes;  // by (tier, Bluestein, odd radix)
  std::vector<crs::DevBuf<int>> d_ring_class;
  std::vector<int> ring_small_order;         // classes by ring count, ascending
  std::vector<crs::RingClass> ring_prefix;   // [k]: the first k + 1 of them merged
  std::vector<crs::DevBuf<int>> d_ring_prefix;
  std::map<int, std::unique_ptr<crs::ShtPlan>> plans;
  std::unique_ptr<crs::GridWork> work;
  int device = 0;
};

namespace crs {

ShtPlan& get_plan(crs_grid g, int lmax, hipStream_t s);

// ------------------------------------------------------------ kernels API
// Legendre stage.  Harmonic inputs are "hat" vectors: u^ = c_m f_lm u.
// Optional skip of finished systems: map j is skipped when
// act[kActStride * mapsys[j]] == 0 (both NULL: nothing is skipped).
constexpr int kActStride = 8;
struct MapSkip {
  const int* mapsys = nullptr;
  const double* act = nullptr;
  __device__ __forceinline__ bool off(int map) const {
    return act != nullptr && act[kActStride * mapsys[map]] == 0.0;
  }
};

struct LegArgs {
  const double* g;        // triangle
  const int* ls;          // [L+1][npairs]
  const double2* ms;      // [L+1][npairs]
  const double* zpair;    // [npairs]
  int lmax, npairs, nring;
  MapSkip skip;
  // optional compaction: the launch's map slots s < *mcount are the maps
  // mlist[s] (ascending), the slots past *mcount are empty; without it slot
  // s is map s.  Both device pointers, set together.
  const int* mlist = nullptr;
  const int* mcount = nullptr;
};
// Which Legendre kernels run for a (ring pairs, L, maps) shape: synthesis on
// the matrix cores or vector FP64 with syn_r ring pairs per lane; adjoint on
// the matrix cores with adj_t 64-pair tiles per wave or vector FP64 with
// adj_r pairs per lane.  leg_choice gives the autotuned choice for the shape
// if one was recorded (leg_autotune), else the measured default rules; the
// environment variables CRS_LEG_MFMA_MIN, CRS_LEG_RS, CRS_LEG_RA and
// CRS_LEG_TA override either (tuning and tests).  A caller takes the choice
// once and passes the same one to leg_adjoint_tiles and the launches.
struct LegChoice {
  int syn_mfma = 0, syn_r = 1;
  int adj_mfma = 0, adj_r = 1, adj_t = 1;
};
LegChoice leg_choice(int npairs, int lmax, int nmaps);
// Times every valid variant of both transforms on the given buffers (their
// contents are overwritten; vpart is allocated internally) and records the
// fastest per transform for the shape.  Returns the recorded choice.
LegChoice leg_autotune(const LegArgs& a, int nmaps, double* uhat, double2* phase, hipStream_t s);
// phase: [nmaps][nring][L+1] double2 (cos, sin parts)
void launch_leg_synth(const LegChoice& c, const LegArgs& a, int nmaps, const double* uhat, int64_t ustride,
                      double2* phase, int64_t pstride, hipStream_t s);
// Adjoint: writes ntiles partial vectors vpart[tile][map][nalm], ntiles as
// returned here for the same choice and square flag as the launch.
int leg_adjoint_tiles(const LegChoice& c, int npairs, bool square);
void launch_leg_adjoint(const LegChoice& c, const LegArgs& a, int nmaps, const double2* phase, int64_t pstride,
                        double* vpart, int64_t vstride, int64_t tstride, bool square,
                        hipStream_t s);

// Ring FFT stage.
enum RingMode { RING_SYNTH = 0, RING_ADJOINT = 1, RING_ROUNDTRIP = 2, RING_DIAG = 3 };
struct RingArgs {
  const int* nphi;
  const int64_t* offset;
  const int* phinum;
  const int* phiden;
  const int* nfac;     // radices of the FFT length of each ring
  const int* fac;
  const unsigned* facm;  // per stage: FastDiv multiplier of the stride Ns before it
  const int* fftn;     // FFT length: Nphi / 2 (even), Nphi (odd) or the Bluestein length
  const int64_t* twoff;
  const double2* tw;   // per distinct Nphi: exp(-i pi t / Nphi), t < 2 Nphi
  const int64_t* bfoff;
  const double2* bf;    // per Bluestein length: filter spectrum [fftn], then the chirp [n0]
  const double2* tw2;
  int nring, lmax;
  int maxn, xcap;      // per launch class: longest ring, LDS data words
  int any_blue;        // per launch class: Bluestein tables present in LDS
  MapSkip skip;
  const int* rings;    // ring list of the launch (set by launch_ring per class)
};
// maps j = 0..nmaps-1 use weight weights[j / maps_per_weight] (RING_ROUNDTRIP).
void launch_ring(crs_grid g, int lmax, RingMode mode, int nmaps, double2* phase, int64_t pstride,
                 const double* map_in, double* map_out, int64_t mstride,
                 const double* const* weights, int maps_per_weight, hipStream_t s,
                 MapSkip skip = MapSkip{});

// Scaling between plain and hat vectors: out[map] = hs * sum_t in[t][map]
// elementwise over the packed alm index (hs = c_m f_lm, ShtPlan::hs).
void launch_tile_sum(const double* hs, int64_t nalm, int nmaps, const double* in, int64_t istride,
                     int ntiles, int64_t tstride, double* out, int64_t ostride, hipStream_t s);
// Same with the scale computed per (l, m) from the f triangle; square: f^2
// without c_m (the M_diag setup).
void launch_hat_scale(const double* f, int lmax, int nmaps, const double* in, int64_t istride,
                      int ntiles, int64_t tstride, double* out, int64_t ostride, bool square,
                      hipStream_t s);

// Profiling hooks (no-ops unless profiling is on).  A scope brackets its
// launches with HIP events on the stream.  On a stream that is being
// captured into a graph the event records become graph nodes; the pairs are
// then handed to the graph's owner (prof_take_captured), which accounts them
// after every replay (prof_account) and frees them (prof_release).
// Work of a launch, three ways: the Legendre flops counted over the (ring
// pair, l, m) triples whose |lambda| reaches the float64 normal range (w[0],
// the headline count), over all triples (w[1], nominal) and over the triples
// the kernels evaluate (w[2], |lambda| >= 2^-100); ring launches carry their
// algorithmic bytes in all three.
struct Work3 {
  double w[3] = {0.0, 0.0, 0.0};
};
struct ProfRecord {
  int family;
  Work3 work;
  int tag;  // owner's label (a group index) for replay-time work, -1: fixed
  hipEvent_t e0, e1;
};
struct ProfScope {
  int family;
  Work3 work;
  int tag;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool captured = false;
  ProfScope(int fam, const Work3& w, hipStream_t st, int tag = -1);
  ~ProfScope();
};
enum { FAM_LEG_SYNTH = 0, FAM_LEG_ADJ = 1, FAM_RING = 2, FAM_COUNT = 3 };
bool prof_enabled();
void prof_disable_in_graphs();  // if a graph cannot hold event records
std::vector<ProfRecord> prof_take_captured();
// Accounts one replay; work (optional) gives each record's work for this
// replay (records of finished systems' maps do less), else the recorded work.
void prof_account(const std::vector<ProfRecord>& recs,
                  const std::function<Work3(const ProfRecord&)>& work = nullptr);
void prof_release(std::vector<ProfRecord>& recs);
Work3 leg_work(const ShtPlan& p, int nmaps);
Work3 bytes_work(double bytes);

}  // namespace crs
