// Internal structures of the system solver shared by model.hip (model
// construction and its tables), exec.hip (operators, right-hand side, PCG on
// a set of independent systems) and batch.hip (many models in one solve).
#pragma once

#include "internal.h"

#include <tuple>

namespace crs {

LegArgs leg_args(crs_grid g, ShtPlan& p);
RingArgs ring_args(crs_grid g, int lmax);
double ring_bytes(crs_grid g, int lmax, int nmaps, int mode);

__host__ __device__ inline int64_t moff_h(int L, int m) {
  return (m == 0) ? 0 : (int64_t)(L + 1) + 2 * ((int64_t)(m - 1) * (L + 1) - (int64_t)(m - 1) * m / 2);
}
__host__ __device__ inline int64_t tri_h(int L, int m) { return (int64_t)m * (L + 1) - (int64_t)m * (m - 1) / 2; }

// (m, part, l - m) of packed index i (0 <= i < (L+1)^2) in the packed m-major
// layout: [m = 0: l = 0..L], then for m >= 1 [cos: l = m..L][sin: l = m..L].
// The m >= 1 blocks up to k hold S(k) = k (2L + 1) - k^2 entries; m - 1 is
// the largest k with S(k) <= i - (L + 1) (root of the quadratic, then exact
// integer correction).
__host__ __device__ inline void unpack_lm(int L, int64_t i, int& m, int& part, int& ll) {
  if (i <= L) {
    m = 0;
    part = 0;
    ll = (int)i;
    return;
  }
  const int64_t j = i - (L + 1);
  const int64_t b = 2LL * L + 1;
  const double bd = (double)b;
  int64_t k = (int64_t)floor((bd - sqrt(bd * bd - 4.0 * (double)j)) * 0.5);
  if (k < 0) k = 0;
  while ((k + 1) * b - (k + 1) * (k + 1) <= j) ++k;
  while (k > 0 && k * b - k * k > j) --k;
  m = (int)k + 1;
  const int64_t w = j - (k * b - k * k);
  const int nsl = L - m + 1;
  part = w >= nsl ? 1 : 0;
  ll = (int)(w - (int64_t)part * nsl);
}

// Work lists of the packed-index kernels: one entry per block, (row, first,
// end) of a contiguous range of one row's packed indices.
constexpr int kWorkBlock = 256;
// per band of a problem in an Exec: {L, group maps, map base, tiles, map stride, dropped from M_PI}
constexpr int kBinfo = 6;

// One spatially varying mixing pair (band nu, component k), eq:Q:
// Q~ = Y^T W Q Y on its grid at the component band-limit.
struct VarMix {
  int nu = 0, k = 0;
  crs_grid grid = nullptr;   // not owned
  DevBuf<double> qw;         // q(n_i) w_i per pixel
  double qeff = 0.0;         // eq:optimal-q, the preconditioners' scalar
};
struct VarMixRun;
struct VarMixRunDel {
  void operator()(VarMixRun* p) const;
};

struct Band {
  crs_grid grid = nullptr;
  int lmax = 0;
  int64_t npix = 0;
  std::vector<double> beam, q, tau_host, w_host;
  DevBuf<double> tau, tplus;  // tau = N^-1 diagonal; tplus = alpha^2 w^2 tau^+
  double alpha2 = 0;
};

// ------------------------------------------------------------ execution
// An Exec runs the operators on a set of independent systems: the right-
// hand sides of one model, or the problems of a batch.  System s belongs to
// problem sys[s].prob and occupies [off, off + n) of the stacked vectors.
// Bands of all systems that share (grid, L) form one group whose Legendre
// and ring launches carry every (system, band) pair as a map.

// Device view of one problem's tables (pointers into its crs_model_s).
struct ProbDev {
  int nc, nb, Lf, Lc;
  const int* lk;
  const int64_t* coff;
  const double* cA;      // [Lf+1][nb][nc]: b_{nu,l} q_{nu,k}
  const double* cP;      // [Lf+1][nb][nc]: U^+ entries of the band rows
  const double* dInv;    // [Lf+1][nc]: C^-1
  const double* dSqrt;   // [Lf+1][nc]: C^-1/2
  const double* dPi;     // [Lf+1][nc][nc]: U^+_pr (U^+_pr)^T
  const double* ftab;    // f_lm triangle at Lf
  const double* Dinv;    // [(Lc+1)^2][nc][nc] M_diag blocks (NULL without)
  const double* const* vptr;  // per band: partial sums of its group (this Exec)
  const int* binfo;           // per band: {L, group maps, map base, tiles, map stride, dropped from M_PI}
  // spatially varying mixing (eq:Q): per (band, component) the pair's index
  // or -1 (NULL: none); y_v = Q~ x_k per system at ybuf + yoff[v] + rhs nalm(L_k)
  const int* vidx;
  const double* ybuf;
  const int64_t* yoff;
};
struct SysDev {
  int prob, rhs;
  int64_t off, n;
};
struct SlotDev {  // one map of a group
  int sys, band;
};

struct ExecGroup {
  crs_grid grid = nullptr;
  int lmax = 0;
  ShtPlan* plan = nullptr;
  LegChoice leg;                      // Legendre kernels of this group (fixed at creation)
  int nmaps = 0, ntiles = 1;
  int64_t nalm = 0, pst = 0;
  std::vector<SlotDev> hslots;
  DevBuf<SlotDev> slots;
  DevBuf<int> mapsys;                 // per map: its system
  DevBuf<int> ident, pikeep;          // per map: its index; 1 if its band takes part in M_PI
  DevBuf<int> mlist, mcount;          // active maps of the launch in progress (k_compact, k_compact_all)
  DevBuf<double> piflag;              // per map (stride kActStride): runs in this M_PI launch
  int pi_maps = 0;                    // maps whose band takes part in M_PI
  std::vector<int> hkeep;             // host copy of pikeep
  DevBuf<const double*> wA, wP, tau;  // per map: tau, alpha^2 w^2 tau^+, tau
  DevBuf<double> uhat, vpart, pix;
  DevBuf<double2> phase;
  DevBuf<const double*> dptr, wptr;   // per map: data / omega_1 maps (right-hand side)
};

// ------------------------------------------- harmonic / map batch operations
// (harmonic.hip).  nm vectors or maps per launch, map j skipped when skip.off(j).
// out_hat[j] = hs f_j[l] (in1_j + in2_j) repacked to LO (in1_j at in1 + off1[j]
// or + j st1; in2 optional at in2 + j st2; f_j = F + mc[j] fst, optional)
void launch_hat_from(double* out, int LO, const double* hs, const double* in1, int L1, const int64_t* off1,
                     int64_t st1, const double* in2, int L2, int64_t st2, const double* F, int fst, const int* mc,
                     int nm, MapSkip skip, hipStream_t s);
// out_j (at out + offo[j] or + j nalm(LO)) (+)= alpha f_j[l] hs sum_t parts[t][j] - g_j[l] sub_j
void launch_from_parts(double* out, const int64_t* offo, int LO, int acc, double alpha, const double* hs,
                       const double* parts, int ntiles, int64_t tstride, const double* F, int fst, const double* sub,
                       int Ls, int64_t sst, const double* Gs, int gst, const int* mc, int nm, MapSkip skip,
                       hipStream_t s);
enum { MOP_MASK = 0, MOP_SCALE = 1, MOP_AXPY_MASK = 2, MOP_POST = 3, MOP_ZERO = 4 };
// MASK: x *= ind; SCALE: x = sm_j b; AXPY_MASK: x += alpha ind y; POST: x += sm_j (b - ind y); ZERO: x = 0
void launch_map_op(int op, double* x, const double* b, const double* y, const double* ind, const double* sm,
                   double alpha, int64_t npix, int nm, MapSkip skip, hipStream_t s);
// Transform scratch sized by reserve() for every (grid, L, maps) it will run;
// the Legendre kernel choice of a (grid, L) is fixed at its first reserve.
struct ShtScratch {
  DevBuf<double> hat, parts;
  DevBuf<double2> phase;
  std::map<std::pair<crs_grid, int>, std::pair<int, LegChoice>> choice;
  void reserve(crs_grid g, int L, int nm, hipStream_t s);
};
// map[j] = Y hat[j] (hat: nm x nalm(L) hat vectors; map stride npix)
void scratch_synth(ShtScratch& w, crs_grid g, int L, int nm, const double* hat, double* map, MapSkip skip,
                   hipStream_t s);
// Y^T map to per-tile partial sums in w.parts ([tile][j][nalm(L)]); returns the tile count
int scratch_adjoint(ShtScratch& w, crs_grid g, int L, int nm, const double* map, MapSkip skip, hipStream_t s);

// Mask-restricted preconditioner (mask.hip): the multigrid hierarchy of a
// model and the per-Exec state of its cycle.
struct MaskMG;
struct MaskRun;
struct MaskMGDel {
  void operator()(MaskMG* p) const;
};
struct MaskRunDel {
  void operator()(MaskRun* p) const;
};

constexpr int kChunk = 8;         // PCG iterations per graph launch
constexpr int kMaxGroupStreams = 8;  // streams the transform groups of an Exec may run on
struct ExecStats {
  int iterations = 0;             // iterations of the slowest system
  int graph_launches = 0;
  int graph_captures = 0;
  int host_syncs = 0;             // host reads of the PCG flags
};

struct Exec {
  std::vector<crs_model> probs;   // not owned
  std::vector<SysDev> hsys;
  int nsys = 0;
  int64_t ntot = 0;
  int Lc = 0;                     // largest component band-limit
  std::vector<ExecGroup> groups;
  DevBuf<ProbDev> dprobs;
  DevBuf<SysDev> dsys;
  DevBuf<int> sys_ident;          // 0 .. nsys-1 (per-system map skipping)
  DevBuf<int2> rows;              // (system, component) rows of the back-mix
  int nrows = 0;
  DevBuf<int4> wl_rows;           // work list over rows: (row, first, end) per block
  int nwl_rows = 0;
  DevBuf<int4> wl_sys;            // work list over systems (component-space index of P.Lc)
  int nwl_sys = 0;
  DevBuf<int2> rng_sys;           // per system: (first block, block count) in wl_sys
  DevBuf<double> wpart;           // per work-list block partial dot products
  DevBuf<double> chi2part;        // per (system, band) partial sums of the chi-square
  std::vector<DevBuf<const double*>> vptr;
  std::vector<DevBuf<int>> binfo;
  bool has_diag = true;
  // host mirror of the activity flags handed to the operators (act): which
  // systems' maps do work; credits profiled launches with that work only
  std::vector<char> hact;
  // PCG workspace
  DevBuf<double> r, z, p, q, t, partial, scal, cand;
  DevBuf<int> dsel;
  double* hscal = nullptr;        // pinned host copy of the scalars [nsys][8]
  int* hsel = nullptr;            // pinned host selection flags [nsys]
  DevBuf<double> xw;              // iterate (the graphs reference only Exec buffers)
  // chunked graphs of the PCG iteration: k iterations per launch with the
  // convergence test on the device (k_iter_end); per chunk iteration a
  // row of residuals (hrows), per system a candidate flag (dcand)
  DevBuf<double> dcand, bbdev, hrows;
  std::vector<char> live;         // per group: some system still iterating
  int chunk_iter = 0;             // iteration within the chunk being captured
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    std::vector<ProfRecord> prof;  // event pairs captured in the graph
    double rtol = 0.0;
    ~GraphEntry();
  };
  // keyed by (preconditioner and profiling, first chunk, iterations, live groups)
  std::map<std::tuple<int, int, int, uint64_t>, std::unique_ptr<GraphEntry>> graphs;
  hipStream_t cap_stream = nullptr;
  ExecStats stats;                // of the last exec_pcg
  std::vector<std::unique_ptr<MaskRun, MaskRunDel>> mask_runs;  // per problem (M_mask)
  std::unique_ptr<VarMixRun, VarMixRunDel> varmix;             // spatially varying mixing
  const int* vm_vidx = nullptr;                                // its device tables (in varmix)
  const double* vm_ybuf = nullptr;
  const int64_t* vm_yoff = nullptr;
  // Transform groups are independent until the back-mix: exec_bands runs
  // them on the caller's stream and on these side streams (default
  // priority), forked from and joined back into the caller's stream by
  // events (inside a graph capture the same calls become graph edges).
  // nstreams: streams the groups run on (1: all on the caller's stream; set
  // by exec_set_streams, part of a captured graph's key).
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  int nstreams = 1;
  ~Exec();
};

// models: the problems; nrhs right-hand sides per problem (systems are
// problem-major).  Allocates all workspaces.
// autotune: time the Legendre kernel variants of every group once per shape
// (leg_autotune) instead of taking the default rules.
std::unique_ptr<Exec> make_exec(const std::vector<crs_model>& models, int nrhs, hipStream_t s,
                                bool autotune = false);
// device bytes make_exec allocates for these models and right-hand-side count
int64_t exec_plan_bytes(const std::vector<crs_model>& models, int nrhs);

enum OpKind { OP_A = 0, OP_PI = 1 };
// act: per-system flags at stride 8 (the PCG scalars' active slot, or the
// candidate flags of a convergence check); systems whose flag is 0 are left
// out (their outputs are not written).  NULL: every system.
// wpart (optional): per block of the system work list (the back-mix runs over
// it), its part of in . out (the system sums are the rng_sys ranges of it).
void exec_apply(Exec& e, OpKind kind, const double* in, double* out, hipStream_t s, const double* act = nullptr,
                double* wpart = nullptr);
// wpart (optional): per block of the system work list, its part of r . z
void exec_diag(Exec& e, const double* r, double* z, hipStream_t s, const double* act = nullptr,
               double* wpart = nullptr);
// algorithmic work of one launch of group gi (family FAM_*) over the maps
// whose system is active in e.hact (masked) or over all of them
Work3 group_work(const Exec& e, int gi, int family, bool masked, bool pi = false);
// the band half of exec_apply: every group's adjoint partial sums, no back-mix
void exec_bands(Exec& e, OpKind kind, const double* in, hipStream_t s, const double* act = nullptr);
// Run the transform groups on up to n streams (1 <= n <= kMaxGroupStreams;
// more than one group is needed for any concurrency); creates the streams.
void exec_set_streams(Exec& e, int n);
void exec_prior_inv(Exec& e, const double* x, double* y, hipStream_t s);
// the band half of exec_rhs (data / omega_1 terms only)
void exec_rhs_bands(Exec& e, const std::vector<std::vector<const double*>>& d,
                    const std::vector<std::vector<const double*>>& w1, hipStream_t s);
void exec_mix_grad(Exec& e, const double* va, int sa0, const double* vb, int sb0, int nrhs, double sign,
                   const double* beamtab, double* dq, hipStream_t s);
// b = sum P^T (tau d + tau^1/2 w1) + C^-1/2 w2; d, w1: per (system, band) host
// tables of device map pointers indexed [sys][band] (NULL = zero); w2 stacked.
void exec_rhs(Exec& e, const std::vector<std::vector<const double*>>& d,
              const std::vector<std::vector<const double*>>& w1, const double* w2, double* b,
              hipStream_t s);
// maps[sys][band] <- P_band x_sys
void exec_project(Exec& e, const double* x, const std::vector<std::vector<double*>>& maps, hipStream_t s);
// y = S^-1 x and val[sys] = 1/2 x^T S^-1 x (val: device, one per system)
void exec_prior_quad(Exec& e, const double* x, double* y, double* val, hipStream_t s);
// res[sys][band] = d - P x and val[sys] = sum_band res^T N^-1 res (device)
void exec_chi2(Exec& e, const double* x, const std::vector<std::vector<const double*>>& d,
               const std::vector<std::vector<double*>>& res, double* val, hipStream_t s);
// out[sys][band] = scale N^-1_band in[sys][band]
void exec_noise_weight(Exec& e, double scale, const std::vector<std::vector<const double*>>& in,
                       const std::vector<std::vector<double*>>& out, hipStream_t s);
// PCG on every system of e.  b, x stacked.  use_graph: run each iteration as
// one captured hipGraph.
int exec_pcg(Exec& e, int precond, const double* b, double* x, double rtol, int maxiter, int* iters,
             double* relres, double* history, bool use_graph, hipStream_t s);

// z (+)= M_mask r on every system whose problem has a mask preconditioner
// (act: skip finished systems, NULL: all)
void exec_mask(Exec& e, const double* r, double* z, bool accumulate, hipStream_t s, const double* act);
bool exec_has_mask(const Exec& e);
// allocates the cycle state of every masked problem of e (before any capture)
void exec_mask_prepare(Exec& e, hipStream_t s);
// Spatially varying mixing (mixmap.hip): y_v = Q~_v x_k of every pair for
// every system (before the forward mix), and out_k += Q~_v (B_nu v_nu) of
// every pair after the transpose mix (v_nu: the band adjoints in the group
// partial sums).  No-ops without mixing maps.
void exec_varmix_fwd(Exec& e, const double* x, hipStream_t s, const double* act);
void exec_varmix_back(Exec& e, double* out, hipStream_t s, const double* act);
bool exec_has_varmix(const Exec& e);
void exec_varmix_prepare(Exec& e, hipStream_t s);
// mixing scalar of (band, component) for the A tables (1 for a varying pair,
// whose map acts through Q~) and for the preconditioners (eq:optimal-q)
double mix_q_a(crs_model m, int nu, int k);
double mix_q_pre(crs_model m, int nu, int k);
// rebuilds the mixing, U^+ and M_diag tables and drops the model's Execs
void model_rebuild_tables(crs_model m, hipStream_t s);
// the model's Exec for nrhs right-hand sides (built on first use)
Exec& model_exec_ref(crs_model m, int nrhs, hipStream_t s);

void launch_philox_normals(uint64_t seed, uint64_t stream, uint64_t rhs0, int nrhs, int64_t n,
                           double* out, hipStream_t s);
void model_draw_omegas(crs_model m, int nrhs, uint64_t seed, std::vector<const double*>& w1,
                       const double*& w2, hipStream_t s);

}  // namespace crs

struct crs_model_s {
  int ncomp = 0, nbands = 0;
  std::vector<int> lk;
  std::vector<std::vector<double>> invcl;
  std::vector<int64_t> coff;
  int64_t n = 0;
  int Lc = 0, Lmax = 0;
  std::vector<crs::Band> bands;
  bool has_diag = false;
  // per-l tables
  crs::DevBuf<double> cA, cP;        // [Lmax+1][nb][nc]
  crs::DevBuf<double> dInv, dSqrt;   // [Lmax+1][nc] diagonal prior terms
  crs::DevBuf<double> dPi;           // [Lmax+1][nc][nc]
  crs::DevBuf<double> ftab;          // f_lm triangle at Lmax
  crs::DevBuf<double> beamtab;       // [Lmax+1][nb] b_{nu,l} (0 above L_nu)
  crs::DevBuf<double> gwork;         // [x; lambda] stacked for the mixing gradient
  crs::DevBuf<double> Dinv;          // [(Lc+1)^2][nc][nc]
  crs::DevBuf<int> d_lk;
  crs::DevBuf<int64_t> d_coff;
  std::vector<double> upinv;         // host copy [Lmax+1][nc][nb+nc]
  // execution state for this model alone, per right-hand-side count, and CR draws
  std::map<int, std::unique_ptr<crs::Exec>> execs;
  crs::DevBuf<double> om1, om2, bcr;
  std::unique_ptr<crs::MaskMG, crs::MaskMGDel> mask;  // M_mask hierarchy (crs_model_set_mask)
  std::vector<crs::VarMix> varmix;   // spatially varying mixing pairs (eq:Q)
  std::vector<int> merge_group;      // per band: observation-merge group (-1: alone), App. A.3
  std::vector<char> pi_drop;         // per band: merged into another band's row of U (no T^+)
  int device = 0;
};
