// Ring grids (HEALPix RING, Gauss-Legendre), per-ring FFT tables and the
// per-(grid, lmax) Legendre plans.
//
// HEALPix RING geometry follows Gorski et al. (2005); the paper uses HEALPix
// sky maps and recommends Gauss-Legendre grids where exact quadrature is
// wanted (Sect. 2.1, Sect. 2.2 below eq:Q).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace crs {

namespace {

// sin(pi x), cos(pi x) with exact argument reduction (x a ratio of integers
// reduced modulo 2 by the caller); accurate to a few ulps.
void host_sincospi(double x, double* s, double* c) {
  x = std::fmod(x, 2.0);
  if (x < 0) x += 2.0;
  // reduce to [0, 0.5] using symmetries
  double sign_s = 1.0, sign_c = 1.0;
  if (x >= 1.0) { x -= 1.0; sign_s = -1.0; sign_c = -1.0; }
  if (x > 0.5) { x = 1.0 - x; sign_c = -sign_c; }
  double ss, cc;
  if (x <= 0.25) {
    ss = std::sin(M_PI * x);
    cc = std::cos(M_PI * x);
  } else {
    double y = 0.5 - x;
    ss = std::cos(M_PI * y);
    cc = std::sin(M_PI * y);
  }
  *s = sign_s * ss;
  *c = sign_c * cc;
}

// Radices of an FFT of length n: the power-of-two part 2^e in as few stages
// as possible (radix 8, with 2^4 as 4 x 4 and a remaining 2^2 as one radix
// 4), then the odd prime factors in increasing order.
std::vector<int> factorize(int n) {
  std::vector<int> f;
  int e = 0;
  while (n % 2 == 0) { ++e; n /= 2; }
  int n8 = e / 3, rest = e % 3;
  if (rest == 1 && n8 > 0) { --n8; rest = 4; }
  for (int i = 0; i < n8; ++i) f.push_back(8);
  if (rest == 4) { f.push_back(4); f.push_back(4); }
  if (rest == 2) f.push_back(4);
  if (rest == 1) f.push_back(2);
  for (int p = 3; p * p <= n; p += 2)
    while (n % p == 0) { f.push_back(p); n /= p; }
  if (n > 1) f.push_back(n);
  if (f.empty()) f.push_back(1);
  return f;
}

// In-place radix-2 complex FFT (forward, exp(-2 pi i jk / n)), n a power of two.
void host_fft_pow2(std::vector<double2>& x) {
  const int n = (int)x.size();
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(x[i], x[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    const int h = len / 2;
    for (int k = 0; k < h; ++k) {
      double sv, cv;
      host_sincospi(-2.0 * k / len, &sv, &cv);
      for (int i = k; i < n; i += len) {
        const double2 u = x[i], v = x[i + h];
        const double2 t = make_double2(v.x * cv - v.y * sv, v.x * sv + v.y * cv);
        x[i] = make_double2(u.x + t.x, u.y + t.y);
        x[i + h] = make_double2(u.x - t.x, u.y - t.y);
      }
    }
  }
}

// Bluestein filter for a length-n DFT by a length-M cyclic convolution
// (M >= 2n - 1): b_d = exp(+i pi d^2 / n) for |d| < n, wrapped to M, and
// its forward DFT divided by M (so that the device inverse FFT needs no
// scaling).  Phases are reduced exactly: d^2 mod 2n.
std::vector<double2> bluestein_filter(int n, int M) {
  std::vector<double2> b(M, make_double2(0.0, 0.0));
  for (int d = 0; d < n; ++d) {
    double sv, cv;
    const long long t = ((long long)d * d) % (2LL * n);
    host_sincospi((double)t / n, &sv, &cv);
    b[d] = make_double2(cv, sv);
    if (d) b[M - d] = b[d];
  }
  host_fft_pow2(b);
  for (auto& v : b) v = make_double2(v.x / M, v.y / M);
  // followed by the chirp w_d = exp(-i pi d^2 / n), d < n
  for (int d = 0; d < n; ++d) {
    double sv, cv;
    const long long t = ((long long)d * d) % (2LL * n);
    host_sincospi((double)t / n, &sv, &cv);
    b.push_back(make_double2(cv, -sv));
  }
  return b;
}

// P_n(cos th) and P_{n-1}(cos th) by the Legendre recurrence written for
// D_j = P_j - P_{j-1} and t = 1 - cos th = 2 sin^2(th / 2):
//   D_j = ((j - 1) D_{j-1} - (2j - 1) t P_{j-1}) / j,   P_j = P_{j-1} + D_j.
// It carries the deviation of P_j from P_j(1) = 1 explicitly, with t taken
// from th, so the values keep full relative precision near the pole (the
// recurrence in x = cos th inherits the rounding of x, which near the poles
// moves P_{n-1} by about 1e-6 relative at n = 4000).
void legendre_theta(int n, double th, double& pn, double& pm1) {
  const double sh = std::sin(0.5 * th);
  const double t = 2.0 * sh * sh;
  double prev = 1.0, p = 1.0 - t, d = -t;  // P_0, P_1, D_1
  for (int j = 2; j <= n; ++j) {
    d = ((j - 1.0) * d - (2.0 * j - 1.0) * t * p) / j;
    prev = p;
    p += d;
  }
  pn = n == 0 ? 1.0 : p;
  pm1 = n == 0 ? 0.0 : prev;
}

// Gauss-Legendre nodes (descending) and weights: Newton iteration on theta
// for the nodes of the northern half (theta <= pi / 2), the southern half by
// symmetry; weights w = 2 sin^2 th / (n P_{n-1}(cos th))^2.
void gl_nodes(int n, std::vector<double>& z, std::vector<double>& st, std::vector<double>& w) {
  z.resize(n);
  st.resize(n);
  w.resize(n);
  for (int k = 0; k < (n + 1) / 2; ++k) {
    double th = M_PI * (k + 0.75) / (n + 0.5);
    double pn = 0, pm1 = 0;
    for (int it = 0; it < 100; ++it) {
      legendre_theta(n, th, pn, pm1);
      // d/dth P_n(cos th) = n (cos th P_n - P_{n-1}) / sin th
      const double dth = pn * std::sin(th) / (n * (std::cos(th) * pn - pm1));
      th -= dth;
      if (std::fabs(dth) < 1e-16) break;
    }
    legendre_theta(n, th, pn, pm1);
    const double s = std::sin(th);
    const double x = (2 * k + 1 == n) ? 0.0 : std::cos(th);
    const double wk = 2.0 * s * s / ((n * pm1) * (n * pm1));
    z[k] = x;
    st[k] = s;
    w[k] = wk;
    z[n - 1 - k] = -x;
    st[n - 1 - k] = s;
    w[n - 1 - k] = wk;
  }
}

}  // namespace

// Uploads per-ring tables (lengths, offsets, phi0, FFT factors, twiddles).
void grid_finalize(crs_grid g, hipStream_t s) {
  int nr = g->nring;
  g->offset.resize(nr);
  int64_t off = 0;
  for (int r = 0; r < nr; ++r) {
    g->offset[r] = off;
    off += g->nphi[r];
  }
  g->npix = off;
  for (int r = 0; r < nr; ++r)
    CRS_CHECK(g->nphi[r] <= kMaxRing, CRS_EUNSUPPORTED,
              "ring length above 8192 pixels is not supported");
  // Per ring: the complex FFT that the ring kernels run.  Even Nphi uses a
  // half-length complex transform (two real samples per complex word); a
  // length whose largest prime factor exceeds 7 goes through Bluestein's
  // chirp convolution with a power-of-two FFT.
  std::vector<int> nfac(nr), fac((size_t)nr * kMaxFactors, 1), fftn(nr);
  std::vector<unsigned> facm((size_t)nr * kMaxFactors, 0u);
  std::vector<int64_t> twoff(nr), bfoff(nr, -1);
  std::map<int, int64_t> tw_of, bf_of;
  std::vector<double2> tw, bf;
  g->ring_classes.clear();
  std::map<int, int> class_of;
  bool any_blue = false;
  for (int r = 0; r < nr; ++r) {
    const int n = g->nphi[r];
    const bool half = (n % 2) == 0;
    const int n0 = half ? n / 2 : n;
    auto f0 = factorize(n0);
    // radices are 2, 4, 8 and primes, so a prime factor above 7 is one > 8
    bool blue = false;
    for (int v : f0) blue = blue || v > 8;
    int nf = n0;
    if (blue) {
      nf = 1;
      while (nf < 2 * n0 - 1) nf *= 2;
      any_blue = true;
      auto it = bf_of.find(n0);
      if (it == bf_of.end()) {
        bf_of[n0] = (int64_t)bf.size();
        bfoff[r] = (int64_t)bf.size();
        auto spec = bluestein_filter(n0, nf);
        bf.insert(bf.end(), spec.begin(), spec.end());
      } else {
        bfoff[r] = it->second;
      }
    }
    CRS_CHECK(nf <= kBlueMax, CRS_EUNSUPPORTED,
              "ring FFT above 8192 points (an odd ring longer than 4096 pixels with a prime factor above 7)");
    auto ff = factorize(nf);
    CRS_CHECK((int)ff.size() <= kMaxFactors, CRS_EUNSUPPORTED, "too many FFT factors");
    nfac[r] = (int)ff.size();
    {
      unsigned ns = 1;
      for (size_t i = 0; i < ff.size(); ++i) {
        fac[(size_t)r * kMaxFactors + i] = ff[i];
        facm[(size_t)r * kMaxFactors + i] = ns <= 1 ? 0u : (unsigned)(0xFFFFFFFFull / ns + 1);
        ns *= (unsigned)ff[i];
      }
    }
    fftn[r] = nf;
    g->ring_maxn = std::max(g->ring_maxn, n);
    auto it = tw_of.find(n);
    if (it == tw_of.end()) {
      int64_t o = (int64_t)tw.size();
      tw_of[n] = o;
      for (int t = 0; t < 2 * n; ++t) {
        double sv, cv;
        host_sincospi((double)t / (double)n, &sv, &cv);
        tw.push_back(make_double2(cv, -sv));
      }
      twoff[r] = o;
    } else {
      twoff[r] = it->second;
    }
    int tier = 0;
    while (ring_tier_maxfft(tier) < nf) ++tier;
    // classes by (tier, Bluestein, odd radix) from the 512-thread tier up: a
    // class without odd radices runs a kernel built for power-of-two FFTs
    // only (72 instead of 115 registers: more blocks per CU), and Bluestein's
    // longer buffers do not set the LDS size of the direct rings.  The
    // smaller tiers stay whole (their kernels differ by a few registers,
    // less than an extra launch costs).
    bool odd = false;
    for (int v : ff) odd = odd || (v % 2) != 0;
    const int key = tier >= 2 ? tier * 4 + (blue ? 2 : 0) + (odd ? 1 : 0) : tier * 4;
    auto ci = class_of.find(key);
    if (ci == class_of.end()) {
      class_of[key] = (int)g->ring_classes.size();
      g->ring_classes.emplace_back();
      g->ring_classes.back().tier = tier;
      ci = class_of.find(key);
    }
    RingClass& rc = g->ring_classes[ci->second];
    rc.rings.push_back(r);
    rc.blue = rc.blue || blue;
    rc.odd = rc.odd || odd;
    rc.xcap = std::max(rc.xcap, std::max(nf, n0));
    rc.maxn = std::max(rc.maxn, n);
    const int nt = ring_tier_threads(tier);
    if (n <= nt) rc.gcap = std::max(rc.gcap, n + n * (nt / n));
  }
  // largest tier first
  std::stable_sort(g->ring_classes.begin(), g->ring_classes.end(),
                   [](const RingClass& x, const RingClass& y) { return x.tier > y.tier; });
  g->d_ring_class.clear();
  for (auto& rc : g->ring_classes) {
    g->d_ring_class.emplace_back();
    g->d_ring_class.back().upload(rc.rings, s);
  }
  // Launches with few maps merge the classes that would have too few blocks
  // to fill the GPU on their own into one launch (run by the kernel of their
  // largest tier).  Which classes are small depends on the map count, but
  // they are always the first ones in order of ring count, so the merged
  // class of every such prefix is prepared here.
  const int ncls = (int)g->ring_classes.size();
  CRS_CHECK(ncls <= kMaxRingClasses, CRS_EUNSUPPORTED, "too many ring classes");
  g->ring_small_order.resize(ncls);
  for (int c = 0; c < ncls; ++c) g->ring_small_order[c] = c;
  std::stable_sort(g->ring_small_order.begin(), g->ring_small_order.end(), [&](int x, int y) {
    return g->ring_classes[x].rings.size() < g->ring_classes[y].rings.size();
  });
  g->ring_prefix.clear();
  g->d_ring_prefix.clear();
  RingClass acc;
  for (int k = 0; k < ncls; ++k) {
    const RingClass& rc = g->ring_classes[g->ring_small_order[k]];
    acc.tier = std::max(acc.tier, rc.tier);
    acc.blue = acc.blue || rc.blue;
    acc.odd = acc.odd || rc.odd;
    acc.xcap = std::max(acc.xcap, rc.xcap);
    acc.maxn = std::max(acc.maxn, rc.maxn);
    acc.rings.insert(acc.rings.end(), rc.rings.begin(), rc.rings.end());
    RingClass m = acc;
    std::sort(m.rings.begin(), m.rings.end());
    // fold scratch for the merged kernel's block size
    const int nt = ring_tier_threads(m.tier);
    m.gcap = 0;
    for (int r : m.rings) {
      const int n = g->nphi[r];
      if (n <= nt) m.gcap = std::max(m.gcap, n + n * (nt / n));
    }
    g->ring_prefix.push_back(m);
    g->d_ring_prefix.emplace_back();
    g->d_ring_prefix.back().upload(m.rings, s);
  }
  if (any_blue) {
    std::vector<double2> t2(kBlueMax);
    for (int t = 0; t < kBlueMax; ++t) {
      double sv, cv;
      host_sincospi(2.0 * t / kBlueMax, &sv, &cv);
      t2[t] = make_double2(cv, -sv);
    }
    g->d_tw2.upload(t2, s);
    g->d_bf.upload(bf, s);
  }
  g->d_fftn.upload(fftn, s);
  g->d_bfoff.upload(bfoff, s);
  int np = (nr + 1) / 2;
  std::vector<double> zp(np), sp(np);
  for (int p = 0; p < np; ++p) {
    zp[p] = g->z[p];
    sp[p] = g->sint[p];
  }
  g->d_nphi.upload(g->nphi, s);
  g->d_offset.upload(g->offset, s);
  g->d_phinum.upload(g->phi0_num, s);
  g->d_phiden.upload(g->phi0_den, s);
  g->d_nfac.upload(nfac, s);
  g->d_fac.upload(fac, s);
  g->d_facm.upload(facm, s);
  g->d_twoff.upload(twoff, s);
  g->d_tw.upload(tw, s);
  g->d_zpair.upload(zp, s);
  g->d_spair.upload(sp, s);
  CRS_HIP(hipStreamSynchronize(s));
}

void build_healpix(crs_grid g, int nside) {
  g->kind = 0;
  g->nside = nside;
  int nr = 4 * nside - 1;
  g->nring = nr;
  g->z.resize(nr);
  g->sint.resize(nr);
  g->nphi.resize(nr);
  g->phi0_num.resize(nr);
  g->phi0_den.resize(nr);
  g->ringw.assign(nr, 4.0 * M_PI / (12.0 * nside * (double)nside));
  double ns = nside;
  for (int k = 0; k < nr; ++k) {
    int i = k + 1;
    if (i < nside || i > 3 * nside) {
      int ii = (i < nside) ? i : 4 * nside - i;
      double om = (double)ii * ii / (3.0 * ns * ns);  // 1 - |z|
      double zz = 1.0 - om;
      g->z[k] = (i < nside) ? zz : -zz;
      g->sint[k] = std::sqrt(om * (2.0 - om));
      g->nphi[k] = 4 * ii;
      g->phi0_num[k] = 1;   // phi0 = pi / (4 ii) = pi / nphi
      g->phi0_den[k] = 4 * ii;
    } else {
      double zz = 4.0 / 3.0 - (2.0 * i) / (3.0 * ns);
      g->z[k] = zz;
      g->sint[k] = std::sqrt((1.0 - zz) * (1.0 + zz));
      g->nphi[k] = 4 * nside;
      bool shifted = ((i - nside) % 2) == 0;
      g->phi0_num[k] = shifted ? 1 : 0;
      g->phi0_den[k] = 4 * nside;
    }
  }
}

void build_gl(crs_grid g, int nrings, int nphi) {
  g->kind = 1;
  g->nring = nrings;
  g->nphi_gl = nphi;
  std::vector<double> w;
  gl_nodes(nrings, g->z, g->sint, w);
  g->nphi.assign(nrings, nphi);
  g->phi0_num.assign(nrings, 0);
  g->phi0_den.assign(nrings, nphi);
  g->ringw.resize(nrings);
  for (int r = 0; r < nrings; ++r) g->ringw[r] = w[r] * 2.0 * M_PI / nphi;
}

// ----------------------------------------------------------- Legendre plan
// mu-recurrence tables.  With a_lm = sqrt((4l^2-1)/(l^2-m^2)),
// b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)) and c_lm = a_lm b_lm the normalised
// associated Legendre functions obey lambda_l = a_l z lambda_{l-1} - c_l lambda_{l-2}.
// Writing lambda_l = f_l mu_l with f_m = f_{m+1} = 1, f_l = c_l f_{l-2} turns
// this into mu_l = g_l z mu_{l-1} - mu_{l-2}, g_l = a_l f_{l-1} / f_l: one
// multiply and one FMA per step.  Triangle layout: entry (l, m) at
// tri(m) + l - m, tri(m) = m (L+1) - m (m-1) / 2.
__host__ __device__ static inline int64_t tri_off(int L, int m) { return (int64_t)m * (L + 1) - (int64_t)m * (m - 1) / 2; }

__global__ void k_start_table(const double* __restrict__ gtab, const double* __restrict__ ftab,
                              const double* __restrict__ zp, const double* __restrict__ sp,
                              const double* __restrict__ pm_mant, const int* __restrict__ pm_exp,
                              int L, int npairs, double thr, int* __restrict__ ls_out,
                              double2* __restrict__ ms_out, double thr_lo, int* __restrict__ lu_out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  int m = blockIdx.y;
  if (p >= npairs || m > L) return;
  double z = zp[p], s = sp[p];
  // lambda_mm = P_m sin^m(theta), carried as mantissa * 2^e
  double mant = pm_mant[m];
  long e = pm_exp[m];
  if (m > 0) {
    if (s == 0.0) {
      mant = 0.0;
    } else {
      int se;
      double sm = frexp(s, &se);
      double r = 1.0;
      long er = 0;
      double base = sm;
      long eb = se;
      int k = m;
      while (k) {
        if (k & 1) {
          int t;
          r = frexp(r * base, &t);
          er += eb + t;
        }
        k >>= 1;
        if (k) {
          int t;
          base = frexp(base * base, &t);
          eb = 2 * eb + t;
        }
      }
      int t;
      mant = frexp(mant * r, &t);
      e += er + t;
    }
  }
  const double* g = gtab + tri_off(L, m) - m;
  const double* f = ftab + tri_off(L, m) - m;
  double mu_prev = 0.0, mu_cur = mant;
  int l = m;
  int lsv = L + 1, luv = L + 1;
  double2 msv = make_double2(0.0, 0.0);
  // threshold tests on |lambda_l| = f_l |mu_l| 2^e: the first l at or above
  // thr_lo (counted, not used by the kernels) and at or above thr (start)
  while (true) {
    double v = fabs(f[l] * mu_cur);
    if (luv > L && v != 0.0 && e > -2000 && ldexp(v, (int)e) >= thr_lo) luv = l;
    if (v != 0.0 && e > -2000 && ldexp(v, (int)e) >= thr) {
      lsv = l;
      msv = make_double2(ldexp(mu_prev, (int)e), ldexp(mu_cur, (int)e));
      break;
    }
    ++l;
    if (l > L) break;
    double nx = g[l] * z * mu_cur - mu_prev;
    mu_prev = mu_cur;
    mu_cur = nx;
    if (fabs(mu_cur) > 0x1p600) {
      mu_cur *= 0x1p-600;
      mu_prev *= 0x1p-600;
      e += 600;
    }
  }
  ls_out[(size_t)m * npairs + p] = lsv;
  ms_out[(size_t)m * npairs + p] = msv;
  lu_out[(size_t)m * npairs + p] = luv;
}

constexpr double kSkipThreshold = 0x1p-100;  // |lambda| below this is not evaluated
constexpr double kFp64Normal = 0x1p-1022;    // smallest normal float64

ShtPlan& get_plan(crs_grid g, int lmax, hipStream_t s) {
  auto it = g->plans.find(lmax);
  if (it != g->plans.end()) return *it->second;
  auto plan = std::make_unique<ShtPlan>();
  int L = lmax;
  plan->lmax = L;
  plan->npairs = (g->nring + 1) / 2;
  int64_t ntri = (int64_t)(L + 1) * (L + 2) / 2;
  // g carries 8 trailing zeros: the MFMA synthesis reads it in aligned groups of 8 past L
  std::vector<double> gt(ntri + 8, 0.0), ft(ntri, 0.0);
  for (int m = 0; m <= L; ++m) {
    int64_t o = tri_off(L, m) - m;
    ft[o + m] = 1.0;
    if (m + 1 <= L) {
      ft[o + m + 1] = 1.0;
      gt[o + m + 1] = std::sqrt(2.0 * m + 3.0);
    }
    for (int l = m + 2; l <= L; ++l) {
      double dl = l, dm = m;
      double a = std::sqrt((4.0 * dl * dl - 1.0) / ((dl - dm) * (dl + dm)));
      double b = std::sqrt(((dl - 1.0 - dm) * (dl - 1.0 + dm)) / (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
      ft[o + l] = a * b * ft[o + l - 2];
      gt[o + l] = a * ft[o + l - 1] / ft[o + l];
    }
  }
  // P_m = lambda_00 prod_{k<=m} sqrt((2k+1)/(2k)) as mantissa/exponent
  std::vector<double> pmm(L + 1);
  std::vector<int> pme(L + 1);
  {
    int e;
    double mant = std::frexp(1.0 / std::sqrt(4.0 * M_PI), &e);
    long ee = e;
    pmm[0] = mant;
    pme[0] = (int)ee;
    for (int m = 1; m <= L; ++m) {
      mant *= std::sqrt((2.0 * m + 1.0) / (2.0 * m));
      int t;
      mant = std::frexp(mant, &t);
      ee += t;
      pmm[m] = mant;
      pme[m] = (int)ee;
    }
  }
  // c_m f_lm in the packed alm layout ([m = 0: l], then per m >= 1 [cos: l][sin: l])
  std::vector<double> hs((size_t)(L + 1) * (L + 1));
  {
    size_t o = 0;
    for (int m = 0; m <= L; ++m) {
      const double cm = m == 0 ? 1.0 : std::sqrt(2.0);
      const int64_t t = tri_off(L, m) - m;
      for (int part = 0; part < (m == 0 ? 1 : 2); ++part)
        for (int l = m; l <= L; ++l) hs[o++] = cm * ft[t + l];
    }
  }
  plan->g.upload(gt, s);
  plan->f.upload(ft, s);
  plan->hs.upload(hs, s);
  DevBuf<double> dpm;
  DevBuf<int> dpe;
  dpm.upload(pmm, s);
  dpe.upload(pme, s);
  plan->ls.alloc((size_t)(L + 1) * plan->npairs);
  plan->ms.alloc((size_t)(L + 1) * plan->npairs);
  DevBuf<int> dlu;
  dlu.alloc((size_t)(L + 1) * plan->npairs);
  dim3 grid((plan->npairs + 127) / 128, L + 1);
  hipLaunchKernelGGL(k_start_table, grid, dim3(128), 0, s, plan->g.p, plan->f.p, g->d_zpair.p,
                     g->d_spair.p, dpm.p, dpe.p, L, plan->npairs, kSkipThreshold, plan->ls.p,
                     plan->ms.p, kFp64Normal, dlu.p);
  CRS_HIP(hipGetLastError());
  std::vector<int> lsh((size_t)(L + 1) * plan->npairs), luh(lsh.size());
  CRS_HIP(hipMemcpyAsync(lsh.data(), plan->ls.p, lsh.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  CRS_HIP(hipMemcpyAsync(luh.data(), dlu.p, luh.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  CRS_HIP(hipStreamSynchronize(s));
  int64_t eff = 0, eff64 = 0;
  for (size_t i = 0; i < lsh.size(); ++i) {
    if (lsh[i] <= L) eff += L - lsh[i] + 1;
    if (luh[i] <= L) eff64 += L - luh[i] + 1;
  }
  plan->eff_triples = eff;
  plan->fp64_triples = eff64;
  plan->nominal_triples = (int64_t)plan->npairs * ntri;
  auto& ref = *plan;
  g->plans[lmax] = std::move(plan);
  return ref;
}

}  // namespace crs

using namespace crs;

extern "C" {

int crs_grid_healpix(int nside, crs_grid* out) {
  return guarded([&] {
    CRS_CHECK(out != nullptr, CRS_EINVAL, "out is NULL");
    CRS_CHECK(nside >= 1, CRS_EINVAL, "nside must be >= 1");
    CRS_CHECK(nside <= 2048, CRS_EUNSUPPORTED, "nside above 2048 is not supported");
    auto g = std::make_unique<crs_grid_s>();
    CRS_HIP(hipGetDevice(&g->device));
    build_healpix(g.get(), nside);
    grid_finalize(g.get(), nullptr);
    *out = g.release();
    return CRS_OK;
  });
}

int crs_grid_gauss_legendre(int nrings, int nphi, crs_grid* out) {
  return guarded([&] {
    CRS_CHECK(out != nullptr, CRS_EINVAL, "out is NULL");
    CRS_CHECK(nrings >= 1 && nphi >= 1, CRS_EINVAL, "nrings and nphi must be >= 1");
    CRS_CHECK(nphi <= kMaxRing, CRS_EUNSUPPORTED, "nphi above 8192 is not supported");
    // an odd ring is transformed at full length: above 4096 pixels its length
    // must be 7-smooth (Bluestein's convolution would exceed 8192 points)
    if (nphi % 2 == 1 && nphi > kMaxRing / 2) {
      int n = nphi;
      for (int p : {3, 5, 7})
        while (n % p == 0) n /= p;
      CRS_CHECK(n == 1, CRS_EUNSUPPORTED, "odd nphi above 4096 must have no prime factor above 7");
    }
    auto g = std::make_unique<crs_grid_s>();
    CRS_HIP(hipGetDevice(&g->device));
    build_gl(g.get(), nrings, nphi);
    grid_finalize(g.get(), nullptr);
    *out = g.release();
    return CRS_OK;
  });
}

int crs_grid_info(crs_grid g, int* nrings, int64_t* npix) {
  return guarded([&] {
    CRS_CHECK(g != nullptr, CRS_EINVAL, "grid is NULL");
    if (nrings) *nrings = g->nring;
    if (npix) *npix = g->npix;
    return CRS_OK;
  });
}

int crs_grid_pixel_centres(crs_grid g, double* z, double* phi) {
  return guarded([&] {
    CRS_CHECK(g != nullptr, CRS_EINVAL, "grid is NULL");
    CRS_CHECK(z != nullptr && phi != nullptr, CRS_EINVAL, "z or phi is NULL");
    for (int r = 0; r < g->nring; ++r) {
      int n = g->nphi[r];
      for (int j = 0; j < n; ++j) {
        z[g->offset[r] + j] = g->z[r];
        // phi = pi * (num/den + 2 j / n)
        double x = (double)g->phi0_num[r] / g->phi0_den[r] + 2.0 * j / n;
        phi[g->offset[r] + j] = M_PI * x;
      }
    }
    return CRS_OK;
  });
}

int crs_grid_weights(crs_grid g, double* w) {
  return guarded([&] {
    CRS_CHECK(g != nullptr, CRS_EINVAL, "grid is NULL");
    CRS_CHECK(w != nullptr, CRS_EINVAL, "w is NULL");
    for (int r = 0; r < g->nring; ++r)
      for (int j = 0; j < g->nphi[r]; ++j) w[g->offset[r] + j] = g->ringw[r];
    return CRS_OK;
  });
}

int crs_grid_destroy(crs_grid g) {
  return guarded([&] {
    delete g;
    return CRS_OK;
  });
}

}  // extern "C"
