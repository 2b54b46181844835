// Ring stage of the spherical harmonic transforms: per-ring FFTs in LDS.
//
// Synthesis, second half of Y (Sect. 2.1): on ring r with Nphi pixels at
// phi_j = phi0 + 2 pi j / Nphi,
//     f_j = Re sum_{m=0..L} (F^c_m - i F^s_m) e^{i m phi_j}.
// The m sum is folded onto Nphi bins (m -> m mod Nphi, conjugate partner
// -m) so that f = inverse DFT of a Hermitian spectrum c; rings with
// Nphi < 2L+1 alias exactly as the dense operator does.
// Adjoint, first half of Y^T (Sect. 3.2): H_m = e^{-i m phi0} F^_{m mod Nphi},
// F^_k = sum_j f_j e^{-2 pi i j k / Nphi}, H^c = Re H, H^s = -Im H.
// Round trip (inside A and T^+): synthesis, multiply by a pixel weight
// (tau for A, alpha^2 w^2 tau^+ for T^+; Sect. 2.3 and Sect. 3.3), adjoint --
// the map never leaves LDS.
// Diagonal setup (M_diag, Sect. 5): for a pixel map t, G^c_m = T^_0 +
// Re(e^{-2 i m phi0} T^_{2m}), G^s_m = T^_0 - Re(...), G_0 = (T^_0, 0):
// sum_j t_j cos^2(m phi_j) = (G^c_m)/2 etc.
//
// Transform layout.  The ring data are real, so an even ring (Nphi = 2H, all
// HEALPix rings) runs a complex FFT of length H on z_n = f_{2n} + i f_{2n+1}:
//   synthesis  Z_k = (c_k + c_{k+H}) + i e^{2 pi i k / Nphi} (c_k - c_{k+H}),
//              z = inverse DFT_H(Z);
//   adjoint    Z = DFT_H(z), E_k = (Z_k + conj Z_{H-k}) / 2,
//              O_k = (Z_k - conj Z_{H-k}) / (2i), F^_k = E_k + e^{-2 pi i k / Nphi} O_k.
// Odd rings run a full complex FFT of length Nphi.  The FFT is a mixed-radix
// Stockham autosort in LDS (radix 8, 4, 2, 3, 5, 7); a length with a prime
// factor above 7 is computed by Bluestein's chirp-z identity
// n k = (n^2 + k^2 - (k - n)^2) / 2 as a cyclic convolution of power-of-two
// length M >= 2n - 1 (filter spectrum precomputed per length on the host).
// One block per (ring, map); rings are launched in classes by FFT length
// (<= 512: 128 threads, <= 1024: 256, <= 4096: 512, <= 8192: 1024) and,
// for the two longer tiers, by Bluestein or direct transform and whether
// the FFT has odd radices; the half-length and Bluestein paths are chosen
// per ring.
#include "internal.h"

namespace crs {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Exact quotient n / d for n * d < 2^32 (multiply-high by ceil(2^32 / d)).
struct FastDiv {
  unsigned d, m;
  __device__ __forceinline__ explicit FastDiv(unsigned dd)
      : d(dd), m(dd <= 1 ? 0u : 0xFFFFFFFFu / dd + 1u) {}  // 32-bit quotient: same value
  // with the multiplier precomputed on the host
  __device__ __forceinline__ FastDiv(unsigned dd, unsigned mm) : d(dd), m(mm) {}
  __device__ __forceinline__ unsigned div(unsigned n) const { return d <= 1 ? n : __umulhi(n, m); }
  __device__ __forceinline__ unsigned mod(unsigned n) const { return n - div(n) * d; }
};

// Twiddles exp(-2 pi i u / Lt) from two LDS tables: Wf[u & 63] Wc[u >> 6]
// (exact table entries; the product adds one rounding).  An FFT of length
// n | Lt reads omega_n^t at u = t * q, q = Lt / n.
struct TwCtx {
  const double2* Wf;
  const double2* Wc;
  int q;
  __device__ __forceinline__ double2 at(int u) const { return cmul(Wc[u >> 6], Wf[u & 63]); }
  __device__ __forceinline__ double2 tw(int t, bool inv) const {
    const double2 w = at(t * q);
    return inv ? conj2(w) : w;
  }
};

// The ring's table exp(-i pi t / Nphi), t < 2 Nphi, read from global memory
// (L2-resident: every ring of that length and every map shares it).  The
// fold reads its phase factors here, so it need not wait for the LDS copy of
// the tables.
struct GlobalTw {
  const double2* __restrict__ T;
  __device__ __forceinline__ double2 at(int t) const { return T[t]; }
};

// cos(2 pi k / R) and sin(2 pi k / R), 1 <= k <= (R-1)/2, for the odd radices
// (values correctly rounded from their closed forms).
__device__ __forceinline__ constexpr double dft_cos(int R, int k) {
  return R == 3 ? -0.5
       : R == 5 ? (k == 1 ? 0.3090169943749474241022934 : -0.8090169943749474241022934)
       : (k == 1 ? 0.6234898018587335305250049
                 : k == 2 ? -0.2225209339563144042889026 : -0.9009688679024191262361023);
}
__device__ __forceinline__ constexpr double dft_sin(int R, int k) {
  return R == 3 ? 0.8660254037844386467637232
       : R == 5 ? (k == 1 ? 0.9510565162951535721164393 : 0.5877852522924731291687060)
       : (k == 1 ? 0.7818314824680298087084445
                 : k == 2 ? 0.9749279121818236070181317 : 0.4338837391175581204757683);
}

template <int R>
__device__ __forceinline__ void small_dft(double2 (&v)[R], bool inv) {
  if constexpr (R == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 8) {
    // X_k = E_k + w^k O_k, X_{k+4} = E_k - w^k O_k (E, O: 4-point DFTs of the
    // even and odd samples; w = exp(-/+ i pi / 4))
    double2 e[4] = {v[0], v[2], v[4], v[6]};
    double2 o[4] = {v[1], v[3], v[5], v[7]};
    small_dft<4>(e, inv);
    small_dft<4>(o, inv);
    constexpr double h = 0.7071067811865475244008444;  // 1 / sqrt(2)
    double2 t[4];
    t[0] = o[0];
    t[1] = inv ? make_double2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
               : make_double2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    t[2] = inv ? make_double2(-o[2].y, o[2].x) : make_double2(o[2].y, -o[2].x);
    t[3] = inv ? make_double2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
               : make_double2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], t[k]);
      v[k + 4] = csub(e[k], t[k]);
    }
  } else if constexpr (R == 4) {
    const double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const double2 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    const double2 mit3 = make_double2(t3.y, -t3.x);  // -i t3
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = inv ? csub(t1, mit3) : cadd(t1, mit3);
    v[3] = inv ? cadd(t1, mit3) : csub(t1, mit3);
  } else {
    // odd R: with a_s = x_s + x_{R-s}, b_s = x_s - x_{R-s},
    //   y_r = x_0 + sum_s a_s cos(2 pi r s / R) -/+ i sum_s b_s sin(2 pi r s / R),
    //   y_{R-r} the same with the sine term's sign flipped.
    constexpr int H = (R - 1) / 2;
    double2 a[H], b[H];
    double2 y0 = v[0];
#pragma unroll
    for (int s = 1; s <= H; ++s) {
      a[s - 1] = cadd(v[s], v[R - s]);
      b[s - 1] = csub(v[s], v[R - s]);
      y0 = cadd(y0, a[s - 1]);
    }
    double2 out[R];
    out[0] = y0;
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      double2 A = v[0], B = make_double2(0.0, 0.0);
#pragma unroll
      for (int s = 1; s <= H; ++s) {
        const int k = (r * s) % R;
        const double c = dft_cos(R, k <= H ? k : R - k);
        const double sn = k <= H ? dft_sin(R, k) : -dft_sin(R, R - k);
        A.x = fma(a[s - 1].x, c, A.x);
        A.y = fma(a[s - 1].y, c, A.y);
        B.x = fma(b[s - 1].x, sn, B.x);
        B.y = fma(b[s - 1].y, sn, B.y);
      }
      const double2 miB = make_double2(B.y, -B.x);  // -i B
      out[r] = inv ? csub(A, miB) : cadd(A, miB);
      out[R - r] = inv ? cadd(A, miB) : csub(A, miB);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = out[r];
  }
}

// One radix-R Stockham stage on x[0..n): butterfly j (k = j mod Ns) reads
// x[j + r n/R], twiddles by omega_n^{r k span} (span = n / (Ns R); powers
// of omega^{k span} by repeated multiplication), and writes x[(j / Ns) Ns R
// + k + r Ns].  Every thread keeps its butterflies in registers across the
// barrier, so the stage works in place.
template <int R, int NT, int MAXN>
__device__ void stage(double2* x, int n, int Ns, unsigned nsm, const TwCtx& C, bool inv) {
  constexpr int MAXIT = (MAXN / R + NT - 1) / NT;
  const int nb = (int)((unsigned)n / (unsigned)R);
  const FastDiv dv((unsigned)Ns, nsm);
  const int span = (int)dv.div((unsigned)nb);  // nb Ns <= n: exact
  const int tid = threadIdx.x;
  double2 v[MAXIT][R];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int j = tid + NT * it;
    if (j < nb) {
      const int k = (int)dv.mod((unsigned)j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = x[j + r * nb];
      if (k != 0) {
        const double2 w1 = C.tw(k * span, inv);
        double2 w = w1;
        v[it][1] = cmul(v[it][1], w);
#pragma unroll
        for (int r = 2; r < R; ++r) {
          w = cmul(w, w1);
          v[it][r] = cmul(v[it][r], w);
        }
      }
      small_dft<R>(v[it], inv);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int j = tid + NT * it;
    if (j < nb) {
      const int q = (int)dv.div((unsigned)j);
      const int idx = q * Ns * R + (j - q * Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) x[idx + r * Ns] = v[it][r];
    }
  }
  __syncthreads();
}

// Radix of stage s of a power-of-two length 2^e, in the order the host's
// factorization gives (radix 8 first, 2^4 as 4 x 4, a remaining 2^2 as 4,
// a remaining 2 last); 0 past the last stage.
__host__ __device__ constexpr int pow2_radix(int e, int s) {
  int n8 = e / 3, rest = e % 3;
  if (rest == 1 && n8 > 0) {
    --n8;
    rest = 4;
  }
  if (s < n8) return 8;
  s -= n8;
  if (rest == 4) return s < 2 ? 4 : 0;
  if (rest == 2) return s == 0 ? 4 : 0;
  if (rest == 1) return s == 0 ? 2 : 0;
  return 0;
}
__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
static_assert(pow2_radix(9, 0) == 8 && pow2_radix(9, 2) == 8 && pow2_radix(9, 3) == 0, "512 = 8 8 8");
static_assert(pow2_radix(8, 1) == 8 && pow2_radix(8, 2) == 4 && pow2_radix(8, 3) == 0, "256 = 8 8 4");
static_assert(pow2_radix(10, 1) == 8 && pow2_radix(10, 2) == 4 && pow2_radix(10, 3) == 4 &&
                  pow2_radix(10, 4) == 0, "1024 = 8 8 4 4");
static_assert(pow2_radix(11, 2) == 8 && pow2_radix(11, 3) == 4 && pow2_radix(11, 4) == 0, "2048 = 8 8 8 4");
static_assert(pow2_radix(13, 3) == 4 && pow2_radix(13, 4) == 4 && pow2_radix(13, 5) == 0, "8192 = 8 8 8 4 4");
static_assert(pow2_radix(1, 0) == 2 && pow2_radix(1, 1) == 0, "2");

// The stages of a power-of-two length N with every length, stride and
// divisor fixed at compile time (the same stages and arithmetic as the
// general loop below, without its per-stage scalar work).
template <int NT, int MAXN, int N, int S = 0, int NS = 1>
__device__ __forceinline__ void fft_fixed(double2* x, const TwCtx& C, bool inv) {
  constexpr int R = pow2_radix(ilog2(N), S);
  if constexpr (R > 0) {
    constexpr unsigned m = NS <= 1 ? 0u : 0xFFFFFFFFu / NS + 1u;
    stage<R, NT, MAXN>(x, N, NS, m, C, inv);
    fft_fixed<NT, MAXN, N, S + 1, NS * R>(x, C, inv);
  }
}

// In-place DFT of x[0..n) in LDS: forward exp(-2 pi i jk/n), inverse exp(+).
// POW2: the length is a power of two (radix 8, 4 and 2 only).  HALF: length
// MAXN / 2 gets its fixed stages too (where that does not cost registers).
template <int NT, int MAXN, bool POW2, bool HALF>
__device__ void fft_lds(double2* x, int n, const int* __restrict__ fac, const unsigned* __restrict__ facm,
                        int nfac, const TwCtx& C, bool inv) {
  if (n == MAXN) {  // the tier's longest length: the Bluestein convolutions and the widest rings
    fft_fixed<NT, MAXN, MAXN>(x, C, inv);
    return;
  }
  // half of it: the belt rings of a HEALPix grid whose largest length sits in
  // the tier
  if constexpr (HALF) {
    if (n == MAXN / 2) {
      fft_fixed<NT, MAXN, MAXN / 2>(x, C, inv);
      return;
    }
  }
  int Ns = 1;
  for (int st = 0; st < nfac; ++st) {
    const int R = fac[st];
    const unsigned m = facm[st];
    if (R == 8) {
      stage<8, NT, MAXN>(x, n, Ns, m, C, inv);
    } else if (R == 4) {
      stage<4, NT, MAXN>(x, n, Ns, m, C, inv);
    } else if (R == 2) {
      stage<2, NT, MAXN>(x, n, Ns, m, C, inv);
    } else if constexpr (!POW2) {
      if (R == 3) stage<3, NT, MAXN>(x, n, Ns, m, C, inv);
      else if (R == 5) stage<5, NT, MAXN>(x, n, Ns, m, C, inv);
      else if (R == 7) stage<7, NT, MAXN>(x, n, Ns, m, C, inv);
    }
    Ns *= R;
  }
}

// DFT of length n0 through Bluestein's identity:
//   X_k = w_k sum_n (x_n w_n) b_{k-n},  w_n = exp(-i pi n^2 / n0), b_d = conj(w_d),
// a cyclic convolution of length M (x holds M words).  The inverse DFT is
// conj(DFT(conj x)).  bf holds the filter spectrum (M words) followed by the
// chirp w_n (n0 words), both precomputed on the host.
template <int NT, int MAXN>
__device__ void dft_bluestein(double2* x, int n0, int M, const double2* __restrict__ bf,
                              const TwCtx& C, const int* __restrict__ fac, const unsigned* __restrict__ facm,
                              int nfac, bool inv) {
  const int tid = threadIdx.x;
  const double2* __restrict__ w = bf + M;
  for (int i = tid; i < M; i += NT) {
    double2 v = make_double2(0.0, 0.0);
    if (i < n0) {
      const double2 a = x[i];
      v = cmul(inv ? conj2(a) : a, w[i]);
    }
    x[i] = v;
  }
  __syncthreads();
  fft_lds<NT, MAXN, true, (MAXN <= 1024)>(x, M, fac, facm, nfac, C, false);
  for (int i = tid; i < M; i += NT) x[i] = cmul(x[i], bf[i]);
  __syncthreads();
  fft_lds<NT, MAXN, true, (MAXN <= 1024)>(x, M, fac, facm, nfac, C, true);
  for (int i = tid; i < n0; i += NT) {
    const double2 v = cmul(x[i], w[i]);
    x[i] = inv ? conj2(v) : v;
  }
  __syncthreads();
}

// Sum of g_m = (F^c_m - i F^s_m) e^{i m phi0} over m = m0, m0 + S, ... <= L,
// e^{i m phi0} = conj(T[t_m]) with t_m = m num mod 2N stepping by tS; four
// loads in flight per step, summed in order of m.
template <class Tw>
__device__ __forceinline__ double2 sum_g(const double2* __restrict__ ph, int m0, int S, int L, int t,
                                         int tS, int twoN, const Tw& ring) {
  double2 acc = make_double2(0.0, 0.0);
  int m = m0;
  auto add = [&](double2 F) {
    acc = cadd(acc, cmulc(make_double2(F.x, -F.y), ring.at(t)));
    t += tS;
    if (t >= twoN) t -= twoN;
  };
  for (; m + 3 * S <= L; m += 4 * S) {
    const double2 F0 = ph[m], F1 = ph[m + S], F2 = ph[m + 2 * S], F3 = ph[m + 3 * S];
    add(F0);
    add(F1);
    add(F2);
    add(F3);
  }
  for (; m <= L; m += S) add(ph[m]);
  return acc;
}

// Folded spectrum c_k = (G_k + conj G_{-k}) / 2 with G_k the sum of g_m over
// m = k mod N (0 <= k < N).
template <class Tw>
__device__ __forceinline__ double2 fold(const double2* __restrict__ ph, int k, int N, int L, int num,
                                        const FastDiv& d2N, int stepN, const Tw& ring) {
  const double2 a = sum_g(ph, k, N, L, (int)d2N.mod((unsigned)k * (unsigned)num), stepN, 2 * N, ring);
  const int m1 = k == 0 ? 0 : N - k;
  const double2 b = sum_g(ph, m1, N, L, (int)d2N.mod((unsigned)m1 * (unsigned)num), stepN, 2 * N, ring);
  return make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
}

// ODD: the class has FFT lengths with radices 3, 5 or 7 (without it only the
// power-of-two stages are compiled, which takes far fewer registers).
template <int NT, int MAXN, bool ODD>
__global__ __launch_bounds__(NT) void k_ring(RingArgs a, int mode, double2* __restrict__ phase,
                                             int64_t pstride, const double* __restrict__ map_in,
                                             double* __restrict__ map_out, int64_t mstride,
                                             const double* const* __restrict__ weights,
                                             int maps_per_weight) {
  extern __shared__ double2 lds[];
  double2* x = lds;
  double2* wf = lds + a.xcap;
  double2* wc = wf + 64;
  double2* wf2 = wc + (2 * a.maxn + 63) / 64;
  double2* wc2 = wf2 + 64;
  double2* G = a.any_blue ? wc2 + kBlueMax / 64 : wf2;  // fold scratch (rings with N <= NT)
  const int r = a.rings[blockIdx.x];
  const int map = blockIdx.y;
  if (a.skip.off(map)) return;  // whole block: before any barrier
  const int tid = threadIdx.x;
  const int L = a.lmax;
  const int N = a.nphi[r];
  const bool half = (N & 1) == 0;     // two real samples per complex word
  const bool blue = a.bfoff[r] >= 0;  // Bluestein convolution
  const int n0 = half ? N / 2 : N;
  const int nf = a.fftn[r];
  const int64_t off = a.offset[r];
  const int num = a.phinum[r];
  const double2* __restrict__ Tg = a.tw + a.twoff[r];
  const int* __restrict__ fac = a.fac + (size_t)r * kMaxFactors;
  const unsigned* __restrict__ facm = a.facm + (size_t)r * kMaxFactors;
  const int nfac = a.nfac[r];
  double2* __restrict__ ph = phase + (int64_t)map * pstride + (int64_t)r * (L + 1);
  const int twoN = 2 * N;
  for (int i = tid; i < 64; i += NT) wf[i] = Tg[i < twoN ? i : 0];
  for (int u = tid; u * 64 < twoN; u += NT) wc[u] = Tg[64 * u];
  if (blue) {
    for (int i = tid; i < 64; i += NT) wf2[i] = a.tw2[i];
    for (int u = tid; u < kBlueMax / 64; u += NT) wc2[u] = a.tw2[64 * u];
  }
  // No barrier here: the LDS tables are first read after the barrier that
  // follows the fold (synthesis) or the input load (adjoint), so the table
  // copy and those global loads are in flight together.
  const TwCtx ring{wf, wc, 1};
  const GlobalTw gring{Tg};
  // the FFT of length n0 (direct) or nf (Bluestein)
  const TwCtx fc = blue ? TwCtx{wf2, wc2, (int)((unsigned)kBlueMax / (unsigned)nf)} : TwCtx{wf, wc, half ? 4 : 2};
  const double2* __restrict__ bf = blue ? a.bf + a.bfoff[r] : nullptr;
  const FastDiv d2N((unsigned)twoN), dN((unsigned)N);
  double* xd = reinterpret_cast<double*>(x);

  // Wide even rings (N >= 2L, every HEALPix belt ring at L <= 2 Nside): each
  // m <= L has its own bin (m = N / 2 = L shares the Nyquist bin with -m), so
  // the fold and the unfold take one phase value per bin and the factors
  // e^{-i pi t / N} straight from the ring's global table, t = m num < 2N
  // (phi0 = pi num / N with num 0 or 1 on every grid built here).
  const bool wide = half && 2 * L <= N;
  auto gval = [&](int m) -> double2 {  // g_m = (F^c_m - i F^s_m) e^{i m phi0}
    const double2 F = ph[m];
    const double2 Fc = make_double2(F.x, -F.y);
    return num ? cmulc(Fc, gring.at(m)) : Fc;
  };
  if (mode == RING_SYNTH || mode == RING_ROUNDTRIP) {
    const int stepN = (int)d2N.mod((unsigned)N * (unsigned)num);
    if (N <= NT && !wide) {
      // short ring: all threads fold.  Thread p < S (S = N floor(NT / N))
      // sums g_m over m = p mod S; G_k then adds the S / N partials of bin k.
      const int S = N * (NT / N);
      double2* P = G + N;
      if (tid < S)
        P[tid] = sum_g(ph, tid, S, L, (int)d2N.mod((unsigned)tid * (unsigned)num),
                       (int)d2N.mod((unsigned)S * (unsigned)num), twoN, gring);
      __syncthreads();
      for (int k = tid; k < N; k += NT) {
        double2 acc = P[k];
        for (int j = k + N; j < S; j += N) acc = cadd(acc, P[j]);
        G[k] = acc;
      }
      __syncthreads();
    }
    auto cfold = [&](int k) -> double2 {
      if (N <= NT) {
        const double2 u = G[k], v = G[k == 0 ? 0 : N - k];
        return make_double2(0.5 * (u.x + v.x), 0.5 * (u.y - v.y));
      }
      return fold(ph, k, N, L, num, d2N, stepN, gring);
    };
    for (int k = tid; k < n0; k += NT) {
      if (wide) {
        // c_0 = Re g_0, c_k = g_k / 2 (0 < k < H), c_{k+H} = conj(g_{H-k}) / 2
        // (0 < k), c_H = Re g_H (H <= L only when N = 2L)
        double2 ck = k <= L ? gval(k) : make_double2(0.0, 0.0);
        double2 ch = n0 - k <= L ? gval(n0 - k) : make_double2(0.0, 0.0);
        if (k == 0) {
          ck.y = 0.0;
          ch.y = 0.0;
        } else {
          ck = make_double2(0.5 * ck.x, 0.5 * ck.y);
          ch = make_double2(0.5 * ch.x, -0.5 * ch.y);
        }
        const double2 e = conj2(gring.at(2 * k));
        const double2 dd = cmul(e, csub(ck, ch));
        x[k] = make_double2(ck.x + ch.x - dd.y, ck.y + ch.y + dd.x);
      } else if (half) {
        const double2 ck = cfold(k);
        const double2 ch = cfold(k + n0);
        // Z_k = (c_k + c_{k+H}) + i e^{+2 pi i k / N} (c_k - c_{k+H})
        const double2 e = conj2(gring.at(2 * k));
        const double2 dd = cmul(e, csub(ck, ch));
        x[k] = make_double2(ck.x + ch.x - dd.y, ck.y + ch.y + dd.x);
      } else {
        x[k] = cfold(k);
      }
    }
    __syncthreads();
    if (blue)
      dft_bluestein<NT, MAXN>(x, n0, nf, bf, fc, fac, facm, nfac, true);
    else
      fft_lds<NT, MAXN, !ODD, (!ODD || MAXN <= 1024)>(x, n0, fac, facm, nfac, fc, true);
    if (mode == RING_SYNTH) {
      double* out = map_out + (int64_t)map * mstride + off;
      if (half) {
        for (int j = tid; j < N; j += NT) out[j] = xd[j];
      } else {
        for (int j = tid; j < N; j += NT) out[j] = x[j].x;
      }
      return;
    }
    const double* __restrict__ w = weights[map / maps_per_weight] + off;
    if (half) {
      for (int j = tid; j < N; j += NT) xd[j] *= w[j];
    } else {
      for (int j = tid; j < N; j += NT) x[j] = make_double2(x[j].x * w[j], 0.0);
    }
    __syncthreads();
  } else {
    const double* in = map_in + (int64_t)map * mstride + off;
    if (half) {
      for (int j = tid; j < N; j += NT) xd[j] = in[j];
    } else {
      for (int j = tid; j < N; j += NT) x[j] = make_double2(in[j], 0.0);
    }
    __syncthreads();
  }
  if (blue)
    dft_bluestein<NT, MAXN>(x, n0, nf, bf, fc, fac, facm, nfac, false);
  else
    fft_lds<NT, MAXN, !ODD, (!ODD || MAXN <= 1024)>(x, n0, fac, facm, nfac, fc, false);

  // forward DFT of the real ring data at bin k (0 <= k < N)
  auto spec = [&](int k) -> double2 {
    if (half) {
      const int kk = k >= n0 ? k - n0 : k;
      const int k2 = kk == 0 ? 0 : n0 - kk;
      const double2 Zk = x[kk], Zc = conj2(x[k2]);
      const double2 E = make_double2(0.5 * (Zk.x + Zc.x), 0.5 * (Zk.y + Zc.y));
      const double2 D = csub(Zk, Zc);
      const double2 O = make_double2(0.5 * D.y, -0.5 * D.x);  // D / (2i)
      return cadd(E, cmul(ring.at(2 * k), O));
    } else {
      return x[k];
    }
  };
  if (mode == RING_DIAG) {
    const double t0 = spec(0).x;
    for (int m = tid; m <= L; m += NT) {
      if (m == 0) {
        ph[0] = make_double2(t0, 0.0);
      } else {
        const unsigned m2 = d2N.mod(2u * (unsigned)m);
        const int k = (int)dN.mod(m2);
        const double2 X = cmul(spec(k), ring.at((int)d2N.mod(m2 * (unsigned)num)));
        ph[m] = make_double2(t0 + X.x, t0 - X.x);
      }
    }
    return;
  }
  if (wide) {
    for (int m = tid; m <= L; m += NT) {
      // F^_m from Z_m and Z_{H-m} (m = H only when N = 2L: bin 0's partner)
      const int kk = m < n0 ? m : m - n0;
      const int k2 = kk == 0 ? 0 : n0 - kk;
      const double2 Zk = x[kk], Zc = conj2(x[k2]);
      const double2 E = make_double2(0.5 * (Zk.x + Zc.x), 0.5 * (Zk.y + Zc.y));
      const double2 D = csub(Zk, Zc);
      const double2 O = make_double2(0.5 * D.y, -0.5 * D.x);
      double2 h = cadd(E, cmul(gring.at(2 * m), O));
      if (num) h = cmul(h, gring.at(m));
      ph[m] = make_double2(h.x, m == 0 ? 0.0 : -h.y);
    }
    return;
  }
  for (int m = tid; m <= L; m += NT) {
    // H_m = e^{-i m phi0} F^_{m mod N};  e^{-i m phi0} = T[m num mod 2N]
    const unsigned mm = d2N.mod((unsigned)m);
    const double2 h = cmul(spec((int)dN.mod(mm)), ring.at((int)d2N.mod(mm * (unsigned)num)));
    ph[m] = make_double2(h.x, m == 0 ? 0.0 : -h.y);
  }
}

}  // namespace

RingArgs ring_args(crs_grid g, int lmax);

void launch_ring(crs_grid g, int lmax, RingMode mode, int nmaps, double2* phase, int64_t pstride,
                 const double* map_in, double* map_out, int64_t mstride,
                 const double* const* weights, int maps_per_weight, hipStream_t s, MapSkip skip) {
  CRS_CHECK(lmax < 65536, CRS_EUNSUPPORTED, "lmax above 65535 is not supported by the ring stage");
  RingArgs base = ring_args(g, lmax);
  base.skip = skip;
  const int mpw = maps_per_weight < 1 ? 1 : maps_per_weight;
  const int md = (int)mode;
  auto launch_class = [&](const RingClass& rc, const int* rings) {
    if (rc.rings.empty()) return;
    RingArgs a = base;
    a.maxn = rc.maxn;
    a.xcap = rc.xcap;
    a.rings = rings;
    const dim3 grid((unsigned)rc.rings.size(), nmaps);
    const size_t words = (size_t)rc.xcap + 64 + (2 * rc.maxn + 63) / 64 +
                         (rc.blue ? 64 + kBlueMax / 64 : 0) + rc.gcap;
    a.any_blue = rc.blue ? 1 : 0;
    const size_t lds = words * sizeof(double2);
    CRS_CHECK(lds <= kMaxLds, CRS_EUNSUPPORTED, "ring class needs " + std::to_string(lds) + " bytes of LDS");
    switch (rc.tier * 2 + (rc.odd ? 1 : 0)) {
#define CRS_RING(T, NT, MAXN, ODD)                                                                   \
  case T * 2 + ODD:                                                                                  \
    hipLaunchKernelGGL((k_ring<NT, MAXN, ODD>), grid, dim3(NT), lds, s, a, md, phase, pstride,       \
                       map_in, map_out, mstride, weights, mpw);                                      \
    break;
      CRS_RING(0, 128, 512, false)
      CRS_RING(0, 128, 512, true)
      CRS_RING(1, 256, 1024, false)
      CRS_RING(1, 256, 1024, true)
      CRS_RING(2, 512, 4096, false)
      CRS_RING(2, 512, 4096, true)
      CRS_RING(3, 1024, 8192, false)
      CRS_RING(3, 1024, 8192, true)
#undef CRS_RING
      default: throw Error{CRS_EUNSUPPORTED, "ring FFT length above 8192"};
    }
    CRS_HIP(hipGetLastError());
  };
  // Launches on a stream run one after another, so a class of a few hundred
  // blocks would leave most CUs idle for a whole block's duration: the
  // classes with fewer than kMinClassBlocks blocks (the first `nsmall` in
  // order of ring count) run together as one launch, the others on their own.
  constexpr int64_t kMinClassBlocks = 1024;
  const int ncls = (int)g->ring_classes.size();
  int nsmall = 0;
  while (nsmall < ncls &&
         (int64_t)g->ring_classes[g->ring_small_order[nsmall]].rings.size() * nmaps < kMinClassBlocks)
    ++nsmall;
  bool small[kMaxRingClasses] = {};
  for (int k = 0; k < nsmall; ++k) small[g->ring_small_order[k]] = true;
  for (int c = 0; c < ncls; ++c)
    if (!small[c]) launch_class(g->ring_classes[c], g->d_ring_class[c].p);
  if (nsmall > 0) launch_class(g->ring_prefix[nsmall - 1], g->d_ring_prefix[nsmall - 1].p);
}

}  // namespace crs
