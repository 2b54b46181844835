// Ring stage of the spherical harmonic transforms: per-ring FFTs in LDS.
//
// Synthesis, second half of Y (Sect. 2.1): on ring r with Nphi pixels at
// phi_j = phi0 + 2 pi j / Nphi,
//     f_j = Re sum_{m=0..L} (F^c_m - i F^s_m) e^{i m phi_j}.
// The m sum is folded onto Nphi bins (m -> m mod Nphi, conjugate partner
// -m) so that f = inverse DFT of a Hermitian spectrum; rings with
// Nphi < 2L+1 alias exactly as the dense operator does.
// Adjoint, first half of Y^T (Sect. 3.2): H_m = e^{-i m phi0} F^_{m mod Nphi},
// F^_k = sum_j f_j e^{-2 pi i j k / Nphi}, H^c = Re H, H^s = -Im H.
// Round trip (inside A and T^+): synthesis, multiply by a pixel weight
// (tau for A, alpha^2 w^2 tau^+ for T^+; Sect. 2.3 eq:A and Sect. 3.3),
// adjoint -- the map never leaves LDS.
// Diagonal setup (M_diag, Sect. 5): for a pixel map t, G^c_m = T^_0 +
// Re(e^{-2 i m phi0} T^_{2m}), G^s_m = T^_0 - Re(...), G_0 = (T^_0, 0):
// sum_j t_j cos^2(m phi_j) = (G^c_m)/2 etc.
//
// FFT: mixed-radix Stockham autosort (radix 4, 2, 3, 5, 7 butterflies and a
// direct stage for larger primes), one block of 256 (Nphi <= 2048) or 512
// threads per ring and map, data resident in LDS (Nphi <= 4096).  Twiddles come from per-length
// tables T[t] = exp(-i pi t / Nphi), t < 2 Nphi; phi0 is 0 or pi / Nphi.
#include "internal.h"

namespace crs {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Twiddles of one ring from two small LDS tables: omega_2N^t = Wc[t >> 6] Wf[t & 63]
// with Wf[i] = exp(-i pi i / N) (i < 64) and Wc[u] = exp(-i pi 64 u / N), both
// copied from the ring's global table at kernel start (exact entries; the
// product adds at most one rounding).
struct Tw {
  const double2* Wf;
  const double2* Wc;
  __device__ __forceinline__ double2 get2(int t2) const { return cmul(Wc[t2 >> 6], Wf[t2 & 63]); }
};
// omega_N^t = exp(-2 pi i t / N) (forward) or its conjugate (inverse)
__device__ __forceinline__ double2 tw_get(const Tw& T, int t, bool inv) {
  const double2 w = T.get2(2 * t);
  return inv ? make_double2(w.x, -w.y) : w;
}

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
    double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    double2 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    // forward: y1 = t1 - i t3, y3 = t1 + i t3 ; inverse swaps
    double2 mit3 = make_double2(t3.y, -t3.x);  // -i * t3
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    if (!inv) {
      v[1] = cadd(t1, mit3);
      v[3] = csub(t1, mit3);
    } else {
      v[1] = csub(t1, mit3);
      v[3] = cadd(t1, mit3);
    }
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

template <int R, int NT, int MAXN>
__device__ void stage_small(double2* x, int N, int Ns, const Tw& T, bool inv) {
  constexpr int MAXIT = (MAXN / R + NT - 1) / NT;
  const int nb = N / R;
  const int tid = threadIdx.x;
  double2 v[MAXIT][R];
  const int span = N / (Ns * R);
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int j = tid + NT * it;
    if (j < nb) {
      const int k = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double2 a = x[j + r * nb];
        v[it][r] = (r == 0 || k == 0) ? a : cmul(a, tw_get(T, r * k * span, inv));
      }
      small_dft<R>(v[it], inv);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int j = tid + NT * it;
    if (j < nb) {
      const int k = j % Ns;
      const int idx = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) x[idx + r * Ns] = v[it][r];
    }
  }
  __syncthreads();
}

// Radix-R stage for a prime R > 7: twiddle the inputs in place, then every
// butterfly is a plain length-R DFT computed output pair by output pair
// (r, R-r) from a_s = x_s + x_{R-s}, b_s = x_s - x_{R-s}:
//   y_r = x_0 + sum_s a_s cos(2 pi r s / R) -/+ i sum_s b_s sin(2 pi r s / R).
// The omega_R^{r s} factors are stepped by complex multiplication and re-read
// from the LDS table every 16 steps to bound rounding growth.
template <int NT, int MAXN>
__device__ void stage_generic(double2* x, double2* wp, int N, int Ns, int R, const Tw& T, bool inv) {
  constexpr int RB = 4;
  // items nb * ceil((h+1)/RB) <= 0.23 N for R >= 11
  constexpr int MAXIT = (MAXN / 4 + NT - 1) / NT;
  const int nb = N / R;
  const int NsR = Ns * R;
  const int span = N / NsR;
  const int tid = threadIdx.x;
  const int h = (R - 1) / 2;
  // (a) input twiddles  x[j + s nb] *= w_N^{s k span},  k = j mod Ns
  for (int e = tid; e < N; e += NT) {
    const int j = e % nb, s = e / nb, k = j % Ns;
    const int t = s * k * span;
    if (t) x[e] = cmul(x[e], tw_get(T, t, inv));
  }
  // (b) forward table omega_R^t = exp(-2 pi i t / R)
  for (int t = tid; t < R; t += NT) wp[t] = T.get2(2 * t * (N / R));
  __syncthreads();
  // (c) a_s, b_s in place
  for (int e = tid; e < nb * h; e += NT) {
    const int j = e % nb, s = 1 + e / nb;
    const double2 u = x[j + s * nb], v = x[j + (R - s) * nb];
    x[j + s * nb] = cadd(u, v);
    x[j + (R - s) * nb] = csub(u, v);
  }
  __syncthreads();
  // (d) output pairs
  const int nrb = (h + 1 + RB - 1) / RB;
  const int items = nb * nrb;
  double2 out0[MAXIT][RB], out1[MAXIT][RB];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int q = tid + NT * it;
    if (q >= items) break;
    const int j = q % nb, r0 = (q / nb) * RB;
    const double2 x0 = x[j];
    double2 A[RB], B[RB], w[RB], st[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      A[i] = make_double2(0.0, 0.0);
      B[i] = make_double2(0.0, 0.0);
      const int r = min(r0 + i, h);
      st[i] = wp[r];  // omega^r (forward)
      w[i] = st[i];   // omega^{r s} at s = 1
    }
    for (int s = 1; s <= h; ++s) {
      const double2 as = x[j + s * nb], bs = x[j + (R - s) * nb];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        // forward omega^{rs} = c - i sn
        const double c = w[i].x, sn = -w[i].y;
        A[i].x = fma(as.x, c, A[i].x);
        A[i].y = fma(as.y, c, A[i].y);
        B[i].x = fma(bs.x, sn, B[i].x);
        B[i].y = fma(bs.y, sn, B[i].y);
        if ((s & 15) == 15) {
          const int r = min(r0 + i, h);
          w[i] = wp[(int)(((long)r * (s + 1)) % R)];
        } else {
          w[i] = cmul(w[i], st[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      // forward: y_r = x0 + A - i B ; y_{R-r} = x0 + A + i B (inverse swaps)
      const double2 miB = make_double2(B[i].y, -B[i].x);
      const double2 base = cadd(x0, A[i]);
      out0[it][i] = inv ? csub(base, miB) : cadd(base, miB);
      out1[it][i] = inv ? cadd(base, miB) : csub(base, miB);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int q = tid + NT * it;
    if (q >= items) break;
    const int j = q % nb, r0 = (q / nb) * RB;
    const int k = j % Ns;
    const int idx = (j / Ns) * NsR + k;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int r = r0 + i;
      if (r > h) break;
      x[idx + r * Ns] = out0[it][i];
      if (r > 0) x[idx + (R - r) * Ns] = out1[it][i];
    }
  }
  __syncthreads();
}

// In-place DFT of x[0..N) in LDS: forward exp(-2 pi i jk/N), inverse exp(+).
template <int NT, int MAXN, bool GEN>
__device__ void fft_lds(double2* x, double2* wp, int N, const int* __restrict__ fac, int nfac,
                        const Tw& T, bool inv) {
  int Ns = 1;
  for (int st = 0; st < nfac; ++st) {
    const int R = fac[st];
    switch (R) {
      case 1: break;
      case 2: stage_small<2, NT, MAXN>(x, N, Ns, T, inv); break;
      case 3: stage_small<3, NT, MAXN>(x, N, Ns, T, inv); break;
      case 4: stage_small<4, NT, MAXN>(x, N, Ns, T, inv); break;
      case 5: stage_small<5, NT, MAXN>(x, N, Ns, T, inv); break;
      case 7: stage_small<7, NT, MAXN>(x, N, Ns, T, inv); break;
      default:
        if constexpr (GEN) stage_generic<NT, MAXN>(x, wp, N, Ns, R, T, inv);
        break;
    }
    Ns *= R;
  }
}

template <int NT, int MAXN, bool GEN>
__global__ __launch_bounds__(NT) void k_ring(RingArgs a, int mode, int nmaps, double2* __restrict__ phase,
                                              int64_t pstride, const double* __restrict__ map_in,
                                              double* __restrict__ map_out, int64_t mstride,
                                              const double* const* __restrict__ weights,
                                              int maps_per_weight) {
  extern __shared__ double2 lds[];
  double2* x = lds;
  double2* wp = lds + a.maxn;
  double2* wf = wp + a.maxp;
  double2* wc = wf + 64;
  const int r = a.rings[blockIdx.x];
  const int map = blockIdx.y;
  const int tid = threadIdx.x;
  const int L = a.lmax;
  const int N = a.nphi[r];
  const int64_t off = a.offset[r];
  const int num = a.phinum[r];
  const double2* __restrict__ Tg = a.tw + a.twoff[r];
  const int* __restrict__ fac = a.fac + (size_t)r * kMaxFactors;
  const int nfac = a.nfac[r];
  double2* __restrict__ ph = phase + (int64_t)map * pstride + (int64_t)r * (L + 1);
  const int twoN = 2 * N;
  for (int i = tid; i < 64; i += NT) wf[i] = Tg[i < twoN ? i : 0];
  for (int u = tid; u * 64 < twoN; u += NT) wc[u] = Tg[64 * u];
  __syncthreads();
  const Tw T{wf, wc};

  if (mode == RING_SYNTH || mode == RING_ROUNDTRIP) {
    // fold the Hermitian spectrum: c_k = (sum_{m=k mod N} g_m + sum_{m=-k mod N} conj g_m) / 2
    // phase index of e^{-i m phi0} in the 2N table: t(m) = m num mod 2N; stepping
    // m by N adds N num mod 2N
    const int stepN = (int)(((unsigned)N * (unsigned)num) % (unsigned)twoN);
    for (int k = tid; k < N; k += NT) {
      double2 acc = make_double2(0.0, 0.0);
      int t = (int)(((unsigned)k * (unsigned)num) % (unsigned)twoN);
      for (int m = k; m <= L; m += N) {
        const double2 F = ph[m];
        // g_m = (F^c - i F^s) e^{+i m phi0}, e^{+i m phi0} = conj(T[t])
        acc = cadd(acc, cmulc(make_double2(F.x, -F.y), T.get2(t)));
        t += stepN;
        if (t >= twoN) t -= twoN;
      }
      const int m1 = (N - k) % N;
      t = (int)(((unsigned)m1 * (unsigned)num) % (unsigned)twoN);
      for (int m = m1; m <= L; m += N) {
        const double2 F = ph[m];
        const double2 g = cmulc(make_double2(F.x, -F.y), T.get2(t));
        acc = cadd(acc, make_double2(g.x, -g.y));
        t += stepN;
        if (t >= twoN) t -= twoN;
      }
      x[k] = make_double2(0.5 * acc.x, 0.5 * acc.y);
    }
    __syncthreads();
    fft_lds<NT, MAXN, GEN>(x, wp, N, fac, nfac, T, /*inv=*/true);
    if (mode == RING_SYNTH) {
      double* out = map_out + (int64_t)map * mstride + off;
      for (int j = tid; j < N; j += NT) out[j] = x[j].x;
      return;
    }
    const double* __restrict__ w = weights[map / maps_per_weight] + off;
    for (int j = tid; j < N; j += NT) x[j] = make_double2(x[j].x * w[j], 0.0);
    __syncthreads();
  } else {
    const double* in = map_in + (int64_t)map * mstride + off;
    for (int j = tid; j < N; j += NT) x[j] = make_double2(in[j], 0.0);
    __syncthreads();
  }
  fft_lds<NT, MAXN, GEN>(x, wp, N, fac, nfac, T, /*inv=*/false);
  if (mode == RING_DIAG) {
    const double t0 = x[0].x;
    for (int m = tid; m <= L; m += NT) {
      if (m == 0) {
        ph[0] = make_double2(t0, 0.0);
      } else {
        const unsigned m2 = (2u * (unsigned)m) % (unsigned)twoN;
        const int k = (int)(m2 % (unsigned)N);
        const double2 X = cmul(x[k], T.get2((int)((m2 * (unsigned)num) % (unsigned)twoN)));
        ph[m] = make_double2(t0 + X.x, t0 - X.x);
      }
    }
    return;
  }
  for (int m = tid; m <= L; m += NT) {
    const double2 F = x[m % N];
    // H_m = e^{-i m phi0} F^_{m mod N};  e^{-i m phi0} = T[m num mod 2N]
    const unsigned mm = (unsigned)m % (unsigned)twoN;
    const double2 h = cmul(F, T.get2((int)((mm * (unsigned)num) % (unsigned)twoN)));
    ph[m] = make_double2(h.x, m == 0 ? 0.0 : -h.y);
  }
}

}  // namespace

RingArgs ring_args(crs_grid g, int lmax);

void launch_ring(crs_grid g, int lmax, RingMode mode, int nmaps, double2* phase, int64_t pstride,
                 const double* map_in, double* map_out, int64_t mstride,
                 const double* const* weights, int maps_per_weight, hipStream_t s) {
  const RingArgs base = ring_args(g, lmax);
  for (size_t c = 0; c < g->ring_classes.size(); ++c) {
    const RingClass& rc = g->ring_classes[c];
    if (rc.rings.empty()) continue;
    RingArgs a = base;
    a.maxn = rc.maxn;
    a.maxp = rc.maxp;
    a.rings = g->d_ring_class[c].p;
    dim3 grid((unsigned)rc.rings.size(), nmaps);
    const size_t lds = (size_t)(a.maxn + a.maxp + 64 + (2 * a.maxn + 63) / 64) * sizeof(double2);
    const int mpw = maps_per_weight < 1 ? 1 : maps_per_weight;
    const bool gen = rc.maxp > 0;
    if (a.maxn > 2048) {
      if (gen)
        hipLaunchKernelGGL((k_ring<512, 4096, true>), grid, dim3(512), lds, s, a, (int)mode, nmaps, phase,
                           pstride, map_in, map_out, mstride, weights, mpw);
      else
        hipLaunchKernelGGL((k_ring<512, 4096, false>), grid, dim3(512), lds, s, a, (int)mode, nmaps, phase,
                           pstride, map_in, map_out, mstride, weights, mpw);
    } else {
      if (gen)
        hipLaunchKernelGGL((k_ring<256, 2048, true>), grid, dim3(256), lds, s, a, (int)mode, nmaps, phase,
                           pstride, map_in, map_out, mstride, weights, mpw);
      else
        hipLaunchKernelGGL((k_ring<256, 2048, false>), grid, dim3(256), lds, s, a, (int)mode, nmaps, phase,
                           pstride, map_in, map_out, mstride, weights, mpw);
    }
    CRS_HIP(hipGetLastError());
  }
}

}  // namespace crs
