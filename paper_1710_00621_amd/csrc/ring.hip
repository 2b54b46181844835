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
// direct stage for larger primes), one block of 256 threads per ring and
// map, data resident in LDS (Nphi <= 4096).  Twiddles come from per-length
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

// omega_N^t = exp(-2 pi i t / N) (forward) or its conjugate (inverse)
__device__ __forceinline__ double2 tw_get(const double2* __restrict__ T, int t, bool inv) {
  double2 w = T[2 * t];
  return inv ? make_double2(w.x, -w.y) : w;
}

template <int R>
__device__ __forceinline__ void small_dft(double2 (&v)[R], const double2* __restrict__ T, int N, bool inv) {
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
    double2 out[R];
    const int step = N / R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double2 acc = v[0];
#pragma unroll
      for (int s = 1; s < R; ++s) acc = cadd(acc, cmul(v[s], tw_get(T, ((r * s) % R) * step, inv)));
      out[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = out[r];
  }
}

template <int R>
__device__ void stage_small(double2* x, int N, int Ns, const double2* __restrict__ T, bool inv) {
  constexpr int MAXIT = (kMaxRing / R + 255) / 256;
  const int nb = N / R;
  const int tid = threadIdx.x;
  double2 v[MAXIT][R];
  const int span = N / (Ns * R);
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int j = tid + 256 * it;
    if (j < nb) {
      const int k = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double2 a = x[j + r * nb];
        v[it][r] = (r == 0 || k == 0) ? a : cmul(a, tw_get(T, r * k * span, inv));
      }
      small_dft<R>(v[it], T, N, inv);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int j = tid + 256 * it;
    if (j < nb) {
      const int k = j % Ns;
      const int idx = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) x[idx + r * Ns] = v[it][r];
    }
  }
  __syncthreads();
}

__device__ void stage_generic(double2* x, int N, int Ns, int R, const double2* __restrict__ T, bool inv) {
  constexpr int MAXIT = (kMaxRing + 255) / 256;
  const int nb = N / R;
  const int tid = threadIdx.x;
  const int NsR = Ns * R;
  const int span = N / NsR;
  double2 v[MAXIT];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int o = tid + 256 * it;
    if (o < N) {
      const int k = o % Ns;
      const int r = (o / Ns) % R;
      const int j = (o / NsR) * Ns + k;
      const int base = r * Ns + k;
      double2 acc = make_double2(0.0, 0.0);
      int t = 0;
      for (int s = 0; s < R; ++s) {
        acc = cadd(acc, cmul(x[j + s * nb], tw_get(T, t * span, inv)));
        t += base;
        if (t >= NsR) t -= NsR * (t / NsR);
      }
      v[it] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int o = tid + 256 * it;
    if (o < N) x[o] = v[it];
  }
  __syncthreads();
}

// In-place DFT of x[0..N) in LDS: forward exp(-2 pi i jk/N), inverse exp(+).
__device__ void fft_lds(double2* x, int N, const int* __restrict__ fac, int nfac,
                        const double2* __restrict__ T, bool inv) {
  int Ns = 1;
  for (int st = 0; st < nfac; ++st) {
    const int R = fac[st];
    switch (R) {
      case 1: break;
      case 2: stage_small<2>(x, N, Ns, T, inv); break;
      case 3: stage_small<3>(x, N, Ns, T, inv); break;
      case 4: stage_small<4>(x, N, Ns, T, inv); break;
      case 5: stage_small<5>(x, N, Ns, T, inv); break;
      case 7: stage_small<7>(x, N, Ns, T, inv); break;
      default: stage_generic(x, N, Ns, R, T, inv); break;
    }
    Ns *= R;
  }
}

__global__ __launch_bounds__(256) void k_ring(RingArgs a, int mode, int nmaps, double2* __restrict__ phase,
                                              int64_t pstride, const double* __restrict__ map_in,
                                              double* __restrict__ map_out, int64_t mstride,
                                              const double* const* __restrict__ weights,
                                              int maps_per_weight) {
  __shared__ double2 x[kMaxRing];
  const int r = blockIdx.x;
  const int map = blockIdx.y;
  const int tid = threadIdx.x;
  const int L = a.lmax;
  const int N = a.nphi[r];
  const int64_t off = a.offset[r];
  const int num = a.phinum[r];
  const double2* __restrict__ T = a.tw + a.twoff[r];
  const int* __restrict__ fac = a.fac + (size_t)r * kMaxFactors;
  const int nfac = a.nfac[r];
  double2* __restrict__ ph = phase + (int64_t)map * pstride + (int64_t)r * (L + 1);
  const int twoN = 2 * N;

  if (mode == RING_SYNTH || mode == RING_ROUNDTRIP) {
    // fold the Hermitian spectrum: c_k = (sum_{m=k mod N} g_m + sum_{m=-k mod N} conj g_m) / 2
    for (int k = tid; k < N; k += 256) {
      double2 acc = make_double2(0.0, 0.0);
      for (int m = k; m <= L; m += N) {
        const double2 F = ph[m];
        // g_m = (F^c - i F^s) e^{+i m phi0}, e^{+i m phi0} = conj(T[m num mod 2N])
        const double2 e = T[(int)(((int64_t)m * num) % twoN)];
        acc = cadd(acc, cmulc(make_double2(F.x, -F.y), e));
      }
      for (int m = (N - k) % N; m <= L; m += N) {
        const double2 F = ph[m];
        const double2 e = T[(int)(((int64_t)m * num) % twoN)];
        const double2 g = cmulc(make_double2(F.x, -F.y), e);
        acc = cadd(acc, make_double2(g.x, -g.y));
      }
      x[k] = make_double2(0.5 * acc.x, 0.5 * acc.y);
    }
    __syncthreads();
    fft_lds(x, N, fac, nfac, T, /*inv=*/true);
    if (mode == RING_SYNTH) {
      double* out = map_out + (int64_t)map * mstride + off;
      for (int j = tid; j < N; j += 256) out[j] = x[j].x;
      return;
    }
    const double* __restrict__ w = weights[map / maps_per_weight] + off;
    for (int j = tid; j < N; j += 256) x[j] = make_double2(x[j].x * w[j], 0.0);
    __syncthreads();
  } else {
    const double* in = map_in + (int64_t)map * mstride + off;
    for (int j = tid; j < N; j += 256) x[j] = make_double2(in[j], 0.0);
    __syncthreads();
  }
  fft_lds(x, N, fac, nfac, T, /*inv=*/false);
  if (mode == RING_DIAG) {
    const double t0 = x[0].x;
    for (int m = tid; m <= L; m += 256) {
      if (m == 0) {
        ph[0] = make_double2(t0, 0.0);
      } else {
        const int k = (int)((2 * (int64_t)m) % N);
        const double2 X = cmul(x[k], T[(int)(((int64_t)2 * m * num) % twoN)]);
        ph[m] = make_double2(t0 + X.x, t0 - X.x);
      }
    }
    return;
  }
  for (int m = tid; m <= L; m += 256) {
    const double2 F = x[m % N];
    // H_m = e^{-i m phi0} F^_{m mod N};  e^{-i m phi0} = T[m num mod 2N]
    const double2 h = cmul(F, T[(int)(((int64_t)m * num) % twoN)]);
    ph[m] = make_double2(h.x, m == 0 ? 0.0 : -h.y);
  }
}

}  // namespace

void launch_ring(const RingArgs& a, RingMode mode, int nmaps, double2* phase, int64_t pstride,
                 const double* map_in, double* map_out, int64_t mstride,
                 const double* const* weights, int maps_per_weight, hipStream_t s) {
  dim3 grid(a.nring, nmaps);
  hipLaunchKernelGGL(k_ring, grid, dim3(256), 0, s, a, (int)mode, nmaps, phase, pstride, map_in,
                     map_out, mstride, weights, maps_per_weight < 1 ? 1 : maps_per_weight);
  CRS_HIP(hipGetLastError());
}

}  // namespace crs
