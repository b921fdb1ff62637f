// Register-resident real <-> band-limited-spectrum transforms for one s-row
// per lane (gfx950, wave64).
//
// A state row holds the Fourier coefficients X_k, k = 0..K, of a real field
// sampled on N points, x_n = sum_{|k|<=K} X_k e^{2 pi i k n / N} (the paper's
// spatial expansion, Sec. V.C.1), with K < N/3 so that quadratic products are
// alias-free for the kept modes.  Each lane owns one whole row: the transform
// runs entirely in VGPRs, twiddles are compile-time literals, and no lane ever
// talks to another during a transform.
//
// Real transforms use the half-length complex trick: the N reals are paired
// as z_m = x_{2m} + i x_{2m+1}, m < M = N/2, and one complex M-point FFT does
// the work; an O(M) pre/post-processing step maps between Z and X.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace ksc {

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------

template <int... Is, class F>
__device__ __forceinline__ void sfor_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
// Unrolled loop whose index is a constant expression inside the body.
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(std::make_integer_sequence<int, N>{}, f);
}

constexpr double kPi = 3.141592653589793238462643383279502884;

// Taylor series of sin and cos on |x| <= pi/4 (terms to x^25; the remainder
// is below 1e-19 there).
constexpr double cx_sin_small(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n <= 12; ++n) {
    term *= -x2 / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos_small(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n <= 12; ++n) {
    term *= -x2 / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}

// cos and sin of 2 pi e / M for integer e, with exact quadrant reduction.
struct CS {
  double c, s;
};
constexpr CS cx_unit(long e, long M) {
  e %= M;
  if (e < 0) e += M;
  // quadrant q = nearest multiple of M/4; remainder angle pi * r / (2M), |r| <= M/2
  long q = (4 * e + M / 2) / M;
  long r = 4 * e - q * M;
  double x = kPi * double(r) / double(2 * M);
  double c = cx_cos_small(x), s = cx_sin_small(x);
  switch (q & 3) {
    case 0: return {c, s};
    case 1: return {-s, c};
    case 2: return {-c, -s};
    default: return {s, -c};
  }
}

template <typename T>
struct cplx {
  T r, i;
};

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev(int v, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
  return r;
}

// ---------------------------------------------------------------------------
// complex M-point FFT in registers, radix-2 decimation in time.
//   SIGN = -1: Z_k = sum_m z_m e^{-2 pi i k m / M}
//   SIGN = +1: Z_k = sum_m z_m e^{+2 pi i k m / M}
// Input in natural order, output in natural order (the bit-reversal is a
// compile-time renaming of registers).  Butterflies with a general twiddle
// use the 6-FMA form a' = a + w b, b' = 2a - a'.
// ---------------------------------------------------------------------------
template <int M, int SIGN, typename T>
__device__ __forceinline__ void fft_c(T (&re)[M], T (&im)[M]) {
  constexpr int LG = ilog2(M);
  static_assert((1 << LG) == M, "power of two");
  T xr[M], xi[M];
  sfor<M>([&](auto I) {
    constexpr int i = I;
    constexpr int s = bitrev(i, LG);
    xr[i] = re[s];
    xi[i] = im[s];
  });
  sfor<LG>([&](auto S) {
    constexpr int h = 1 << int(S);  // half-size of the sub-DFTs being merged
    sfor<M / 2>([&](auto B) {
      constexpr int b = B;
      constexpr int blk = b / h, j = b % h;
      constexpr int a0 = blk * 2 * h + j, a1 = a0 + h;
      constexpr int e = j * (M / (2 * h));  // twiddle exponent, angle 2 pi e / M
      if constexpr (e == 0) {
        T tr = xr[a1], ti = xi[a1];
        xr[a1] = xr[a0] - tr;
        xi[a1] = xi[a0] - ti;
        xr[a0] = xr[a0] + tr;
        xi[a0] = xi[a0] + ti;
      } else if constexpr (4 * e == M) {
        // w = SIGN * i : w*b = (-SIGN b.i, SIGN b.r)
        T tr = (SIGN > 0) ? -xi[a1] : xi[a1];
        T ti = (SIGN > 0) ? xr[a1] : -xr[a1];
        xr[a1] = xr[a0] - tr;
        xi[a1] = xi[a0] - ti;
        xr[a0] = xr[a0] + tr;
        xi[a0] = xi[a0] + ti;
      } else {
        constexpr CS w = cx_unit(e, M);
        constexpr T wr = T(w.c);
        constexpr T wi = T(SIGN * w.s);
        T ar = xr[a0], ai = xi[a0], br = xr[a1], bi = xi[a1];
        T nr = fmaT(-wi, bi, fmaT(wr, br, ar));
        T ni = fmaT(wi, br, fmaT(wr, bi, ai));
        xr[a0] = nr;
        xi[a0] = ni;
        xr[a1] = fmaT(T(2), ar, -nr);
        xi[a1] = fmaT(T(2), ai, -ni);
      }
    });
  });
  sfor<M>([&](auto I) {
    constexpr int i = I;
    re[i] = xr[i];
    im[i] = xi[i];
  });
}

// ---------------------------------------------------------------------------
// Band-limited spectrum -> real samples.
//   x_n = sum_{|k|<=K} X_k e^{2 pi i k n / N},  X_{-k} = conj(X_k), Im X_0 ignored.
// X has KM = K+1 entries; out has N entries.
// ---------------------------------------------------------------------------
// TI is the storage type of the coefficients (converted to the arithmetic
// type T as they are read).
template <int N, int KM, typename T, typename TI = T>
__device__ __forceinline__ void spec_to_phys(const cplx<TI> (&X)[KM], T (&out)[N]) {
  constexpr int M = N / 2;
  static_assert(KM - 1 < M, "K must be below N/2");
  T zr[M], zi[M];
  // Z_k = E_k + i O_k with E_k = X_k + conj(X_{M-k}), O_k = w^k (X_k - conj(X_{M-k})),
  // w = e^{2 pi i / N}.  For the partner M - k, E_{M-k} = conj(E_k) and, since
  // w^{M-k} = -conj(w^k), O_{M-k} = conj(O_k): one product serves both.
  sfor<M / 2 + 1>([&](auto Kk) {
    constexpr int k = Kk;
    constexpr int kb = M - k;  // partner index; kb == M means X_M (zero)
    T ar = T(0), ai = T(0), br = T(0), bi = T(0);
    if constexpr (k < KM) {
      ar = T(X[k].r);
      ai = (k == 0) ? T(0) : T(X[k].i);
    }
    if constexpr (kb < KM) {
      br = T(X[kb].r);
      bi = -T(X[kb].i);  // conj
    }
    // (a partner above K is zero: its sums and differences are not formed)
    T er = (kb < KM) ? ar + br : ar, ei = (kb < KM) ? ai + bi : ai;
    T dr = (kb < KM) ? ar - br : ar, di = (kb < KM) ? ai - bi : ai;
    T orr, oi;
    if constexpr (k == 0) {
      orr = dr;
      oi = di;
    } else {
      constexpr CS w = cx_unit(k, N);
      constexpr T wr = T(w.c), wi = T(w.s);
      orr = fmaT(wr, dr, -wi * di);
      oi = fmaT(wr, di, wi * dr);
    }
    zr[k] = er - oi;
    zi[k] = ei + orr;
    if constexpr (k != 0 && k != M / 2) {
      zr[M - k] = er + oi;   // conj(E) + i conj(O)
      zi[M - k] = orr - ei;
    }
  });
  fft_c<M, +1, T>(zr, zi);
  sfor<M>([&](auto Mm) {
    constexpr int m = Mm;
    out[2 * m] = zr[m];
    out[2 * m + 1] = zi[m];
  });
}

// ---------------------------------------------------------------------------
// Real samples -> kept modes, unnormalized and doubled:
//   X_k = 2 * sum_n x_n e^{-2 pi i k n / N},  k = 0..K
// (X_k / (2N) is the Fourier coefficient; callers fold 1/(2N) into the
// per-mode constants they multiply by anyway).  Outputs above K are never
// formed; the dead butterflies of the last FFT stage are removed by the
// compiler.
// ---------------------------------------------------------------------------
template <int N, int KM, typename T>
__device__ __forceinline__ void phys_to_spec2(const T (&x)[N], cplx<T> (&X)[KM]) {
  constexpr int M = N / 2;
  T zr[M], zi[M];
  sfor<M>([&](auto Mm) {
    constexpr int m = Mm;
    zr[m] = x[2 * m];
    zi[m] = x[2 * m + 1];
  });
  fft_c<M, -1, T>(zr, zi);
  // X_k = D_k - i V_k with D = Z_k + conj(Z_{M-k}), S = Z_k - conj(Z_{M-k}),
  // V = w^{-k} S.  For a partner M - k that is also kept, D_{M-k} = conj(D_k),
  // S_{M-k} = -conj(S_k) and w^{-(M-k)} = -w^k, so X_{M-k} = conj(D_k + i V_k).
  sfor<KM>([&](auto Kk) {
    constexpr int k = Kk;
    constexpr int kb = (M - k) % M;
    constexpr bool paired_low = (k != 0) && (2 * k < M) && (M - k < KM);  // forms X_{M-k} too
    constexpr bool paired_high = (2 * k > M) && (M - k < KM);           // formed by M - k
    if constexpr (k == 0) {
      X[0].r = (zr[0] + zr[0]) + (zi[0] + zi[0]);
      X[0].i = T(0);
    } else if constexpr (!paired_high) {
      constexpr CS w = cx_unit(k, N);
      constexpr T c = T(w.c), s = T(w.s);
      const T Dr = zr[k] + zr[kb], Di = zi[k] - zi[kb];
      const T Sr = zr[k] - zr[kb], Si = zi[k] + zi[kb];
      // V = (c - i s) S
      const T Vr = fmaT(c, Sr, s * Si), Vi = fmaT(c, Si, -s * Sr);
      X[k].r = Dr + Vi;
      X[k].i = Di - Vr;
      if constexpr (paired_low) {
        X[M - k].r = Dr - Vi;
        X[M - k].i = -(Di + Vr);
      }
    }
  });
}

// Real samples -> Fourier coefficients X_k = (1/N) sum_n x_n e^{-2 pi i k n / N}.
template <int N, int KM, typename T>
__device__ __forceinline__ void phys_to_spec(const T (&x)[N], cplx<T> (&X)[KM]) {
  phys_to_spec2<N, KM, T>(x, X);
  constexpr T h = T(0.5 / N);
  sfor<KM>([&](auto Kk) {
    constexpr int k = Kk;
    X[k].r *= h;
    X[k].i *= h;
  });
}

// ---------------------------------------------------------------------------
// Lane pairs: two neighbouring lanes (p = lane & 1) share one row, for grids
// whose whole-row transform would not fit one lane's registers.
//
// Spectrum side, lane p holds X_k for k = 2i + p, i = 0..KH-1 (entries with
// k > K are zero).  Physical side, lane p holds the samples x_n with
// n in [p N/2, (p+1) N/2).
//
// With M = N/2 (half-length trick) and Q = M/2, the complex M-point DFT splits
// as z_{m1 + Q m2} = sum_{k2} (-1)^{m2 k2} w_M^{m1 k2} sum_{k1} w_Q^{m1 k1}
// Z_{2 k1 + k2}: each lane runs a Q-point FFT over its decimated spectrum, a
// lane-dependent twiddle, and one radix-2 stage across the pair (a DPP lane
// swap).  The forward transform runs the same steps in reverse order.
// ---------------------------------------------------------------------------

// Value of the other lane of the pair (DPP quad_perm [1, 0, 3, 2]).
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xf, 0xf, false));
}
__device__ __forceinline__ double pair_swap(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp(int(b), 0xB1, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), 0xB1, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Complex product of (xr, xi) with the compile-time unit number e^{2 pi i e / n}
// (SIGN = +1) or its conjugate (SIGN = -1).
template <long E, long NN, int SIGN, typename T>
__device__ __forceinline__ void cmul_unit(T& xr, T& xi) {
  constexpr CS w = cx_unit(E, NN);
  constexpr T c = T(w.c), s = T(SIGN * w.s);
  const T r = fmaT(c, xr, -s * xi);
  xi = fmaT(c, xi, s * xr);
  xr = r;
}

// Band-limited spectrum -> this lane's half of the samples (see above).
//   x_n = sum_{|k|<=K} X_k e^{2 pi i k n / N},  Im X_0 ignored.
// pf is 0 on lane 0 and 1 on lane 1 of the pair.  Lane-dependent factors are
// formed as both candidates from compile-time constants followed by a select
// of the two results (never a select between two constants, which would keep
// the constants in registers across the caller's loops).  pf passes through an
// empty asm statement so that nothing derived from it is hoisted either.
template <int N, int KH, typename T, typename TI = T>
__device__ __forceinline__ void spec_to_phys_pair(const cplx<TI> (&X)[KH], T pf, T (&out)[N / 2]) {
  constexpr int M = N / 2, Q = M / 2;
  static_assert(2 * KH <= M + 1, "K must be below N/2");
  __asm__ volatile("" : "+v"(pf));
  const bool odd = pf != T(0);
  const T sgn = odd ? T(-1) : T(1);
  T zr[Q], zi[Q];
  sfor<Q>([&](auto K1) {
    constexpr int k1 = K1;
    // k = 2 k1 + p; its partner M - k is entry Q - k1 - p of this lane
    constexpr int ib0 = Q - k1, ib1 = Q - k1 - 1;
    T ar = T(0), ai = T(0);
    if constexpr (k1 < KH) {
      ar = T(X[k1].r);
      ai = T(X[k1].i);
      if constexpr (k1 == 0) ai = odd ? ai : T(0);  // Im X_0 (lane 0, entry 0)
    }
    T b0r = T(0), b0i = T(0), b1r = T(0), b1i = T(0);
    if constexpr (ib0 < KH && ib0 < Q) {
      b0r = T(X[ib0].r);
      b0i = T(X[ib0].i);
    }
    if constexpr (ib1 < KH) {
      b1r = T(X[ib1].r);
      b1i = T(X[ib1].i);
    }
    const T br = odd ? b1r : b0r, bi = -(odd ? b1i : b0i);  // conj(X_{M-k})
    const T er = ar + br, ei = ai + bi;
    T dr = ar - br, di = ai - bi;
    // O_k = w^k D_k, w = e^{2 pi i / N}: lane 1 takes one more factor w
    T d1r = dr, d1i = di;
    cmul_unit<1, N, +1, T>(d1r, d1i);
    dr = odd ? d1r : dr;
    di = odd ? d1i : di;
    if constexpr (k1 != 0) cmul_unit<2 * k1, N, +1, T>(dr, di);
    zr[k1] = er - di;  // Z_k = E_k + i O_k
    zi[k1] = ei + dr;
  });
  fft_c<Q, +1, T>(zr, zi);
  sfor<Q>([&](auto M1) {
    constexpr int m1 = M1;
    T tr = zr[m1], ti = zi[m1];
    if constexpr (m1 != 0) {  // lane 1: times e^{2 pi i m1 / M}
      T ur = tr, ui = ti;
      cmul_unit<m1, M, +1, T>(ur, ui);
      tr = odd ? ur : tr;
      ti = odd ? ui : ti;
    }
    const T yr = pair_swap(tr), yi = pair_swap(ti);
    out[2 * m1] = fmaT(sgn, tr, yr);      // lane 0: T0 + T1, lane 1: T0 - T1
    out[2 * m1 + 1] = fmaT(sgn, ti, yi);
    // keep the swaps next to their uses (clustered, their results spill)
    if constexpr (m1 % 8 == 7) __builtin_amdgcn_sched_barrier(0);
  });
}

// This lane's half of the samples -> its kept modes, unnormalized and doubled:
//   X_k = 2 sum_n x_n e^{-2 pi i k n / N},  k = 2i + p <= K.
template <int N, int KH, typename T>
__device__ __forceinline__ void phys_to_spec2_pair(const T (&x)[N / 2], T pf, cplx<T> (&X)[KH]) {
  constexpr int M = N / 2, Q = M / 2;
  __asm__ volatile("" : "+v"(pf));
  const bool odd = pf != T(0);
  const T sgn = odd ? T(-1) : T(1);
  T zr[Q], zi[Q];
  sfor<Q>([&](auto M1) {
    constexpr int m1 = M1;
    const T xr = x[2 * m1], xi = x[2 * m1 + 1];
    const T yr = pair_swap(xr), yi = pair_swap(xi);
    T tr = fmaT(sgn, xr, yr), ti = fmaT(sgn, xi, yi);  // lane 0: z + z', lane 1: z - z'
    if constexpr (m1 != 0) {  // lane 1: times e^{-2 pi i m1 / M}
      T ur = tr, ui = ti;
      cmul_unit<m1, M, -1, T>(ur, ui);
      tr = odd ? ur : tr;
      ti = odd ? ui : ti;
    }
    zr[m1] = tr;
    zi[m1] = ti;
    if constexpr (m1 % 8 == 7) __builtin_amdgcn_sched_barrier(0);
  });
  fft_c<Q, -1, T>(zr, zi);
  sfor<KH>([&](auto K1) {
    constexpr int k1 = K1;
    // Z_{M-k} is entry (Q - k1 - p) mod Q of this lane
    constexpr int ib0 = (Q - k1) % Q, ib1 = Q - k1 - 1;
    const T br = odd ? zr[ib1] : zr[ib0], bi = odd ? zi[ib1] : zi[ib0];
    const T Dr = zr[k1] + br, Di = zi[k1] - bi;
    T Sr = zr[k1] - br, Si = zi[k1] + bi;
    // X_k = D - i w^{-k} S: lane 1 takes one more factor w^{-1}
    T s1r = Sr, s1i = Si;
    cmul_unit<1, N, -1, T>(s1r, s1i);
    Sr = odd ? s1r : Sr;
    Si = odd ? s1i : Si;
    if constexpr (k1 != 0) cmul_unit<2 * k1, N, -1, T>(Sr, Si);
    X[k1].r = Dr + Si;
    X[k1].i = Di - Sr;
  });
}

}  // namespace ksc
