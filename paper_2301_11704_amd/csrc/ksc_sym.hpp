// Real transforms of fields that are odd or even in x (the inversion-symmetric
// subspace), one row per lane in registers, built on the complex FFT of
// ksc_fft.hpp.
#pragma once

#include "ksc_fft.hpp"

namespace ksc {

// ---------------------------------------------------------------------------
// Sine and cosine transforms for fields that are odd or even in x (the
// inversion-symmetric subspace), with m = N/2:
//   DST-I  F_j = sum_{k=1}^{m-1} f_k sin(pi k j / m),
//   DCT-I  C_n = g_0/2 + (-1)^n g_m/2 + sum_{k=1}^{m-1} g_k cos(pi k n / m).
// Split-radix recursion on the output parity (pairing k with m - k, h = m/2):
//   C_{2i}   = DCT-I_h (s),   s_k = g_k + g_{m-k} (s_0 = g_0 + g_m, s_h = 2 g_h),
//   C_{2i+1} = DCT-III_h (e), e_k = g_k - g_{m-k} (e_0 = g_0 - g_m),
//   F_{2i}   = DST-I_h (d),   d_k = f_k - f_{m-k},
//   F_{2i+1} = (-1)^i DCT-III_h (b),  b_0 = 2 f_h, b_k = f_{h-k} + f_{h+k},
// where DCT-III_h(b)_n = b_0/2 + sum_{k=1}^{h-1} b_k cos(pi k (2n+1) / (2h)).
// A DCT-III of length h is one Hermitian inverse DFT of h points (Makhoul's
// reordering: V_k = e^{i pi k/(2h)} (b_k - i b_{h-k}), v = sum_k V_k e^{2 pi i k n/h},
// x_{2n} = v_n / 2, x_{2n+1} = v_{h-1-n} / 2), i.e. a complex FFT of h/2 points.
// Every output is a direct transform of the input: no output is formed from
// another by a running sum, whose rounding errors would add up along the
// outputs.  The levels together take about as many FFT points as one real DFT
// of m points.  All functions return twice the transform.
// ---------------------------------------------------------------------------

// v_n = sum_{k=0}^{H-1} V_k e^{2 pi i k n / H}, n = 0..H-1, for a Hermitian V
// given by V_0 .. V_{H/2} (V_0 and V_{H/2} real): the half-length trick with
// one complex FFT of H/2 points (as spec_to_phys, with the Nyquist term kept).
template <int H, typename T>
__device__ __forceinline__ void herm_to_real(const cplx<T> (&V)[H / 2 + 1], T (&out)[H]) {
  constexpr int M = H / 2;
  T zr[M], zi[M];
  // Z_k = E_k + i O_k, E_k = V_k + conj(V_{M-k}), O_k = w^k (V_k - conj(V_{M-k})),
  // w = e^{2 pi i / H}; the partner M - k has conj(E_k) and conj(O_k).
  sfor<M / 2 + 1>([&](auto Kk) {
    constexpr int k = Kk;
    constexpr int kb = M - k;
    const T ar = V[k].r, ai = (k == 0) ? T(0) : V[k].i;
    const T br = V[kb].r, bi = (kb == M) ? T(0) : -V[kb].i;  // conj
    const T er = ar + br, ei = ai + bi;
    const T dr = ar - br, di = ai - bi;
    T orr, oi;
    if constexpr (k == 0) {
      orr = dr;
      oi = di;
    } else {
      constexpr CS w = cx_unit(k, H);
      constexpr T wr = T(w.c), wi = T(w.s);
      orr = fmaT(wr, dr, -wi * di);
      oi = fmaT(wr, di, wi * dr);
    }
    zr[k] = er - oi;
    zi[k] = ei + orr;
    if constexpr (k != 0 && 2 * k != M) {
      zr[M - k] = er + oi;
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

// x[n] = 2 DCT-III_H(b)_n = b_0 + 2 sum_{k=1}^{H-1} b_k cos(pi k (2n+1) / (2H)).
template <int H, typename T>
__device__ __forceinline__ void dct3_x2(const T (&b)[H], T (&x)[H]) {
  if constexpr (H == 1) {
    x[0] = b[0];
  } else {
    cplx<T> V[H / 2 + 1];
    sfor<H / 2 + 1>([&](auto Kk) {
      constexpr int k = Kk;
      if constexpr (k == 0) {
        V[0] = cplx<T>{b[0], T(0)};
      } else if constexpr (2 * k == H) {
        V[k] = cplx<T>{T(1.4142135623730950488) * b[k], T(0)};
      } else {
        constexpr CS w = cx_unit(k, 4 * H);  // e^{i pi k / (2H)}
        constexpr T c = T(w.c), s = T(w.s);
        V[k] = cplx<T>{fmaT(c, b[k], s * b[H - k]), fmaT(s, b[k], -c * b[H - k])};
      }
    });
    T v[H];
    herm_to_real<H, T>(V, v);
    sfor<H / 2>([&](auto Nn) {
      constexpr int n = Nn;
      x[2 * n] = v[n];
      x[2 * n + 1] = v[H - 1 - n];
    });
  }
}

// out[n] = 2 C_n for n = 0..NOUT-1 (NOUT <= m + 1); g[k] for k = 0..m.
template <int M2, int NOUT, typename T>
__device__ __forceinline__ void dct1_x2(const T (&g)[M2 + 1], T (&out)[NOUT]) {
  static_assert(NOUT <= M2 + 1, "outputs 0..m");
  if constexpr (M2 == 1) {
    out[0] = g[0] + g[1];
    if constexpr (NOUT > 1) out[1] = g[0] - g[1];
  } else {
    constexpr int h = M2 / 2;
    constexpr int NE = (NOUT + 1) / 2;  // even outputs 2i < NOUT
    T sv[h + 1], ev[h];
    sfor<h + 1>([&](auto Kk) {
      constexpr int k = Kk;
      if constexpr (k == 0) {
        sv[0] = g[0] + g[M2];
        ev[0] = g[0] - g[M2];
      } else if constexpr (k == h) {
        sv[h] = g[h] + g[h];
      } else {
        sv[k] = g[k] + g[M2 - k];
        ev[k] = g[k] - g[M2 - k];
      }
    });
    T ce[NE], co[h];
    dct1_x2<h, NE, T>(sv, ce);
    dct3_x2<h, T>(ev, co);
    sfor<NOUT>([&](auto Nn) {
      constexpr int n = Nn;
      if constexpr (n % 2 == 0)
        out[n] = ce[n / 2];
      else
        out[n] = co[n / 2];
    });
  }
}

// out[j] = 2 F_j for j = 0..NOUT-1 (NOUT <= m; out[0] = 0); f[k] for k = 1..m-1
// (f[0] unused).
template <int M2, int NOUT, typename T>
__device__ __forceinline__ void dst1_x2(const T (&f)[M2], T (&out)[NOUT]) {
  static_assert(NOUT <= M2, "outputs 0..m-1");
  if constexpr (M2 == 1) {
    out[0] = T(0);
  } else {
    constexpr int h = M2 / 2;
    constexpr int NE = (NOUT + 1) / 2;  // even outputs 2i < NOUT
    T dv[h], bv[h];
    sfor<h>([&](auto Kk) {
      constexpr int k = Kk;
      if constexpr (k == 0) {
        dv[0] = T(0);
        bv[0] = f[h] + f[h];
      } else {
        dv[k] = f[k] - f[M2 - k];
        bv[k] = f[h - k] + f[h + k];
      }
    });
    T fe[NE], fo[h];
    dst1_x2<h, NE, T>(dv, fe);
    dct3_x2<h, T>(bv, fo);
    sfor<NOUT>([&](auto Jj) {
      constexpr int j = Jj;
      if constexpr (j % 2 == 0)
        out[j] = fe[j / 2];
      else if constexpr ((j / 2) % 2 == 0)
        out[j] = fo[j / 2];
      else
        out[j] = -fo[j / 2];
    });
  }
}

}  // namespace ksc
