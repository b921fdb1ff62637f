// Fused per-tile evaluation of the KS connecting-curve residual, the cost J^2,
// the adjoint L^dagger(u; r) and either the Euclidean gradient of J^2 or one
// semi-implicit descent step (Ashtari & Schneider, arXiv:2301.11704: residual
// eq. KSE_residual, cost eq. cost_function_general, adjoint Sec. V.A and
// Appendix A, descent eq. KSE_G with the semi-implicit Euler of Sec. V.C.3).
//
// Work decomposition: a workgroup of 64*W lanes owns one tile of consecutive
// s-rows of one curve; lane t computes the residual of row jr = j0 - 1 + t,
// so the tile evaluates 64W residual rows and emits the 64W - 2 interior ones
// (the first and last lane supply the s-halo of the adjoint's d/ds).  The
// state rows j0-2 .. j0+64W-1 are staged once in LDS (mode-major, so that
// lane-consecutive accesses hit consecutive banks); each HBM byte of the state
// is read once per tile and each output byte written once.
#pragma once

#include "ksc_fft.hpp"

namespace ksc {

enum Mode : int { MODE_J = 0, MODE_GRAD = 1, MODE_STEP = 2 };

// Per-curve descriptor as seen by the kernels.
struct CurveDev {
  long long off;       // offset of row 0 in complex elements of the state
  long long poff;      // offset of row 0 in physical samples
  int n_s, n_x, km;    // rows, grid points, kept modes (K+1)
  int row_off;         // offset into the per-row tables
  int mode_off;        // offset into the per-mode tables
  int tile_begin;      // first tile of this curve in the tile list
  int n_tiles;
  int pad_;
};

struct TileDev {
  int curve;
  int j0;  // first emitted row
};

template <typename T>
struct KernelArgs {
  const cplx<T>* __restrict__ in;     // state
  cplx<T>* __restrict__ out;          // gradient (MODE_GRAD) or next state (MODE_STEP)
  const CurveDev* __restrict__ curves;
  const TileDev* __restrict__ tiles;
  const T* __restrict__ cs;           // per row: g_j / (2 dsigma)
  const T* __restrict__ wlT;          // per row: w_j L (run precision)
  const double* __restrict__ wlD;     // per row: w_j L (FP64, cost reduction)
  const T* __restrict__ q;            // per mode: 2 pi k / L
  const T* __restrict__ A;            // per mode: q^2 - q^4
  const T* __restrict__ pre;          // per mode: 1 / (1 + dtau A^2)   (MODE_STEP)
  const double* __restrict__ scale;   // per curve gradient scale, nullable
  const unsigned char* __restrict__ active;  // per curve, nullable
  double* __restrict__ partials;      // per tile: J^2, J_arc numerator, J_arc denominator
  T dtau;
  int n_tiles;
  int tile_base;
};

template <typename T>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum three per-lane FP64 values over the workgroup in a fixed order and
// store them as the tile's partials.
template <int W>
__device__ __forceinline__ void reduce_partials(double a, double b, double c, double* red,
                                                double* dst) {
  a = wave_sum<double>(a);
  b = wave_sum<double>(b);
  c = wave_sum<double>(c);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[3 * wv + 0] = a;
    red[3 * wv + 1] = b;
    red[3 * wv + 2] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      s0 += red[3 * w + 0];
      s1 += red[3 * w + 1];
      s2 += red[3 * w + 2];
    }
    dst[0] = s0;
    dst[1] = s1;
    dst[2] = s2;
  }
}

// LDS bytes a tile needs for KM modes.
template <typename T, int W>
constexpr int tile_lds_bytes(int km) {
  return (64 * W + 2) * km * int(sizeof(cplx<T>)) + 3 * W * int(sizeof(double));
}

template <int NX, typename T, int W, int MODE>
__device__ __forceinline__ void tile_body(const KernelArgs<T>& a, const CurveDev& cd, int c,
                                          int j0, int tile, cplx<T>* buf, double* red) {
  constexpr int KM = (NX - 1) / 3 + 1;
  constexpr int ROWS = 64 * W;   // residual rows per tile
  constexpr int BR = ROWS + 2;   // staged state rows
  const int t = threadIdx.x;
  const int n_s = cd.n_s;
  const cplx<T>* __restrict__ src = a.in + cd.off;
  const int jr = j0 - 1 + t;

  __syncthreads();  // the previous tile of a persistent workgroup is done with the LDS
  // ---- stage the state rows j0-2 .. j0+ROWS-1 in LDS (mode-major) ----
  cplx<T> X[KM];
  {
    const bool ok = (jr >= 0) && (jr < n_s);
    const cplx<T>* row = src + (long long)(ok ? jr : 0) * KM;
    sfor<KM>([&](auto Kk) {
      constexpr int k = Kk;
      cplx<T> v = ok ? row[k] : cplx<T>{T(0), T(0)};
      if (k == 0) v.i = T(0);
      X[k] = v;
      buf[k * BR + t + 1] = v;
    });
    if (t < 2) {
      const int je = (t == 0) ? (j0 - 2) : (j0 - 1 + ROWS);
      const int be = (t == 0) ? 0 : (BR - 1);
      const bool oke = (je >= 0) && (je < n_s);
      const cplx<T>* rowe = src + (long long)(oke ? je : 0) * KM;
      sfor<KM>([&](auto Kk) {
        constexpr int k = Kk;
        cplx<T> v = oke ? rowe[k] : cplx<T>{T(0), T(0)};
        if (k == 0) v.i = T(0);
        buf[k * BR + be] = v;
      });
    }
  }
  __syncthreads();

  const T* __restrict__ qv = a.q + cd.mode_off;
  const T* __restrict__ Av = a.A + cd.mode_off;
  const bool interior = (jr >= 1) && (jr <= n_s - 2);
  const bool owned = interior && (t >= 1) && (t <= ROWS - 2);
  const T csj = interior ? a.cs[cd.row_off + jr] : T(0);

  // ---- u = physical field of row jr; N_hat = spectrum of u^2 ----
  T u[NX];
  spec_to_phys<NX, KM, T>(X, u);
  cplx<T> R[KM];
  T rowR = T(0), rowD = T(0);
  {
    T p[NX];
    sfor<NX>([&](auto Nn) {
      constexpr int n = Nn;
      p[n] = u[n] * u[n];
    });
    cplx<T> Nh[KM];
    phys_to_spec<NX, KM, T>(p, Nh, T(1) / T(NX));
    // r_hat = -g (u_{j+1} - u_{j-1}) / (2 dsigma) + A u_hat - (i q / 2) N_hat
    sfor<KM>([&](auto Kk) {
      constexpr int k = Kk;
      constexpr T ck = (k == 0) ? T(1) : T(2);
      const cplx<T> xm = buf[k * BR + t];
      const cplx<T> xp = buf[k * BR + t + 2];
      const T dr = xp.r - xm.r, di = xp.i - xm.i;
      const T qh = T(0.5) * qv[k];
      const T Ak = Av[k];
      T rr = fmaT(-csj, dr, fmaT(Ak, X[k].r, qh * Nh[k].i));
      T ri = fmaT(-csj, di, fmaT(Ak, X[k].i, -qh * Nh[k].r));
      if (k == 0) ri = T(0);
      if (!interior) {
        rr = T(0);
        ri = T(0);
      }
      R[k].r = rr;
      R[k].i = ri;
      rowR = fmaT(ck * rr, rr, fmaT(ck * ri, ri, rowR));
      rowD = fmaT(ck * dr, dr, fmaT(ck * di, di, rowD));
    });
  }
  {
    double pj = 0.0, pn = 0.0, pd = 0.0;
    if (owned) {
      const double rR = double(rowR), rD = double(rowD);
      pj = a.wlD[cd.row_off + jr] * rR;
      pn = sqrt(rR * rD);
      pd = sqrt(rD);
    }
    reduce_partials<W>(pj, pn, pd, red, a.partials + 3ll * tile);
  }
  if constexpr (MODE == MODE_J) {
    return;
  } else {
    __syncthreads();  // everyone has read the staged state
    sfor<KM>([&](auto Kk) {
      constexpr int k = Kk;
      buf[k * BR + t] = R[k];
    });
    __syncthreads();

    // ---- rho = physical field of r_x; Q_hat = spectrum of u * rho ----
    cplx<T> Q[KM];
    {
      cplx<T> Y[KM];
      sfor<KM>([&](auto Kk) {
        constexpr int k = Kk;
        const T qk = qv[k];
        Y[k].r = -qk * R[k].i;
        Y[k].i = qk * R[k].r;
      });
      T rho[NX];
      spec_to_phys<NX, KM, T>(Y, rho);
      sfor<NX>([&](auto Nn) {
        constexpr int n = Nn;
        rho[n] = u[n] * rho[n];
      });
      phys_to_spec<NX, KM, T>(rho, Q, T(1) / T(NX));
    }

    // ---- L^dagger r = g (r_{j+1} - r_{j-1}) / (2 dsigma) + Q_hat + A r_hat ----
    const int tm = (t >= 1) ? t - 1 : 0;
    const int tp = (t <= ROWS - 2) ? t + 1 : ROWS - 1;
    cplx<T>* __restrict__ dstrow = a.out + cd.off + (long long)jr * KM;
    if constexpr (MODE == MODE_GRAD) {
      const T sc = (a.scale != nullptr) ? T(a.scale[c]) : T(1);
      const T two_wl = owned ? T(2) * a.wlT[cd.row_off + jr] * sc : T(0);
      if (owned) {
        sfor<KM>([&](auto Kk) {
          constexpr int k = Kk;
          constexpr T ck = (k == 0) ? T(1) : T(2);
          const cplx<T> rm = buf[k * BR + tm];
          const cplx<T> rp = buf[k * BR + tp];
          const T Ak = Av[k];
          T gr = fmaT(csj, rp.r - rm.r, fmaT(Ak, R[k].r, Q[k].r));
          T gi = fmaT(csj, rp.i - rm.i, fmaT(Ak, R[k].i, Q[k].i));
          const T f = two_wl * ck;
          cplx<T> o;
          o.r = f * gr;
          o.i = (k == 0) ? T(0) : f * gi;
          dstrow[k] = o;
        });
      } else if ((jr == 0 || jr == n_s - 1) && jr >= 0 && jr < n_s) {
        sfor<KM>([&](auto Kk) {
          constexpr int k = Kk;
          dstrow[k] = cplx<T>{T(0), T(0)};
        });
      }
    } else {  // MODE_STEP
      const T* __restrict__ pv = a.pre + cd.mode_off;
      if (owned) {
        sfor<KM>([&](auto Kk) {
          constexpr int k = Kk;
          const cplx<T> rm = buf[k * BR + tm];
          const cplx<T> rp = buf[k * BR + tp];
          const T Ak = Av[k];
          T gr = fmaT(csj, rp.r - rm.r, fmaT(Ak, R[k].r, Q[k].r));
          T gi = fmaT(csj, rp.i - rm.i, fmaT(Ak, R[k].i, Q[k].i));
          const T f = -a.dtau * pv[k];
          cplx<T> o;
          o.r = fmaT(f, gr, X[k].r);
          o.i = (k == 0) ? T(0) : fmaT(f, gi, X[k].i);
          dstrow[k] = o;
        });
      } else if ((jr == 0 || jr == n_s - 1) && jr >= 0 && jr < n_s) {
        sfor<KM>([&](auto Kk) {
          constexpr int k = Kk;
          dstrow[k] = X[k];
        });
      }
    }
  }
}

// Inactive curve in a descent: the tile copies its rows unchanged.
template <int NX, typename T, int W>
__device__ __forceinline__ void tile_copy(const KernelArgs<T>& a, const CurveDev& cd, int j0,
                                          int tile, double* red) {
  constexpr int KM = (NX - 1) / 3 + 1;
  constexpr int ROWS = 64 * W;
  const int t = threadIdx.x;
  const int jr = j0 - 1 + t;
  const bool interior = (jr >= 1) && (jr <= cd.n_s - 2);
  const bool owned = interior && (t >= 1) && (t <= ROWS - 2);
  const bool pinned = (jr == 0 || jr == cd.n_s - 1) && jr >= 0 && jr < cd.n_s;
  if (owned || pinned) {
    const cplx<T>* s = a.in + cd.off + (long long)jr * KM;
    cplx<T>* d = a.out + cd.off + (long long)jr * KM;
    for (int k = 0; k < KM; ++k) d[k] = s[k];
  }
  reduce_partials<W>(0.0, 0.0, 0.0, red, a.partials + 3ll * tile);
}

}  // namespace ksc
