// Fused per-tile evaluation restricted to the inversion-symmetric subspace,
// u(-x) = -u(x) (the inversion operator of the paper's symmetry-preservation
// subsection, eq. reflection).  The residual and the adjoint commute with the
// inversion, so the descent (eq. KSE_G) keeps a curve that starts in the
// subspace inside it, and the gradient of J^2 restricted to the subspace is
// the restriction of the full gradient.
//
// In the subspace u_hat_k = i b_k with real b_k (k = 1..K, u_hat_0 = 0), so a
// state row is K reals and
//   u(x)   = -2 sum_k b_k sin(q_k x)        (a sine series),
//   u^2    is even: a cosine series, N_hat_k real,
//   r_hat  = i rho_k,  rho_k = -g (b_{j+1} - b_{j-1}) / (2 dsigma) + A_k b_k - q_k N_hat_k / 2,
//   r_x    = -2 sum_k q_k rho_k cos(q_k x),
//   u r_x  is odd:  Q_hat_k = i Im Q_hat_k,
//   L^dagger r = i (g (rho_{j+1} - rho_{j-1}) / (2 dsigma) + Im Q_hat_k + A_k rho_k).
// With m = N_x / 2 samples per half period every transform is a DST-I or
// DCT-I of length m (ksc_sym.hpp), so a row
// costs about half the flops of the full space and moves half the bytes.
//
// Tiles, staging, the boundary-row edge workspace and the per-wave partial
// sums are those of the full-space kernel (ksc_tile.hpp); rows are K reals
// instead of K+1 complex values.
#pragma once

#include "ksc_sym.hpp"
#include "ksc_tile.hpp"

namespace ksc {

// One lane per row whenever the half-period samples of a row fit (m reals of
// the field kept for the adjoint plus m of transform work space).
template <int NX, typename T>
constexpr bool odd_supported() {
  return (NX / 2) * int(sizeof(T)) <= 512 && (NX - 1) / 3 >= 1;
}

template <int NX, typename T, int W, int MODE>
__device__ __forceinline__ void tile_body_odd(const KernelArgs<T>& a, const CurveDev& cd, int c,
                                              int j0, int tile, T* buf) {
  constexpr int K = (NX - 1) / 3;  // sine modes k = 1..K, element k-1 of a row
  constexpr int M2 = NX / 2;       // samples x_0 .. x_{m-1} of the half period
  constexpr int ROWS = 64 * W;     // rows per tile
  constexpr int BR = ROWS + 2;     // staged rows: j0-1 .. j0+ROWS
  constexpr int E = 16 / int(sizeof(T));
  const int t = threadIdx.x;
  const int n_s = cd.n_s;
  const int jr = j0 + t;
  const bool interior = (jr >= 1) && (jr <= n_s - 2);
  const T* __restrict__ gin = reinterpret_cast<const T*>(a.in);

  // LDS row-major: staged row b (= state row j0-1+b) starts at buf[sh + b*K]
  const long long base = cd.off + (long long)(j0 - 1) * K;
  const int sh = int(((base % E) + E) % E);
  __syncthreads();  // the previous tile of a persistent workgroup is done with the LDS
  stage_block<T, ROWS, BR * K + E>(buf, gin, base, sh, BR * K + sh,
                                   cd.off + (long long)(j0 > 0 ? j0 - 1 : 0) * K,
                                   cd.off + (long long)min(n_s, j0 + ROWS + 1) * K);
  __syncthreads();
  T* __restrict__ rows = buf + sh;

  const T csj = interior ? a.cs[cd.row_off + jr] : T(0);
  const T q1s = T(cd.q1 * cd.q1);          // q_k^2 = k^2 q1^2
  const T qN1 = T(cd.q1 / (2.0 * NX));     // q_k N_hat_k / 2 = k qN1 * (2 C_k)
  constexpr T iN = T(1.0 / NX);            // Im Q_hat_k = -(2 F_k) / N

  // ---- u on x_0 .. x_{m-1} (u_m = 0) and the cosine coefficients of u^2 ----
  T u[M2];
  {
    T f[M2];
    sfor<M2>([&](auto Kk) {
      constexpr int k = Kk;
      if constexpr (k >= 1 && k <= K)
        f[k] = -rows[(t + 1) * K + (k - 1)];
      else
        f[k] = T(0);
    });
    dst1_x2<M2, M2, T>(f, u);  // 2 F_n with f = -b is u_n
  }
  T C2[K + 1];  // 2 C_k of u^2 = N N_hat_k
  {
    T g[M2 + 1];
    sfor<M2>([&](auto Nn) {
      constexpr int n = Nn;
      g[n] = u[n] * u[n];
    });
    g[M2] = T(0);
    dct1_x2<M2, K + 1, T>(g, C2);
  }

  // ---- rho_k = -cs (b_{j+1} - b_{j-1}) + A_k b_k - (q_k / (2N)) (2 C_k) ----
  // LDS reads in batches of CH modes, the next batch in flight during the
  // arithmetic of the current one (as in the full-space kernel).
  constexpr int CH = 8;
  constexpr int NCH = (K + CH - 1) / CH;
  T rowR = T(0), rowD = T(0);
  T R[K];
  {
    T q1s_r = q1s, qN1_r = qN1;
    __asm__ volatile("" : "+v"(q1s_r), "+v"(qN1_r));
    T xm[2][CH], x0[2][CH], xp[2][CH];
    auto load = [&](auto Cc, auto Bb) {
      constexpr int e0 = int(Cc) * CH;
      sfor<CH>([&](auto Ii) {
        constexpr int e = e0 + int(Ii);
        if constexpr (e < K) {
          xm[Bb][Ii] = rows[t * K + e];
          x0[Bb][Ii] = rows[(t + 1) * K + e];
          xp[Bb][Ii] = rows[(t + 2) * K + e];
        }
      });
    };
    load(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    sfor<NCH>([&](auto Cc) {
      constexpr int e0 = int(Cc) * CH;
      constexpr int B = int(Cc) % 2;
      if constexpr (int(Cc) + 1 < NCH)
        load(std::integral_constant<int, int(Cc) + 1>{}, std::integral_constant<int, 1 - B>{});
      __builtin_amdgcn_sched_barrier(0);
      sfor<CH>([&](auto Ii) {
        constexpr int i = Ii;
        constexpr int e = e0 + i;
        if constexpr (e < K) {
          constexpr int k = e + 1;
          const T db = xp[B][i] - xm[B][i];
          const T qn = T(k) * qN1_r;
          const T q2 = T(k * k) * q1s_r;
          const T Ak = fmaT(-q2, q2, q2);
          const T rho = fmaT(-csj, db, fmaT(Ak, x0[B][i], -qn * C2[k]));
          rowR = fmaT(rho, rho, rowR);
          if constexpr (MODE == MODE_J) rowD = fmaT(db, db, rowD);
          R[e] = interior ? rho : T(0);
        }
      });
      __asm__ volatile("" : "+v"(rowR), "+v"(rowD));
      __builtin_amdgcn_sched_barrier(0);
    });
  }
  // |r_hat_0|^2 + 2 sum_k |r_hat_k|^2 = 2 sum_k rho_k^2 (likewise for d/ds u)
  double pj = 0.0, pn = 0.0, pd = 0.0;
  if (interior) {
    const double rR = 2.0 * double(rowR);
    pj = a.wlD[cd.row_off + jr] * rR;
    if constexpr (MODE == MODE_J) {
      const double rD = 2.0 * double(rowD);
      pn = sqrt(rR * rD);
      pd = sqrt(rD);
    }
  }
  store_wave_partials<W, (MODE == MODE_J) ? 3 : 1>(pj, pn, pd, tile_partials(a, cd, c, tile, W));

  if constexpr (MODE != MODE_J) {
    // exchange residual rows through the staging buffer (outside rows read as 0)
    __syncthreads();
    sfor<K>([&](auto Ee) {
      constexpr int e = Ee;
      rows[(t + 1) * K + e] = R[e];
    });
    for (int i = t; i < 2 * K; i += ROWS) rows[(i < K) ? i : (BR - 2) * K + i] = T(0);
    __syncthreads();

    // ---- r_x on the half period, then Im Q_hat from the sine series of u r_x ----
    T G2[K + 1];  // 2 F_k of u r_x = -N Im Q_hat_k
    {
      T rx[M2];
      {
        T q1_r = T(cd.q1);
        __asm__ volatile("" : "+v"(q1_r));
        T g[M2 + 1];
        sfor<M2 + 1>([&](auto Kk) {
          constexpr int k = Kk;
          if constexpr (k >= 1 && k <= K)
            g[k] = -(T(k) * q1_r) * R[k - 1];
          else
            g[k] = T(0);
        });
        dct1_x2<M2, M2, T>(g, rx);  // 2 C_n with g = -q rho is r_x at x_n
      }
      T w[M2];
      sfor<M2>([&](auto Nn) {
        constexpr int n = Nn;
        w[n] = u[n] * rx[n];
      });
      dst1_x2<M2, K + 1, T>(w, G2);
    }

    // ---- L^dagger r (imaginary parts) = cs (rho_{j+1} - rho_{j-1}) + Im Q_hat + A rho ----
    const bool fix_lo = interior && t == 0 && jr - 1 >= 1;
    const bool fix_hi = interior && t == ROWS - 1 && jr + 1 <= n_s - 2;
    T D[K];
    {
      T q1s_d = q1s;
      __asm__ volatile("" : "+v"(q1s_d));
      T rm[2][CH], r0[2][CH], rp[2][CH];
      auto load_r = [&](auto Cc, auto Bb) {
        constexpr int e0 = int(Cc) * CH;
        sfor<CH>([&](auto Ii) {
          constexpr int e = e0 + int(Ii);
          if constexpr (e < K) {
            rm[Bb][Ii] = rows[t * K + e];
            r0[Bb][Ii] = rows[(t + 1) * K + e];
            rp[Bb][Ii] = rows[(t + 2) * K + e];
          }
        });
      };
      load_r(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
      sfor<NCH>([&](auto Cc) {
        constexpr int e0 = int(Cc) * CH;
        constexpr int B = int(Cc) % 2;
        if constexpr (int(Cc) + 1 < NCH)
          load_r(std::integral_constant<int, int(Cc) + 1>{}, std::integral_constant<int, 1 - B>{});
        __builtin_amdgcn_sched_barrier(0);
        sfor<CH>([&](auto Ii) {
          constexpr int i = Ii;
          constexpr int e = e0 + i;
          if constexpr (e < K) {
            constexpr int k = e + 1;
            const T q2 = T(k * k) * q1s_d;
            const T Ak = fmaT(-q2, q2, q2);
            D[e] = fmaT(csj, rp[B][i] - rm[B][i], fmaT(Ak, r0[B][i], -iN * G2[k]));
          }
        });
        __builtin_amdgcn_sched_barrier(0);
      });
    }
    if (fix_lo || fix_hi) {
      // edge workspace as reals: [tile][slot][partial adjoint | residual][km_max]
      T* e = reinterpret_cast<T*>(a.edge) + ((long long)tile * 4 + (fix_hi ? 2 : 0)) * a.km_max;
      sfor<K>([&](auto Ee) {
        constexpr int i = Ee;
        e[i] = D[i];
        e[a.km_max + i] = rows[(t + 1) * K + i];
      });
    }
    // ---- the tile's output rows, staged in LDS and written back coalesced ----
    // GRAD: 2 (2 w L) L^dagger (0 on the end rows);  STEP: the increment
    // -dtau L^dagger / (1 + dtau A^2) (0 on the end rows), added to the input.
    const long long obase = cd.off + (long long)j0 * K;
    const int osh = int(obase % E);
    T* __restrict__ orow = buf + osh + t * K;
    __syncthreads();  // every lane has read its residual neighbours
    if constexpr (MODE == MODE_GRAD) {
      const T sc = (a.scale != nullptr) ? T(a.scale[c]) : T(1);
      const T f2 = interior ? T(2) * (a.wlT[cd.row_off + jr] * sc) : T(0);
      sfor<K>([&](auto Ee) {
        constexpr int i = Ee;
        orow[i] = f2 * D[i];
      });
    } else {
      const T* __restrict__ pv = a.pre + cd.mode_off + 1;  // mode k = element + 1
      const T m = interior ? T(1) : T(0);
      sfor<K>([&](auto Ee) {
        constexpr int i = Ee;
        orow[i] = (m * pv[i]) * D[i];
      });
    }
    __syncthreads();
    flush_block<T, ROWS, ROWS * K + E, MODE == MODE_STEP>(
        reinterpret_cast<T*>(a.out), gin, buf, obase, osh, ROWS * K + osh, obase,
        cd.off + (long long)min(n_s, j0 + ROWS) * K);
  }
}

// Inactive curve in a descent: the tile copies its rows unchanged.
template <int NX, typename T, int W>
__device__ __forceinline__ void tile_copy_odd(const KernelArgs<T>& a, const CurveDev& cd, int c,
                                              int j0, int tile) {
  constexpr int K = (NX - 1) / 3;
  const int jr = j0 + int(threadIdx.x);
  if (jr < cd.n_s) {
    const T* s = reinterpret_cast<const T*>(a.in) + cd.off + (long long)jr * K;
    T* d = reinterpret_cast<T*>(a.out) + cd.off + (long long)jr * K;
    for (int k = 0; k < K; ++k) d[k] = s[k];
  }
  store_wave_partials<W, 1>(0.0, 0.0, 0.0, tile_partials(a, cd, c, tile, W));
}

}  // namespace ksc
