// Rows split over L lanes: the fused tile evaluation for grids whose row is
// too wide for one lane (N_x = 256 in FP32), with every row's transforms
// spread over L = sqrt(N_x) consecutive lanes so that a long curve fills the
// chip (a 8190-row curve at N_x = 256 gets 2048 waves, two per SIMD).
//
// Layout of one row over its L lanes (lane p = 0..L-1 of the row's group),
// with the half-length trick z_m = x_{2m} + i x_{2m+1}, m < M = N/2 = L Q,
// L = 2Q:
//   spectrum side: lane p holds the coefficients k = L k1 + p, k1 < Q;
//   sample side:   lane p = 2 m1 + h holds z_m for m = m1 + Q (j + Q h),
//                  j < Q.
// The M-point DFT splits as z_{m1 + Q m2} = sum_p w_L^{m2 p} w_M^{m1 p}
// sum_{k1} w_Q^{m1 k1} Z_{L k1 + p}: a Q-point FFT in each lane, a twiddle
// w_M^{m1 p}, a transpose of the row's Q x L block through LDS that gives
// lane (m1, h) the entries p = 2 pp + h of line m1, a Q-point FFT over pp in
// each lane (the even / odd half of the L-point DFT over p), and one radix-2
// step across the lane pair, E + w_L^j O and E - w_L^j O, with the partner's
// values from a DPP lane swap.  The forward transform runs the same steps in
// reverse.
//
// LDS banks: block entry (m1, q) sits at m1 (L + 2) + q.  The L lanes of a
// row then touch 16-byte groups on distinct banks both when each writes its
// own q of a line and when the pairs read their half-lines; in the state
// dtype the blocks of neighbouring rows are an odd multiple of 128 bytes
// apart, and so are the FP64 residual rows.
//
// Pass 0 (u = c2r(u_hat), N_hat = r2c(u^2), the residual) runs in FP64 as in
// the one-lane kernel; the residual rows are exchanged between neighbouring
// rows in FP64 as well, so that the adjoint's d/ds differences unrounded
// residuals.
#pragma once

#include "ksc_tile.hpp"

namespace ksc {

// LDS footprint (bytes) of the L-lane tile of R rows: staging rows (state
// dtype), residual rows (FP64), the transpose blocks (FP64, one per tile
// row) and the twiddle tables.
constexpr int lanes_stage_bytes(int KM, int R, int esize) {
  return ((((R + 2) * KM + 2) * 2 * esize) + 15) / 16 * 16;
}
// Padded strides (complex FP64 entries): residual rows and transpose blocks
// (Q lines of L entries, each padded by 2).
constexpr int lanes_rstride(int KM) { return (KM + 7) / 16 * 16 + 8; }
constexpr int lanes_bstride(int NX, int L) { return (NX / 2 / L) * (L + 2); }
// Twiddle tables: e^{2 pi i k / N} for k < N/2 and e^{2 pi i m1 p / M}, in
// FP64 and in the state dtype.
constexpr int lanes_lds_bytes(int NX, int KM, int R, int L, int esize) {
  return lanes_stage_bytes(KM, R, esize) + (R + 2) * lanes_rstride(KM) * 16 +
         R * lanes_bstride(NX, L) * 16 + NX * (16 + 8);
}

namespace lanes_detail {

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cplx<T>{fmaT(a.r, b.r, -a.i * b.i), fmaT(a.r, b.i, a.i * b.r)};
}
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {  // a conj(b)
  return cplx<T>{fmaT(a.r, b.r, a.i * b.i), fmaT(a.i, b.r, -a.r * b.i)};
}

// The L lanes of a row sit in one wave, and the LDS performs a wave's
// accesses in the order they were issued, so the transposes of a row need no
// workgroup barrier: only the compiler must keep each access on its side.
__device__ __forceinline__ void row_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace lanes_detail

// Band-limited spectrum -> this lane's samples (layout above).  X(k) returns
// coefficient k (0 for k > K; Im of mode 0 ignored); tb: the row's transpose
// block in LDS; tw: e^{2 pi i k / N}, k < N/2, and tw2: e^{2 pi i m1 p / M}
// at m1 L + p, both in LDS in the arithmetic type.  All L lanes of the row
// call it together.
template <int N, int L, typename T, class XF>
__device__ __forceinline__ void c2r_lanes_split(XF X, int p, cplx<T>* tb, const cplx<T>* tw,
                                                const cplx<T>* tw2, T (&out)[N / L]) {
  using namespace lanes_detail;
  constexpr int M = N / 2, Q = M / L;
  static_assert(L == 2 * Q && 64 % L == 0, "split layout: L = 2Q lanes in one wave");
  T zr[Q], zi[Q];
  sfor<Q>([&](auto K1) {
    constexpr int k1 = K1;
    const int k = L * k1 + p;
    const cplx<T> a = X(k);
    cplx<T> b = X(M - k);  // zero for k = 0 (coefficient M is above K)
    b.i = -b.i;            // conj
    const cplx<T> E{a.r + b.r, a.i + b.i};
    const cplx<T> O = cmul(cplx<T>{a.r - b.r, a.i - b.i}, tw[k]);
    zr[k1] = E.r - O.i;  // Z = E + i O
    zi[k1] = E.i + O.r;
  });
  fft_c<Q, +1, T>(zr, zi);
  cplx<T>* const tw_ = tb + p;  // entries (m1, p), m1 < Q
  sfor<Q>([&](auto M1) {
    constexpr int m1 = M1;
    tw_[m1 * (L + 2)] = cmul(cplx<T>{zr[m1], zi[m1]}, tw2[m1 * L + p]);
  });
  row_sync();
  const int h = p & 1;
  const cplx<T>* const tr_ = tb + (p >> 1) * (L + 2) + h;  // entries (p / 2, 2 pp + h)
  T vr[Q], vi[Q];
  sfor<Q>([&](auto Pp) {
    constexpr int pp = Pp;
    const cplx<T> v = tr_[2 * pp];
    vr[pp] = v.r;
    vi[pp] = v.i;
  });
  row_sync();
  fft_c<Q, +1, T>(vr, vi);  // E (h = 0) or O (h = 1) at j
  const T sg = h ? T(-1) : T(1);
  sfor<Q>([&](auto J) {
    constexpr int j = J;
    constexpr CS c = cx_unit(j, L);
    // own value E (h = 0) or w^j O (h = 1); the pair forms E + w^j O on
    // lane 0 and E - w^j O on lane 1
    T orr = vr[j], oi = vi[j];
    if constexpr (j != 0) {
      const T gr = fmaT(T(c.c), vr[j], -T(c.s) * vi[j]);
      const T gi = fmaT(T(c.c), vi[j], T(c.s) * vr[j]);
      orr = h ? gr : orr;
      oi = h ? gi : oi;
    }
    out[2 * j] = fmaT(sg, orr, pair_swap(orr));
    out[2 * j + 1] = fmaT(sg, oi, pair_swap(oi));
  });
}

// This lane's samples -> its kept coefficients, unnormalized and doubled:
//   X_k = 2 sum_n x_n e^{-2 pi i k n / N} for k = L i + p <= K (X[i]).
template <int N, int KM, int L, typename T>
__device__ __forceinline__ void r2c_lanes_split(const T (&in)[N / L], int p, cplx<T>* tb,
                                                const cplx<T>* tw, const cplx<T>* tw2,
                                                cplx<T> (&X)[(KM + L - 1) / L]) {
  using namespace lanes_detail;
  constexpr int M = N / 2, Q = M / L, KL = (KM + L - 1) / L;
  static_assert(L == 2 * Q && KL <= Q, "split layout");
  const int h = p & 1;
  const T sg = h ? T(-1) : T(1);
  T vr[Q], vi[Q];
  sfor<Q>([&](auto J) {
    constexpr int j = J;
    constexpr CS c = cx_unit(j, L);
    // lane 0: a + b, lane 1: (a - b) w^{-j}, with a = z_{m1 + Q j} (lane 0)
    // and b = z_{m1 + Q (j + Q)} (lane 1)
    const T ar = in[2 * j], ai = in[2 * j + 1];
    const T tr = fmaT(sg, ar, pair_swap(ar)), ti = fmaT(sg, ai, pair_swap(ai));
    vr[j] = tr;
    vi[j] = ti;
    if constexpr (j != 0) {
      const T gr = fmaT(T(c.c), tr, T(c.s) * ti);
      const T gi = fmaT(T(c.c), ti, -T(c.s) * tr);
      vr[j] = h ? gr : tr;
      vi[j] = h ? gi : ti;
    }
  });
  fft_c<Q, -1, T>(vr, vi);  // entries (p / 2, 2 pp + h)
  cplx<T>* const tr_ = tb + (p >> 1) * (L + 2) + h;
  sfor<Q>([&](auto Pp) {
    constexpr int pp = Pp;
    tr_[2 * pp] = cplx<T>{vr[pp], vi[pp]};
  });
  row_sync();
  T zr[Q], zi[Q];
  const cplx<T>* const tw_ = tb + p;  // entries (m1, p)
  sfor<Q>([&](auto M1) {
    constexpr int mm = M1;
    const cplx<T> w = cmulc(tw_[mm * (L + 2)], tw2[mm * L + p]);
    zr[mm] = w.r;
    zi[mm] = w.i;
  });
  row_sync();
  fft_c<Q, -1, T>(zr, zi);  // Z_{L k1 + p} at k1
  sfor<Q>([&](auto K1) {
    constexpr int k1 = K1;
    tb[L * k1 + p] = cplx<T>{zr[k1], zi[k1]};
  });
  row_sync();
  sfor<KL>([&](auto I) {
    constexpr int i = I;
    const int k = L * i + p;
    const cplx<T> zb = tb[(M - k) % M];  // Z_{M-k}
    const T Dr = zr[i] + zb.r, Di = zi[i] - zb.i;
    const cplx<T> S{zr[i] - zb.r, zi[i] + zb.i};
    const cplx<T> V = cmulc(S, tw[k]);  // e^{-2 pi i k / N} S
    X[i] = cplx<T>{Dr + V.i, Di - V.r};
  });
  row_sync();
}

// The fused tile evaluation (as tile_body in ksc_tile.hpp: staging, pass 0 in
// FP64, the residual and its partial sums, the residual exchange, pass 1, the
// adjoint, the output) with the R = 64W/L rows of the tile spread over L
// lanes each.
template <int NX, typename T, int W, int MODE, int L>
__device__ __forceinline__ void tile_body_lanes(const KernelArgs<T>& a, const CurveDev& cd, int c,
                                                int j0, int tile, cplx<T>* buf) {
  using namespace lanes_detail;
  constexpr int KM = (NX - 1) / 3 + 1;
  constexpr int KL = (KM + L - 1) / L;  // modes per lane
  constexpr int NT = 64 * W;            // lanes
  constexpr int ROWS = NT / L;          // rows per tile
  constexpr int BR = ROWS + 2;          // staged rows: j0-1 .. j0+ROWS
  constexpr int E = 16 / int(sizeof(cplx<T>));
  constexpr int M = NX / 2;
  constexpr int NS = NX / L;            // samples per lane
  static_assert(L * L == NX, "L = sqrt(N_x) lanes per row");
  const int t = threadIdx.x / L;        // row within the tile
  const int p = threadIdx.x % L;
  const int n_s = cd.n_s;
  const int jr = j0 + t;
  const bool interior = (jr >= 1) && (jr <= n_s - 2);

  // LDS: staging rows (dtype T), residual rows (FP64), transpose blocks
  // (FP64), twiddles e^{2 pi i j / N} and e^{2 pi i m1 p / M} (FP64, then the
  // same rounded to the state dtype for pass 1)
  constexpr int RS = lanes_rstride(KM), BS = lanes_bstride(NX, L);
  cplx<double>* r64 = reinterpret_cast<cplx<double>*>(
      reinterpret_cast<char*>(buf) + lanes_stage_bytes(KM, ROWS, int(sizeof(T))));
  cplx<double>* tbd = r64 + BR * RS + t * BS;  // this row's transpose block
  cplx<double>* tw = r64 + BR * RS + ROWS * BS;
  cplx<double>* tw2 = tw + M;
  cplx<T>* twT = reinterpret_cast<cplx<T>*>(tw2 + M);
  cplx<T>* tw2T = twT + M;

  const long long base = cd.off + (long long)(j0 - 1) * KM;
  const int sh = int(((base % E) + E) % E);
  __syncthreads();  // the previous tile of a persistent workgroup is done with the LDS
  for (int j = threadIdx.x; j < M; j += NT) {
    double s, co;
    sincospi(2.0 * j / NX, &s, &co);
    tw[j] = cplx<double>{co, s};
    twT[j] = cplx<T>{T(co), T(s)};
  }
  for (int j = threadIdx.x; j < M; j += NT) {
    double s, co;
    sincospi(2.0 * ((j / L) * (j % L)) / M, &s, &co);
    tw2[j] = cplx<double>{co, s};
    tw2T[j] = cplx<T>{T(co), T(s)};
  }
  stage_block<cplx<T>, NT, BR * KM + E>(buf, a.in, base, sh, BR * KM + sh,
                                        cd.off + (long long)(j0 > 0 ? j0 - 1 : 0) * KM,
                                        cd.off + (long long)min(n_s, j0 + ROWS + 1) * KM);
  __syncthreads();
  cplx<T>* __restrict__ rows = buf + sh;
  const cplx<T>* __restrict__ my = rows + (t + 1) * KM;

  const T x0i = my[0].i;  // raw Im u_hat_0 (lane 0 of the row uses it)
  const T csj = interior ? a.cs[cd.row_off + jr] : T(0);

  // ---- pass 0 in FP64: u, S0 = r2c(u^2) = 2 N_x N_hat of the lane's modes ----
  T u[MODE == MODE_J ? 1 : NS];
  cplx<double> S0[KL];
  {
    double v[NS];
    c2r_lanes_split<NX, L, double>(
        [&](int k) {
          cplx<double> x{0.0, 0.0};
          if (k < KM) {
            const cplx<T> y = my[k];
            x = cplx<double>{double(y.r), k == 0 ? 0.0 : double(y.i)};
          }
          return x;
        },
        p, tbd, tw, tw2, v);
    if constexpr (MODE != MODE_J) {
      sfor<NS>([&](auto Nn) {
        constexpr int n = Nn;
        u[n] = T(v[n]);
      });
    }
    sfor<NS>([&](auto Nn) {
      constexpr int n = Nn;
      v[n] = v[n] * v[n];
    });
    r2c_lanes_split<NX, KM, L, double>(v, p, tbd, tw, tw2, S0);
  }

  // ---- residual of the lane's modes (FP64), its row sums ----
  double rowR = 0.0, rowD = 0.0;  // sum of c_k |r_k|^2, c_k |du_k|^2 over the lane's modes
  cplx<double> R[KL];
  {
    const double q1 = cd.q1, qN1 = cd.q1 / (4.0 * NX), cs_r = double(csj);
    sfor<KL>([&](auto I) {
      constexpr int i = I;
      const int k = L * i + p;
      double rr = 0.0, ri = 0.0, dr = 0.0, di = 0.0;
      if (k < KM) {
        const cplx<T> xm = rows[t * KM + k], x0 = my[k], xp = rows[(t + 2) * KM + k];
        dr = double(xp.r) - double(xm.r);
        di = (k == 0) ? 0.0 : double(xp.i) - double(xm.i);
        const double qk = double(k) * q1;
        const double q2 = qk * qk;
        const double Ak = fmaT(-q2, q2, q2);
        const double qn = double(k) * qN1;
        rr = fmaT(-cs_r, dr, fmaT(Ak, double(x0.r), qn * S0[i].i));
        ri = (k == 0) ? 0.0 : fmaT(-cs_r, di, fmaT(Ak, double(x0.i), -qn * S0[i].r));
      }
      if (!interior) rr = ri = 0.0;
      R[i] = cplx<double>{rr, ri};
      const double ck = (k == 0) ? 1.0 : 2.0;
      rowR = fmaT(ck, fmaT(rr, rr, ri * ri), rowR);
      if constexpr (MODE == MODE_J) rowD = fmaT(ck, fmaT(dr, dr, di * di), rowD);
    });
    double pj = 0.0, pn = 0.0, pd = 0.0;
    const double wl = interior ? a.wlD[cd.row_off + jr] : 0.0;
    pj = wl * rowR;
    if constexpr (MODE == MODE_J) {
      // J_arc needs whole-row norms: add the L lanes' shares
      double rRrow = rowR, rDrow = rowD;
      sfor<ilog2(L)>([&](auto B) {
        constexpr int b = 1 << int(B);
        rRrow += __shfl_xor(rRrow, b, 64);
        rDrow += __shfl_xor(rDrow, b, 64);
      });
      if (interior && p == 0) {
        pn = sqrt(rRrow * rDrow);
        pd = sqrt(rDrow);
      }
    }
    store_wave_partials<W, (MODE == MODE_J) ? 3 : 1>(pj, pn, pd, tile_partials(a, cd, c, tile, W));
  }
  if constexpr (MODE != MODE_J) {
  // ---- exchange residual rows (FP64) ----
  sfor<KL>([&](auto I) {
    constexpr int i = I;
    const int k = L * i + p;
    if (k < KM) r64[(t + 1) * RS + k] = R[i];
  });
  for (int i = threadIdx.x; i < 2 * KM; i += NT)
    r64[(i < KM) ? i : (BR - 1) * RS + i - KM] = cplx<double>{0.0, 0.0};
  __syncthreads();

  // ---- pass 1 in the state dtype: S = r2c(u * c2r(i q r_hat / (2 N_x))) = Q_hat ----
  cplx<T> S[KL];
  {
    const cplx<double>* rme = r64 + (t + 1) * RS;
    const T qY1 = T(cd.q1 / (2.0 * NX));
    // the row's block in the state dtype, packed at BS entries of that type
    // (an odd multiple of 128 bytes in FP32)
    cplx<T>* tbt = reinterpret_cast<cplx<T>*>(r64 + BR * RS) + t * BS;
    T v[NS];
    c2r_lanes_split<NX, L, T>(
        [&](int k) {
          cplx<T> x{T(0), T(0)};
          if (k < KM) {
            const cplx<double> y = rme[k];
            const T qk = T(k) * qY1;
            x = cplx<T>{-qk * T(y.i), qk * T(y.r)};
          }
          return x;
        },
        p, tbt, twT, tw2T, v);
    sfor<NS>([&](auto Nn) {
      constexpr int n = Nn;
      v[n] = u[n] * v[n];
    });
    r2c_lanes_split<NX, KM, L, T>(v, p, tbt, twT, tw2T, S);
  }

  // ---- L^dagger r = g (r_{j+1} - r_{j-1}) / (2 dsigma) + Q_hat + A r_hat ----
  const bool fix_lo = interior && t == 0 && jr - 1 >= 1;
  const bool fix_hi = interior && t == ROWS - 1 && jr + 1 <= n_s - 2;
  cplx<T> D[KL];
  {
    const double q1 = cd.q1, cs_r = double(csj);
    sfor<KL>([&](auto I) {
      constexpr int i = I;
      const int k = L * i + p;
      D[i] = cplx<T>{T(0), T(0)};
      if (k < KM) {
        const cplx<double> rm = r64[t * RS + k], rp = r64[(t + 2) * RS + k];
        const double qk = double(k) * q1;
        const double q2 = qk * qk;
        const double Ak = fmaT(-q2, q2, q2);
        const double dr = fmaT(cs_r, rp.r - rm.r, fmaT(Ak, R[i].r, double(S[i].r)));
        const double di = fmaT(cs_r, rp.i - rm.i, fmaT(Ak, R[i].i, double(S[i].i)));
        D[i] = cplx<T>{T(dr), (k == 0) ? T(0) : T(di)};
      }
    });
  }
  if (fix_lo || fix_hi) {
    cplx<T>* e = a.edge + ((long long)tile * 4 + (fix_hi ? 2 : 0)) * a.km_max;
    sfor<KL>([&](auto I) {
      constexpr int i = I;
      const int k = L * i + p;
      if (k < KM) {
        e[k] = D[i];
        e[a.km_max + k] = cplx<T>{T(R[i].r), T(R[i].i)};
      }
    });
  }
  // ---- the tile's output rows, staged in LDS and written back coalesced ----
  const long long obase = cd.off + (long long)j0 * KM;
  const int osh = int(obase % E);
  cplx<T>* __restrict__ orow = buf + osh + t * KM;
  __syncthreads();  // every lane has read its state rows
  if constexpr (MODE == MODE_GRAD) {
    const T sc = (a.scale != nullptr) ? T(a.scale[c]) : T(1);
    const T f0 = interior ? a.wlT[cd.row_off + jr] * sc : T(0);
    sfor<KL>([&](auto I) {
      constexpr int i = I;
      const int k = L * i + p;
      const T f = (k == 0) ? f0 : T(2) * f0;  // c_0 = 1, c_k = 2
      if (k < KM) orow[k] = cplx<T>{f * D[i].r, f * D[i].i};
    });
  } else {
    const T* __restrict__ pv = a.pre + cd.mode_off;
    const T m = interior ? T(1) : T(0);
    sfor<KL>([&](auto I) {
      constexpr int i = I;
      const int k = L * i + p;
      if (k < KM) {
        const T f = m * pv[k];
        orow[k] = cplx<T>{f * D[i].r, (k == 0) ? -x0i : f * D[i].i};
      }
    });
  }
  __syncthreads();
  flush_block<cplx<T>, NT, ROWS * KM + E, MODE == MODE_STEP>(
      a.out, a.in, buf, obase, osh, ROWS * KM + osh, obase,
      cd.off + (long long)min(n_s, j0 + ROWS) * KM);
  }  // MODE != MODE_J
}

}  // namespace ksc
