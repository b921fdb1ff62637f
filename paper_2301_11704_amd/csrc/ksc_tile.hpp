// Fused per-tile evaluation of the KS connecting-curve residual, the cost J^2,
// the adjoint L^dagger(u; r) and either the Euclidean gradient of J^2 or one
// semi-implicit descent step (Ashtari & Schneider, arXiv:2301.11704: residual
// eq. KSE_residual, cost eq. cost_function_general, adjoint Sec. V.A and
// Appendix A, descent eq. KSE_G with the semi-implicit Euler of Sec. V.C.3).
//
// Work decomposition: a workgroup of 64*W lanes owns the rows j0 .. j0+64W-1
// of one curve, one row per lane; tiles do not overlap, so every row's
// transforms are computed exactly once.  The state rows j0-1 .. j0+64W are
// staged in LDS (mode-major: lane-consecutive accesses hit consecutive
// banks) for the d/ds of the residual; the residual rows are then exchanged
// through the same buffer for the d/ds of the adjoint.  The two rows at a
// tile boundary lack one neighbouring residual row: their lanes store the
// partial adjoint and their residual in a small edge workspace, and the post
// kernel (which runs after every fused launch anyway to reduce the cost)
// adds the missing term and writes those rows.  (Finishing them inside the
// fused kernel by the last workgroup of a curve needs a device-scope release
// per workgroup, i.e. an L2 write-back on every XCD holding the fresh output;
// measured, that doubled the kernel time.)
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
  double q1;           // 2 pi / L: q_k = k q1
};

struct TileDev {
  int curve;
  int j0;  // first row of the tile
};

template <typename T>
struct KernelArgs {
  const cplx<T>* __restrict__ in;     // state
  cplx<T>* __restrict__ out;          // gradient (MODE_GRAD) or next state (MODE_STEP)
  const CurveDev* __restrict__ curves;
  const TileDev* __restrict__ tiles;
  const T* __restrict__ cs;           // per row: g_j / (2 dsigma), 0 on the end rows
  const T* __restrict__ wlT;          // per row: 2 w_j L (run precision)
  const double* __restrict__ wlD;     // per row: w_j L (FP64, cost reduction)
  const T* __restrict__ pre;          // per mode: -dtau / (1 + dtau A^2)   (MODE_STEP)
  const double* __restrict__ scale;   // per curve gradient scale, nullable
  const unsigned char* __restrict__ active;  // per curve, nullable
  double* __restrict__ partials;      // per tile and wave: J^2, J_arc numerator, J_arc denominator
  int part_stride;                    // > 0: curve c's slots start at c * part_stride; 0: tile order
  cplx<T>* __restrict__ edge;         // per tile: [2 slots][partial adjoint, residual][km_max]
  int km_max;                         // stride of the edge workspace
  int n_tiles;
  int tile_base;
};

// One DPP lane move of an FP64 value (both 32-bit halves); lanes outside
// ROW_MASK or reading an invalid source get 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes of a wave with a fixed DPP pattern (inclusive scan
// within 16-lane rows, then row broadcasts); lane 63 ends with the total.
// The order of the additions is fixed, so the result is deterministic.
__device__ __forceinline__ double wave_sum_to_lane63(double v) {
  v += dpp_f64<0x111, 0xf>(v);  // row_shr:1
  v += dpp_f64<0x112, 0xf>(v);  // row_shr:2
  v += dpp_f64<0x114, 0xf>(v);  // row_shr:4
  v += dpp_f64<0x118, 0xf>(v);  // row_shr:8
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// First partial-sum slot of a tile: per curve at a fixed stride (so the post
// kernel finds a curve's slots without reading its descriptor), or in tile
// order when that layout would waste too much memory.
template <typename T>
__device__ __forceinline__ double* tile_partials(const KernelArgs<T>& a, const CurveDev& cd, int c,
                                                 int tile, int W) {
  const long long slot = (a.part_stride > 0)
                             ? (long long)c * a.part_stride + (long long)(tile - cd.tile_begin) * W
                             : (long long)tile * W;
  return a.partials + 3 * slot;
}

// Each wave stores its partial sums (J^2, J_arc numerator, denominator) of
// the tile; the post kernel adds them in a fixed order.
template <int W, int NV>
__device__ __forceinline__ void store_wave_partials(double a, double b, double c, double* dst) {
  a = wave_sum_to_lane63(a);
  if constexpr (NV > 1) {
    b = wave_sum_to_lane63(b);
    c = wave_sum_to_lane63(c);
  }
  if ((threadIdx.x & 63) == 63) {
    double* d = dst + 3 * (threadIdx.x >> 6);
    d[0] = a;
    d[1] = (NV > 1) ? b : 0.0;
    d[2] = (NV > 1) ? c : 0.0;
  }
}

// 16-byte vector of the state's scalar type (four FP32 or two FP64 values).
template <typename T>
struct alignas(16) vec16 {
  T v[4 / (sizeof(T) / 4)];
};

// State elements as seen by the staging copies: a complex Fourier
// coefficient (full space) or one real coefficient (odd subspace), held in a
// 16-byte chunk of scalars.
template <typename V>
struct elem {
  using S = V;
  static constexpr int n = 1;  // scalars per element
  __device__ __forceinline__ static void put(vec16<S>& w, int h, V x) { w.v[h] = x; }
  __device__ __forceinline__ static V get(const vec16<S>& w, int h) { return w.v[h]; }
  __device__ __forceinline__ static V zero() { return V(0); }
};
template <typename T>
struct elem<cplx<T>> {
  using S = T;
  static constexpr int n = 2;
  __device__ __forceinline__ static void put(vec16<S>& w, int h, cplx<T> x) {
    w.v[2 * h] = x.r;
    w.v[2 * h + 1] = x.i;
  }
  __device__ __forceinline__ static cplx<T> get(const vec16<S>& w, int h) {
    return cplx<T>{w.v[2 * h], w.v[2 * h + 1]};
  }
  __device__ __forceinline__ static cplx<T> zero() { return cplx<T>{T(0), T(0)}; }
};

// Copy the contiguous complex range [G_lo, G_hi) of global memory `g` into LDS
// `buf`, global index G landing at buf[G - base + shift]; everything else of
// the n elements starting at buf[0] is zero-filled.  `base - shift` is
// 16-byte aligned, so whole 16-byte chunks move with one load and one LDS
// store; a chunk straddling the valid range is moved element by element.
template <typename V, int NT, int NMAX>
__device__ __forceinline__ void stage_block(V* __restrict__ buf, const V* __restrict__ g,
                                            long long base, int shift, int n, long long G_lo,
                                            long long G_hi) {
  using T = typename elem<V>::S;
  constexpr int E = 16 / int(sizeof(V));  // elements per chunk
  constexpr int NQ = (NMAX + E * NT - 1) / (E * NT);  // chunks per thread, at most
  const long long G0 = base - shift;             // global index of buf[0]
  const int nq = (n + E - 1) / E;
  // (opaque thread index: the per-chunk offsets are formed here, not hoisted
  // out of the caller's tile loop where they would stay live)
  int tid = threadIdx.x;
  __asm__ volatile("" : "+v"(tid));
  vec16<T> w[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {  // every load in flight before the first LDS store
    const int q = tid + i * NT;
    const long long G = G0 + (long long)q * E;
    if (q < nq && G >= G_lo && G + E <= G_hi) {
      w[i] = *reinterpret_cast<const vec16<T>*>(g + G);
    } else {
#pragma unroll
      for (int h = 0; h < E; ++h) {
        const bool ok = q < nq && (G + h >= G_lo) && (G + h < G_hi);
        elem<V>::put(w[i], h, ok ? g[G + h] : elem<V>::zero());
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = tid + i * NT;
    if (q < nq) reinterpret_cast<vec16<T>*>(buf)[q] = w[i];
  }
}

// Write LDS rows back: global index G in [G_lo, G_hi) receives buf[G - base + shift]
// (ADD: plus the input g_in[G], the state update of a descent step).  Chunks
// are 16-byte aligned in both spaces; a chunk straddling the range is written
// element by element so no row outside [G_lo, G_hi) is touched.  A thread's
// chunks go in groups of GB: every read of a group (LDS, and global with ADD)
// is issued before its first store, so their latencies overlap.
template <typename V, int NT, int NMAX, bool ADD>
__device__ __forceinline__ void flush_block(V* __restrict__ gout, const V* __restrict__ gin,
                                            const V* __restrict__ buf, long long base,
                                            int shift, int n, long long G_lo, long long G_hi) {
  using T = typename elem<V>::S;
  constexpr int E = 16 / int(sizeof(V));
  constexpr int NQ = (NMAX + E * NT - 1) / (E * NT);  // chunks per thread, at most
  constexpr int GB = 8;
  const long long G0 = base - shift;
  const int nq = (n + E - 1) / E;
  int tid = threadIdx.x;  // (opaque, as in stage_block)
  __asm__ volatile("" : "+v"(tid));
#pragma unroll 1
  for (int i0 = 0; i0 < NQ; i0 += GB) {
    vec16<T> w[GB];
#pragma unroll
    for (int i = 0; i < GB; ++i) {
      const int q = tid + (i0 + i) * NT;
      if (q < nq) w[i] = reinterpret_cast<const vec16<T>*>(buf)[q];
    }
    if constexpr (ADD) {
      vec16<T> x[GB];
#pragma unroll
      for (int i = 0; i < GB; ++i) {
        const int q = tid + (i0 + i) * NT;
        const long long G = G0 + (long long)q * E;
        if (q < nq && G >= G_lo && G + E <= G_hi) {
          x[i] = *reinterpret_cast<const vec16<T>*>(gin + G);
        } else {
#pragma unroll
          for (int h = 0; h < E; ++h) {
            const bool ok = q < nq && (G + h >= G_lo) && (G + h < G_hi);
            elem<V>::put(x[i], h, ok ? gin[G + h] : elem<V>::zero());
          }
        }
      }
#pragma unroll
      for (int i = 0; i < GB; ++i)
#pragma unroll
        for (int h = 0; h < E * elem<V>::n; ++h) w[i].v[h] += x[i].v[h];
    }
#pragma unroll
    for (int i = 0; i < GB; ++i) {
      const int q = tid + (i0 + i) * NT;
      const long long G = G0 + (long long)q * E;
      if (q < nq && G >= G_lo && G + E <= G_hi) {
        // streaming store: the output is not read again by this kernel
        typedef float f4_t __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(*reinterpret_cast<const f4_t*>(&w[i]),
                                    reinterpret_cast<f4_t*>(gout + G));
      } else if (q < nq) {
#pragma unroll
        for (int h = 0; h < E; ++h)
          if (G + h >= G_lo && G + h < G_hi) gout[G + h] = elem<V>::get(w[i], h);
      }
    }
  }
}

// Samples of the physical field u that a lane parks in LDS between the two
// passes of the gradient (the rest stay in registers).  Only where pass 0's
// FP64 transform work space would not fit next to the whole field: N_x = 128
// with one FP32 row per lane (64 of its 128 samples).  The host adds
// lanes * u_stash * esize bytes to the staging buffer's LDS.
constexpr int u_stash_n(int nx, int esize) {
  return (nx == 128 && esize == 4) ? 64 : 0;
}
template <int NX, typename T>
constexpr int u_stash() {
  return u_stash_n(NX, int(sizeof(T)));
}

template <int NX, typename T, int W, int MODE>
__device__ __forceinline__ void tile_body(const KernelArgs<T>& a, const CurveDev& cd, int c,
                                          int j0, int tile, cplx<T>* buf, double* red) {
  constexpr int KM = (NX - 1) / 3 + 1;
  constexpr int ROWS = 64 * W;   // rows per tile
  constexpr int BR = ROWS + 2;   // staged rows: j0-1 .. j0+ROWS
  constexpr int E = 16 / int(sizeof(cplx<T>));
  const int t = threadIdx.x;
  const int n_s = cd.n_s;
  const int jr = j0 + t;
  const bool inrow = jr < n_s;
  const bool interior = (jr >= 1) && (jr <= n_s - 2);

  // LDS row-major: staged row b (= state row j0-1+b) starts at buf[sh + b*KM];
  // sh aligns the block so that 16-byte chunks line up with global memory.
  const long long base = cd.off + (long long)(j0 - 1) * KM;
  const int sh = int(((base % E) + E) % E);
  __syncthreads();  // the previous tile of a persistent workgroup is done with the LDS
  stage_block<cplx<T>, ROWS, BR * KM + E>(buf, a.in, base, sh, BR * KM + sh,
                       cd.off + (long long)(j0 > 0 ? j0 - 1 : 0) * KM,
                       cd.off + (long long)min(n_s, j0 + ROWS + 1) * KM);
  __syncthreads();
  cplx<T>* __restrict__ rows = buf + sh;

  const T x0i = rows[(t + 1) * KM].i;  // raw Im u_hat_0 (zeroed in the output)
  const T csj = interior ? a.cs[cd.row_off + jr] : T(0);
  const T q1s = T(cd.q1 * cd.q1);                  // q1^2:  q_k^2 = k^2 q1^2
  const T qY1 = T(cd.q1 / (2.0 * NX));             // q1 / (2 N_x): Q_hat = r2c/(2 N_x)
  constexpr int CH = 5;                            // modes per LDS read batch (15 reads)
  constexpr int NCH = (KM + CH - 1) / CH;

  // ---- pass 0, in FP64 whatever the state dtype: u = c2r(u_hat), the
  // nonlinear term S = r2c(u * u) = 2 N_x N_hat and the residual.  In FP32 the
  // rounding of N_hat differs from row to row and the adjoint's d/ds below
  // differences neighbouring residual rows with a weight that grows like N_s;
  // FP64 here (the same issue rate as non-packed FP32 on this chip) keeps
  // the FP32 gradient within 1e-5 of the exact one at every curve length.
  cplx<T> In[KM];
  sfor<KM>([&](auto Kk) {
    constexpr int k = Kk;
    cplx<T> v = rows[(t + 1) * KM + k];
    if (k == 0) v.i = T(0);
    In[k] = v;
  });
  // u: the first US samples in LDS after the staging buffer (sample n of
  // lane t at ust[n * ROWS + t]: consecutive lanes, consecutive banks), the
  // others in registers
  constexpr int US = (MODE == MODE_J) ? 0 : u_stash<NX, T>();
  T u[MODE == MODE_J ? 1 : NX - US];
  T* __restrict__ ust = reinterpret_cast<T*>(buf + (BR * KM + E)) + t;
  cplx<double> S0[KM];
  {
    double v[NX];
    spec_to_phys<NX, KM, double, T>(In, v);
    if constexpr (MODE != MODE_J) {
      sfor<NX>([&](auto Nn) {
        constexpr int n = Nn;
        if constexpr (n < US)
          ust[n * ROWS] = T(v[n]);
        else
          u[n - US] = T(v[n]);
      });
    }
    sfor<NX>([&](auto Nn) {
      constexpr int n = Nn;
      v[n] = v[n] * v[n];
    });
    phys_to_spec2<NX, KM, double>(v, S0);
  }
  cplx<T> R[KM];
  {
    // r_hat = -g (u_{j+1} - u_{j-1}) / (2 dsigma) + A u_hat - (i q / 2) N_hat in
    // FP64 (the inputs are exact in it), rounded once to the state dtype; the
    // state rows are read from LDS in batches of CH modes (all reads of a batch
    // issued before its arithmetic), keeping few values live.
    double rowR0 = 0.0, rowR = 0.0, rowD0 = 0.0, rowD = 0.0;
    // (the empty asm keeps the per-mode constants below from being hoisted
    // and kept live across the transforms)
    double q1s_r = cd.q1 * cd.q1, qN1_r = cd.q1 / (4.0 * NX), cs_r = double(csj);
    __asm__ volatile("" : "+v"(q1s_r), "+v"(qN1_r), "+v"(cs_r));
    // two batches of LDS reads in flight: batch c+1 is issued before the
    // arithmetic of batch c
    cplx<T> xm[2][CH], x0[2][CH], xp[2][CH];
    auto load = [&](auto Cc, auto Bb) {
      constexpr int k0 = int(Cc) * CH;
      sfor<CH>([&](auto Ii) {
        constexpr int k = k0 + int(Ii);
        if constexpr (k < KM) {
          xm[Bb][Ii] = rows[t * KM + k];
          x0[Bb][Ii] = rows[(t + 1) * KM + k];
          xp[Bb][Ii] = rows[(t + 2) * KM + k];
        }
      });
    };
    load(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    sfor<NCH>([&](auto Cc) {
      constexpr int k0 = int(Cc) * CH;
      constexpr int B = int(Cc) % 2;
      if constexpr (int(Cc) + 1 < NCH)
        load(std::integral_constant<int, int(Cc) + 1>{}, std::integral_constant<int, 1 - B>{});
      __builtin_amdgcn_sched_barrier(0);
      sfor<CH>([&](auto Ii) {
        constexpr int i = Ii;
        constexpr int k = k0 + i;
        if constexpr (k < KM) {
          const double dr = double(xp[B][i].r) - double(xm[B][i].r);
          double rr, ri;
          if constexpr (k == 0) {
            rr = -cs_r * dr;
            ri = 0.0;
            rowR0 = rr * rr;
            if constexpr (MODE == MODE_J) rowD0 = dr * dr;
          } else {
            const double di = double(xp[B][i].i) - double(xm[B][i].i);
            const double qn = double(k) * qN1_r;
            const double q2 = double(k * k) * q1s_r;
            const double Ak = fmaT(-q2, q2, q2);
            rr = fmaT(-cs_r, dr, fmaT(Ak, double(x0[B][i].r), qn * S0[k].i));
            ri = fmaT(-cs_r, di, fmaT(Ak, double(x0[B][i].i), -qn * S0[k].r));
            rowR = fmaT(rr, rr, fmaT(ri, ri, rowR));
            if constexpr (MODE == MODE_J) rowD = fmaT(dr, dr, fmaT(di, di, rowD));
          }
          R[k] = interior ? cplx<T>{T(rr), T(ri)} : cplx<T>{T(0), T(0)};
        }
      });
      // finish this batch's sums here (J-only mode has no other use of the
      // residual, and sinking its arithmetic keeps every batch's reads live)
      __asm__ volatile("" : "+v"(rowR0), "+v"(rowR), "+v"(rowD0), "+v"(rowD));
      __builtin_amdgcn_sched_barrier(0);
    });
    double pj = 0.0, pn = 0.0, pd = 0.0;
    if (interior) {
      const double rR = rowR0 + 2.0 * rowR;
      pj = a.wlD[cd.row_off + jr] * rR;
      if constexpr (MODE == MODE_J) {
        const double rD = rowD0 + 2.0 * rowD;
        pn = sqrt(rR * rD);
        pd = sqrt(rD);
      }
    }
    store_wave_partials<W, (MODE == MODE_J) ? 3 : 1>(pj, pn, pd, tile_partials(a, cd, c, tile, W));
  }
  cplx<T> S[KM];
  if constexpr (MODE != MODE_J) {
    // exchange residual rows through the staging buffer (outside rows read as 0)
    __syncthreads();
    T qY1_r = qY1;
    __asm__ volatile("" : "+v"(qY1_r));
    sfor<KM>([&](auto Kk) {
      constexpr int k = Kk;
      rows[(t + 1) * KM + k] = R[k];
      const T qk = T(k) * qY1_r;
      In[k] = cplx<T>{-qk * R[k].i, qk * R[k].r};
    });
    for (int i = t; i < 2 * KM; i += ROWS)
      rows[(i < KM) ? i : (BR - 2) * KM + i] = cplx<T>{T(0), T(0)};
    __syncthreads();
    // ---- pass 1, in the state dtype: rho = c2r(i q r_hat / (2 N_x)),
    // S = r2c(u * rho) = Q_hat ----
    T v[NX];
    spec_to_phys<NX, KM, T>(In, v);
    sfor<NX>([&](auto Nn) {
      constexpr int n = Nn;
      if constexpr (n < US)
        v[n] = ust[n * ROWS] * v[n];
      else
        v[n] = u[n - US] * v[n];
    });
    phys_to_spec2<NX, KM, T>(v, S);
  }

  if constexpr (MODE != MODE_J) {
    // ---- L^dagger r = g (r_{j+1} - r_{j-1}) / (2 dsigma) + Q_hat + A r_hat ----
    const bool fix_lo = interior && t == 0 && jr - 1 >= 1;
    const bool fix_hi = interior && t == ROWS - 1 && jr + 1 <= n_s - 2;
    cplx<T> D[KM];
    T q1s_d = q1s;
    __asm__ volatile("" : "+v"(q1s_d));
    cplx<T> rm[2][CH], r0[2][CH], rp[2][CH];
    auto load_r = [&](auto Cc, auto Bb) {
      constexpr int k0 = int(Cc) * CH;
      sfor<CH>([&](auto Ii) {
        constexpr int k = k0 + int(Ii);
        if constexpr (k < KM) {
          rm[Bb][Ii] = rows[t * KM + k];
          r0[Bb][Ii] = rows[(t + 1) * KM + k];
          rp[Bb][Ii] = rows[(t + 2) * KM + k];
        }
      });
    };
    load_r(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    sfor<NCH>([&](auto Cc) {
      constexpr int k0 = int(Cc) * CH;
      constexpr int B = int(Cc) % 2;
      if constexpr (int(Cc) + 1 < NCH)
        load_r(std::integral_constant<int, int(Cc) + 1>{}, std::integral_constant<int, 1 - B>{});
      __builtin_amdgcn_sched_barrier(0);
      sfor<CH>([&](auto Ii) {
        constexpr int i = Ii;
        constexpr int k = k0 + i;
        if constexpr (k < KM) {
          const T q2 = T(k * k) * q1s_d;
          const T Ak = fmaT(-q2, q2, q2);
          D[k].r = fmaT(csj, rp[B][i].r - rm[B][i].r, fmaT(Ak, r0[B][i].r, S[k].r));
          D[k].i = (k == 0) ? T(0)
                            : fmaT(csj, rp[B][i].i - rm[B][i].i, fmaT(Ak, r0[B][i].i, S[k].i));
        }
      });
      __builtin_amdgcn_sched_barrier(0);
    });
    if (fix_lo || fix_hi) {
      cplx<T>* e = a.edge + ((long long)tile * 4 + (fix_hi ? 2 : 0)) * a.km_max;
      sfor<KM>([&](auto Kk) {
        constexpr int k = Kk;
        e[k] = D[k];
        e[a.km_max + k] = rows[(t + 1) * KM + k];
      });
    }
    // ---- the tile's output rows, staged in LDS and written back coalesced ----
    // GRAD: 2 w L c_k L^dagger (0 on the end rows);  STEP: the increment
    // -dtau L^dagger / (1 + dtau A^2) (0 on the end rows), added to the input
    // while writing.  The increment of Im u_hat_0 cancels its raw input value.
    const long long obase = cd.off + (long long)j0 * KM;
    const int osh = int(obase % E);
    cplx<T>* __restrict__ orow = buf + osh + t * KM;
    __syncthreads();  // every lane has read its residual neighbours
    if constexpr (MODE == MODE_GRAD) {
      const T sc = (a.scale != nullptr) ? T(a.scale[c]) : T(1);
      const T f0 = interior ? a.wlT[cd.row_off + jr] * sc : T(0);
      sfor<KM>([&](auto Kk) {
        constexpr int k = Kk;
        constexpr T ck = (k == 0) ? T(1) : T(2);
        orow[k] = cplx<T>{(ck * f0) * D[k].r, (ck * f0) * D[k].i};
      });
    } else {
      const T* __restrict__ pv = a.pre + cd.mode_off;
      const T m = interior ? T(1) : T(0);
      sfor<KM>([&](auto Kk) {
        constexpr int k = Kk;
        const T f = m * pv[k];
        orow[k] = cplx<T>{f * D[k].r, (k == 0) ? -x0i : f * D[k].i};
      });
    }
    __syncthreads();
    flush_block<cplx<T>, ROWS, ROWS * KM + E, MODE == MODE_STEP>(a.out, a.in, buf, obase, osh, ROWS * KM + osh, obase,
                                            cd.off + (long long)min(n_s, j0 + ROWS) * KM);
  }
}

// Lanes per row of the FP32 N_x = 256 tile kernel (ksc_lanes.hpp): 16 lanes
// give a 8190-row curve 2048 waves, two per SIMD.
constexpr int kLanesF32N256 = 16;

// Lanes per row: one whole row per lane while its transform fits the
// registers (N_x reals of the field kept for the adjoint plus N_x of
// transform work space), else a lane pair per row.
template <int NX, typename T>
constexpr int lanes_per_row() {
  if (sizeof(T) == 4 && NX == 256) return kLanesF32N256;
  return (NX * int(sizeof(T)) > 512) ? 2 : 1;
}

// Waves per SIMD that a tile kernel is compiled for: the 16-lane kernel keeps
// two resident (at most 256 VGPRs each), the others one.
template <int NX, typename T>
constexpr int tile_waves_per_simd() {
  return (lanes_per_row<NX, T>() * lanes_per_row<NX, T>() == NX) ? 2 : 1;
}

// The same evaluation with two lanes per row (lane 2r + p holds modes
// k = 2i + p and samples [p N/2, (p+1) N/2) of row j0 + r): a tile is 32W rows.
// It serves FP64 rows of N_x >= 128, so both passes run in the state dtype.
template <int NX, typename T, int W, int MODE>
__device__ __forceinline__ void tile_body2(const KernelArgs<T>& a, const CurveDev& cd, int c,
                                           int j0, int tile, cplx<T>* buf) {
  constexpr int KM = (NX - 1) / 3 + 1;
  constexpr int KH = (KM + 1) / 2;  // modes per lane
  constexpr int ROWS = 32 * W;      // rows per tile
  constexpr int NT = 64 * W;        // lanes
  constexpr int BR = ROWS + 2;      // staged rows: j0-1 .. j0+ROWS
  constexpr int E = 16 / int(sizeof(cplx<T>));
  constexpr int NH = NX / 2;        // samples per lane
  const int t = threadIdx.x >> 1;   // row within the tile
  const int p = threadIdx.x & 1;
  const bool odd = p != 0;
  const T pf = T(p);
  const int n_s = cd.n_s;
  const int jr = j0 + t;
  const bool interior = (jr >= 1) && (jr <= n_s - 2);

  const long long base = cd.off + (long long)(j0 - 1) * KM;
  const int sh = int(((base % E) + E) % E);
  __syncthreads();
  stage_block<cplx<T>, NT, BR * KM + E>(buf, a.in, base, sh, BR * KM + sh,
                                  cd.off + (long long)(j0 > 0 ? j0 - 1 : 0) * KM,
                                  cd.off + (long long)min(n_s, j0 + ROWS + 1) * KM);
  __syncthreads();
  static_assert(sizeof(T) == 8, "lane pairs serve FP64 rows");
  cplx<T>* __restrict__ rows = buf + sh;
  // this lane's entry i of a row is mode 2i + p; the last entry of lane 1 may
  // lie past K (odd KM): it reads as zero and is never written
  auto ok = [&](int i) { return 2 * i + p < KM; };

  const T x0i = rows[(t + 1) * KM].i;  // raw Im u_hat_0 (lane 0 uses it)
  const T csj = interior ? a.cs[cd.row_off + jr] : T(0);
  const T q1 = T(cd.q1);
  const T qY1 = T(cd.q1 / (2.0 * NX));
  constexpr int CH = 7;
  constexpr int NCH = (KH + CH - 1) / CH;

  cplx<T> In[KH];
  sfor<KH>([&](auto Ii) {
    constexpr int i = Ii;
    In[i] = ok(i) ? rows[(t + 1) * KM + 2 * i + p] : cplx<T>{T(0), T(0)};
  });
  T u[MODE == MODE_J ? 1 : NH];
  cplx<T> R[KH];
  // r_hat from S0 = r2c(u^2), the cost partials
  auto residual = [&](const cplx<double>(&S0)[KH]) {
    double rowR0 = 0.0, rowR = 0.0, rowD0 = 0.0, rowD = 0.0;
    double q1_r = cd.q1, qN1_r = cd.q1 / (4.0 * NX), pf_r = double(p), cs_r = double(csj);
    __asm__ volatile("" : "+v"(q1_r), "+v"(qN1_r), "+v"(pf_r), "+v"(cs_r));
    sfor<NCH>([&](auto Cc) {
      constexpr int i0 = int(Cc) * CH;
      cplx<T> xm[CH], x0[CH], xp[CH];
      sfor<CH>([&](auto Ii) {
        constexpr int i = i0 + int(Ii);
        if constexpr (i < KH) {
          const int k = 2 * i + p;
          const bool v = ok(i);
          xm[Ii] = v ? rows[t * KM + k] : cplx<T>{T(0), T(0)};
          x0[Ii] = v ? rows[(t + 1) * KM + k] : cplx<T>{T(0), T(0)};
          xp[Ii] = v ? rows[(t + 2) * KM + k] : cplx<T>{T(0), T(0)};
        }
      });
      __builtin_amdgcn_sched_barrier(0);
      sfor<CH>([&](auto Ii) {
        constexpr int ii = Ii;
        constexpr int i = i0 + ii;
        if constexpr (i < KH) {
          const double kf = double(2 * i) + pf_r;  // mode number k = 2i + p
          const double qn = kf * qN1_r;
          const double qk = kf * q1_r;
          const double q2 = qk * qk;
          const double Ak = fmaT(-q2, q2, q2);
          const double dr = double(xp[ii].r) - double(xm[ii].r);
          const double di = double(xp[ii].i) - double(xm[ii].i);
          double rr = fmaT(-cs_r, dr, fmaT(Ak, double(x0[ii].r), qn * S0[i].i));
          double ri = fmaT(-cs_r, di, fmaT(Ak, double(x0[ii].i), -qn * S0[i].r));
          if constexpr (i == KH - 1) {
            // past K on lane 1 when K+1 is odd: the transform still produced
            // a coefficient there, which must not enter the cost or the adjoint
            rr = ok(i) ? rr : 0.0;
            ri = ok(i) ? ri : 0.0;
          }
          if constexpr (i == 0) {
            // lane 0 entry 0 is mode 0: real, weight 1 in the Parseval sum
            ri = odd ? ri : 0.0;
            const double e = fmaT(rr, rr, ri * ri);
            rowR0 = odd ? 0.0 : e;
            rowR = odd ? e : 0.0;
            if constexpr (MODE == MODE_J) {
              const double d = odd ? fmaT(dr, dr, di * di) : dr * dr;
              rowD0 = odd ? 0.0 : d;
              rowD = odd ? d : 0.0;
            }
          } else {
            rowR = fmaT(rr, rr, fmaT(ri, ri, rowR));
            if constexpr (MODE == MODE_J) rowD = fmaT(dr, dr, fmaT(di, di, rowD));
          }
          R[i] = interior ? cplx<T>{T(rr), T(ri)} : cplx<T>{T(0), T(0)};
        }
      });
      // finish this batch's sums here (J-only mode has no other use of the
      // residual, and sinking its arithmetic keeps every batch's reads live)
      __asm__ volatile("" : "+v"(rowR0), "+v"(rowR), "+v"(rowD0), "+v"(rowD));
      __builtin_amdgcn_sched_barrier(0);
    });
    double pj = 0.0, pn = 0.0, pd = 0.0;
    if (interior) {
      // each lane holds its share of the row sums; J_arc needs whole rows
      const double rR = rowR0 + 2.0 * rowR;
      pj = a.wlD[cd.row_off + jr] * rR;
      if constexpr (MODE == MODE_J) {
        const double rD = rowD0 + 2.0 * rowD;
        const double rRrow = rR + pair_swap(rR), rDrow = rD + pair_swap(rD);
        pn = odd ? 0.0 : sqrt(rRrow * rDrow);
        pd = odd ? 0.0 : sqrt(rDrow);
      }
    }
    store_wave_partials<W, (MODE == MODE_J) ? 3 : 1>(pj, pn, pd, tile_partials(a, cd, c, tile, W));
  };
  // the residual rows to the staging buffer (for the neighbours' d/ds) and
  // In = i q r_hat / (2 N_x), the input of pass 1
  auto exchange = [&]() {
    __syncthreads();
    T qY1_r = qY1, pf_y = pf;
    __asm__ volatile("" : "+v"(qY1_r), "+v"(pf_y));
    sfor<KH>([&](auto Ii) {
      constexpr int i = Ii;
      if (ok(i)) rows[(t + 1) * KM + 2 * i + p] = R[i];
      const T qk = (T(2 * i) + pf_y) * qY1_r;
      In[i] = cplx<T>{-qk * R[i].i, qk * R[i].r};
    });
    for (int i = threadIdx.x; i < 2 * KM; i += NT)
      rows[(i < KM) ? i : (BR - 2) * KM + i] = cplx<T>{T(0), T(0)};
    __syncthreads();
  };
  cplx<T> S[KH];
  {
    // both passes through one copy of the transforms (a runtime loop of two
    // iterations keeps the code, and the register allocation, of one pass)
    constexpr int NPASS = (MODE == MODE_J) ? 1 : 2;
#pragma clang loop unroll(disable)
    for (int pass = 0; pass < NPASS; ++pass) {
      {
        T v[NH];
        spec_to_phys_pair<NX, KH, T>(In, pf, v);
        if constexpr (MODE == MODE_J) {
          sfor<NH>([&](auto Nn) {
            constexpr int n = Nn;
            v[n] = v[n] * v[n];
          });
        } else {
          if (pass == 0) {
            sfor<NH>([&](auto Nn) {
              constexpr int n = Nn;
              u[n] = v[n];
            });
          }
          sfor<NH>([&](auto Nn) {
            constexpr int n = Nn;
            v[n] = u[n] * v[n];
          });
        }
        phys_to_spec2_pair<NX, KH, T>(v, pf, S);
      }
      if (pass == 0) {
        residual(S);
        if constexpr (MODE != MODE_J) exchange();
      }
    }
  }

  if constexpr (MODE != MODE_J) {
    const bool fix_lo = interior && t == 0 && jr - 1 >= 1;
    const bool fix_hi = interior && t == ROWS - 1 && jr + 1 <= n_s - 2;
    cplx<T> D[KH];
    T q1_d = q1, pf_d = pf;
    __asm__ volatile("" : "+v"(q1_d), "+v"(pf_d));
    sfor<NCH>([&](auto Cc) {
      constexpr int i0 = int(Cc) * CH;
      cplx<T> rm[CH], r0[CH], rp[CH];
      sfor<CH>([&](auto Ii) {
        constexpr int i = i0 + int(Ii);
        if constexpr (i < KH) {
          const int k = 2 * i + p;
          const bool v = ok(i);
          rm[Ii] = v ? rows[t * KM + k] : cplx<T>{T(0), T(0)};
          r0[Ii] = v ? rows[(t + 1) * KM + k] : cplx<T>{T(0), T(0)};
          rp[Ii] = v ? rows[(t + 2) * KM + k] : cplx<T>{T(0), T(0)};
        }
      });
      __builtin_amdgcn_sched_barrier(0);
      sfor<CH>([&](auto Ii) {
        constexpr int ii = Ii;
        constexpr int i = i0 + ii;
        if constexpr (i < KH) {
          const T qk = (T(2 * i) + pf_d) * q1_d;
          const T q2 = qk * qk;
          const T Ak = fmaT(-q2, q2, q2);
          D[i].r = fmaT(csj, rp[ii].r - rm[ii].r, fmaT(Ak, r0[ii].r, S[i].r));
          const T di = fmaT(csj, rp[ii].i - rm[ii].i, fmaT(Ak, r0[ii].i, S[i].i));
          D[i].i = (i == 0 && !odd) ? T(0) : di;
        }
      });
      __builtin_amdgcn_sched_barrier(0);
    });
    if (fix_lo || fix_hi) {
      int pe = p;  // (opaque: keeps the per-mode addresses below from being hoisted)
      __asm__ volatile("" : "+v"(pe));
      cplx<T>* e = a.edge + ((long long)tile * 4 + (fix_hi ? 2 : 0)) * a.km_max + pe;
      cplx<T>* e2 = e + a.km_max;
      const cplx<T>* rr = rows + (t + 1) * KM + pe;
      sfor<KH>([&](auto Ii) {
        constexpr int i = Ii;
        if (ok(i)) {
          e[2 * i] = D[i];
          e2[2 * i] = rr[2 * i];
        }
      });
    }
    const long long obase = cd.off + (long long)j0 * KM;
    const int osh = int(obase % E);
    int po = p;
    __asm__ volatile("" : "+v"(po));
    cplx<T>* __restrict__ orow = buf + osh + t * KM + po;  // this lane's modes: orow[2i]
    __syncthreads();
    if constexpr (MODE == MODE_GRAD) {
      const T sc = (a.scale != nullptr) ? T(a.scale[c]) : T(1);
      const T f0 = interior ? a.wlT[cd.row_off + jr] * sc : T(0);
      const T f2 = T(2) * f0;
      sfor<KH>([&](auto Ii) {
        constexpr int i = Ii;
        const T f = (i == 0 && !odd) ? f0 : f2;  // c_0 = 1, c_k = 2
        if (ok(i)) orow[2 * i] = cplx<T>{f * D[i].r, f * D[i].i};
      });
    } else {
      const T* __restrict__ pv = a.pre + cd.mode_off + po;
      const T m = interior ? T(1) : T(0);
      sfor<KH>([&](auto Ii) {
        constexpr int i = Ii;
        if (ok(i)) {
          const T f = m * pv[2 * i];
          orow[2 * i] = cplx<T>{f * D[i].r, (i == 0 && !odd) ? -x0i : f * D[i].i};
        }
      });
    }
    __syncthreads();
    flush_block<cplx<T>, NT, ROWS * KM + E, MODE == MODE_STEP>(a.out, a.in, buf, obase, osh, ROWS * KM + osh, obase,
                                          cd.off + (long long)min(n_s, j0 + ROWS) * KM);
  }
}

// Inactive curve in a descent: the tile copies its rows unchanged.
template <int NX, typename T, int W>
__device__ __forceinline__ void tile_copy(const KernelArgs<T>& a, const CurveDev& cd, int c, int j0,
                                          int tile) {
  constexpr int KM = (NX - 1) / 3 + 1;
  constexpr int ROWS = 64 * W / lanes_per_row<NX, T>();
  const int jr = j0 + int(threadIdx.x);
  if (int(threadIdx.x) < ROWS && jr < cd.n_s) {
    const cplx<T>* s = a.in + cd.off + (long long)jr * KM;
    cplx<T>* d = a.out + cd.off + (long long)jr * KM;
    for (int k = 0; k < KM; ++k) d[k] = s[k];
  }
  store_wave_partials<W, 1>(0.0, 0.0, 0.0, tile_partials(a, cd, c, tile, W));
}

}  // namespace ksc
