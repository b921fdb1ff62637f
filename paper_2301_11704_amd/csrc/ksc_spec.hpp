// Evaluation with the paper's spectral d/ds: the rational Chebyshev
// differentiation matrix D_t (Sec. IV, eq. rational_diff_matrix) applied along
// s, instead of the central difference of the tile kernels.
//
// D_t is dense, so one evaluation is three launches (plus the cost reduction):
//   1. Y = D_t U per curve, a matrix product along s (MFMA, spec_gemm);
//   2. per row (spec_row_body): r_hat = -Y + A u_hat - (i q / 2) N_hat, the
//      cost partials, and the row-local part of the adjoint
//      P = Q_hat + A r_hat (Q_hat: the u r_x term); the row writes
//      WR = 2 w L r_hat and P;
//   3. Z' = D_t^T WR per curve (MFMA), whose epilogue forms the output:
//      L^dagger r = P - Z' / (2 w L) (the s-part -(1/w) D_t^T (w r) is the
//      exact discrete adjoint of -D_t in the weighted inner product), and the
//      gradient 2 w L c_k L^dagger r = c_k (2 w L P - Z') or the step
//      u_hat - dtau L^dagger r / (1 + dtau A^2).
// The matrix pool holds D~ = S D_t per distinct N_s (it does not depend on S)
// in FP64; 1/S is applied in the epilogues.  The products run on FP64 matrix
// cores for both state dtypes: the sums along s cancel heavily (at N_s = 552
// the sum of the magnitudes of the terms of the adjoint's s-part is ~3e3 times
// the result), so FP32 storage of D~ or FP32 accumulation would lose about
// three digits, while FP32 rounding of the state and of the residual alone
// stays near 1e-6 of the gradient.
#pragma once

#include "ksc_sym.hpp"
#include "ksc_tile.hpp"

namespace ksc {

// Per-curve descriptor of the spectral launches.
struct SpecDev {
  long long off;   // offset of row 0 in complex elements of the state
  long long dmat;  // offset of the curve's D~ (n_s x n_s, row-major) in the matrix pool
  long long dmatT; // offset of its transpose
  int n_s, km, row_off, mode_off;
  int c, pad_;     // index of the curve in the problem
  double inv_S;    // 1 / S
};

template <typename T>
struct SpecArgs {
  const double* __restrict__ dpool;     // D~ matrices (FP64)
  const SpecDev* __restrict__ curves;
  const T* __restrict__ b;              // GEMM right operand (state layout)
  T* __restrict__ out;                  // GEMM result or final output (state layout)
  const T* __restrict__ u;              // state (STEP epilogue)
  const T* __restrict__ p;              // row-local adjoint part P (GRAD/STEP epilogue)
  const T* __restrict__ wlT;            // per row: 2 w L
  const T* __restrict__ pre;            // per mode: -dtau / (1 + dtau A^2)
  const double* __restrict__ scale;     // per curve gradient scale, nullable
  const unsigned char* __restrict__ active;  // per curve, nullable (STEP)
  double* __restrict__ part;            // split k: partial products, [kparts][state scalars]
  long long part_stride;                // scalars per partial (the state's scalar count)
  int kparts;                           // parts of the k range (1: no split)
};

enum SpecEpi : int { EPI_Y = 0, EPI_GRAD = 1, EPI_STEP = 2 };

// A group of curves that share n_x and n_s (one D~), as one launch sees it:
// its workgroups are [block0, block0 + row_blocks * curve_blocks).
struct SpecGroupDev {
  int first;       // first curve (index into the SpecDev array)
  int count;       // curves in the group
  int row_blocks;  // ceil(n_s / 64)
  int block0;      // first workgroup of the group in the launch
};

// Row kernel arguments: the tile machinery's KernelArgs (state in a.in, tiles,
// tables, partials) plus the derivative rows Y and the two output arrays.
template <typename T>
struct SpecRowArgs {
  KernelArgs<T> a;
  const cplx<T>* __restrict__ y;  // D_t U
  cplx<T>* __restrict__ wr;       // 2 w L r_hat (0 on the end rows)
  cplx<T>* __restrict__ pl;       // Q_hat + A r_hat (0 on the end rows)
};

// One tile of 64W rows, one row per lane (N_x sizeof(T) <= 512 B): the
// residual from the precomputed d/ds rows, the cost and J_arc partials and,
// unless MODE_J, the row-local adjoint part.
template <int NX, typename T, int W, int MODE>
__device__ __forceinline__ void spec_row_body(const SpecRowArgs<T>& sa, const CurveDev& cd, int c,
                                              int j0, int tile, cplx<T>* buf) {
  const KernelArgs<T>& a = sa.a;
  constexpr int KM = (NX - 1) / 3 + 1;
  constexpr int ROWS = 64 * W;
  constexpr int E = 16 / int(sizeof(cplx<T>));
  constexpr int NB = ROWS * KM + 2 * E;  // one staged block, with alignment slack
  const int t = threadIdx.x;
  const int n_s = cd.n_s;
  const int jr = j0 + t;
  const bool interior = (jr >= 1) && (jr <= n_s - 2);
  const long long base = cd.off + (long long)j0 * KM;
  const long long G_hi = cd.off + (long long)min(n_s, j0 + ROWS) * KM;
  const int sh = int(base % E);
  cplx<T>* __restrict__ bu = buf;       // state rows
  cplx<T>* __restrict__ by = buf + NB;  // d/ds rows
  __syncthreads();
  stage_block<cplx<T>, ROWS, ROWS * KM + E>(bu, a.in, base, sh, ROWS * KM + sh, base, G_hi);
  stage_block<cplx<T>, ROWS, ROWS * KM + E>(by, sa.y, base, sh, ROWS * KM + sh, base, G_hi);
  __syncthreads();
  const cplx<T>* __restrict__ urow = bu + sh + t * KM;
  const cplx<T>* __restrict__ yrow = by + sh + t * KM;

  const T q1s = T(cd.q1 * cd.q1);
  const T qN1 = T(cd.q1 / (4.0 * NX));  // q1 / (4 N_x): S is 2 N_x N_hat
  const T qY1 = T(cd.q1 / (2.0 * NX));  // q1 / (2 N_x): Q_hat = r2c/(2 N_x)

  cplx<T> In[KM];
  sfor<KM>([&](auto Kk) {
    constexpr int k = Kk;
    cplx<T> v = urow[k];
    if (k == 0) v.i = T(0);
    In[k] = v;
  });
  T u[NX];
  cplx<T> S[KM];
  {
    T v[NX];
    spec_to_phys<NX, KM, T>(In, v);
    sfor<NX>([&](auto Nn) {
      constexpr int n = Nn;
      if constexpr (MODE != MODE_J) u[n] = v[n];
      v[n] = v[n] * v[n];
    });
    phys_to_spec2<NX, KM, T>(v, S);
  }
  // r_hat = -D_t u_hat + A u_hat - (i q / 2) N_hat,  S = 2 N_x N_hat
  cplx<T> R[KM];
  T rowR0 = T(0), rowR = T(0), rowD0 = T(0), rowD = T(0);
  sfor<KM>([&](auto Kk) {
    constexpr int k = Kk;
    const cplx<T> yk = yrow[k];
    T rr, ri;
    if constexpr (k == 0) {
      rr = -yk.r;
      ri = T(0);
      rowR0 = rr * rr;
      rowD0 = yk.r * yk.r;
    } else {
      const T qn = T(k) * qN1;
      const T q2 = T(k * k) * q1s;
      const T Ak = fmaT(-q2, q2, q2);
      rr = fmaT(Ak, In[k].r, fmaT(qn, S[k].i, -yk.r));
      ri = fmaT(Ak, In[k].i, fmaT(-qn, S[k].r, -yk.i));
      rowR = fmaT(rr, rr, fmaT(ri, ri, rowR));
      rowD = fmaT(yk.r, yk.r, fmaT(yk.i, yk.i, rowD));
    }
    R[k] = interior ? cplx<T>{rr, ri} : cplx<T>{T(0), T(0)};
  });
  double pj = 0.0, pn = 0.0, pd = 0.0;
  if (interior) {
    const double rR = double(rowR0) + 2.0 * double(rowR);
    const double wl = a.wlD[cd.row_off + jr];  // w_j L
    pj = wl * rR;
    if constexpr (MODE == MODE_J) {
      // J_arc: |u_s| ds = |D_t u|_j w_j (the common factor L cancels)
      const double rD = double(rowD0) + 2.0 * double(rowD);
      pn = wl * sqrt(rR * rD);
      pd = wl * sqrt(rD);
    }
  }
  store_wave_partials<W, (MODE == MODE_J) ? 3 : 1>(pj, pn, pd, tile_partials(a, cd, c, tile, W));
  if constexpr (MODE != MODE_J) {
    // Q_hat = r2c(u * c2r((i q / (2 N_x)) r_hat))
    sfor<KM>([&](auto Kk) {
      constexpr int k = Kk;
      const T qk = T(k) * qY1;
      In[k] = cplx<T>{-qk * R[k].i, qk * R[k].r};
    });
    {
      T v[NX];
      spec_to_phys<NX, KM, T>(In, v);
      sfor<NX>([&](auto Nn) {
        constexpr int n = Nn;
        v[n] = u[n] * v[n];
      });
      phys_to_spec2<NX, KM, T>(v, S);
    }
    const T f0 = interior ? a.wlT[cd.row_off + jr] : T(0);  // 2 w L
    // outputs through the staging buffers (coalesced writes)
    __syncthreads();
    cplx<T>* __restrict__ ow = bu + sh + t * KM;
    cplx<T>* __restrict__ op = by + sh + t * KM;
    sfor<KM>([&](auto Kk) {
      constexpr int k = Kk;
      const T q2 = T(k * k) * q1s;
      const T Ak = fmaT(-q2, q2, q2);
      ow[k] = cplx<T>{f0 * R[k].r, f0 * R[k].i};
      const T pr = fmaT(Ak, R[k].r, S[k].r);
      const T pi = (k == 0) ? T(0) : fmaT(Ak, R[k].i, S[k].i);
      op[k] = interior ? cplx<T>{pr, pi} : cplx<T>{T(0), T(0)};
    });
    __syncthreads();
    flush_block<cplx<T>, ROWS, ROWS * KM + E, false>(sa.wr, nullptr, bu, base, sh, ROWS * KM + sh,
                                                     base, G_hi);
    flush_block<cplx<T>, ROWS, ROWS * KM + E, false>(sa.pl, nullptr, by, base, sh, ROWS * KM + sh,
                                                     base, G_hi);
  }
}

// The same in the inversion-symmetric subspace (rows of K reals b_k,
// u_hat_k = i b_k; transforms as in ksc_odd.hpp): rho_k = -y_k + A_k b_k
// - (q_k / (2N)) (2 C_k) with y = D_t b, the row-local adjoint part
// P = Im Q_hat + A rho, and WR = 2 w L rho.  The pointers of sa are read as
// real arrays.
template <int NX, typename T, int W, int MODE>
__device__ __forceinline__ void spec_row_body_odd(const SpecRowArgs<T>& sa, const CurveDev& cd,
                                                  int c, int j0, int tile, T* buf) {
  const KernelArgs<T>& a = sa.a;
  constexpr int K = (NX - 1) / 3;
  constexpr int M2 = NX / 2;
  constexpr int ROWS = 64 * W;
  constexpr int E = 16 / int(sizeof(T));
  constexpr int NB = ROWS * K + 2 * E;
  const int t = threadIdx.x;
  const int n_s = cd.n_s;
  const int jr = j0 + t;
  const bool interior = (jr >= 1) && (jr <= n_s - 2);
  const long long base = cd.off + (long long)j0 * K;
  const long long G_hi = cd.off + (long long)min(n_s, j0 + ROWS) * K;
  const int sh = int(base % E);
  T* __restrict__ bu = buf;
  T* __restrict__ by = buf + NB;
  __syncthreads();
  stage_block<T, ROWS, ROWS * K + E>(bu, reinterpret_cast<const T*>(a.in), base, sh, ROWS * K + sh,
                                     base, G_hi);
  stage_block<T, ROWS, ROWS * K + E>(by, reinterpret_cast<const T*>(sa.y), base, sh, ROWS * K + sh,
                                     base, G_hi);
  __syncthreads();
  const T* __restrict__ brow = bu + sh + t * K;
  const T* __restrict__ yrow = by + sh + t * K;
  const T q1s = T(cd.q1 * cd.q1);
  const T qN1 = T(cd.q1 / (2.0 * NX));
  constexpr T iN = T(1.0 / NX);

  T u[M2];
  {
    T f[M2];
    sfor<M2>([&](auto Kk) {
      constexpr int k = Kk;
      if constexpr (k >= 1 && k <= K)
        f[k] = -brow[k - 1];
      else
        f[k] = T(0);
    });
    dst1_x2<M2, M2, T>(f, u);
  }
  T C2[K + 1];
  {
    T g[M2 + 1];
    sfor<M2>([&](auto Nn) {
      constexpr int n = Nn;
      g[n] = u[n] * u[n];
    });
    g[M2] = T(0);
    dct1_x2<M2, K + 1, T>(g, C2);
  }
  T R[K];
  T rowR = T(0), rowD = T(0);
  sfor<K>([&](auto Ee) {
    constexpr int e = Ee;
    constexpr int k = e + 1;
    const T yk = yrow[e];
    const T qn = T(k) * qN1;
    const T q2 = T(k * k) * q1s;
    const T Ak = fmaT(-q2, q2, q2);
    const T rho = fmaT(Ak, brow[e], fmaT(-qn, C2[k], -yk));
    rowR = fmaT(rho, rho, rowR);
    rowD = fmaT(yk, yk, rowD);
    R[e] = interior ? rho : T(0);
  });
  double pj = 0.0, pn = 0.0, pd = 0.0;
  if (interior) {
    const double rR = 2.0 * double(rowR);
    const double wl = a.wlD[cd.row_off + jr];
    pj = wl * rR;
    if constexpr (MODE == MODE_J) {
      const double rD = 2.0 * double(rowD);
      pn = wl * sqrt(rR * rD);
      pd = wl * sqrt(rD);
    }
  }
  store_wave_partials<W, (MODE == MODE_J) ? 3 : 1>(pj, pn, pd, tile_partials(a, cd, c, tile, W));
  if constexpr (MODE != MODE_J) {
    T G2[K + 1];  // 2 F_k of u r_x = -N Im Q_hat_k
    {
      T rx[M2];
      {
        const T q1 = T(cd.q1);
        T g[M2 + 1];
        sfor<M2 + 1>([&](auto Kk) {
          constexpr int k = Kk;
          if constexpr (k >= 1 && k <= K)
            g[k] = -(T(k) * q1) * R[k - 1];
          else
            g[k] = T(0);
        });
        dct1_x2<M2, M2, T>(g, rx);
      }
      T w[M2];
      sfor<M2>([&](auto Nn) {
        constexpr int n = Nn;
        w[n] = u[n] * rx[n];
      });
      dst1_x2<M2, K + 1, T>(w, G2);
    }
    const T f0 = interior ? a.wlT[cd.row_off + jr] : T(0);  // 2 w L
    __syncthreads();
    T* __restrict__ ow = bu + sh + t * K;
    T* __restrict__ op = by + sh + t * K;
    sfor<K>([&](auto Ee) {
      constexpr int e = Ee;
      constexpr int k = e + 1;
      const T q2 = T(k * k) * q1s;
      const T Ak = fmaT(-q2, q2, q2);
      ow[e] = f0 * R[e];
      op[e] = interior ? fmaT(Ak, R[e], -iN * G2[k]) : T(0);
    });
    __syncthreads();
    flush_block<T, ROWS, ROWS * K + E, false>(reinterpret_cast<T*>(sa.wr), nullptr, bu, base, sh,
                                              ROWS * K + sh, base, G_hi);
    flush_block<T, ROWS, ROWS * K + E, false>(reinterpret_cast<T*>(sa.pl), nullptr, by, base, sh,
                                              ROWS * K + sh, base, G_hi);
  }
}

// ---------------------------------------------------------------------------
// C = op(D~) B / S per curve on FP64 matrix cores: D~ is n_s x n_s (op = transpose
// for TRANS), B the curve's state viewed as an n_s x NC real matrix (NC =
// 2(K+1), row stride NC).  A workgroup of four waves computes 64 rows of CB
// curves that share n_s (NCP = NC rounded up to 16 columns each, CB chosen for
// about six column tiles per wave, so one A tile feeds six accumulators); wave
// w owns rows 16w .. 16w+15 and all column tiles; the k loop walks n_s in
// steps of 32, the next step's operands loaded into registers while the
// current step's products run.
//
// 16x16x4 MFMA lane layout: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator r of lane l holds C[i][l % 16] with
// i = 4 (l / 16) + r for FP32 and i = l / 16 + 4 r for FP64 (checked on the
// device against a host product).
// ---------------------------------------------------------------------------
template <typename T>
struct mfma_acc;
template <>
struct mfma_acc<float> {
  typedef float v __attribute__((ext_vector_type(4)));
  __device__ __forceinline__ static v mac(float a, float b, v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct mfma_acc<double> {
  typedef double v __attribute__((ext_vector_type(4)));
  __device__ __forceinline__ static v mac(double a, double b, v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// Curves per workgroup of the products: one where a curve already gives a
// wave three or more 16-column tiles (a larger block would leave too few
// workgroups to fill the chip for batches of a few hundred rows per curve),
// else enough curves for about three tiles.
template <int NCP>
constexpr int spec_cb() {
  return (NCP / 16) >= 3 ? 1 : (NCP / 16) == 2 ? 2 : 3;
}
// Columns of a curve's state viewed as a real matrix, and the scalar offset
// of its row 0: full space 2(K+1) (col = 2k + re/im), odd subspace K
// (col = k - 1, the reals b_k).
template <bool ODD>
__device__ __forceinline__ int spec_cols(const SpecDev& cd) {
  return ODD ? cd.km - 1 : 2 * cd.km;
}
template <bool ODD>
__device__ __forceinline__ long long spec_base(const SpecDev& cd) {
  return ODD ? cd.off : 2 * cd.off;
}

// The output of element (row, col) of curve cd's product C = op(D~) B (before
// the 1/S): the product rounded to the state dtype (EPI_Y) or the gradient /
// stepped state formed from it as in the row kernels.  In the odd subspace
// every kept mode k = col + 1 has c_k = 2.
template <typename T, int EPI, bool ODD>
__device__ __forceinline__ void spec_store(const SpecArgs<T>& sa, const SpecDev& cd, int row,
                                           int col, double acc) {
  const int NC = spec_cols<ODD>(cd);
  const int n_s = cd.n_s;
  const int k = ODD ? col + 1 : col >> 1;
  const bool im0 = !ODD && (col == 1);
  const long long idx = spec_base<ODD>(cd) + (long long)row * NC + col;
  const T z = T(acc * cd.inv_S);
  const bool interior = row >= 1 && row <= n_s - 2;
  if constexpr (EPI == EPI_Y) {
    sa.out[idx] = z;
  } else if constexpr (EPI == EPI_GRAD) {
    const T sc = (sa.scale != nullptr) ? T(sa.scale[cd.c]) : T(1);
    const T pv = sa.p[idx];
    const T f = sa.wlT[cd.row_off + row];
    const T ck = (k == 0) ? T(1) : T(2);
    sa.out[idx] = (interior && !im0) ? (ck * sc) * fmaT(f, pv, -z) : T(0);
  } else {
    const bool act = (sa.active == nullptr) || sa.active[cd.c] != 0;
    const T uv = sa.u[idx];
    T o = uv;
    if (interior && act) {
      const T pv = sa.p[idx];
      const T f = sa.wlT[cd.row_off + row];
      o = fmaT(sa.pre[cd.mode_off + k], pv - z / f, uv);
    }
    sa.out[idx] = im0 ? T(0) : o;
  }
}

// LDS of one product workgroup (doubles): the A and B tiles with padded rows.
template <int NCP>
constexpr int spec_gemm_lds() {
  constexpr int BW = spec_cb<NCP>() * NCP;
  return 32 * (64 + 16) + 32 * (BW + ((48 - BW % 32) % 32));
}

// Rows row0 .. row0+63 of C for the curves cbase .. cbase+CB-1 of a group of
// `count` curves that share n_s (and hence D~).
// Part kp of sa.kparts of the k range: with one part the epilogue writes the
// output; with several, the raw partial products go to sa.part and
// spec_reduce forms the output.
template <typename T, int NCP, bool TRANS, int EPI, bool ODD>
__device__ __forceinline__ void spec_gemm_body(const SpecArgs<T>& sa, int count, int cbase,
                                               int row0, int kp, double* lds) {
  using mma = mfma_acc<double>;
  using acc_t = typename mma::v;
  constexpr int BM = 64, BK = 32;
  constexpr int AE = BM * BK / 256;          // A elements per thread and k step
  constexpr int CB = spec_cb<NCP>();
  constexpr int NT = NCP / 16;               // column tiles per curve
  constexpr int NJ = CB * NT;                // column tiles per wave
  constexpr int BW = CB * NCP;               // B tile width
  // LDS row strides: the four 16-lane groups of an MFMA operand read hit
  // alternating halves of the 64 banks (stride = 16 mod 32 doubles)
  constexpr int SA = BM + 16;
  constexpr int SB = BW + ((48 - BW % 32) % 32);
  constexpr int BE = (BK * BW) / 256;        // B elements per thread and k step
  static_assert((BK * BW) % 256 == 0, "B tile must split evenly over 256 threads");
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const SpecDev c0 = sa.curves[cbase];
  const int n_s = c0.n_s;
  const int NC = spec_cols<ODD>(c0);
  // op(D~)[i][k] is read as M[k][i] from M = D~^T (untransposed product) or
  // M = D~ (transposed product): a wave reads 64 consecutive doubles of one
  // row of M and writes them to 64 consecutive LDS words
  const double* __restrict__ D = sa.dpool + (TRANS ? c0.dmat : c0.dmatT);
  long long boff[CB];  // scalar offset of each curve's state block, -1 past the group
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
    boff[cb] = (cbase + cb < count) ? spec_base<ODD>(sa.curves[cbase + cb]) : -1;
  double* As = lds;               // [BK][SA]
  double* Bs = lds + BK * SA;     // [BK][SB]

  // B is held in the state's dtype until it is written to LDS, so that an
  // FP32 state's conversion does not wait on its load right after issuing it
  double ra[AE];
  T rb[BE];
  // A tile element e of thread t: (i, kk) with i < 64, kk < BK
  auto a_index = [&](int e, int& i, int& kk) {
    i = t % BM;
    kk = (t / BM) * AE + e;
  };
  auto load = [&](int k0) {
    // A tile: op(D~)[row0 + i][k0 + kk]
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      int i, kk;
      a_index(e, i, kk);
      const int gi = row0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < n_s && gk < n_s) v = D[(long long)gk * n_s + gi];
      ra[e] = v;
    }
    // B tile: row k0 + kk of each curve's n_s x NC block, curves side by side
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int q = t + 256 * e;
      const int kk = q / BW, rem = q % BW;
      const int cb = rem / NCP, col = rem % NCP;
      const int gk = k0 + kk;
      long long o = -1;
#pragma unroll
      for (int x = 0; x < CB; ++x) o = (cb == x) ? boff[x] : o;
      rb[e] = (gk < n_s && col < NC && o >= 0) ? sa.b[o + (long long)gk * NC + col] : T(0);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      int i, kk;
      a_index(e, i, kk);
      As[kk * SA + i] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int q = t + 256 * e;
      Bs[(q / BW) * SB + q % BW] = double(rb[e]);  // [kk][cb*NCP + col]
    }
  };

  // this part's k range, whole k steps
  const int nk = (n_s + BK - 1) / BK;
  const int per = (nk + sa.kparts - 1) / sa.kparts;
  const int k_lo = kp * per * BK, k_hi = min(n_s, (kp + 1) * per * BK);
  acc_t acc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) acc[j] = acc_t{0.0, 0.0, 0.0, 0.0};
  if (k_lo < k_hi) load(k_lo);
  for (int k0 = k_lo; k0 < k_hi; k0 += BK) {
    __syncthreads();  // the previous step's reads of the tiles are done
    store();
    __syncthreads();
    if (k0 + BK < k_hi) load(k0 + BK);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      const int kk = 4 * s + (lane >> 4);
      const double av = As[kk * SA + 16 * w + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const double bv = Bs[kk * SB + 16 * j + (lane & 15)];
        acc[j] = mma::mac(av, bv, acc[j]);
      }
    }
  }

  // epilogue: element (row, col) of curve cb's C
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    if (cbase + cb >= count) break;
    const SpecDev cd = sa.curves[cbase + cb];
#pragma unroll
    for (int jt = 0; jt < NT; ++jt) {
      const int j = cb * NT + jt;
      const int col = 16 * jt + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + 16 * w + mma::row(lane, r);
        if (row >= n_s || col >= NC) continue;
        if (sa.kparts == 1)
          spec_store<T, EPI, ODD>(sa, cd, row, col, acc[j][r]);
        else
          sa.part[kp * sa.part_stride + spec_base<ODD>(cd) + (long long)row * NC + col] = acc[j][r];
      }
    }
  }
}

// Sum of the kparts (at most 8) partial products of one element in part order
// (deterministic) and the epilogue.  The elements of a product workgroup's
// tile (64 rows x CB curves x NC columns) are spread over `chunk` workgroups
// of 256 threads, one element per thread, so that the partial loads of all
// elements are in flight together.
template <typename T, int NCP, int EPI, bool ODD>
__device__ __forceinline__ void spec_reduce_body(const SpecArgs<T>& sa, int count, int cbase,
                                                 int row0, int chunk) {
  const SpecDev c0 = sa.curves[cbase];
  const int NC = spec_cols<ODD>(c0);
  const int e = chunk * 256 + threadIdx.x;
  const int cb = e / (64 * NC), rem = e % (64 * NC);
  const int row = row0 + rem / NC, col = rem % NC;
  if (cb >= spec_cb<NCP>() || cbase + cb >= count || row >= c0.n_s) return;
  const SpecDev cd = sa.curves[cbase + cb];
  const long long idx = spec_base<ODD>(cd) + (long long)row * NC + col;
  double v[8];
#pragma unroll
  for (int kp = 0; kp < 8; ++kp) v[kp] = (kp < sa.kparts) ? sa.part[kp * sa.part_stride + idx] : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int kp = 0; kp < 8; ++kp) acc += v[kp];
  spec_store<T, EPI, ODD>(sa, cd, row, col, acc);
}

}  // namespace ksc
