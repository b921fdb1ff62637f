// The implicit-in-s descent step: for every curve and kept mode k, solve
//
//   (I + dtau B_k) delta = -dtau L^dagger_k,   B_k = A_k^2 - D m D,
//
// on the interior rows and write u_hat + delta.  D is the central difference
// along s, g_j (q_{j+1} - q_{j-1}) / (2 dsigma), and m zeroes the end rows of
// the residual, so B_k is the part of L^dagger(u; r(u)) that is linear in u
// (Sec. V.A: r = f(u) - u_s and L^dagger r = r_s + u r_x - r_xx - r_xxxx; the
// cross terms A_k u_s cancel).  The paper's step (Sec. V.C.3) keeps only A_k^2
// implicit; this one also removes the s-stiffness of the central difference.
//
// D m D couples row j only to rows j - 2 and j + 2, so the interior rows split
// into two chains (odd rows, even rows), each a tridiagonal system with
//   b_j = 1 + dtau A_k^2 + dtau beta_j (beta_{j+1} + beta_{j-1}),
//   a_j = -dtau beta_j beta_{j-1},  c_j = -dtau beta_j beta_{j+1},
// beta_j = g_j / (2 dsigma) (0 on the end rows); couplings to the fixed end
// rows are dropped.  The matrix is strictly diagonally dominant (margin
// 1 + dtau A_k^2), so elimination without pivoting is stable.
//
// Parallel solve (partition method): a workgroup takes one chain of one curve
// for CW mode columns; each column's chain is cut into P chunks, one thread
// per chunk.  A thread eliminates its chunk's interior rows in registers,
// writing each as y + l s_left + r s_right in terms of the last rows of its
// own chunk and of the chunk before (the interface unknowns s_p); the P
// interface equations form a tridiagonal system solved by parallel cyclic
// reduction in LDS; then every thread recovers its rows.  The right-hand side
// -dtau L^dagger_k is the gradient G = 2 w_j L c_k L^dagger_k of the fused
// kernel, rescaled per row.
//
// Optional heavy-ball momentum (Polyak): with beta > 0 the interior rows get
// u_hat + delta + beta (u_hat - u_prev), u_prev being what the output buffer
// holds on entry (in a ping-pong descent: the state one step before u_hat).
// A curve whose cost rose at this step's evaluation drops the momentum term
// for the step (a restart from rest, after O'Donoghue & Candes' adaptive
// restart of accelerated gradient schemes), so the iteration cannot coast
// away from the basin it is descending in.
#include "ksc_launch_simp.hpp"

namespace ksc {

namespace {

// 1/x: the hardware reciprocal in FP32 (1 ulp; every pivot is bounded away
// from zero by the diagonal dominance), a correctly rounded division in FP64
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// State element (column mc, row) of NV scalars: one 8- or 16-byte access for
// a complex mode.
template <typename T, int NV>
struct simp_vec;
template <typename T>
struct simp_vec<T, 1> {
  T v[1];
};
template <typename T>
struct alignas(2 * sizeof(T)) simp_vec<T, 2> {
  T v[2];
};

template <typename T, int NV, int MM>
__global__ __launch_bounds__(kSimpThreads) void simp_kernel(SimpArgs<T> a) {
  using V = simp_vec<T, NV>;
  __shared__ T sA[kSimpThreads], sB[kSimpThreads], sC[kSimpThreads], sD[NV][kSimpThreads];
  __shared__ T xY[NV][kSimpThreads], xL[kSimpThreads], xR[kSimpThreads];
  __shared__ int xF[kSimpThreads];

  // The dispatcher deals workgroups to the 8 XCDs in turn; map them so that
  // consecutive table entries (the chains and column groups of one curve,
  // which share cache lines) run on one XCD and its L2.
  int b = blockIdx.x;
  const int per_xcd = gridDim.x / 8;
  if (b < 8 * per_xcd) b = (b % 8) * per_xcd + b / 8;
  const SimpBlock blk = a.blocks[b];
  const CurveDev cd = a.curves[blk.curve];
  const int t = threadIdx.x;
  const int P = 1 << blk.log2p;
  const int CW = kSimpThreads >> blk.log2p;
  const int ci = t & (CW - 1);         // mode column within the group
  const int p = t >> (kSimpLog2Threads - blk.log2p);  // chunk
  const int NM = a.odd ? cd.km - 1 : cd.km;                   // mode columns (NV scalars each)
  const long long base = cd.off;  // row 0 in elements (complex modes, or reals in the odd space)
  const int mc = blk.col0 + ci;
  const bool col_ok = mc < NM;
  const int mcc = col_ok ? mc : NM - 1;                        // clamped for loads
  const int k = a.odd ? mcc + 1 : mcc;
  const int n_s = cd.n_s;
  const int j0 = 1 + blk.parity;
  const int n = (n_s - 1 - blk.parity) / 2;                    // rows of the chain
  const int m = (n + P - 1) >> blk.log2p;                      // chunk length (<= MM)
  const int q0 = p * m;
  const int mp = max(0, min(m, n - q0));                       // rows of this chunk
  const int mi = mp - 1;                                       // interior rows (the last is the interface)
  const T* __restrict__ cs = a.cs + cd.row_off;
  const T* __restrict__ wl = a.wlT + cd.row_off;
  const V* __restrict__ vin = reinterpret_cast<const V*>(a.in);
  const V* __restrict__ vgr = reinterpret_cast<const V*>(a.grad);
  V* __restrict__ vout = reinterpret_cast<V*>(a.out);
  auto eidx = [&](int row) { return base + (long long)row * NM + mcc; };
  // Im of mode 0 is identically zero in the full space
  auto clean = [&](V x) {
    if (NV == 2 && k == 0) x.v[NV - 1] = T(0);
    return x;
  };

  const bool is_active = (a.active == nullptr) || a.active[blk.curve] != 0;
  // end rows: copied by the odd-row chain's workgroup, one thread per column
  if (blk.parity == 0 && p == 0 && col_ok) {
    const long long i0 = eidx(0), i1 = eidx(n_s - 1);
    vout[i0] = is_active ? clean(vin[i0]) : vin[i0];
    vout[i1] = is_active ? clean(vin[i1]) : vin[i1];
  }
  if (!is_active) {  // uniform over the workgroup
    if (col_ok)
      for (int i = 0; i < mp; ++i) {
        const long long ix = eidx(j0 + 2 * (q0 + i));
        vout[ix] = vin[ix];
      }
    return;
  }

  // The system scaled row by row by w_j = 1 / (2 beta_j) is symmetric:
  //   diag_j = w_j (1 + dtau A_k^2) + dtau/2 (beta_{j+1} + beta_{j-1}),
  //   off-diagonal to row j +- 2: -dtau/2 beta_{j+-1},
  //   right-hand side -dtau w_j L^dagger_j = -dtau G_j / (2 L c_k).
  const T dtau = a.dtau, hdt = T(0.5) * dtau;
  const T Ak = a.A[cd.mode_off + k];
  const T ck = (a.odd || k > 0) ? T(2) : T(1);
  const T inv2L = T(cd.q1 / (4.0 * M_PI));                     // 1 / (2L), q1 = 2 pi / L
  const T dfac = (T(1) + dtau * Ak * Ak) * inv2L;              // times wl_j = 2 w_j L
  const T rfac = -dtau * inv2L / ck;

  // loads: right-hand sides, states and the metric of the chunk's rows, all
  // issued before the first use (the states only where registers allow:
  // not for 16 FP64 rows)
  constexpr bool PF = !(sizeof(T) == 8 && MM == 16);
  T y[MM][NV], wj[MM], bn[MM];
  V xin[PF ? MM : 1];
  T bprev;  // beta of the row before the chunk's first row
  bprev = cs[j0 + 2 * min(q0, n - 1) - 1];
#pragma unroll
  for (int i = 0; i < MM; ++i) {
    const int j = j0 + 2 * min(q0 + i, n - 1);  // in range for every thread
    wj[i] = wl[j];
    bn[i] = cs[j + 1];
    const V g = vgr[eidx(j)];
    if constexpr (PF) xin[i] = vin[eidx(j)];
#pragma unroll
    for (int v = 0; v < NV; ++v) y[i][v] = g.v[v] * rfac;
  }
  auto coef = [&](int i, T& ai, T& bi, T& ci_) {
    const T bm = (i == 0) ? bprev : bn[i - 1];  // beta_{j-1}
    const int q = q0 + i;
    bi = wj[i] * dfac + hdt * (bn[i] + bm);
    ai = (q > 0) ? -hdt * bm : T(0);
    ci_ = (q < n - 1) ? -hdt * bn[i] : T(0);
  };

  // forward elimination of the interior rows 0 .. mi-1
  T cp[MM], l[MM], r[MM];
  T cprev = T(0), lprev = T(0), rlast = T(0);
  T yprev[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) yprev[v] = T(0);
#pragma unroll
  for (int i = 0; i < MM; ++i) {
    if (i < mi) {
      T ai, bi, ci_;
      coef(i, ai, bi, ci_);
      const T inv = rcp(bi - ai * cprev);
      cp[i] = ci_ * inv;
#pragma unroll
      for (int v = 0; v < NV; ++v) y[i][v] = (y[i][v] - ai * yprev[v]) * inv;
      l[i] = -ai * (i == 0 ? T(1) : lprev) * inv;
      if (i == mi - 1) rlast = -ci_ * inv;
      cprev = cp[i];
      lprev = l[i];
#pragma unroll
      for (int v = 0; v < NV; ++v) yprev[v] = y[i][v];
    }
  }
  // back substitution: interior row i = y_i + l_i s_{p-1} + r_i s_p
  {
    T yn[NV], ln = T(0), rn = T(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) yn[v] = T(0);
#pragma unroll
    for (int i = MM - 1; i >= 0; --i) {
      if (i < mi) {
        if (i == mi - 1) {
          r[i] = rlast;
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) y[i][v] -= cp[i] * yn[v];
          l[i] -= cp[i] * ln;
          r[i] = -cp[i] * rn;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) yn[v] = y[i][v];
        ln = l[i];
        rn = r[i];
      }
    }
  }

  // publish the first interior row for the chunk before
  xF[t] = (mi >= 1) ? 1 : 0;
  xL[t] = (mi >= 1) ? l[0] : T(0);
  xR[t] = (mi >= 1) ? r[0] : T(0);
#pragma unroll
  for (int v = 0; v < NV; ++v) xY[v][t] = (mi >= 1) ? y[0][v] : T(0);
  __syncthreads();

  // interface equation of chunk p: A s_{p-1} + B s_p + C s_{p+1} = D
  T eA = T(0), eB = T(1), eC = T(0), eD[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) eD[v] = T(0);
  if (mp > 0) {
    T ae = T(0), be = T(1), ce = T(0), de[NV], yl[NV], ll = T(0), rl = T(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      de[v] = T(0);
      yl[v] = T(0);
    }
#pragma unroll
    for (int i = 0; i < MM; ++i) {
      if (i == mi) {
        coef(i, ae, be, ce);
#pragma unroll
        for (int v = 0; v < NV; ++v) de[v] = y[i][v];
      }
      if (i == mi - 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) yl[v] = y[i][v];
        ll = l[i];
        rl = r[i];
      }
    }
    // the row before the interface: interior row mi-1, or s_{p-1} itself
    const bool has_int = mi >= 1;
    // the row after: the next chunk's first interior row, or s_{p+1} itself
    const int tn = t + CW;  // same column, chunk p + 1
    const bool nxt = (p + 1 < P) && xF[tn] != 0;
    const T l0n = nxt ? xL[tn] : T(0), r0n = nxt ? xR[tn] : T(0);
    eA = ae * (has_int ? ll : T(1));
    eB = be + ae * (has_int ? rl : T(0)) + ce * l0n;
    eC = ce * (nxt ? r0n : T(1));
#pragma unroll
    for (int v = 0; v < NV; ++v)
      eD[v] = de[v] - ae * (has_int ? yl[v] : T(0)) - ce * (nxt ? xY[v][tn] : T(0));
  }

  // parallel cyclic reduction over the P interface equations of the column
  sA[t] = eA;
  sB[t] = eB;
  sC[t] = eC;
#pragma unroll
  for (int v = 0; v < NV; ++v) sD[v][t] = eD[v];
  __syncthreads();
  for (int st = 1; st < P; st <<= 1) {
    const bool lo = p - st >= 0, hi = p + st < P;
    const int tl = t - st * CW, th = t + st * CW;
    const T Al = lo ? sA[tl] : T(0), Bl = lo ? sB[tl] : T(1), Cl = lo ? sC[tl] : T(0);
    const T Ah = hi ? sA[th] : T(0), Bh = hi ? sB[th] : T(1), Ch = hi ? sC[th] : T(0);
    T Dl[NV], Dh[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Dl[v] = lo ? sD[v][tl] : T(0);
      Dh[v] = hi ? sD[v][th] : T(0);
    }
    const T k1 = eA * rcp(Bl), k2 = eC * rcp(Bh);
    eB = eB - Cl * k1 - Ah * k2;
#pragma unroll
    for (int v = 0; v < NV; ++v) eD[v] = eD[v] - Dl[v] * k1 - Dh[v] * k2;
    eA = -Al * k1;
    eC = -Ch * k2;
    __syncthreads();
    sA[t] = eA;
    sB[t] = eB;
    sC[t] = eC;
#pragma unroll
    for (int v = 0; v < NV; ++v) sD[v][t] = eD[v];
    __syncthreads();
  }
  T s_me[NV];
  const T invB = rcp(eB);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    s_me[v] = eD[v] * invB;
    xY[v][t] = s_me[v];  // every thread has passed the last barrier's reads of xY
  }
  __syncthreads();
  T s_left[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) s_left[v] = (p > 0) ? xY[v][t - CW] : T(0);

  if (!col_ok) return;
#pragma unroll
  for (int i = 0; i < MM; ++i) {
    if (i < mp) {
      const long long ix = eidx(j0 + 2 * (q0 + i));
      V x;
      if constexpr (PF)
        x = xin[i];
      else
        x = vin[ix];
      V mom;
#pragma unroll
      for (int v = 0; v < NV; ++v) mom.v[v] = T(0);
      if (a.beta != T(0) && !(a.rose != nullptr && a.rose[blk.curve] != 0)) {  // uniform per workgroup
        const V prev = vout[ix];
#pragma unroll
        for (int v = 0; v < NV; ++v) mom.v[v] = a.beta * (x.v[v] - prev.v[v]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v)
        x.v[v] += ((i < mi) ? y[i][v] + l[i] * s_left[v] + r[i] * s_me[v] : s_me[v]) + mom.v[v];
      vout[ix] = clean(x);
    }
  }
}

template <typename T, int MM>
void launch_simp_mm(int n_blocks, hipStream_t s, const SimpArgs<T>& a) {
  if (a.odd)
    hipLaunchKernelGGL((simp_kernel<T, 1, MM>), dim3(n_blocks), dim3(kSimpThreads), 0, s, a);
  else
    hipLaunchKernelGGL((simp_kernel<T, 2, MM>), dim3(n_blocks), dim3(kSimpThreads), 0, s, a);
}

template <typename T>
hipError_t launch_simp(int chunk, int n_blocks, hipStream_t s, const SimpArgs<T>& a) {
  if (n_blocks <= 0) return hipSuccess;
  if (chunk == 8)
    launch_simp_mm<T, 8>(n_blocks, s, a);
  else if (chunk == 16)
    launch_simp_mm<T, 16>(n_blocks, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_simp_f32(int chunk, int n_blocks, hipStream_t s, const SimpArgs<float>& a) {
  return launch_simp<float>(chunk, n_blocks, s, a);
}
hipError_t launch_simp_f64(int chunk, int n_blocks, hipStream_t s, const SimpArgs<double>& a) {
  return launch_simp<double>(chunk, n_blocks, s, a);
}

}  // namespace ksc
