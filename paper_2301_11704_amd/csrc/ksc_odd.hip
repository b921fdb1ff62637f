// Fused tile kernels of the inversion-symmetric subspace for one (dtype, n_x)
// pair: compiled once per pair with -DKSC_T=<float|double> -DKSC_TNAME=<f32|f64>
// -DKSC_NX=<8..256>, and once per dtype with -DKSC_ODD_CONV for the boundary
// conversions.
#include "ksc_launch_odd.hpp"

#ifndef KSC_T
#error "KSC_T must be defined"
#endif

#define KSC_CAT2(a, b) a##b
#define KSC_CAT(a, b) KSC_CAT2(a, b)

namespace ksc {

#ifndef KSC_ODD_CONV
// The fused kernel of the inversion-symmetric subspace (rows of K reals).
template <int NX, typename T, int W, int MODE>
__global__ __launch_bounds__(64 * W) void odd_kernel(KernelArgs<T> a) {
  extern __shared__ __align__(16) double smem_d[];
  T* buf = reinterpret_cast<T*>(smem_d);
  for (int i = blockIdx.x; i < a.n_tiles; i += gridDim.x) {
    const int tile = a.tile_base + i;
    const TileDev td = a.tiles[tile];
    const CurveDev cd = a.curves[td.curve];
    if (MODE == MODE_STEP && a.active != nullptr && a.active[td.curve] == 0) {
      tile_copy_odd<NX, T, W>(a, cd, td.curve, td.j0, tile);
      continue;
    }
    tile_body_odd<NX, T, W, MODE>(a, cd, td.curve, td.j0, tile, buf);
  }
}

template <typename T, int W, int NX>
constexpr bool odd_tile_fits() {
  constexpr int K = (NX - 1) / 3;
  return odd_supported<NX, T>() && ((64 * W + 2) * K * int(sizeof(T)) + 32 <= 160 * 1024);
}

template <int NX, typename T, int W>
static hipError_t launch_odd_w(int mode, int grid, size_t lds, hipStream_t s, const KernelArgs<T>& a,
                               hipEvent_t e0, hipEvent_t e1) {
  if constexpr (!odd_tile_fits<T, W, NX>()) {
    return hipErrorInvalidValue;
  } else {
  switch (mode) {
    case MODE_J:
      hipExtLaunchKernelGGL((odd_kernel<NX, T, W, MODE_J>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
      break;
    case MODE_GRAD:
      hipExtLaunchKernelGGL((odd_kernel<NX, T, W, MODE_GRAD>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
      break;
    default:
      hipExtLaunchKernelGGL((odd_kernel<NX, T, W, MODE_STEP>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
      break;
  }
  return hipGetLastError();
  }
}

hipError_t KSC_CAT(KSC_CAT(KSC_CAT(launch_odd_, KSC_TNAME), _), KSC_NX)(
    int W, int mode, int grid, size_t lds, hipStream_t s, const KernelArgs<KSC_T>& a, hipEvent_t e0,
    hipEvent_t e1) {
  switch (W) {
    case 1: return launch_odd_w<KSC_NX, KSC_T, 1>(mode, grid, lds, s, a, e0, e1);
    case 2: return launch_odd_w<KSC_NX, KSC_T, 2>(mode, grid, lds, s, a, e0, e1);
    default: return launch_odd_w<KSC_NX, KSC_T, 4>(mode, grid, lds, s, a, e0, e1);
  }
}


#else
// Inversion-symmetric subspace conversions, one row per lane.
//   spec -> phys: u_n = -2 sum_k b_k sin(2 pi k n / N) for n = 0..N-1.
//   phys -> spec: b_k = Im u_hat_k = -(1/N) sum_n u_n sin(2 pi k n / N); only
//   the odd part u_n - u_{N-n} contributes, so a field outside the subspace
//   is projected onto it.
template <int NX, typename T>
__global__ __launch_bounds__(64) void p2s_odd_kernel(int rows, const T* __restrict__ phys,
                                                     T* __restrict__ spec) {
  constexpr int K = (NX - 1) / 3, M2 = NX / 2;
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= rows) return;
  const T* x = phys + (long long)r * NX;
  T f[M2];
  sfor<M2>([&](auto Nn) {
    constexpr int n = Nn;
    if constexpr (n == 0)
      f[0] = T(0);
    else
      f[n] = x[n] - x[NX - n];
  });
  T F2[K + 1];
  dst1_x2<M2, K + 1, T>(f, F2);
  constexpr T h = T(-0.5 / NX);
  sfor<K>([&](auto Ee) {
    constexpr int e = Ee;
    spec[(long long)r * K + e] = h * F2[e + 1];
  });
}

template <int NX, typename T>
__global__ __launch_bounds__(64) void s2p_odd_kernel(int rows, const T* __restrict__ spec,
                                                     T* __restrict__ phys) {
  constexpr int K = (NX - 1) / 3, M2 = NX / 2;
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= rows) return;
  T f[M2];
  sfor<M2>([&](auto Kk) {
    constexpr int k = Kk;
    if constexpr (k >= 1 && k <= K)
      f[k] = -spec[(long long)r * K + (k - 1)];
    else
      f[k] = T(0);
  });
  T u[M2];
  dst1_x2<M2, M2, T>(f, u);
  T* x = phys + (long long)r * NX;
  sfor<NX>([&](auto Nn) {
    constexpr int n = Nn;
    if constexpr (n < M2)
      x[n] = u[n];
    else if constexpr (n == M2)
      x[n] = T(0);
    else
      x[n] = -u[NX - n];
  });
}

template <typename T>
static hipError_t conv_odd(bool to_spec, int nx, int rows, hipStream_t s, const T* src, T* dst) {
  const int g = (rows + 63) / 64;
#define KSC_CONV_ODD_CASE(N)                                                                  \
  case N:                                                                                     \
    if constexpr (odd_supported<N, T>()) {                                                    \
      if (to_spec)                                                                            \
        hipLaunchKernelGGL((p2s_odd_kernel<N, T>), dim3(g), dim3(64), 0, s, rows, src, dst);  \
      else                                                                                    \
        hipLaunchKernelGGL((s2p_odd_kernel<N, T>), dim3(g), dim3(64), 0, s, rows, src, dst);  \
      break;                                                                                  \
    } else {                                                                                  \
      return hipErrorInvalidValue;                                                            \
    }
  switch (nx) {
    KSC_CONV_ODD_CASE(8)
    KSC_CONV_ODD_CASE(16)
    KSC_CONV_ODD_CASE(32)
    KSC_CONV_ODD_CASE(64)
    KSC_CONV_ODD_CASE(128)
    KSC_CONV_ODD_CASE(256)
    default: return hipErrorInvalidValue;
  }
#undef KSC_CONV_ODD_CASE
  return hipGetLastError();
}

hipError_t KSC_CAT(launch_p2s_odd_, KSC_TNAME)(int nx, int rows, hipStream_t s, const KSC_T* phys,
                                               KSC_T* spec) {
  return conv_odd<KSC_T>(true, nx, rows, s, phys, spec);
}
hipError_t KSC_CAT(launch_s2p_odd_, KSC_TNAME)(int nx, int rows, hipStream_t s, const KSC_T* spec,
                                               KSC_T* phys) {
  return conv_odd<KSC_T>(false, nx, rows, s, spec, phys);
}

#endif

}  // namespace ksc
