// Fused tile kernels for one (dtype, n_x) pair.  Compiled once per pair with
// -DKSC_T=<float|double> -DKSC_TNAME=<f32|f64> -DKSC_NX=<8..256>, or with
// -DKSC_MIXED for the mixed-n_x kernel.
#include "ksc_launch.hpp"

#ifndef KSC_T
#error "KSC_T must be defined"
#endif

namespace ksc {

template <int NX, typename T, int W, int MODE>
__global__ __launch_bounds__(64 * W, (tile_waves_per_simd<NX, T>())) void fused_kernel(KernelArgs<T> a) {
  extern __shared__ __align__(16) double smem_d[];
  constexpr int KM = (NX - 1) / 3 + 1;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_d);
  double* red = nullptr;
  for (int i = blockIdx.x; i < a.n_tiles; i += gridDim.x) {
    const int tile = a.tile_base + i;
    const TileDev td = a.tiles[tile];
    const CurveDev cd = a.curves[td.curve];
    if (MODE == MODE_STEP && a.active != nullptr && a.active[td.curve] == 0) {
      tile_copy<NX, T, W>(a, cd, td.curve, td.j0, tile);
      continue;
    }
    if constexpr (lanes_per_row<NX, T>() > 2)
      tile_body_lanes<NX, T, W, MODE, lanes_per_row<NX, T>()>(a, cd, td.curve, td.j0, tile, buf);
    else if constexpr (lanes_per_row<NX, T>() == 2)
      tile_body2<NX, T, W, MODE>(a, cd, td.curve, td.j0, tile, buf);
    else
      tile_body<NX, T, W, MODE>(a, cd, td.curve, td.j0, tile, buf, red);
  }
}

#ifdef KSC_MIXED
template <typename T, int W, int MODE>
__global__ __launch_bounds__(64 * W) void mixed_kernel(KernelArgs<T> a) {
  extern __shared__ __align__(16) double smem_d[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_d);
  double* red = nullptr;
  for (int i = blockIdx.x; i < a.n_tiles; i += gridDim.x) {
    const int tile = a.tile_base + i;
    const TileDev td = a.tiles[tile];
    const CurveDev cd = a.curves[td.curve];
    // the tile's grid size is the same on every lane: branch on it as a
    // wave-uniform (scalar) value, not as a per-lane condition
    const int nx = __builtin_amdgcn_readfirstlane(cd.n_x);
    if (MODE == MODE_STEP && a.active != nullptr && a.active[td.curve] == 0) {
      switch (nx) {
        case 32: tile_copy<32, T, W>(a, cd, td.curve, td.j0, tile); break;
        case 64: tile_copy<64, T, W>(a, cd, td.curve, td.j0, tile); break;
        default: tile_copy<128, T, W>(a, cd, td.curve, td.j0, tile); break;
      }
      continue;
    }
    switch (nx) {
      case 32: tile_body<32, T, W, MODE>(a, cd, td.curve, td.j0, tile, buf, red); break;
      case 64: tile_body<64, T, W, MODE>(a, cd, td.curve, td.j0, tile, buf, red); break;
      default:
        if constexpr (lanes_per_row<128, T>() == 2)
          tile_body2<128, T, W, MODE>(a, cd, td.curve, td.j0, tile, buf);
        else
          tile_body<128, T, W, MODE>(a, cd, td.curve, td.j0, tile, buf, red);
        break;
    }
  }
}
#endif

template <int NX, typename T>
__global__ __launch_bounds__(64) void p2s_kernel(int rows, const T* __restrict__ phys,
                                                 cplx<T>* __restrict__ spec) {
  constexpr int KM = (NX - 1) / 3 + 1;
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= rows) return;
  T x[NX];
  sfor<NX>([&](auto Nn) {
    constexpr int n = Nn;
    x[n] = phys[(long long)r * NX + n];
  });
  cplx<T> X[KM];
  phys_to_spec<NX, KM, T>(x, X);
  sfor<KM>([&](auto Kk) {
    constexpr int k = Kk;
    spec[(long long)r * KM + k] = X[k];
  });
}

template <int NX, typename T>
__global__ __launch_bounds__(64) void s2p_kernel(int rows, const cplx<T>* __restrict__ spec,
                                                 T* __restrict__ phys) {
  constexpr int KM = (NX - 1) / 3 + 1;
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= rows) return;
  cplx<T> X[KM];
  sfor<KM>([&](auto Kk) {
    constexpr int k = Kk;
    X[k] = spec[(long long)r * KM + k];
  });
  T x[NX];
  spec_to_phys<NX, KM, T>(X, x);
  sfor<NX>([&](auto Nn) {
    constexpr int n = Nn;
    phys[(long long)r * NX + n] = x[n];
  });
}

}  // namespace ksc

#define KSC_CAT2(a, b) a##b
#define KSC_CAT(a, b) KSC_CAT2(a, b)

namespace ksc {

// Tile shapes whose LDS staging buffer exceeds the 160 KB of a gfx950 CU are
// not instantiated.
template <typename T, int W, int NX>
constexpr bool tile_fits() {
  constexpr int KM = (NX - 1) / 3 + 1;
  constexpr int R = 64 * W / lanes_per_row<NX, T>();
  if constexpr (lanes_per_row<NX, T>() > 2)
    return lanes_lds_bytes(NX, KM, R, lanes_per_row<NX, T>(), int(sizeof(T))) <= 160 * 1024;
  return ((R + 2) * KM + 2) * int(sizeof(cplx<T>)) + 64 * W * u_stash<NX, T>() * int(sizeof(T)) <=
         160 * 1024;
}

#ifndef KSC_MIXED
template <int NX, typename T, int W>
static hipError_t launch_w(int mode, int grid, size_t lds, hipStream_t s, const KernelArgs<T>& a,
                           hipEvent_t e0, hipEvent_t e1) {
  if constexpr (!tile_fits<T, W, NX>()) {
    return hipErrorInvalidValue;
  } else {
  switch (mode) {
    case MODE_J:
      hipExtLaunchKernelGGL((fused_kernel<NX, T, W, MODE_J>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
      break;
    case MODE_GRAD:
      hipExtLaunchKernelGGL((fused_kernel<NX, T, W, MODE_GRAD>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
      break;
    default:
      hipExtLaunchKernelGGL((fused_kernel<NX, T, W, MODE_STEP>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
      break;
  }
  return hipGetLastError();
  }
}

hipError_t KSC_CAT(KSC_CAT(KSC_CAT(launch_fused_, KSC_TNAME), _), KSC_NX)(
    int W, int mode, int grid, size_t lds, hipStream_t s, const KernelArgs<KSC_T>& a, hipEvent_t e0,
    hipEvent_t e1) {
  switch (W) {
    case 1: return launch_w<KSC_NX, KSC_T, 1>(mode, grid, lds, s, a, e0, e1);
    case 2: return launch_w<KSC_NX, KSC_T, 2>(mode, grid, lds, s, a, e0, e1);
    default: return launch_w<KSC_NX, KSC_T, 4>(mode, grid, lds, s, a, e0, e1);
  }
}

#else
template <typename T, int W>
static hipError_t launch_mw(int mode, int grid, size_t lds, hipStream_t s, const KernelArgs<T>& a,
                            hipEvent_t e0, hipEvent_t e1) {
  if constexpr (!(tile_fits<T, W, 128>() && tile_fits<T, W, 64>())) {
    return hipErrorInvalidValue;
  } else {
  switch (mode) {
    case MODE_J:  // J-only mixed batches launch per grid size (host)
      return hipErrorInvalidValue;
    case MODE_GRAD:
      hipExtLaunchKernelGGL((mixed_kernel<T, W, MODE_GRAD>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
      break;
    default:
      hipExtLaunchKernelGGL((mixed_kernel<T, W, MODE_STEP>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
      break;
  }
  return hipGetLastError();
  }
}

hipError_t KSC_CAT(launch_mixed_, KSC_TNAME)(int W, int mode, int grid, size_t lds, hipStream_t s,
                                            const KernelArgs<KSC_T>& a, hipEvent_t e0,
                                            hipEvent_t e1) {
  switch (W) {
    case 1: return launch_mw<KSC_T, 1>(mode, grid, lds, s, a, e0, e1);
    case 2: return launch_mw<KSC_T, 2>(mode, grid, lds, s, a, e0, e1);
    default: return launch_mw<KSC_T, 4>(mode, grid, lds, s, a, e0, e1);
  }
}

template <typename T>
static hipError_t conv(bool to_spec, int nx, int rows, hipStream_t s, const void* src, void* dst) {
  const int g = (rows + 63) / 64;
#define KSC_CONV_CASE(N)                                                                      \
  case N:                                                                                     \
    if (to_spec)                                                                              \
      hipLaunchKernelGGL((p2s_kernel<N, T>), dim3(g), dim3(64), 0, s, rows,                   \
                         static_cast<const T*>(src), static_cast<cplx<T>*>(dst));             \
    else                                                                                      \
      hipLaunchKernelGGL((s2p_kernel<N, T>), dim3(g), dim3(64), 0, s, rows,                   \
                         static_cast<const cplx<T>*>(src), static_cast<T*>(dst));             \
    break;
  switch (nx) {
    KSC_CONV_CASE(8)
    KSC_CONV_CASE(16)
    KSC_CONV_CASE(32)
    KSC_CONV_CASE(64)
    KSC_CONV_CASE(128)
    KSC_CONV_CASE(256)
    default: return hipErrorInvalidValue;
  }
#undef KSC_CONV_CASE
  return hipGetLastError();
}

hipError_t KSC_CAT(KSC_CAT(launch_p2s_, KSC_TNAME), )(int nx, int rows, hipStream_t s,
                                                      const KSC_T* phys, cplx<KSC_T>* spec) {
  return conv<KSC_T>(true, nx, rows, s, phys, spec);
}
hipError_t KSC_CAT(KSC_CAT(launch_s2p_, KSC_TNAME), )(int nx, int rows, hipStream_t s,
                                                      const cplx<KSC_T>* spec, KSC_T* phys) {
  return conv<KSC_T>(false, nx, rows, s, spec, phys);
}
#endif

}  // namespace ksc
