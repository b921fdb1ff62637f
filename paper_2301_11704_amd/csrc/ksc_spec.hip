// Spectral-d/ds kernels for one (dtype, n_x) pair: the D~ products on matrix
// cores, the deterministic split-k reduction and the row kernels (full space
// and inversion-symmetric subspace).  Compiled once per pair with
// -DKSC_T=<float|double> -DKSC_TNAME=<f32|f64> -DKSC_NX=<8..128>.
#include "ksc_launch_spec.hpp"

#ifndef KSC_T
#error "KSC_T must be defined"
#endif

#define KSC_CAT2(a, b) a##b
#define KSC_CAT(a, b) KSC_CAT2(a, b)

namespace ksc {

// One workgroup per (group, row block of 64, block of spec_cb<NCP>() curves)
// over all the groups of one n_x (a group: curves that share n_s), times
// grid.y parts of the k range; the workgroup finds its group in the small
// group table.
struct SpecTile {
  int count, cbase, row0, first;
};
__device__ __forceinline__ SpecTile spec_tile(const SpecGroupDev* __restrict__ groups,
                                              int n_groups, int bid, int cb) {
  int g = 0;
  while (g + 1 < n_groups && bid >= groups[g + 1].block0) ++g;  // uniform over the workgroup
  const SpecGroupDev G = groups[g];
  const int local = bid - G.block0;
  return SpecTile{G.count, (local / G.row_blocks) * cb, (local % G.row_blocks) * kSpecRowsPerBlock,
                  G.first};
}

template <typename T, int NCP, bool TRANS, int EPI, bool ODD>
__global__ __launch_bounds__(256, 3) void spec_gemm_kernel(SpecArgs<T> sa,
                                                        const SpecGroupDev* __restrict__ groups,
                                                        int n_groups) {
  __shared__ __align__(16) double lds[spec_gemm_lds<NCP>()];
  const SpecTile tl = spec_tile(groups, n_groups, blockIdx.x, spec_cb<NCP>());
  SpecArgs<T> ga = sa;
  ga.curves = sa.curves + tl.first;
  spec_gemm_body<T, NCP, TRANS, EPI, ODD>(ga, tl.count, tl.cbase, tl.row0, blockIdx.y, lds);
}

template <typename T, int NCP, int EPI, bool ODD>
__global__ __launch_bounds__(256) void spec_reduce_kernel(SpecArgs<T> sa,
                                                          const SpecGroupDev* __restrict__ groups,
                                                          int n_groups) {
  const SpecTile tl = spec_tile(groups, n_groups, blockIdx.x, spec_cb<NCP>());
  SpecArgs<T> ga = sa;
  ga.curves = sa.curves + tl.first;
  spec_reduce_body<T, NCP, EPI, ODD>(ga, tl.count, tl.cbase, tl.row0, blockIdx.y);
}

template <int NX, typename T, int W, int MODE, bool ODD>
__global__ __launch_bounds__(64 * W) void spec_row_kernel(SpecRowArgs<T> sa) {
  extern __shared__ __align__(16) double smem_d[];
  for (int i = blockIdx.x; i < sa.a.n_tiles; i += gridDim.x) {
    const int tile = sa.a.tile_base + i;
    const TileDev td = sa.a.tiles[tile];
    const CurveDev cd = sa.a.curves[td.curve];
    if constexpr (ODD)
      spec_row_body_odd<NX, T, W, MODE>(sa, cd, td.curve, td.j0, tile, reinterpret_cast<T*>(smem_d));
    else
      spec_row_body<NX, T, W, MODE>(sa, cd, td.curve, td.j0, tile,
                                    reinterpret_cast<cplx<T>*>(smem_d));
  }
}

// Staging buffers of one row tile: state rows and d/ds rows, each with slack.
template <typename T, int W, int NX, bool ODD>
constexpr bool spec_row_fits() {
  constexpr int K = (NX - 1) / 3;
  constexpr int bytes = ODD ? 2 * (64 * W * K + 2 * (16 / int(sizeof(T)))) * int(sizeof(T))
                            : 2 * (64 * W * (K + 1) + 2 * (16 / int(sizeof(cplx<T>)))) *
                                  int(sizeof(cplx<T>));
  return bytes <= 160 * 1024;
}

template <int NX, typename T, int W, bool ODD>
static hipError_t launch_row_w(int mode, int grid, size_t lds, hipStream_t s,
                               const SpecRowArgs<T>& a, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (!(spec_supported<NX, T>() && spec_row_fits<T, W, NX, ODD>())) {
    return hipErrorInvalidValue;
  } else {
    switch (mode) {
      case MODE_J:
        hipExtLaunchKernelGGL((spec_row_kernel<NX, T, W, MODE_J, ODD>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
        break;
      default:
        hipExtLaunchKernelGGL((spec_row_kernel<NX, T, W, MODE_GRAD, ODD>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
        break;
    }
    return hipGetLastError();
  }
}

template <bool ODD>
static hipError_t launch_row(int W, int mode, int grid, size_t lds, hipStream_t s,
                             const SpecRowArgs<KSC_T>& a, hipEvent_t e0, hipEvent_t e1) {
  switch (W) {
    case 1: return launch_row_w<KSC_NX, KSC_T, 1, ODD>(mode, grid, lds, s, a, e0, e1);
    case 2: return launch_row_w<KSC_NX, KSC_T, 2, ODD>(mode, grid, lds, s, a, e0, e1);
    default: return launch_row_w<KSC_NX, KSC_T, 4, ODD>(mode, grid, lds, s, a, e0, e1);
  }
}

hipError_t KSC_CAT(KSC_CAT(KSC_CAT(launch_spec_row_, KSC_TNAME), _), KSC_NX)(
    int odd, int W, int mode, int grid, size_t lds, hipStream_t s, const SpecRowArgs<KSC_T>& a,
    hipEvent_t e0, hipEvent_t e1) {
  return odd ? launch_row<true>(W, mode, grid, lds, s, a, e0, e1)
             : launch_row<false>(W, mode, grid, lds, s, a, e0, e1);
}

template <bool ODD>
static hipError_t launch_gemm(int epi, const SpecGroupDev* groups, int n_groups, int n_blocks,
                              hipStream_t s, const SpecArgs<KSC_T>& a, hipEvent_t e0,
                              hipEvent_t e1) {
  constexpr int NCP = spec_ncp(KSC_NX, ODD);
  static_assert(spec_curves_per_block(KSC_NX, ODD) == spec_cb<NCP>(),
                "host and kernel blocking agree");
  if constexpr (!spec_supported<KSC_NX, KSC_T>()) {
    return hipErrorInvalidValue;
  } else {
    const dim3 grid(n_blocks, a.kparts);
    const bool split = a.kparts > 1;
    hipEvent_t eg = split ? nullptr : e1;  // the last launch stamps the end
    using T = KSC_T;
    switch (epi) {
      case EPI_Y:
        hipExtLaunchKernelGGL((spec_gemm_kernel<T, NCP, false, EPI_Y, ODD>), grid, dim3(256), 0, s, e0, eg, 0, a, groups, n_groups);
        break;
      case EPI_GRAD:
        hipExtLaunchKernelGGL((spec_gemm_kernel<T, NCP, true, EPI_GRAD, ODD>), grid, dim3(256), 0, s, e0, eg, 0, a, groups, n_groups);
        break;
      default:
        hipExtLaunchKernelGGL((spec_gemm_kernel<T, NCP, true, EPI_STEP, ODD>), grid, dim3(256), 0, s, e0, eg, 0, a, groups, n_groups);
        break;
    }
    if (split) {
      // one thread per element of a product tile (64 rows x CB curves x NCP columns)
      const dim3 rg(n_blocks, (64 * spec_cb<NCP>() * NCP + 255) / 256);
      switch (epi) {
        case EPI_Y:
          hipExtLaunchKernelGGL((spec_reduce_kernel<T, NCP, EPI_Y, ODD>), rg, dim3(256), 0, s, nullptr, e1, 0, a, groups, n_groups);
          break;
        case EPI_GRAD:
          hipExtLaunchKernelGGL((spec_reduce_kernel<T, NCP, EPI_GRAD, ODD>), rg, dim3(256), 0, s, nullptr, e1, 0, a, groups, n_groups);
          break;
        default:
          hipExtLaunchKernelGGL((spec_reduce_kernel<T, NCP, EPI_STEP, ODD>), rg, dim3(256), 0, s, nullptr, e1, 0, a, groups, n_groups);
          break;
      }
    }
    return hipGetLastError();
  }
}

hipError_t KSC_CAT(KSC_CAT(KSC_CAT(launch_spec_gemm_, KSC_TNAME), _), KSC_NX)(
    int odd, int epi, const SpecGroupDev* groups, int n_groups, int n_blocks, hipStream_t s,
    const SpecArgs<KSC_T>& a, hipEvent_t e0, hipEvent_t e1) {
  return odd ? launch_gemm<true>(epi, groups, n_groups, n_blocks, s, a, e0, e1)
             : launch_gemm<false>(epi, groups, n_groups, n_blocks, s, a, e0, e1);
}

}  // namespace ksc
