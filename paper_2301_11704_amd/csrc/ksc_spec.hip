// Spectral-d/ds kernels for one (dtype, n_x) pair: the D~ products on matrix
// cores and the row kernel.  Compiled once per pair with -DKSC_T=<float|double>
// -DKSC_TNAME=<f32|f64> -DKSC_NX=<8..128>.
#include "ksc_launch_spec.hpp"

#ifndef KSC_T
#error "KSC_T must be defined"
#endif

#define KSC_CAT2(a, b) a##b
#define KSC_CAT(a, b) KSC_CAT2(a, b)

namespace ksc {

// One workgroup per (group, row block of 64, block of spec_cb<NCP>() curves)
// over all the groups of one n_x (a group: curves that share n_s); the
// workgroup finds its group in the small group table.
template <typename T, int NCP, bool TRANS, int EPI>
__global__ __launch_bounds__(256) void spec_gemm_kernel(SpecArgs<T> sa,
                                                        const SpecGroupDev* __restrict__ groups,
                                                        int n_groups) {
  __shared__ __align__(16) double lds[spec_gemm_lds<NCP>()];
  const int bid = blockIdx.x;
  int g = 0;
  while (g + 1 < n_groups && bid >= groups[g + 1].block0) ++g;  // uniform over the workgroup
  const SpecGroupDev G = groups[g];
  const int local = bid - G.block0;
  SpecArgs<T> ga = sa;
  ga.curves = sa.curves + G.first;
  spec_gemm_body<T, NCP, TRANS, EPI>(ga, G.count, (local / G.row_blocks) * spec_cb<NCP>(),
                                     (local % G.row_blocks) * kSpecRowsPerBlock, lds);
}

template <int NX, typename T, int W, int MODE>
__global__ __launch_bounds__(64 * W) void spec_row_kernel(SpecRowArgs<T> sa) {
  extern __shared__ __align__(16) double smem_d[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_d);
  for (int i = blockIdx.x; i < sa.a.n_tiles; i += gridDim.x) {
    const int tile = sa.a.tile_base + i;
    const TileDev td = sa.a.tiles[tile];
    const CurveDev cd = sa.a.curves[td.curve];
    spec_row_body<NX, T, W, MODE>(sa, cd, td.curve, td.j0, tile, buf);
  }
}

// Staging buffers of one row tile: state rows and d/ds rows, each with slack.
template <typename T, int W, int NX>
constexpr bool spec_row_fits() {
  constexpr int KM = (NX - 1) / 3 + 1;
  constexpr int E = 16 / int(sizeof(cplx<T>));
  return 2 * (64 * W * KM + 2 * E) * int(sizeof(cplx<T>)) <= 160 * 1024;
}

template <int NX, typename T, int W>
static hipError_t launch_row_w(int mode, int grid, size_t lds, hipStream_t s,
                               const SpecRowArgs<T>& a, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (!(spec_supported<NX, T>() && spec_row_fits<T, W, NX>())) {
    return hipErrorInvalidValue;
  } else {
    switch (mode) {
      case MODE_J:
        hipExtLaunchKernelGGL((spec_row_kernel<NX, T, W, MODE_J>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
        break;
      default:
        hipExtLaunchKernelGGL((spec_row_kernel<NX, T, W, MODE_GRAD>), dim3(grid), dim3(64 * W), lds, s, e0, e1, 0, a);
        break;
    }
    return hipGetLastError();
  }
}

hipError_t KSC_CAT(KSC_CAT(KSC_CAT(launch_spec_row_, KSC_TNAME), _), KSC_NX)(
    int W, int mode, int grid, size_t lds, hipStream_t s, const SpecRowArgs<KSC_T>& a, hipEvent_t e0,
    hipEvent_t e1) {
  switch (W) {
    case 1: return launch_row_w<KSC_NX, KSC_T, 1>(mode, grid, lds, s, a, e0, e1);
    case 2: return launch_row_w<KSC_NX, KSC_T, 2>(mode, grid, lds, s, a, e0, e1);
    default: return launch_row_w<KSC_NX, KSC_T, 4>(mode, grid, lds, s, a, e0, e1);
  }
}

hipError_t KSC_CAT(KSC_CAT(KSC_CAT(launch_spec_gemm_, KSC_TNAME), _), KSC_NX)(
    int epi, const SpecGroupDev* groups, int n_groups, int n_blocks, hipStream_t s,
    const SpecArgs<KSC_T>& a, hipEvent_t e0, hipEvent_t e1) {
  constexpr int NCP = spec_ncp(KSC_NX);
  static_assert(spec_curves_per_block(KSC_NX) == spec_cb<NCP>(), "host and kernel blocking agree");
  const dim3 grid(n_blocks);
  if constexpr (!spec_supported<KSC_NX, KSC_T>()) {
    return hipErrorInvalidValue;
  } else {
    switch (epi) {
      case EPI_Y:
        hipExtLaunchKernelGGL((spec_gemm_kernel<KSC_T, NCP, false, EPI_Y>), grid, dim3(256), 0, s, e0, e1, 0, a, groups, n_groups);
        break;
      case EPI_GRAD:
        hipExtLaunchKernelGGL((spec_gemm_kernel<KSC_T, NCP, true, EPI_GRAD>), grid, dim3(256), 0, s, e0, e1, 0, a, groups, n_groups);
        break;
      default:
        hipExtLaunchKernelGGL((spec_gemm_kernel<KSC_T, NCP, true, EPI_STEP>), grid, dim3(256), 0, s, e0, e1, 0, a, groups, n_groups);
        break;
    }
    return hipGetLastError();
  }
}

}  // namespace ksc
