// Launchers of the spectral-d/ds kernels (ksc_spec.hip), between the host
// runtime and the kernel translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "ksc_spec.hpp"

namespace ksc {

// Rows of a D~ product tile and the padded column count of one curve's state
// viewed as a real matrix (2(K+1) columns in the full space, K in the odd
// subspace, rounded up to 16).
constexpr int kSpecRowsPerBlock = 64;
constexpr int spec_ncp(int nx, bool odd = false) {
  return (((odd ? (nx - 1) / 3 : 2 * ((nx - 1) / 3 + 1)) + 15) / 16) * 16;
}

// One row per lane is required (N_x sizeof(T) <= 512 B).
template <int NX, typename T>
constexpr bool spec_supported() {
  return NX * int(sizeof(T)) <= 512;
}

// Curves per workgroup of the products (ksc_spec.hpp spec_cb) for n_x.
constexpr int spec_curves_per_block(int nx, bool odd = false) {
  return (spec_ncp(nx, odd) / 16) >= 3 ? 1 : (spec_ncp(nx, odd) / 16) == 2 ? 2 : 3;
}

// epi: EPI_Y (Y = D_t B), EPI_GRAD or EPI_STEP (with op(D~) = D~^T) over the
// n_groups groups (device table) of curves with this n_x, n_blocks workgroups
// in all; a.curves is the SpecDev array the groups index.
// odd != 0: the inversion-symmetric subspace (rows of K reals).
#define KSC_DECLARE_SPEC(TNAME, T, NX)                                                          \
  hipError_t launch_spec_gemm_##TNAME##_##NX(int odd, int epi, const SpecGroupDev* groups,      \
                                             int n_groups, int n_blocks, hipStream_t s,          \
                                             const SpecArgs<T>& a, hipEvent_t e0, hipEvent_t e1); \
  hipError_t launch_spec_row_##TNAME##_##NX(int odd, int W, int mode, int grid, size_t lds,      \
                                            hipStream_t s, const SpecRowArgs<T>& a, hipEvent_t e0, \
                                            hipEvent_t e1);
KSC_DECLARE_SPEC(f32, float, 8)
KSC_DECLARE_SPEC(f32, float, 16)
KSC_DECLARE_SPEC(f32, float, 32)
KSC_DECLARE_SPEC(f32, float, 64)
KSC_DECLARE_SPEC(f32, float, 128)
KSC_DECLARE_SPEC(f64, double, 8)
KSC_DECLARE_SPEC(f64, double, 16)
KSC_DECLARE_SPEC(f64, double, 32)
KSC_DECLARE_SPEC(f64, double, 64)
#undef KSC_DECLARE_SPEC

}  // namespace ksc
