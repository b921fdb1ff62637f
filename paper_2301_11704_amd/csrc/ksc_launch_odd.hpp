// Launchers of the inversion-symmetric subspace kernels (ksc_odd.hip), between
// the host runtime and the kernel translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "ksc_odd.hpp"

namespace ksc {

// Fused tile kernel on rows of K reals for curves with n_x == NX; arguments as
// for launch_fused_* (ksc_launch.hpp).  Returns hipErrorInvalidValue for a
// (dtype, n_x, W) without a kernel (odd_supported, LDS size).
#define KSC_DECLARE_ODD(TNAME, T, NX)                                                       \
  hipError_t launch_odd_##TNAME##_##NX(int W, int mode, int grid, size_t lds, hipStream_t s, \
                                       const KernelArgs<T>& a, hipEvent_t e0, hipEvent_t e1);
KSC_DECLARE_ODD(f32, float, 8)
KSC_DECLARE_ODD(f32, float, 16)
KSC_DECLARE_ODD(f32, float, 32)
KSC_DECLARE_ODD(f32, float, 64)
KSC_DECLARE_ODD(f32, float, 128)
KSC_DECLARE_ODD(f32, float, 256)
KSC_DECLARE_ODD(f64, double, 8)
KSC_DECLARE_ODD(f64, double, 16)
KSC_DECLARE_ODD(f64, double, 32)
KSC_DECLARE_ODD(f64, double, 64)
KSC_DECLARE_ODD(f64, double, 128)
KSC_DECLARE_ODD(f64, double, 256)
#undef KSC_DECLARE_ODD

// Boundary conversions: phys (N_x samples per row) <-> K sine coefficients
// b_k = Im u_hat_k per row (phys -> spec keeps the odd part).
hipError_t launch_p2s_odd_f32(int nx, int rows, hipStream_t s, const float* phys, float* spec);
hipError_t launch_s2p_odd_f32(int nx, int rows, hipStream_t s, const float* spec, float* phys);
hipError_t launch_p2s_odd_f64(int nx, int rows, hipStream_t s, const double* phys, double* spec);
hipError_t launch_s2p_odd_f64(int nx, int rows, hipStream_t s, const double* spec, double* phys);

}  // namespace ksc
