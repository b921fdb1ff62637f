// Internal launcher interface between the host runtime and the kernel
// translation units (one per dtype and grid size, compiled in parallel).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "ksc_lanes.hpp"

namespace ksc {

// Fused tile kernel for curves that all have n_x == NX.
//   W     waves per workgroup (1, 2 or 4): a tile emits 64W - 2 rows
//   mode  MODE_J, MODE_GRAD or MODE_STEP
//   grid  workgroups; grid < a.n_tiles makes each workgroup walk the tile
//         list with stride grid (persistent launch)
//   e0,e1 nullable HIP events stamped by the dispatch itself at kernel start
//         and end (kernel timing)
#define KSC_DECLARE_LAUNCH(TNAME, T, NX)                                                      \
  hipError_t launch_fused_##TNAME##_##NX(int W, int mode, int grid, size_t lds, hipStream_t s, \
                                         const KernelArgs<T>& a, hipEvent_t e0, hipEvent_t e1);
KSC_DECLARE_LAUNCH(f32, float, 8)
KSC_DECLARE_LAUNCH(f32, float, 16)
KSC_DECLARE_LAUNCH(f32, float, 32)
KSC_DECLARE_LAUNCH(f32, float, 64)
KSC_DECLARE_LAUNCH(f32, float, 128)
KSC_DECLARE_LAUNCH(f32, float, 256)
KSC_DECLARE_LAUNCH(f64, double, 8)
KSC_DECLARE_LAUNCH(f64, double, 16)
KSC_DECLARE_LAUNCH(f64, double, 32)
KSC_DECLARE_LAUNCH(f64, double, 64)
KSC_DECLARE_LAUNCH(f64, double, 128)
KSC_DECLARE_LAUNCH(f64, double, 256)
#undef KSC_DECLARE_LAUNCH

// One launch over curves of mixed n_x in {32, 64, 128}: every workgroup
// dispatches each tile to the body compiled for that tile's grid size.
hipError_t launch_mixed_f32(int W, int mode, int grid, size_t lds, hipStream_t s,
                            const KernelArgs<float>& a, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_mixed_f64(int W, int mode, int grid, size_t lds, hipStream_t s,
                            const KernelArgs<double>& a, hipEvent_t e0, hipEvent_t e1);

// Boundary conversions for one curve of grid size nx (rows handled one per lane).
hipError_t launch_p2s_f32(int nx, int rows, hipStream_t s, const float* phys, cplx<float>* spec);
hipError_t launch_s2p_f32(int nx, int rows, hipStream_t s, const cplx<float>* spec, float* phys);
hipError_t launch_p2s_f64(int nx, int rows, hipStream_t s, const double* phys, cplx<double>* spec);
hipError_t launch_s2p_f64(int nx, int rows, hipStream_t s, const cplx<double>* spec, double* phys);

}  // namespace ksc
