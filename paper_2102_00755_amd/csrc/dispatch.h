// Run-time dispatch from grid sizes to the compile-time FFT lengths.
#pragma once

#include "kernels.h"

namespace fwi {

// Supported FFT lengths (axis lengths ny, nz and half lengths nx/2).
#define FWI_LENGTHS(X) \
  X(8) X(12) X(16) X(24) X(32) X(40) X(48) X(56) X(64) X(80) X(96) X(112) X(128) X(160) X(192) X(224) \
  X(240) X(256) X(320) X(384) X(448) X(480) X(512)

inline bool length_supported(int L) {
  switch (L) {
#define FWI_CASE_TRUE(N) case N: return true;
    FWI_LENGTHS(FWI_CASE_TRUE)
#undef FWI_CASE_TRUE
    default: return false;
  }
}

// Each returns hipErrorInvalidValue for an unsupported length or tile width
// (tb = row segment of an axis-pass tile in bytes: 64 or 128); plan = radix
// plan of the transforms (0 or 1, make_plan; lengths whose plans coincide
// run plan 0).
template <typename T>
hipError_t launch_axis_y(int L, bool inv, int tb, int plan, dim3 grid, hipStream_t st, const AxisArgs<T>& a);
template <typename T>
hipError_t launch_axis_z(int L, bool inv, int tb, int plan, dim3 grid, hipStream_t st, const AxisArgs<T>& a);
template <typename T>
hipError_t launch_axis_zm(int L, int tb, int plan, dim3 grid, hipStream_t st, const AxisArgs<T>& a);
// the Z1 of the lossy step with the A[d] output (k_axis_z_minus_ad, grid.y = slots)
template <typename T>
hipError_t launch_axis_zma(int L, int tb, int plan, dim3 grid, hipStream_t st, const AxisArgs<T>& a);
template <typename T>
hipError_t launch_axis_zp(int L, int tb, int plan, dim3 grid, hipStream_t st, const AxisArgs<T>& a);
template <typename T>
hipError_t launch_axis_ys(int L, int tb, int plan, dim3 grid, hipStream_t st, const AxisArgs<T>& a);
// the inverse y pass of the time step (k_axis_y_div, grid.y = slots)
template <typename T>
hipError_t launch_axis_yd(int L, int tb, int plan, dim3 grid, hipStream_t st, const AxisArgs<T>& a);
template <typename T>
hipError_t launch_axis_yv(int L, int tb, int plan, dim3 grid, hipStream_t st, const AxisArgs<T>& a);
// absorption z pass (k_axis_z_frac)
template <typename T>
hipError_t launch_axis_zf(int L, int tb, int plan, dim3 grid, hipStream_t st, const AxisArgs<T>& a);
// lossy x passes: part 0 = k_x_lossy_rho, part 1 = k_x_lossy_eos; kind = SpKind
template <typename T>
hipError_t launch_x_lossy(int M, int part, int kind, dim3 grid, hipStream_t st, const X2Args<T>& a);
// plan: radix plan of the x transforms (0 or 1, make_plan)
template <typename T> hipError_t launch_x_vel(int M, int plan, dim3 grid, hipStream_t st, const XArgs<T>& a);
template <typename T>
hipError_t launch_x_den(int M, int mode, int plan, dim3 grid, hipStream_t st, const X2Args<T>& a);
template <typename T> hipError_t launch_x_r2c(int M, dim3 grid, hipStream_t st, const XArgs<T>& a, const T* in, int f);
template <typename T>
hipError_t launch_x_c2r(int M, dim3 grid, hipStream_t st, const XArgs<T>& a, T* out, int f, const cplx<T>* mult);

template <typename T> inline int x_lines_per_block(int M) { return x_lpb<T>(M); }
template <typename T> inline int x_lines_per_block_vel(int M) { return x_lpb_vel<T>(M); }
template <typename T> inline int x_lines_per_block_den(int M) { return x_lpb_den<T>(M); }
template <typename T> inline int x_lines_per_block_den(int M, int mode) { return x_lpb_den_mode<T>(M, mode); }
template <typename T> inline int x_lines_per_block_eos(int M) { return x_lpb_eos<T>(M); }

}  // namespace fwi
