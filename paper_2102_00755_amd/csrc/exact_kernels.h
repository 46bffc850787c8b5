// Pointwise kernels of the exact discrete gradient: reverse-mode
// differentiation of the forward iteration (App. B, Alg. 1's forward loop;
// Sec. 2.1's absorption operator L when set), run backwards in time over the
// adjoint variables of the velocities (vb), split densities (rb) and
// pressure (pb).  The spectral parts of the reverse step (the transposed
// staggered derivatives d-^T = -d+, d+^T = -d-, and the fractional Laplacians
// A = |k|^{y-2}, B = |k|^{y-1}, both symmetric) run through the library's
// derivative and transform passes; these kernels hold the rest.
#pragma once

#include "fwi_common.h"

namespace fwi {

// pb[receiver voxel] += r^n: the residual row n (traces - observed, or a
// given residual) at the receivers (the loss term M^T r^n)
template <typename T>
__global__ void k_ex_inject(T* pb, const int32_t* rec_lin, const T* traces, const T* obs, int is_resid, int n,
                            int n_rec) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rec) return;
  const size_t k = (size_t)n * n_rec + r;
  const T v = is_resid ? obs[k] : traces[k] - obs[k];
  pb[rec_lin[r]] += v;
}

// gacc[g] += pb[Gamma voxel g] * hist[g]: the c0-derivative of the equation
// of state of step n against its adjoint pressure (FP64 accumulation)
template <typename T>
__global__ void k_ex_accum(double* gacc, const T* pb, const int32_t* gam_lin, const T* hist, int n_gam) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_gam; g += gridDim.x * blockDim.x)
    gacc[g] += (double)pb[gam_lin[g]] * (double)hist[g];
}

// Inputs of the transposed absorption terms: eP = eta c0^2 pb, tP = tau c0^2 pb
// with tau = -2 alpha0 c0^{y-1}, eta = 2 alpha0 c0^y tan(pi y / 2)
template <typename T>
__global__ void k_ex_coef(const T* c, const T* alpha0, T alpha0_u, double y, double two_tan, const T* pb, T* eP,
                          T* tP, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double cv = (double)c[i];
    const double al = alpha0 ? (double)alpha0[i] : (double)alpha0_u;
    const double cy1 = pow(cv, y - 1.0);
    const double q = cv * cv * (double)pb[i];
    eP[i] = (T)(two_tan * al * cv * cy1 * q);
    tP[i] = (T)(-2.0 * al * cy1 * q);
  }
}

// Transposed density update of axis a (rho_a <- L_a (L_a rho_a - dt rho0 u_a),
// s = sum rho_a, p = c0^2 (s + tau A[rho0 sum u] - eta B[s])):
//   sb = c0^2 pb - FB   (FB = B[eta c0^2 pb]; absent without absorption)
//   t  = L_a (rb_a + sb),  rb_a <- L_a t,  ub = rho0 FA - dt rho0 t
// (FA = A[tau c0^2 pb]); L_a is the normal-grid PML factor along axis a.
template <typename T>
__global__ void k_ex_rho(const T* c, const T* pb, const T* FB, const T* FA, T* rb, T* ub, const T* lam, int axis,
                         Dims d, T dt_rho0, T rho0) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < d.nfield;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % d.nx);
    const long long r = i / d.nx;
    const int y = (int)(r % d.ny), z = (int)(r / d.ny);
    const T la = lam[axis == 0 ? x : (axis == 1 ? y : z)];
    const T cv = c[i];
    T sb = cv * cv * pb[i];
    if (FB) sb -= FB[i];
    const T t = la * (rb[i] + sb);
    rb[i] = la * t;
    ub[i] = (FA ? rho0 * FA[i] : (T)0) - dt_rho0 * t;
  }
}

// Transposed velocity update of axis a (v_a <- Ls_a (Ls_a v_a - dt/rho0 d+_a p)):
// t = Ls_a vb_a, vb_a <- Ls_a t; t goes to out (then pb += dt/rho0 d-_a t)
template <typename T>
__global__ void k_ex_vel(T* vb, T* out, const T* lam_s, int axis, Dims d) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < d.nfield;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % d.nx);
    const long long r = i / d.nx;
    const int y = (int)(r % d.ny), z = (int)(r / d.ny);
    const T la = lam_s[axis == 0 ? x : (axis == 1 ? y : z)];
    const T t = la * vb[i];
    vb[i] = la * t;
    out[i] = t;
  }
}

}  // namespace fwi
