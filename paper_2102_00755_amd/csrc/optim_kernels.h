// Device vector kernels of the stochastic L-BFGS outer loop (App. D,
// Algorithm 2): deterministic FP64 dot products, the two-loop recursion with
// its scalars kept in device memory (no host round trip), axpby, projection
// onto bounds, the squared-slowness parametrisation u = 1/c0^2 (Sec. 2.4)
// and the gather / scatter between the grid and Gamma-compact vectors.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fwi_common.h"

namespace fwi {

constexpr int RED_BLOCKS = 512;   // partial sums of a dot product (fixed: deterministic)
constexpr int RED_NT = 256;

// part[b] = sum over the grid-stride share of block b of a[i] b[i] (FP64)
template <typename T>
__global__ void __launch_bounds__(RED_NT) k_dot_partial(const T* a, const T* b, long long n, double* part) {
  __shared__ double red[RED_NT];
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)RED_NT + threadIdx.x; i < n; i += (long long)gridDim.x * RED_NT)
    s += (double)gld(a + i) * (double)gld(b + i);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = RED_NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) gst(part + blockIdx.x, red[0]);
}

// Finish a dot product d = sum(part) in a fixed order and store
//   mode 0: out[0] = d
//   mode 1: out[0] = 1 / d                       (rho_j = 1 / y_j^T s_j)
//   mode 2: out[0] = rho[0] * d                  (alpha_j = rho_j s_j^T q)
//   mode 3: out[0] = alpha[0] - rho[0] * d       (alpha_j - beta_j)
__global__ void __launch_bounds__(RED_NT) k_dot_final(const double* part, int np, int mode, const double* rho,
                                                      const double* alpha, double* out) {
  __shared__ double red[RED_NT];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += RED_NT) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = RED_NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double d = red[0];
    double v = d;
    if (mode == 1) v = 1.0 / d;
    else if (mode == 2) v = rho[0] * d;
    else if (mode == 3) v = alpha[0] - rho[0] * d;
    out[0] = v;
  }
}

// y[i] += sign * coef[0] * x[i] with the coefficient read from device memory
template <typename T>
__global__ void k_axpy_dev(T* y, const T* x, const double* coef, double sign, long long n) {
  const T c = (T)(sign * coef[0]);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    gst(y + i, gld(y + i) + c * gld(x + i));
}

// y = a x + b y (x may be null: y = b y); with b == 0 y is not read, so it
// may hold anything (a copy into uninitialised memory)
template <typename T>
__global__ void k_axpby(long long n, T a, const T* x, T b, T* y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    gst(y + i, (x ? a * gld(x + i) : (T)0) + (b != (T)0 ? b * gld(y + i) : (T)0));
}

template <typename T>
__global__ void k_clip(long long n, T* x, T lo, T hi) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    gst(x + i, max(min(gld(x + i), hi), lo));
}

// squared slowness u = 1 / c^2:
//   mode 0: out = 1 / in^2                (c -> u)
//   mode 1: out = 1 / sqrt(in)            (u -> c)
//   mode 2: out = -1/2 aux^3 in           (dJ/du from dJ/dc at c = aux: dc/du = -c^3 / 2)
template <typename T>
__global__ void k_sqslowness(long long n, int mode, const T* in, const T* aux, T* out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const T v = gld(in + i);
    T r;
    if (mode == 0) r = (T)1 / (v * v);
    else if (mode == 1) r = (T)1 / sqrt(v);
    else {
      const T c = gld(aux + i);
      r = (T)-0.5 * c * c * c * v;
    }
    gst(out + i, r);
  }
}

// compact[k] = full[idx[k]]  /  full[idx[k]] = compact[k]
template <typename T>
__global__ void k_gather(const T* full, const int32_t* idx, long long n, T* compact) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    gst(compact + k, gld(full + gld(idx + k)));
}
template <typename T>
__global__ void k_scatter(const T* compact, const int32_t* idx, long long n, T* full) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    gst(full + gld(idx + k), gld(compact + k));
}

}  // namespace fwi
