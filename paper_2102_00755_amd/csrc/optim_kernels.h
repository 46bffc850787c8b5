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

// ---- grid transfers of the coarse-to-fine scheme (Sec. 2.4, App. C) --------

// Blackman window over signed frequency index k of a coarse axis with Nyquist
// index K: 0.42 + 0.5 cos(pi k/K) + 0.08 cos(2 pi k/K), zero beyond |k| = K
__device__ __forceinline__ double blackman_k(double k, double K) {
  const double a = fabs(k) / K;
  if (a > 1.0) return 0.0;
  return 0.42 + 0.5 * cos(3.14159265358979323846 * a) + 0.08 * cos(2.0 * 3.14159265358979323846 * a);
}

// Source index and factor of fine frequency k (signed) on an axis of coarse
// length nc embedded in fine length nf >= nc: returns the coarse index, or -1
// when k lies outside the coarse band; `half` is set for the even Nyquist bin
// split over +-nc/2.
__device__ __forceinline__ int embed_index(int k, int nc, int nf, bool* half) {
  *half = false;
  if (nc % 2 == 0) {
    const int K = nc / 2;
    if (k > -K && k < K) return k < 0 ? k + nc : k;
    if (k == K || k == -K) {
      if (nf > nc) { *half = true; return K; }
      return k == -K ? K : -1;     // equal sizes: the single Nyquist bin (stored at -K)
    }
    return -1;
  }
  const int K = (nc - 1) / 2;
  if (k >= -K && k <= K) return k < 0 ? k + nc : k;
  return -1;
}

// Fine half spectrum [nz_f][ny_f][px_f] from the coarse one: the coarse DFT
// embedded in the fine frequency grid (zero elsewhere, the even Nyquist bin
// split in halves), times the separable Blackman window of the coarse band
// when window != 0, times scale (1 / N_coarse: the transforms are
// unnormalised).
template <typename T>
__global__ void k_spec_embed(const cplx<T>* cs, Dims dc, cplx<T>* fs, Dims df, int window, double scale) {
  using C = cplx<T>;
  const long long nf = (long long)df.px * df.ny * df.nz;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nf; e += (long long)gridDim.x * blockDim.x) {
    const int kx = (int)(e % df.px);
    const long long r = e / df.px;
    const int iy = (int)(r % df.ny), iz = (int)(r / df.ny);
    const int ky = iy < (df.ny + 1) / 2 ? iy : iy - df.ny;
    const int kz = iz < (df.nz + 1) / 2 ? iz : iz - df.nz;
    C v = cmake<C>((T)0, (T)0);
    bool hx = false, hy, hz;
    int cx = -1;
    if (kx <= df.M) {
      if (kx < dc.M) cx = kx;
      else if (kx == dc.M) { cx = kx; hx = df.M > dc.M; }
    }
    const int cy = embed_index(ky, dc.ny, df.ny, &hy);
    const int cz = embed_index(kz, dc.nz, df.nz, &hz);
    if (cx >= 0 && cy >= 0 && cz >= 0) {
      double f = scale * (hx ? 0.5 : 1.0) * (hy ? 0.5 : 1.0) * (hz ? 0.5 : 1.0);
      if (window)
        f *= blackman_k(kx, 0.5 * dc.nx) * blackman_k(ky, 0.5 * dc.ny) * blackman_k(kz, 0.5 * dc.nz);
      const C c = gld(cs + ((size_t)cz * dc.ny + cy) * dc.px + cx);
      v = cmake<C>((T)(f * (double)c.x), (T)(f * (double)c.y));
    }
    gst(fs + e, v);
  }
}

// I0(x), the modified Bessel function of the first kind of order 0, from its
// power series sum_k ((x/2)^2)^k / (k!)^2 (terms until they stop changing the sum)
__device__ __forceinline__ double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((double)k * (double)k);
    const double next = sum + term;
    if (next == sum) break;
    sum = next;
  }
  return sum;
}

// Kaiser-windowed sinc resampling of time series in [nt_in][nch] to
// out [nt_out][nch] (one thread per output value, taps summed in increasing n):
//   out[m] = scale sum_n in[n] 2 fc dt_in sinc(2 fc tau) I0(beta sqrt(1-(tau/tw)^2)) / I0(beta),
//   tau = m dt_out - n dt_in, |tau| <= tw
template <typename T>
__global__ void k_resample_time(const T* in, int nt_in, int nch, double dt_in, T* out, int nt_out, double dt_out,
                                double fc, double beta, double tw, double scale) {
  // tau = t_m - n dt_in rounded as written (no fused multiply-add): taps lying
  // exactly on the window edge are then included exactly as the definition says
#pragma clang fp contract(off)
  const double pi = 3.14159265358979323846;
  const double i0b = bessel_i0(beta);
  const long long total = (long long)nt_out * nch;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(e / nch), ch = (int)(e % nch);
    const double tm = m * dt_out;
    // candidate taps one wider on each side; the support test |tau| <= tw is
    // applied to each tap's own tau so that taps exactly on the edge count
    int n0 = (int)floor((tm - tw) / dt_in) - 1, n1 = (int)ceil((tm + tw) / dt_in) + 1;
    n0 = max(n0, 0);
    n1 = min(n1, nt_in - 1);
    double acc = 0.0;
    for (int n = n0; n <= n1; ++n) {
      const double tau = tm - n * dt_in;
      if (fabs(tau) > tw) continue;
      const double x = 2.0 * fc * tau;
      const double sinc = (x == 0.0) ? 1.0 : sin(pi * x) / (pi * x);
      const double r = fmax(1.0 - (tau / tw) * (tau / tw), 0.0);
      const double win = bessel_i0(beta * sqrt(r)) / i0b;
      acc += (double)gld(in + (size_t)n * nch + ch) * 2.0 * fc * dt_in * sinc * win;
    }
    gst(out + e, (T)(scale * acc));
  }
}

}  // namespace fwi
