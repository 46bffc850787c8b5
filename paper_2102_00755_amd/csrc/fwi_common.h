// Common device types of the MI355X k-space TR-gradient library.
//
// Field layout: [nz][ny][nx] reals, x fastest.  Spectra: [nz][ny][px]
// complex, where px >= nx/2 + 1 is the row pitch of the half spectrum along
// x (real-to-complex along x, complex along y and z).  px is a multiple of
// 128 bytes, so that every axis-pass tile row starts on a cache line.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fwi {

template <typename T> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename T> using cplx = typename cplx_t<T>::type;

template <typename C> __device__ __forceinline__ C cmake(decltype(C::x) a, decltype(C::x) b) {
  C r; r.x = a; r.y = b; return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return cmake<C>(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse): rot<false>(a) = -i a
template <bool INV, typename C> __device__ __forceinline__ C crot(C a) {
  return INV ? cmake<C>(-a.y, a.x) : cmake<C>(a.y, -a.x);
}

// Global-memory loads and stores through address space 1.  Pointers read
// from memory (the slot table) are generic to the compiler, and generic
// (flat) accesses count against the LDS wait counter as well: every LDS wait
// of a transform would then also wait for the HBM loads still in flight.
#define FWI_GAS __attribute__((address_space(1)))
template <int N> struct gword;
template <> struct gword<4> { typedef unsigned int type; };
template <> struct gword<8> { typedef unsigned int type __attribute__((ext_vector_type(2))); };
template <> struct gword<16> { typedef unsigned int type __attribute__((ext_vector_type(4))); };
template <typename V> __device__ __forceinline__ V gld(const V* p) {
  using W = typename gword<sizeof(V)>::type;
  return __builtin_bit_cast(V, *(const FWI_GAS W*)p);
}
template <typename V> __device__ __forceinline__ void gst(V* p, V v) {
  using W = typename gword<sizeof(V)>::type;
  *(FWI_GAS W*)p = __builtin_bit_cast(W, v);
}

// Operator tables of one handle (device pointers), all built on the host in
// FP64 and rounded once to T.
template <typename T> struct Tables {
  const cplx<T>* tw_x;     // W_{M}^m, m < M (M = nx/2), forward sign
  const cplx<T>* tw_y;     // W_{ny}^m
  const cplx<T>* tw_z;     // W_{nz}^m
  const cplx<T>* rtw;      // W_{nx}^k, k <= M (real<->complex along x)
  const T* ksq[3];         // k_a^2 per axis (x: k < M+1; y: ny; z: nz)
  const cplx<T>* sfac_p[3];  // i k_a exp(+i k_a dx / 2) per axis
  const cplx<T>* sfac_m[3];  // i k_a exp(-i k_a dx / 2)
  const T* pml_n[3];       // Lambda on the normal grid per axis
  const T* pml_s[3];       // Lambda^s on the staggered grid per axis
};

// Pointers of one simulation slot (one wave simulation of one problem).
template <typename T> struct Slot {
  T* v[3];
  T* rho[3];
  cplx<T>* spec[3];
};

// Sparse geometry per x-line (line = y + ny * z), CSR over lines.
struct LineGeom {
  const int32_t* src_off;   // [nlines+1] -> src_x / src_id
  const int16_t* src_x;
  const int32_t* src_id;
  const int32_t* rec_off;   // [nlines+1] -> rec_x / rec_id
  const int16_t* rec_x;
  const int32_t* rec_id;
  const int32_t* bnd_off;   // [nlines+1] -> tape index range of the line
  const int16_t* bnd_x;     // x of every dGamma voxel, tape order
  const int32_t* gam_off;   // [nlines+1] -> Gamma index range of the line
  const int16_t* gam_x;     // x of every Gamma voxel, Gamma order
};

struct Dims {
  int nx, ny, nz;     // grid
  int M;              // nx / 2
  int px;             // spectrum row pitch (complex elements)
  long long nfield;   // nx*ny*nz
  long long nspec;    // px*ny*nz
  int nlines;         // ny*nz
  int n_src, n_rec, n_bnd, n_gam;
  int nt;
};

}  // namespace fwi
