// HIP kernels of one k-space time step (App. B) and of the TR gradient
// (Alg. 1), written for gfx950.
//
// One time step of one simulation is eight launches, each one HBM pass:
//   Y3  forward y-FFT of p_hat                       (1 field in place)
//   Z2  forward z-FFT, x kappa * i k_a e^{+i k_a dx/2} for a = x,y,z,
//       inverse z-FFT                                 (1 field -> 3 fields)
//   Y4  inverse y-FFT                                 (3 fields in place)
//   X1  inverse x (C2R) -> d+_a p, velocity update with PML, forward x (R2C)
//   Y1  forward y-FFT                                 (3 fields)
//   Z1  forward z-FFT, x kappa * i k_a e^{-i k_a dx/2}, inverse z-FFT
//   Y2  inverse y-FFT                                 (3 fields)
//   X2  inverse x (C2R) -> d-_a v_a, split-density update with PML, source /
//       adjoint injection or Dirichlet imposition, equation of state, sensor
//       sampling, boundary tape, gradient accumulation, forward x (R2C) of p
// The k-space operator kappa = sinc(c_ref dt |k| / 2) is evaluated on the
// fly (a Taylor series in u = (c_ref dt |k| / 2)^2) instead of being read
// from HBM, and the 1/(nx ny nz) normalisation of the three unnormalised
// inverse transforms is folded into the same multiplier.
#pragma once

#include "fft_engine.h"

namespace fwi {

// ----------------------------------------------------------------------------
// launch geometry
// ----------------------------------------------------------------------------
// axis-pass tile width: 64-byte row segments (8 FP32 / 4 FP64 complex); measured
// faster than 128-byte segments because twice as many tiles fit in LDS per CU
template <typename T> constexpr int axis_tw() { return 64 / (int)(2 * sizeof(T)); }
constexpr int axis_nt(int L, int TW) {
  int n = L * TW / 8;
  n = n < 64 ? 64 : (n > 256 ? 256 : n);
  return (n + 63) / 64 * 64;
}
// x-lines per workgroup of the x passes.  LDS regions hold the lines as
// columns without padding, so their column counts (LPB, 2 LPB, 3 LPB) must
// keep 64-bit accesses conflict-free: an odd LPB gives odd or 2-mod-4
// strides, measured conflict-free on gfx950 (strides with a factor of 4 and
// gapped runs are not).
template <typename T> constexpr int odd_lpb(int budget, int M) {
  int l = budget / (M * (int)sizeof(T));
  if (l > 15) l = 15;
  if (l < 1) l = 1;
  if ((l & 1) == 0) l -= 1;
  return l;
}
template <typename T> constexpr int x_lpb_vel(int M) { return odd_lpb<T>(5120, M); }
template <typename T> constexpr int x_lpb_den(int M) { return odd_lpb<T>(3072, M); }
template <typename T> constexpr int x_lpb(int M) { return odd_lpb<T>(4096, M); }
constexpr int X_NT = 256;

// sinc(sqrt(u)) = sum_n (-1)^n u^n / (2n+1)!, n = 0..10 (accurate to double
// rounding for sqrt(u) <= pi/2; the host rejects larger arguments)
template <typename T> __device__ __forceinline__ T sinc_u(T u) {
  T r = (T)(1.0 / 51090942171709440000.0);
  r = r * u - (T)(1.0 / 121645100408832000.0);
  r = r * u + (T)(1.0 / 355687428096000.0);
  r = r * u - (T)(1.0 / 1307674368000.0);
  r = r * u + (T)(1.0 / 6227020800.0);
  r = r * u - (T)(1.0 / 39916800.0);
  r = r * u + (T)(1.0 / 362880.0);
  r = r * u - (T)(1.0 / 5040.0);
  r = r * u + (T)(1.0 / 120.0);
  r = r * u - (T)(1.0 / 6.0);
  r = r * u + (T)1.0;
  return r;
}

// ----------------------------------------------------------------------------
// axis passes (y and z), tiles of L rows x TW consecutive kx columns
// ----------------------------------------------------------------------------
// Slots processed by one launch: i < na -> slot0 + i, else slot1 + (i - na)
// (the adjoint slots and the forward / TR slots live in two ranges).
template <typename T> struct AxisArgs {
  const Slot<T>* slots;
  int slot0;   // first slot of the first range
  int na;      // slots in the first range
  int slot1;   // first slot of the second range
  int nf;      // fields per slot
  int f0;      // first field
  Dims d;
  Tables<T> tb;
  T scale;     // 1 / (nx ny nz)
  T kap_a;     // (c_ref dt / 2)^2
};

__device__ __forceinline__ int slot_of(int i, int slot0, int na, int slot1) {
  return i < na ? slot0 + i : slot1 + (i - na);
}

// All global loads of a thread are issued before the first LDS store so that
// the whole tile is in flight at once (memory-level parallelism is what
// bounds a streaming pass).
template <typename T, int L, int TW, int NT>
__device__ __forceinline__ void tile_load(cplx<T>* buf, const cplx<T>* g, size_t rstride, int ncol) {
  using C = cplx<T>;
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
  C tmp[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    const int r = e / TW, c = e % TW;
    tmp[i] = (c < ncol && (E % NT == 0 || e < E)) ? g[(size_t)r * rstride + c] : cmake<C>((T)0, (T)0);
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if (E % NT == 0 || e < E) buf[e] = tmp[i];
  }
}
template <typename T, int L, int TW, int NT>
__device__ __forceinline__ void tile_store(const cplx<T>* buf, cplx<T>* g, size_t rstride, int ncol) {
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    const int r = e / TW, c = e % TW;
    if (c < ncol && (E % NT == 0 || e < E)) g[(size_t)r * rstride + c] = buf[e];
  }
}

// ---- persistent axis passes -------------------------------------------------
// Each workgroup walks the tile list with stride gridDim.x.  The global loads
// of the next tile are issued into registers right after the current tile has
// been written to LDS, so they are in flight during the current tile's FFTs
// and stores (one tile of prefetch per workgroup).
template <typename T> struct TileRef {
  cplx<T>* g;   // first element of the tile in its field
  int ncol;     // valid columns (ragged last tile)
  int kx0;      // first kx column
  int outer;    // z (y pass) or y (z pass)
  int s, f;     // slot and field
};

template <typename T, int TW>
__device__ __forceinline__ TileRef<T> tile_ref(const AxisArgs<T>& a, int item, int nouter, int nf_tile,
                                               size_t outer_stride) {
  const int ntx = (a.d.M + TW) / TW;
  const int per = ntx * nouter;
  const int si = item / per;
  const int rem = item % per;
  const int outer = rem / ntx, tile = rem % ntx;
  TileRef<T> t;
  t.s = slot_of(si / nf_tile, a.slot0, a.na, a.slot1);
  t.f = a.f0 + si % nf_tile;
  t.kx0 = tile * TW;
  t.g = a.slots[t.s].spec[t.f] + (size_t)outer * outer_stride + (size_t)t.kx0;
  t.ncol = min(TW, a.d.M + 1 - t.kx0);
  t.outer = outer;
  return t;
}

template <typename T, int L, int TW, int NT>
__device__ __forceinline__ void tile_prefetch(cplx<T>* pre, const cplx<T>* g, int ncol, size_t rstride) {
  using C = cplx<T>;
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    const int r = e / TW, c = e % TW;
    pre[i] = (c < ncol && (E % NT == 0 || e < E)) ? g[(size_t)r * rstride + c] : cmake<C>((T)0, (T)0);
  }
}
template <typename T, int L, int TW, int NT>
__device__ __forceinline__ void tile_commit(cplx<T>* buf, const cplx<T>* pre) {
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if (E % NT == 0 || e < E) buf[e] = pre[i];
  }
}

// kappa * scale * i k_f exp(sign i k_f dx / 2) at row r (kz), column kx, y
template <typename T>
__device__ __forceinline__ cplx<T> zmult(const AxisArgs<T>& a, const cplx<T>* const* sfac, int f, int kx, int y,
                                         int r, T ky2) {
  const T u = a.kap_a * (a.tb.ksq[0][kx] + ky2 + a.tb.ksq[2][r]);
  const T kap = sinc_u(u) * a.scale;
  const cplx<T> sf = (f == 0) ? sfac[0][kx] : ((f == 1) ? sfac[1][y] : sfac[2][r]);
  return cscale(sf, kap);
}

enum AxisKind { AK_Y = 0, AK_ZMINUS = 1, AK_ZPLUS = 2 };

// Persistent axis pass over nitems tiles:
//   AK_Y      in-place FFT along y (forward or inverse by INV) of nf fields
//   AK_ZMINUS field f -> F_z^-1 m-_f F_z field f                (Z1)
//   AK_ZPLUS  field 0 -> fields 0,1,2 = F_z^-1 m+_a F_z field 0  (Z2)
template <typename T, int L, int KIND, bool INV>
__global__ void __launch_bounds__(axis_nt(L, axis_tw<T>()))
k_axis_persist(AxisArgs<T> a, int nitems) {
  using C = cplx<T>;
  constexpr int TW = axis_tw<T>();
  constexpr int NT = axis_nt(L, TW);
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
  __shared__ C buf[L * TW];
  const size_t px = a.d.px;
  const int nouter = (KIND == AK_Y) ? a.d.nz : a.d.ny;
  const size_t ostride = (KIND == AK_Y) ? (size_t)a.d.ny * px : px;
  const size_t rstride = (KIND == AK_Y) ? px : (size_t)a.d.ny * px;
  const int nf_tile = (KIND == AK_ZPLUS) ? 1 : a.nf;
  C pre[EPT];
  int item = blockIdx.x;
  if (item < nitems) {
    const TileRef<T> t = tile_ref<T, TW>(a, item, nouter, nf_tile, ostride);
    tile_prefetch<T, L, TW, NT>(pre, t.g, t.ncol, rstride);
  }
  for (; item < nitems; item += gridDim.x) {
    const TileRef<T> t = tile_ref<T, TW>(a, item, nouter, nf_tile, ostride);
    tile_commit<T, L, TW, NT>(buf, pre);
    __syncthreads();
    const int next = item + gridDim.x;
    if (next < nitems) {
      const TileRef<T> tn = tile_ref<T, TW>(a, next, nouter, nf_tile, ostride);
      tile_prefetch<T, L, TW, NT>(pre, tn.g, tn.ncol, rstride);
    }
    if (KIND == AK_Y) {
      lds_fft<T, L, TW, TW, NT, INV>(buf, a.tb.tw_y);
      tile_store<T, L, TW, NT>(buf, t.g, rstride, t.ncol);
    } else if (KIND == AK_ZMINUS) {
      lds_fft<T, L, TW, TW, NT, false>(buf, a.tb.tw_z);
      const T ky2 = a.tb.ksq[1][t.outer];
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = (int)threadIdx.x + i * NT;
        const int r = e / TW, c = e % TW;
        if ((E % NT == 0 || e < E) && c < t.ncol)
          buf[e] = cmul(zmult<T>(a, a.tb.sfac_m, t.f, t.kx0 + c, t.outer, r, ky2), buf[e]);
      }
      __syncthreads();
      lds_fft<T, L, TW, TW, NT, true>(buf, a.tb.tw_z);
      tile_store<T, L, TW, NT>(buf, t.g, rstride, t.ncol);
    } else {
      lds_fft<T, L, TW, TW, NT, false>(buf, a.tb.tw_z);
      const T ky2 = a.tb.ksq[1][t.outer];
      C xr[EPT];
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = (int)threadIdx.x + i * NT;
        if (E % NT == 0 || e < E) xr[i] = buf[e];
      }
      const size_t off = (size_t)(t.g - a.slots[t.s].spec[0]);
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
          const int e = (int)threadIdx.x + i * NT;
          const int r = e / TW, c = e % TW;
          if (E % NT == 0 || e < E) {
            const int kx = min(t.kx0 + c, a.d.M);
            buf[e] = cmul(zmult<T>(a, a.tb.sfac_p, f, kx, t.outer, r, ky2), xr[i]);
          }
        }
        __syncthreads();
        lds_fft<T, L, TW, TW, NT, true>(buf, a.tb.tw_z);
        tile_store<T, L, TW, NT>(buf, a.slots[t.s].spec[f] + off, rstride, t.ncol);
      }
    }
    __syncthreads();
  }
}

// Y pass: in-place FFT along y of nf fields per slot.  L == ny.
template <typename T, int L, bool INV>
__global__ void __launch_bounds__(axis_nt(L, axis_tw<T>()))
k_axis_y(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = axis_tw<T>();
  constexpr int NT = axis_nt(L, TW);
  __shared__ C buf[L * TW];
  const int ntx = (a.d.M + TW) / TW;
  const int tile = blockIdx.x % ntx;
  const int z = blockIdx.x / ntx;
  const int s = slot_of(blockIdx.y / a.nf, a.slot0, a.na, a.slot1);
  const int f = a.f0 + blockIdx.y % a.nf;
  const size_t px = a.d.px;
  C* g = a.slots[s].spec[f] + (size_t)z * L * px + (size_t)tile * TW;
  const int ncol = min(TW, a.d.M + 1 - tile * TW);
  tile_load<T, L, TW, NT>(buf, g, px, ncol);
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, INV>(buf, a.tb.tw_y);
  tile_store<T, L, TW, NT>(buf, g, px, ncol);
}

// Z pass of the velocity divergence terms: field f -> F_z^-1 m-_f F_z field f
// (eq. DisPartDevSt with the minus shift).  L == nz.
template <typename T, int L>
__global__ void __launch_bounds__(axis_nt(L, axis_tw<T>()))
k_axis_z_minus(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = axis_tw<T>();
  constexpr int NT = axis_nt(L, TW);
  __shared__ C buf[L * TW];
  const int ntx = (a.d.M + TW) / TW;
  const int tile = blockIdx.x % ntx;
  const int y = blockIdx.x / ntx;
  const int s = slot_of(blockIdx.y / a.nf, a.slot0, a.na, a.slot1);
  const int f = a.f0 + blockIdx.y % a.nf;
  const size_t px = a.d.px;
  const size_t rstride = (size_t)a.d.ny * px;
  C* g = a.slots[s].spec[f] + (size_t)y * px + (size_t)tile * TW;
  const int ncol = min(TW, a.d.M + 1 - tile * TW);
  tile_load<T, L, TW, NT>(buf, g, rstride, ncol);
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, false>(buf, a.tb.tw_z);
  const T ky2 = a.tb.ksq[1][y];
  const C sfy = a.tb.sfac_m[1][y];
#pragma unroll 4
  for (int e = threadIdx.x; e < L * TW; e += NT) {
    const int r = e / TW, c = e % TW;
    if (c < ncol) {
      const int kx = tile * TW + c;
      const T u = a.kap_a * (a.tb.ksq[0][kx] + ky2 + a.tb.ksq[2][r]);
      const T kap = sinc_u(u) * a.scale;
      const C sf = (f == 0) ? a.tb.sfac_m[0][kx] : ((f == 1) ? sfy : a.tb.sfac_m[2][r]);
      buf[e] = cscale(cmul(sf, buf[e]), kap);
    }
  }
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, true>(buf, a.tb.tw_z);
  tile_store<T, L, TW, NT>(buf, g, rstride, ncol);
}

// Z pass of the pressure gradient: field 0 (p_hat) -> fields 0,1,2 =
// F_z^-1 m+_a F_z p_hat for a = x, y, z.  L == nz.
template <typename T, int L>
__global__ void __launch_bounds__(axis_nt(L, axis_tw<T>()))
k_axis_z_plus(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = axis_tw<T>();
  constexpr int NT = axis_nt(L, TW);
  constexpr int EPT = (L * TW + NT - 1) / NT;
  __shared__ C buf[L * TW];
  const int ntx = (a.d.M + TW) / TW;
  const int tile = blockIdx.x % ntx;
  const int y = blockIdx.x / ntx;
  const int s = slot_of(blockIdx.y, a.slot0, a.na, a.slot1);
  const size_t px = a.d.px;
  const size_t rstride = (size_t)a.d.ny * px;
  const size_t off = (size_t)y * px + (size_t)tile * TW;
  const Slot<T> sl = a.slots[s];
  const int ncol = min(TW, a.d.M + 1 - tile * TW);
  tile_load<T, L, TW, NT>(buf, sl.spec[0] + off, rstride, ncol);
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, false>(buf, a.tb.tw_z);
  C xr[EPT];
  T kr[EPT];
  const T ky2 = a.tb.ksq[1][y];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < L * TW) {
      const int r = e / TW, c = e % TW;
      xr[i] = buf[e];
      const int kx = min(tile * TW + c, a.d.M);
      const T u = a.kap_a * (a.tb.ksq[0][kx] + ky2 + a.tb.ksq[2][r]);
      kr[i] = sinc_u(u) * a.scale;
    }
  }
  const C sfy = a.tb.sfac_p[1][y];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * NT;
      if (e < L * TW) {
        const int r = e / TW, c = e % TW;
        const int kx = min(tile * TW + c, a.d.M);
        const C sf = (f == 0) ? a.tb.sfac_p[0][kx] : ((f == 1) ? sfy : a.tb.sfac_p[2][r]);
        buf[e] = cscale(cmul(sf, xr[i]), kr[i]);
      }
    }
    __syncthreads();
    lds_fft<T, L, TW, TW, NT, true>(buf, a.tb.tw_z);
    tile_store<T, L, TW, NT>(buf, sl.spec[f] + off, rstride, ncol);
  }
}

// ----------------------------------------------------------------------------
// x passes: LPB consecutive x-lines per workgroup, real <-> half spectrum
// ----------------------------------------------------------------------------
// 2D lane layout of the x passes: KT lanes (a power of two >= NK, at most
// the block) run along the fast index k of a line, RT = X_NT / KT rows of
// lanes along the slow index r (line, region or column).  Thread t owns
// k = t % KT + KT ik and r = t / KT + RT ir: every address is a per-thread
// base plus a compile-time offset, and consecutive lanes touch consecutive k.
constexpr int pow2_at_least(int n) {
  int p = 64;
  while (p < n && p < X_NT) p *= 2;
  return p;
}
template <int NR, int NK> struct Lanes {
  static constexpr int KT = pow2_at_least(NK);
  static constexpr int RT = X_NT / KT;
  static constexpr int KI = (NK + KT - 1) / KT;
  static constexpr int RI = (NR + RT - 1) / RT;
  static constexpr int NI = RI * KI;   // items per thread
};
template <int NR, int NK, typename F>
__device__ __forceinline__ void lanes2d(F&& fn) {
  using Ly = Lanes<NR, NK>;
  const int kq = (int)threadIdx.x % Ly::KT;
  const int rq = (int)threadIdx.x / Ly::KT;
#pragma unroll
  for (int ir = 0; ir < Ly::RI; ++ir) {
#pragma unroll
    for (int ik = 0; ik < Ly::KI; ++ik) {
      const int r = rq + ir * Ly::RT;
      const int k = kq + ik * Ly::KT;
      if ((NR % Ly::RT == 0 || r < NR) && (NK % Ly::KT == 0 || k < NK)) fn(ir * Ly::KI + ik, r, k);
    }
  }
}

// Spectra lines (M+1 complex) of NREG regions x LPB lines <-> LDS columns
// col0 + f LPB + l, rows 0..M.
template <typename T, int M, int LPB, int NREG>
__device__ __forceinline__ void x_prefetch_spectra(cplx<T>* pre, cplx<T>* const* spec, int l0, int nl, size_t px) {
  using C = cplx<T>;
  lanes2d<NREG * LPB, M + 1>([&](int i, int r, int k) {
    const int f = r / LPB, l = r % LPB;
    pre[i] = (l < nl) ? spec[f][(size_t)(l0 + l) * px + k] : cmake<C>((T)0, (T)0);
  });
}
template <typename T, int M, int LPB, int TWP, int NREG>
__device__ __forceinline__ void x_commit_spectra(cplx<T>* buf, const cplx<T>* pre, int col0) {
  lanes2d<NREG * LPB, M + 1>([&](int i, int r, int k) {
    const int f = r / LPB, l = r % LPB;
    buf[k * TWP + col0 + f * LPB + l] = pre[i];
  });
}
template <typename T, int M, int LPB, int NREG> struct SpecRegs {
  static constexpr int N = Lanes<NREG * LPB, M + 1>::NI;
};
template <typename T, int M, int LPB, int TWP, int NREG>
__device__ __forceinline__ void x_load_spectra(cplx<T>* buf, cplx<T>* const* spec, int col0, int l0, int nl,
                                               size_t px) {
  cplx<T> tmp[SpecRegs<T, M, LPB, NREG>::N];
  x_prefetch_spectra<T, M, LPB, NREG>(tmp, spec, l0, nl, px);
  x_commit_spectra<T, M, LPB, TWP, NREG>(buf, tmp, col0);
}
template <typename T, int M, int LPB, int TWP, int NREG>
__device__ __forceinline__ void x_store_spectra(const cplx<T>* buf, cplx<T>* const* spec, int col0, int l0,
                                                int nl, size_t px) {
  lanes2d<NREG * LPB, M + 1>([&](int, int r, int k) {
    const int f = r / LPB, l = r % LPB;
    if (l < nl) spec[f][(size_t)(l0 + l) * px + k] = buf[k * TWP + col0 + f * LPB + l];
  });
}

// Half spectrum X[0..M] of a length-2M real line -> Z[0..M-1] whose
// unnormalised length-M inverse DFT is (y[2n] + i y[2n+1]) with y the
// unnormalised length-2M inverse DFT of the Hermitian extension of X:
//   Z[k] = (X[k] + conj X[M-k]) + i (X[k] - conj X[M-k]) W_2M^{-k}
// Imaginary parts of X[0] and X[M] are dropped (real part of the inverse).
template <typename T, int M, int TWP, int NCOL>
__device__ __forceinline__ void c2r_pre(cplx<T>* buf, const cplx<T>* __restrict__ rtw) {
  using C = cplx<T>;
  lanes2d<NCOL, M / 2 + 1>([&](int, int col, int k) {
    if (k == 0) {
      const C x0 = buf[col], xm = buf[M * TWP + col];
      buf[col] = cmake<C>(x0.x + xm.x, x0.x - xm.x);
    } else {
      const C A = buf[k * TWP + col], B = buf[(M - k) * TWP + col];
      const C w = rtw[k];
      const C s1 = cadd(A, cconj(B)), d1 = csub(A, cconj(B));
      const C t1 = cmul(d1, cconj(w));                      // d1 W^{-k}
      buf[k * TWP + col] = cmake<C>(s1.x - t1.y, s1.y + t1.x);  // s1 + i t1
      if (k != M - k) {
        const C s2 = cadd(B, cconj(A)), d2 = csub(B, cconj(A));
        const C t2 = cmul(d2, cmake<C>(-w.x, -w.y));          // d2 W^{-(M-k)} = -d2 W^k
        buf[(M - k) * TWP + col] = cmake<C>(s2.x - t2.y, s2.y + t2.x);
      }
    }
  });
}

// Z[0..M-1] = DFT_M(x[2n] + i x[2n+1]) -> half spectrum X[0..M] of x:
//   X[k] = (Z[k] + conj Z[M-k]) / 2 - i W_2M^k (Z[k] - conj Z[M-k]) / 2
template <typename T, int M, int TWP, int NCOL>
__device__ __forceinline__ void r2c_post(cplx<T>* buf, const cplx<T>* __restrict__ rtw) {
  using C = cplx<T>;
  const T h = (T)0.5;
  lanes2d<NCOL, M / 2 + 1>([&](int, int col, int k) {
    if (k == 0) {
      const C z0 = buf[col];
      buf[col] = cmake<C>(z0.x + z0.y, (T)0);
      buf[M * TWP + col] = cmake<C>(z0.x - z0.y, (T)0);
    } else {
      const C A = buf[k * TWP + col], B = buf[(M - k) * TWP + col];
      const C w = rtw[k];
      const C s1 = cadd(A, cconj(B)), d1 = csub(A, cconj(B));
      const C t1 = cmul(w, d1);                                  // W^k d1
      buf[k * TWP + col] = cmake<C>(h * (s1.x + t1.y), h * (s1.y - t1.x));  // (s1 - i t1)/2
      if (k != M - k) {
        const C s2 = cadd(B, cconj(A)), d2 = csub(B, cconj(A));
        const C t2 = cmul(cmake<C>(-w.x, w.y), d2);             // W^{M-k} = -conj(W^k)
        buf[(M - k) * TWP + col] = cmake<C>(h * (s2.x + t2.y), h * (s2.y - t2.x));
      }
    }
  });
}

template <typename T> struct XArgs {
  const Slot<T>* slots;
  int slot0, na, slot1;   // slot ranges as in AxisArgs
  Dims d;
  Tables<T> tb;
  T dt_rho;   // dt / rho0
};

// X1: d+_a p (C2R of the three Z2/Y4 spectra), velocity update
// v_a <- L^s_a (L^s_a v_a - dt/rho0 d+_a p) (Alg. 1 momentum step), R2C of v_a.
template <typename T, int M>
__global__ void __launch_bounds__(X_NT) k_x_velocity(XArgs<T> a) {
  using C = cplx<T>;
  constexpr int LPB = x_lpb_vel<T>(M);
  constexpr int NC = 3 * LPB;
  constexpr int TWP = NC;
  __shared__ C buf[(M + 1) * TWP];
  const int l0 = blockIdx.x * LPB;
  const int nl = min(LPB, a.d.nlines - l0);
  const Slot<T> sl = a.slots[slot_of(blockIdx.y, a.slot0, a.na, a.slot1)];
  const size_t px = a.d.px;
  const int nx = a.d.nx;
  // prefetch the velocities: in flight during the C2R transforms
  C vv[Lanes<LPB, M>::NI][3];
  lanes2d<LPB, M>([&](int i, int l, int n) {
#pragma unroll
    for (int f = 0; f < 3; ++f)
      vv[i][f] = (l < nl) ? reinterpret_cast<const C*>(sl.v[f] + (size_t)(l0 + l) * nx)[n] : cmake<C>((T)0, (T)0);
  });
  x_load_spectra<T, M, LPB, TWP, 3>(buf, sl.spec, 0, l0, nl, px);
  __syncthreads();
  c2r_pre<T, M, TWP, NC>(buf, a.tb.rtw);
  __syncthreads();
  lds_fft<T, M, NC, TWP, X_NT, true>(buf, a.tb.tw_x);
  lanes2d<LPB, M>([&](int i, int l, int n) {
    if (l >= nl) return;
    const int line = l0 + l;
    const int yy = line % a.d.ny, zz = line / a.d.ny;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const C dp = buf[n * TWP + f * LPB + l];
      T lx, ly;
      if (f == 0) { lx = a.tb.pml_s[0][2 * n]; ly = a.tb.pml_s[0][2 * n + 1]; }
      else if (f == 1) { lx = ly = a.tb.pml_s[1][yy]; }
      else { lx = ly = a.tb.pml_s[2][zz]; }
      const C vn = cmake<C>(lx * (lx * vv[i][f].x - a.dt_rho * dp.x), ly * (ly * vv[i][f].y - a.dt_rho * dp.y));
      reinterpret_cast<C*>(sl.v[f] + (size_t)line * nx)[n] = vn;
      buf[n * TWP + f * LPB + l] = vn;
    }
  });
  __syncthreads();
  lds_fft<T, M, NC, TWP, X_NT, false>(buf, a.tb.tw_x);
  r2c_post<T, M, TWP, NC>(buf, a.tb.rtw);
  __syncthreads();
  x_store_spectra<T, M, LPB, TWP, 3>(buf, sl.spec, 0, l0, nl, px);
}

// Persistent X1: workgroups walk the (slot, line group) items with stride
// gridDim.x.  The next item's spectra are loaded into registers right after
// the current item's spectra reach LDS and its velocities right after the
// current velocities are consumed, so HBM traffic overlaps the transforms.
template <typename T, int M>
__global__ void __launch_bounds__(X_NT) k_x_velocity_persist(XArgs<T> a, int nitems) {
  using C = cplx<T>;
  constexpr int LPB = x_lpb_vel<T>(M);
  constexpr int NC = 3 * LPB;
  constexpr int TWP = NC;
  __shared__ C buf[(M + 1) * TWP];
  const int ngroups = (a.d.nlines + LPB - 1) / LPB;
  const size_t px = a.d.px;
  const int nx = a.d.nx;
  C pre[SpecRegs<T, M, LPB, 3>::N];
  C vv[Lanes<LPB, M>::NI][3];
  auto item_slot = [&](int it) { return a.slots[slot_of(it / ngroups, a.slot0, a.na, a.slot1)]; };
  auto prefetch_v = [&](const Slot<T>& sl, int l0, int nl) {
    lanes2d<LPB, M>([&](int i, int l, int n) {
#pragma unroll
      for (int f = 0; f < 3; ++f)
        vv[i][f] = (l < nl) ? reinterpret_cast<const C*>(sl.v[f] + (size_t)(l0 + l) * nx)[n] : cmake<C>((T)0, (T)0);
    });
  };
  int item = blockIdx.x;
  if (item < nitems) {
    const Slot<T> sl = item_slot(item);
    const int l0 = (item % ngroups) * LPB;
    const int nl = min(LPB, a.d.nlines - l0);
    prefetch_v(sl, l0, nl);
    x_prefetch_spectra<T, M, LPB, 3>(pre, sl.spec, l0, nl, px);
  }
  for (; item < nitems; item += gridDim.x) {
    const Slot<T> sl = item_slot(item);
    const int l0 = (item % ngroups) * LPB;
    const int nl = min(LPB, a.d.nlines - l0);
    const int next = item + gridDim.x;
    const bool has_next = next < nitems;
    x_commit_spectra<T, M, LPB, TWP, 3>(buf, pre, 0);
    __syncthreads();
    if (has_next) {
      const Slot<T> sn = item_slot(next);
      const int n0 = (next % ngroups) * LPB;
      x_prefetch_spectra<T, M, LPB, 3>(pre, sn.spec, n0, min(LPB, a.d.nlines - n0), px);
    }
    c2r_pre<T, M, TWP, NC>(buf, a.tb.rtw);
    __syncthreads();
    lds_fft<T, M, NC, TWP, X_NT, true>(buf, a.tb.tw_x);
    lanes2d<LPB, M>([&](int i, int l, int n) {
      if (l >= nl) return;
      const int line = l0 + l;
      const int yy = line % a.d.ny, zz = line / a.d.ny;
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        const C dp = buf[n * TWP + f * LPB + l];
        T lx, ly;
        if (f == 0) { lx = a.tb.pml_s[0][2 * n]; ly = a.tb.pml_s[0][2 * n + 1]; }
        else if (f == 1) { lx = ly = a.tb.pml_s[1][yy]; }
        else { lx = ly = a.tb.pml_s[2][zz]; }
        const C vn = cmake<C>(lx * (lx * vv[i][f].x - a.dt_rho * dp.x), ly * (ly * vv[i][f].y - a.dt_rho * dp.y));
        reinterpret_cast<C*>(sl.v[f] + (size_t)line * nx)[n] = vn;
        buf[n * TWP + f * LPB + l] = vn;
      }
    });
    if (has_next) {
      const Slot<T> sn = item_slot(next);
      const int n0 = (next % ngroups) * LPB;
      prefetch_v(sn, n0, min(LPB, a.d.nlines - n0));
    }
    __syncthreads();
    lds_fft<T, M, NC, TWP, X_NT, false>(buf, a.tb.tw_x);
    r2c_post<T, M, TWP, NC>(buf, a.tb.rtw);
    __syncthreads();
    x_store_spectra<T, M, LPB, TWP, 3>(buf, sl.spec, 0, l0, nl, px);
    __syncthreads();
  }
}

enum XMode { XM_FWD = 0, XM_PAIR = 1, XM_TRONLY = 2, XM_ADJONLY = 3 };

template <typename T> struct X2Args {
  const Slot<T>* slots;
  int B;          // problems in this launch (grid.y)
  int tr_off;     // slot index of problem b's forward/TR simulation = tr_off + b
  Dims d;
  Tables<T> tb;
  LineGeom g;
  T dt_rho0;      // dt * rho0
  T src_k;        // 2 dt / (3 dx): mass-source conversion (divided by c0 at the voxel)
  int step;       // forward iteration n, or adjoint iteration j
  const T* c;            // [B][nfield]
  const T* src_sig;      // [B][nt][n_src]
  const int8_t* w;       // [B][n_src]
  T* traces;             // [B][nt][n_rec]
  T* tape;               // [B][nt][n_bnd] or null
  const T* adj_src;      // [B][nt][n_rec]: a^j (reversed running sum of the residual)
  int tape_row;          // TR: tape row imposed in this step
  int tr_state_mode;     // TR initialisation: 0 step, 1 zero state, 2 keep densities
  T* ring;               // [B][3][n_gam]
  int ring_a, ring_b, ring_c;
  double* gacc;          // [B][n_gam]
  // When non-null the step index is read from device memory (replayed graph
  // of one time step); tape row and ring slots then follow from it.
  const int* step_dev;
};

// Per-launch step indices of an X2 launch.
struct StepIdx {
  int step, tape_row, ra, rb, rc;
};

template <typename T, int MODE>
__device__ __forceinline__ StepIdx step_indices(const X2Args<T>& a) {
  StepIdx s{a.step, a.tape_row, a.ring_a, a.ring_b, a.ring_c};
  if (a.step_dev) {
    const int j = *a.step_dev;
    s.step = j;
    if (MODE == XM_PAIR) {   // adjoint iteration j pairs with TR step k = j + 2
      s.tape_row = a.d.nt - 3 - j;
      s.ra = j % 3;
      s.rb = (j + 1) % 3;
      s.rc = (j + 2) % 3;
    }
  }
  return s;
}

// advance the device step counter of a replayed time-step graph
static __global__ void k_step_count(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] += 1;
}

enum SpKind { SP_SOURCE = 0, SP_ADJOINT = 1, SP_DIRICHLET = 2 };

// Locate the local line of sparse entry i given the CSR offsets of lines
// l0 .. l0+nl.
__device__ __forceinline__ int local_line(const int32_t* off, int l0, int nl, int i) {
  int l = 0;
  while (l + 1 < nl && i >= off[l0 + l + 1]) ++l;
  return l;
}

// Density update of one simulation slot for the workgroup's lines: C2R of
// d-_a v_a, rho_a <- L_a (L_a rho_a - dt rho0 d-_a v_a) (+ injection, or
// Dirichlet on dGamma), p = c0^2 sum_a rho_a written to column pcol of buf.
// state_mode: 0 = one density step, 1 = zero state (TR start from the tape
// only), 2 = keep the stored densities (TR start from the final forward state)
template <typename T, int M, int LPB, int TWP, int TWPP, int KIND>
__device__ __forceinline__ void density_update(const X2Args<T>& a, const StepIdx& si, const Slot<T>& sl, int b,
                                               int l0, int nl, int state_mode, int pcol, cplx<T>* buf,
                                               cplx<T>* bufp, cplx<T>* spv, uint8_t* spm) {
  const bool zero_state = state_mode == 1;
  const bool no_step = state_mode != 0;
  using C = cplx<T>;
  constexpr int NC = 3 * LPB;
  const int nx = a.d.nx;
  const size_t px = a.d.px;
  const T* cb = a.c + (size_t)b * a.d.nfield;
  // prefetch c0 and the split densities: in flight during the C2R transforms
  constexpr int EB = Lanes<LPB, M>::NI;
  C cc[EB], rr[EB][3];
  lanes2d<LPB, M>([&](int i, int l, int n) {
    const bool ok = l < nl;
    const size_t lo = (size_t)(l0 + l) * nx;
    cc[i] = ok ? reinterpret_cast<const C*>(cb + lo)[n] : cmake<C>((T)0, (T)0);
#pragma unroll
    for (int f = 0; f < 3; ++f)
      rr[i][f] = (ok && !zero_state) ? reinterpret_cast<const C*>(sl.rho[f] + lo)[n] : cmake<C>((T)0, (T)0);
  });
  if (!no_step) x_load_spectra<T, M, LPB, TWP, 3>(buf, sl.spec, 0, l0, nl, px);
  for (int e = threadIdx.x; e < M * LPB; e += X_NT) {
    spv[e] = cmake<C>((T)0, (T)0);
    if (KIND == SP_DIRICHLET) { spm[2 * e] = 0; spm[2 * e + 1] = 0; }
  }
  __syncthreads();
  // sparse inputs of this step
  if (KIND == SP_SOURCE) {
    const int i0 = a.g.src_off[l0], i1 = a.g.src_off[l0 + nl];
    for (int i = i0 + (int)threadIdx.x; i < i1; i += X_NT) {
      const int l = local_line(a.g.src_off, l0, nl, i);
      const int x = a.g.src_x[i], id = a.g.src_id[i];
      const T cv = cb[(size_t)(l0 + l) * nx + x];
      const T val = a.src_k / cv * (T)a.w[(size_t)b * a.d.n_src + id] *
                    a.src_sig[((size_t)b * a.d.nt + si.step) * a.d.n_src + id];
      T* sp = reinterpret_cast<T*>(spv);
      sp[2 * ((x >> 1) * LPB + l) + (x & 1)] = val;
    }
  } else if (KIND == SP_ADJOINT) {
    const int i0 = a.g.rec_off[l0], i1 = a.g.rec_off[l0 + nl];
    for (int i = i0 + (int)threadIdx.x; i < i1; i += X_NT) {
      const int l = local_line(a.g.rec_off, l0, nl, i);
      const int x = a.g.rec_x[i], id = a.g.rec_id[i];
      const T val = a.adj_src[((size_t)b * a.d.nt + si.step) * a.d.n_rec + id] * (T)(1.0 / 3.0);
      T* sp = reinterpret_cast<T*>(spv);
      sp[2 * ((x >> 1) * LPB + l) + (x & 1)] = val;
    }
  } else {
    const int i0 = a.g.bnd_off[l0], i1 = a.g.bnd_off[l0 + nl];
    const T* trow = a.tape + ((size_t)b * a.d.nt + si.tape_row) * a.d.n_bnd;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += X_NT) {
      const int l = local_line(a.g.bnd_off, l0, nl, i);
      const int x = a.g.bnd_x[i];
      const T cv = cb[(size_t)(l0 + l) * nx + x];
      const T val = trow[i] / ((T)3 * cv * cv);           // g / (3 c0^2)
      T* sp = reinterpret_cast<T*>(spv);
      const int q = 2 * ((x >> 1) * LPB + l) + (x & 1);
      sp[q] = val;
      spm[q] = 1;
    }
  }
  if (!no_step) {
    c2r_pre<T, M, TWP, NC>(buf, a.tb.rtw);
    __syncthreads();
    lds_fft<T, M, NC, TWP, X_NT, true>(buf, a.tb.tw_x);
  } else {
    __syncthreads();
  }
  lanes2d<LPB, M>([&](int i, int l, int n) {
    if (l >= nl) return;
    const int line = l0 + l;
    const int yy = line % a.d.ny, zz = line / a.d.ny;
    const C c2 = cc[i];
    const C sv = spv[n * LPB + l];
    C sum = cmake<C>((T)0, (T)0);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      C* rp = reinterpret_cast<C*>(sl.rho[f] + (size_t)line * nx) + n;
      C rn;
      if (zero_state) {
        rn = cmake<C>((T)0, (T)0);
      } else if (no_step) {
        rn = rr[i][f];
      } else {
        const C dv = buf[n * TWP + f * LPB + l];
        T lx, ly;
        if (f == 0) { lx = a.tb.pml_n[0][2 * n]; ly = a.tb.pml_n[0][2 * n + 1]; }
        else if (f == 1) { lx = ly = a.tb.pml_n[1][yy]; }
        else { lx = ly = a.tb.pml_n[2][zz]; }
        rn = cmake<C>(lx * (lx * rr[i][f].x - a.dt_rho0 * dv.x), ly * (ly * rr[i][f].y - a.dt_rho0 * dv.y));
      }
      if (KIND == SP_DIRICHLET) {
        if (spm[2 * (n * LPB + l)]) rn.x = sv.x;
        if (spm[2 * (n * LPB + l) + 1]) rn.y = sv.y;
      } else {
        rn = cadd(rn, sv);
      }
      *rp = rn;
      sum = cadd(sum, rn);
    }
    bufp[n * TWPP + pcol + l] = cmake<C>(c2.x * c2.x * sum.x, c2.y * c2.y * sum.y);
  });
  __syncthreads();
}

// read p at voxel x of local line l from the packed column pcol
template <typename T, int TWPP>
__device__ __forceinline__ T p_at(const cplx<T>* bufp, int pcol, int l, int x) {
  const cplx<T> z = bufp[(x >> 1) * TWPP + pcol + l];
  return (x & 1) ? z.y : z.x;
}

// X2: density / EOS pass.  MODE selects which simulations of problem b the
// workgroup advances:
//   XM_FWD     forward slot: sources, traces f^n, boundary tape g^n
//   XM_PAIR    adjoint slot (receiver injection a^j/3) and TR slot (Dirichlet
//              from the tape), gradient accumulation, TR ring update
//   XM_TRONLY  TR slot only (initial state and the TR pre-step), ring update
//   XM_ADJONLY adjoint slot and gradient with p_tr = 0 (last two iterations)
template <typename T, int M, int MODE>
__global__ void __launch_bounds__(X_NT) k_x_density(X2Args<T> a) {
  using C = cplx<T>;
  constexpr int LPB = x_lpb_den<T>(M);
  constexpr int NP = (MODE == XM_PAIR) ? 2 : 1;
  constexpr int TWP = 3 * LPB;        // d-_a v_a of the three axes
  constexpr int TWPP = NP * LPB;      // new pressure(s), packed for the R2C
  __shared__ C buf[(M + 1) * TWP];
  __shared__ C bufp[(M + 1) * TWPP];
  __shared__ C spv[M * LPB];
  __shared__ uint8_t spm[(MODE == XM_PAIR || MODE == XM_TRONLY) ? 2 * M * LPB : 1];
  const int l0 = blockIdx.x * LPB;
  const int nl = min(LPB, a.d.nlines - l0);
  const int b = blockIdx.y;
  const int nx = a.d.nx;
  const size_t px = a.d.px;
  const int PA = 0;                         // column of the adjoint / forward pressure
  const int PT = (NP == 2) ? LPB : 0;       // column of the TR pressure
  const Slot<T> s_adj = a.slots[b];
  const Slot<T> s_tr = a.slots[a.tr_off + b];
  const StepIdx si = step_indices<T, MODE>(a);

  if (MODE == XM_FWD) {
    density_update<T, M, LPB, TWP, TWPP, SP_SOURCE>(a, si, s_tr, b, l0, nl, 0, PA, buf, bufp, spv, spm);
    // sensors f^n = M p and boundary tape g^n = p(dGamma)
    const int i0 = a.g.rec_off[l0], i1 = a.g.rec_off[l0 + nl];
    for (int i = i0 + (int)threadIdx.x; i < i1; i += X_NT) {
      const int l = local_line(a.g.rec_off, l0, nl, i);
      a.traces[((size_t)b * a.d.nt + si.step) * a.d.n_rec + a.g.rec_id[i]] =
          p_at<T, TWPP>(bufp, PA, l, a.g.rec_x[i]);
    }
    if (a.tape) {
      const int j0 = a.g.bnd_off[l0], j1 = a.g.bnd_off[l0 + nl];
      T* trow = a.tape + ((size_t)b * a.d.nt + si.step) * a.d.n_bnd;
      for (int i = j0 + (int)threadIdx.x; i < j1; i += X_NT) {
        const int l = local_line(a.g.bnd_off, l0, nl, i);
        trow[i] = p_at<T, TWPP>(bufp, PA, l, a.g.bnd_x[i]);
      }
    }
  }
  if (MODE == XM_PAIR || MODE == XM_ADJONLY) {
    density_update<T, M, LPB, TWP, TWPP, SP_ADJOINT>(a, si, s_adj, b, l0, nl, 0, PA, buf, bufp, spv, spm);
  }
  if (MODE == XM_PAIR || MODE == XM_TRONLY) {
    density_update<T, M, LPB, TWP, TWPP, SP_DIRICHLET>(a, si, s_tr, b, l0, nl, a.tr_state_mode, PT, buf, bufp,
                                                       spv, spm);
  }
  if (MODE != XM_FWD) {
    // ring update and gradient: G += 2/c0^3 p_adj (p_tr^(j) - 2 p_tr^(j+1) + p_tr^(j+2))
    const int i0 = a.g.gam_off[l0], i1 = a.g.gam_off[l0 + nl];
    const T* cb = a.c + (size_t)b * a.d.nfield;
    T* ring = a.ring + (size_t)b * 3 * a.d.n_gam;
    double* gacc = a.gacc + (size_t)b * a.d.n_gam;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += X_NT) {
      const int l = local_line(a.g.gam_off, l0, nl, i);
      const int x = a.g.gam_x[i];
      // p_tr^(k) = 0 for k >= N: the ring slot is written in every mode so
      // that the next iteration never reads a stale entry
      const T ptr = (MODE == XM_ADJONLY) ? (T)0 : p_at<T, TWPP>(bufp, PT, l, x);
      if (MODE != XM_TRONLY) {
        const T padj = p_at<T, TWPP>(bufp, PA, l, x);
        const T cv = cb[(size_t)(l0 + l) * nx + x];
        const T pm = ring[(size_t)si.ra * a.d.n_gam + i];
        const T p0 = ring[(size_t)si.rb * a.d.n_gam + i];
        const T inc = (T)2 / (cv * cv * cv) * padj * (pm - (T)2 * p0 + ptr);
        gacc[i] += (double)inc;
      }
      ring[(size_t)si.rc * a.d.n_gam + i] = ptr;
    }
  }
  __syncthreads();
  // forward x-transform of the new pressure(s)
  lds_fft<T, M, TWPP, TWPP, X_NT, false>(bufp, a.tb.tw_x);
  r2c_post<T, M, TWPP, TWPP>(bufp, a.tb.rtw);
  __syncthreads();
  if (NP == 2) {
    cplx<T>* specs[2] = {s_adj.spec[0], s_tr.spec[0]};
    x_store_spectra<T, M, LPB, TWPP, 2>(bufp, specs, 0, l0, nl, px);
  } else {
    cplx<T>* specs[1] = {(MODE == XM_TRONLY || MODE == XM_FWD) ? s_tr.spec[0] : s_adj.spec[0]};
    x_store_spectra<T, M, LPB, TWPP, 1>(bufp, specs, 0, l0, nl, px);
  }
}

// ----------------------------------------------------------------------------
// small kernels
// ----------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* p, long long n, T v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
__global__ void k_scale(T* p, long long n, T v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] *= v;
}

// Residual r^n = f^n - f^delta_n (or a given residual), adjoint source
// a^j = sum_{i<=j} r^{N-1-i} and per-block FP64 partial sums of r^2.
// grid: x over receivers (256 per block), y over problems.
template <typename T>
__global__ void __launch_bounds__(256) k_residual(const T* traces, const T* obs, int obs_is_residual, T* adj,
                                                  double* partial, int nt, int n_rec) {
  __shared__ double red[256];
  const int b = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  double s2 = 0.0;
  if (r < n_rec) {
    const size_t base = (size_t)b * nt * n_rec;
    double acc = 0.0;
    for (int j = 0; j < nt; ++j) {
      const size_t src = base + (size_t)(nt - 1 - j) * n_rec + r;
      const double rv = obs_is_residual ? (double)obs[src] : (double)traces[src] - (double)obs[src];
      acc += rv;
      s2 += rv * rv;
      adj[base + (size_t)j * n_rec + r] = (T)acc;
    }
  }
  red[threadIdx.x] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)b * gridDim.x + blockIdx.x] = red[0];
}

static __global__ void k_misfit_final(const double* partial, int nblk, double* misfit, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) {
    double s = 0.0;
    for (int i = 0; i < nblk; ++i) s += partial[(size_t)b * nblk + i];
    misfit[b] = 0.5 * s;
  }
}

template <typename T>
__global__ void k_grad_scatter(const double* gacc, const int32_t* gam_lin, int n_gam, long long nfield, T* grad,
                               int B) {
  const int b = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_gam; i += gridDim.x * blockDim.x)
    grad[(size_t)b * nfield + gam_lin[i]] = (T)gacc[(size_t)b * n_gam + i];
}

// flag |= 1 if any value lies outside [lo, hi] or is not finite
template <typename T>
__global__ void k_check_range(const T* p, long long n, T lo, T hi, int* flag) {
  int bad = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const T v = p[i];
    if (!(v >= lo && v <= hi)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

}  // namespace fwi

namespace fwi {

// Plain real-to-complex / complex-to-real x passes (used by the standalone
// spectral derivative; the time step uses the fused X1 / X2 passes).
template <typename T, int M>
__global__ void __launch_bounds__(X_NT) k_x_r2c(XArgs<T> a, const T* in, int f) {
  using C = cplx<T>;
  constexpr int LPB = x_lpb<T>(M);
  constexpr int TWP = LPB;
  __shared__ C buf[(M + 1) * TWP];
  const int l0 = blockIdx.x * LPB;
  const int nl = min(LPB, a.d.nlines - l0);
  const Slot<T> sl = a.slots[a.slot0];
  lanes2d<LPB, M>([&](int, int l, int n) {
    buf[n * TWP + l] = (l < nl) ? reinterpret_cast<const C*>(in + (size_t)(l0 + l) * a.d.nx)[n]
                                : cmake<C>((T)0, (T)0);
  });
  __syncthreads();
  lds_fft<T, M, LPB, TWP, X_NT, false>(buf, a.tb.tw_x);
  r2c_post<T, M, TWP, LPB>(buf, a.tb.rtw);
  __syncthreads();
  cplx<T>* specs[1] = {sl.spec[f]};
  x_store_spectra<T, M, LPB, TWP, 1>(buf, specs, 0, l0, nl, a.d.px);
}

template <typename T, int M>
__global__ void __launch_bounds__(X_NT) k_x_c2r(XArgs<T> a, T* out, int f) {
  using C = cplx<T>;
  constexpr int LPB = x_lpb<T>(M);
  constexpr int TWP = LPB;
  __shared__ C buf[(M + 1) * TWP];
  const int l0 = blockIdx.x * LPB;
  const int nl = min(LPB, a.d.nlines - l0);
  const Slot<T> sl = a.slots[a.slot0];
  cplx<T>* specs[1] = {sl.spec[f]};
  x_load_spectra<T, M, LPB, TWP, 1>(buf, specs, 0, l0, nl, a.d.px);
  __syncthreads();
  c2r_pre<T, M, TWP, LPB>(buf, a.tb.rtw);
  __syncthreads();
  lds_fft<T, M, LPB, TWP, X_NT, true>(buf, a.tb.tw_x);
  lanes2d<LPB, M>([&](int, int l, int n) {
    if (l < nl) reinterpret_cast<C*>(out + (size_t)(l0 + l) * a.d.nx)[n] = buf[n * TWP + l];
  });
}

}  // namespace fwi
