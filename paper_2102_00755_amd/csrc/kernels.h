// HIP kernels of one k-space time step (App. B) and of the TR gradient
// (Alg. 1), written for gfx950.
//
// One time step of one simulation is eight launches, each one HBM pass:
//   Y3  forward y-FFT of p_hat                       (1 field in place)
//   Z2  forward z-FFT, x kappa (Q) and x kappa i k_z e^{+i k_z dz/2} (R),
//       inverse z-FFT; Q is stored, R advances v_z, which is kept as its
//       x-y spectrum W_z (its PML factor depends on z alone)
//   Y4q inverse y-FFT of Q; the same after x i k_y e^{+i k_y dy/2}, which
//       advances the x spectrum of v_y, then its forward y-FFT
//   X1  x i k_x e^{+i k_x dx/2}, inverse x (C2R) -> d+_x p, v_x update with
//       PML, forward x (R2C)
//   Y1  forward y-FFT of the x spectrum of v_x        (1 field)
//   Z1  forward z-FFT, x kappa * i k_a e^{-i k_a dx/2}, inverse z-FFT
//       (v_z: read from W_z, which it leaves in place)
//   Y2  inverse y-FFT of the 3 fields; d-_y v_y + d-_z v_z summed on the
//       x-lines outside the y and z PML slabs
//   X2  inverse x (C2R) -> d-_a v_a, split-density update with PML (the
//       densities kept compactly outside the slabs), source / adjoint
//       injection or Dirichlet imposition, equation of state, sensor
//       sampling, boundary tape, gradient accumulation, forward x (R2C) of p
// With absorption Z1 also forms A[d] and X2 is replaced by the lossy passes.
// The k-space operator kappa = sinc(c_ref dt |k| / 2) is evaluated on the
// fly (a Taylor series in u = (c_ref dt |k| / 2)^2) instead of being read
// from HBM, and the 1/(nx ny nz) normalisation of the three unnormalised
// inverse transforms is folded into the same multiplier.
#pragma once

#include "fft_engine.h"

namespace fwi {

// ----------------------------------------------------------------------------
// launch geometry (tuning macros: set with build.py --define)
// ----------------------------------------------------------------------------
// FWI_Y_TILE_BYTES     default row segment of a y-pass tile in bytes (64 or 128;
//                      per handle at run time: fwi_set_tuning)
// FWI_ZM_TILE_BYTES    the same for the Z1 pass (z_minus)
// FWI_ZP_TILE_BYTES    the same for the Z2 pass (z_plus: one field in, two out)
// FWI_AXIS_MAX_NT      largest axis-pass workgroup (one thread per 8 elements)
// FWI_PITCH_BYTES      the spectrum row pitch px is a multiple of this
// FWI_XVEL_LDS_BUDGET  x-lines per X1 workgroup = budget / (M sizeof(T)), odd
// FWI_XDEN_LDS_BUDGET  the same for X2 (and the lossy density pass)
// FWI_XDEN_PAIR_LDS_BUDGET  the same for the paired (adjoint + TR) X2: one line
//                      at M = 224 FP32 (0.79 ms per launch against 0.83 with
//                      three; the forward X2 is faster with three, 0.35 vs 0.42)
// FWI_XEOS_LDS_BUDGET  the same for the lossy equation-of-state pass (3, 5, 7
//                      lines at M = 224 FP32: 192, 221, 210 us per launch)
// Measured on the 448x448x224 FP32 gradient (same box, alternating runs),
// with the nine-pass step: 128-byte y tiles with 64-byte z tiles (XCD-paired,
// see tile_linear) gave 25 140 Mcell-steps/s against 24 995 with 128-byte z
// tiles and 24 600 with 64-byte y tiles (Z1 now runs 128-byte tiles, see the
// plans below); the pitch stays 128 bytes (a 64-byte pitch makes half of
// the 128-byte rows straddle two cache lines, a 256-byte pitch slows the y and
// z passes), and 256-byte z tiles are slower (fewer workgroups per CU).
#ifndef FWI_Y_TILE_BYTES
#define FWI_Y_TILE_BYTES 128
#endif
#ifndef FWI_ZM_TILE_BYTES
#define FWI_ZM_TILE_BYTES 128
#endif
#ifndef FWI_ZP_TILE_BYTES
#define FWI_ZP_TILE_BYTES 64
#endif
#ifndef FWI_AXIS_MAX_NT
#define FWI_AXIS_MAX_NT 512
#endif
#ifndef FWI_XVEL_LDS_BUDGET
#define FWI_XVEL_LDS_BUDGET 5120
#endif
#ifndef FWI_XDEN_LDS_BUDGET
#define FWI_XDEN_LDS_BUDGET 3072
#endif
#ifndef FWI_XDEN_PAIR_LDS_BUDGET
#define FWI_XDEN_PAIR_LDS_BUDGET 896
#endif
#ifndef FWI_XEOS_LDS_BUDGET
#define FWI_XEOS_LDS_BUDGET 3072
#endif
// FWI_Y_PLAN, FWI_ZM_PLAN, FWI_ZP_PLAN, FWI_X_PLAN
//                      default radix plans (make_plan: 0 or 1) of the y passes,
//                      Z1, Z2 and the velocity / density x passes.  At
//                      448x448x224 FP32 (same box, alternating runs) plan 1 of
//                      Z2 (224 = 7*4*8) gives 25 410 Mcell-steps/s against
//                      25 190 with plan 0: Z2 itself is 3 % slower, but its
//                      stores leave the caches in a state the following inverse
//                      y passes and X1 read 2-3 % faster; the other kinds'
//                      plans change the total by less than 0.1 %.  Since v_z
//                      moved into Z2 (bricked) and Y2 pairs its fields, the
//                      autotuner picks 128-byte Z1 tiles and Z2 plan 0 (Z1
//                      0.452 -> 0.424 ms, Y2 0.338 -> 0.325 ms, step -2.6 %;
//                      Z2's plan no longer matters), the defaults now.
#ifndef FWI_Y_PLAN
#define FWI_Y_PLAN 0
#endif
#ifndef FWI_ZM_PLAN
#define FWI_ZM_PLAN 0
#endif
#ifndef FWI_ZP_PLAN
#define FWI_ZP_PLAN 0
#endif
#ifndef FWI_X_PLAN
#define FWI_X_PLAN 0
#endif
enum AxisKind { AK_Y = 0, AK_ZMINUS = 1, AK_ZPLUS = 2 };
// axis-pass tile width in complex elements for a row segment of TB bytes
template <typename T, int TB> constexpr int tile_tw() { return TB / (int)(2 * sizeof(T)); }
// The spectrum row pitch px is a multiple of FWI_PITCH_BYTES; a tile at the
// end of a row may extend past px and then holds only its first columns in
// memory.
#ifndef FWI_PITCH_BYTES
#define FWI_PITCH_BYTES 128
#endif
template <typename T> constexpr int pitch_tw() { return FWI_PITCH_BYTES / (int)(2 * sizeof(T)); }
constexpr int axis_nt(int L, int TW) {
  int n = L * TW / 8;
  n = n < 64 ? 64 : (n > FWI_AXIS_MAX_NT ? FWI_AXIS_MAX_NT : n);
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
template <typename T> constexpr int x_lpb_vel(int M) { return odd_lpb<T>(FWI_XVEL_LDS_BUDGET, M); }
template <typename T> constexpr int x_lpb_den(int M) { return odd_lpb<T>(FWI_XDEN_LDS_BUDGET, M); }
// lines per X2 workgroup of mode m (XMode: 1 = the paired adjoint + TR pass)
template <typename T> constexpr int x_lpb_den_mode(int M, int m) {
  return m == 1 ? odd_lpb<T>(FWI_XDEN_PAIR_LDS_BUDGET, M) : x_lpb_den<T>(M);
}
template <typename T> constexpr int x_lpb_eos(int M) { return odd_lpb<T>(FWI_XEOS_LDS_BUDGET, M); }
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
  T vcoef;     // nx dt / rho0: velocity update of the x-spectrum states
  T half_e0;   // absorption pass: |k|^{2 half_e0} on field 0 (B[s]: (y - 1) / 2)
  T half_e1;   //                  |k|^{2 half_e1} on field 1 (A[d]: (y - 2) / 2)
  int vz_state;  // time step: Z2 advances W_z (slot v[2]) with R instead of
                 // storing R, and Z1 reads field 2 from W_z
  int pml[3];    // PML cells at both ends of x, y, z (Y2: storage of d-_y v_y, d-_z v_z)
  // absorption: the spectrum A[d] per slot (slot s at ad + s ad_stride),
  // written by the Z1 of the lossy step, inverse-y transformed by Y2; null
  // without absorption.  ad_coef = rho0.
  cplx<T>* ad;
  long long ad_stride;
  T ad_coef;
};

__device__ __forceinline__ int slot_of(int i, int slot0, int na, int slot1) {
  return i < na ? slot0 + i : slot1 + (i - na);
}

// Tiles are moved whole within the row pitch: the padding columns of the last
// tile (kx > M) are in bounds, transformed with the valid columns (columns
// never mix) and never read by the x passes.  ncol = min(TW, px - kx0) is the
// number of tile columns that exist in memory (less than TW only for a
// 128-byte tile at the end of a row).  Loads are unpredicated, from clamped
// columns, so that a thread's loads are all in flight before the first wait;
// stores are predicated on c < ncol and otherwise write full row segments.
template <typename T, int L, int TW, int NT>
__device__ __forceinline__ void tile_prefetch(cplx<T>* tmp, const cplx<T>* g, size_t rstride, int ncol) {
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = min((int)threadIdx.x + i * NT, E - 1);
    tmp[i] = gld(g + (size_t)(e / TW) * rstride + min(e % TW, ncol - 1));
  }
}
template <typename T, int L, int TW, int NT>
__device__ __forceinline__ void tile_commit(cplx<T>* buf, const cplx<T>* tmp) {
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
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
    if ((E % NT == 0 || e < E) && e % TW < ncol) gst(g + (size_t)(e / TW) * rstride + e % TW, buf[e]);
  }
}

// Twiddle table W_N^m, m < N, staged in LDS by each workgroup: the stages of
// a transform then read their twiddles with the butterfly operands instead
// of waiting for an L2 round trip per stage.  Issued with the tile loads.
template <int N, int NT> struct TwRegs {
  static constexpr int N_PER = (N + NT - 1) / NT;
};
template <typename T, int N, int NT>
__device__ __forceinline__ void tw_prefetch(cplx<T>* tt, const cplx<T>* tw) {
#pragma unroll
  for (int i = 0; i < TwRegs<N, NT>::N_PER; ++i) tt[i] = gld(tw + min((int)threadIdx.x + i * NT, N - 1));
}
template <typename T, int N, int NT>
__device__ __forceinline__ void tw_commit(cplx<T>* twl, const cplx<T>* tt) {
#pragma unroll
  for (int i = 0; i < TwRegs<N, NT>::N_PER; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if (N % NT == 0 || e < N) twl[e] = tt[i];
  }
}

// Tile and twiddles into LDS (loads of both in flight together).
template <typename T, int L, int TW, int NT>
__device__ __forceinline__ void tile_load(cplx<T>* buf, const cplx<T>* g, size_t rstride, int ncol, cplx<T>* twl,
                                          const cplx<T>* tw) {
  cplx<T> tmp[(L * TW + NT - 1) / NT], tt[TwRegs<L, NT>::N_PER];
  tile_prefetch<T, L, TW, NT>(tmp, g, rstride, ncol);
  tw_prefetch<T, L, NT>(tt, tw);
  tile_commit<T, L, TW, NT>(buf, tmp);
  tw_commit<T, L, NT>(twl, tt);
}

// Linear tile index of an axis-pass workgroup.  With 64-byte row segments two
// neighbouring tiles share every 128-byte line.  Workgroups are dispatched
// round-robin over the eight XCDs, each with its own L2, so within every group
// of 16 workgroups the mapping gives both halves of a line to workgroups b and
// b + 8, which run on the same XCD at the same time: their half-line writes
// merge in that L2 instead of reaching HBM as read-modify-writes.  Measured at
// 448x448x224 FP32 with 64-byte z tiles: Z2 2.9 -> 3.6 TB/s.  128-byte tiles
// keep the identity.
template <int TBYTES> __device__ __forceinline__ int tile_linear() {
  const int b = blockIdx.x;
  if (TBYTES >= 128) return b;
  const int g16 = gridDim.x & ~15;
  return b < g16 ? (b & ~15) + 2 * (b & 7) + ((b >> 3) & 1) : b;
}

// Y pass: in-place FFT along y of nf fields per slot.  L == ny.
template <typename T, int L, bool INV, int TB, int PL = 0>
__global__ void __launch_bounds__(axis_nt(L, tile_tw<T, TB>()))
k_axis_y(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = tile_tw<T, TB>();
  constexpr int NT = axis_nt(L, TW);
  __shared__ C buf[L * TW];
  __shared__ C twl[L];
  const int ntx = (a.d.px + TW - 1) / TW;   // tiles per spectrum row
  const int tl = tile_linear<TB>();
  const int tile = tl % ntx;
  const int z = tl / ntx;
  const int s = slot_of(blockIdx.y / a.nf, a.slot0, a.na, a.slot1);
  const int f = a.f0 + blockIdx.y % a.nf;
  const size_t px = a.d.px;
  C* g = a.slots[s].spec[f] + (size_t)z * L * px + (size_t)tile * TW;
  const int ncol = min(TW, (int)px - tile * TW);
  tile_load<T, L, TW, NT>(buf, g, px, ncol, twl, a.tb.tw_y);
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, INV, PL>(buf, twl);
  tile_store<T, L, TW, NT>(buf, g, px, ncol);
}

// Waves per SIMD the velocity y pass is compiled for: 4 (two workgroups of
// 8 waves per CU) in FP32 where a thread holds at most 14 tile elements, else
// the compiler's choice (FP64 would spill)
template <typename T, int L, int TB> constexpr int yv_waves() {
  return sizeof(T) == 4 &&
                 (L * tile_tw<T, TB>() + axis_nt(L, tile_tw<T, TB>()) - 1) / axis_nt(L, tile_tw<T, TB>()) <= 14
             ? 4
             : 1;
}

// Inverse y pass of the time step (Y2), one launch per step (grid.y = slots).
// The first ntx nz workgroups transform field 0 (d-_x v_x) in place in TW-wide
// tiles (with absorption the next ntx nz the slot's A[d] spectrum).  The others transform fields 1 and 2 (d-_y v_y, d-_z v_z) side by
// side: an LDS tile of TW columns holds the same TW/2 spectrum columns of both
// fields.  On the x-lines outside the y and z PML slabs the density pass only
// needs their sum (the split densities are stored compactly there, see
// X2Args), so field 1 receives d-_y v_y + d-_z v_z, read from the two halves of
// the tile, and field 2 is not written; lines in a slab receive both.  The
// half-width tiles are XCD-paired like 64-byte z tiles.  L == ny.
__device__ __forceinline__ bool in_pml_slab(int i, int n, int P) { return i < P || i > n - 1 - P; }
template <typename T, int L, int TB, int PL = 0>
__global__ void __launch_bounds__(axis_nt(L, tile_tw<T, TB>()))
k_axis_y_div(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = tile_tw<T, TB>();
  constexpr int H = TW / 2;                 // columns of each field in a paired tile
  static_assert(TW % 2 == 0, "paired y tile: TW must be even");
  constexpr int NT = axis_nt(L, TW);
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
  constexpr int TPT = TwRegs<L, NT>::N_PER;
  __shared__ C buf[L * TW];
  __shared__ C twl[L];
  const Slot<T>& sl = a.slots[slot_of(blockIdx.y, a.slot0, a.na, a.slot1)];
  const size_t px = a.d.px;
  const int ntx = ((int)px + TW - 1) / TW;
  const int n0 = ntx * a.d.nz;              // field-0 workgroups
  const int b = blockIdx.x;
  const int nad = a.ad ? n0 : 0;            // A[d] workgroups (absorption)
  if (b < n0 + nad) {
    const int bb = b < n0 ? b : b - n0;
    const int tile = bb % ntx, z = bb / ntx;
    C* const base = b < n0 ? sl.spec[0] : a.ad + (size_t)slot_of(blockIdx.y, a.slot0, a.na, a.slot1) * a.ad_stride;
    C* g = base + (size_t)z * L * px + (size_t)tile * TW;
    const int ncol = min(TW, (int)px - tile * TW);
    tile_load<T, L, TW, NT>(buf, g, px, ncol, twl, a.tb.tw_y);
    __syncthreads();
    lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
    tile_store<T, L, TW, NT>(buf, g, px, ncol);
    return;
  }
  const int nh = ((int)px + H - 1) / H;     // paired tiles per spectrum row
  const int n1 = nh * a.d.nz;
  int t1 = b - n0 - nad;
  t1 = t1 < (n1 & ~15) ? (t1 & ~15) + 2 * (t1 & 7) + ((t1 >> 3) & 1) : t1;
  const int tile = t1 % nh, z = t1 / nh;
  const size_t off = (size_t)z * L * px + (size_t)tile * H;
  const int ncol = min(H, (int)px - tile * H);
  C* const g1 = sl.spec[1] + off;
  C* const g2 = sl.spec[2] + off;
  {
    C tmp[EPT], tt[TPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = min((int)threadIdx.x + i * NT, E - 1);
      const int c = e % TW;
      tmp[i] = gld((c < H ? g1 : g2) + (size_t)(e / TW) * px + min(c % H, ncol - 1));
    }
    tw_prefetch<T, L, NT>(tt, a.tb.tw_y);
    tile_commit<T, L, TW, NT>(buf, tmp);
    tw_commit<T, L, NT>(twl, tt);
  }
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
  const bool zslab = in_pml_slab(z, a.d.nz, a.pml[2]);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    const int c = e % TW, cc = c % H;
    if ((E % NT == 0 || e < E) && cc < ncol) {
      const int y = e / TW;
      const bool full = zslab || in_pml_slab(y, L, a.pml[1]);
      if (c < H) gst(g1 + (size_t)y * px + cc, full ? buf[e] : cadd(buf[e], buf[e + H]));
      else if (full) gst(g2 + (size_t)y * px + cc, buf[e]);
    }
  }
}

// Plain z pass: in-place FFT along z of nf fields per slot (grid transfers of
// the coarse-to-fine scheme).  L == nz.
template <typename T, int L, bool INV, int TB, int PL = 0>
__global__ void __launch_bounds__(axis_nt(L, tile_tw<T, TB>()))
k_axis_z(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = tile_tw<T, TB>();
  constexpr int NT = axis_nt(L, TW);
  __shared__ C buf[L * TW];
  __shared__ C twl[L];
  const int ntx = (a.d.px + TW - 1) / TW;   // tiles per spectrum row
  const int tl = tile_linear<TB>();
  const int tile = tl % ntx;
  const int y = tl / ntx;
  const int s = slot_of(blockIdx.y / a.nf, a.slot0, a.na, a.slot1);
  const int f = a.f0 + blockIdx.y % a.nf;
  const size_t px = a.d.px;
  const size_t rstride = (size_t)a.d.ny * px;
  C* g = a.slots[s].spec[f] + (size_t)y * px + (size_t)tile * TW;
  const int ncol = min(TW, (int)px - tile * TW);
  tile_load<T, L, TW, NT>(buf, g, rstride, ncol, twl, a.tb.tw_z);
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, INV, PL>(buf, twl);
  tile_store<T, L, TW, NT>(buf, g, rstride, ncol);
}

// k-space multipliers of the elements a thread owns in a z tile: thread t
// owns rows r_i = t / TW + i NT / TW of column c = t % TW (NT is a multiple
// of TW), so kx is fixed per thread.  The tables are read before the tile's
// data arrives (their latency overlaps the tile load).
template <typename T, int L, int TW, int NT>
__device__ __forceinline__ void z_kappa(const AxisArgs<T>& a, int kx, int y, T* kap) {
  static_assert(NT % TW == 0, "z tile: NT must be a multiple of TW");
  constexpr int EPT = (L * TW + NT - 1) / NT;
  const T base = a.tb.ksq[0][kx] + a.tb.ksq[1][y];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int r = (int)threadIdx.x / TW + i * (NT / TW);
    if ((L * TW) % NT == 0 || r < L) kap[i] = sinc_u(a.kap_a * (base + a.tb.ksq[2][r])) * a.scale;
  }
}
// kappa * scale * s_f with the shift factor s_f = i k_f exp(+-i k_f dx / 2)
// of field f (sfac = sfac_p or sfac_m)
template <typename T, int L, int TW, int NT>
__device__ __forceinline__ void z_mult(const AxisArgs<T>& a, const cplx<T>* const* sfac, int f, int kx, int y,
                                       const T* kap, cplx<T>* m) {
  constexpr int EPT = (L * TW + NT - 1) / NT;
  if (f == 2) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int r = (int)threadIdx.x / TW + i * (NT / TW);
      if ((L * TW) % NT == 0 || r < L) m[i] = cscale(sfac[2][r], kap[i]);
    }
  } else {
    const cplx<T> sf = (f == 0) ? sfac[0][kx] : sfac[1][y];
#pragma unroll
    for (int i = 0; i < EPT; ++i) m[i] = cscale(sf, kap[i]);
  }
}
template <typename T, int L, int TW, int NT>
__device__ __forceinline__ void z_apply(cplx<T>* buf, const cplx<T>* m, const cplx<T>* x) {
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if (E % NT == 0 || e < E) buf[e] = cmul(m[i], x ? x[i] : buf[e]);
  }
}

// Storage of W_z (the x-y spectrum of v_z, slot v[2]), which only the z
// passes touch: z-contiguous bricks of WB = 64 bytes of columns,
// [y][px / WB][nz][WB], so that a z tile reads and writes it as contiguous
// 64-byte rows of one block (the spectra are [z][y][px], where a z tile's rows
// lie ny px apart).  px is a multiple of WB and a z tile spans whole bricks.
template <typename T> constexpr int wz_bw() { return 64 / (int)sizeof(cplx<T>); }
// the first element of the tile of columns [k0, k0 + TW) at spectrum row y
template <typename T>
__device__ __forceinline__ size_t wz_tile(const Dims& d, int y, int k0) {
  constexpr int WB = wz_bw<T>();
  return ((size_t)y * (d.px / WB) + k0 / WB) * (size_t)d.nz * WB;
}
// offset of element (row r = z, column c) within the tile
template <typename T, int L>
__device__ __forceinline__ int wz_el(int r, int c) {
  constexpr int WB = wz_bw<T>();
  return (c / WB) * L * WB + r * WB + c % WB;
}

// Z pass of the velocity divergence terms: field f -> F_z^-1 m-_f F_z field f
// (eq. DisPartDevSt with the minus shift).  L == nz.
template <typename T, int L, int TB, int PL = 0>
__global__ void __launch_bounds__(axis_nt(L, tile_tw<T, TB>()))
k_axis_z_minus(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = tile_tw<T, TB>();
  constexpr int NT = axis_nt(L, TW);
  constexpr int EPT = (L * TW + NT - 1) / NT;
  __shared__ C buf[L * TW];
  __shared__ C twl[L];
  const int ntx = (a.d.px + TW - 1) / TW;   // tiles per spectrum row
  const int tl = tile_linear<TB>();
  const int tile = tl % ntx;
  const int y = tl / ntx;
  const int s = slot_of(blockIdx.y / a.nf, a.slot0, a.na, a.slot1);
  const int f = a.f0 + blockIdx.y % a.nf;
  const size_t px = a.d.px;
  const size_t rstride = (size_t)a.d.ny * px;
  const size_t off = (size_t)y * px + (size_t)tile * TW;
  C* g = a.slots[s].spec[f] + off;
  const bool wz_in = a.vz_state && f == 2;   // v_z from its z-contiguous state
  const int ncol = min(TW, (int)px - tile * TW);
  const int kx = min(tile * TW + (int)threadIdx.x % TW, a.d.M);
  T kap[EPT];
  C m[EPT];
  z_kappa<T, L, TW, NT>(a, kx, y, kap);
  z_mult<T, L, TW, NT>(a, a.tb.sfac_m, f, kx, y, kap, m);
  if (wz_in) {
    const C* gw = reinterpret_cast<const C*>(a.slots[s].v[2]) + wz_tile<T>(a.d, y, tile * TW);
    C tmp[EPT], tt[TwRegs<L, NT>::N_PER];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = min((int)threadIdx.x + i * NT, L * TW - 1);
      tmp[i] = gld(gw + wz_el<T, L>(e / TW, min(e % TW, ncol - 1)));
    }
    tw_prefetch<T, L, NT>(tt, a.tb.tw_z);
    tile_commit<T, L, TW, NT>(buf, tmp);
    tw_commit<T, L, NT>(twl, tt);
  } else {
    tile_load<T, L, TW, NT>(buf, g, rstride, ncol, twl, a.tb.tw_z);
  }
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, false, PL>(buf, twl);
  z_apply<T, L, TW, NT>(buf, m, nullptr);
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
  tile_store<T, L, TW, NT>(buf, g, rstride, ncol);
}

// x^e for normal x > 0 in the kernel's precision.  FP32: 2^(e log2 x) with
// the hardware base-2 logarithm and exponential (about 1 ulp each, a relative
// error near 1e-6 here, against ~100 instructions of powf, which made the
// absorption passes ALU-bound); FP64: pow.
__device__ __forceinline__ float real_pow(float x, float e) {
  return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(x));
}
__device__ __forceinline__ double real_pow(double x, double e) { return pow(x, e); }

// Z1 of the lossy step: one workgroup per tile runs the three fields of
// k_axis_z_minus one after the other and also forms the absorption term
// A[d] = F^-1 |k|^{y-2} F d of d = rho0 sum_a d-_a v_a (Sec. 2.1) from the same
// z spectra: the products m_a F v_a of the three fields are summed in
// registers, multiplied by rho0 |k|^{y-2} (0 at k = 0; the 1/(nx ny nz) of
// the unnormalised transforms is already in m_a) and inverse z transformed
// into the slot's A[d] spectrum, which the inverse y pass then finishes.
// L == nz.
template <typename T, int L, int TB, int PL = 0>
__global__ void __launch_bounds__(axis_nt(L, tile_tw<T, TB>()))
k_axis_z_minus_ad(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = tile_tw<T, TB>();
  constexpr int NT = axis_nt(L, TW);
  constexpr int EPT = (L * TW + NT - 1) / NT;
  __shared__ C buf[L * TW];
  __shared__ C twl[L];
  const int ntx = (a.d.px + TW - 1) / TW;   // tiles per spectrum row
  const int tl = tile_linear<TB>();
  const int tile = tl % ntx;
  const int y = tl / ntx;
  const int s = slot_of(blockIdx.y, a.slot0, a.na, a.slot1);
  const size_t px = a.d.px;
  const size_t rstride = (size_t)a.d.ny * px;
  const size_t off = (size_t)y * px + (size_t)tile * TW;
  const int ncol = min(TW, (int)px - tile * TW);
  const int kx = min(tile * TW + (int)threadIdx.x % TW, a.d.M);
  T kap[EPT];
  C acc[EPT];
  z_kappa<T, L, TW, NT>(a, kx, y, kap);
#pragma unroll
  for (int i = 0; i < EPT; ++i) acc[i] = cmake<C>((T)0, (T)0);
  for (int f = 0; f < 3; ++f) {
    C* g = a.slots[s].spec[f] + off;
    C m[EPT];
    z_mult<T, L, TW, NT>(a, a.tb.sfac_m, f, kx, y, kap, m);
    if (f == 0) {
      tile_load<T, L, TW, NT>(buf, g, rstride, ncol, twl, a.tb.tw_z);
    } else {
      C tmp[EPT];
      if (f == 2 && a.vz_state) {
        const C* gw = reinterpret_cast<const C*>(a.slots[s].v[2]) + wz_tile<T>(a.d, y, tile * TW);
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
          const int e = min((int)threadIdx.x + i * NT, L * TW - 1);
          tmp[i] = gld(gw + wz_el<T, L>(e / TW, min(e % TW, ncol - 1)));
        }
      } else {
        tile_prefetch<T, L, TW, NT>(tmp, g, rstride, ncol);
      }
      __syncthreads();   // the previous field's stores have read buf
      tile_commit<T, L, TW, NT>(buf, tmp);
    }
    __syncthreads();
    lds_fft<T, L, TW, TW, NT, false, PL>(buf, twl);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = (int)threadIdx.x + i * NT;
      if ((L * TW) % NT == 0 || e < L * TW) {
        const C v = cmul(m[i], buf[e]);
        buf[e] = v;
        acc[i] = cadd(acc[i], v);
      }
    }
    __syncthreads();
    lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
    tile_store<T, L, TW, NT>(buf, g, rstride, ncol);
  }
  // A[d]: rho0 |k|^{y-2} times the summed spectra
  const T base = a.tb.ksq[0][kx] + a.tb.ksq[1][y];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    const int r = (int)threadIdx.x / TW + i * (NT / TW);
    if ((L * TW) % NT == 0 || e < L * TW) {
      const T q = base + a.tb.ksq[2][r];
      const T mA = q > (T)0 ? real_pow(q, a.half_e1) * a.ad_coef : (T)0;
      buf[e] = cscale(acc[i], mA);
    }
  }
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
  tile_store<T, L, TW, NT>(buf, a.ad + (size_t)s * a.ad_stride + off, rstride, ncol);
}

// Z pass of the pressure gradient, field 0 (p_hat) -> two fields:
//   field 0: Q = F_z^-1 kappa F_z p_hat                (for d+_x and d+_y)
//   field 2: R = F_z^-1 kappa i k_z e^{+i k_z dz/2} F_z p_hat   (d+_z)
// The shift factors i k_a e^{+i k_a da/2} of x and y are separable and are
// applied later, in the y pass (y) and the x pass (x), where those wave
// numbers are at hand: one spectrum less is written here and read there.
// In the time step (vz_state) R is not stored: it advances v_z at once.
// v_z is kept as W_z = F_y F_x v_z (z in real space); its PML factor
// Lambda^s_z(z) is constant in x and y, so the momentum step
// v_z <- L_z (L_z v_z - dt/rho0 d+_z p) commutes with F_y F_x, and with
// F_y F_x d+_z p = nx ny R (R being the y-x spectrum of d+_z p / (nx ny),
// since the normalisation is folded into kappa) it reads
//   W_z <- L_z (L_z W_z - ny vcoef R),  vcoef = nx dt / rho0.
// L == nz.
template <typename T, int L, int TB, int PL = 0>
__global__ void __launch_bounds__(axis_nt(L, tile_tw<T, TB>()))
k_axis_z_plus(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = tile_tw<T, TB>();
  constexpr int NT = axis_nt(L, TW);
  constexpr int EPT = (L * TW + NT - 1) / NT;
  __shared__ C buf[L * TW];
  __shared__ C twl[L];
  const int ntx = (a.d.px + TW - 1) / TW;   // tiles per spectrum row
  const int tl = tile_linear<TB>();
  const int tile = tl % ntx;
  const int y = tl / ntx;
  const int s = slot_of(blockIdx.y, a.slot0, a.na, a.slot1);
  const size_t px = a.d.px;
  const size_t rstride = (size_t)a.d.ny * px;
  const size_t off = (size_t)y * px + (size_t)tile * TW;
  const int ncol = min(TW, (int)px - tile * TW);
  const int kx = min(tile * TW + (int)threadIdx.x % TW, a.d.M);
  C* const s0 = a.slots[s].spec[0];
  C* const s2 = a.slots[s].spec[2];
  T kap[EPT];
  C m[EPT];
  z_kappa<T, L, TW, NT>(a, kx, y, kap);
  z_mult<T, L, TW, NT>(a, a.tb.sfac_p, 2, kx, y, kap, m);
  tile_load<T, L, TW, NT>(buf, s0 + off, rstride, ncol, twl, a.tb.tw_z);
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, false, PL>(buf, twl);
  C xr[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if ((L * TW) % NT == 0 || e < L * TW) xr[i] = buf[e];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if ((L * TW) % NT == 0 || e < L * TW) buf[e] = cscale(xr[i], kap[i]);
  }
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
  tile_store<T, L, TW, NT>(buf, s0 + off, rstride, ncol);
  __syncthreads();
  z_apply<T, L, TW, NT>(buf, m, xr);
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
  if (!a.vz_state) {
    tile_store<T, L, TW, NT>(buf, s2 + off, rstride, ncol);
    return;
  }
  C* const gw = reinterpret_cast<C*>(a.slots[s].v[2]) + wz_tile<T>(a.d, y, tile * TW);
  C w[EPT];
  T lz[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = min((int)threadIdx.x + i * NT, L * TW - 1);
    w[i] = gld(gw + wz_el<T, L>(e / TW, min(e % TW, ncol - 1)));
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) lz[i] = gld(a.tb.pml_s[2] + min(((int)threadIdx.x + i * NT) / TW, L - 1));
  const T cf = a.vcoef * (T)a.d.ny;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if (((L * TW) % NT == 0 || e < L * TW) && e % TW < ncol) {
      const C r = buf[e];
      const C wn = cmake<C>(lz[i] * (lz[i] * w[i].x - cf * r.x), lz[i] * (lz[i] * w[i].y - cf * r.y));
      gst(gw + wz_el<T, L>(e / TW, e % TW), wn);
    }
  }
}

// Z pass of the absorption operators (Sec. 2.1, the fractional Laplacians of
// L): field f -> F_z^-1 m_f F_z field f with the radial multiplier
// m_f = |k|^{2 e_f} / (nx ny nz), |k|^2 = kx^2 + ky^2 + kz^2, and m_f = 0 at
// k = 0: e_0 = (y - 1) / 2 for s (field 0), e_1 = (y - 2) / 2 for d (field 1).
// L == nz.
template <typename T, int L, int TB, int PL = 0>
__global__ void __launch_bounds__(axis_nt(L, tile_tw<T, TB>()))
k_axis_z_frac(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = tile_tw<T, TB>();
  constexpr int NT = axis_nt(L, TW);
  constexpr int EPT = (L * TW + NT - 1) / NT;
  static_assert(NT % TW == 0, "z tile: NT must be a multiple of TW");
  __shared__ C buf[L * TW];
  __shared__ C twl[L];
  const int ntx = (a.d.px + TW - 1) / TW;   // tiles per spectrum row
  const int tl = tile_linear<TB>();
  const int tile = tl % ntx;
  const int y = tl / ntx;
  const int s = slot_of(blockIdx.y / a.nf, a.slot0, a.na, a.slot1);
  const int f = a.f0 + blockIdx.y % a.nf;
  const size_t px = a.d.px;
  const size_t rstride = (size_t)a.d.ny * px;
  C* g = a.slots[s].spec[f] + (size_t)y * px + (size_t)tile * TW;
  const int ncol = min(TW, (int)px - tile * TW);
  const int kx = min(tile * TW + (int)threadIdx.x % TW, a.d.M);
  const T he = (f == 0) ? a.half_e0 : a.half_e1;
  // tile and twiddle loads in flight while the multipliers are computed
  C tmp[EPT], tt[TwRegs<L, NT>::N_PER];
  tile_prefetch<T, L, TW, NT>(tmp, g, rstride, ncol);
  tw_prefetch<T, L, NT>(tt, a.tb.tw_z);
  const T base = a.tb.ksq[0][kx] + a.tb.ksq[1][y];
  T m[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int r = (int)threadIdx.x / TW + i * (NT / TW);
    if ((L * TW) % NT == 0 || r < L) {
      const T q = base + a.tb.ksq[2][r];
      m[i] = q > (T)0 ? real_pow(q, he) * a.scale : (T)0;
    }
  }
  tile_commit<T, L, TW, NT>(buf, tmp);
  tw_commit<T, L, NT>(twl, tt);
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, false, PL>(buf, twl);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if ((L * TW) % NT == 0 || e < L * TW) buf[e] = cscale(buf[e], m[i]);
  }
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
  tile_store<T, L, TW, NT>(buf, g, rstride, ncol);
}

// Inverse y pass after Z2: per slot, part 0 reads Q (field 0) and writes
// F_y^-1 Q to field 0 and F_y^-1 (i k_y e^{+i k_y dy/2} Q) to field 1; part 1
// transforms R (field 2) in place.  grid.y = 2 x slots.  L == ny.
template <typename T, int L, int TB, int PL = 0>
__global__ void __launch_bounds__(axis_nt(L, tile_tw<T, TB>()))
k_axis_y_split(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = tile_tw<T, TB>();
  constexpr int NT = axis_nt(L, TW);
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
  __shared__ C buf[L * TW];
  __shared__ C twl[L];
  __shared__ C sfl[L];
  const int ntx = (a.d.px + TW - 1) / TW;   // tiles per spectrum row
  const int tl = tile_linear<TB>();
  const int tile = tl % ntx;
  const int z = tl / ntx;
  const int part = blockIdx.y & 1;
  const int s = slot_of(blockIdx.y >> 1, a.slot0, a.na, a.slot1);
  const size_t px = a.d.px;
  const size_t off = (size_t)z * L * px + (size_t)tile * TW;
  const int ncol = min(TW, (int)px - tile * TW);
  C* const g = a.slots[s].spec[part == 0 ? 0 : 2] + off;
  C tmp[EPT], tt[TwRegs<L, NT>::N_PER], ts[TwRegs<L, NT>::N_PER];
  tile_prefetch<T, L, TW, NT>(tmp, g, px, ncol);
  tw_prefetch<T, L, NT>(tt, a.tb.tw_y);
  if (part == 0) tw_prefetch<T, L, NT>(ts, a.tb.sfac_p[1]);
  tile_commit<T, L, TW, NT>(buf, tmp);
  tw_commit<T, L, NT>(twl, tt);
  if (part == 0) tw_commit<T, L, NT>(sfl, ts);
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
  tile_store<T, L, TW, NT>(buf, g, px, ncol);
  if (part == 0) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = (int)threadIdx.x + i * NT;
      if (E % NT == 0 || e < E) buf[e] = cmul(sfl[e / TW], tmp[i]);
    }
    __syncthreads();
    lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
    tile_store<T, L, TW, NT>(buf, a.slots[s].spec[1] + off, px, ncol);
  }
}

// Inverse y pass of the time step, fused with the velocity update of v_y and
// its forward y transform.  v_y is kept as its x spectrum V_y = F_x v_y
// (unnormalised R2C, rows of px complex): its PML factor Lambda^s_y depends
// on y only, i.e. it is a constant along every x-line, so
// v_y <- L_y (L_y v_y - dt/rho0 d+_y p) (Alg. 1 momentum step) commutes with
// F_x and is applied here, where F_x d+_y p is at hand.  Per slot (grid.y =
// slots): Q (field 0) -> F_y^-1 Q to field 0 (d+_x p, finished by X1);
//   G = F_y^-1 (i k_y e^{+i k_y dy/2} Q) = F_x(d+_y p) / nx;
//   V_y <- L_y (L_y V_y - nx dt/rho0 G);  F_y V_y -> field 1.
// (v_z, whose factor depends on z, is advanced in the Z2 pass; v_x in X1.)
// L == ny.
// Inverse transform of the tile in LDS (G), V <- lam (lam V - vcoef G) on the
// state rows of gv (loaded only now, so that no tile is held in registers
// through the transform), then the forward transform of V to gout.
template <typename T, int L, int TW, int NT, int PL>
__device__ __forceinline__ void y_vel_update(cplx<T>* buf, const cplx<T>* twl, const T* lam_row, T vcoef, cplx<T>* gv,
                                             cplx<T>* gout, size_t px, int ncol) {
  using C = cplx<T>;
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
  lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
  C vs[EPT];
  tile_prefetch<T, L, TW, NT>(vs, gv, px, ncol);
  // each thread updates the elements it loaded (same element map as the tile load)
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if (E % NT == 0 || e < E) {
      const T lam = lam_row[e / TW];
      const C g = buf[e];
      const C vn = cmake<C>(lam * (lam * vs[i].x - vcoef * g.x), lam * (lam * vs[i].y - vcoef * g.y));
      buf[e] = vn;
      if (e % TW < ncol) gst(gv + (size_t)(e / TW) * px + e % TW, vn);
    }
  }
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, false, PL>(buf, twl);
  tile_store<T, L, TW, NT>(buf, gout, px, ncol);
}

template <typename T, int L, int TB, int PL = 0>
__global__ void __launch_bounds__(axis_nt(L, tile_tw<T, TB>()))
__attribute__((amdgpu_waves_per_eu(yv_waves<T, L, TB>()))) k_axis_y_vel(AxisArgs<T> a) {
  using C = cplx<T>;
  constexpr int TW = tile_tw<T, TB>();
  constexpr int NT = axis_nt(L, TW);
  constexpr int E = L * TW;
  constexpr int EPT = (E + NT - 1) / NT;
  constexpr int TPT = TwRegs<L, NT>::N_PER;
  __shared__ C buf[L * TW];
  __shared__ C twl[L];
  __shared__ C sfl[L];   // i k_y e^{+i k_y dy/2}
  __shared__ T lml[L];   // Lambda^s_y
  const int ntx = (a.d.px + TW - 1) / TW;   // tiles per spectrum row
  const int tl = tile_linear<TB>();
  const int tile = tl % ntx;
  const int z = tl / ntx;
  const Slot<T>& sl = a.slots[slot_of(blockIdx.y, a.slot0, a.na, a.slot1)];
  const size_t px = a.d.px;
  const size_t off = (size_t)z * L * px + (size_t)tile * TW;
  const int ncol = min(TW, (int)px - tile * TW);
  C* const gq = sl.spec[0] + off;
  C q[EPT];
  {
    C tt[TPT], ts[TPT];
    T tl[TPT];
    tile_prefetch<T, L, TW, NT>(q, gq, px, ncol);
    tw_prefetch<T, L, NT>(tt, a.tb.tw_y);
    tw_prefetch<T, L, NT>(ts, a.tb.sfac_p[1]);
#pragma unroll
    for (int i = 0; i < TPT; ++i) tl[i] = gld(a.tb.pml_s[1] + min((int)threadIdx.x + i * NT, L - 1));
    tile_commit<T, L, TW, NT>(buf, q);
    tw_commit<T, L, NT>(twl, tt);
    tw_commit<T, L, NT>(sfl, ts);
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      const int e = (int)threadIdx.x + i * NT;
      if (L % NT == 0 || e < L) lml[e] = tl[i];
    }
  }
  __syncthreads();
  lds_fft<T, L, TW, TW, NT, true, PL>(buf, twl);
  tile_store<T, L, TW, NT>(buf, gq, px, ncol);     // F_y^-1 Q
  __syncthreads();
  // Q again from F_y^-1 Q (a forward transform in LDS gives L Q) instead of
  // keeping the loaded tile in registers through the first transform: with
  // the velocity state loaded only after the next transform, the kernel
  // fits 128 VGPRs, two 448-row groups run per CU, and the pass takes 11 %
  // less time (448x448x224 FP32)
  lds_fft<T, L, TW, TW, NT, false, PL>(buf, twl);
  const T inv_l = (T)1 / (T)L;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if (E % NT == 0 || e < E) buf[e] = cscale(cmul(sfl[e / TW], buf[e]), inv_l);
  }
  C* const gv = reinterpret_cast<C*>(sl.v[1]) + off;
  __syncthreads();
  y_vel_update<T, L, TW, NT, PL>(buf, twl, lml, a.vcoef, gv, sl.spec[1] + off, px, ncol);
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

// Same walk over every item of the thread, in range or not, with r and k
// clamped into range and ok telling whether the item is in range: loads are
// issued unpredicated from a valid address (a predicated load in its own
// branch is waited for before the next one is issued).
template <int NR, int NK, typename F>
__device__ __forceinline__ void lanes2d_all(F&& fn) {
  using Ly = Lanes<NR, NK>;
  const int kq = (int)threadIdx.x % Ly::KT;
  const int rq = (int)threadIdx.x / Ly::KT;
#pragma unroll
  for (int ir = 0; ir < Ly::RI; ++ir) {
#pragma unroll
    for (int ik = 0; ik < Ly::KI; ++ik) {
      const int r = rq + ir * Ly::RT;
      const int k = kq + ik * Ly::KT;
      const bool ok = (NR % Ly::RT == 0 || r < NR) && (NK % Ly::KT == 0 || k < NK);
      fn(ir * Ly::KI + ik, min(r, NR - 1), min(k, NK - 1), ok);
    }
  }
}

// Spectra lines (M+1 complex) of NREG regions x LPB lines <-> LDS columns
// col0 + f LPB + l, rows 0..M.  The region loop is unrolled so that every
// spectrum pointer is selected at compile time (a run-time index into the
// pointer array would place it in scratch memory).
template <typename T, int M, int LPB, int NREG> struct SpecRegs {
  static constexpr int PER = Lanes<LPB, M + 1>::NI;
  static constexpr int N = NREG * PER;
};
template <typename T, int M, int LPB, int NREG>
__device__ __forceinline__ void x_prefetch_spectra(cplx<T>* pre, cplx<T>* const* spec, int l0, int nl, size_t px) {
  using C = cplx<T>;
  constexpr int PER = SpecRegs<T, M, LPB, NREG>::PER;
#pragma unroll
  for (int f = 0; f < NREG; ++f) {
    const C* s = spec[f];
    lanes2d_all<LPB, M + 1>([&](int i, int l, int k, bool) {
      const C v = gld(s + (size_t)(l0 + min(l, nl - 1)) * px + k);
      pre[f * PER + i] = (l < nl) ? v : cmake<C>((T)0, (T)0);
    });
  }
}
template <typename T, int M, int LPB, int TWP, int NREG>
__device__ __forceinline__ void x_commit_spectra(cplx<T>* buf, const cplx<T>* pre, int col0) {
  constexpr int PER = SpecRegs<T, M, LPB, NREG>::PER;
#pragma unroll
  for (int f = 0; f < NREG; ++f)
    lanes2d<LPB, M + 1>([&](int i, int l, int k) { buf[k * TWP + col0 + f * LPB + l] = pre[f * PER + i]; });
}
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
  // Whole rows up to the pitch, zeros past k = M: every store covers full
  // 128-byte lines.  A partial last line per row (1800 of 1920 bytes at
  // nx = 448) made the x passes 9 % slower: the memory side merges partial
  // lines by read-modify-write.  The zero padding stays zero through the y and
  // z passes (columns never mix).
  constexpr int PT = pitch_tw<T>();
  constexpr int NK = (M + 1 + PT - 1) / PT * PT;
#pragma unroll
  for (int f = 0; f < NREG; ++f) {
    cplx<T>* s = spec[f];
    lanes2d<LPB, NK>([&](int, int l, int k) {
      if (l < nl)
        gst(s + (size_t)(l0 + l) * px + k,
            (NK == M + 1 || k <= M) ? buf[k * TWP + col0 + f * LPB + l] : cmake<cplx<T>>((T)0, (T)0));
    });
  }
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

// x-pass twiddles staged in LDS: W_M^m (m < M) of the complex length-M
// transform followed by W_2M^k (k <= M/2) of the real <-> half-spectrum
// pre / post processing.
template <int M> struct XTw {
  static constexpr int N = M + M / 2 + 1;
  static constexpr int PER = (N + X_NT - 1) / X_NT;
};
template <typename T, int M>
__device__ __forceinline__ void x_tw_prefetch(cplx<T>* tt, const Tables<T>& tb) {
#pragma unroll
  for (int i = 0; i < XTw<M>::PER; ++i) {
    const int e = min((int)threadIdx.x + i * X_NT, XTw<M>::N - 1);
    tt[i] = gld(e < M ? tb.tw_x + e : tb.rtw + (e - M));
  }
}
template <typename T, int M>
__device__ __forceinline__ void x_tw_commit(cplx<T>* twl, const cplx<T>* tt) {
#pragma unroll
  for (int i = 0; i < XTw<M>::PER; ++i) {
    const int e = (int)threadIdx.x + i * X_NT;
    if (XTw<M>::N % X_NT == 0 || e < XTw<M>::N) twl[e] = tt[i];
  }
}

template <typename T> struct XArgs {
  const Slot<T>* slots;
  int slot0, na, slot1;   // slot ranges as in AxisArgs
  Dims d;
  Tables<T> tb;
  T dt_rho;   // dt / rho0
};

// X1: d+_x p (C2R of field 0 after the shift factor i k_x e^{+i k_x dx/2}),
// v_x <- L^s_x (L^s_x v_x - dt/rho0 d+_x p) with L^s_x varying along x (Alg. 1
// momentum step), R2C of v_x into field 0.  (v_y and v_z are advanced by the
// inverse y pass, k_axis_y_vel.)
template <typename T, int M, int PL = 0>
__global__ void __launch_bounds__(X_NT) __attribute__((amdgpu_waves_per_eu(4))) k_x_velocity(XArgs<T> a) {
  using C = cplx<T>;
  constexpr int LPB = x_lpb_vel<T>(M);
  constexpr int NC = LPB;
  constexpr int TWP = NC;
  __shared__ C buf[(M + 1) * TWP];
  __shared__ C twl[XTw<M>::N];
  const int l0 = blockIdx.x * LPB;
  const int nl = min(LPB, a.d.nlines - l0);
  const Slot<T> sl = a.slots[slot_of(blockIdx.y, a.slot0, a.na, a.slot1)];
  const size_t px = a.d.px;
  const int nx = a.d.nx;
  // velocities and PML factors are prefetched: in flight during the C2R
  using Ly = Lanes<LPB, M>;
  C vv[Ly::NI];
  C l0f[Ly::NI];          // (Lambda^s_x at x = 2n, 2n + 1)
  lanes2d_all<LPB, M>([&](int i, int l, int n, bool) {
    const size_t lo = (size_t)(l0 + min(l, nl - 1)) * nx;
    vv[i] = gld(reinterpret_cast<const C*>(sl.v[0] + lo) + n);
    l0f[i] = gld(reinterpret_cast<const C*>(a.tb.pml_s[0]) + n);
  });
  {
    C pre[SpecRegs<T, M, LPB, 1>::N], tt[XTw<M>::PER], sx[Lanes<LPB, M + 1>::NI];
    x_prefetch_spectra<T, M, LPB, 1>(pre, sl.spec, l0, nl, px);
    x_tw_prefetch<T, M>(tt, a.tb);
    lanes2d_all<LPB, M + 1>([&](int i, int, int k, bool) { sx[i] = gld(a.tb.sfac_p[0] + k); });
#pragma unroll
    for (int i = 0; i < Lanes<LPB, M + 1>::NI; ++i) pre[i] = cmul(sx[i], pre[i]);
    x_commit_spectra<T, M, LPB, TWP, 1>(buf, pre, 0);
    x_tw_commit<T, M>(twl, tt);
  }
  __syncthreads();
  c2r_pre<T, M, TWP, NC>(buf, twl + M);
  __syncthreads();
  lds_fft<T, M, NC, TWP, X_NT, true, PL>(buf, twl);
  lanes2d<LPB, M>([&](int i, int l, int n) {
    if (l >= nl) return;
    const C dp = buf[n * TWP + l];
    const T lx = l0f[i].x, ly = l0f[i].y;
    const C vn = cmake<C>(lx * (lx * vv[i].x - a.dt_rho * dp.x), ly * (ly * vv[i].y - a.dt_rho * dp.y));
    gst(reinterpret_cast<C*>(sl.v[0] + (size_t)(l0 + l) * nx) + n, vn);
    buf[n * TWP + l] = vn;
  });
  __syncthreads();
  lds_fft<T, M, NC, TWP, X_NT, false, PL>(buf, twl);
  r2c_post<T, M, TWP, NC>(buf, twl + M);
  __syncthreads();
  x_store_spectra<T, M, LPB, TWP, 1>(buf, sl.spec, 0, l0, nl, px);
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
  const int32_t* delay;  // [B][n_src] whole-step source delays, or null (none)
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
  // absorption (lossy passes only)
  T rho0;
  const T* alpha0;       // [nfield] per-voxel alpha0 or null (then alpha0_u)
  T alpha0_u;            // uniform alpha0, Np (rad/s)^-y m^-1
  T y1;                  // y - 1
  T two_tan;             // 2 tan(pi y / 2)
  T tr_tau_sign;         // sign of tau in the TR simulation (-1: switched)
  T* padj;               // [B][n_gam]: adjoint pressure on Gamma of this step
  // exact gradient: [nt][n_gam] dp/dc0 at fixed state on Gamma per forward
  // step (problem 0), or null
  T* hist;
  int pml[3];            // PML cells at both ends of x, y, z (normal grid: Lambda != 1 there)
  const cplx<T>* ad;     // absorption: A[d] per slot (AxisArgs::ad), read by the lossy EOS
  long long ad_stride;
};

// Storage of the split densities (three real fields per slot).  Inside the
// PML of axis a the component rho_a is damped by Lambda_a and must be kept
// apart; elsewhere the components evolve alike (rho_a <- rho_a - dt rho0
// d-_a v_a) and only their sum enters the equation of state.  So an x-line
// outside the y and z PML slabs (most lines) keeps in field 0 the undamped
// part u = sum of the components with Lambda_a = 1 (all three, or rho_y +
// rho_z on the x-PML voxels), and in field 1 rho_x on the x-PML voxels only;
// field 2 is not used there.  Lines in a y or z slab keep the three
// components.  Same arithmetic, 2 + 4 P_x / nx instead of 6 field accesses
// per voxel on those lines.  On the same lines the inverse y pass delivers
// d-_y v_y + d-_z v_z as the second spectrum and no third one (k_axis_y_div).
template <typename T> __device__ __forceinline__ bool full_split_line(const X2Args<T>& a, int line) {
  return in_pml_slab(line % a.d.ny, a.d.ny, a.pml[1]) || in_pml_slab(line / a.d.ny, a.d.nz, a.pml[2]);
}
// the voxel pair (2n, 2n+1) of an x-line touches the x PML
template <typename T> __device__ __forceinline__ bool x_pml_pair(const X2Args<T>& a, int n) {
  return in_pml_slab(2 * n, a.d.nx, a.pml[0]) || in_pml_slab(2 * n + 1, a.d.nx, a.pml[0]);
}

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
// STAGE_TW: this call also stages the x twiddles in twl (the first call of
// the workgroup); later calls find them there.
// LOSSY: instead of p, column pcol receives s = sum_a rho_a, which is also
// stored as a real field in the slot's third spectrum buffer (rows of px
// complex), for the lossy equation of state (A[d] comes from the z pass).
// The update runs in phases around the C2R so that the paired pass can
// transform the derivative spectra of both of its simulations at once:
// density_load (registers: c0, densities, PML factors; the three spectra into
// LDS columns col0 + f LPB; the sparse inputs into spv / spm), one C2R of all
// TWP columns (density_c2r), density_finish (the update; p or s to column
// pcol of bufp).  density_update runs the three for one slot.
template <typename T, int M, int LPB> struct DensRegs {
  static constexpr int EB = Lanes<LPB, M>::NI;
  cplx<T> cc[EB], rr[EB][3], l0f[EB];
  T l1f[EB], l2f[EB];
};
template <typename T, int M, int LPB, int TWP, int KIND, bool STAGE_TW, bool LOSSY>
__device__ __forceinline__ void density_load(const X2Args<T>& a, const StepIdx& si, const Slot<T>& sl, int b, int l0,
                                             int nl, int state_mode, int col0, cplx<T>* buf, cplx<T>* spv,
                                             uint8_t* spm, cplx<T>* twl, DensRegs<T, M, LPB>& r) {
  const bool zero_state = state_mode == 1;
  const bool no_step = state_mode != 0;
  using C = cplx<T>;
  const int nx = a.d.nx;
  const size_t px = a.d.px;
  const T* cb = a.c + (size_t)b * a.d.nfield;
  // prefetch c0, the split densities and the PML factors: in flight during
  // the C2R transforms
  C* const cc = r.cc;
  C(*const rr)[3] = r.rr;
  C* const l0f = r.l0f;
  T* const l1f = r.l1f;
  T* const l2f = r.l2f;
  lanes2d_all<LPB, M>([&](int i, int l, int n, bool) {
    const int line = l0 + min(l, nl - 1);
    const size_t lo = (size_t)line * nx;
    if (!LOSSY) cc[i] = gld(reinterpret_cast<const C*>(cb + lo) + n);
    if (!zero_state) {
      const bool full = full_split_line(a, line);
      rr[i][0] = gld(reinterpret_cast<const C*>(sl.rho[0] + lo) + n);
      rr[i][1] = (full || x_pml_pair(a, n)) ? gld(reinterpret_cast<const C*>(sl.rho[1] + lo) + n) : cmake<C>((T)0, (T)0);
      rr[i][2] = full ? gld(reinterpret_cast<const C*>(sl.rho[2] + lo) + n) : cmake<C>((T)0, (T)0);
    }
    if (!no_step) {
      l0f[i] = gld(reinterpret_cast<const C*>(a.tb.pml_n[0]) + n);
      l1f[i] = gld(a.tb.pml_n[1] + line % a.d.ny);
      l2f[i] = gld(a.tb.pml_n[2] + line / a.d.ny);
    }
  });
  {
    C pre[SpecRegs<T, M, LPB, 3>::N], tt[XTw<M>::PER];
    if (!no_step) {
      // fields 0 and 1; field 2 only on the lines that keep the split (zeros
      // elsewhere: field 1 holds d-_y v_y + d-_z v_z there)
      x_prefetch_spectra<T, M, LPB, 2>(pre, sl.spec, l0, nl, px);
      constexpr int PER = SpecRegs<T, M, LPB, 3>::PER;
      lanes2d_all<LPB, M + 1>([&](int i, int l, int k, bool) {
        const bool rd = l < nl && full_split_line(a, l0 + l);
        pre[2 * PER + i] = rd ? gld(sl.spec[2] + (size_t)(l0 + l) * px + k) : cmake<C>((T)0, (T)0);
      });
    }
    if (STAGE_TW) x_tw_prefetch<T, M>(tt, a.tb);
    if (!no_step) x_commit_spectra<T, M, LPB, TWP, 3>(buf, pre, col0);
    if (STAGE_TW) x_tw_commit<T, M>(twl, tt);
  }
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
      // delayed encoding (eq. DelaySE): source id fires its signal d_id steps late
      const int k = a.delay ? si.step - a.delay[(size_t)b * a.d.n_src + id] : si.step;
      const T sv = k >= 0 ? a.src_sig[((size_t)b * a.d.nt + k) * a.d.n_src + id] : (T)0;
      const T val = a.src_k / cv * (T)a.w[(size_t)b * a.d.n_src + id] * sv;
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
}
// inverse x transforms of all TWP columns of buf (after density_load)
template <typename T, int M, int TWP, int PL>
__device__ __forceinline__ void density_c2r(cplx<T>* buf, const cplx<T>* twl) {
  c2r_pre<T, M, TWP, TWP>(buf, twl + M);
  __syncthreads();
  lds_fft<T, M, TWP, TWP, X_NT, true, PL>(buf, twl);
}
template <typename T, int M, int LPB, int TWP, int TWPP, int KIND, bool LOSSY>
__device__ __forceinline__ void density_finish(const X2Args<T>& a, const Slot<T>& sl, int l0, int nl,
                                               int state_mode, int col0, int pcol, const cplx<T>* buf,
                                               cplx<T>* bufp, const cplx<T>* spv, const uint8_t* spm,
                                               const DensRegs<T, M, LPB>& r) {
  const bool zero_state = state_mode == 1;
  const bool no_step = state_mode != 0;
  using C = cplx<T>;
  const int nx = a.d.nx;
  const size_t px = a.d.px;
  const C* const cc = r.cc;
  const C(*const rr)[3] = r.rr;
  const C* const l0f = r.l0f;
  const T* const l1f = r.l1f;
  const T* const l2f = r.l2f;
  lanes2d<LPB, M>([&](int i, int l, int n) {
    if (l >= nl) return;
    const int line = l0 + l;
    const C c2 = cc[i];
    const C sv = spv[n * LPB + l];
    C sum = cmake<C>((T)0, (T)0);
    if (!full_split_line(a, line)) {
      // undamped part u in field 0, rho_x on the x-PML pairs in field 1
      const bool xp = x_pml_pair(a, n);
      const T nu = xp ? (T)2 : (T)3;   // components in u
      C u, rx = cmake<C>((T)0, (T)0);
      if (zero_state) {
        u = cmake<C>((T)0, (T)0);
      } else if (no_step) {
        u = rr[i][0];
        rx = rr[i][1];
      } else {
        const C d0 = buf[n * TWP + col0 + l], d1 = buf[n * TWP + col0 + LPB + l],
                d2 = buf[n * TWP + col0 + 2 * LPB + l];
        const C du = xp ? cadd(d1, d2) : cadd(cadd(d0, d1), d2);
        u = cmake<C>(rr[i][0].x - a.dt_rho0 * du.x, rr[i][0].y - a.dt_rho0 * du.y);
        if (xp) {
          const T lx = l0f[i].x, ly = l0f[i].y;
          rx = cmake<C>(lx * (lx * rr[i][1].x - a.dt_rho0 * d0.x), ly * (ly * rr[i][1].y - a.dt_rho0 * d0.y));
        }
      }
      if (KIND == SP_DIRICHLET) {
        if (spm[2 * (n * LPB + l)]) { u.x = nu * sv.x; rx.x = sv.x; }
        if (spm[2 * (n * LPB + l) + 1]) { u.y = nu * sv.y; rx.y = sv.y; }
      } else {
        u = cmake<C>(u.x + nu * sv.x, u.y + nu * sv.y);
        rx = cadd(rx, sv);
      }
      const size_t lo = (size_t)line * nx;
      gst(reinterpret_cast<C*>(sl.rho[0] + lo) + n, u);
      if (xp) gst(reinterpret_cast<C*>(sl.rho[1] + lo) + n, rx);
      sum = xp ? cadd(u, rx) : u;
    } else
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      C* rp = reinterpret_cast<C*>(sl.rho[f] + (size_t)line * nx) + n;
      C rn;
      if (zero_state) {
        rn = cmake<C>((T)0, (T)0);
      } else if (no_step) {
        rn = rr[i][f];
      } else {
        const C dv = buf[n * TWP + col0 + f * LPB + l];
        const T lx = f == 0 ? l0f[i].x : (f == 1 ? l1f[i] : l2f[i]);
        const T ly = f == 0 ? l0f[i].y : (f == 1 ? l1f[i] : l2f[i]);
        rn = cmake<C>(lx * (lx * rr[i][f].x - a.dt_rho0 * dv.x), ly * (ly * rr[i][f].y - a.dt_rho0 * dv.y));
      }
      if (KIND == SP_DIRICHLET) {
        if (spm[2 * (n * LPB + l)]) rn.x = sv.x;
        if (spm[2 * (n * LPB + l) + 1]) rn.y = sv.y;
      } else {
        rn = cadd(rn, sv);
      }
      gst(rp, rn);
      sum = cadd(sum, rn);
    }
    if (LOSSY) {
      bufp[n * TWPP + pcol + l] = sum;
      gst(sl.spec[2] + (size_t)line * px + n, sum);
    } else {
      bufp[n * TWPP + pcol + l] = cmake<C>(c2.x * c2.x * sum.x, c2.y * c2.y * sum.y);
    }
  });
  __syncthreads();
}
template <typename T, int M, int LPB, int TWP, int TWPP, int KIND, bool STAGE_TW, bool LOSSY = false, int PL = 0>
__device__ __forceinline__ void density_update(const X2Args<T>& a, const StepIdx& si, const Slot<T>& sl, int b,
                                               int l0, int nl, int state_mode, int pcol, cplx<T>* buf,
                                               cplx<T>* bufp, cplx<T>* spv, uint8_t* spm, cplx<T>* twl) {
  static_assert(TWP == 3 * LPB, "one slot: three spectra of LPB lines");
  DensRegs<T, M, LPB> r;
  density_load<T, M, LPB, TWP, KIND, STAGE_TW, LOSSY>(a, si, sl, b, l0, nl, state_mode, 0, buf, spv, spm, twl, r);
  if (state_mode == 0) density_c2r<T, M, TWP, PL>(buf, twl);
  else __syncthreads();
  density_finish<T, M, LPB, TWP, TWPP, KIND, LOSSY>(a, sl, l0, nl, state_mode, 0, pcol, buf, bufp, spv, spm, r);
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
template <typename T, int M, int MODE, int PL = 0>
__global__ void __launch_bounds__(X_NT) k_x_density(X2Args<T> a) {
  using C = cplx<T>;
  constexpr int LPB = x_lpb_den_mode<T>(M, MODE);
  constexpr int NP = (MODE == XM_PAIR) ? 2 : 1;
  constexpr int TWP = 3 * LPB * NP;   // d-_a v_a of the three axes (per simulation)
  constexpr int TWPP = NP * LPB;      // new pressure(s), packed for the R2C
  __shared__ C buf[(M + 1) * TWP];
  __shared__ C bufp[(M + 1) * TWPP];
  __shared__ C spv[M * LPB * NP];
  __shared__ uint8_t spm[(MODE == XM_PAIR || MODE == XM_TRONLY) ? 2 * M * LPB : 1];
  __shared__ C twl[XTw<M>::N];
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

  if constexpr (MODE == XM_FWD) {
    density_update<T, M, LPB, TWP, TWPP, SP_SOURCE, true, false, PL>(a, si, s_tr, b, l0, nl, 0, PA, buf, bufp, spv, spm,
                                                          twl);
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
    if (a.hist) {
      // exact gradient: dp/dc0 of p = c0^2 sum rho at a fixed state, (2/c0) p
      const int j0 = a.g.gam_off[l0], j1 = a.g.gam_off[l0 + nl];
      T* hrow = a.hist + (size_t)si.step * a.d.n_gam;
      for (int i = j0 + (int)threadIdx.x; i < j1; i += X_NT) {
        const int l = local_line(a.g.gam_off, l0, nl, i);
        const int x = a.g.gam_x[i];
        hrow[i] = (T)2 / a.c[(size_t)(l0 + l) * nx + x] * p_at<T, TWPP>(bufp, PA, l, x);
      }
    }
  }
  if constexpr (MODE == XM_PAIR) {
    // adjoint (columns 0 ..) and TR (columns 3 LPB ..) through one C2R
    DensRegs<T, M, LPB> ra, rt;
    C* const spv_t = spv + M * LPB;
    density_load<T, M, LPB, TWP, SP_ADJOINT, true, false>(a, si, s_adj, b, l0, nl, 0, 0, buf, spv, nullptr, twl, ra);
    density_load<T, M, LPB, TWP, SP_DIRICHLET, false, false>(a, si, s_tr, b, l0, nl, a.tr_state_mode, 3 * LPB, buf,
                                                             spv_t, spm, twl, rt);
    density_c2r<T, M, TWP, PL>(buf, twl);
    density_finish<T, M, LPB, TWP, TWPP, SP_ADJOINT, false>(a, s_adj, l0, nl, 0, 0, PA, buf, bufp, spv, nullptr, ra);
    density_finish<T, M, LPB, TWP, TWPP, SP_DIRICHLET, false>(a, s_tr, l0, nl, a.tr_state_mode, 3 * LPB, PT, buf, bufp,
                                                              spv_t, spm, rt);
  }
  if constexpr (MODE == XM_ADJONLY) {
    density_update<T, M, LPB, TWP, TWPP, SP_ADJOINT, true, false, PL>(a, si, s_adj, b, l0, nl, 0, PA, buf, bufp, spv,
                                                           spm, twl);
  }
  if constexpr (MODE == XM_TRONLY) {
    density_update<T, M, LPB, TWP, TWPP, SP_DIRICHLET, MODE == XM_TRONLY, false, PL>(a, si, s_tr, b, l0, nl, a.tr_state_mode,
                                                                          PT, buf, bufp, spv, spm, twl);
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
  lds_fft<T, M, TWPP, TWPP, X_NT, false, PL>(bufp, twl);
  r2c_post<T, M, TWPP, TWPP>(bufp, twl + M);
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
// lossy passes (power-law absorption, Sec. 2.1): the density update is split
// from the equation of state, which needs the fractional Laplacians of s and d
// (three axis passes in between: forward y, k_axis_z_frac, inverse y)
// ----------------------------------------------------------------------------
// XL1: C2R of d-_a v_a, split-density update with PML and the injection or
// imposition of KIND (SP_SOURCE forward, SP_ADJOINT adjoint, SP_DIRICHLET TR
// with a.tr_state_mode as in X2), then s = sum_a rho_a (also kept as a real
// field in the third spectrum buffer), whose forward x transform goes to
// field 0.  (A[d] of d = rho0 sum_a d-_a v_a is formed by the lossy Z1.)
template <typename T, int M, int KIND>
__global__ void __launch_bounds__(X_NT) k_x_lossy_rho(X2Args<T> a) {
  using C = cplx<T>;
  constexpr int LPB = x_lpb_den<T>(M);
  constexpr int TWP = 3 * LPB;        // d-_a v_a of the three axes
  constexpr int TWPP = LPB;           // s
  __shared__ C buf[(M + 1) * TWP];
  __shared__ C bufp[(M + 1) * TWPP];
  __shared__ C spv[M * LPB];
  __shared__ uint8_t spm[KIND == SP_DIRICHLET ? 2 * M * LPB : 1];
  __shared__ C twl[XTw<M>::N];
  const int l0 = blockIdx.x * LPB;
  const int nl = min(LPB, a.d.nlines - l0);
  const int b = blockIdx.y;
  const Slot<T> sl = a.slots[KIND == SP_ADJOINT ? b : a.tr_off + b];
  // forward steps count n, adjoint / TR steps the paired iteration j (a
  // replayed step graph reads either from a.step_dev)
  const StepIdx si = KIND == SP_SOURCE ? step_indices<T, XM_FWD>(a) : step_indices<T, XM_PAIR>(a);
  const int state_mode = KIND == SP_DIRICHLET ? a.tr_state_mode : 0;
  density_update<T, M, LPB, TWP, TWPP, KIND, true, true>(a, si, sl, b, l0, nl, state_mode, 0, buf, bufp, spv,
                                                         spm, twl);
  lds_fft<T, M, TWPP, TWPP, X_NT, false>(bufp, twl);
  r2c_post<T, M, TWPP, TWPP>(bufp, twl + M);
  __syncthreads();
  cplx<T>* specs[1] = {sl.spec[0]};
  x_store_spectra<T, M, LPB, TWPP, 1>(bufp, specs, 0, l0, nl, a.d.px);
}

// XL2: C2R of field 0 (B[s] = F^-1 |k|^{y-1} F s) and of the slot's A[d] =
// F^-1 |k|^{y-2} F d (zero when the TR starts without a density step), lossy
// equation of state
//   p = c0^2 (s + sgn tau A[d] - eta B[s]),
//   tau = -2 alpha0 c0^{y-1},  eta = 2 alpha0 c0^y tan(pi y / 2),
// sgn = a.tr_tau_sign for the TR (KIND SP_DIRICHLET), else +1; then the
// outputs of KIND (forward: traces f^n and tape g^n; adjoint: p on Gamma to
// a.padj; TR: p on Gamma to ring slot a.ring_c, or (j + 2) mod 3 in a replayed
// step graph) and the forward x transform
// of p into field 0.
template <typename T, int M, int KIND>
__global__ void __launch_bounds__(X_NT) k_x_lossy_eos(X2Args<T> a) {
  using C = cplx<T>;
  constexpr int LPB = x_lpb_eos<T>(M);
  constexpr int TWP = 2 * LPB;        // B[s] in columns 0.., A[d] in LPB..
  __shared__ C buf[(M + 1) * TWP];
  __shared__ C twl[XTw<M>::N];
  const int l0 = blockIdx.x * LPB;
  const int nl = min(LPB, a.d.nlines - l0);
  const int b = blockIdx.y;
  const int nx = a.d.nx;
  const size_t px = a.d.px;
  const Slot<T> sl = a.slots[KIND == SP_ADJOINT ? b : a.tr_off + b];
  const T* cb = a.c + (size_t)b * a.d.nfield;
  const T sgn = KIND == SP_DIRICHLET ? a.tr_tau_sign : (T)1;
  const StepIdx si = KIND == SP_SOURCE ? step_indices<T, XM_FWD>(a) : step_indices<T, XM_PAIR>(a);
  using Ly = Lanes<LPB, M>;
  C ss[Ly::NI], cc[Ly::NI], aa[Ly::NI];
  lanes2d_all<LPB, M>([&](int i, int l, int n, bool) {
    const int line = l0 + min(l, nl - 1);
    ss[i] = gld(sl.spec[2] + (size_t)line * px + n);
    cc[i] = gld(reinterpret_cast<const C*>(cb + (size_t)line * nx) + n);
    aa[i] = a.alpha0 ? gld(reinterpret_cast<const C*>(a.alpha0 + (size_t)line * nx) + n)
                     : cmake<C>(a.alpha0_u, a.alpha0_u);
  });
  {
    const bool no_step = KIND == SP_DIRICHLET && a.tr_state_mode != 0;
    cplx<T>* specs[2] = {sl.spec[0],
                         const_cast<C*>(a.ad) + (size_t)(KIND == SP_ADJOINT ? b : a.tr_off + b) * a.ad_stride};
    C pre[SpecRegs<T, M, LPB, 2>::N], tt[XTw<M>::PER];
    x_prefetch_spectra<T, M, LPB, 2>(pre, specs, l0, nl, px);
    x_tw_prefetch<T, M>(tt, a.tb);
    if (no_step) {
#pragma unroll
      for (int i = 0; i < SpecRegs<T, M, LPB, 2>::PER; ++i) pre[SpecRegs<T, M, LPB, 2>::PER + i] = cmake<C>((T)0, (T)0);
    }
    x_commit_spectra<T, M, LPB, TWP, 2>(buf, pre, 0);
    x_tw_commit<T, M>(twl, tt);
  }
  __syncthreads();
  c2r_pre<T, M, TWP, TWP>(buf, twl + M);
  __syncthreads();
  lds_fft<T, M, TWP, TWP, X_NT, true>(buf, twl);
  auto eos = [&](T s, T A, T B, T c, T al) -> T {
    const T cy1 = real_pow(c, a.y1);               // c0^{y-1}
    const T tau = (T)-2 * al * cy1;
    const T eta = a.two_tan * al * (c * cy1);
    return c * c * (s + sgn * tau * A - eta * B);
  };
  // exact gradient: dp/dc0 at a fixed state, (2/c0) p + c0^2 (tau' A - eta' B)
  // with tau' = -2 alpha0 (y-1) c0^{y-2}, eta' = 2 alpha0 y c0^{y-1} tan(pi y/2)
  auto dpdc = [&](T p, T A, T B, T c, T al) -> T {
    const T cy1 = real_pow(c, a.y1);               // c0^{y-1}
    const T dtau = (T)-2 * al * a.y1 * cy1 / c;
    const T deta = (a.y1 + (T)1) * a.two_tan * al * cy1;
    return (T)2 / c * p + c * c * (dtau * A - deta * B);
  };
  const bool want_hist = KIND == SP_SOURCE && a.hist != nullptr;
  lanes2d<LPB, M>([&](int i, int l, int n) {
    if (l >= nl) return;
    const C Bv = buf[n * TWP + l];
    const C Av = buf[n * TWP + LPB + l];
    const C pv = cmake<C>(eos(ss[i].x, Av.x, Bv.x, cc[i].x, aa[i].x), eos(ss[i].y, Av.y, Bv.y, cc[i].y, aa[i].y));
    buf[n * TWP + l] = pv;
    if (want_hist)   // A is not needed any more: its column takes dp/dc0
      buf[n * TWP + LPB + l] = cmake<C>(dpdc(pv.x, Av.x, Bv.x, cc[i].x, aa[i].x),
                                        dpdc(pv.y, Av.y, Bv.y, cc[i].y, aa[i].y));
  });
  __syncthreads();
  if (want_hist) {
    const int j0 = a.g.gam_off[l0], j1 = a.g.gam_off[l0 + nl];
    T* hrow = a.hist + (size_t)si.step * a.d.n_gam;
    for (int i = j0 + (int)threadIdx.x; i < j1; i += X_NT) {
      const int l = local_line(a.g.gam_off, l0, nl, i);
      hrow[i] = p_at<T, TWP>(buf, LPB, l, a.g.gam_x[i]);
    }
  }
  if (KIND == SP_SOURCE) {
    const int i0 = a.g.rec_off[l0], i1 = a.g.rec_off[l0 + nl];
    for (int i = i0 + (int)threadIdx.x; i < i1; i += X_NT) {
      const int l = local_line(a.g.rec_off, l0, nl, i);
      a.traces[((size_t)b * a.d.nt + si.step) * a.d.n_rec + a.g.rec_id[i]] = p_at<T, TWP>(buf, 0, l, a.g.rec_x[i]);
    }
    if (a.tape) {
      const int j0 = a.g.bnd_off[l0], j1 = a.g.bnd_off[l0 + nl];
      T* trow = a.tape + ((size_t)b * a.d.nt + si.step) * a.d.n_bnd;
      for (int i = j0 + (int)threadIdx.x; i < j1; i += X_NT) {
        const int l = local_line(a.g.bnd_off, l0, nl, i);
        trow[i] = p_at<T, TWP>(buf, 0, l, a.g.bnd_x[i]);
      }
    }
  } else {
    T* dst = KIND == SP_ADJOINT ? a.padj + (size_t)b * a.d.n_gam
                                : a.ring + ((size_t)b * 3 + si.rc) * a.d.n_gam;
    const int i0 = a.g.gam_off[l0], i1 = a.g.gam_off[l0 + nl];
    for (int i = i0 + (int)threadIdx.x; i < i1; i += X_NT) {
      const int l = local_line(a.g.gam_off, l0, nl, i);
      dst[i] = p_at<T, TWP>(buf, 0, l, a.g.gam_x[i]);
    }
  }
  __syncthreads();
  lds_fft<T, M, LPB, TWP, X_NT, false>(buf, twl);
  r2c_post<T, M, TWP, LPB>(buf, twl + M);
  __syncthreads();
  cplx<T>* specs[1] = {sl.spec[0]};
  x_store_spectra<T, M, LPB, TWP, 1>(buf, specs, 0, l0, nl, px);
}

// Gradient step of the lossy TR gradient (Alg. 1 form):
//   G += 2 / c0^3 p_adj (p_tr^(j) - 2 p_tr^(j+1) + p_tr^(j+2))
// with p_tr^(j+2) = 0 (and that ring slot cleared) when adj_only; with
// step_dev non-null the ring slots follow from the device iteration counter j.
// grid: x over Gamma voxels, y over problems.
template <typename T>
__global__ void k_lossy_grad(const T* c, const int32_t* gam_lin, const T* padj, T* ring, double* gacc, int n_gam,
                             long long nfield, int ra, int rb, int rc, int adj_only, const int* step_dev) {
  if (step_dev) {
    const int j = *step_dev;
    ra = j % 3;
    rb = (j + 1) % 3;
    rc = (j + 2) % 3;
  }
  const int b = blockIdx.y;
  T* rg = ring + (size_t)b * 3 * n_gam;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_gam; i += gridDim.x * blockDim.x) {
    T ptr;
    if (adj_only) {
      ptr = (T)0;
      rg[(size_t)rc * n_gam + i] = ptr;
    } else {
      ptr = rg[(size_t)rc * n_gam + i];
    }
    const T cv = c[(size_t)b * nfield + gam_lin[i]];
    const T pm = rg[(size_t)ra * n_gam + i];
    const T p0 = rg[(size_t)rb * n_gam + i];
    const T inc = (T)2 / (cv * cv * cv) * padj[(size_t)b * n_gam + i] * (pm - (T)2 * p0 + ptr);
    gacc[(size_t)b * n_gam + i] += (double)inc;
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

// Sum of v over the 64 lanes of a wavefront by butterfly shuffles (every
// lane ends with the same sum; the pairing order is fixed: deterministic).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Residual r^n = f^n - f^delta_n (or a given residual), adjoint source
// a^j = sum_{i<=j} r^{N-1-i} and per-block FP64 partial sums of r^2
// (wavefront shuffles, then the four wavefront sums in order).
// grid: x over receivers (256 per block), y over problems.
template <typename T>
__global__ void __launch_bounds__(256) k_residual(const T* traces, const T* obs, int obs_is_residual, T* adj,
                                                  double* partial, int nt, int n_rec) {
  __shared__ double red[4];
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
  s2 = wave_sum(s2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
  __syncthreads();
  if (threadIdx.x == 0) partial[(size_t)b * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
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

// Mean of the B gradients of one batched call (averaging of independent
// encoded realisations, Sec. 3.2): grad[gamma voxel i] = (1/B) sum_b G_b[i],
// summed in FP64 over b = 0..B-1 in that order (deterministic), rounded once.
template <typename T>
__global__ void k_grad_mean_scatter(const double* gacc, const int32_t* gam_lin, int n_gam, T* grad, int B) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_gam; i += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += gacc[(size_t)b * n_gam + i];
    grad[gam_lin[i]] = (T)(s / (double)B);
  }
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
  lanes2d<LPB, M>([&](int, int l, int n) {
    buf[n * TWP + l] = (l < nl) ? gld(reinterpret_cast<const C*>(in + (size_t)(l0 + l) * a.d.nx) + n)
                                : cmake<C>((T)0, (T)0);
  });
  __syncthreads();
  lds_fft<T, M, LPB, TWP, X_NT, false>(buf, a.tb.tw_x);
  r2c_post<T, M, TWP, LPB>(buf, a.tb.rtw);
  __syncthreads();
  cplx<T>* specs[1] = {a.slots[a.slot0].spec[f]};
  x_store_spectra<T, M, LPB, TWP, 1>(buf, specs, 0, l0, nl, a.d.px);
}

// mult (may be null): per-kx factor applied before the inverse transform
template <typename T, int M>
__global__ void __launch_bounds__(X_NT) k_x_c2r(XArgs<T> a, T* out, int f, const cplx<T>* mult) {
  using C = cplx<T>;
  constexpr int LPB = x_lpb<T>(M);
  constexpr int TWP = LPB;
  __shared__ C buf[(M + 1) * TWP];
  const int l0 = blockIdx.x * LPB;
  const int nl = min(LPB, a.d.nlines - l0);
  cplx<T>* specs[1] = {a.slots[a.slot0].spec[f]};
  x_load_spectra<T, M, LPB, TWP, 1>(buf, specs, 0, l0, nl, a.d.px);
  __syncthreads();
  if (mult) {
    lanes2d<LPB, M + 1>([&](int, int l, int k) { buf[k * TWP + l] = cmul(gld(mult + k), buf[k * TWP + l]); });
    __syncthreads();
  }
  c2r_pre<T, M, TWP, LPB>(buf, a.tb.rtw);
  __syncthreads();
  lds_fft<T, M, LPB, TWP, X_NT, true>(buf, a.tb.tw_x);
  lanes2d<LPB, M>([&](int, int l, int n) {
    if (l < nl) gst(reinterpret_cast<C*>(out + (size_t)(l0 + l) * a.d.nx) + n, buf[n * TWP + l]);
  });
}

}  // namespace fwi
