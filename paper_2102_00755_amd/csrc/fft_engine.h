// LDS-resident mixed-radix Stockham FFT for many short columns at once.
//
// A workgroup holds TW independent sequences ("columns") of length L in LDS,
// element (row r, column c) at buf[r * TWP + c].  Consecutive lanes work on
// consecutive columns of the same row, so every LDS access of a stage is a
// run of consecutive 8/16-byte words (no bank conflicts when TWP*sizeof
// is 128 B, or when TWP is odd).
//
// Each stage of radix R (Ns = product of the radices already applied) is the
// Stockham autosort step of Govindaraju et al. (SC'08, "High performance
// discrete Fourier transforms on graphics processors"): butterfly j reads
// rows j + t L/R, multiplies input t by W_L^{t (j mod Ns) L/(Ns R)}, applies
// an R-point DFT and writes rows (j/Ns) Ns R + (j mod Ns) + u Ns.  Every
// thread first loads all its butterflies into registers, the workgroup
// synchronises, then results are stored in place.  Twiddles come from a
// table W_L^m computed in FP64 on the host and rounded once.
//
// Radices: 2, 3, 4, 5, 7, 8.  Odd radices use the symmetric form
// y_k = x0 + sum_j (x_j + x_{R-j}) cos(2 pi j k / R) -+ i (x_j - x_{R-j}) sin(...).
// Forward transforms use exp(-2 pi i / L); inverse ones are unnormalised.
#pragma once

#include "fwi_common.h"

namespace fwi {

struct RadixPlan {
  int n;
  int r[8];
};

// Radix plan of length L.  Plan 0: the odd radices (7, 5, 3) first, then
// the power-of-two part as radix-8 stages with one radix-4 or radix-2 stage
// (two radix-4 stages for 16) last.  Plan 1: the same radices with the
// power-of-two stages in reverse order (e.g. 224 = 7 * 8 * 4 -> 7 * 4 * 8).
// Both compute the same DFT; they differ in rounding, in the thread mapping
// of each stage and in the twiddle pattern, and so in speed (a run-time
// choice of the x passes: fwi_set_tuning).
constexpr RadixPlan make_plan(int L, int PL = 0) {
  RadixPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0}};
  int m = L;
  while (m % 7 == 0) { p.r[p.n++] = 7; m /= 7; }
  while (m % 5 == 0) { p.r[p.n++] = 5; m /= 5; }
  while (m % 3 == 0) { p.r[p.n++] = 3; m /= 3; }
  const int first2 = p.n;
  while (m > 1) {
    if (m == 16) { p.r[p.n++] = 4; p.r[p.n++] = 4; m = 1; }
    else if (m % 8 == 0) { p.r[p.n++] = 8; m /= 8; }
    else if (m % 4 == 0) { p.r[p.n++] = 4; m /= 4; }
    else { p.r[p.n++] = 2; m /= 2; }
  }
  if (PL == 1) {
    for (int i = first2, j = p.n - 1; i < j; ++i, --j) {
      const int t = p.r[i];
      p.r[i] = p.r[j];
      p.r[j] = t;
    }
  }
  return p;
}

// Plan 1 differs from plan 0 (otherwise only plan 0 is instantiated)
constexpr bool plan_differs(int L) {
  const RadixPlan a = make_plan(L, 0), b = make_plan(L, 1);
  for (int i = 0; i < a.n; ++i)
    if (a.r[i] != b.r[i]) return true;
  return false;
}

constexpr bool plan_ok(int L) {
  int m = L;
  while (m % 7 == 0) m /= 7;
  while (m % 5 == 0) m /= 5;
  while (m % 3 == 0) m /= 3;
  while (m % 2 == 0) m /= 2;
  return m == 1 && L >= 2;
}

constexpr int plan_prefix(int L, int s, int PL = 0) {
  RadixPlan p = make_plan(L, PL);
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= p.r[i];
  return ns;
}

// cos / sin of 2 pi m / R for the odd radices (m taken mod R)
template <int R> struct OddConst;
template <> struct OddConst<3> {
  static constexpr double c(int m) { return m == 0 ? 1.0 : -0.5; }
  static constexpr double s(int m) {
    return m == 0 ? 0.0 : (m == 1 ? 0.8660254037844386467637231708 : -0.8660254037844386467637231708);
  }
};
template <> struct OddConst<5> {
  static constexpr double c(int m) {
    return m == 0 ? 1.0 : (m == 1 || m == 4) ? 0.3090169943749474241022934172 : -0.8090169943749474241022934172;
  }
  static constexpr double s(int m) {
    return m == 0 ? 0.0 : m == 1 ? 0.9510565162951535721164393334 : m == 2 ? 0.5877852522924731291687059546
         : m == 3 ? -0.5877852522924731291687059546 : -0.9510565162951535721164393334;
  }
};
template <> struct OddConst<7> {
  static constexpr double c(int m) {
    return m == 0 ? 1.0 : (m == 1 || m == 6) ? 0.6234898018587335305250048840
         : (m == 2 || m == 5) ? -0.2225209339563144042889025645 : -0.9009688679024191262361023195;
  }
  static constexpr double s(int m) {
    return m == 0 ? 0.0 : m == 1 ? 0.7818314824680298087084445267 : m == 2 ? 0.9749279121818236070181316830
         : m == 3 ? 0.4338837391175581204757683328 : m == 4 ? -0.4338837391175581204757683328
         : m == 5 ? -0.9749279121818236070181316830 : -0.7818314824680298087084445267;
  }
};

// R-point DFT in place: y_u = sum_t x_t exp(-+ 2 pi i t u / R)
template <int R, bool INV, typename C> struct Bfly;

template <bool INV, typename C> struct Bfly<2, INV, C> {
  static __device__ __forceinline__ void run(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV, typename C> struct Bfly<4, INV, C> {
  static __device__ __forceinline__ void run(C* v) {
    C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    C c = cadd(v[1], v[3]), d = crot<INV>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};

template <bool INV, typename C> struct Bfly<8, INV, C> {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(C::x);
    const T h = (T)0.7071067811865475244008443621;
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    Bfly<4, INV, C>::run(e);
    Bfly<4, INV, C>::run(o);
    // W8^u o_u, W8 = exp(-+ i pi / 4)
    C t1 = INV ? cmake<C>(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
               : cmake<C>(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    C t2 = crot<INV>(o[2]);
    C t3 = INV ? cmake<C>(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
               : cmake<C>(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], t1);
    v[5] = csub(e[1], t1);
    v[2] = cadd(e[2], t2);
    v[6] = csub(e[2], t2);
    v[3] = cadd(e[3], t3);
    v[7] = csub(e[3], t3);
  }
};

template <int R, bool INV, typename C> struct BflyOdd {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(C::x);
    constexpr int H = (R - 1) / 2;
    C sp[H + 1], sm[H + 1];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      sp[j] = cadd(v[j], v[R - j]);
      sm[j] = csub(v[j], v[R - j]);
    }
    C y0 = v[0];
#pragma unroll
    for (int j = 1; j <= H; ++j) y0 = cadd(y0, sp[j]);
    C out[R];
    out[0] = y0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      C a = v[0];
      C b = cmake<C>((T)0, (T)0);
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const T cc = (T)OddConst<R>::c((j * k) % R);
        const T ss = (T)OddConst<R>::s((j * k) % R);
        a.x += sp[j].x * cc;
        a.y += sp[j].y * cc;
        b.x += sm[j].x * ss;
        b.y += sm[j].y * ss;
      }
      // forward: y_k = a - i b, y_{R-k} = a + i b ; inverse: swapped
      C mib = cmake<C>(b.y, -b.x);  // -i b
      if (INV) {
        out[k] = csub(a, mib);
        out[R - k] = cadd(a, mib);
      } else {
        out[k] = cadd(a, mib);
        out[R - k] = csub(a, mib);
      }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = out[u];
  }
};
template <bool INV, typename C> struct Bfly<3, INV, C> : BflyOdd<3, INV, C> {};
template <bool INV, typename C> struct Bfly<5, INV, C> : BflyOdd<5, INV, C> {};
template <bool INV, typename C> struct Bfly<7, INV, C> : BflyOdd<7, INV, C> {};

// Thread mapping of one stage.  Work items are (c, jj, k): column c < TW,
// position jj < NS inside the current sub-transforms, sub-transform k < K
// (K = L / (NS R)); butterfly j = k NS + jj.  Threads are laid out c fastest,
// then jj, then k, so LDS reads of a stage are contiguous, and each thread's
// items differ by compile-time strides: every address is a per-thread base
// plus a constant, and when TW NS <= NT a thread keeps one jj for all its
// items, so its twiddles are loaded once per stage.
constexpr int largest_divisor_le(int n, int cap) {
  int best = 1;
  for (int d = 1; d <= n && d <= cap; ++d)
    if (n % d == 0) best = d;
  return best;
}

template <int TW, int NS, int K, int NT> struct StageMap {
  static constexpr bool A = TW * NS <= NT;                       // one jj per thread
  static constexpr int KB = A ? largest_divisor_le(K, NT / (TW * NS)) : 1;
  static constexpr int JB = A ? NS : largest_divisor_le(NS, NT / TW);
  static constexpr int TU = A ? TW * NS * KB : TW * JB;          // threads with work
  static constexpr int NJ = A ? 1 : NS / JB;                     // jj values per thread
  static constexpr int NK = A ? K / KB : K;                      // k values per thread
};

template <typename T, int L, int TW, int TWP, int NT, bool INV, int S, int PL>
struct Stage {
  static __device__ __forceinline__ void run(cplx<T>* buf, const cplx<T>* __restrict__ tw) {
    constexpr RadixPlan P = make_plan(L, PL);
    if constexpr (S < P.n) {
      using C = cplx<T>;
      constexpr int R = P.r[S];
      constexpr int NS = plan_prefix(L, S, PL);
      constexpr int LR = L / R;
      constexpr int K = L / (NS * R);
      constexpr int TSTEP = L / (NS * R);
      using Map = StageMap<TW, NS, K, NT>;
      const int tid = threadIdx.x;
      const bool active = tid < Map::TU;
      const int c = tid % TW;
      const int jq = tid / TW;                                   // jj (+ NS kb) or jb
      const int jj0 = Map::A ? (jq % NS) : jq;
      const int kb = Map::A ? (jq / NS) : 0;
      C v[Map::NJ][Map::NK][R];
      if (active) {
#pragma unroll
        for (int a = 0; a < Map::NJ; ++a) {
          const int jj = jj0 + a * Map::JB;
          C w[R];
          if (NS > 1) {
#pragma unroll
            for (int t = 1; t < R; ++t) {
              C x = tw[t * jj * TSTEP];
              w[t] = INV ? cconj(x) : x;
            }
          }
#pragma unroll
          for (int b = 0; b < Map::NK; ++b) {
            const int k = kb + b * Map::KB;
            const int j = k * NS + jj;
#pragma unroll
            for (int t = 0; t < R; ++t) {
              C x = buf[(j + t * LR) * TWP + c];
              if (NS > 1 && t > 0) x = cmul(x, w[t]);
              v[a][b][t] = x;
            }
          }
        }
      }
      __syncthreads();
      if (active) {
#pragma unroll
        for (int a = 0; a < Map::NJ; ++a) {
          const int jj = jj0 + a * Map::JB;
#pragma unroll
          for (int b = 0; b < Map::NK; ++b) {
            const int k = kb + b * Map::KB;
            Bfly<R, INV, C>::run(v[a][b]);
#pragma unroll
            for (int u = 0; u < R; ++u) buf[(k * NS * R + jj + u * NS) * TWP + c] = v[a][b][u];
          }
        }
      }
      __syncthreads();
      Stage<T, L, TW, TWP, NT, INV, S + 1, PL>::run(buf, tw);
    }
  }
};

// In-place length-L FFT of TW columns in LDS.  Must be called by all NT
// threads of the workgroup; begins and ends with the LDS contents valid for
// every thread (the caller synchronises before the call).
template <typename T, int L, int TW, int TWP, int NT, bool INV, int PL = 0>
__device__ __forceinline__ void lds_fft(cplx<T>* buf, const cplx<T>* __restrict__ tw) {
  static_assert(plan_ok(L), "FFT length must factor into 2, 3, 5, 7");
  Stage<T, L, TW, TWP, NT, INV, 0, PL>::run(buf, tw);
}

}  // namespace fwi
