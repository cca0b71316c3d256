// Radix-2/4/8/16 FFT building blocks for gfx950 (device code).
//
// Pencil FFTs of power-of-two length L are done by a team of L/E threads,
// each holding E elements in registers: thread t holds x[t + (L/E) e],
// e = 0..E-1. The transform runs as Stockham autosort stages of radix R <= E
// (each thread does E/R radix-R butterflies per stage, in registers); between
// stages the team exchanges data through LDS. Both the first stage's input
// and the last stage's output sit at the positions t + (L/E) e, so global
// loads and stores are coalesced across the team, and a forward transform
// leaves in registers exactly the elements the inverse transform starts
// from (the per-wave-vector apply is done there, with no exchange).
//
// The DFT sign is a template argument: SIGN = +1 computes
// X_k = sum_n x_n e^{+2 pi i n k / L} (the forward sign of Sec. 4 of the
// paper), SIGN = -1 the inverse sign. Transforms are unnormalised.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qw {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
// Complex products written as one multiply and one FMA per part, so that
// their rounding does not depend on how the compiler contracts them in a
// given kernel: every kernel that runs the same transform steps then gives
// the same bits.
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -(a.x * b.y)));
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }

// cos(2 pi k / 16), k = 0..15, and sin(2 pi k / 16) = cos(2 pi (k - 4) / 16).
__device__ constexpr double kCos16[16] = {
    1.0,
    0.92387953251128675613,
    0.70710678118654752440,
    0.38268343236508977173,
    0.0,
    -0.38268343236508977173,
    -0.70710678118654752440,
    -0.92387953251128675613,
    -1.0,
    -0.92387953251128675613,
    -0.70710678118654752440,
    -0.38268343236508977173,
    0.0,
    0.38268343236508977173,
    0.70710678118654752440,
    0.92387953251128675613};

// d * exp(SIGN * 2 pi i idx / 16) for a compile-time-foldable idx.
template <int SIGN, typename T>
__device__ __forceinline__ cx<T> rot16(cx<T> d, int idx) {
  if (idx == 0) return d;
  if (idx == 8) return mk(-d.x, -d.y);
  if (idx == 4) return SIGN > 0 ? mk(-d.y, d.x) : mk(d.y, -d.x);
  if (idx == 12) return SIGN > 0 ? mk(d.y, -d.x) : mk(-d.y, d.x);
  const T c = (T)kCos16[idx];
  const T s = (T)(SIGN * kCos16[(idx + 12) & 15]);
  return mk(fma(d.x, c, -(d.y * s)), fma(d.x, s, d.y * c));
}

__host__ __device__ constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b)
    if (i & (1 << b)) r |= 1 << (bits - 1 - b);
  return r;
}
__host__ __device__ constexpr int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

// In-register DFT of size R (2, 4, 8 or 16), natural order in and out.
// Decimation in frequency, then a compile-time bit-reversal (register renaming).
template <int R, int SIGN, typename T>
__device__ __forceinline__ void dft_reg(cx<T>* a) {
  static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 16, "radix");
  if constexpr (R > 1) {
#pragma unroll
    for (int span = R / 2; span >= 1; span >>= 1) {
#pragma unroll
      for (int start = 0; start < R; start += 2 * span) {
#pragma unroll
        for (int k = 0; k < span; ++k) {
          const cx<T> x = a[start + k];
          const cx<T> y = a[start + k + span];
          a[start + k] = x + y;
          a[start + k + span] = rot16<SIGN>(x - y, k * (16 / (2 * span)));
        }
      }
    }
    cx<T> t[R];
    constexpr int B = ilog2(R);
#pragma unroll
    for (int i = 0; i < R; ++i) t[i] = a[bitrev(i, B)];
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = t[i];
  }
}

// Twiddle table: tw[j] = exp(-2 pi i j / TWN), generated in FP64 on the host.
constexpr int TWN = 4096;

template <int SIGN, typename T>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* __restrict__ tw, int j) {
  const cx<T> w = tw[j];
  return SIGN > 0 ? mk(w.x, -w.y) : w;
}

// LDS slot of pencil position `pos`. With PAD one slot is skipped after every
// 16, which spreads the stride-R writes of the early stages over the banks.
template <bool PAD>
__device__ __forceinline__ int lds_slot(int pos) {
  return PAD ? pos + (pos >> 4) : pos;
}
template <bool PAD>
__host__ __device__ constexpr int lds_len(int L) {
  return PAD ? L + L / 16 : L;
}

// LDS slot of pencil position `pos` in the multi-component team transform
// with E elements per thread: the low five bits (in 8- or 16-byte words)
// are XORed with bits lg E .. lg E + 4. Every exchange of the transform
// (stage writes base + r NS, reads t + (L/E) e) then touches 32 distinct
// words per 32 lanes, i.e. all LDS banks once, and no padding is needed.
// Bits 5 and up are unchanged and bits lg E .. 4 can be recovered from them,
// so the map is a bijection on [0, L) for every power-of-two L.
template <int E>
__device__ __forceinline__ int lds_swz(int pos) {
  constexpr int lg = E >= 16 ? 4 : (E >= 8 ? 3 : (E >= 4 ? 2 : (E >= 2 ? 1 : 0)));
  return pos ^ ((pos >> lg) & 31);
}

// One Stockham stage (and, recursively, the rest). NS = product of the radices
// already done. LDS addressing: element at pencil position `pos` lives at
// lds[lds_slot<PAD>(pos) * ls] (the caller offsets lds to its pencil).
template <typename T, int L, int E, int SIGN, int NS, bool PAD>
struct Stages {
  static constexpr int REM = L / NS;
  static constexpr int R = REM >= E ? E : REM;
  static constexpr bool LAST = (NS * R == L);
  static constexpr int TT = L / E;
  static constexpr int NB = E / R;

  __device__ __forceinline__ static void run(cx<T> (&v)[E], cx<T>* lds, int ls, int t,
                                             const cx<T>* __restrict__ tw) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + b * TT;
      const int k = j & (NS - 1);
      cx<T> a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = v[b + r * NB];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) a[r] = cmul(a[r], twiddle<SIGN>(tw, r * k * (TWN / (NS * R))));
      }
      dft_reg<R, SIGN>(a);
      if constexpr (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[b + r * NB] = a[r];
      } else {
        const int base = (j / NS) * (NS * R) + k;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lds_slot<PAD>(base + r * NS) * ls] = a[r];
      }
    }
    if constexpr (!LAST) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = lds[lds_slot<PAD>(t + TT * e) * ls];
      __syncthreads();
      Stages<T, L, E, SIGN, NS * R, PAD>::run(v, lds, ls, t, tw);
    }
  }
};

// Full length-L transform of the team's registers (see the file comment).
template <typename T, int L, int E, int SIGN, bool PAD = false>
__device__ __forceinline__ void fft_team(cx<T> (&v)[E], cx<T>* lds, int ls, int t,
                                         const cx<T>* __restrict__ tw) {
  static_assert((L & (L - 1)) == 0 && L >= 1 && L <= TWN, "length");
  static_assert(E <= L && (E & (E - 1)) == 0, "elements per thread");
  Stages<T, L, E, SIGN, 1, PAD>::run(v, lds, ls, t, tw);
}

// Orders a team's LDS writes before its reads of what other lanes wrote, and
// those reads before the next writes. A team of at most 64 threads lies in
// one wavefront, whose LDS operations complete in order, so a wavefront-level
// fence and barrier suffice and the other wavefronts of the workgroup run on
// (a workgroup-wide barrier would stall them at every exchange); larger
// teams take the workgroup barrier.
template <int TT>
__device__ __forceinline__ void team_sync() {
  if constexpr (TT <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// The same transform applied to S pencils in lockstep (the spinor components
// of one lattice row): twiddles and LDS slots are computed once per stage and
// shared, and each exchange is one write/barrier/read/barrier for all S.
// Component c of the team's pencil lives at lds + c * cstride (cstride >= L),
// position pos at slot lds_swz<E>(pos). Teams of fewer than 32 threads share
// a wave: their regions should be S * L + L / E elements apart, which puts
// the teams of one wave on disjoint banks.
template <typename T, int L, int E, int SIGN, int NS, int S>
struct StagesMulti {
  static constexpr int REM = L / NS;
  static constexpr int R = REM >= E ? E : REM;
  static constexpr bool LAST = (NS * R == L);
  static constexpr int TT = L / E;
  static constexpr int NB = E / R;

  __device__ __forceinline__ static void run(cx<T> (&v)[S][E], cx<T>* lds, int cstride, int t,
                                             const cx<T>* __restrict__ tw) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + b * TT;
      const int k = j & (NS - 1);
      cx<T> w[R];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) w[r] = twiddle<SIGN>(tw, r * k * (TWN / (NS * R)));
      }
      const int base = (j / NS) * (NS * R) + k;
#pragma unroll
      for (int c = 0; c < S; ++c) {
        cx<T> a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = v[c][b + r * NB];
        if constexpr (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) a[r] = cmul(a[r], w[r]);
        }
        dft_reg<R, SIGN>(a);
        if constexpr (LAST) {
#pragma unroll
          for (int r = 0; r < R; ++r) v[c][b + r * NB] = a[r];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) lds[c * cstride + lds_swz<E>(base + r * NS)] = a[r];
        }
      }
    }
    if constexpr (!LAST) {
      team_sync<TT>();
#pragma unroll
      for (int c = 0; c < S; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) v[c][e] = lds[c * cstride + lds_swz<E>(t + TT * e)];
      team_sync<TT>();
      StagesMulti<T, L, E, SIGN, NS * R, S>::run(v, lds, cstride, t, tw);
    }
  }
};

template <typename T, int L, int E, int SIGN, int S>
__device__ __forceinline__ void fft_team_multi(cx<T> (&v)[S][E], cx<T>* lds, int cstride, int t,
                                               const cx<T>* __restrict__ tw) {
  static_assert((L & (L - 1)) == 0 && L >= 1 && L <= TWN, "length");
  StagesMulti<T, L, E, SIGN, 1, S>::run(v, lds, cstride, t, tw);
}

// Twiddles of a team transform held in registers. The twiddles a thread
// applies depend only on its position t in the team and on the stage, not
// on the pencil or on the direction (the inverse takes their conjugates), so
// a thread that transforms many pencils, forward and back, loads them once.
// Entries: for every stage after the first, NB groups of R - 1 table
// values, in the order the stages consume them.
template <int L, int E>
__host__ __device__ constexpr int team_twiddle_count() {
  int n = 0;
  for (int NS = 1; NS < L;) {
    const int REM = L / NS;
    const int R = REM >= E ? E : REM;
    if (NS > 1) n += (E / R) * (R - 1);
    NS *= R;
  }
  return n;
}

template <typename T, int L, int E, int NS, int OFF>
__device__ __forceinline__ void load_team_twiddles_from(cx<T>* w, int t,
                                                        const cx<T>* __restrict__ tw) {
  if constexpr (NS < L) {
    constexpr int REM = L / NS;
    constexpr int R = REM >= E ? E : REM;
    constexpr int NB = E / R;
    constexpr int TT = L / E;
    if constexpr (NS > 1) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int k = (t + b * TT) & (NS - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) w[OFF + b * (R - 1) + r - 1] = tw[r * k * (TWN / (NS * R))];
      }
      load_team_twiddles_from<T, L, E, NS * R, OFF + NB * (R - 1)>(w, t, tw);
    } else {
      load_team_twiddles_from<T, L, E, NS * R, OFF>(w, t, tw);
    }
  }
}

template <typename T, int L, int E>
__device__ __forceinline__ void load_team_twiddles(cx<T>* w, int t, const cx<T>* __restrict__ tw) {
  load_team_twiddles_from<T, L, E, 1, 0>(w, t, tw);
}

// StagesMulti with the twiddles from a register cache (load_team_twiddles).
template <typename T, int L, int E, int SIGN, int NS, int S, int OFF>
struct StagesMultiC {
  static constexpr int REM = L / NS;
  static constexpr int R = REM >= E ? E : REM;
  static constexpr bool LAST = (NS * R == L);
  static constexpr int TT = L / E;
  static constexpr int NB = E / R;

  __device__ __forceinline__ static void run(cx<T> (&v)[S][E], cx<T>* lds, int cstride, int t,
                                             const cx<T>* wc) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t + b * TT;
      const int k = j & (NS - 1);
      cx<T> w[R];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> x = wc[OFF + b * (R - 1) + r - 1];
          w[r] = SIGN > 0 ? mk(x.x, -x.y) : x;
        }
      }
      const int base = (j / NS) * (NS * R) + k;
#pragma unroll
      for (int c = 0; c < S; ++c) {
        cx<T> a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = v[c][b + r * NB];
        if constexpr (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) a[r] = cmul(a[r], w[r]);
        }
        dft_reg<R, SIGN>(a);
        if constexpr (LAST) {
#pragma unroll
          for (int r = 0; r < R; ++r) v[c][b + r * NB] = a[r];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) lds[c * cstride + lds_swz<E>(base + r * NS)] = a[r];
        }
      }
    }
    if constexpr (!LAST) {
      team_sync<TT>();
#pragma unroll
      for (int c = 0; c < S; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) v[c][e] = lds[c * cstride + lds_swz<E>(t + TT * e)];
      team_sync<TT>();
      StagesMultiC<T, L, E, SIGN, NS * R, S, (NS > 1 ? OFF + NB * (R - 1) : OFF)>::run(
          v, lds, cstride, t, wc);
    }
  }
};

template <typename T, int L, int E, int SIGN, int S>
__device__ __forceinline__ void fft_team_multi_c(cx<T> (&v)[S][E], cx<T>* lds, int cstride, int t,
                                                 const cx<T>* wc) {
  static_assert((L & (L - 1)) == 0 && L >= 1 && L <= TWN, "length");
  StagesMultiC<T, L, E, SIGN, 1, S, 0>::run(v, lds, cstride, t, wc);
}

}  // namespace qw
