// FFT passes along a strided lattice axis, and the transpose used by the 1D
// four-step transform when a natural-order spectrum is asked for.
//
// Data is viewed as [O][L][I]: the transform runs along the middle axis of
// length L (stride I elements) for every (o, i). A workgroup takes P
// consecutive columns i0..i0+P-1 of one o, so each of its global loads and
// stores touches P contiguous elements (P * 8 or 16 bytes, at least one
// 128-byte line), and keeps the P pencils in registers (E per thread) with
// LDS for the exchanges between radix stages. The column index is the
// fastest-varying thread index, so LDS is addressed [pos][column]: the lanes
// of a wave touch consecutive words.
#include <algorithm>
#include <atomic>

#include "qw_internal.h"

namespace qw {

// Outer index o of a launch covers `ocount` consecutive planes o0.. of each
// of several components, components `ostride` elements apart (a slab of the
// lattice); a whole-field launch has ocount = O, o0 = 0. hints: kNtStore,
// kNtLoad bits (non-temporal stores of the results, loads of the input).
struct OuterMap {
  int64_t ocount, o0, ostride;
  int hints;
};

// Workgroup b runs on XCD b % 8 (each XCD has its own L2 and translation
// caches). For complex128 the work is numbered so that each XCD takes a
// contiguous eighth of it (for an n1 pass, a contiguous range of columns of
// every row it reads): 256^3 evolution 2.28 -> 2.23 ms, its n2 passes 0.42 ->
// 0.38 ms. For complex64 the natural order is kept: there the same numbering
// made the n1 forward pass 0.221 -> 0.252 ms and the evolution 1.05 -> 1.09 ms.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t n, bool on) {
  return (on && (n & 7) == 0) ? (b & 7) * (n >> 3) + (b >> 3) : b;
}

template <typename T, int L, int E, int SIGN>
__global__ __launch_bounds__(1024) void k_fft_strided(cx<T>* __restrict__ out,
                                                      const cx<T>* __restrict__ in, int64_t I,
                                                      int lgP, int64_t nblk_i, OuterMap om,
                                                      const cx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int TT = L / E;
  const int P = 1 << lgP;
  const int tid = threadIdx.x;
  const int p = tid & (P - 1);
  const int t = tid >> lgP;
  const int64_t blk = xcd_order(blockIdx.x, gridDim.x, sizeof(T) == 8);
  const int64_t o = blk / nblk_i;
  const int64_t i0 = (blk - o * nblk_i) << lgP;
  const int64_t comp = o / om.ocount;
  const int64_t plane = om.o0 + (o - comp * om.ocount);
  const int64_t base = comp * om.ostride + plane * (int64_t)L * I + i0 + p;
  cx<T> v[E];
  if (om.hints & kNtLoad) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = load_nt(&in[base + (int64_t)(t + TT * e) * I]);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = in[base + (int64_t)(t + TT * e) * I];
  }
  fft_team<T, L, E, SIGN>(v, lds + p, P, t, tw);
  if (om.hints & kNtStore) {
#pragma unroll
    for (int e = 0; e < E; ++e) store_nt(&out[base + (int64_t)(t + TT * e) * I], v[e]);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) out[base + (int64_t)(t + TT * e) * I] = v[e];
  }
}

// Strided passes with their loads staged through LDS by the global-to-LDS
// loads of gfx950 (16 bytes per lane), double-buffered: a workgroup of 512
// threads takes kStagedTiles tiles in turn, and the next tile's loads are in
// flight while the current one is transformed and stored, without holding
// registers. The tiles and their arithmetic are those of the register
// kernel at the same length and precision (COLS columns per tile, E
// elements per thread: thread (p, t), p < COLS, holds rows t + TT e of
// column p, TT = L / E), so both give the same bits.
//
// Each wave stages exactly the rows its own threads read: a wave holds
// TPW = 64 / COLS values of t and RPW = TPW E rows, and slot
// (t / TPW) RPW + TPW e + t % TPW of the buffer holds row t + TT e, so a
// wave waits for its own loads only.
//
// Tiles per workgroup, measured on the n1 inverse pass at 256^3 complex64
// (8192 tiles): 8 tiles 0.197 ms (1024 workgroups, four per CU in turn), 4
// tiles 0.207, 2 tiles 0.219, 1 tile 0.243, against 0.213 for the register
// kernel; 6 and 12 (workgroup counts not a multiple of the 256 CUs) 0.227
// and 0.217. Launches of fewer than kStagedMinTiles tiles (four workgroups
// of eight tiles per CU) keep the register kernel.
constexpr int kStagedTiles = 8;
constexpr int64_t kStagedMinTiles = 8192;

// Workgroup barrier that orders LDS accesses only: this wave's LDS
// operations complete, then all waves meet. Unlike __syncthreads it does not
// wait for the vector memory counter, so loads into LDS issued earlier stay
// in flight.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// This wave's vector memory operations (its loads into LDS among them)
// complete. Written out: the compiler does not count loads into LDS issued
// in an earlier iteration of a loop as outstanding at their use.
__device__ __forceinline__ void vm_drain() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

typedef float qw_f2 __attribute__((ext_vector_type(2)));
typedef float qw_f4 __attribute__((ext_vector_type(4)));
typedef double qw_d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ qw_f2 f2(cx<float> z) { return qw_f2{z.x, z.y}; }
__device__ __forceinline__ qw_d2 d2(cx<double> z) { return qw_d2{z.x, z.y}; }

template <typename T>
__device__ __forceinline__ unsigned lds_addr(const T* p) {
  typedef __attribute__((address_space(3))) const T* lds_ptr;
  return (unsigned)(size_t)(lds_ptr)p;
}

// The exchanges of the staged transforms are written out with their waits
// (compiled LDS accesses would also wait for the next tile's loads into the
// other buffer, which the compiler cannot tell apart from the one being
// transformed), and their twiddles sit in registers (any global load issued
// after the next tile's loads would wait for them too).

// y[e] = the 8-byte value at LDS bytes a + 4096 e (e = 0..15), then the
// workgroup barrier.
__device__ __forceinline__ void lds_read16_st64(unsigned a, cx<float> (&y)[16]) {
  qw_f4 q0, q1, q2, q3, q4, q5, q6, q7;
  asm volatile(
      "ds_read2st64_b64 %0, %8 offset0:0 offset1:8\n\t"
      "ds_read2st64_b64 %1, %8 offset0:16 offset1:24\n\t"
      "ds_read2st64_b64 %2, %8 offset0:32 offset1:40\n\t"
      "ds_read2st64_b64 %3, %8 offset0:48 offset1:56\n\t"
      "ds_read2st64_b64 %4, %8 offset0:64 offset1:72\n\t"
      "ds_read2st64_b64 %5, %8 offset0:80 offset1:88\n\t"
      "ds_read2st64_b64 %6, %8 offset0:96 offset1:104\n\t"
      "ds_read2st64_b64 %7, %8 offset0:112 offset1:120\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      "s_barrier"
      : "=&v"(q0), "=&v"(q1), "=&v"(q2), "=&v"(q3), "=&v"(q4), "=&v"(q5), "=&v"(q6), "=&v"(q7)
      : "v"(a)
      : "memory");
  const qw_f4 q[8] = {q0, q1, q2, q3, q4, q5, q6, q7};
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    y[2 * i] = mk(q[i].x, q[i].y);
    y[2 * i + 1] = mk(q[i].z, q[i].w);
  }
}

// The 8-byte values y[r] to LDS bytes a + 128 r (r = 0..15), in the 8-byte
// units of ds_write2_b64, then the workgroup barrier.
__device__ __forceinline__ void lds_write16_b64_s128(unsigned a, const cx<float> (&y)[16]) {
  asm volatile(
      "ds_write2_b64 %0, %1, %2 offset0:0 offset1:16\n\t"
      "ds_write2_b64 %0, %3, %4 offset0:32 offset1:48\n\t"
      "ds_write2_b64 %0, %5, %6 offset0:64 offset1:80\n\t"
      "ds_write2_b64 %0, %7, %8 offset0:96 offset1:112\n\t"
      "ds_write2_b64 %0, %9, %10 offset0:128 offset1:144\n\t"
      "ds_write2_b64 %0, %11, %12 offset0:160 offset1:176\n\t"
      "ds_write2_b64 %0, %13, %14 offset0:192 offset1:208\n\t"
      "ds_write2_b64 %0, %15, %16 offset0:224 offset1:240\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      "s_barrier" ::"v"(a),
      "v"(f2(y[0])), "v"(f2(y[1])), "v"(f2(y[2])), "v"(f2(y[3])), "v"(f2(y[4])), "v"(f2(y[5])),
      "v"(f2(y[6])), "v"(f2(y[7])), "v"(f2(y[8])), "v"(f2(y[9])), "v"(f2(y[10])), "v"(f2(y[11])),
      "v"(f2(y[12])), "v"(f2(y[13])), "v"(f2(y[14])), "v"(f2(y[15]))
      : "memory");
}

// The same at a + 256 r (r < 8) and a + 2048 + 256 (r - 8).
__device__ __forceinline__ void lds_write16_b64_s256(unsigned a, const cx<float> (&y)[16]) {
  asm volatile(
      "ds_write2_b64 %0, %2, %3 offset0:0 offset1:32\n\t"
      "ds_write2_b64 %0, %4, %5 offset0:64 offset1:96\n\t"
      "ds_write2_b64 %0, %6, %7 offset0:128 offset1:160\n\t"
      "ds_write2_b64 %0, %8, %9 offset0:192 offset1:224\n\t"
      "ds_write2_b64 %1, %10, %11 offset0:0 offset1:32\n\t"
      "ds_write2_b64 %1, %12, %13 offset0:64 offset1:96\n\t"
      "ds_write2_b64 %1, %14, %15 offset0:128 offset1:160\n\t"
      "ds_write2_b64 %1, %16, %17 offset0:192 offset1:224\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      "s_barrier" ::"v"(a),
      "v"(a + 2048u), "v"(f2(y[0])), "v"(f2(y[1])), "v"(f2(y[2])), "v"(f2(y[3])), "v"(f2(y[4])),
      "v"(f2(y[5])), "v"(f2(y[6])), "v"(f2(y[7])), "v"(f2(y[8])), "v"(f2(y[9])), "v"(f2(y[10])),
      "v"(f2(y[11])), "v"(f2(y[12])), "v"(f2(y[13])), "v"(f2(y[14])), "v"(f2(y[15]))
      : "memory");
}

// The same at a + 2048 r (r = 0..15), in the 512-byte units of
// ds_write2st64_b64.
__device__ __forceinline__ void lds_write16_st64_s2048(unsigned a, const cx<float> (&y)[16]) {
  asm volatile(
      "ds_write2st64_b64 %0, %1, %2 offset0:0 offset1:4\n\t"
      "ds_write2st64_b64 %0, %3, %4 offset0:8 offset1:12\n\t"
      "ds_write2st64_b64 %0, %5, %6 offset0:16 offset1:20\n\t"
      "ds_write2st64_b64 %0, %7, %8 offset0:24 offset1:28\n\t"
      "ds_write2st64_b64 %0, %9, %10 offset0:32 offset1:36\n\t"
      "ds_write2st64_b64 %0, %11, %12 offset0:40 offset1:44\n\t"
      "ds_write2st64_b64 %0, %13, %14 offset0:48 offset1:52\n\t"
      "ds_write2st64_b64 %0, %15, %16 offset0:56 offset1:60\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      "s_barrier" ::"v"(a),
      "v"(f2(y[0])), "v"(f2(y[1])), "v"(f2(y[2])), "v"(f2(y[3])), "v"(f2(y[4])), "v"(f2(y[5])),
      "v"(f2(y[6])), "v"(f2(y[7])), "v"(f2(y[8])), "v"(f2(y[9])), "v"(f2(y[10])), "v"(f2(y[11])),
      "v"(f2(y[12])), "v"(f2(y[13])), "v"(f2(y[14])), "v"(f2(y[15]))
      : "memory");
}

// Eight 16-byte values to LDS bytes a + OFF k (k = 0..7), then the
// workgroup barrier.
template <int OFF>
__device__ __forceinline__ void lds_write8_b128(unsigned a, const cx<double> (&y)[8]) {
  asm volatile(
      "ds_write_b128 %0, %1\n\t"
      "ds_write_b128 %0, %2 offset:%c9\n\t"
      "ds_write_b128 %0, %3 offset:%c10\n\t"
      "ds_write_b128 %0, %4 offset:%c11\n\t"
      "ds_write_b128 %0, %5 offset:%c12\n\t"
      "ds_write_b128 %0, %6 offset:%c13\n\t"
      "ds_write_b128 %0, %7 offset:%c14\n\t"
      "ds_write_b128 %0, %8 offset:%c15\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      "s_barrier" ::"v"(a),
      "v"(d2(y[0])), "v"(d2(y[1])), "v"(d2(y[2])), "v"(d2(y[3])), "v"(d2(y[4])), "v"(d2(y[5])),
      "v"(d2(y[6])), "v"(d2(y[7])), "i"(OFF), "i"(2 * OFF), "i"(3 * OFF), "i"(4 * OFF),
      "i"(5 * OFF), "i"(6 * OFF), "i"(7 * OFF)
      : "memory");
}

// y[k] = the 16-byte value at LDS bytes a + 8192 k (k = 0..7), then the
// workgroup barrier.
__device__ __forceinline__ void lds_read8_b128(unsigned a, cx<double> (&y)[8]) {
  qw_d2 q0, q1, q2, q3, q4, q5, q6, q7;
  asm volatile(
      "ds_read_b128 %0, %8\n\t"
      "ds_read_b128 %1, %8 offset:8192\n\t"
      "ds_read_b128 %2, %8 offset:16384\n\t"
      "ds_read_b128 %3, %8 offset:24576\n\t"
      "ds_read_b128 %4, %8 offset:32768\n\t"
      "ds_read_b128 %5, %8 offset:40960\n\t"
      "ds_read_b128 %6, %8 offset:49152\n\t"
      "ds_read_b128 %7, %8 offset:57344\n\t"
      "s_waitcnt lgkmcnt(0)\n\t"
      "s_barrier"
      : "=&v"(q0), "=&v"(q1), "=&v"(q2), "=&v"(q3), "=&v"(q4), "=&v"(q5), "=&v"(q6), "=&v"(q7)
      : "v"(a)
      : "memory");
  const qw_d2 q[8] = {q0, q1, q2, q3, q4, q5, q6, q7};
#pragma unroll
  for (int k = 0; k < 8; ++k) y[k] = mk(q[k].x, q[k].y);
}

// The staged shapes: each gives COLS and E (the register kernel's), whether
// its workgroups go in XCD order (measured per shape: at 256^3 complex128
// the staged n1 inverse pass gained nothing without it; at 512^3, either
// precision, it was slower with it), its twiddles and its transform.
// fft(v, X, t, W):
// the register kernel's Stockham stages for thread t's values v, with the
// element at (position pos, this thread's column) at LDS bytes
// X + pos * COLS * sizeof(cx<T>).
template <typename T, int L>
struct Staged;

// Length 256, complex64: radix 16, 16.
template <>
struct Staged<float, 256> {
  static constexpr int COLS = 32, E = 16;
  static constexpr bool XCD = false;
  template <int SIGN>
  struct Tw {
    cx<float> w[16];
    __device__ __forceinline__ void load(const cx<float>* __restrict__ tw, int t) {
#pragma unroll
      for (int r = 1; r < 16; ++r) w[r] = twiddle<SIGN>(tw, r * t * (TWN / 256));
    }
  };
  template <int SIGN>
  __device__ __forceinline__ static void fft(cx<float> (&v)[16], unsigned X, int t,
                                             const Tw<SIGN>& W) {
    dft_reg<16, SIGN>(v);
    lds_write16_b64_s256(X + 4096u * t, v);  // positions 16 t + r
    lds_read16_st64(X + 256u * t, v);        // positions t + 16 e
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], W.w[r]);
    dft_reg<16, SIGN>(v);
  }
};

// Length 512, complex64: radix 16, 16, 2.
template <>
struct Staged<float, 512> {
  static constexpr int COLS = 16, E = 16;
  static constexpr bool XCD = false;
  template <int SIGN>
  struct Tw {
    cx<float> w2[16], w3[8];  // stage 2 (k = t & 15), stage 3 (k = t + 32 b)
    __device__ __forceinline__ void load(const cx<float>* __restrict__ tw, int t) {
#pragma unroll
      for (int r = 1; r < 16; ++r) w2[r] = twiddle<SIGN>(tw, r * (t & 15) * (TWN / 256));
#pragma unroll
      for (int b = 0; b < 8; ++b) w3[b] = twiddle<SIGN>(tw, (t + 32 * b) * (TWN / 512));
    }
  };
  template <int SIGN>
  __device__ __forceinline__ static void fft(cx<float> (&v)[16], unsigned X, int t,
                                             const Tw<SIGN>& W) {
    dft_reg<16, SIGN>(v);
    lds_write16_b64_s128(X + 2048u * t, v);  // positions 16 t + r
    lds_read16_st64(X + 128u * t, v);        // positions t + 32 e
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], W.w2[r]);
    dft_reg<16, SIGN>(v);
    // positions (t >> 4) 256 + (t & 15) + 16 r
    lds_write16_st64_s2048(X + 128u * ((t >> 4) * 256 + (t & 15)), v);
    lds_read16_st64(X + 128u * t, v);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      cx<float> a[2] = {v[b], cmul(v[b + 8], W.w3[b])};
      dft_reg<2, SIGN>(a);
      v[b] = a[0];
      v[b + 8] = a[1];
    }
  }
};

// Length 256, complex128: radix 8, 8, 4.
template <>
struct Staged<double, 256> {
  static constexpr int COLS = 16, E = 8;
  static constexpr bool XCD = true;
  template <int SIGN>
  struct Tw {
    cx<double> w2[8], w3[2][4];  // stage 2 (k = t & 7), stage 3 (k = t + 32 b)
    __device__ __forceinline__ void load(const cx<double>* __restrict__ tw, int t) {
#pragma unroll
      for (int r = 1; r < 8; ++r) w2[r] = twiddle<SIGN>(tw, r * (t & 7) * (TWN / 64));
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 1; r < 4; ++r)
          w3[b][r] = twiddle<SIGN>(tw, r * ((t + 32 * b) & 63) * (TWN / 256));
    }
  };
  template <int SIGN>
  __device__ __forceinline__ static void fft(cx<double> (&v)[8], unsigned X, int t,
                                             const Tw<SIGN>& W) {
    dft_reg<8, SIGN>(v);
    lds_write8_b128<256>(X + 2048u * t, v);  // positions 8 t + r
    lds_read8_b128(X + 256u * t, v);         // positions t + 32 e
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], W.w2[r]);
    dft_reg<8, SIGN>(v);
    // positions (t >> 3) 64 + (t & 7) + 8 r
    lds_write8_b128<2048>(X + 256u * ((t >> 3) * 64 + (t & 7)), v);
    lds_read8_b128(X + 256u * t, v);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cx<double> a[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = v[b + 2 * r];
#pragma unroll
      for (int r = 1; r < 4; ++r) a[r] = cmul(a[r], W.w3[b][r]);
      dft_reg<4, SIGN>(a);
#pragma unroll
      for (int r = 0; r < 4; ++r) v[b + 2 * r] = a[r];
    }
  }
};

// Length 512, complex128: radix 8, 8, 8.
template <>
struct Staged<double, 512> {
  static constexpr int COLS = 8, E = 8;
  static constexpr bool XCD = false;
  template <int SIGN>
  struct Tw {
    cx<double> w2[8], w3[8];  // stage 2 (k = t & 7), stage 3 (k = t)
    __device__ __forceinline__ void load(const cx<double>* __restrict__ tw, int t) {
#pragma unroll
      for (int r = 1; r < 8; ++r) {
        w2[r] = twiddle<SIGN>(tw, r * (t & 7) * (TWN / 64));
        w3[r] = twiddle<SIGN>(tw, r * t * (TWN / 512));
      }
    }
  };
  template <int SIGN>
  __device__ __forceinline__ static void fft(cx<double> (&v)[8], unsigned X, int t,
                                             const Tw<SIGN>& W) {
    dft_reg<8, SIGN>(v);
    lds_write8_b128<128>(X + 1024u * t, v);  // positions 8 t + r
    lds_read8_b128(X + 128u * t, v);         // positions t + 64 e
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], W.w2[r]);
    dft_reg<8, SIGN>(v);
    // positions (t >> 3) 64 + (t & 7) + 8 r
    lds_write8_b128<1024>(X + 128u * ((t >> 3) * 64 + (t & 7)), v);
    lds_read8_b128(X + 128u * t, v);
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], W.w3[r]);
    dft_reg<8, SIGN>(v);
  }
};

// One tile (L rows of COLS columns from `tile`, row stride I) into buf:
// each instruction loads RPI whole rows, slots RPI j .. RPI j + RPI - 1 of
// this wave.
// Cache policy of the global-to-LDS loads: 0, or kAuxNt (the nt bit of
// gfx950's cache-policy field: the input's lines are not kept in the caches).
constexpr int kAuxNt = 2;

template <typename T, int L, int AUX = 0>
struct StagedTile {
  __device__ __forceinline__ static void load(cx<T>* __restrict__ buf,
                                              const cx<T>* __restrict__ in, int64_t tile,
                                              int64_t I, int tid) {
    using S = Staged<T, L>;
    constexpr int TT = L / S::E, TPW = 64 / S::COLS, RPW = TPW * S::E;
    constexpr int EPL = 16 / (int)sizeof(cx<T>);  // elements per lane
    constexpr int LPR = S::COLS / EPL;             // lanes per row
    constexpr int RPI = 64 / LPR;                  // rows per instruction
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
#pragma unroll
    for (int j = 0; j < RPW / RPI; ++j) {
      const int q = RPI * j + l / LPR;
      const int64_t r = TPW * w + q % TPW + TT * (q / TPW);
      __builtin_amdgcn_global_load_lds(in + tile + r * I + EPL * (l % LPR),
                                       buf + (w * RPW + RPI * j) * S::COLS, 16, 0, AUX);
    }
  }
};

// The tile loop: tiles blockIdx.x * kStagedTiles + k (workgroups in XCD
// order where the shape says so) of the nblk (nblk_i per outer index), each
// transformed and handed to epi(v, tile, first element of the tile) with the
// thread's E values, rows t + TT e of column p. buf: 2 L COLS elements of
// LDS.
template <typename T, int L, int SIGN, int AUX = 0, typename Epi>
__device__ __forceinline__ void staged_loop(cx<T>* __restrict__ buf,
                                            const cx<T>* __restrict__ in, int64_t I,
                                            int64_t nblk_i, int64_t nblk, const OuterMap& om,
                                            const cx<T>* __restrict__ tw, Epi epi) {
  using S = Staged<T, L>;
  constexpr int COLS = S::COLS, E = S::E, TPW = 64 / COLS, RPW = TPW * E;
  const int tid = threadIdx.x;
  const int p = tid % COLS, t = tid / COLS;
  typename S::template Tw<SIGN> W;
  W.load(tw, t);
  auto tile_base = [&](int64_t blk) -> int64_t {
    const int64_t o = blk / nblk_i;
    const int64_t i0 = (blk - o * nblk_i) * COLS;
    const int64_t comp = o / om.ocount;
    const int64_t plane = om.o0 + (o - comp * om.ocount);
    return comp * om.ostride + plane * L * I + i0;
  };
  const int64_t first = xcd_order(blockIdx.x, gridDim.x, S::XCD) * kStagedTiles;
  if (first >= nblk) return;
  const int n = nblk - first < kStagedTiles ? (int)(nblk - first) : kStagedTiles;
  int64_t cur = tile_base(first);
  StagedTile<T, L, AUX>::load(buf, in, cur, I, tid);
  const int s0 = (t / TPW) * RPW + t % TPW;
  for (int k = 0; k < n; ++k) {
    cx<T>* X = buf + (k & 1) * (L * COLS);
    cx<T>* Y = buf + ((k + 1) & 1) * (L * COLS);
    vm_drain();
    cx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = X[(s0 + TPW * e) * COLS + p];
    // every wave has its rows before the exchange writes X, and the last
    // reads of Y (the previous tile's exchange and epilogue) are done
    lds_barrier();
    int64_t nxt = 0;
    if (k + 1 < n) {
      nxt = tile_base(first + k + 1);
      StagedTile<T, L, AUX>::load(Y, in, nxt, I, tid);
    }
    S::template fft<SIGN>(v, lds_addr(X + p), t, W);
    epi(v, first + k, cur);
    cur = nxt;
  }
}

// NT: non-temporal stores (a template parameter: as a branch inside the
// loop the two store forms were merged into plain stores).
template <typename T, int L, int SIGN, bool NT, int AUX = 0>
__global__ __launch_bounds__(512) void k_fft_strided_staged(cx<T>* __restrict__ out,
                                                            const cx<T>* __restrict__ in,
                                                            int64_t I, int64_t nblk_i,
                                                            int64_t nblk, OuterMap om,
                                                            const cx<T>* __restrict__ tw) {
  using S = Staged<T, L>;
  constexpr int COLS = S::COLS, E = S::E, TT = L / E;
  __shared__ __align__(16) cx<T> buf[2 * L * COLS];
  const int p = threadIdx.x % COLS, t = threadIdx.x / COLS;
  staged_loop<T, L, SIGN, AUX>(buf, in, I, nblk_i, nblk, om, tw,
                          [&](const cx<T>(&v)[E], int64_t, int64_t base) {
                            const int64_t b = base + p;
#pragma unroll
                            for (int e = 0; e < E; ++e) {
                              if constexpr (NT)
                                store_nt(&out[b + (int64_t)(t + TT * e) * I], v[e]);
                              else
                                out[b + (int64_t)(t + TT * e) * I] = v[e];
                            }
                          });
}

// The staged kernels take a pass when they apply, unless switched off
// (qw_set_fft_kernel): lengths 256 and 512, whole tiles, at least
// kStagedMinTiles of them, and
// * complex64, length 256: the inverse direction. The forward passes
//   measured slower staged (0.246 and 0.210 ms against 0.226 and 0.190 at
//   256^3; in XCD order 0.240 and 0.183, but the fused pass after them then
//   took 0.245 against 0.238 ms; the n1 pass with its cache hints 0.223
//   against 0.205 ms for the register kernel with the same hints), where the
//   inverse ones went 0.187 -> 0.174 ms and 0.213 -> 0.197 ms (in XCD order
//   0.190 and 0.195).
// * complex64, length 512: both directions. At 512^3 the n1 forward pass
//   2.82 -> 2.17 ms, n2 forward 1.77 -> 1.63, n2 inverse 1.83 -> 1.61, n1
//   inverse 2.37 -> 2.08 (the jump 10.8 -> 9.5 ms); in XCD order slightly
//   slower (9.66 ms).
// * complex128: rows at least 4096 elements apart, both directions. At
//   256^3 the n1 passes 0.490 -> 0.451 ms and 0.456 -> 0.418 ms (the jump
//   2.26 -> 2.19 ms), where the n2 passes (4 KB apart) measured slower
//   (0.382 -> 0.394 and 0.384 -> 0.392 ms); at 512^3 the n1 passes 4.83 ->
//   4.32 and 4.64 -> 4.32 ms (in XCD order 4.44 and 4.42), where the n2
//   passes (8 KB apart) measured slower (3.05 -> 3.37 ms).
static std::atomic<bool> g_staged{true};

void set_fft_staged(bool on) { g_staged.store(on, std::memory_order_relaxed); }

static bool use_staged(bool dbl, int sign, int64_t L, int64_t O, int64_t I) {
  if (!g_staged.load(std::memory_order_relaxed) || (L != 256 && L != 512)) return false;
  const int cols = dbl ? (L == 256 ? Staged<double, 256>::COLS : Staged<double, 512>::COLS)
                       : (L == 256 ? Staged<float, 256>::COLS : Staged<float, 512>::COLS);
  if (I % cols != 0 || O * (I / cols) < kStagedMinTiles) return false;
  if (dbl) return I >= 4096;
  return L == 512 || sign < 0;
}

// The staged kernel of a direction and store form, loads of cache policy AUX.
template <typename T, int L, int AUX>
static auto staged_kernel(int sign, bool nt) {
  return sign > 0 ? (nt ? k_fft_strided_staged<T, L, 1, true, AUX>
                        : k_fft_strided_staged<T, L, 1, false, AUX>)
                  : (nt ? k_fft_strided_staged<T, L, -1, true, AUX>
                        : k_fft_strided_staged<T, L, -1, false, AUX>);
}

template <typename T, int L>
static hipError_t run_staged(cx<T>* out, const cx<T>* in, int64_t O, int64_t I,
                             const OuterMap& om, const cx<T>* tw, hipStream_t st, int sign) {
  const int64_t nblk_i = I / Staged<T, L>::COLS;
  const int64_t nblk = O * nblk_i;
  const int64_t ng = (nblk + kStagedTiles - 1) / kStagedTiles;
  if (ng > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool nt = om.hints & kNtStore;
  auto kern = (om.hints & kNtLoad) ? staged_kernel<T, L, kAuxNt>(sign, nt)
                                   : staged_kernel<T, L, 0>(sign, nt);
  hipLaunchKernelGGL(kern, dim3((unsigned)ng), dim3(512), 0, st, out, in, I, nblk_i, nblk, om, tw);
  return hipGetLastError();
}

template <typename T>
static hipError_t dispatch_staged(int64_t L, cx<T>* out, const cx<T>* in, int64_t O, int64_t I,
                                  const OuterMap& om, const cx<T>* tw, hipStream_t st, int sign) {
  return L == 256 ? run_staged<T, 256>(out, in, O, I, om, tw, st, sign)
                  : run_staged<T, 512>(out, in, O, I, om, tw, st, sign);
}

// Columns per workgroup of a strided pass: 256 bytes of each row (32
// complex64 or 16 complex128 columns), at least 256 threads; then at most
// 1024 threads, and at most 64 KB of LDS unless rows would drop below 128
// bytes; at most the I columns there are. Measured on the 256^3 complex64
// evolution: 16 columns (128-byte rows) 1.175 ms, 32 columns 1.131 ms,
// 64 columns (128 KB of LDS, one workgroup per CU) 1.160 ms.
// Workgroup size of a strided pass with unlimited columns (the launch
// bound of the fused kernel, so that the compiler may use the registers the
// actual workgroups leave free).
template <typename T, int L>
constexpr int strided_max_threads() {
  constexpr int Emax = sizeof(T) == 8 ? 8 : 16;
  constexpr int E = L < Emax ? L : Emax;
  constexpr int TT = L / E;
  constexpr int row128 = 128 / (int)sizeof(cx<T>);
  int P = 2 * row128;
  while (TT * P < 256) P <<= 1;
  while (TT * P > 1024 && P > 1) P >>= 1;
  while ((size_t)P * L * sizeof(cx<T>) > 65536 && P > row128) P >>= 1;
  return TT * P;
}

template <typename T, int L>
static int strided_cols(int64_t I) {
  constexpr int Emax = sizeof(T) == 8 ? 8 : 16;
  constexpr int E = L < Emax ? L : Emax;
  constexpr int TT = L / E;
  constexpr int row128 = 128 / (int)sizeof(cx<T>);
  int P = 2 * row128;
  while (TT * P < 256) P <<= 1;
  while (TT * P > 1024 && P > 1) P >>= 1;
  while ((size_t)P * L * sizeof(cx<T>) > 65536 && P > row128) P >>= 1;
  if (P > I) P = (int)I;
  return P;
}

template <typename T, int L, int SIGN>
static hipError_t run_strided(cx<T>* out, const cx<T>* in, int64_t O, int64_t I,
                              const OuterMap& om, const cx<T>* tw, hipStream_t st) {
  constexpr int Emax = sizeof(T) == 8 ? 8 : 16;
  constexpr int E = L < Emax ? L : Emax;
  constexpr int TT = L / E;
  int P = strided_cols<T, L>(I);
  if (TT * P > 1024) return hipErrorInvalidValue;
  const int lgP = ilog2(P);
  const size_t lds = (size_t)P * L * sizeof(cx<T>);
  auto kern = k_fft_strided<T, L, E, SIGN>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t nblk_i = I / P;
  const int64_t nblk = O * nblk_i;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(TT * P), lds, st, out, in, I, lgP, nblk_i, om,
                     tw);
  return hipGetLastError();
}

template <typename T, int SIGN>
static hipError_t dispatch_strided(int64_t L, cx<T>* out, const cx<T>* in, int64_t O, int64_t I,
                                   const OuterMap& om, const cx<T>* tw, hipStream_t st) {
  switch (L) {
    case 1:
      return hipErrorInvalidValue;
    case 2: return run_strided<T, 2, SIGN>(out, in, O, I, om, tw, st);
    case 4: return run_strided<T, 4, SIGN>(out, in, O, I, om, tw, st);
    case 8: return run_strided<T, 8, SIGN>(out, in, O, I, om, tw, st);
    case 16: return run_strided<T, 16, SIGN>(out, in, O, I, om, tw, st);
    case 32: return run_strided<T, 32, SIGN>(out, in, O, I, om, tw, st);
    case 64: return run_strided<T, 64, SIGN>(out, in, O, I, om, tw, st);
    case 128: return run_strided<T, 128, SIGN>(out, in, O, I, om, tw, st);
    case 256: return run_strided<T, 256, SIGN>(out, in, O, I, om, tw, st);
    case 512: return run_strided<T, 512, SIGN>(out, in, O, I, om, tw, st);
    case 1024: return run_strided<T, 1024, SIGN>(out, in, O, I, om, tw, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fft_strided_slab(bool dbl, int sign, int64_t L, void* out, const void* in,
                                   int64_t ncomp, int64_t ocount, int64_t o0, int64_t ostride,
                                   int64_t I, const void* tw, hipStream_t st, int hints) {
  const OuterMap om{ocount, o0, ostride, hints};
  const int64_t O = ncomp * ocount;
  if (use_staged(dbl, sign, L, O, I))
    return dbl ? dispatch_staged<double>(L, (cx<double>*)out, (const cx<double>*)in, O, I, om,
                                         (const cx<double>*)tw, st, sign)
               : dispatch_staged<float>(L, (cx<float>*)out, (const cx<float>*)in, O, I, om,
                                        (const cx<float>*)tw, st, sign);
  if (dbl) {
    auto o = (cx<double>*)out;
    auto i = (const cx<double>*)in;
    auto w = (const cx<double>*)tw;
    return sign > 0 ? dispatch_strided<double, 1>(L, o, i, O, I, om, w, st)
                    : dispatch_strided<double, -1>(L, o, i, O, I, om, w, st);
  }
  auto o = (cx<float>*)out;
  auto i = (const cx<float>*)in;
  auto w = (const cx<float>*)tw;
  return sign > 0 ? dispatch_strided<float, 1>(L, o, i, O, I, om, w, st)
                  : dispatch_strided<float, -1>(L, o, i, O, I, om, w, st);
}

hipError_t launch_fft_strided(bool dbl, int sign, int64_t L, void* out, const void* in, int64_t O,
                              int64_t I, const void* tw, hipStream_t st, int hints) {
  if (L == 1) {
    if (out != in)
      return hipMemcpyAsync(out, in, (dbl ? 16 : 8) * O * I, hipMemcpyDeviceToDevice, st);
    return hipSuccess;
  }
  return launch_fft_strided_slab(dbl, sign, L, out, in, 1, O, 0, 0, I, tw, st, hints);
}

// Last inverse pass of an evolution with the Sec. 5.2 reductions fused: the
// transformed values are reduced where they are produced (the field need
// not be read again, nor written at all when only the reductions are
// wanted). Whole fields: outer index o = b * s + component.
//
// The arithmetic of the reductions of one tile of P columns, shared by the
// register and the staged kernel so that both give the same partials:
// (1) over the thread's E values (rows t + TT e of column col): only the
// axis-0 displacement varies along the pass, so three moments in it
// suffice (the other axes are fixed per column);
// Every operation is rounded on its own (no contraction into FMAs), so
// that the register and the staged kernels give the same sums.
template <typename T, int L, int E>
__device__ __forceinline__ void obs_thread_moments(const cx<T> (&v)[E], int t, int64_t I,
                                                   int64_t col, int dim, const AxisImage32& a0,
                                                   double& S0, double& S1, double& S11) {
#pragma clang fp contract(off)
  constexpr int TT = L / E;
  S0 = 0.0;
  S1 = 0.0;
  S11 = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int pos = t + TT * e;
    const double w = min_image32(dim == 1 ? pos * (int)I + (int)col : pos, a0);
    const double x = (double)v[e].x, y = (double)v[e].y;
    const double pr = x * x + y * y;
    const double wp = w * pr;
    S0 += pr;
    S1 += wp;
    S11 += w * wp;
  }
}

// (2) the ten moment fields of column cc from its sums c0, c1, c2 over the
// pass (the other axes' displacements wb, wc fixed per column);
__device__ __forceinline__ void obs_column_disp(int64_t cc, const double (&org)[3],
                                                const ObsFuse& f, double& wb, double& wc) {
  wb = 0.0;
  wc = 0.0;
  if (f.dim == 2) {
    wb = min_image(cc, axis_image(org[1], f.N[1]));
  } else if (f.dim == 3) {
    wb = min_image(cc >> f.lg[2], axis_image(org[1], f.N[1]));
    wc = min_image(cc & (f.N[2] - 1), axis_image(org[2], f.N[2]));
  }
}

__device__ __forceinline__ double obs_field(int k, double c0, double c1, double c2, double wb,
                                            double wc) {
  switch (k) {
    case 0: return c0;
    case 1: return c1;
    case 2: return wb * c0;
    case 3: return wc * c0;
    case 4: return c2;
    case 5: return wb * wb * c0;
    case 6: return wc * wc * c0;
    case 7: return wb * c1;
    case 8: return wc * c1;
    default: return wb * wc * c0;
  }
}

__device__ __forceinline__ void obs_column_fields(double c0, double c1, double c2, int64_t cc,
                                                  const double (&org)[3], const ObsFuse& f,
                                                  double (&acc)[10]) {
  double wb, wc;
  obs_column_disp(cc, org, f, wb, wc);
#pragma unroll
  for (int k = 0; k < 10; ++k) acc[k] = obs_field(k, c0, c1, c2, wb, wc);
}

// (3) over the columns: a shuffle sum over the 64 lanes of a wave (lane 0
// takes the result).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <typename T, int L, int E>
__global__ __launch_bounds__((strided_max_threads<T, L>())) void k_fft_strided_obs(cx<T>* __restrict__ out,
                                                          const cx<T>* __restrict__ in, int64_t I,
                                                          int lgP, int64_t nblk_i, int s,
                                                          ObsFuse f,
                                                          const cx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int TT = L / E;
  const int P = 1 << lgP;
  const int tid = threadIdx.x;
  const int p = tid & (P - 1);
  const int t = tid >> lgP;
  const int64_t blk = xcd_order(blockIdx.x, gridDim.x, sizeof(T) == 8);
  const int64_t o = blk / nblk_i;
  const int64_t col = ((blk - o * nblk_i) << lgP) + p;
  const int64_t base = o * (int64_t)L * I + col;
  cx<T> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = in[base + (int64_t)(t + TT * e) * I];
  fft_team<T, L, E, -1>(v, lds + p, P, t, tw);
  if (f.store) {
#pragma unroll
    for (int e = 0; e < E; ++e) out[base + (int64_t)(t + TT * e) * I] = v[e];
  }
  const int64_t b = o / s;
  double org[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) org[a] = f.origins ? f.origins[3 * b + a] : f.c[a];
  double S0, S1, S11;
  obs_thread_moments<T, L, E>(v, t, I, col, f.dim, axis_image32(axis_image(org[0], f.N[0])), S0,
                              S1, S11);
  // Over the TT threads of each column, through LDS (free once the
  // transform is done; the launch sizes it for 3 doubles per thread).
  const int nth = TT * P;
  double* red = reinterpret_cast<double*>(smem_raw);
  __syncthreads();
  red[tid] = S0;
  red[nth + tid] = S1;
  red[2 * nth + tid] = S11;
  __syncthreads();
  double acc[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) acc[k] = 0.0;
  if (tid < P) {
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
    for (int r = 0; r < TT; ++r) {
      const int i = r * P + tid;
      c0 += red[i];
      c1 += red[nth + i];
      c2 += red[2 * nth + i];
    }
    obs_column_fields(c0, c1, c2, col - p + tid, org, f, acc);
  }
  // Only the waves holding column sums shuffle.
  __shared__ double red2[10][16];
  const int lane = tid & 63, wave = tid >> 6;
  const int nwc = (P + 63) >> 6;
  if (wave < nwc) {
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      const double vv = wave_sum(acc[k]);
      if (lane == 0) red2[k][wave] = vv;
    }
  }
  __syncthreads();
  if (tid < kObsFields) {
    double sum = 0.0;
    if (tid < 10)
      for (int w = 0; w < nwc; ++w) sum += red2[tid][w];
    f.partials[blk * kObsFields + tid] = sum;
  }
}

// The same pass staged through LDS (see k_fft_strided_staged), length 256,
// for calls with one origin (f.origins null): the same tiles and
// arithmetic, so the same field and partial vectors. Its LDS accesses inside
// the tile loop are written out with their waits (compiled ones would also
// wait for the next tile's loads in flight), and the reduction area is LDS
// of its own, which the loop's barriers order against the previous tile's
// readers. The reduction tail would stall the workgroup on one wave, so the
// ten fields are spread over seven waves by the column sum they take: c0:
// {0, 2}, {3, 5}, {6, 9}; c1: {1}, {7}, {8}; c2: {4}; the last wave writes
// the zero fields. The COLS columns sit in lanes 0..COLS-1 of a reducing
// wave and the other lanes hold zeros, so the register kernel's shuffle
// steps over lanes COLS and up add 0.0.

// c = sum over the TT rows r (in that order) of the doubles at LDS bytes
// a + 8 COLS r (COLS = 512 / TT).
template <int TT>
__device__ __forceinline__ double lds_column_sum(unsigned a) {
  static_assert(TT == 16 || TT == 32, "rows of a column");
  constexpr unsigned kHalf = 2048;  // bytes of TT / 2 rows
  double c = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    qw_d2 y0, y1, y2, y3, y4, y5, y6, y7;
    if constexpr (TT == 16) {
      // 256-byte rows: four pairs per half
      asm volatile(
          "ds_read2_b64 %0, %4 offset0:0 offset1:32\n\t"
          "ds_read2_b64 %1, %4 offset0:64 offset1:96\n\t"
          "ds_read2_b64 %2, %4 offset0:128 offset1:160\n\t"
          "ds_read2_b64 %3, %4 offset0:192 offset1:224\n\t"
          "s_waitcnt lgkmcnt(0)"
          : "=&v"(y0), "=&v"(y1), "=&v"(y2), "=&v"(y3)
          : "v"(a + kHalf * h)
          : "memory");
      y4 = y5 = y6 = y7 = qw_d2{0.0, 0.0};
    } else {
      // 128-byte rows: eight pairs per half
      asm volatile(
          "ds_read2_b64 %0, %8 offset0:0 offset1:16\n\t"
          "ds_read2_b64 %1, %8 offset0:32 offset1:48\n\t"
          "ds_read2_b64 %2, %8 offset0:64 offset1:80\n\t"
          "ds_read2_b64 %3, %8 offset0:96 offset1:112\n\t"
          "ds_read2_b64 %4, %8 offset0:128 offset1:144\n\t"
          "ds_read2_b64 %5, %8 offset0:160 offset1:176\n\t"
          "ds_read2_b64 %6, %8 offset0:192 offset1:208\n\t"
          "ds_read2_b64 %7, %8 offset0:224 offset1:240\n\t"
          "s_waitcnt lgkmcnt(0)"
          : "=&v"(y0), "=&v"(y1), "=&v"(y2), "=&v"(y3), "=&v"(y4), "=&v"(y5), "=&v"(y6),
            "=&v"(y7)
          : "v"(a + kHalf * h)
          : "memory");
    }
    const qw_d2 y[8] = {y0, y1, y2, y3, y4, y5, y6, y7};
#pragma unroll
    for (int i = 0; i < TT / 4; ++i) {
      c += y[i].x;
      c += y[i].y;
    }
  }
  return c;
}

// wave_sum for a wave whose lanes COLS..63 hold zeros.
template <int COLS>
__device__ __forceinline__ double wave_sum_cols(double v) {
#pragma unroll
  for (int off = 32; off >= COLS; off >>= 1) v = v + 0.0;
#pragma unroll
  for (int off = COLS / 2; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// NT: the field (when f.store) is written with non-temporal stores.
template <typename T, int AUX = 0, bool NT = false>
__global__ __launch_bounds__(512) void k_fft_strided_obs_staged(cx<T>* __restrict__ out,
                                                                const cx<T>* __restrict__ in,
                                                                int64_t I, int64_t nblk_i,
                                                                int64_t nblk, ObsFuse f,
                                                                const cx<T>* __restrict__ tw) {
  using S = Staged<T, 256>;
  constexpr int COLS = S::COLS, E = S::E, TT = 256 / E;
  __shared__ __align__(16) cx<T> buf[2 * 256 * COLS];
  __shared__ __align__(16) double red[3 * 512];
  const int tid = threadIdx.x;
  const int p = tid % COLS, t = tid / COLS;
  const OuterMap om{nblk / nblk_i, 0, 0, 0};
  const AxisImage32 a0 = axis_image32(axis_image(f.c[0], f.N[0]));
  const double org[3] = {f.c[0], f.c[1], f.c[2]};
  const unsigned ra = lds_addr(red + tid);
  const unsigned rl = lds_addr(red + (tid & 63));  // the column of a reducing lane
  staged_loop<T, 256, -1, AUX>(buf, in, I, nblk_i, nblk, om, tw,
                          [&](const cx<T>(&v)[E], int64_t blk, int64_t base) {
                            if (f.store) {
#pragma unroll
                              for (int e = 0; e < E; ++e) {
                                if constexpr (NT)
                                  store_nt(&out[base + p + (int64_t)(t + TT * e) * I], v[e]);
                                else
                                  out[base + p + (int64_t)(t + TT * e) * I] = v[e];
                              }
                            }
                            const int64_t o = blk / nblk_i;
                            const int64_t col = base - o * 256 * I + p;
                            double S0, S1, S11;
                            obs_thread_moments<T, 256, E>(v, t, I, col, f.dim, a0, S0, S1, S11);
                            // red[tid], red[512 + tid], red[1024 + tid]; then
                            // all threads' moments are there
                            asm volatile(
                                "ds_write_b64 %0, %1\n\t"
                                "ds_write_b64 %0, %2 offset:4096\n\t"
                                "ds_write_b64 %0, %3 offset:8192\n\t"
                                "s_waitcnt lgkmcnt(0)\n\t"
                                "s_barrier" ::"v"(ra),
                                "v"(S0), "v"(S1), "v"(S11)
                                : "memory");
                            const int wave = tid >> 6, lane = tid & 63;
                            if (wave < 7) {
                              const int m = wave < 3 ? 0 : (wave < 6 ? 1 : 2);
                              // the wave's fields as nibbles of one constant (15: none)
                              const int k0 = (0x04871630 >> (4 * wave)) & 15;
                              const int k1r = (0x0FFFF952 >> (4 * wave)) & 15;
                              const int k1 = k1r == 15 ? -1 : k1r;
                              double v0 = 0.0, v1 = 0.0;
                              if (lane < COLS) {
                                const double c = lds_column_sum<TT>(rl + 4096u * m);
                                double wb, wc;
                                obs_column_disp(col - p + lane, org, f, wb, wc);
                                v0 = obs_field(k0, c, c, c, wb, wc);
                                if (k1 >= 0) v1 = obs_field(k1, c, c, c, wb, wc);
                              }
                              v0 = wave_sum_cols<COLS>(v0);
                              if (k1 >= 0) v1 = wave_sum_cols<COLS>(v1);
                              if (lane == 0) {
                                double* dst = f.partials + blk * kObsFields;
                                dst[k0] = 0.0 + v0;
                                if (k1 >= 0) dst[k1] = 0.0 + v1;
                              }
                            } else if (lane == 0) {
                              double* dst = f.partials + blk * kObsFields;
                              for (int k = 10; k < kObsFields; ++k) dst[k] = 0.0;
                            }
                          });
}

template <typename T, int L>
static hipError_t run_strided_obs(cx<T>* out, const cx<T>* in, int s, int B, int64_t I,
                                  const ObsFuse& f, const cx<T>* tw, hipStream_t st, int hints) {
  constexpr int Emax = sizeof(T) == 8 ? 8 : 16;
  constexpr int E = L < Emax ? L : Emax;
  constexpr int TT = L / E;
  const int P = strided_cols<T, L>(I);
  if (TT * P > 1024 || (TT * P) % 64 != 0) return hipErrorInvalidValue;
  const int lgP = ilog2(P);
  const int64_t nblk_i = I / P;
  const int64_t nblk = (int64_t)s * B * nblk_i;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  if constexpr (L == 256) {
    if (!f.origins && use_staged(sizeof(T) == 8, -1, L, (int64_t)s * B, I)) {
      static_assert(TT * Staged<T, 256>::COLS == 512, "staged tiles are the register kernel's");
      const int64_t ng = (nblk + kStagedTiles - 1) / kStagedTiles;
      const bool ntl = hints & kNtLoad, nts = hints & kNtStore;
      auto kern = ntl ? (nts ? k_fft_strided_obs_staged<T, kAuxNt, true>
                             : k_fft_strided_obs_staged<T, kAuxNt, false>)
                      : (nts ? k_fft_strided_obs_staged<T, 0, true>
                             : k_fft_strided_obs_staged<T, 0, false>);
      hipLaunchKernelGGL(kern, dim3((unsigned)ng), dim3(512), 0, st, out, in, I, nblk_i, nblk, f,
                         tw);
      return hipGetLastError();
    }
  }
  // the transform's exchanges, then 3 doubles per thread for the reduction
  const size_t lds = std::max((size_t)P * L * sizeof(cx<T>), (size_t)TT * P * 3 * sizeof(double));
  auto kern = k_fft_strided_obs<T, L, E>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(TT * P), lds, st, out, in, I, lgP, nblk_i, s,
                     f, tw);
  return hipGetLastError();
}

template <typename T>
static int64_t obs_blocks_t(int64_t L, int64_t I) {
  // Longer complex64 (1024) and complex128 (512, 1024) passes would spill
  // registers with the reduction fused; those take a separate reduction.
  if (L > (sizeof(T) == 4 ? 512 : 256)) return 0;
  int P = 0, TT = 0;
  switch (L) {
#define QW_CASE(LL)                                           \
  case LL: {                                                  \
    constexpr int Emax = sizeof(T) == 8 ? 8 : 16;             \
    TT = LL / (LL < Emax ? LL : Emax);                        \
    P = strided_cols<T, LL>(I);                               \
    break;                                                    \
  }
    QW_CASE(2) QW_CASE(4) QW_CASE(8) QW_CASE(16) QW_CASE(32) QW_CASE(64) QW_CASE(128)
    QW_CASE(256) QW_CASE(512) QW_CASE(1024)
#undef QW_CASE
    default: return 0;
  }
  if (TT * P > 1024 || (TT * P) % 64 != 0) return 0;
  return I / P;
}

int64_t strided_obs_blocks(bool dbl, int64_t L, int64_t I) {
  return dbl ? obs_blocks_t<double>(L, I) : obs_blocks_t<float>(L, I);
}

template <typename T>
static hipError_t dispatch_strided_obs(int64_t L, cx<T>* out, const cx<T>* in, int s, int B,
                                       int64_t I, const ObsFuse& f, const cx<T>* tw,
                                       hipStream_t st, int hints) {
  switch (L) {
    case 2: return run_strided_obs<T, 2>(out, in, s, B, I, f, tw, st, hints);
    case 4: return run_strided_obs<T, 4>(out, in, s, B, I, f, tw, st, hints);
    case 8: return run_strided_obs<T, 8>(out, in, s, B, I, f, tw, st, hints);
    case 16: return run_strided_obs<T, 16>(out, in, s, B, I, f, tw, st, hints);
    case 32: return run_strided_obs<T, 32>(out, in, s, B, I, f, tw, st, hints);
    case 64: return run_strided_obs<T, 64>(out, in, s, B, I, f, tw, st, hints);
    case 128: return run_strided_obs<T, 128>(out, in, s, B, I, f, tw, st, hints);
    case 256: return run_strided_obs<T, 256>(out, in, s, B, I, f, tw, st, hints);
    case 512: return run_strided_obs<T, 512>(out, in, s, B, I, f, tw, st, hints);
    case 1024: return run_strided_obs<T, 1024>(out, in, s, B, I, f, tw, st, hints);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fft_strided_obs(bool dbl, int64_t L, void* out, const void* in, int s, int B,
                                  int64_t I, const ObsFuse& f, const void* tw, hipStream_t st,
                                  int hints) {
  if (dbl)
    return dispatch_strided_obs<double>(L, (cx<double>*)out, (const cx<double>*)in, s, B, I, f,
                                        (const cx<double>*)tw, st, hints);
  return dispatch_strided_obs<float>(L, (cx<float>*)out, (const cx<float>*)in, s, B, I, f,
                                     (const cx<float>*)tw, st, hints);
}

// out[p][c][r] = in[p][r][c] for planes p of an R x C matrix (32 x 32 tiles).
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(cx<T>* __restrict__ out,
                                                   const cx<T>* __restrict__ in, int64_t R,
                                                   int64_t C, int64_t tiles_c, int64_t tiles_r) {
  __shared__ cx<T> tile[32][33];
  const int64_t blk = blockIdx.x;
  const int64_t per_plane = tiles_c * tiles_r;
  const int64_t plane = blk / per_plane;
  const int64_t rem = blk - plane * per_plane;
  const int64_t tr = rem / tiles_c;
  const int64_t tc = rem - tr * tiles_c;
  const cx<T>* src = in + plane * R * C;
  cx<T>* dst = out + plane * R * C;
  const int tx = threadIdx.x & 31;
  const int ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t r = tr * 32 + yy, c = tc * 32 + tx;
    if (r < R && c < C) tile[yy][tx] = src[r * C + c];
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t c = tc * 32 + yy, r = tr * 32 + tx;
    if (r < R && c < C) dst[c * R + r] = tile[tx][yy];
  }
}

hipError_t launch_transpose(bool dbl, void* out, const void* in, int64_t planes, int64_t R,
                            int64_t C, hipStream_t st) {
  const int64_t tc = (C + 31) / 32, tr = (R + 31) / 32;
  const int64_t nblk = planes * tc * tr;
  if (dbl)
    hipLaunchKernelGGL(k_transpose<double>, dim3((unsigned)nblk), dim3(256), 0, st,
                       (cx<double>*)out, (const cx<double>*)in, R, C, tc, tr);
  else
    hipLaunchKernelGGL(k_transpose<float>, dim3((unsigned)nblk), dim3(256), 0, st,
                       (cx<float>*)out, (const cx<float>*)in, R, C, tc, tr);
  return hipGetLastError();
}

}  // namespace qw
