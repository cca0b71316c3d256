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

#include "qw_internal.h"

namespace qw {

// Outer index o of a launch covers `ocount` consecutive planes o0.. of each
// of several components, components `ostride` elements apart (a slab of the
// lattice); a whole-field launch has ocount = O, o0 = 0. nt: the results are
// written with non-temporal stores.
struct OuterMap {
  int64_t ocount, o0, ostride;
  int nt;
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
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = in[base + (int64_t)(t + TT * e) * I];
  fft_team<T, L, E, SIGN>(v, lds + p, P, t, tw);
  if (om.nt) {
#pragma unroll
    for (int e = 0; e < E; ++e) store_nt(&out[base + (int64_t)(t + TT * e) * I], v[e]);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) out[base + (int64_t)(t + TT * e) * I] = v[e];
  }
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
                                   int64_t I, const void* tw, hipStream_t st, bool nt) {
  const OuterMap om{ocount, o0, ostride, nt ? 1 : 0};
  const int64_t O = ncomp * ocount;
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
                              int64_t I, const void* tw, hipStream_t st, bool nt) {
  if (L == 1) {
    if (out != in)
      return hipMemcpyAsync(out, in, (dbl ? 16 : 8) * O * I, hipMemcpyDeviceToDevice, st);
    return hipSuccess;
  }
  return launch_fft_strided_slab(dbl, sign, L, out, in, 1, O, 0, 0, I, tw, st, nt);
}

// Last inverse pass of an evolution with the Sec. 5.2 reductions fused: the
// transformed values are reduced where they are produced (the field need
// not be read again, nor written at all when only the reductions are
// wanted). Whole fields: outer index o = b * s + component.
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
  const AxisImage32 a0 = axis_image32(axis_image(org[0], f.N[0]));
  // (1) Over the thread's elements: only the axis-0 displacement varies
  // along the pass, so three moments in it suffice (the other axes are
  // fixed per column).
  double S0 = 0.0, S1 = 0.0, S11 = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int pos = t + TT * e;
    const double w = min_image32(f.dim == 1 ? pos * (int)I + (int)col : pos, a0);
    const double x = (double)v[e].x, y = (double)v[e].y;
    const double pr = x * x + y * y;
    const double wp = w * pr;
    S0 += pr;
    S1 += wp;
    S11 += w * wp;
  }
  // (2) Over the TT threads of each column, through LDS (free once the
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
    const int64_t cc = col - p + tid;  // the column these sums belong to
    double wb = 0.0, wc = 0.0;
    if (f.dim == 2) {
      wb = min_image(cc, axis_image(org[1], f.N[1]));
    } else if (f.dim == 3) {
      wb = min_image(cc >> f.lg[2], axis_image(org[1], f.N[1]));
      wc = min_image(cc & (f.N[2] - 1), axis_image(org[2], f.N[2]));
    }
    acc[0] = c0;
    acc[1] = c1;
    acc[2] = wb * c0;
    acc[3] = wc * c0;
    acc[4] = c2;
    acc[5] = wb * wb * c0;
    acc[6] = wc * wc * c0;
    acc[7] = wb * c1;
    acc[8] = wc * c1;
    acc[9] = wb * wc * c0;
  }
  // (3) Over the columns: only the waves holding column sums shuffle.
  __shared__ double red2[10][16];
  const int lane = tid & 63, wave = tid >> 6;
  const int nwc = (P + 63) >> 6;
  if (wave < nwc) {
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      double vv = acc[k];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) vv += __shfl_down(vv, off, 64);
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

template <typename T, int L>
static hipError_t run_strided_obs(cx<T>* out, const cx<T>* in, int s, int B, int64_t I,
                                  const ObsFuse& f, const cx<T>* tw, hipStream_t st) {
  constexpr int Emax = sizeof(T) == 8 ? 8 : 16;
  constexpr int E = L < Emax ? L : Emax;
  constexpr int TT = L / E;
  const int P = strided_cols<T, L>(I);
  if (TT * P > 1024 || (TT * P) % 64 != 0) return hipErrorInvalidValue;
  const int lgP = ilog2(P);
  // the transform's exchanges, then 3 doubles per thread for the reduction
  const size_t lds = std::max((size_t)P * L * sizeof(cx<T>), (size_t)TT * P * 3 * sizeof(double));
  auto kern = k_fft_strided_obs<T, L, E>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t nblk_i = I / P;
  const int64_t nblk = (int64_t)s * B * nblk_i;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
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
                                       hipStream_t st) {
  switch (L) {
    case 2: return run_strided_obs<T, 2>(out, in, s, B, I, f, tw, st);
    case 4: return run_strided_obs<T, 4>(out, in, s, B, I, f, tw, st);
    case 8: return run_strided_obs<T, 8>(out, in, s, B, I, f, tw, st);
    case 16: return run_strided_obs<T, 16>(out, in, s, B, I, f, tw, st);
    case 32: return run_strided_obs<T, 32>(out, in, s, B, I, f, tw, st);
    case 64: return run_strided_obs<T, 64>(out, in, s, B, I, f, tw, st);
    case 128: return run_strided_obs<T, 128>(out, in, s, B, I, f, tw, st);
    case 256: return run_strided_obs<T, 256>(out, in, s, B, I, f, tw, st);
    case 512: return run_strided_obs<T, 512>(out, in, s, B, I, f, tw, st);
    case 1024: return run_strided_obs<T, 1024>(out, in, s, B, I, f, tw, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fft_strided_obs(bool dbl, int64_t L, void* out, const void* in, int s, int B,
                                  int64_t I, const ObsFuse& f, const void* tw, hipStream_t st) {
  if (dbl)
    return dispatch_strided_obs<double>(L, (cx<double>*)out, (const cx<double>*)in, s, B, I, f,
                                        (const cx<double>*)tw, st);
  return dispatch_strided_obs<float>(L, (cx<float>*)out, (const cx<float>*)in, s, B, I, f,
                                     (const cx<float>*)tw, st);
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
