// Position-space step of the walk (Sec. 2 of the paper, update rule):
//   psi(n, t+1) = sum_h U_h psi(n + h, t)   on the periodic N^d torus,
// with the transition matrices U_h derived by the plan from the symbol.
// The generic kernels use one thread per output site for all s components,
// with neighbour reads served by L1/L2. Large 3D lattices stage planes of a
// tile in LDS instead: the plane-ring kernel (Dirac, complex64), the tile
// kernel (Dirac, complex128 fields beyond the cache), the Weyl and the
// cubic-supercell tile kernels (complex64).
#include <algorithm>

#include "qw_internal.h"

namespace qw {

__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc + a b as four chained FMAs (the plain expression compiles to a
// multiply, an FMA and an add per real part).
template <typename T>
__device__ __forceinline__ cx<T> fma_c(cx<T> acc, cx<T> a, cx<T> b) {
  acc.x = fma_r(a.x, b.x, acc.x);
  acc.x = fma_r(a.y, -b.y, acc.x);
  acc.y = fma_r(a.x, b.y, acc.y);
  acc.y = fma_r(a.y, b.x, acc.y);
  return acc;
}

// One 1D site: U_{+1} acts on psi(n+1) (r), U_{-1} on psi(n-1) (l), U_0 on
// psi(n) (p). Shared by the streaming and the LDS-resident kernels, so both
// give bitwise the same result.
template <typename T>
__device__ __forceinline__ void site1d(const StencilCoef<T>& C, cx<T> p0, cx<T> p1, cx<T> r0,
                                       cx<T> r1, cx<T> l0, cx<T> l1, cx<T>& a0, cx<T>& a1) {
  a0 = mk((T)0, (T)0);
  a1 = a0;
  a0 = fma_c(a0, C.up[0][0][0], r0); a0 = fma_c(a0, C.up[0][0][1], r1);
  a1 = fma_c(a1, C.up[0][1][0], r0); a1 = fma_c(a1, C.up[0][1][1], r1);
  a0 = fma_c(a0, C.up[1][0][0], l0); a0 = fma_c(a0, C.up[1][0][1], l1);
  a1 = fma_c(a1, C.up[1][1][0], l0); a1 = fma_c(a1, C.up[1][1][1], l1);
  a0 = fma_c(a0, C.onsite[0][0], p0); a0 = fma_c(a0, C.onsite[0][1], p1);
  a1 = fma_c(a1, C.onsite[1][0], p0); a1 = fma_c(a1, C.onsite[1][1], p1);
}

// Instance blockIdx.y of a batch of fields back to back, with its own
// coefficients coefs[blockIdx.y].
template <typename T>
__global__ __launch_bounds__(256) void k_step1d(cx<T>* __restrict__ out_all,
                                               const cx<T>* __restrict__ in_all, StencilGeom g,
                                               const StencilCoef<T>* __restrict__ coefs) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.V) return;
  const int64_t V = g.V;
  const cx<T>* __restrict__ in = in_all + (int64_t)blockIdx.y * 2 * V;
  cx<T>* __restrict__ out = out_all + (int64_t)blockIdx.y * 2 * V;
  const StencilCoef<T> C = coefs[blockIdx.y];
  const int64_t msk = g.N[0] - 1;
  const int64_t r = (n + 1) & msk, l = (n - 1) & msk;
  cx<T> a0, a1;
  site1d(C, in[n], in[V + n], in[r], in[V + r], in[l], in[V + l], a0, a1);
  out[n] = a0;
  out[V + n] = a1;
}

// 1D lattices whose field fits in LDS: one workgroup per instance keeps the
// field in LDS for all `nsteps` steps (one global read and write in total).
// Each thread updates sites tid, tid + blockDim, ...: new values are formed
// in registers from the LDS copy, then written back after a barrier.
constexpr int kResThreads = 1024;
// Sites per thread: N <= 8192 (complex64) or 4096 (complex128), the sizes
// whose two components fit in 160 KB of LDS.
template <typename T>
constexpr int res_max_sites() { return sizeof(T) == 4 ? 8 : 4; }

template <typename T>
__global__ __launch_bounds__(kResThreads) void k_step1d_resident(
    cx<T>* __restrict__ psi_all, StencilGeom g, const StencilCoef<T>* __restrict__ coefs,
    int64_t nsteps) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* f0 = reinterpret_cast<cx<T>*>(smem_raw);
  const int N = (int)g.N[0];
  cx<T>* f1 = f0 + N;
  cx<T>* __restrict__ psi = psi_all + (int64_t)blockIdx.y * 2 * N;
  const StencilCoef<T> C = coefs[blockIdx.y];
  const int tid = threadIdx.x;
  const int msk = N - 1;
  for (int n = tid; n < N; n += kResThreads) {
    f0[n] = psi[n];
    f1[n] = psi[N + n];
  }
  __syncthreads();
  constexpr int MS = res_max_sites<T>();
  for (int64_t k = 0; k < nsteps; ++k) {
    cx<T> a0[MS], a1[MS];
#pragma unroll
    for (int j = 0; j < MS; ++j) {
      const int n = tid + j * kResThreads;
      if (n < N) {
        const int r = (n + 1) & msk, l = (n - 1) & msk;
        site1d(C, f0[n], f1[n], f0[r], f1[r], f0[l], f1[l], a0[j], a1[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MS; ++j) {
      const int n = tid + j * kResThreads;
      if (n < N) {
        f0[n] = a0[j];
        f1[n] = a1[j];
      }
    }
    __syncthreads();
  }
  for (int n = tid; n < N; n += kResThreads) {
    psi[n] = f0[n];
    psi[N + n] = f1[n];
  }
}

// Workgroup b runs on XCD b % 8 (each XCD has its own L2). With a grid that
// divides into eight, XCD x gets the contiguous range of blocks
// [x n/8, (x+1) n/8): the neighbour rows and planes a site reads then sit in
// the same L2 instead of being fetched by several XCDs.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t n) {
  return (n & 7) == 0 ? (b & 7) * (n >> 3) + (b >> 3) : b;
}

__device__ constexpr int kOff2[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
__device__ constexpr int kOff3[8][3] = {{1, 0, 0},  {0, -1, 0}, {0, 0, -1}, {-1, -1, -1},
                                        {-1, 0, 0}, {0, 1, 0},  {0, 0, 1},  {1, 1, 1}};

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_step_nd(cx<T>* __restrict__ out_all,
                                                const cx<T>* __restrict__ in_all, StencilGeom g,
                                                const StencilCoef<T>* __restrict__ coefs) {
  const int64_t idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (idx >= g.V) return;
  const int64_t V = g.V;
  const cx<T>* __restrict__ in = in_all + (int64_t)blockIdx.y * 4 * V;
  cx<T>* __restrict__ out = out_all + (int64_t)blockIdx.y * 4 * V;
  const StencilCoef<T> C = coefs[blockIdx.y];
  int64_t n[3];
  const int64_t m[3] = {g.N[0] - 1, g.N[1] - 1, g.N[2] - 1};
  if constexpr (DIM == 3) {
    n[2] = idx & m[2];
    n[1] = (idx >> g.lg[2]) & m[1];
    n[0] = idx >> (g.lg[2] + g.lg[1]);
  } else {
    n[1] = idx & m[1];
    n[0] = idx >> g.lg[1];
  }
  constexpr int K = DIM == 3 ? 8 : 4;
  cx<T> a0 = mk((T)0, (T)0), a1 = a0, a2 = a0, a3 = a0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int64_t nb;
    if constexpr (DIM == 3) {
      const int64_t x = (n[0] + kOff3[k][0]) & m[0];
      const int64_t y = (n[1] + kOff3[k][1]) & m[1];
      const int64_t z = (n[2] + kOff3[k][2]) & m[2];
      nb = (((x << g.lg[1]) | y) << g.lg[2]) | z;
    } else {
      const int64_t x = (n[0] + kOff2[k][0]) & m[0];
      const int64_t y = (n[1] + kOff2[k][1]) & m[1];
      nb = (x << g.lg[1]) | y;
    }
    const cx<T> q0 = in[nb], q1 = in[V + nb], q2 = in[2 * V + nb], q3 = in[3 * V + nb];
    a0 = fma_c(a0, C.up[k][0][0], q0); a0 = fma_c(a0, C.up[k][0][1], q1);
    a1 = fma_c(a1, C.up[k][1][0], q0); a1 = fma_c(a1, C.up[k][1][1], q1);
    a2 = fma_c(a2, C.lo[k][0][0], q2); a2 = fma_c(a2, C.lo[k][0][1], q3);
    a3 = fma_c(a3, C.lo[k][1][0], q2); a3 = fma_c(a3, C.lo[k][1][1], q3);
  }
  const cx<T> mass = C.onsite[0][0];
  a0 = fma_c(a0, mass, in[2 * V + idx]);
  a1 = fma_c(a1, mass, in[3 * V + idx]);
  a2 = fma_c(a2, mass, in[idx]);
  a3 = fma_c(a3, mass, in[V + idx]);
  if (g.nt) {
    store_nt(&out[idx], a0);
    store_nt(&out[V + idx], a1);
    store_nt(&out[2 * V + idx], a2);
    store_nt(&out[3 * V + idx], a3);
  } else {
    out[idx] = a0;
    out[V + idx] = a1;
    out[2 * V + idx] = a2;
    out[3 * V + idx] = a3;
  }
}


// Two-component Weyl walk of d = 2, 3 (Sec. 3.1): the same neighbour offsets
// as the Dirac walk, with the Weyl transition matrices in `up` (the upper
// blocks of the Dirac walk at m = 0) and no on-site term. One thread per
// output site; each instance (blockIdx.y) is a field of 2 V entries.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_step_weyl(cx<T>* __restrict__ out_all,
                                                  const cx<T>* __restrict__ in_all, StencilGeom g,
                                                  const StencilCoef<T>* __restrict__ coefs) {
  const int64_t idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (idx >= g.V) return;
  const int64_t V = g.V;
  const cx<T>* __restrict__ in = in_all + (int64_t)blockIdx.y * 2 * V;
  cx<T>* __restrict__ out = out_all + (int64_t)blockIdx.y * 2 * V;
  const StencilCoef<T>& C = coefs[blockIdx.y];
  int64_t n[3];
  const int64_t m[3] = {g.N[0] - 1, g.N[1] - 1, g.N[2] - 1};
  if constexpr (DIM == 3) {
    n[2] = idx & m[2];
    n[1] = (idx >> g.lg[2]) & m[1];
    n[0] = idx >> (g.lg[2] + g.lg[1]);
  } else {
    n[1] = idx & m[1];
    n[0] = idx >> g.lg[1];
  }
  constexpr int K = DIM == 3 ? 8 : 4;
  cx<T> a0 = mk((T)0, (T)0), a1 = a0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int64_t nb;
    if constexpr (DIM == 3) {
      const int64_t x = (n[0] + kOff3[k][0]) & m[0];
      const int64_t y = (n[1] + kOff3[k][1]) & m[1];
      const int64_t z = (n[2] + kOff3[k][2]) & m[2];
      nb = (((x << g.lg[1]) | y) << g.lg[2]) | z;
    } else {
      const int64_t x = (n[0] + kOff2[k][0]) & m[0];
      const int64_t y = (n[1] + kOff2[k][1]) & m[1];
      nb = (x << g.lg[1]) | y;
    }
    const cx<T> q0 = in[nb], q1 = in[V + nb];
    a0 = fma_c(a0, C.up[k][0][0], q0); a0 = fma_c(a0, C.up[k][0][1], q1);
    a1 = fma_c(a1, C.up[k][1][0], q0); a1 = fma_c(a1, C.up[k][1][1], q1);
  }
  if (g.nt) {
    store_nt(&out[idx], a0);
    store_nt(&out[V + idx], a1);
  } else {
    out[idx] = a0;
    out[V + idx] = a1;
  }
}

// LDS-tiled 3D Weyl step (two components). A workgroup owns a kWtR x kWtC
// tile of (n1, n2) and a chunk of planes of axis 0; each plane of the tile
// with a one-site halo in n1 and n2 is read from global memory once into a
// ring of three LDS planes (n0 - 1, n0, n0 + 1), from which all eight terms
// of the output plane n0 are formed. Each thread owns every fourth row of a
// column of the tile, so a plane's barrier covers several sites per thread.
// Tiles of kWtR rows: 16 at complex64 (four sites per thread, 57 KB of LDS),
// 8 at complex128 (two, 63 KB), two workgroups per CU either way. At
// complex128 the staged values take 80 B per lane of scratch memory.
template <typename T>
constexpr int wt_rows() { return sizeof(T) == 4 ? 16 : 8; }
constexpr int kWtC = 64;
constexpr int kWtHC = kWtC + 2;
constexpr int kWtThreads = 256;
constexpr int kWtRowStep = kWtThreads / kWtC;  // 4

// Halo site k of a tile of R rows as local (row, column): rows 0 and R + 1
// in full, then columns 0 and kWtHC - 1 of rows 1..R.
template <int R>
__device__ __forceinline__ void wt_halo_site(int k, int& lr, int& lc) {
  constexpr int kWtHR = R + 2;
  if (k < 2 * kWtHC) {
    lr = k < kWtHC ? 0 : kWtHR - 1;
    lc = k < kWtHC ? k : k - kWtHC;
  } else {
    const int q = k - 2 * kWtHC;
    lr = 1 + (q >> 1);
    lc = (q & 1) ? kWtHC - 1 : 0;
  }
}

template <typename T>
__global__ __launch_bounds__(kWtThreads) void k_step_weyl_tile(cx<T>* __restrict__ out_all,
                                                               const cx<T>* __restrict__ in_all,
                                                               StencilGeom g,
                                                               const StencilCoef<T>* __restrict__ coefs,
                                                               int lgL) {
  constexpr int kWtR = wt_rows<T>();
  constexpr int kWtSites = (kWtR + 2) * kWtHC;     // tile plus halo
  constexpr int kWtHalo = kWtSites - kWtR * kWtC;
  constexpr int kWtRowsPerThread = kWtR * kWtC / kWtThreads;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);  // [slot 3][component 2][kWtSites]
  const int64_t V = g.V;
  const cx<T>* __restrict__ in = in_all + (int64_t)blockIdx.y * 2 * V;
  cx<T>* __restrict__ out = out_all + (int64_t)blockIdx.y * 2 * V;
  const StencilCoef<T>& C = coefs[blockIdx.y];
  const int64_t m0 = g.N[0] - 1, m1 = g.N[1] - 1, m2 = g.N[2] - 1;
  const int lg2 = g.lg[2], lg12 = g.lg[1] + g.lg[2];
  const int64_t tiles2 = g.N[2] / kWtC, tiles1 = g.N[1] / kWtR;
  const int64_t w = xcd_block(blockIdx.x, gridDim.x);
  const int64_t b2 = (w % tiles2) * kWtC;
  const int64_t b1 = ((w / tiles2) % tiles1) * kWtR;
  const int64_t c0 = (w / (tiles2 * tiles1)) << lgL;
  const int tid = threadIdx.x;
  const int r = tid / kWtC, c = tid % kWtC;
  const bool has_halo = tid < kWtHalo;
  int hr = 0, hc = 0;
  if (has_halo) wt_halo_site<kWtR>(tid, hr, hc);
  const int64_t hcol = (((b1 - 1 + hr) & m1) << lg2) | ((b2 - 1 + hc) & m2);
  const int lh = hr * kWtHC + hc;
  int64_t col[kWtRowsPerThread];
#pragma unroll
  for (int h = 0; h < kWtRowsPerThread; ++h) col[h] = ((b1 + r + h * kWtRowStep) << lg2) | (b2 + c);

  cx<T> v[kWtRowsPerThread][2], vh0 = mk((T)0, (T)0), vh1 = vh0;
  auto fetch = [&](int64_t p) {
    const int64_t base = (p & m0) << lg12;
#pragma unroll
    for (int h = 0; h < kWtRowsPerThread; ++h) {
      v[h][0] = in[base + col[h]];
      v[h][1] = in[V + base + col[h]];
    }
    if (has_halo) {
      vh0 = in[base + hcol];
      vh1 = in[V + base + hcol];
    }
  };
  auto stage = [&](int slot) {
    cx<T>* P = lds + slot * 2 * kWtSites;
#pragma unroll
    for (int h = 0; h < kWtRowsPerThread; ++h) {
      const int l = (r + h * kWtRowStep + 1) * kWtHC + c + 1;
      P[l] = v[h][0];
      P[kWtSites + l] = v[h][1];
    }
    if (has_halo) {
      P[lh] = vh0;
      P[kWtSites + lh] = vh1;
    }
  };

  const int L = 1 << lgL;
  fetch(c0 - 1);
  stage(0);
  fetch(c0);
  stage(1);
  fetch(c0 + 1);
  int sm = 0, s0 = 1, sp = 2;  // ring slots of planes n0 - 1, n0, n0 + 1
  for (int i = 0; i < L; ++i) {
    const int64_t n0 = c0 + i;
    __syncthreads();  // the previous plane's reads of slot sp are done
    stage(sp);
    __syncthreads();
    if (i + 1 < L) fetch(n0 + 2);
    const cx<T>* Pm = lds + sm * 2 * kWtSites;
    const cx<T>* P0 = lds + s0 * 2 * kWtSites;
    const cx<T>* Pp = lds + sp * 2 * kWtSites;
    const int64_t plane = (n0 & m0) << lg12;
#pragma unroll
    for (int h = 0; h < kWtRowsPerThread; ++h) {
      const int ls = (r + h * kWtRowStep + 1) * kWtHC + c + 1;
      cx<T> a0 = mk((T)0, (T)0), a1 = a0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int o1 = kOff3[k][0], o2 = kOff3[k][1], o3 = kOff3[k][2];
        const cx<T>* P = (o1 > 0 ? Pp : (o1 < 0 ? Pm : P0)) + ls + o2 * kWtHC + o3;
        const cx<T> q0 = P[0], q1 = P[kWtSites];
        a0 = fma_c(a0, C.up[k][0][0], q0); a0 = fma_c(a0, C.up[k][0][1], q1);
        a1 = fma_c(a1, C.up[k][1][0], q0); a1 = fma_c(a1, C.up[k][1][1], q1);
      }
      const int64_t idx = plane | col[h];
      if (g.nt) {
        store_nt(&out[idx], a0);
        store_nt(&out[V + idx], a1);
      } else {
        out[idx] = a0;
        out[V + idx] = a1;
      }
    }
    const int t = sm;
    sm = s0;
    s0 = sp;
    sp = t;
  }
}

bool step_weyl_tile_ok(const StencilGeom& g, bool dbl) {
  return g.dim == 3 && g.weyl && g.N[1] >= (dbl ? wt_rows<double>() : wt_rows<float>()) &&
         g.N[2] >= kWtC;
}

hipError_t launch_step_weyl_tile(bool dbl, const StencilGeom& g, int B, void* out, const void* in,
                                 const void* coefs, hipStream_t st) {
  // Planes per workgroup: 16, halved (down to 2) until there are at least
  // 1024 workgroups per instance, and at most the length of axis 0 (at 256^3
  // complex64: 16 planes, 0.130 ms per step; 8 planes and 2048 workgroups,
  // 0.133).
  const int R = dbl ? wt_rows<double>() : wt_rows<float>();
  const int64_t tiles = (g.N[1] / R) * (g.N[2] / kWtC);
  int lgL = 4;
  while (lgL > 1 && (tiles * g.N[0]) >> lgL < 1024) --lgL;
  if (lgL > g.lg[0]) lgL = g.lg[0];
  const int64_t nblk = tiles * (g.N[0] >> lgL);
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = 3 * 2 * (size_t)(R + 2) * kWtHC * (dbl ? sizeof(cx<double>) : sizeof(cx<float>));
  if (dbl) {
    hipLaunchKernelGGL(k_step_weyl_tile<double>, dim3((unsigned)nblk, (unsigned)B),
                       dim3(kWtThreads), lds, st, (cx<double>*)out, (const cx<double>*)in, g,
                       (const StencilCoef<double>*)coefs, lgL);
  } else {
    hipLaunchKernelGGL(k_step_weyl_tile<float>, dim3((unsigned)nblk, (unsigned)B),
                       dim3(kWtThreads), lds, st, (cx<float>*)out, (const cx<float>*)in, g,
                       (const StencilCoef<float>*)coefs, lgL);
  }
  return hipGetLastError();
}


// LDS-tiled 3D Dirac step for complex128 fields of at least kNtBytes (the
// complex64 lattices take the plane-ring kernel below). A workgroup owns a kDtR x kDtC tile of (n1, n2)
// and a chunk of planes of axis 0; each plane of the tile with a one-site
// halo is read from global memory once into a ring of three LDS planes, from
// which the eight neighbour terms and the mass term of the output plane are
// formed, in the order of the one-thread-per-site kernel. One site per
// thread: the ring of 3 x 4 components x 396 sites takes 76 KB, two
// workgroups per CU.
constexpr int kDtR = 4, kDtC = 64;
constexpr int kDtHR = kDtR + 2, kDtHC = kDtC + 2;
constexpr int kDtSites = kDtHR * kDtHC;          // 396
constexpr int kDtHalo = kDtSites - kDtR * kDtC;  // 140
constexpr int kDtThreads = kDtR * kDtC;

// Halo site k < kDtHalo as local (row, column): rows 0 and kDtHR - 1 in
// full, then columns 0 and kDtHC - 1 of rows 1..kDtR.
__device__ __forceinline__ void dt_halo_site(int k, int& lr, int& lc) {
  if (k < 2 * kDtHC) {
    lr = k < kDtHC ? 0 : kDtHR - 1;
    lc = k < kDtHC ? k : k - kDtHC;
  } else {
    const int q = k - 2 * kDtHC;
    lr = 1 + (q >> 1);
    lc = (q & 1) ? kDtHC - 1 : 0;
  }
}

template <typename T>
__global__ __launch_bounds__(kDtThreads) void k_step3d_tile(cx<T>* __restrict__ out_all,
                                                            const cx<T>* __restrict__ in_all,
                                                            StencilGeom g,
                                                            const StencilCoef<T>* __restrict__ coefs,
                                                            int lgL) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);  // [slot 3][component 4][kDtSites]
  constexpr int PL = 4 * kDtSites;
  const int64_t V = g.V;
  const cx<T>* __restrict__ in = in_all + (int64_t)blockIdx.y * 4 * V;
  cx<T>* __restrict__ out = out_all + (int64_t)blockIdx.y * 4 * V;
  const StencilCoef<T>& C = coefs[blockIdx.y];
  const int64_t m0 = g.N[0] - 1, m1 = g.N[1] - 1, m2 = g.N[2] - 1;
  const int lg2 = g.lg[2], lg12 = g.lg[1] + g.lg[2];
  const int64_t tiles2 = g.N[2] / kDtC, tiles1 = g.N[1] / kDtR;
  const int64_t w = xcd_block(blockIdx.x, gridDim.x);
  const int64_t b2 = (w % tiles2) * kDtC;
  const int64_t b1 = ((w / tiles2) % tiles1) * kDtR;
  const int64_t c0 = (w / (tiles2 * tiles1)) << lgL;
  const int tid = threadIdx.x;
  const int r = tid / kDtC, c = tid % kDtC;
  const bool has_halo = tid < kDtHalo;
  int hr = 0, hc = 0;
  if (has_halo) dt_halo_site(tid, hr, hc);
  const int64_t hcol = (((b1 - 1 + hr) & m1) << lg2) | ((b2 - 1 + hc) & m2);
  const int64_t col = ((b1 + r) << lg2) | (b2 + c);
  const int lh = hr * kDtHC + hc;
  const int ls = (r + 1) * kDtHC + c + 1;

  cx<T> v0, v1, v2, v3, h0, h1, h2, h3;
  h0 = h1 = h2 = h3 = mk((T)0, (T)0);
  auto fetch = [&](int64_t p) __attribute__((always_inline)) {
    const int64_t s = ((p & m0) << lg12) | col;
    v0 = in[s]; v1 = in[V + s]; v2 = in[2 * V + s]; v3 = in[3 * V + s];
    if (has_halo) {
      const int64_t sh = ((p & m0) << lg12) | hcol;
      h0 = in[sh]; h1 = in[V + sh]; h2 = in[2 * V + sh]; h3 = in[3 * V + sh];
    }
  };
  auto stage = [&](int slot) __attribute__((always_inline)) {
    cx<T>* P = lds + slot * PL;
    P[ls] = v0; P[kDtSites + ls] = v1; P[2 * kDtSites + ls] = v2; P[3 * kDtSites + ls] = v3;
    if (has_halo) {
      P[lh] = h0; P[kDtSites + lh] = h1; P[2 * kDtSites + lh] = h2; P[3 * kDtSites + lh] = h3;
    }
  };

  const int L = 1 << lgL;
  fetch(c0 - 1);
  stage(0);
  fetch(c0);
  stage(1);
  fetch(c0 + 1);
  int sm = 0, s0 = 1, sp = 2;  // ring slots of planes n0 - 1, n0, n0 + 1
  const cx<T> mass = C.onsite[0][0];
  for (int i = 0; i < L; ++i) {
    const int64_t n0 = c0 + i;
    __syncthreads();  // the previous plane's reads of slot sp are done
    stage(sp);
    __syncthreads();
    if (i + 1 < L) fetch(n0 + 2);
    const cx<T>* Pm = lds + sm * PL;
    const cx<T>* P0 = lds + s0 * PL;
    const cx<T>* Pp = lds + sp * PL;
    cx<T> a0 = mk((T)0, (T)0), a1 = a0, a2 = a0, a3 = a0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int o1 = kOff3[k][0], o2 = kOff3[k][1], o3 = kOff3[k][2];
      const cx<T>* P = (o1 > 0 ? Pp : (o1 < 0 ? Pm : P0)) + ls + o2 * kDtHC + o3;
      const cx<T> q0 = P[0], q1 = P[kDtSites], q2 = P[2 * kDtSites], q3 = P[3 * kDtSites];
      a0 = fma_c(a0, C.up[k][0][0], q0); a0 = fma_c(a0, C.up[k][0][1], q1);
      a1 = fma_c(a1, C.up[k][1][0], q0); a1 = fma_c(a1, C.up[k][1][1], q1);
      a2 = fma_c(a2, C.lo[k][0][0], q2); a2 = fma_c(a2, C.lo[k][0][1], q3);
      a3 = fma_c(a3, C.lo[k][1][0], q2); a3 = fma_c(a3, C.lo[k][1][1], q3);
    }
    a0 = fma_c(a0, mass, P0[2 * kDtSites + ls]);
    a1 = fma_c(a1, mass, P0[3 * kDtSites + ls]);
    a2 = fma_c(a2, mass, P0[ls]);
    a3 = fma_c(a3, mass, P0[kDtSites + ls]);
    const int64_t idx = ((n0 & m0) << lg12) | col;
    if (g.nt) {
      store_nt(&out[idx], a0);
      store_nt(&out[V + idx], a1);
      store_nt(&out[2 * V + idx], a2);
      store_nt(&out[3 * V + idx], a3);
    } else {
      out[idx] = a0;
      out[V + idx] = a1;
      out[2 * V + idx] = a2;
      out[3 * V + idx] = a3;
    }
    const int t = sm;
    sm = s0;
    s0 = sp;
    sp = t;
  }
}

bool step3d_tile_ok(const StencilGeom& g) {
  return g.dim == 3 && !g.weyl && g.N[1] >= kDtR && g.N[2] >= kDtC;
}

hipError_t launch_step3d_tile(const StencilGeom& g, int B, void* out, const void* in,
                              const void* coefs, hipStream_t st) {
  // Planes per workgroup: 16, halved (down to 2) until there are at least
  // 2048 workgroups per instance, and at most the length of axis 0.
  const int64_t tiles = (g.N[1] / kDtR) * (g.N[2] / kDtC);
  int lgL = 4;
  while (lgL > 1 && (tiles * g.N[0]) >> lgL < 2048) --lgL;
  if (lgL > g.lg[0]) lgL = g.lg[0];
  const int64_t nblk = tiles * (g.N[0] >> lgL);
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = 3 * 4 * kDtSites * sizeof(cx<double>);
  auto kern = k_step3d_tile<double>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk, (unsigned)B), dim3(kDtThreads), lds, st,
                     (cx<double>*)out, (const cx<double>*)in, g, (const StencilCoef<double>*)coefs,
                     lgL);
  return hipGetLastError();
}

// Cubic-supercell BCC field (Sec. 4): two sublattice arrays of N1 x N2 x N3
// sites, f_j(m) at the Cartesian site x = 2m + j t, t = (1,1,1). One step of
// the update rule of Sec. 2, psi(x) <- sum_k U_k psi(x + c_k) + mass term,
// with c_k the Cartesian displacement H o_k of the k-th neighbour offset o_k
// (kOff3; H has the generators h1 = (1,1,1), h2 = (1,-1,-1), h3 = (-1,1,-1)
// as columns). Every c_k has entries +-1, so x + c_k lies on the other
// sublattice: at m + (c_k - t)/2 from sublattice 0 and at m + (c_k + t)/2 from
// sublattice 1 (periodic in m). The mass term couples the upper and lower
// components of the site itself.
//
// The eight sites read for output m therefore form a 2 x 2 x 2 block of the
// other sublattice, {m + s a : a in {0,1}^3} with s = -1 for sublattice 0 and
// s = +1 for sublattice 1. A thread marches along axis 0 through a chunk of
// kBccChunk outputs at fixed (m1, m2): the quad of sites in plane m0 + s (or
// m0) read for one output is the quad in plane m0 (or m0 + s) of the next, so
// it is kept in registers and each output loads one new quad (16 values) and
// its own four components, instead of eight sites.
__device__ constexpr int kCart3[8][3] = {{1, 1, 1},    {-1, 1, 1},  {1, -1, 1},  {-1, -1, 1},
                                         {-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1}};
constexpr int kLgBccChunk = 4;  // kBccChunk = 16 planes per thread
constexpr int kLgBccStrip = 5;  // rows of axis 1 a workgroup range covers

// The four sites (m0, m1 + s a1, m2 + s a2), a1, a2 in {0,1}, of the plane at
// offset plane_off, all four components: P[2 a1 + a2][c].
template <typename T, int SH>
__device__ __forceinline__ void load_quad(cx<T> (&P)[4][4], const cx<T>* __restrict__ src,
                                          int64_t V, int64_t plane_off, int64_t n1, int64_t n2,
                                          int64_t m1, int64_t m2, int lg2) {
  const int64_t r0 = plane_off + (n1 << lg2);
  const int64_t r1 = plane_off + (((n1 + SH) & m1) << lg2);
  const int64_t z1 = (n2 + SH) & m2;
  const int64_t idx[4] = {r0 + n2, r0 + z1, r1 + n2, r1 + z1};
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) P[q][c] = src[c * V + idx[q]];
}

template <typename T, int SH>
__device__ __forceinline__ void bcc_column(cx<T>* __restrict__ dst, const cx<T>* __restrict__ src,
                                           const cx<T>* __restrict__ own, const StencilGeom& g,
                                           const StencilCoef<T>& C, int64_t c0, int len,
                                           int64_t n1, int64_t n2) {
  const int64_t V = g.V;
  const int64_t m0 = g.N[0] - 1, m1 = g.N[1] - 1, m2 = g.N[2] - 1;
  const int lg12 = g.lg[1] + g.lg[2];
  const int64_t col = (n1 << g.lg[2]) | n2;
  // H: the quad of the plane loaded last; Q: the new one. For s = +1 plane
  // m0 is H and m0 + 1 is Q; for s = -1 plane m0 - 1 is H and m0 is Q.
  cx<T> H[4][4], Q[4][4];
  load_quad<T, SH>(H, src, V, (SH > 0 ? c0 : ((c0 - 1) & m0)) << lg12, n1, n2, m1, m2, g.lg[2]);
  const cx<T> mass = C.onsite[0][0];
  for (int i = 0; i < len; ++i) {
    const int64_t n0 = c0 + i;
    load_quad<T, SH>(Q, src, V, (SH > 0 ? ((n0 + 1) & m0) : n0) << lg12, n1, n2, m1, m2, g.lg[2]);
    const int64_t site = (n0 << lg12) | col;
    const cx<T> o0 = own[site], o1 = own[V + site], o2 = own[2 * V + site],
                o3 = own[3 * V + site];
    cx<T> a0 = mk((T)0, (T)0), a1 = a0, a2 = a0, a3 = a0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      // a_i = 1 where the k-th displacement is s along axis i
      const int b0 = (kCart3[k][0] * SH + 1) >> 1;
      const int b1 = (kCart3[k][1] * SH + 1) >> 1;
      const int b2 = (kCart3[k][2] * SH + 1) >> 1;
      const bool fresh = (b0 == 1) == (SH > 0);
      const int qi = 2 * b1 + b2;
      const cx<T> q0 = fresh ? Q[qi][0] : H[qi][0], q1 = fresh ? Q[qi][1] : H[qi][1];
      const cx<T> q2 = fresh ? Q[qi][2] : H[qi][2], q3 = fresh ? Q[qi][3] : H[qi][3];
      a0 = fma_c(a0, C.up[k][0][0], q0); a0 = fma_c(a0, C.up[k][0][1], q1);
      a1 = fma_c(a1, C.up[k][1][0], q0); a1 = fma_c(a1, C.up[k][1][1], q1);
      a2 = fma_c(a2, C.lo[k][0][0], q2); a2 = fma_c(a2, C.lo[k][0][1], q3);
      a3 = fma_c(a3, C.lo[k][1][0], q2); a3 = fma_c(a3, C.lo[k][1][1], q3);
    }
    a0 = fma_c(a0, mass, o2);
    a1 = fma_c(a1, mass, o3);
    a2 = fma_c(a2, mass, o0);
    a3 = fma_c(a3, mass, o1);
    if (g.nt) {
      store_nt(&dst[site], a0);
      store_nt(&dst[V + site], a1);
      store_nt(&dst[2 * V + site], a2);
      store_nt(&dst[3 * V + site], a3);
    } else {
      dst[site] = a0;
      dst[V + site] = a1;
      dst[2 * V + site] = a2;
      dst[3 * V + site] = a3;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c) H[q][c] = Q[q][c];
  }
}

// Thread order (a bijection onto the columns of both arrays), fastest first:
// m2, a row of a strip of 2^kLgBccStrip rows of axis 1, the sublattice, the
// strip, the chunk of axis 0. Each XCD takes a contiguous range of it
// (xcd_block): the workgroups resident on one XCD cover a few strips of both
// arrays and march through the same planes together, so the rows and planes
// they share are fetched from HBM about once.
template <typename T>
__global__ __launch_bounds__(256) void k_step_bcc(cx<T>* __restrict__ out,
                                                 const cx<T>* __restrict__ in, StencilGeom g,
                                                 const StencilCoef<T>* __restrict__ coefs) {
  const int lgL = g.lg[0] < kLgBccChunk ? g.lg[0] : kLgBccChunk;
  const int lgR = g.lg[1] < kLgBccStrip ? g.lg[1] : kLgBccStrip;
  const int64_t V = g.V;
  const int64_t w = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (w >= (2 * V) >> lgL) return;
  const int64_t n2 = w & (g.N[2] - 1);
  int64_t q = w >> g.lg[2];
  const int64_t r = q & ((int64_t(1) << lgR) - 1);
  q >>= lgR;
  const int j = (int)(q & 1);
  q >>= 1;
  const int64_t n1 = ((q & ((int64_t(1) << (g.lg[1] - lgR)) - 1)) << lgR) | r;
  const int64_t c0 = (q >> (g.lg[1] - lgR)) << lgL;
  cx<T>* __restrict__ dst = out + (int64_t)j * 4 * V;
  const cx<T>* __restrict__ own = in + (int64_t)j * 4 * V;
  const cx<T>* __restrict__ src = in + (int64_t)(1 - j) * 4 * V;  // the other sublattice
  if (j == 0)
    bcc_column<T, -1>(dst, src, own, g, coefs[0], c0, 1 << lgL, n1, n2);
  else
    bcc_column<T, 1>(dst, src, own, g, coefs[0], c0, 1 << lgL, n1, n2);
}

// LDS-tiled form of the same step. A workgroup owns a kBtR x kBtC tile of
// (m1, m2) and a chunk of planes of axis 0, and forms the outputs of both
// sublattice arrays there: output m of sublattice 0 reads sublattice 1 at
// m - a and output m of sublattice 1 reads sublattice 0 at m + a, a in
// {0,1}^3. Per plane it stages the sublattice-1 tile with a one-site halo on
// the low side of axes 1 and 2 and the sublattice-0 tile with one on the high
// side, each in a ring of two planes (m0 - 1 and m0 of sublattice 1, m0 and
// m0 + 1 of sublattice 0). Each input value is then fetched once per
// workgroup (plus its share of halo), every read of the eight neighbours and
// of the site's own components (the mass term) is served from LDS, and a
// barrier per plane keeps the workgroup's waves on the same plane.
constexpr int kBtR = 4, kBtC = 64;
constexpr int kBtHC = kBtC + 1;
constexpr int kBtSites = (kBtR + 1) * kBtHC;     // tile plus halo: 325
constexpr int kBtHalo = kBtSites - kBtR * kBtC;  // 69
constexpr int kBtThreads = kBtR * kBtC;          // one tile site per thread

// Halo site k < kBtHalo of a staged plane as local (row, column): for
// sublattice 1 (halo low) row 0 in full, then column 0 of rows 1..kBtR; for
// sublattice 0 (halo high) row kBtR in full, then column kBtC of rows
// 0..kBtR-1.
__device__ __forceinline__ void bt_halo_site(int sub, int k, int& lr, int& lc) {
  if (k < kBtHC) {
    lr = sub ? 0 : kBtR;
    lc = k;
  } else {
    lr = sub ? k - kBtHC + 1 : k - kBtHC;
    lc = sub ? 0 : kBtC;
  }
}

// Per-thread staging of the tiled cubic step: the thread's own tile site of
// a sublattice-1 plane p1 and a sublattice-0 plane p0, and its halo site (of
// plane p1 or p0), held in registers between the global loads and the LDS
// writes.
template <typename T>
struct BtRegs {
  cx<T> v1[4], v0[4], vh[4];
};
struct BtSite {
  int64_t col, hcol;  // (m1, m2) offsets of the tile site and of the halo site
  int lh, l1, l0;     // LDS offsets: halo site, tile site in the two staged layouts
  int hsub;           // sublattice of the halo site
  bool has_halo;
};

template <typename T>
__device__ __forceinline__ void bt_fetch(BtRegs<T>& v, const cx<T>* __restrict__ f0,
                                         const cx<T>* __restrict__ f1, int64_t V, int64_t m0,
                                         int lg12, const BtSite& S, int64_t p1, int64_t p0) {
  const int64_t s1 = ((p1 & m0) << lg12) | S.col, s0 = ((p0 & m0) << lg12) | S.col;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v.v1[q] = f1[q * V + s1];
    v.v0[q] = f0[q * V + s0];
  }
  if (S.has_halo) {
    const cx<T>* __restrict__ hsrc = S.hsub ? f1 : f0;
    const int64_t sh = (((S.hsub ? p1 : p0) & m0) << lg12) | S.hcol;
#pragma unroll
    for (int q = 0; q < 4; ++q) v.vh[q] = hsrc[q * V + sh];
  }
}

template <typename T>
__device__ __forceinline__ void bt_stage(const BtRegs<T>& v, cx<T>* lds, const BtSite& S,
                                         int slot) {
  cx<T>* s1 = lds + (2 + slot) * 4 * kBtSites;
  cx<T>* s0 = lds + slot * 4 * kBtSites;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    s1[q * kBtSites + S.l1] = v.v1[q];
    s0[q * kBtSites + S.l0] = v.v0[q];
  }
  if (S.has_halo) {
    cx<T>* sh = S.hsub ? s1 : s0;
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[q * kBtSites + S.lh] = v.vh[q];
  }
}

template <typename T>
__global__ __launch_bounds__(kBtThreads) void k_step_bcc_tile(cx<T>* __restrict__ out,
                                                              const cx<T>* __restrict__ in,
                                                              StencilGeom g,
                                                              const StencilCoef<T>* __restrict__ coefs,
                                                              int lgL) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);  // [sub][slot][comp][kBtSites]
  const int64_t V = g.V;
  const int64_t m0 = g.N[0] - 1, m1 = g.N[1] - 1, m2 = g.N[2] - 1;
  const int lg12 = g.lg[1] + g.lg[2];
  const int64_t tiles2 = g.N[2] / kBtC, tiles1 = g.N[1] / kBtR;
  const int64_t w = xcd_block(blockIdx.x, gridDim.x);
  const int64_t b2 = (w % tiles2) * kBtC;
  const int64_t b1 = ((w / tiles2) % tiles1) * kBtR;
  const int64_t c0 = (w / (tiles2 * tiles1)) << lgL;
  const int tid = threadIdx.x;
  const int r = tid / kBtC, c = tid % kBtC;
  const cx<T>* __restrict__ f0 = in;
  const cx<T>* __restrict__ f1 = in + 4 * V;
  // The halo site this thread stages, if any: sublattice 1 for tid < kBtHalo,
  // sublattice 0 for kBtHalo <= tid < 2 kBtHalo.
  const int hsub = tid < kBtHalo ? 1 : 0;
  const bool has_halo = tid < 2 * kBtHalo;
  int hr = 0, hc = 0;
  if (has_halo) bt_halo_site(hsub, hsub ? tid : tid - kBtHalo, hr, hc);
  const int64_t hcol = hsub ? ((((b1 - 1 + hr) & m1) << g.lg[2]) | ((b2 - 1 + hc) & m2))
                            : ((((b1 + hr) & m1) << g.lg[2]) | ((b2 + hc) & m2));
  const int64_t col = ((b1 + r) << g.lg[2]) | (b2 + c);
  const BtSite S{col, hcol, hr * kBtHC + hc, (r + 1) * kBtHC + c + 1, r * kBtHC + c, hsub,
                 has_halo};
  BtRegs<T> v;
  const StencilCoef<T>& C = coefs[0];
  const cx<T> mass = C.onsite[0][0];
  const int L = 1 << lgL;
  cx<T>* __restrict__ d0 = out;
  cx<T>* __restrict__ d1 = out + 4 * V;
  bt_fetch(v, f0, f1, V, m0, lg12, S, c0 - 1, c0);  // the older planes of the first output plane
  bt_stage(v, lds, S, 0);
  bt_fetch(v, f0, f1, V, m0, lg12, S, c0, c0 + 1);
  for (int i = 0; i < L; ++i) {
    const int oslot = i & 1, nslot = oslot ^ 1;
    __syncthreads();  // the previous plane's reads of slot nslot are done
    bt_stage(v, lds, S, nslot);
    __syncthreads();
    const int64_t n0 = c0 + i;
    if (i + 1 < L) bt_fetch(v, f0, f1, V, m0, lg12, S, n0 + 1, n0 + 2);
    const cx<T>* o1 = lds + (2 + oslot) * 4 * kBtSites;  // sublattice 1, plane n0 - 1
    const cx<T>* n1p = lds + (2 + nslot) * 4 * kBtSites; // sublattice 1, plane n0
    const cx<T>* o0 = lds + oslot * 4 * kBtSites;        // sublattice 0, plane n0
    const cx<T>* n0p = lds + nslot * 4 * kBtSites;       // sublattice 0, plane n0 + 1
    const int64_t site = (n0 << lg12) | col;
    // Sublattice 0: neighbours m - a on sublattice 1, own components at m.
    {
      cx<T> a0 = mk((T)0, (T)0), a1 = a0, a2 = a0, a3 = a0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e0 = (1 - kCart3[k][0]) >> 1, e1 = (1 - kCart3[k][1]) >> 1,
                  e2 = (1 - kCart3[k][2]) >> 1;
        const cx<T>* P = e0 ? o1 : n1p;
        const int l = (r + 1 - e1) * kBtHC + (c + 1 - e2);
        const cx<T> q0 = P[l], q1 = P[kBtSites + l], q2 = P[2 * kBtSites + l],
                    q3 = P[3 * kBtSites + l];
        a0 = fma_c(a0, C.up[k][0][0], q0); a0 = fma_c(a0, C.up[k][0][1], q1);
        a1 = fma_c(a1, C.up[k][1][0], q0); a1 = fma_c(a1, C.up[k][1][1], q1);
        a2 = fma_c(a2, C.lo[k][0][0], q2); a2 = fma_c(a2, C.lo[k][0][1], q3);
        a3 = fma_c(a3, C.lo[k][1][0], q2); a3 = fma_c(a3, C.lo[k][1][1], q3);
      }
      const int l = r * kBtHC + c;
      a0 = fma_c(a0, mass, o0[2 * kBtSites + l]);
      a1 = fma_c(a1, mass, o0[3 * kBtSites + l]);
      a2 = fma_c(a2, mass, o0[l]);
      a3 = fma_c(a3, mass, o0[kBtSites + l]);
      if (g.nt) {
        store_nt(&d0[site], a0); store_nt(&d0[V + site], a1);
        store_nt(&d0[2 * V + site], a2); store_nt(&d0[3 * V + site], a3);
      } else {
        d0[site] = a0; d0[V + site] = a1; d0[2 * V + site] = a2; d0[3 * V + site] = a3;
      }
    }
    // Sublattice 1: neighbours m + a on sublattice 0, own components at m.
    {
      cx<T> a0 = mk((T)0, (T)0), a1 = a0, a2 = a0, a3 = a0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int e0 = (1 + kCart3[k][0]) >> 1, e1 = (1 + kCart3[k][1]) >> 1,
                  e2 = (1 + kCart3[k][2]) >> 1;
        const cx<T>* P = e0 ? n0p : o0;
        const int l = (r + e1) * kBtHC + (c + e2);
        const cx<T> q0 = P[l], q1 = P[kBtSites + l], q2 = P[2 * kBtSites + l],
                    q3 = P[3 * kBtSites + l];
        a0 = fma_c(a0, C.up[k][0][0], q0); a0 = fma_c(a0, C.up[k][0][1], q1);
        a1 = fma_c(a1, C.up[k][1][0], q0); a1 = fma_c(a1, C.up[k][1][1], q1);
        a2 = fma_c(a2, C.lo[k][0][0], q2); a2 = fma_c(a2, C.lo[k][0][1], q3);
        a3 = fma_c(a3, C.lo[k][1][0], q2); a3 = fma_c(a3, C.lo[k][1][1], q3);
      }
      const int l = (r + 1) * kBtHC + c + 1;
      a0 = fma_c(a0, mass, n1p[2 * kBtSites + l]);
      a1 = fma_c(a1, mass, n1p[3 * kBtSites + l]);
      a2 = fma_c(a2, mass, n1p[l]);
      a3 = fma_c(a3, mass, n1p[kBtSites + l]);
      if (g.nt) {
        store_nt(&d1[site], a0); store_nt(&d1[V + site], a1);
        store_nt(&d1[2 * V + site], a2); store_nt(&d1[3 * V + site], a3);
      } else {
        d1[site] = a0; d1[V + site] = a1; d1[2 * V + site] = a2; d1[3 * V + site] = a3;
      }
    }
  }
}

hipError_t launch_step_bcc(bool dbl, const StencilGeom& g, void* out, const void* in,
                           const void* coefs, hipStream_t st) {
  if (g.dim != 3 || g.weyl) return hipErrorInvalidValue;
  StencilGeom gn = g;
  gn.nt = 2 * 4 * (size_t)g.V * (dbl ? 16 : 8) >= kNtBytes;
  // complex64 lattices that hold a whole tile take the LDS-tiled kernel;
  // complex128 takes the marching one, whose staging registers the compiler
  // keeps out of scratch memory (the tiled kernel's it does not, at double).
  if (!dbl && g.N[1] >= kBtR && g.N[2] >= kBtC) {
    // Planes per workgroup: 16, halved (down to 2) until there are at least
    // 2048 workgroups, and at most the length of axis 0.
    const int64_t tiles = (g.N[1] / kBtR) * (g.N[2] / kBtC);
    int lgL = 4;
    while (lgL > 1 && (tiles * g.N[0]) >> lgL < 2048) --lgL;
    if (lgL > g.lg[0]) lgL = g.lg[0];
    const int64_t nblk = tiles * (g.N[0] >> lgL);
    if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = 2 * 2 * 4 * kBtSites * sizeof(cx<float>);
    hipLaunchKernelGGL(k_step_bcc_tile<float>, dim3((unsigned)nblk), dim3(kBtThreads), lds, st,
                       (cx<float>*)out, (const cx<float>*)in, gn, (const StencilCoef<float>*)coefs,
                       lgL);
    return hipGetLastError();
  }
  const int lgL = g.lg[0] < kLgBccChunk ? g.lg[0] : kLgBccChunk;
  const int64_t nblk = (((2 * g.V) >> lgL) + 255) / 256;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  if (dbl)
    hipLaunchKernelGGL(k_step_bcc<double>, dim3((unsigned)nblk), dim3(256), 0, st,
                       (cx<double>*)out, (const cx<double>*)in, gn,
                       (const StencilCoef<double>*)coefs);
  else
    hipLaunchKernelGGL(k_step_bcc<float>, dim3((unsigned)nblk), dim3(256), 0, st,
                       (cx<float>*)out, (const cx<float>*)in, gn, (const StencilCoef<float>*)coefs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3D step with an LDS ring of lattice planes. A workgroup owns a TN2 x TN3
// tile of (n2, n3) and marches along n1 through a chunk of planes. Each input
// plane of the tile, with a one-site halo in n2 and n3, is read from global
// memory once into a ring of three LDS planes (n1-1, n1, n1+1), from which
// all nine terms of the output plane n1 are formed. The next plane's loads
// are issued before the current plane is computed. Workgroups are numbered
// so that the tiles handled by one XCD (workgroup index mod 8) are adjacent,
// which keeps the halos that neighbouring tiles share in that XCD's L2.
// ---------------------------------------------------------------------------
constexpr int kTN2 = 8, kTN3 = 64;
constexpr int kH2 = kTN2 + 2, kH3 = kTN3 + 2;
constexpr int kPlaneSites = kH2 * kH3;               // tile + halo
constexpr int kHalo = kPlaneSites - kTN2 * kTN3;     // 148 halo sites
constexpr int kStepThreads = kTN2 * kTN3 / 2;        // two tile sites per thread

template <typename T>
struct PlaneRegs {
  cx<T> own[2][4];
  cx<T> halo[4];
};

// Site (i2, i3) of the halo'd tile, i2 in [0, kH2), i3 in [0, kH3), for the
// k-th halo site (k < kHalo): rows 0 and kH2-1 in full, then columns 0 and kH3-1.
__device__ __forceinline__ void halo_site(int k, int& i2, int& i3) {
  if (k < 2 * kH3) {
    i2 = k < kH3 ? 0 : kH2 - 1;
    i3 = k < kH3 ? k : k - kH3;
  } else {
    const int r = k - 2 * kH3;  // 0 .. 2*kTN2-1
    i2 = 1 + (r >> 1);
    i3 = (r & 1) ? kH3 - 1 : 0;
  }
}

template <typename T>
__device__ __forceinline__ void load_plane(PlaneRegs<T>& R, const cx<T>* __restrict__ in,
                                           int64_t V, int64_t plane_off, int64_t m2, int64_t m3,
                                           int lg3, int64_t b2, int64_t b3, int tid) {
  // own sites: rows tid / kTN3 and tid / kTN3 + kTN2 / 2, column tid % kTN3
  const int c3 = tid & (kTN3 - 1);
  const int r0 = tid / kTN3;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t n2 = (b2 + r0 + h * (kTN2 / 2)) & m2;
    const int64_t n3 = (b3 + c3) & m3;
    const int64_t idx = plane_off + (n2 << lg3) + n3;
#pragma unroll
    for (int c = 0; c < 4; ++c) R.own[h][c] = in[c * V + idx];
  }
  // Every thread loads (threads past the halo repeat halo site 0 and never
  // store it): unconditional loads keep the wait counts exact.
  {
    int i2, i3;
    halo_site(tid < kHalo ? tid : 0, i2, i3);
    const int64_t n2 = (b2 + i2 - 1) & m2;
    const int64_t n3 = (b3 + i3 - 1) & m3;
    const int64_t idx = plane_off + (n2 << lg3) + n3;
#pragma unroll
    for (int c = 0; c < 4; ++c) R.halo[c] = in[c * V + idx];
  }
}

template <typename T>
__device__ __forceinline__ void store_plane(const PlaneRegs<T>& R, cx<T>* ring, int tid) {
  const int c3 = tid & (kTN3 - 1);
  const int r0 = tid / kTN3;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i2 = 1 + r0 + h * (kTN2 / 2), i3 = 1 + c3;
#pragma unroll
    for (int c = 0; c < 4; ++c) ring[(c * kH2 + i2) * kH3 + i3] = R.own[h][c];
  }
  if (tid < kHalo) {
    int i2, i3;
    halo_site(tid, i2, i3);
#pragma unroll
    for (int c = 0; c < 4; ++c) ring[(c * kH2 + i2) * kH3 + i3] = R.halo[c];
  }
}

// The eight neighbour terms and the mass term of one output site of the 3D
// Dirac step, read from planes n1-1 (Pm), n1 (P0) and n1+1 (Pp) of a tile
// staged in LDS with rows of W sites and components CS sites apart. Shared
// by the one-step and the two-step plane-ring kernels, so that both form
// every site with the same operations in the same order (same bits).
template <typename T, bool SPARSE, int W, int CS>
__device__ __forceinline__ void site3d_lds(const cx<T>* Pm, const cx<T>* P0, const cx<T>* Pp,
                                           int site, const StencilCoef<T>& C, cx<T>& a0,
                                           cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  a0 = mk((T)0, (T)0);
  a1 = a0;
  a2 = a0;
  a3 = a0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int o1 = kOff3[k][0], o2 = kOff3[k][1], o3 = kOff3[k][2];
    const cx<T>* P = (o1 > 0 ? Pp : (o1 < 0 ? Pm : P0)) + site + o2 * W + o3;
    const cx<T> q0 = P[0], q1 = P[CS];
    if constexpr (SPARSE) {
      // rank-one blocks: offsets 0..3 feed output 0 and read component 3,
      // offsets 4..7 feed output 1 and read component 2
      if (k < 4) {
        const cx<T> q3 = P[3 * CS];
        a0 = fma_c(a0, C.up[k][0][0], q0); a0 = fma_c(a0, C.up[k][0][1], q1);
        a2 = fma_c(a2, C.lo[k][0][1], q3); a3 = fma_c(a3, C.lo[k][1][1], q3);
      } else {
        const cx<T> q2 = P[2 * CS];
        a1 = fma_c(a1, C.up[k][1][0], q0); a1 = fma_c(a1, C.up[k][1][1], q1);
        a2 = fma_c(a2, C.lo[k][0][0], q2); a3 = fma_c(a3, C.lo[k][1][0], q2);
      }
    } else {
      const cx<T> q2 = P[2 * CS], q3 = P[3 * CS];
      a0 = fma_c(a0, C.up[k][0][0], q0); a0 = fma_c(a0, C.up[k][0][1], q1);
      a1 = fma_c(a1, C.up[k][1][0], q0); a1 = fma_c(a1, C.up[k][1][1], q1);
      a2 = fma_c(a2, C.lo[k][0][0], q2); a2 = fma_c(a2, C.lo[k][0][1], q3);
      a3 = fma_c(a3, C.lo[k][1][0], q2); a3 = fma_c(a3, C.lo[k][1][1], q3);
    }
  }
  const cx<T> mass = C.onsite[0][0];
  a0 = fma_c(a0, mass, P0[site + 2 * CS]);
  a1 = fma_c(a1, mass, P0[site + 3 * CS]);
  a2 = fma_c(a2, mass, P0[site]);
  a3 = fma_c(a3, mass, P0[site + CS]);
}

// NT: outputs are written with non-temporal stores (fields of at least
// kNtBytes: 256^3 complex64 0.230 -> 0.214 ms per step; at 128^3 they would
// cost 0.030 -> 0.035 ms, the next step's read hitting the cache).
template <typename T, int PF, bool SPARSE, bool NT>
__global__ __launch_bounds__(kStepThreads) void k_step3d_ring(cx<T>* __restrict__ out_all,
                                                             const cx<T>* __restrict__ in_all,
                                                             StencilGeom g,
                                                             const StencilCoef<T>* __restrict__ coefs,
                                                             int chunk, int64_t tiles2,
                                                             int64_t tiles3, int64_t nchunks) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const cx<T>* __restrict__ in = in_all + (int64_t)blockIdx.y * 4 * g.V;
  cx<T>* __restrict__ out = out_all + (int64_t)blockIdx.y * 4 * g.V;
  const StencilCoef<T> C = coefs[blockIdx.y];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int PL = 4 * kPlaneSites;  // elements per ring plane
  const int tid = threadIdx.x;
  // XCD-aware numbering: workgroup b runs on XCD b % 8; give each XCD a
  // contiguous range of (chunk, tile) indices.
  const int64_t nblk = (int64_t)gridDim.x;
  const int64_t b = blockIdx.x;
  int64_t w = b;
  if ((nblk & 7) == 0) w = (b & 7) * (nblk >> 3) + (b >> 3);
  const int64_t t3 = w % tiles3;
  const int64_t t2 = (w / tiles3) % tiles2;
  const int64_t ch = w / (tiles3 * tiles2);
  (void)nchunks;
  const int64_t b2 = t2 * kTN2, b3 = t3 * kTN3;
  const int64_t m1 = g.N[0] - 1, m2 = g.N[1] - 1, m3 = g.N[2] - 1;
  const int lg3 = g.lg[2];
  const int64_t planeN = g.N[1] * g.N[2];
  const int64_t V = g.V;
  const int64_t a = ch * chunk;

  // Ring slot of (unwrapped) plane p is (p - a + 1) mod 3. The register sets
  // R[0..PF-1] hold the next PF planes in flight: at iteration n1, set
  // (n1 - a) mod PF holds plane n1+1; once it is in LDS it is refilled with
  // plane n1+1+PF. The loop is unrolled by PF so every set is addressed
  // statically.
  PlaneRegs<T> R[PF];
  load_plane(R[0], in, V, ((a - 1) & m1) * planeN, m2, m3, lg3, b2, b3, tid);
  store_plane(R[0], lds, tid);  // plane a-1 -> slot 0
  load_plane(R[0], in, V, (a & m1) * planeN, m2, m3, lg3, b2, b3, tid);
  store_plane(R[0], lds + PL, tid);  // plane a -> slot 1
#pragma unroll
  for (int u = 0; u < PF; ++u)
    load_plane(R[u], in, V, ((a + 1 + u) & m1) * planeN, m2, m3, lg3, b2, b3, tid);

  const int c3 = tid & (kTN3 - 1);
  const int r0 = tid / kTN3;
  // One output plane n1 from ring slots; set u of the registers holds plane
  // n1+1 on entry and, with REFILL, plane n1+1+PF on exit.
  auto plane_step = [&](int64_t n1, int u, bool refill) {
    const int64_t n0 = n1 & m1;
    const int sm = (int)((n1 - a) % 3), s0 = (int)((n1 - a + 1) % 3), sp = (int)((n1 - a + 2) % 3);
    store_plane(R[u], lds + sp * PL, tid);  // plane n1+1 into its slot
    __syncthreads();
    if (refill) load_plane(R[u], in, V, ((n1 + 1 + PF) & m1) * planeN, m2, m3, lg3, b2, b3, tid);
    const cx<T>* Pm = lds + sm * PL;
    const cx<T>* P0 = lds + s0 * PL;
    const cx<T>* Pp = lds + sp * PL;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i2 = 1 + r0 + h * (kTN2 / 2), i3 = 1 + c3;
      const int site = i2 * kH3 + i3;
      cx<T> a0, a1, a2, a3;
      site3d_lds<T, SPARSE, kH3, kH2 * kH3>(Pm, P0, Pp, site, C, a0, a1, a2, a3);
      const int64_t n2 = b2 + r0 + h * (kTN2 / 2), n3 = b3 + c3;
      const int64_t idx = n0 * planeN + (n2 << lg3) + n3;
      if constexpr (NT) {
        store_nt(&out[idx], a0);
        store_nt(&out[V + idx], a1);
        store_nt(&out[2 * V + idx], a2);
        store_nt(&out[3 * V + idx], a3);
      } else {
        out[idx] = a0;
        out[V + idx] = a1;
        out[2 * V + idx] = a2;
        out[3 * V + idx] = a3;
      }
    }
    __syncthreads();  // slot of plane n1-1 is rewritten next iteration
  };
  // chunk is a multiple of PF: all but the last PF planes refill their set
  // unconditionally; the last PF planes load nothing.
  for (int64_t nb = a; nb < a + chunk - PF; nb += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) plane_step(nb + u, u, true);
  }
#pragma unroll
  for (int u = 0; u < PF; ++u) plane_step(a + chunk - PF + u, u, false);
}

bool step3d_ring_ok(const StencilGeom& g) {
  return g.dim == 3 && g.N[1] >= kTN2 && g.N[2] >= kTN3 && g.N[0] >= 4;
}

// complex64 only: the complex128 ring kernel spills registers and ran slower
// than one thread per site at every size measured (64^3: 72 vs 11 us,
// 128^3: 115 vs 86 us per step).
hipError_t launch_step3d_ring(const StencilGeom& g, int B, void* out, const void* in,
                              const void* coefs, hipStream_t st) {
  const int64_t tiles2 = g.N[1] / kTN2, tiles3 = g.N[2] / kTN3;
  // Planes per workgroup: N2 N3 / 2048 within [2, 32], i.e. about 4 N1
  // workgroups for cubic lattices. Measured best at 64^3 (2 planes: 8.0 us
  // per step against 27.9 with 16), 128^3 (8: 28.9 against 32.7) and 256^3
  // (32: 217 us).
  const int64_t planeN = g.N[1] * g.N[2];
  int chunk = (int)std::min<int64_t>(32, std::max<int64_t>(2, planeN / 2048));
  while (chunk > 2 && g.N[0] % chunk) chunk >>= 1;
  if (chunk > g.N[0]) chunk = (int)g.N[0];  // N1 >= 4 is a power of two: chunk >= 2 = PF
  const int64_t nchunks = g.N[0] / chunk;
  const int64_t nblk = tiles2 * tiles3 * nchunks;
  const size_t lds = 3 * 4 * kPlaneSites * sizeof(cx<float>);
  const bool nt = (size_t)B * 4 * (size_t)g.V * sizeof(cx<float>) >= kNtBytes;
  auto kern = g.sparse3 ? (nt ? k_step3d_ring<float, 2, true, true> : k_step3d_ring<float, 2, true, false>)
                        : (nt ? k_step3d_ring<float, 2, false, true> : k_step3d_ring<float, 2, false, false>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk, (unsigned)B), dim3(kStepThreads), lds, st,
                     (cx<float>*)out, (const cx<float>*)in, g, (const StencilCoef<float>*)coefs,
                     chunk, tiles2, tiles3, nchunks);
  return hipGetLastError();
}

// Two steps per launch (temporal blocking of the update rule of Sec. 2):
// psi(t+2) from psi(t) with one read and one write of the field. A
// workgroup owns a TN2 x TN3 tile of (n2, n3) outputs and a chunk of planes
// of axis 0, and keeps two rings of three LDS planes: psi(t) on the tile with
// a two-site halo, and psi(t+1) on the tile with a one-site halo. Per output
// plane n1 it stages psi(t) plane n1+2 (loaded PF planes ahead into
// registers), forms psi(t+1) plane n1+1 on its haloed region from the first
// ring, and psi(t+2) plane n1 on the tile from the second. psi(t+1) on the
// halo is formed by every tile that borders it (the price of reading psi once
// for two steps), and each site is formed by site3d_lds, as in the one-step
// kernel, so that one launch gives the same bits as two one-step launches.
// One output site per thread; the first step's halo sites go to the first
// threads, one more site each.
template <int TN2, int TN3>
struct Ring2 {
  static constexpr int A2 = TN2 + 4, A3 = TN3 + 4, AS = A2 * A3;  // psi(t) region
  static constexpr int B2 = TN2 + 2, B3 = TN3 + 2, BS = B2 * B3;  // psi(t+1) region
  static constexpr int NT = TN2 * TN3;                            // threads
  static constexpr int BH = BS - NT;                              // halo of the psi(t+1) region
  static constexpr int AX = AS - NT;                              // second psi(t) site per thread
  static constexpr size_t lds_bytes(size_t elem) { return 3 * 4 * (size_t)(AS + BS) * elem; }
};

// Halo site k < BH of the psi(t+1) region as (row, column): rows 0 and
// B2 - 1 in full, then columns 0 and B3 - 1 of the rows between.
template <int B2, int B3>
__device__ __forceinline__ void ring2_halo(int k, int& r, int& c) {
  if (k < 2 * B3) {
    r = k < B3 ? 0 : B2 - 1;
    c = k < B3 ? k : k - B3;
  } else {
    const int q = k - 2 * B3;
    r = 1 + (q >> 1);
    c = (q & 1) ? B3 - 1 : 0;
  }
}

template <typename T, int TN2, int TN3, int PF, bool SPARSE, bool NT>
__global__ __launch_bounds__(TN2 * TN3) void k_step3d_ring2(cx<T>* __restrict__ out_all,
                                                           const cx<T>* __restrict__ in_all,
                                                           StencilGeom g,
                                                           const StencilCoef<T>* __restrict__ coefs,
                                                           int chunk, int64_t tiles2,
                                                           int64_t tiles3) {
  using G = Ring2<TN2, TN3>;
  static_assert(G::AX > 0 && G::AX <= G::NT && G::BH > 0 && G::BH <= G::NT, "tile shape");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* ringA = reinterpret_cast<cx<T>*>(smem_raw);  // [slot 3][component 4][AS]
  cx<T>* ringB = ringA + 3 * 4 * G::AS;                // [slot 3][component 4][BS]
  constexpr int PA = 4 * G::AS, PB = 4 * G::BS;
  const int64_t V = g.V;
  const cx<T>* __restrict__ in = in_all + (int64_t)blockIdx.y * 4 * V;
  cx<T>* __restrict__ out = out_all + (int64_t)blockIdx.y * 4 * V;
  const StencilCoef<T> C = coefs[blockIdx.y];
  const int tid = threadIdx.x;
  // XCD-aware numbering: each XCD steps a contiguous range of (chunk, tile).
  const int64_t w = xcd_block(blockIdx.x, gridDim.x);
  const int64_t t3 = w % tiles3;
  const int64_t t2 = (w / tiles3) % tiles2;
  const int64_t ch = w / (tiles3 * tiles2);
  const int64_t b2 = t2 * TN2, b3 = t3 * TN3;
  const int64_t m1 = g.N[0] - 1, m2 = g.N[1] - 1, m3 = g.N[2] - 1;
  const int lg3 = g.lg[2];
  const int64_t planeN = g.N[1] * g.N[2];
  const int64_t a = ch * chunk;

  // psi(t) sites this thread loads: region sites tid and NT + tid (the
  // latter for tid < AX). Threads without a second site load the first one
  // twice (in bounds, never staged): unconditional loads keep the wait
  // counts exact.
  const bool twoA = tid < G::AX;
  int sA[2];
  int64_t offA[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int sidx = (h == 0 || twoA) ? tid + h * G::NT : tid;
    const int r = sidx / G::A3, c = sidx % G::A3;
    sA[h] = sidx;
    offA[h] = (((b2 - 2 + r) & m2) << lg3) | ((b3 - 2 + c) & m3);
  }
  cx<T> ld[PF][2][4];
  auto fetch = [&](cx<T> (&dst)[2][4], int64_t p) __attribute__((always_inline)) {
    const int64_t po = (p & m1) * planeN;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < 4; ++c) dst[h][c] = in[c * V + po + offA[h]];
  };
  auto stage = [&](const cx<T> (&src)[2][4], int slot) __attribute__((always_inline)) {
    cx<T>* P = ringA + slot * PA;
#pragma unroll
    for (int c = 0; c < 4; ++c) P[c * G::AS + sA[0]] = src[0][c];
    if (twoA) {
#pragma unroll
      for (int c = 0; c < 4; ++c) P[c * G::AS + sA[1]] = src[1][c];
    }
  };
  // psi(t+1) sites this thread forms: the tile site of the thread, and for
  // tid < BH one halo site. Index in region B and of the same site in A.
  const bool twoB = tid < G::BH;
  int sB[2], sBA[2];
  {
    const int r = tid / TN3 + 1, c = tid % TN3 + 1;
    sB[0] = r * G::B3 + c;
    sBA[0] = (r + 1) * G::A3 + (c + 1);
    int hr = 0, hc = 0;
    ring2_halo<G::B2, G::B3>(twoB ? tid : 0, hr, hc);
    sB[1] = hr * G::B3 + hc;
    sBA[1] = (hr + 1) * G::A3 + (hc + 1);
  }
  auto first = [&](int sm, int s0, int sp, int slotB) __attribute__((always_inline)) {
    const cx<T>* Pm = ringA + sm * PA;
    const cx<T>* P0 = ringA + s0 * PA;
    const cx<T>* Pp = ringA + sp * PA;
    cx<T>* Q = ringB + slotB * PB;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 0 || twoB) {
        cx<T> a0, a1, a2, a3;
        site3d_lds<T, SPARSE, G::A3, G::AS>(Pm, P0, Pp, sBA[h], C, a0, a1, a2, a3);
        Q[sB[h]] = a0;
        Q[G::BS + sB[h]] = a1;
        Q[2 * G::BS + sB[h]] = a2;
        Q[3 * G::BS + sB[h]] = a3;
      }
    }
  };
  const int64_t offO = ((b2 + tid / TN3) << lg3) | (b3 + tid % TN3);
  auto second = [&](int sm, int s0, int sp, int64_t p) __attribute__((always_inline)) {
    cx<T> a0, a1, a2, a3;
    site3d_lds<T, SPARSE, G::B3, G::BS>(ringB + sm * PB, ringB + s0 * PB, ringB + sp * PB, sB[0],
                                        C, a0, a1, a2, a3);
    const int64_t idx = (p & m1) * planeN + offO;
    if constexpr (NT) {
      store_nt(&out[idx], a0);
      store_nt(&out[V + idx], a1);
      store_nt(&out[2 * V + idx], a2);
      store_nt(&out[3 * V + idx], a3);
    } else {
      out[idx] = a0;
      out[V + idx] = a1;
      out[2 * V + idx] = a2;
      out[3 * V + idx] = a3;
    }
  };

  // Ring slots: psi(t) plane p in slot (p - a + 2) mod 3, psi(t+1) plane p in
  // slot (p - a + 1) mod 3. Prologue: psi(t+1) planes a-1 and a.
  fetch(ld[0], a - 2);
  stage(ld[0], 0);
  fetch(ld[0], a - 1);
  stage(ld[0], 1);
  fetch(ld[0], a);
  stage(ld[0], 2);
  fetch(ld[0], a + 1);
  __syncthreads();
  first(0, 1, 2, 0);  // psi(t+1) plane a - 1
  __syncthreads();
  stage(ld[0], 0);  // psi(t) plane a + 1 replaces plane a - 2
#pragma unroll
  for (int u = 0; u < PF; ++u) fetch(ld[u], a + 2 + u);
  __syncthreads();
  first(1, 2, 0, 1);  // psi(t+1) plane a
  __syncthreads();

  // Output plane p = a + i: stage psi(t) plane p+2 (register set i mod PF,
  // refilled with plane p+2+PF), psi(t+1) plane p+1, psi(t+2) plane p. The
  // barrier after the psi(t+1) plane also orders the next stage after this
  // plane's reads of ring A; the barrier after the stage orders the psi(t+1)
  // writes after the previous plane's reads of ring B.
  int a0s = 2, a1s = 0, a2s = 1;  // ring A slots of psi(t) planes p, p+1, p+2
  int bm = 0, b0 = 1, bp = 2;     // ring B slots of psi(t+1) planes p-1, p, p+1
  auto plane = [&](int64_t p, int u, bool refill) __attribute__((always_inline)) {
    stage(ld[u], a2s);
    if (refill) fetch(ld[u], p + 2 + PF);
    __syncthreads();
    first(a0s, a1s, a2s, bp);
    __syncthreads();
    second(bm, b0, bp, p);
    const int ta = a0s;
    a0s = a1s;
    a1s = a2s;
    a2s = ta;
    const int tb = bm;
    bm = b0;
    b0 = bp;
    bp = tb;
  };
  // chunk is a multiple of PF: all but the last PF planes refill their set.
  for (int64_t p = a; p < a + chunk - PF; p += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) plane(p + u, u, true);
  }
#pragma unroll
  for (int u = 0; u < PF; ++u) plane(a + chunk - PF + u, u, false);
}

bool step3d_ring2_ok(const StencilGeom& g) {
  return g.dim == 3 && !g.weyl && g.N[1] >= 8 && g.N[2] >= 16 && g.N[0] >= 2;
}

// Tile shape of the two-step kernel (16 x 32: 612 first-step sites per 512
// outputs, 128 KB of LDS; 8 x 64: 660, 141 KB; 16 x 16: 324 per 256, 70 KB;
// 8 x 32: 340 per 256, 74 KB — the last two fit two workgroups per CU).
static int g_ring2_shape = 0;  // 0: 16 x 32, 1: 8 x 64, 2: 16 x 16, 3: 8 x 32
static int g_ring2_chunk = 0;  // planes per workgroup; 0: from the lattice

template <int TN2, int TN3, int PF>
static hipError_t launch_ring2_t(const StencilGeom& g, int B, void* out, const void* in,
                                 const void* coefs, hipStream_t st) {
  using G = Ring2<TN2, TN3>;
  if (g.N[1] < TN2 || g.N[2] < TN3) return hipErrorInvalidValue;
  const int64_t tiles2 = g.N[1] / TN2, tiles3 = g.N[2] / TN3;
  // Planes per workgroup: 32, fewer while there would be under 2 workgroups
  // per CU (256 CUs) per instance, at least PF, at most N1.
  int chunk = 32;
  if (g_ring2_chunk > 0) {
    chunk = g_ring2_chunk;
  } else {
    while (chunk > 2 * PF && tiles2 * tiles3 * (g.N[0] / chunk) < 512) chunk >>= 1;
  }
  if (chunk > g.N[0]) chunk = (int)g.N[0];
  if (chunk < PF || chunk % PF || g.N[0] % chunk) return hipErrorInvalidValue;
  const int64_t nblk = tiles2 * tiles3 * (g.N[0] / chunk);
  if (nblk > 0x7fffffffLL || B < 1 || B > 65535) return hipErrorInvalidValue;
  const size_t lds = G::lds_bytes(sizeof(cx<float>));
  const bool nt = (size_t)B * 4 * (size_t)g.V * sizeof(cx<float>) >= kNtBytes;
  auto kern = g.sparse3 ? (nt ? k_step3d_ring2<float, TN2, TN3, PF, true, true>
                              : k_step3d_ring2<float, TN2, TN3, PF, true, false>)
                        : (nt ? k_step3d_ring2<float, TN2, TN3, PF, false, true>
                              : k_step3d_ring2<float, TN2, TN3, PF, false, false>);
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk, (unsigned)B), dim3(G::NT), lds, st,
                     (cx<float>*)out, (const cx<float>*)in, g, (const StencilCoef<float>*)coefs,
                     chunk, tiles2, tiles3);
  return hipGetLastError();
}

bool step2_ok(bool dbl, const StencilGeom& g) {
  if (dbl || !step3d_ring2_ok(g)) return false;
  switch (g_ring2_shape) {
    case 0: return g.N[1] >= 16 && g.N[2] >= 32;
    case 1: return g.N[1] >= 8 && g.N[2] >= 64;
    case 2: return g.N[1] >= 16 && g.N[2] >= 16;
    default: return g.N[1] >= 8 && g.N[2] >= 32;
  }
}

hipError_t launch_step2(bool dbl, const StencilGeom& g, int B, void* out, const void* in,
                        const void* coefs, hipStream_t st) {
  if (!step2_ok(dbl, g)) return hipErrorInvalidValue;
  switch (g_ring2_shape) {
    case 0: return launch_ring2_t<16, 32, 2>(g, B, out, in, coefs, st);
    case 1: return launch_ring2_t<8, 64, 2>(g, B, out, in, coefs, st);
    case 2: return launch_ring2_t<16, 16, 2>(g, B, out, in, coefs, st);
    default: return launch_ring2_t<8, 32, 2>(g, B, out, in, coefs, st);
  }
}

void set_step2_config(int shape, int chunk) {
  g_ring2_shape = shape;
  g_ring2_chunk = chunk;
}

hipError_t launch_step(bool dbl, const StencilGeom& g, int B, void* out, const void* in,
                       const void* coefs, hipStream_t st) {
  if (B < 1 || B > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((g.V + 255) / 256), (unsigned)B);
  StencilGeom gn = g;
  gn.nt = (size_t)B * (g.weyl ? 2 : (g.dim == 1 ? 2 : 4)) * (size_t)g.V * (dbl ? 16 : 8) >= kNtBytes;
  if (g.weyl) {
    if (g.dim < 2) return hipErrorInvalidValue;
    // complex64 lattices that hold a tile, and complex128 fields beyond the
    // last-level cache, take the LDS tile kernel (256^3 complex128: 0.351 ->
    // 0.306 ms per step); smaller complex128 fields one thread per site.
    if (step_weyl_tile_ok(g, dbl) && (!dbl || (size_t)B * 2 * (size_t)g.V * 16 >= kNtBytes))
      return launch_step_weyl_tile(dbl, gn, B, out, in, coefs, st);
    if (dbl) {
      auto C = (const StencilCoef<double>*)coefs;
      auto o = (cx<double>*)out;
      auto i = (const cx<double>*)in;
      if (g.dim == 2) hipLaunchKernelGGL((k_step_weyl<double, 2>), grid, dim3(256), 0, st, o, i, gn, C);
      else hipLaunchKernelGGL((k_step_weyl<double, 3>), grid, dim3(256), 0, st, o, i, gn, C);
    } else {
      auto C = (const StencilCoef<float>*)coefs;
      auto o = (cx<float>*)out;
      auto i = (const cx<float>*)in;
      if (g.dim == 2) hipLaunchKernelGGL((k_step_weyl<float, 2>), grid, dim3(256), 0, st, o, i, gn, C);
      else hipLaunchKernelGGL((k_step_weyl<float, 3>), grid, dim3(256), 0, st, o, i, gn, C);
    }
    return hipGetLastError();
  }
  if (!dbl && step3d_ring_ok(g)) return launch_step3d_ring(g, B, out, in, coefs, st);
  // complex128 steps whose fields (the whole batch: its instances are
  // stepped together and share the cache) exceed the last-level cache take
  // the LDS tile kernel (256^3: 0.89 -> 0.68 ms per step); smaller ones,
  // whose neighbour reads hit the cache, one thread per site (128^3: 0.070 ms
  // against 0.112). The Weyl walk uses the same rule.
  if (dbl && step3d_tile_ok(g) && (size_t)B * 4 * (size_t)g.V * 16 >= kNtBytes)
    return launch_step3d_tile(gn, B, out, in, coefs, st);
  if (dbl) {
    auto C = (const StencilCoef<double>*)coefs;
    auto o = (cx<double>*)out;
    auto i = (const cx<double>*)in;
    if (g.dim == 1) hipLaunchKernelGGL(k_step1d<double>, grid, dim3(256), 0, st, o, i, gn, C);
    else if (g.dim == 2) hipLaunchKernelGGL((k_step_nd<double, 2>), grid, dim3(256), 0, st, o, i, gn, C);
    else hipLaunchKernelGGL((k_step_nd<double, 3>), grid, dim3(256), 0, st, o, i, gn, C);
  } else {
    auto C = (const StencilCoef<float>*)coefs;
    auto o = (cx<float>*)out;
    auto i = (const cx<float>*)in;
    if (g.dim == 1) hipLaunchKernelGGL(k_step1d<float>, grid, dim3(256), 0, st, o, i, gn, C);
    else if (g.dim == 2) hipLaunchKernelGGL((k_step_nd<float, 2>), grid, dim3(256), 0, st, o, i, gn, C);
    else hipLaunchKernelGGL((k_step_nd<float, 3>), grid, dim3(256), 0, st, o, i, gn, C);
  }
  return hipGetLastError();
}

bool step1d_resident_ok(bool dbl, const StencilGeom& g) {
  const int ms = dbl ? res_max_sites<double>() : res_max_sites<float>();
  return g.dim == 1 && g.N[0] <= (int64_t)kResThreads * ms &&
         2 * g.N[0] * (dbl ? 16 : 8) <= 160 * 1024;
}

hipError_t launch_step1d_resident(bool dbl, const StencilGeom& g, int B, void* psi,
                                  const void* coefs, int64_t nsteps, hipStream_t st) {
  if (!step1d_resident_ok(dbl, g) || B < 1 || B > 65535) return hipErrorInvalidValue;
  const size_t lds = 2 * (size_t)g.N[0] * (dbl ? 16 : 8);
  if (dbl) {
    auto kern = k_step1d_resident<double>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(1, (unsigned)B), dim3(kResThreads), lds, st, (cx<double>*)psi,
                       g, (const StencilCoef<double>*)coefs, nsteps);
  } else {
    auto kern = k_step1d_resident<float>;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(1, (unsigned)B), dim3(kResThreads), lds, st, (cx<float>*)psi, g,
                       (const StencilCoef<float>*)coefs, nsteps);
  }
  return hipGetLastError();
}

}  // namespace qw
