// Position-space step of the walk (Sec. 2 of the paper, update rule):
//   psi(n, t+1) = sum_h U_h psi(n + h, t)   on the periodic N^d torus,
// with the transition matrices U_h derived by the plan from the symbol.
// One thread per output site computes all s components; neighbour reads are
// served by L1/L2 (each input is used by up to 2d+3 sites).
#include "qw_internal.h"

namespace qw {

template <typename T>
__device__ __forceinline__ cx<T> fma_c(cx<T> acc, cx<T> a, cx<T> b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
  return acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_step1d(cx<T>* __restrict__ out, const cx<T>* __restrict__ in,
                                               StencilGeom g, StencilCoef<T> C) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.V) return;
  const int64_t msk = g.N[0] - 1;
  const int64_t r = (n + 1) & msk, l = (n - 1) & msk;
  const int64_t V = g.V;
  const cx<T> p0 = in[n], p1 = in[V + n];
  const cx<T> r0 = in[r], r1 = in[V + r];
  const cx<T> l0 = in[l], l1 = in[V + l];
  cx<T> a0 = mk((T)0, (T)0), a1 = a0;
  // U_{+1} acts on psi(n+1), U_{-1} on psi(n-1), U_0 on psi(n).
  a0 = fma_c(a0, C.up[0][0][0], r0); a0 = fma_c(a0, C.up[0][0][1], r1);
  a1 = fma_c(a1, C.up[0][1][0], r0); a1 = fma_c(a1, C.up[0][1][1], r1);
  a0 = fma_c(a0, C.up[1][0][0], l0); a0 = fma_c(a0, C.up[1][0][1], l1);
  a1 = fma_c(a1, C.up[1][1][0], l0); a1 = fma_c(a1, C.up[1][1][1], l1);
  a0 = fma_c(a0, C.onsite[0][0], p0); a0 = fma_c(a0, C.onsite[0][1], p1);
  a1 = fma_c(a1, C.onsite[1][0], p0); a1 = fma_c(a1, C.onsite[1][1], p1);
  out[n] = a0;
  out[V + n] = a1;
}

__device__ constexpr int kOff2[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
__device__ constexpr int kOff3[8][3] = {{1, 0, 0},  {0, -1, 0}, {0, 0, -1}, {-1, -1, -1},
                                        {-1, 0, 0}, {0, 1, 0},  {0, 0, 1},  {1, 1, 1}};

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_step_nd(cx<T>* __restrict__ out, const cx<T>* __restrict__ in,
                                                StencilGeom g, StencilCoef<T> C) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.V) return;
  const int64_t V = g.V;
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
  out[idx] = a0;
  out[V + idx] = a1;
  out[2 * V + idx] = a2;
  out[3 * V + idx] = a3;
}

hipError_t launch_step(bool dbl, const StencilGeom& g, void* out, const void* in,
                       const void* coef, hipStream_t st) {
  const unsigned nblk = (unsigned)((g.V + 255) / 256);
  if (dbl) {
    const StencilCoef<double>& C = *(const StencilCoef<double>*)coef;
    auto o = (cx<double>*)out;
    auto i = (const cx<double>*)in;
    if (g.dim == 1) hipLaunchKernelGGL(k_step1d<double>, dim3(nblk), dim3(256), 0, st, o, i, g, C);
    else if (g.dim == 2) hipLaunchKernelGGL((k_step_nd<double, 2>), dim3(nblk), dim3(256), 0, st, o, i, g, C);
    else hipLaunchKernelGGL((k_step_nd<double, 3>), dim3(nblk), dim3(256), 0, st, o, i, g, C);
  } else {
    const StencilCoef<float>& C = *(const StencilCoef<float>*)coef;
    auto o = (cx<float>*)out;
    auto i = (const cx<float>*)in;
    if (g.dim == 1) hipLaunchKernelGGL(k_step1d<float>, dim3(nblk), dim3(256), 0, st, o, i, g, C);
    else if (g.dim == 2) hipLaunchKernelGGL((k_step_nd<float, 2>), dim3(nblk), dim3(256), 0, st, o, i, g, C);
    else hipLaunchKernelGGL((k_step_nd<float, 3>), dim3(nblk), dim3(256), 0, st, o, i, g, C);
  }
  return hipGetLastError();
}

}  // namespace qw
