// Reductions over a field (Sec. 5.2 position expectation, Sec. 5.1 overlap)
// and the particle-state preparation of Sec. 5.1 (Definition 1) and Sec. 5.2
// (particle/antiparticle superposition). Accumulation is FP64 for both field
// precisions; each workgroup writes one partial vector, a second one-block
// kernel adds the partials in a fixed order (deterministic results).
#include "qw_internal.h"

namespace qw {

// Each thread takes UNR sites per round, all loads of a round issued before
// any arithmetic; FP64 accumulation.
template <typename T, int DIM, bool REF, int S>
__global__ __launch_bounds__(256) void k_observables(const cx<T>* __restrict__ psi_all,
                                                     const cx<T>* __restrict__ ref_all, ObsGeom g,
                                                     const double* __restrict__ origins,
                                                     double* __restrict__ partials_all) {
  constexpr int UNR = 4;
  const int64_t inst = blockIdx.y;
  const cx<T>* __restrict__ psi = psi_all + inst * S * g.V;
  const cx<T>* __restrict__ ref = REF ? ref_all + inst * S * g.V : nullptr;
  double* __restrict__ partials = partials_all + inst * (int64_t)gridDim.x * kObsFields;
  double acc[kObsFields];
#pragma unroll
  for (int f = 0; f < kObsFields; ++f) acc[f] = 0.0;
  AxisImage ax[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) ax[i] = axis_image(origins ? origins[3 * inst + i] : g.c[i], g.N[i]);
  const int64_t V = g.V;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  auto site = [&](int64_t idx, const cx<T> (&a)[S], const cx<T> (&r)[S]) {
    double p = 0.0, ore = 0.0, oim = 0.0, rn = 0.0;
#pragma unroll
    for (int c = 0; c < S; ++c) {
      const double ax_ = (double)a[c].x, ay = (double)a[c].y;
      p += ax_ * ax_ + ay * ay;
      if constexpr (REF) {
        const double rx = (double)r[c].x, ry = (double)r[c].y;
        ore += rx * ax_ + ry * ay;
        oim += rx * ay - ry * ax_;
        rn += rx * rx + ry * ry;
      }
    }
    double w0 = 0.0, w1 = 0.0, w2 = 0.0;
    if constexpr (DIM == 1) {
      w0 = min_image(idx, ax[0]);
    } else if constexpr (DIM == 2) {
      w1 = min_image(idx & (g.N[1] - 1), ax[1]);
      w0 = min_image(idx >> g.lg[1], ax[0]);
    } else {
      w2 = min_image(idx & (g.N[2] - 1), ax[2]);
      w1 = min_image((idx >> g.lg[2]) & (g.N[1] - 1), ax[1]);
      w0 = min_image(idx >> (g.lg[2] + g.lg[1]), ax[0]);
    }
    acc[0] += p;
    acc[1] += w0 * p;
    acc[2] += w1 * p;
    acc[3] += w2 * p;
    acc[4] += w0 * w0 * p;
    acc[5] += w1 * w1 * p;
    acc[6] += w2 * w2 * p;
    acc[7] += w0 * w1 * p;
    acc[8] += w0 * w2 * p;
    acc[9] += w1 * w2 * p;
    if constexpr (REF) {
      acc[10] += ore;
      acc[11] += oim;
      acc[12] += rn;
    }
  };
  int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // Full rounds: every load unconditional, all issued before any use.
  for (; i0 + (UNR - 1) * stride < V; i0 += UNR * stride) {
    cx<T> a[UNR][S], r[UNR][S];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int c = 0; c < S; ++c) {
        a[u][c] = psi[c * V + i0 + u * stride];
        if constexpr (REF) r[u][c] = ref[c * V + i0 + u * stride];
      }
#pragma unroll
    for (int u = 0; u < UNR; ++u) site(i0 + u * stride, a[u], r[u]);
  }
  // Tail: at most UNR - 1 sites per thread.
  for (; i0 < V; i0 += stride) {
    cx<T> a[S], r[S];
#pragma unroll
    for (int c = 0; c < S; ++c) {
      a[c] = psi[c * V + i0];
      if constexpr (REF) r[c] = ref[c * V + i0];
    }
    site(i0, a, r);
  }
  block_reduce_store<kObsFields>(acc, partials + (int64_t)blockIdx.x * kObsFields);
}

// Per-instance final sums: block b adds the nblk partial vectors of instance b.
template <int NF>
__global__ __launch_bounds__(256) void k_reduce_final_b(const double* __restrict__ partials,
                                                        int nblk, double* __restrict__ result) {
  const int64_t b = blockIdx.x;
  double acc[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = 0.0;
  const double* p = partials + b * (int64_t)nblk * NF;
  for (int k = threadIdx.x; k < nblk; k += 256)
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] += p[(int64_t)k * NF + f];
  block_reduce_store<NF>(acc, result + b * NF);
}

// Chunked first stage: block (g, b) adds chunk g of instance b's partials.
template <int NF>
__global__ __launch_bounds__(256) void k_reduce_chunks(const double* __restrict__ partials,
                                                       int64_t nblk, double* __restrict__ mid) {
  const int64_t b = blockIdx.y;
  const int64_t ng = gridDim.x;
  const int64_t lo = nblk * blockIdx.x / ng, hi = nblk * (blockIdx.x + 1) / ng;
  double acc[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = 0.0;
  const double* p = partials + b * nblk * NF;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256)
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] += p[k * NF + f];
  block_reduce_store<NF>(acc, mid + (b * ng + blockIdx.x) * NF);
}

hipError_t launch_reduce_partials(int B, int64_t nb, const double* partials, double* mid,
                                  double* result, hipStream_t st) {
  if (nb <= 1024) {
    hipLaunchKernelGGL(k_reduce_final_b<kObsFields>, dim3((unsigned)B), dim3(256), 0, st,
                       partials, (int)nb, result);
    return hipGetLastError();
  }
  const int ng = 64;
  hipLaunchKernelGGL(k_reduce_chunks<kObsFields>, dim3(ng, (unsigned)B), dim3(256), 0, st,
                     partials, nb, mid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final_b<kObsFields>, dim3((unsigned)B), dim3(256), 0, st, mid, ng,
                     result);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k-space drift (Sec. 5.1, drift vector; Sec. 5.2, the classical part of the
// mean position). On the spectrum in the storage order of the fused pass:
//   w(q)     = |hat psi(q)|^2,
//   wd(q)    = |P+ hat psi|^2 - |P- hat psi|^2 = Re(hat psi^dag M_q hat psi) / sin(omega)
//              (P+- = (I +- M_q / sin(omega)) / 2; 0 where sin(omega) < 1e-12),
//   grad(q)  = d omega / d q_j = -n (d u / d q_j) / sin(omega)   (cos(omega) = n u),
// summed in FP64: fields 0: sum w, 1: sum wd, 2..4: sum grad_j wd.
// u is differentiated through the Cartesian k(q) of the lattice (3D:
// k = ((q1+q2)/2, (q1+q3)/2, -(q2+q3)/2); 2D: ((q1+q2)/2, (q1-q2)/2); 1D: k = q).
template <int DIM>
__device__ __forceinline__ void weyl_du(const PassGeom& g, int64_t j1, int64_t j2, int64_t j3,
                                        double (&du)[3]) {
  const int64_t twoNc = 2 * (int64_t)g.Nc;
  const int64_t a1 = j1 << g.shift[0];
  du[0] = du[1] = du[2] = 0.0;
  if constexpr (DIM == 1) {
    du[0] = -g.cs[2 * ((2 * a1) & (twoNc - 1)) + 1];
  } else if constexpr (DIM == 2) {
    const int64_t a2 = j2 << g.shift[1];
    const int64_t jx = (a1 + a2) & (twoNc - 1), jy = (a1 - a2 + twoNc) & (twoNc - 1);
    const double cx_ = g.cs[2 * jx], sx = g.cs[2 * jx + 1];
    const double cy = g.cs[2 * jy], sy = g.cs[2 * jy + 1];
    const double dx = -sx * cy, dy = -cx_ * sy;
    du[0] = 0.5 * (dx + dy);
    du[1] = 0.5 * (dx - dy);
  } else {
    const int64_t a2 = j2 << g.shift[1], a3 = j3 << g.shift[2];
    const int64_t jx = (a1 + a2) & (twoNc - 1), jy = (a1 + a3) & (twoNc - 1),
                  jz = (a2 + a3) & (twoNc - 1);
    const double cx_ = g.cs[2 * jx], sx = g.cs[2 * jx + 1];
    const double cy = g.cs[2 * jy], sy = g.cs[2 * jy + 1];
    const double cz = g.cs[2 * jz], sz = -g.cs[2 * jz + 1];
    const double dx = -sx * cy * cz + cx_ * sy * sz;
    const double dy = -cx_ * sy * cz + sx * cy * sz;
    const double dz = -cx_ * cy * sz + sx * sy * cz;
    du[0] = 0.5 * (dx + dy);
    du[1] = 0.5 * (dx - dz);
    du[2] = 0.5 * (dy - dz);
  }
}

// a^dag (sigma . n~) a for a two-spinor a.
template <typename T>
__device__ __forceinline__ double sigma_form(cx<T> a0, cx<T> a1, double n1, double n2, double n3) {
  const double x0 = a0.x, y0 = a0.y, x1 = a1.x, y1 = a1.y;
  const double re = x0 * x1 + y0 * y1, im = x0 * y1 - y0 * x1;  // conj(a0) a1
  return 2.0 * (n1 * re + n2 * im) + n3 * (x0 * x0 + y0 * y0 - x1 * x1 - y1 * y1);
}

template <typename T, int DIM, int S>
__global__ __launch_bounds__(256) void k_kdrift(const cx<T>* __restrict__ spec, PassGeom g,
                                               int lgL, double* __restrict__ partials) {
  double acc[kObsFields];
#pragma unroll
  for (int f = 0; f < kObsFields; ++f) acc[f] = 0.0;
  const int64_t V = g.V;
  const double nn = g.single.n, m = g.single.m;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < V; idx += stride) {
    const int64_t pen = idx >> lgL, z = idx & ((int64_t(1) << lgL) - 1);
    int64_t j1, j2, j3;
    q_index<DIM>(g, pen, z, j1, j2, j3);
    double u, n1, n2, n3;
    weyl_un(DIM, g.cs, g.Nc, g.shift, j1, j2, j3, u, n1, n2, n3);
    cx<T> y[S];
#pragma unroll
    for (int c = 0; c < S; ++c) y[c] = spec[c * V + idx];
    double w = 0.0;
#pragma unroll
    for (int c = 0; c < S; ++c) w += (double)y[c].x * y[c].x + (double)y[c].y * y[c].y;
    double form;  // Re(hat psi^dag M hat psi)
    if constexpr (S == 4) {
      const double cross = (double)y[0].x * y[2].x + (double)y[0].y * y[2].y +
                           (double)y[1].x * y[3].x + (double)y[1].y * y[3].y;
      form = nn * (sigma_form<T>(y[0], y[1], n1, n2, n3) - sigma_form<T>(y[2], y[3], n1, n2, n3)) -
             2.0 * m * cross;
    } else if constexpr (DIM == 1) {
      // M = n sin(q) sigma_z - m sigma_x
      const double cross = (double)y[0].x * y[1].x + (double)y[0].y * y[1].y;
      form = nn * n3 * ((double)y[0].x * y[0].x + (double)y[0].y * y[0].y -
                        (double)y[1].x * y[1].x - (double)y[1].y * y[1].y) -
             2.0 * m * cross;
    } else {
      form = sigma_form<T>(y[0], y[1], n1, n2, n3);  // Weyl walk: M = sigma . n~
    }
    const double sinw = sqrt(nn * nn * (n1 * n1 + n2 * n2 + n3 * n3) + m * m);
    acc[0] += w;
    if (sinw >= 1e-12) {
      const double isw = 1.0 / sinw;
      const double wd = form * isw;
      double du[3];
      weyl_du<DIM>(g, j1, j2, j3, du);
      acc[1] += wd;
#pragma unroll
      for (int j = 0; j < 3; ++j) acc[2 + j] += -nn * du[j] * isw * wd;
    }
  }
  block_reduce_store<kObsFields>(acc, partials + (int64_t)blockIdx.x * kObsFields);
}

// At most 2048 workgroups: their partials and the 64 of the middle stage
// fit the plan's partials buffer (at least 13 * 4096 doubles) at any shape.
int64_t kdrift_blocks(int64_t V) {
  int64_t nb = (V + 1023) / 1024;
  if (nb > 2048) nb = 2048;
  return nb < 1 ? 1 : nb;
}

hipError_t launch_kdrift(bool dbl, const PassGeom& g, int64_t L, const void* spec,
                         double* partials, double* result, hipStream_t st) {
  const int64_t nb = kdrift_blocks(g.V);
  const dim3 grid((unsigned)nb);
  int lgL = 0;
  while ((int64_t(1) << lgL) < L) ++lgL;
  if ((int64_t(1) << lgL) != L) return hipErrorInvalidValue;
#define QW_KD(T, D, S) \
  hipLaunchKernelGGL((k_kdrift<T, D, S>), grid, dim3(256), 0, st, (const cx<T>*)spec, g, lgL, partials)
  if (dbl) {
    if (g.dim == 1) QW_KD(double, 1, 2);
    else if (g.dim == 2) { if (g.s == 2) QW_KD(double, 2, 2); else QW_KD(double, 2, 4); }
    else { if (g.s == 2) QW_KD(double, 3, 2); else QW_KD(double, 3, 4); }
  } else {
    if (g.dim == 1) QW_KD(float, 1, 2);
    else if (g.dim == 2) { if (g.s == 2) QW_KD(float, 2, 2); else QW_KD(float, 2, 4); }
    else { if (g.s == 2) QW_KD(float, 3, 2); else QW_KD(float, 3, 4); }
  }
#undef QW_KD
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_partials(1, nb, partials, partials + nb * kObsFields, result, st);
}

// Cubic-supercell field (two sublattice arrays of 4 V entries, the site of
// index m in array j at the Cartesian x = 2m + j (1,1,1)): norm and Cartesian
// position moments about the Cartesian point g.c on the torus of period
// 2 N_i (Sec. 5.2, minimum image), in the field layout of k_observables.
template <typename T>
__global__ __launch_bounds__(256) void k_bcc_obs(const cx<T>* __restrict__ f, ObsGeom g,
                                                double* __restrict__ partials) {
  double acc[kObsFields];
#pragma unroll
  for (int k = 0; k < kObsFields; ++k) acc[k] = 0.0;
  AxisImage ax[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) ax[i] = axis_image(g.c[i], 2 * g.N[i]);
  const int64_t V = g.V;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < 2 * V; gid += stride) {
    const int64_t j = gid >= V ? 1 : 0;
    const int64_t site = gid - j * V;
    const cx<T>* __restrict__ p = f + j * 4 * V + site;
    double w = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cx<T> a = p[c * V];
      w += (double)a.x * a.x + (double)a.y * a.y;
    }
    const int64_t m2 = site & (g.N[2] - 1);
    const int64_t m1 = (site >> g.lg[2]) & (g.N[1] - 1);
    const int64_t m0 = site >> (g.lg[2] + g.lg[1]);
    const double w0 = min_image(2 * m0 + j, ax[0]);
    const double w1 = min_image(2 * m1 + j, ax[1]);
    const double w2 = min_image(2 * m2 + j, ax[2]);
    acc[0] += w;
    acc[1] += w0 * w;
    acc[2] += w1 * w;
    acc[3] += w2 * w;
    acc[4] += w0 * w0 * w;
    acc[5] += w1 * w1 * w;
    acc[6] += w2 * w2 * w;
    acc[7] += w0 * w1 * w;
    acc[8] += w0 * w2 * w;
    acc[9] += w1 * w2 * w;
  }
  block_reduce_store<kObsFields>(acc, partials + (int64_t)blockIdx.x * kObsFields);
}

hipError_t launch_bcc_observables(bool dbl, const ObsGeom& g, const void* f, double* partials,
                                  double* result, hipStream_t st) {
  int64_t nb = (2 * g.V + 1023) / 1024;
  if (nb > 2048) nb = 2048;  // partials and the middle stage fit 13 * 4096 doubles
  if (dbl)
    hipLaunchKernelGGL(k_bcc_obs<double>, dim3((unsigned)nb), dim3(256), 0, st,
                       (const cx<double>*)f, g, partials);
  else
    hipLaunchKernelGGL(k_bcc_obs<float>, dim3((unsigned)nb), dim3(256), 0, st,
                       (const cx<float>*)f, g, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_partials(1, nb, partials, partials + nb * kObsFields, result, st);
}

// The number of workgroups (and so the summation order) depends on the shape
// only, never on the batch: an instance reduces identically alone or batched.
int64_t observables_blocks(const ObsGeom& g, int B) {
  (void)B;
  int64_t nb = (g.V + 1023) / 1024;
  if (nb > kObsBlocks) nb = kObsBlocks;
  return nb < 1 ? 1 : nb;
}

template <typename T>
static void launch_obs_t(const ObsGeom& g, int B, const void* psi, const void* ref,
                         const double* origins, double* partials, unsigned nb, hipStream_t st) {
  auto p = (const cx<T>*)psi;
  auto r = (const cx<T>*)ref;
  const dim3 grid(nb, (unsigned)B);
#define QW_OBS(D, R, S) \
  hipLaunchKernelGGL((k_observables<T, D, R, S>), grid, dim3(256), 0, st, p, r, g, origins, partials)
  // S = 2: the 1D Dirac walk and the two-component Weyl walks of d = 2, 3.
  if (g.dim == 1) {
    if (ref) QW_OBS(1, true, 2); else QW_OBS(1, false, 2);
  } else if (g.dim == 2) {
    if (g.s == 2) { if (ref) QW_OBS(2, true, 2); else QW_OBS(2, false, 2); }
    else { if (ref) QW_OBS(2, true, 4); else QW_OBS(2, false, 4); }
  } else {
    if (g.s == 2) { if (ref) QW_OBS(3, true, 2); else QW_OBS(3, false, 2); }
    else { if (ref) QW_OBS(3, true, 4); else QW_OBS(3, false, 4); }
  }
#undef QW_OBS
}

hipError_t launch_observables(bool dbl, const ObsGeom& g, int B, const void* psi, const void* ref,
                              const double* origins, double* partials, double* result,
                              hipStream_t st) {
  const int64_t nb = observables_blocks(g, B);
  if (dbl)
    launch_obs_t<double>(g, B, psi, ref, origins, partials, (unsigned)nb, st);
  else
    launch_obs_t<float>(g, B, psi, ref, origins, partials, (unsigned)nb, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final_b<kObsFields>, dim3((unsigned)B), dim3(256), 0, st, partials,
                     (int)nb, result);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Marginals. Each workgroup accumulates its sites into a histogram in LDS
// (the order of the LDS atomic adds within a workgroup is not fixed, so
// results agree to rounding between runs); the per-workgroup histograms are
// then added bin by bin in a fixed order.
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_marginals(const cx<T>* __restrict__ psi, MargGeom g,
                                                   double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* hist = reinterpret_cast<double*>(smem_raw);
  for (int i = threadIdx.x; i < g.total; i += blockDim.x) hist[i] = 0.0;
  __syncthreads();
  const int64_t V = g.V;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < V; idx += stride) {
    double pr = 0.0;
    for (int c = 0; c < g.s; ++c) {
      const cx<T> a = psi[c * V + idx];
      pr += (double)a.x * (double)a.x + (double)a.y * (double)a.y;
    }
    int w[3] = {0, 0, 0};
    int64_t rem = idx;
#pragma unroll
    for (int j = DIM - 1; j >= 0; --j) {
      const int n = (int)(rem & (g.N[j] - 1));
      rem >>= g.lg[j];
      const int half = (int)(g.N[j] / 2);
      w[j] = ((n - g.c[j] + half) & (int)(g.N[j] - 1)) - half;
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      int X = 0;
#pragma unroll
      for (int j = 0; j < DIM; ++j) X += g.H[i][j] * w[j];
      atomicAdd(&hist[g.off[i] + X - g.xmin[i]], pr);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < g.total; i += blockDim.x)
    partials[(int64_t)blockIdx.x * g.total + i] = hist[i];
}

// 1D: every site is its own bin (no reduction).
template <typename T>
__global__ __launch_bounds__(256) void k_marginals1d(const cx<T>* __restrict__ psi, MargGeom g,
                                                     double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.V) return;
  const cx<T> a = psi[idx], b = psi[g.V + idx];
  const double pr = (double)a.x * (double)a.x + (double)a.y * (double)a.y +
                    (double)b.x * (double)b.x + (double)b.y * (double)b.y;
  const int half = (int)(g.N[0] / 2);
  const int w = (((int)idx - g.c[0] + half) & (int)(g.N[0] - 1)) - half;
  out[w - g.xmin[0]] = pr;
}

__global__ __launch_bounds__(256) void k_marginals_final(const double* __restrict__ partials,
                                                         int64_t nblk, int total,
                                                         double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  double sum = 0.0;
  for (int64_t b = 0; b < nblk; ++b) sum += partials[b * total + i];
  out[i] = sum;
}

int64_t marginal_blocks(const MargGeom& g) {
  int64_t nb = (g.V + 255) / 256;
  if (nb > 512) nb = 512;
  return nb < 1 ? 1 : nb;
}

hipError_t launch_marginals(bool dbl, const MargGeom& g, const void* psi, double* partials,
                            double* out_dev, hipStream_t st) {
  if (g.dim == 1) {
    const unsigned nb = (unsigned)((g.V + 255) / 256);
    if (dbl)
      hipLaunchKernelGGL(k_marginals1d<double>, dim3(nb), dim3(256), 0, st,
                         (const cx<double>*)psi, g, out_dev);
    else
      hipLaunchKernelGGL(k_marginals1d<float>, dim3(nb), dim3(256), 0, st, (const cx<float>*)psi,
                         g, out_dev);
    return hipGetLastError();
  }
  const size_t lds = sizeof(double) * (size_t)g.total;
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const int64_t nb = marginal_blocks(g);
#define QW_MARG(T, D)                                                                      \
  hipLaunchKernelGGL((k_marginals<T, D>), dim3((unsigned)nb), dim3(256), lds, st,          \
                     (const cx<T>*)psi, g, partials)
  if (dbl) {
    if (g.dim == 2) QW_MARG(double, 2); else QW_MARG(double, 3);
  } else {
    if (g.dim == 2) QW_MARG(float, 2); else QW_MARG(float, 3);
  }
#undef QW_MARG
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_marginals_final, dim3((unsigned)((g.total + 255) / 256)), dim3(256), 0, st,
                     partials, nb, g.total, out_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Particle states. For every q on the grid:
//   a_s(q) = exp(-sigma^2 |dq|^2 / 2) e^{+i q.c} P_s(q) chi_s,
//   P_s = (I + s M_q / sin(omega)) / 2  (I/2 where sin(omega) < 1e-12),
// with M_q and sin(omega) as in the per-q evolution, dq_j = q_j - q'_j wrapped
// to [-pi, pi). The squared norms of a_+ and a_- are reduced per instance,
// then the fill pass writes c+ a+/|a+| + c- a-/|a-|, scaled so that the
// unnormalised inverse DFT has unit norm (Parseval: |psi|^2 = V |hat psi|^2
// and the two sectors are orthogonal at every q).
// ---------------------------------------------------------------------------
// Phase t T(dk) of the dispersive approximation at wrapped dq (lattice axes).
__device__ __forceinline__ double dispersive_phase(int dim, const StateInst& si, const double* dq) {
  double k[3] = {0.0, 0.0, 0.0};
  if (dim == 1) {
    k[0] = dq[0];
  } else if (dim == 2) {
    k[0] = 0.5 * (dq[0] + dq[1]);
    k[1] = 0.5 * (dq[0] - dq[1]);
  } else {
    k[0] = 0.5 * (dq[0] + dq[1]);
    k[1] = 0.5 * (dq[0] + dq[2]);
    k[2] = -0.5 * (dq[1] + dq[2]);
  }
  const double* c = si.tay;
  double T = c[0];
  if (si.order >= 1) T += c[1] * k[0] + c[2] * k[1] + c[3] * k[2];
  if (si.order >= 2)
    T += c[4] * k[0] * k[0] + c[5] * k[1] * k[1] + c[6] * k[2] * k[2] + c[7] * k[0] * k[1] +
         c[8] * k[0] * k[2] + c[9] * k[1] * k[2];
  return si.tdisp * T;
}

// DIM is a template parameter so that every loop over axes and components
// unrolls and the per-site arrays stay in registers.
// Wrapped q_i - q0_i of lattice index j on axis i.
__device__ __forceinline__ double wrapped_dq(const StateGeom& g, const StateInst& si, int i,
                                             int64_t j) {
  const double twopi = 2.0 * M_PI;
  const double q = twopi * (double)j / (double)g.N[i];
  double d = q - si.q0[i] + M_PI;
  return d - twopi * floor(d / twopi) - M_PI;
}

// The Gaussian and the carrier factorise over the lattice axes: per instance
// a table of exp(-sigma^2 dq_i^2 / 2) e^{+i q_i c_i} for every axis i and
// index j (axis i at offset N_0 + .. + N_{i-1}), complex FP64.
__global__ __launch_bounds__(256) void k_state_table(StateGeom g, const StateInst* __restrict__ inst,
                                                     double* __restrict__ tab_all, int nsum) {
  const int64_t b = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsum) return;
  const StateInst& si = inst[b];
  int i = 0, j = t;
  while (i < g.dim - 1 && j >= g.N[i]) {
    j -= (int)g.N[i];
    ++i;
  }
  const double d = wrapped_dq(g, si, i, j);
  const double q = 2.0 * M_PI * (double)j / (double)g.N[i];
  const double amp = exp(-0.5 * si.sigma * si.sigma * d * d);
  double sp, cp;
  sincos(q * si.center[i], &sp, &cp);
  double* tab = tab_all + 2 * (b * nsum + t);
  tab[0] = amp * cp;
  tab[1] = amp * sp;
}

template <int DIM>
__device__ __forceinline__ void state_amplitudes(const StateGeom& g, const StateInst& si,
                                                 const double* __restrict__ tab, int64_t idx,
                                                 double ap[4][2], double am[4][2]) {
  constexpr int S = DIM == 1 ? 2 : 4;
  int64_t j[3] = {0, 0, 0};
  int64_t rem = idx;
#pragma unroll
  for (int i = DIM - 1; i >= 0; --i) {
    j[i] = rem & (g.N[i] - 1);
    rem >>= g.lg[i];
  }
  // g(q) = product of the per-axis factors
  double gr = tab[2 * j[0]], gi = tab[2 * j[0] + 1];
  int64_t off = g.N[0];
#pragma unroll
  for (int i = 1; i < DIM; ++i) {
    const double tr = tab[2 * (off + j[i])], ti = tab[2 * (off + j[i]) + 1];
    const double r = gr * tr - gi * ti;
    gi = gr * ti + gi * tr;
    gr = r;
    off += g.N[i];
  }

  double u, n1, n2, n3;
  weyl_un(DIM, g.cs, g.Nc, g.shift, j[0], j[1], j[2], u, n1, n2, n3);
  (void)u;
  const double nn = si.n, m = si.m;
  const double sinw = sqrt(nn * nn * (n1 * n1 + n2 * n2 + n3 * n3) + m * m);
  const double inv = sinw >= 1e-12 ? 1.0 / sinw : 0.0;
  // Mh = M / sin(omega), applied to chi (complex) for both sectors.
  auto apply_mh = [&](const double chi[4][2], double out[4][2]) {
    if constexpr (DIM == 1) {
      const double a = nn * n3 * inv, gg = -m * inv;
      out[0][0] = a * chi[0][0] + gg * chi[1][0];
      out[0][1] = a * chi[0][1] + gg * chi[1][1];
      out[1][0] = gg * chi[0][0] - a * chi[1][0];
      out[1][1] = gg * chi[0][1] - a * chi[1][1];
      return;
    }
    const double a = nn * n3 * inv, b = nn * n1 * inv, e = nn * n2 * inv, gg = -m * inv;
    // upper: n sigma.n~ chi_u - m chi_l; lower: -m chi_u - n sigma.n~ chi_l, over sin(omega)
    const double* c0 = chi[0];
    const double* c1 = chi[1];
    const double* c2 = chi[2];
    const double* c3 = chi[3];
    out[0][0] = a * c0[0] + (b * c1[0] + e * c1[1]) + gg * c2[0];
    out[0][1] = a * c0[1] + (b * c1[1] - e * c1[0]) + gg * c2[1];
    out[1][0] = (b * c0[0] - e * c0[1]) - a * c1[0] + gg * c3[0];
    out[1][1] = (b * c0[1] + e * c0[0]) - a * c1[1] + gg * c3[1];
    out[2][0] = gg * c0[0] - a * c2[0] - (b * c3[0] + e * c3[1]);
    out[2][1] = gg * c0[1] - a * c2[1] - (b * c3[1] - e * c3[0]);
    out[3][0] = gg * c1[0] - (b * c2[0] - e * c2[1]) + a * c3[0];
    out[3][1] = gg * c1[1] - (b * c2[1] + e * c2[0]) + a * c3[1];
  };
  double mp[4][2], mm[4][2];
  apply_mh(si.chi_p, mp);
  apply_mh(si.chi_m, mm);
  // Sector factors g(q) e^{-+i t T}: equal to g(q) unless dispersive.
  double gpr = gr, gpi = gi, gmr = gr, gmi = gi;
  if (si.order >= 0) {
    double dq[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < DIM; ++i) dq[i] = wrapped_dq(g, si, i, j[i]);
    double s1, c1;
    sincos(dispersive_phase(DIM, si, dq), &s1, &c1);
    gpr = gr * c1 + gi * s1;  // g e^{-i theta}
    gpi = gi * c1 - gr * s1;
    gmr = gr * c1 - gi * s1;  // g e^{+i theta}
    gmi = gi * c1 + gr * s1;
  }
#pragma unroll
  for (int c = 0; c < S; ++c) {
    // P_+ chi = (chi + Mh chi)/2, P_- chi = (chi - Mh chi)/2, times g(q).
    const double pr = 0.5 * (si.chi_p[c][0] + mp[c][0]), pi = 0.5 * (si.chi_p[c][1] + mp[c][1]);
    const double mr = 0.5 * (si.chi_m[c][0] - mm[c][0]), mi = 0.5 * (si.chi_m[c][1] - mm[c][1]);
    ap[c][0] = gpr * pr - gpi * pi;
    ap[c][1] = gpr * pi + gpi * pr;
    am[c][0] = gmr * mr - gmi * mi;
    am[c][1] = gmr * mi + gmi * mr;
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_state_norms(StateGeom g, const StateInst* __restrict__ inst,
                                                     const double* __restrict__ tab_all, int nsum,
                                                     double* __restrict__ partials) {
  constexpr int S = DIM == 1 ? 2 : 4;
  const int64_t b = blockIdx.y;
  const StateInst& si = inst[b];
  const double* __restrict__ tab = tab_all + 2 * b * nsum;
  double acc[2] = {0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < g.V; idx += stride) {
    double ap[4][2], am[4][2];
    state_amplitudes<DIM>(g, si, tab, idx, ap, am);
#pragma unroll
    for (int c = 0; c < S; ++c) {
      acc[0] += ap[c][0] * ap[c][0] + ap[c][1] * ap[c][1];
      acc[1] += am[c][0] * am[c][0] + am[c][1] * am[c][1];
    }
  }
  block_reduce_store<2>(acc, partials + (b * gridDim.x + blockIdx.x) * 2);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_state_fill(StateGeom g, const StateInst* __restrict__ inst,
                                                    const double* __restrict__ tab_all, int nsum,
                                                    const double* __restrict__ norms,
                                                    cx<T>* __restrict__ out_all) {
  constexpr int S = DIM == 1 ? 2 : 4;
  const int64_t b = blockIdx.y;
  const StateInst& si = inst[b];
  const double* __restrict__ tab = tab_all + 2 * b * nsum;
  const double np = norms[2 * b], nm = norms[2 * b + 1];
  const double total = sqrt((double)g.V * (si.c_plus * si.c_plus + si.c_minus * si.c_minus));
  const double coef_p = (si.c_plus != 0.0 && np > 0.0) ? si.c_plus / sqrt(np) / total : 0.0;
  const double coef_m = (si.c_minus != 0.0 && nm > 0.0) ? si.c_minus / sqrt(nm) / total : 0.0;
  cx<T>* __restrict__ out = out_all + b * S * g.V;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < g.V; idx += stride) {
    double ap[4][2], am[4][2];
    state_amplitudes<DIM>(g, si, tab, idx, ap, am);
#pragma unroll
    for (int c = 0; c < S; ++c) {
      const double re = coef_p * ap[c][0] + coef_m * am[c][0];
      const double im = coef_p * ap[c][1] + coef_m * am[c][1];
      out[c * g.V + idx] = mk((T)re, (T)im);
    }
  }
}

int64_t state_blocks(const StateGeom& g, int B) {
  (void)B;
  int64_t nb = (g.V + 255) / 256;
  if (nb > 1024) nb = 1024;
  return nb < 1 ? 1 : nb;
}

int64_t state_scratch_doubles(const StateGeom& g, int B) {
  int64_t nsum = 0;
  for (int i = 0; i < g.dim; ++i) nsum += g.N[i];
  return (int64_t)B * (2 * state_blocks(g, B) + 2 * nsum);
}

hipError_t launch_state_prepare(bool dbl, const StateGeom& g, int B, const StateInst* inst,
                                double* scratch, double* norms, void* out, hipStream_t st) {
  const int64_t nb = state_blocks(g, B);
  int nsum = 0;
  for (int i = 0; i < g.dim; ++i) nsum += (int)g.N[i];
  double* partials = scratch;
  double* tab = scratch + (size_t)B * nb * 2;
  hipLaunchKernelGGL(k_state_table, dim3((unsigned)((nsum + 255) / 256), (unsigned)B), dim3(256), 0,
                     st, g, inst, tab, nsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 gn((unsigned)nb, (unsigned)B);
  if (g.dim == 1) hipLaunchKernelGGL(k_state_norms<1>, gn, dim3(256), 0, st, g, inst, tab, nsum, partials);
  else if (g.dim == 2) hipLaunchKernelGGL(k_state_norms<2>, gn, dim3(256), 0, st, g, inst, tab, nsum, partials);
  else hipLaunchKernelGGL(k_state_norms<3>, gn, dim3(256), 0, st, g, inst, tab, nsum, partials);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final_b<2>, dim3((unsigned)B), dim3(256), 0, st, partials, (int)nb,
                     norms);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t nf = (g.V + 255) / 256;
  if (nf > 65536) nf = 65536;
  const dim3 gf((unsigned)nf, (unsigned)B);
#define QW_FILL(T, D) \
  hipLaunchKernelGGL((k_state_fill<T, D>), gf, dim3(256), 0, st, g, inst, tab, nsum, norms, (cx<T>*)out)
  if (dbl) {
    if (g.dim == 1) QW_FILL(double, 1); else if (g.dim == 2) QW_FILL(double, 2); else QW_FILL(double, 3);
  } else {
    if (g.dim == 1) QW_FILL(float, 1); else if (g.dim == 2) QW_FILL(float, 2); else QW_FILL(float, 3);
  }
#undef QW_FILL
  return hipGetLastError();
}

}  // namespace qw
