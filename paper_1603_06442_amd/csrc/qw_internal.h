// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/qw.h"
#include "qw_fft.h"

namespace qw {

// ---------------------------------------------------------------------------
// Per-wave-vector apply parameters (fused contiguous FFT pass).
// ---------------------------------------------------------------------------
struct InstParam {  // per batch instance, device resident for batched calls
  double m, n;      // mass and n = sqrt(1 - m^2)
  double t;         // time (integer for the walk itself, any real for the interpolation)
};

struct PassGeom {
  int dim;           // 1, 2, 3
  int s;             // spinor components
  int64_t V;         // sites per instance
  int64_t N[3];      // lattice sizes
  int64_t pencils;   // pencils (of all s components) in this launch, over all instances
  int64_t ppi;       // pencils per instance in this launch
  int lg_ppi;        // log2 ppi when ppi is a power of two, else -1
  int64_t pen0;      // first pencil of each instance in this launch (slabs)
  int block_threads; // target workgroup size of the contiguous pass (0 = 256)
  int groups_per_wg; // pencil groups per workgroup (loads one group ahead); 1 = none
  int Nc;            // common denominator for the cos/sin(pi j / Nc) table
  int shift[3];      // log2(Nc / N_i)
  int lgN1;          // log2 N[1] (3D pencil index -> (j1, j2))
  int fourstep;      // 1D four-step: N = N1 * L, pencil = row k1
  int64_t N1;        // four-step rows
  const double* cs;  // cos/sin(pi j / Nc), j in [0, 2 Nc), as (cos, sin) pairs
  const float* csf;  // the same table rounded to FP32 (complex64 evolution with the omega table)
  const void* tw4;   // four-step twiddles exp(-2 pi i j / N), j in [0, N)
  double inv_scale;  // 1 / V
  InstParam single;  // used when inst == nullptr
  const InstParam* inst;
  const double* omega;  // MODE_EVOLVE_TAB: omega(q) of the plan's mass, q in storage order
};

// MODE_EVOLVE evaluates omega(q) per wave-vector (any per-instance mass);
// MODE_EVOLVE_TAB reads it from the plan's FP64 table (the plan's mass).
// MODE_APPLY_INV starts from a spectrum already in storage order (a state
// prepared in momentum space): per-instance apply, then the inverse only.
// MODE_PROJ_INV also starts from a spectrum: instance b gets the sector
// projector P_s = (I + s M_q / sin(omega)) / 2 with s = + for even b, - for
// odd b (I/2 where sin(omega) < 1e-12), times 1/V, then the inverse.
// The MODE_BCC* modes work on the cubic-supercell BCC field (Sec. 4,
// eq:bcc-dft / eq:bcc-idft) of a 3D plan whose N1 x N2 x N3 are the sizes of
// the two sublattice arrays: one launch holds a single field of 2s = 8
// components (the s components of the even sublattice, sites 2n, then those
// of the odd sublattice, sites 2n + t). MODE_BCC: forward, the a_k combine,
// D^t at kappa = pi k / N and at kappa + pi e_x, recombination, inverse.
// MODE_BCC_FWD: forward and combine (the two-sublattice spectrum);
// MODE_BCC_INV: recombination of a two-sublattice spectrum and inverse.
enum {
  MODE_EVOLVE = 0,
  MODE_FWD = 1,
  MODE_INV = 2,
  MODE_EVOLVE_TAB = 3,
  MODE_APPLY_INV = 4,
  MODE_PROJ_INV = 5,
  MODE_BCC = 6,
  MODE_BCC_FWD = 7,
  MODE_BCC_INV = 8,
  MODE_WEYL = 9,  // two-component Weyl walk (d = 2, 3): W_q^t, omega per wave-vector
  MODE_BCC_TAB = 10,  // MODE_BCC with omega(kappa) from the plan's cubic-supercell table
  MODE_WEYL_TAB = 11,  // MODE_WEYL with omega(q) from the plan's table
  MODE_APPLY_INV_TAB = 12  // MODE_APPLY_INV, one instance, omega(q) from the plan's table
};

constexpr bool is_bcc_mode(int mode) {
  return mode == MODE_BCC || mode == MODE_BCC_FWD || mode == MODE_BCC_INV || mode == MODE_BCC_TAB;
}
// Components per pencil of the contiguous pass.
constexpr int contig_components(int dim, int mode) {
  return is_bcc_mode(mode) ? 8
                           : ((dim == 1 || mode == MODE_WEYL || mode == MODE_WEYL_TAB) ? 2 : 4);
}

// ---------------------------------------------------------------------------
// Stencil coefficients, in the kernel's precision. Offsets per dimension:
//   1D: +1, -1                    (2 neighbours, full 2x2 matrices)
//   2D: (1,0), (-1,0), (0,1), (0,-1)
//   3D: (1,0,0), (0,-1,0), (0,0,-1), (-1,-1,-1),  (-1,0,0), (0,1,0), (0,0,1), (1,1,1)
// For d = 2, 3 each neighbour matrix is block diagonal: `up` acts on
// components 0,1 and `lo` on components 2,3. The on-site matrix couples the
// two halves as mass * I (components 0<->2, 1<->3); in 1D the on-site
// matrix is a full 2x2.
// ---------------------------------------------------------------------------
template <typename T>
struct StencilCoef {
  cx<T> up[8][2][2];
  cx<T> lo[8][2][2];
  cx<T> onsite[2][2];  // 1D on-site matrix; for d = 2, 3 onsite[0][0] = mass coupling
};

// 3D sparsity the plan verifies on the derived matrices: for the first four
// offsets (1,0,0), (0,-1,0), (0,0,-1), (-1,-1,-1) only row 0 of `up` and
// column 1 of `lo` are non-zero; for the other four only row 1 of `up` and
// column 0 of `lo`. (Every Weyl block of the BCC walk has rank one.)

struct StencilGeom {
  int dim;
  int64_t N[3];
  int lg[3];  // log2 N_i
  int64_t V;
  int sparse3;  // the 3D coefficients have the rank-one pattern above
  int weyl;     // two-component Weyl walk (d = 2, 3): the `up` blocks only
  int nt;       // non-temporal stores of the results (set by the launchers)
};

// Fields of at least this many bytes are written with non-temporal stores
// by the streaming passes (stencils, whole-field n2 FFT passes): larger than
// the 256 MB last-level cache, the next pass could not find them cached
// anyway, and leaving the cache to the lines still in use gains 3-6% per pass
// at 256^3; a smaller field (a 128^3 complex128 one, 134 MB) would be read
// back from the cache, and there plain stores are 20-35% faster.
constexpr size_t kNtBytes = size_t(256) << 20;

// ---------------------------------------------------------------------------
// Launchers (defined in the kernel translation units).
// ---------------------------------------------------------------------------
// Cache hints of a strided pass (bit set): kNtStore writes the results with
// non-temporal stores (for fields larger than the last-level cache whose next
// reader gains nothing from cached lines); kNtLoad reads the input with
// non-temporal loads (input read once by this pass and not again soon), in
// the LDS-staged kernels with the nt cache policy on their global-to-LDS loads.
enum : int { kNtStore = 1, kNtLoad = 2 };
hipError_t launch_fft_strided(bool dbl, int sign, int64_t L, void* out, const void* in, int64_t O,
                              int64_t I, const void* tw, hipStream_t st, int hints = 0);
// Length-256 complex64 inverse passes of large fields staged through LDS
// (on by default; the same bits either way).
void set_fft_staged(bool on);
// Planes o0 .. o0+ocount-1 of each of ncomp components (ostride elements apart).
hipError_t launch_fft_strided_slab(bool dbl, int sign, int64_t L, void* out, const void* in,
                                   int64_t ncomp, int64_t ocount, int64_t o0, int64_t ostride,
                                   int64_t I, const void* tw, hipStream_t st, int hints = 0);
// E: elements per thread of the contiguous pass (4 or 8; 0 = default 8).
hipError_t launch_fft_contig(bool dbl, int mode, int64_t L, void* out, const void* in,
                             const PassGeom& g, const void* tw, hipStream_t st, int E = 0);
hipError_t launch_omega_table(const PassGeom& g, int64_t L, double* omega, hipStream_t st);
// omega(kappa) of the cubic-supercell field at kappa = pi j / N (sublattice
// frequency indices in storage order), at the plan's mass; V doubles.
hipError_t launch_omega_bcc_table(const PassGeom& g, int64_t L, double* omega, hipStream_t st);
hipError_t launch_transpose(bool dbl, void* out, const void* in, int64_t planes, int64_t R,
                            int64_t C, hipStream_t st);
// One step of B fields back to back; coefs: DEVICE array of B StencilCoef of
// the field precision (instance b uses coefs[b]). B <= 65535.
hipError_t launch_step(bool dbl, const StencilGeom& g, int B, void* out, const void* in,
                       const void* coefs, hipStream_t st);
// Two steps of B fields in one launch (3D Dirac walk, complex64, planes of at
// least 16 x 32 sites): psi(t+2) into out from psi(t) in in (distinct).
bool step2_ok(bool dbl, const StencilGeom& g);
hipError_t launch_step2(bool dbl, const StencilGeom& g, int B, void* out, const void* in,
                        const void* coefs, hipStream_t st);
// Measurement: tile shape (0: 16 x 32, 1: 8 x 64) and planes per workgroup
// (0: chosen from the lattice) of the two-step kernel.
void set_step2_config(int shape, int chunk);
// One step of the cubic-supercell field (two sublattice arrays of 4 * V
// entries each; out and in distinct).
hipError_t launch_step_bcc(bool dbl, const StencilGeom& g, void* out, const void* in,
                           const void* coefs, hipStream_t st);
// 1D lattices with 2 N b <= 160 KB and N <= 8192: nsteps steps of B fields in
// place, each field held in LDS by one workgroup.
bool step1d_resident_ok(bool dbl, const StencilGeom& g);
hipError_t launch_step1d_resident(bool dbl, const StencilGeom& g, int B, void* psi,
                                  const void* coefs, int64_t nsteps, hipStream_t st);

// Reductions over B fields of one shape. Instance b's origin is
// origins[3b..3b+2] if `origins` is given, else c[] (B = 1).
struct ObsGeom {
  int dim;
  int s;
  int64_t N[3];
  int lg[3];
  int64_t V;
  double c[3];
};
constexpr int kObsFields = 13;  // norm2, s1[3], s2[6], ov_re, ov_im, ref_norm2
constexpr int kObsBlocks = 4096;
// Workgroups per instance of the reduction (partials need B * this * 13 doubles).
int64_t observables_blocks(const ObsGeom& g, int B);
// k-space drift sums over a spectrum in the storage order of the fused pass
// (pencils of length L): result[0] = sum |hat psi|^2, result[1] =
// sum (|P+ hat psi|^2 - |P- hat psi|^2), result[2..4] = sum grad_q omega times
// the latter (FP64; at most 2048 workgroups; partials needs (2048 + 64) *
// kObsFields doubles). L is a power of two.
hipError_t launch_kdrift(bool dbl, const PassGeom& g, int64_t L, const void* spec,
                         double* partials, double* result, hipStream_t st);
// Norm and Cartesian moments of a cubic-supercell field about g.c (Cartesian,
// torus of period 2 N_i); result in the field layout of the observables.
hipError_t launch_bcc_observables(bool dbl, const ObsGeom& g, const void* f, double* partials,
                                  double* result, hipStream_t st);
hipError_t launch_observables(bool dbl, const ObsGeom& g, int B, const void* psi, const void* ref,
                              const double* origins, double* partials, double* result,
                              hipStream_t st);

// Minimum image of n - c in [-N/2, N/2) for integer n (N a power of two),
// written with integer arithmetic: c = ci + cf with ci = floor(c), cf in
// [0, 1); for cf = 0 the image is ((n - ci + N/2) mod N) - N/2, otherwise
// ((n - ci + N/2 - 1) mod N) + 1 - cf - N/2.
struct AxisImage {
  int64_t ci;
  double cf;
  int64_t half, mask;
};

__device__ __forceinline__ AxisImage axis_image(double c, int64_t N) {
  AxisImage a;
  const double fl = floor(c);
  a.ci = (int64_t)fl;
  a.cf = c - fl;
  a.half = N / 2;
  a.mask = N - 1;
  return a;
}

__device__ __forceinline__ double min_image(int64_t n, const AxisImage& a) {
  if (a.cf == 0.0) return (double)(((n - a.ci + a.half) & a.mask) - a.half);
  return (double)(((n - a.ci + a.half - 1) & a.mask) - a.half) + (1.0 - a.cf);
}

// The same for 0 <= n < 2^30 in 32-bit arithmetic (the image depends on ci
// only modulo N, and N <= 2^16 here), for per-element use in hot loops.
struct AxisImage32 {
  int ci, half, mask;
  double cf1;  // 1 - cf, or 0 when cf = 0
  int off;     // 0 when cf = 0, else 1
};

__device__ __forceinline__ AxisImage32 axis_image32(const AxisImage& a) {
  AxisImage32 b;
  b.ci = (int)(a.ci & a.mask);
  b.half = (int)a.half;
  b.mask = (int)a.mask;
  b.off = a.cf == 0.0 ? 0 : 1;
  b.cf1 = a.cf == 0.0 ? 0.0 : 1.0 - a.cf;
  return b;
}

__device__ __forceinline__ double min_image32(int n, const AxisImage32& a) {
  return (double)(((n - a.ci + a.half - a.off) & a.mask) - a.half) + a.cf1;
}

// Block sum of NF doubles per thread, for blockDim.x a multiple of 64 up to
// 1024; thread f < NF writes field f to dst[f].
template <int NF>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NF], double* __restrict__ dst) {
  __shared__ double red[NF][16];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    double v = acc[f];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[f][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < NF) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
    dst[threadIdx.x] = s;
  }
}

// The Sec. 5.2 reductions fused into the last (inverse, strided) pass of an
// evolution. The pass runs along axis 0 of the lattice (d = 2, 3: position
// n_1 = index along the pass, the column index holds the other axes) or,
// for the 1D four-step, along n1 of x = n1 * I + column. Every workgroup
// writes one partial vector of kObsFields doubles (overlap fields zero).
struct ObsFuse {
  int dim;
  int64_t N[3];
  int lg[3];
  double c[3];             // origin of instance 0 when origins is null
  const double* origins;   // [B][3] or null
  double* partials;        // [B][s * column blocks][kObsFields]
  int store;               // write the transformed field too
};
// Column blocks per component of the fused pass (partials per instance are
// s times this), or 0 if the pass cannot take the fused reduction (workgroup
// not a multiple of 64 threads).
int64_t strided_obs_blocks(bool dbl, int64_t L, int64_t I);
// Inverse transform along L (stride I) of B instances of s components,
// whole fields, with the reductions of `f`. hints: kNtLoad, kNtStore, taken
// by the LDS-staged form of the pass (the register forms ignore them).
hipError_t launch_fft_strided_obs(bool dbl, int64_t L, void* out, const void* in, int s, int B,
                                  int64_t I, const ObsFuse& f, const void* tw, hipStream_t st,
                                  int hints = 0);
// Sums nb partial vectors of kObsFields doubles per instance into
// result[B][kObsFields], through `mid` (B * 64 * kObsFields doubles), in a
// fixed order.
hipError_t launch_reduce_partials(int B, int64_t nb, const double* partials, double* mid,
                                  double* result, hipStream_t st);

// Marginals along the Cartesian axes: site n adds |psi(n)|^2 to bin
// off[i] + (H w)_i - xmin[i] of axis i, w the minimum image of n - c for the
// integer origin c (taken modulo N).
struct MargGeom {
  int dim;
  int64_t N[3];
  int lg[3];
  int64_t V;
  int s;
  int c[3];      // origin modulo N
  int H[3][3];   // generators as rows of Cartesian components
  int xmin[3];
  int off[3];
  int total;     // bins over all axes
};
// Workgroups of the marginal reduction (partials need this * total doubles).
int64_t marginal_blocks(const MargGeom& g);
// out_dev[total]: the marginals; partials: marginal_blocks * total doubles.
hipError_t launch_marginals(bool dbl, const MargGeom& g, const void* psi, double* partials,
                            double* out_dev, hipStream_t st);

// Particle states: shape, and the per-instance parameters (device array).
struct StateGeom {
  int dim;
  int s;
  int64_t N[3];
  int lg[3];
  int64_t V;
  int Nc;
  int shift[3];
  const double* cs;
};
struct StateInst {
  double m, n, sigma, c_plus, c_minus;
  double q0[3];
  double center[3];
  double chi_p[4][2];  // chi_+ (re, im)
  double chi_m[4][2];  // chi_-
  // Dispersive approximation (order >= 0): the + sector is multiplied by
  // e^{-i tdisp T(dk)}, the - sector by e^{+i tdisp T(dk)}, with T the Taylor
  // polynomial of omega about k0 in dk = k(q) - k0 (wrapped q):
  // tay[0] + tay[1..3] . dk + tay[4..6] . dk^2 + tay[7] dk_x dk_y
  // + tay[8] dk_x dk_z + tay[9] dk_y dk_z.
  int order;  // -1: none
  double tdisp;
  double tay[10];
};
int64_t state_blocks(const StateGeom& g, int B);
// norms[2b], norms[2b+1]: squared norms of the two sector amplitudes of
// instance b; the fill pass writes the normalised spectrum of every instance.
// scratch: state_scratch_doubles(g, B) doubles (partial sums and the
// per-axis Gaussian/carrier tables of every instance).
int64_t state_scratch_doubles(const StateGeom& g, int B);
hipError_t launch_state_prepare(bool dbl, const StateGeom& g, int B, const StateInst* inst,
                                double* scratch, double* norms, void* out, hipStream_t st);

// Non-temporal store of one complex value (not kept in the caches).
template <typename T>
__device__ __forceinline__ void store_nt(cx<T>* p, cx<T> v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<v2*>(p));
}

// Non-temporal load of one complex value.
template <typename T>
__device__ __forceinline__ cx<T> load_nt(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 w = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return mk(w.x, w.y);
}

// Kernel-side helpers shared by the apply and the state preparation:
// u_k and n~_k of the Weyl symbol at lattice frequency indices (j1, j2, j3),
// q_i = 2 pi j_i / N_i, read from the (cos, sin)(pi j / Nc) table.
__device__ __forceinline__ void weyl_un(int dim, const double* __restrict__ cs, int Nc,
                                        const int* shift, int64_t j1, int64_t j2, int64_t j3,
                                        double& u, double& n1, double& n2, double& n3) {
  const int64_t twoNc = 2 * (int64_t)Nc;
  const int64_t a1 = j1 << shift[0];
  if (dim == 1) {
    const int64_t jj = (2 * a1) & (twoNc - 1);
    u = cs[2 * jj];
    n1 = 0.0;
    n2 = 0.0;
    n3 = cs[2 * jj + 1];
    return;
  }
  const int64_t a2 = j2 << shift[1];
  if (dim == 2) {
    // k_x = (q1 + q2) / 2, k_y = (q1 - q2) / 2.
    const int64_t jx = (a1 + a2) & (twoNc - 1);
    const int64_t jy = (a1 - a2 + twoNc) & (twoNc - 1);
    const double cx_ = cs[2 * jx], sx = cs[2 * jx + 1];
    const double cy = cs[2 * jy], sy = cs[2 * jy + 1];
    u = cx_ * cy;
    n1 = sx * cy;
    n2 = cx_ * sy;
    n3 = sx * sy;
    return;
  }
  // 3D: k_x = (q1 + q2)/2, k_y = (q1 + q3)/2, k_z = -(q2 + q3)/2.
  const int64_t a3 = j3 << shift[2];
  const int64_t jx = (a1 + a2) & (twoNc - 1);
  const int64_t jy = (a1 + a3) & (twoNc - 1);
  const int64_t jz = (a2 + a3) & (twoNc - 1);
  const double cx_ = cs[2 * jx], sx = cs[2 * jx + 1];
  const double cy = cs[2 * jy], sy = cs[2 * jy + 1];
  const double cz = cs[2 * jz], sz = -cs[2 * jz + 1];
  u = cx_ * cy * cz + sx * sy * sz;
  n1 = sx * cy * cz - cx_ * sy * sz;
  n2 = cx_ * sy * cz + sx * cy * sz;
  n3 = cx_ * cy * sz - sx * sy * cz;
}

// Map (pencil, position) of the contiguous pass to lattice frequency indices.
template <int DIM>
__device__ __forceinline__ void q_index(const PassGeom& g, int64_t pen, int64_t z, int64_t& j1,
                                        int64_t& j2, int64_t& j3) {
  j2 = 0;
  j3 = 0;
  if constexpr (DIM == 3) {
    j1 = pen >> g.lgN1;
    j2 = pen & (g.N[1] - 1);
    j3 = z;
  } else if constexpr (DIM == 2) {
    j1 = pen;
    j2 = z;
  } else {
    j1 = g.fourstep ? pen + g.N1 * z : z;
  }
}

}  // namespace qw
