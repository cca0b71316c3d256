// C ABI of libqw: plans, argument validation, the pass schedule of the
// Fourier evolution, stepping, reductions and state preparation.
//
// Host-side arithmetic of the walk (FP64): the Weyl/Dirac symbols of
// Sec. 3.1-3.2 of the paper, the transition matrices U_h of the update rule
// obtained from the symbol by an exact inverse DFT on a 4^d grid (Sec. 2.1:
// U_k = sum_h e^{-ik.h} U_h; the symbol's support is within one cell, so a
// grid of 4 points per axis separates the offsets -1, 0, 1), the check of
// the unitarity conditions of Sec. 2 on them, and the spinors chi_s of the
// particle states.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <mutex>
#include <new>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "plan.h"

using namespace qw;

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace qw {
qw_status fail(qw_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}
}  // namespace qw

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int lg2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}

// --- symbols (Sec. 3.1, 3.2) ------------------------------------------------

// u_k and n~_k of the Weyl walk at Cartesian k.
void weyl_un_host(int dim, const double k[3], double& u, double nt[3]) {
  if (dim == 1) {
    u = cos(k[0]);
    nt[0] = 0.0;
    nt[1] = 0.0;
    nt[2] = sin(k[0]);
    return;
  }
  const double cx = cos(k[0]), sx = sin(k[0]), cy = cos(k[1]), sy = sin(k[1]);
  if (dim == 2) {
    u = cx * cy;
    nt[0] = sx * cy;
    nt[1] = cx * sy;
    nt[2] = sx * sy;
    return;
  }
  const double cz = cos(k[2]), sz = sin(k[2]);
  u = cx * cy * cz + sx * sy * sz;
  nt[0] = sx * cy * cz - cx * sy * sz;
  nt[1] = cx * sy * cz + sx * cy * sz;
  nt[2] = cx * cy * sz - sx * sy * cz;
}

// Cartesian k of lattice q (q_j = k . h_j).
void k_of_q(int dim, const double q[3], double k[3]) {
  k[0] = k[1] = k[2] = 0.0;
  if (dim == 1) {
    k[0] = q[0];
  } else if (dim == 2) {
    k[0] = 0.5 * (q[0] + q[1]);
    k[1] = 0.5 * (q[0] - q[1]);
  } else {
    k[0] = 0.5 * (q[0] + q[1]);
    k[1] = 0.5 * (q[0] + q[2]);
    k[2] = -0.5 * (q[1] + q[2]);
  }
}

// Lattice q of Cartesian k.
void q_of_k(int dim, const double k[3], double q[3]) {
  q[0] = q[1] = q[2] = 0.0;
  if (dim == 1) {
    q[0] = k[0];
  } else if (dim == 2) {
    q[0] = k[0] + k[1];
    q[1] = k[0] - k[1];
  } else {
    q[0] = k[0] + k[1] + k[2];
    q[1] = k[0] - k[1] - k[2];
    q[2] = -k[0] + k[1] - k[2];
  }
}

// M of D = cos(omega) I - i M at Cartesian k (block form of Sec. 3.2), and sin(omega).
void dirac_M(int dim, const double k[3], double m, zc M[4][4], double& cosw, double& sinw) {
  const double n = sqrt(1.0 - m * m);
  double u, nt[3];
  weyl_un_host(dim, k, u, nt);
  cosw = n * u;
  sinw = sqrt(n * n * (nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]) + m * m);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) M[i][j] = 0.0;
  if (dim == 1) {
    M[0][0] = n * nt[2];
    M[1][1] = -n * nt[2];
    M[0][1] = -m;
    M[1][0] = -m;
    return;
  }
  const zc sn[2][2] = {{nt[2], zc(nt[0], -nt[1])}, {zc(nt[0], nt[1]), -nt[2]}};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      M[i][j] = n * sn[i][j];
      M[i + 2][j + 2] = -n * sn[i][j];
    }
  for (int i = 0; i < 2; ++i) {
    M[i][i + 2] = -m;
    M[i + 2][i] = -m;
  }
}

// The Dirac symbol D(q) at lattice q: [[n W, i m], [i m, n W^dag]] (1D: 2x2 form).
void dirac_symbol(int dim, const double q[3], double m, zc D[4][4]) {
  double k[3];
  k_of_q(dim, q, k);
  const double n = sqrt(1.0 - m * m);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) D[i][j] = 0.0;
  if (dim == 1) {
    D[0][0] = n * std::exp(zc(0.0, -k[0]));
    D[1][1] = n * std::exp(zc(0.0, k[0]));
    D[0][1] = zc(0.0, m);
    D[1][0] = zc(0.0, m);
    return;
  }
  double u, nt[3];
  weyl_un_host(dim, k, u, nt);
  // W = u I - i sigma . n~
  const zc W[2][2] = {{zc(u, -nt[2]), zc(-nt[1], -nt[0])}, {zc(nt[1], -nt[0]), zc(u, nt[2])}};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      D[i][j] = n * W[i][j];
      D[i + 2][j + 2] = n * std::conj(W[j][i]);
    }
  for (int i = 0; i < 2; ++i) {
    D[i][i + 2] = zc(0.0, m);
    D[i + 2][i] = zc(0.0, m);
  }
}

// --- transition matrices ----------------------------------------------------


int off_index(int dim, const int* o) {
  int idx = 0;
  for (int i = 0; i < dim; ++i) idx = idx * 3 + (o[i] + 1);
  return idx;
}

// U_h = 4^-d sum_{q in grid} e^{+i q.h} D(q); also reports any weight at offset 2.
double derive_table(int dim, double m, Table& T) {
  const int s = dim == 1 ? 2 : 4;
  T.dim = dim;
  T.s = s;
  const int L = 4;
  int npts = 1;
  for (int i = 0; i < dim; ++i) npts *= L;
  double leak = 0.0;
  std::vector<zc> acc(4 * 4 * 64, zc(0.0));  // offsets in {-1,0,1,2}^d -> 4^d slots
  for (int p = 0; p < npts; ++p) {
    double q[3] = {0, 0, 0};
    int j[3] = {0, 0, 0};
    int r = p;
    for (int i = dim - 1; i >= 0; --i) {
      j[i] = r % L;
      r /= L;
      q[i] = 2.0 * M_PI * j[i] / L;
    }
    zc D[4][4];
    dirac_symbol(dim, q, m, D);
    for (int o = 0; o < npts; ++o) {
      int off[3] = {0, 0, 0};
      int rr = o;
      for (int i = dim - 1; i >= 0; --i) {
        off[i] = rr % L - 1;  // -1, 0, 1, 2
        rr /= L;
      }
      double ph = 0.0;
      for (int i = 0; i < dim; ++i) ph += q[i] * off[i];
      const zc e = std::exp(zc(0.0, ph));
      for (int a = 0; a < s; ++a)
        for (int b = 0; b < s; ++b) acc[(o * 4 + a) * 4 + b] += e * D[a][b];
    }
  }
  for (int i = 0; i < 27; ++i)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) T.U[i][a][b] = 0.0;
  for (int o = 0; o < npts; ++o) {
    int off[3] = {0, 0, 0};
    int rr = o;
    bool far = false;
    for (int i = dim - 1; i >= 0; --i) {
      off[i] = rr % L - 1;
      rr /= L;
      if (off[i] == 2) far = true;
    }
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) {
        zc v = acc[(o * 4 + a) * 4 + b] / (double)npts;
        if (std::abs(v.real()) < 1e-15) v.real(0.0);
        if (std::abs(v.imag()) < 1e-15) v.imag(0.0);
        if (far)
          leak = fmax(leak, std::abs(v));
        else
          T.U[off_index(dim, off)][a][b] = v;
      }
  }
  return leak;
}

// Largest violation of the unitarity conditions (Sec. 2) over the table.
double unitarity_defect(const Table& T) {
  const int dim = T.dim, s = T.s;
  int n = 1;
  for (int i = 0; i < dim; ++i) n *= 3;
  double worst = 0.0;
  // sum_h U_h^dag U_{h + d} and sum_h U_{h + d} U_h^dag for every shift d in {-2..2}^dim
  int nd = 1;
  for (int i = 0; i < dim; ++i) nd *= 5;
  for (int di = 0; di < nd; ++di) {
    int dd[3] = {0, 0, 0};
    int r = di;
    bool zero = true;
    for (int i = dim - 1; i >= 0; --i) {
      dd[i] = r % 5 - 2;
      r /= 5;
      if (dd[i]) zero = false;
    }
    zc A[4][4], B[4][4];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) A[a][b] = B[a][b] = 0.0;
    for (int h = 0; h < n; ++h) {
      int o[3] = {0, 0, 0}, o2[3] = {0, 0, 0};
      int rr = h;
      bool ok = true;
      for (int i = dim - 1; i >= 0; --i) {
        o[i] = rr % 3 - 1;
        rr /= 3;
        o2[i] = o[i] + dd[i];
        if (o2[i] < -1 || o2[i] > 1) ok = false;
      }
      if (!ok) continue;
      const int h2 = off_index(dim, o2);
      for (int a = 0; a < s; ++a)
        for (int b = 0; b < s; ++b)
          for (int c = 0; c < s; ++c) {
            A[a][b] += std::conj(T.U[h][c][a]) * T.U[h2][c][b];
            B[a][b] += T.U[h2][a][c] * std::conj(T.U[h][b][c]);
          }
    }
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) {
        const double id = (zero && a == b) ? 1.0 : 0.0;
        worst = fmax(worst, std::abs(A[a][b] - id));
        worst = fmax(worst, std::abs(B[a][b] - id));
      }
  }
  return worst;
}

const int kOff2h[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
const int kOff3h[8][3] = {{1, 0, 0},  {0, -1, 0}, {0, 0, -1}, {-1, -1, -1},
                          {-1, 0, 0}, {0, 1, 0},  {0, 0, 1},  {1, 1, 1}};

// Fill the kernel coefficient struct; check that everything the kernel does
// not read is zero (block-diagonal neighbours, mass coupling on site).
// The rank-one pattern of the 3D neighbour blocks that k_step3d_ring<SPARSE>
// relies on: for offsets 0..3 row 1 of `up` and column 0 of `lo` are zero,
// for offsets 4..7 row 0 of `up` and column 1 of `lo`.
static bool coef_sparse3(const StencilCoef<double>& C) {
  for (int k = 0; k < 8; ++k) {
    const int ur = k < 4 ? 1 : 0, lc = k < 4 ? 0 : 1;
    for (int j = 0; j < 2; ++j) {
      const cx<double> a = C.up[k][ur][j], b = C.lo[k][j][lc];
      if (a.x != 0.0 || a.y != 0.0 || b.x != 0.0 || b.y != 0.0) return false;
    }
  }
  return true;
}

template <typename T>
bool pack_coef(const Table& Tb, double m, StencilCoef<T>& C, std::string& why) {
  memset(&C, 0, sizeof C);
  const int dim = Tb.dim;
  std::vector<bool> used(27, false);
  auto put = [](cx<T>& dst, zc v) {
    dst.x = (T)v.real();
    dst.y = (T)v.imag();
  };
  const double tol = 1e-14;
  if (dim == 1) {
    const int op[1] = {1}, om[1] = {-1}, o0[1] = {0};
    const int ip = off_index(1, op), im = off_index(1, om), i0 = off_index(1, o0);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        put(C.up[0][a][b], Tb.U[ip][a][b]);
        put(C.up[1][a][b], Tb.U[im][a][b]);
        put(C.onsite[a][b], Tb.U[i0][a][b]);
      }
    return true;
  }
  const int K = dim == 3 ? 8 : 4;
  for (int k = 0; k < K; ++k) {
    const int* o = dim == 3 ? kOff3h[k] : kOff2h[k];
    const int idx = off_index(dim, o);
    used[idx] = true;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        put(C.up[k][a][b], Tb.U[idx][a][b]);
        put(C.lo[k][a][b], Tb.U[idx][a + 2][b + 2]);
        if (std::abs(Tb.U[idx][a][b + 2]) > tol || std::abs(Tb.U[idx][a + 2][b]) > tol) {
          why = "neighbour matrix is not block diagonal";
          return false;
        }
      }
  }
  const int o0[3] = {0, 0, 0};
  const int i0 = off_index(dim, o0);
  used[i0] = true;
  const zc mass = Tb.U[i0][0][2];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const zc want = (b == (a ^ 2)) ? mass : zc(0.0);
      if (std::abs(Tb.U[i0][a][b] - want) > tol) {
        why = "on-site matrix is not mass * I between the two halves";
        return false;
      }
    }
  put(C.onsite[0][0], mass);
  (void)m;
  int n = 1;
  for (int i = 0; i < dim; ++i) n *= 3;
  for (int h = 0; h < n; ++h) {
    if (used[h]) continue;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        if (std::abs(Tb.U[h][a][b]) > tol) {
          why = "transition matrix outside the expected neighbourhood";
          return false;
        }
  }
  return true;
}

}  // namespace

namespace qw {

// Optional per-pass event recorder (measurement entry point only).
struct PassTimer {
  hipEvent_t ev[9];
  int n = 0;
  hipStream_t st = nullptr;
};
thread_local PassTimer* g_timer = nullptr;
thread_local bool g_mark_off = false;  // inside a slab loop: one mark for the group

inline void mark() {
  if (g_timer && !g_mark_off && g_timer->n < 9)
    (void)hipEventRecord(g_timer->ev[g_timer->n++], g_timer->st);
}

// The plan's buffers only grow. A buffer that is replaced is kept (retired)
// until qw_destroy, not freed: kernels enqueued before the growth, and graphs
// a caller captured before it, still hold its address. Growth therefore
// needs no device synchronisation and never stalls other streams.
qw_status ensure_scratch(qw_plan_t p, size_t bytes) {
  if (p->scratch_bytes >= bytes) return QW_OK;
  void* q = nullptr;
  HIP_TRY(hipMalloc(&q, bytes));
  if (p->d_scratch) p->retired_dev.push_back(p->d_scratch);
  p->d_scratch = q;
  p->scratch_bytes = bytes;
  return QW_OK;
}

qw_status ensure_inst(qw_plan_t p, int B) {
  if (p->inst_cap >= B) return QW_OK;
  int cap = 64;
  while (cap < B) cap <<= 1;
  InstParam* d = nullptr;
  InstParam* h = nullptr;
  HIP_TRY(hipMalloc(&d, sizeof(InstParam) * cap));
  hipError_t e = hipHostMalloc((void**)&h, sizeof(InstParam) * cap, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(d);
    HIP_TRY(e);
  }
  if (p->d_inst) p->retired_dev.push_back(p->d_inst);
  if (p->h_inst) p->retired_host.push_back(p->h_inst);
  p->d_inst = d;
  p->h_inst = h;
  p->inst_cap = cap;
  return QW_OK;
}

qw_status ensure_coefs(qw_plan_t p, int B) {
  if (p->coefs_cap >= B) return QW_OK;
  int cap = 16;
  while (cap < B) cap <<= 1;
  const size_t one = sizeof(StencilCoef<double>);
  void* d = nullptr;
  unsigned char* h = nullptr;
  HIP_TRY(hipMalloc(&d, one * cap));
  hipError_t e = hipHostMalloc((void**)&h, one * cap, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(d);
    HIP_TRY(e);
  }
  if (p->d_coefs) p->retired_dev.push_back(p->d_coefs);
  if (p->h_coefs) p->retired_host.push_back(p->h_coefs);
  p->d_coefs = d;
  p->h_coefs = h;
  p->coefs_cap = cap;
  return QW_OK;
}

template <typename T>
std::vector<cx<T>> make_twiddles(int64_t n) {
  std::vector<cx<T>> v((size_t)n);
  for (int64_t j = 0; j < n; ++j) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)n;
    v[(size_t)j].x = (T)cosl(a);
    v[(size_t)j].y = (T)sinl(a);
  }
  return v;
}

qw_status check_plan(qw_plan_t p) {
  if (!p) return fail(QW_ERR_INVALID, "plan is NULL");
  return QW_OK;
}

// Calls defined for the Dirac walk only (per-instance masses, particle states,
// sector projectors, the cubic supercell) refuse a Weyl plan.
qw_status dirac_only(qw_plan_t p, const char* what) {
  if (p->weyl) return fail(QW_ERR_UNSUPPORTED, "%s is not defined for a Weyl plan", what);
  return QW_OK;
}

// log2 x for a power of two x > 0, else -1.
static int lg_pow2(int64_t x) {
  if (x <= 0 || (x & (x - 1))) return -1;
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

PassGeom pass_geom(qw_plan_t p, int64_t L, int B) {
  PassGeom g;
  memset(&g, 0, sizeof g);
  g.dim = p->dim;
  g.s = p->s;
  g.V = p->V;
  for (int i = 0; i < 3; ++i) g.N[i] = p->N[i];
  g.ppi = p->V / L;
  g.lg_ppi = lg_pow2(g.ppi);
  g.pencils = g.ppi * B;
  g.pen0 = 0;
  g.block_threads = p->cb;
  g.groups_per_wg = p->gw;
  g.Nc = p->Nc;
  for (int i = 0; i < 3; ++i) g.shift[i] = p->shift[i];
  g.lgN1 = p->lg[1];
  g.fourstep = p->fourstep ? 1 : 0;
  g.N1 = p->fs_N1;
  g.cs = p->d_cs;
  g.csf = p->d_csf;
  g.tw4 = p->d_tw4;
  g.inv_scale = 1.0 / (double)p->V;
  g.single.m = p->m;
  g.single.n = p->n;
  g.single.t = 0;
  g.inst = nullptr;
  g.omega = nullptr;
  return g;
}

// The last inverse pass of the schedule (axis 0; the 1D four-step's n1),
// with the reductions fused when `fuse` is given.
// The complex64 3D n1 inverse pass reads its input non-temporally when the
// field reaches kNtBytes (256^3, staged: 0.197 -> 0.188 ms, fused with the
// reductions 1.031 -> 1.022 ms per jump). The same hint on the n2 inverse
// pass before it made that pass 0.173 -> 0.198 ms, so it stays there. It
// also writes the evolved field non-temporally, as the other streaming
// passes do for fields beyond the last-level cache: with plain stores the
// pass ends sooner (0.190 against 0.214 ms) but leaves its lines dirty in
// that cache, and the next kernel pays for writing them back (the stencil
// step after a jump 0.258 against 0.215 ms); the benchmark's step (fused
// jump, two stencil steps) 1.493 -> 1.461 ms, a loop of fused jumps alone
// 1.019 -> 1.034 ms per jump.
static qw_status last_pass(qw_plan_t p, int64_t L, void* out, const void* in, int B, int64_t I,
                           hipStream_t st, const ObsFuse* fuse) {
  const int hints = (p->dim == 3 && !p->dbl && p->field_bytes * (size_t)B >= kNtBytes)
                        ? kNtLoad | kNtStore
                        : 0;
  if (fuse)
    HIP_TRY(launch_fft_strided_obs(p->dbl, L, out, in, p->s, B, I, *fuse, p->d_tw, st, hints));
  else
    HIP_TRY(launch_fft_strided(p->dbl, -1, L, out, in, (int64_t)p->s * B, I, p->d_tw, st, hints));
  mark();
  return QW_OK;
}

int64_t fused_obs_blocks_of(int dim, const int64_t* N, bool dbl) {
  if (dim == 3) return strided_obs_blocks(dbl, N[0], N[1] * N[2]);
  if (dim == 2) return strided_obs_blocks(dbl, N[0], N[1]);
  if (N[0] > kFourStepL) return strided_obs_blocks(dbl, N[0] / kFourStepL, kFourStepL);
  return 0;
}

int64_t fused_obs_blocks(qw_plan_t p) { return fused_obs_blocks_of(p->dim, p->N, p->dbl); }

ObsFuse make_fuse(qw_plan_t p, const double* origin, const double* origins, double* partials,
                  bool store) {
  ObsFuse f;
  memset(&f, 0, sizeof f);
  f.dim = p->dim;
  for (int i = 0; i < 3; ++i) {
    f.N[i] = p->N[i];
    f.lg[i] = p->lg[i];
    f.c[i] = (origin && i < p->dim) ? origin[i] : 0.0;
  }
  f.origins = origins;
  f.partials = partials;
  f.store = store ? 1 : 0;
  return f;
}

// Strided passes of the schedule: all axes but the contiguous one.
qw_status strided_passes(qw_plan_t p, int sign, void* out, const void* in, int B,
                         hipStream_t st, const ObsFuse* fuse) {
  const int s = p->s;
  if (p->dim == 3) {
    const int64_t N1 = p->N[0], N2 = p->N[1], N3 = p->N[2];
    // Cache hints when the field reaches kNtBytes. The n2 passes write with
    // non-temporal stores (256^3 complex64: 0.199 -> 0.191 ms and 0.197 ->
    // 0.184 ms). At complex64 the n1 forward pass, which reads the input
    // once, also reads it and writes its results non-temporally: 256^3 n1
    // pass 0.231 -> 0.205 ms and the n2 pass after it 0.197 -> 0.181 ms (jump
    // 1.035 -> 0.992 ms); 512^3 n1 pass (staged) 2.19 -> 2.14 ms. Either hint
    // alone loses there: the stores alone cost the n1 pass 0.231 -> 0.251
    // ms, the loads alone the n2 pass 0.197 -> 0.213 ms. At complex128 the
    // same stores slow the staged n1 pass (256^3: 0.46 -> 0.48 ms, 512^3:
    // 4.35 -> 5.3 ms), while non-temporal loads serve the n1 forward pass and
    // both n2 passes: 256^3 jump 2.17 -> 2.08 ms (n1 forward 0.450 -> 0.430,
    // n2 forward 0.391 -> 0.381, the fused pass after it 0.52 -> 0.50, n2
    // inverse 0.395 -> 0.375, the n1 inverse pass after it 0.415 -> 0.395),
    // 512^3 jump 19.4 -> 19.0 ms.
    const bool nt = p->field_bytes * (size_t)B >= kNtBytes;
    int n1_hints = 0, n2_hints = 0;
    if (nt) {
      n1_hints = p->dbl ? kNtLoad : kNtStore | kNtLoad;
      n2_hints = p->dbl ? kNtStore | kNtLoad : kNtStore;
    }
    if (sign > 0) {
      HIP_TRY(launch_fft_strided(p->dbl, 1, N1, out, in, (int64_t)s * B, N2 * N3, p->d_tw, st,
                                 n1_hints));
      mark();
      HIP_TRY(launch_fft_strided(p->dbl, 1, N2, out, out, (int64_t)s * B * N1, N3, p->d_tw, st,
                                 n2_hints));
      mark();
    } else {
      HIP_TRY(launch_fft_strided(p->dbl, -1, N2, out, in, (int64_t)s * B * N1, N3, p->d_tw, st,
                                 n2_hints));
      mark();
      return last_pass(p, N1, out, out, B, N2 * N3, st, fuse);
    }
  } else if (p->dim == 2) {
    if (sign < 0) return last_pass(p, p->N[0], out, in, B, p->N[1], st, fuse);
    HIP_TRY(launch_fft_strided(p->dbl, sign, p->N[0], out, in, (int64_t)s * B, p->N[1], p->d_tw, st));
    mark();
  } else if (p->fourstep) {
    if (sign < 0) return last_pass(p, p->fs_N1, out, in, B, p->fs_N2, st, fuse);
    HIP_TRY(launch_fft_strided(p->dbl, sign, p->fs_N1, out, in, (int64_t)s * B, p->fs_N2, p->d_tw, st));
    mark();
  } else if (out != in) {
    HIP_TRY(hipMemcpyAsync(out, in, p->field_bytes * B, hipMemcpyDeviceToDevice, st));
  }
  return QW_OK;
}

int64_t contig_len(qw_plan_t p) {
  if (p->dim == 3) return p->N[2];
  if (p->dim == 2) return p->N[1];
  return p->fourstep ? p->fs_N2 : p->N[0];
}

bool has_strided(qw_plan_t p) { return p->dim > 1 || p->fourstep; }

// The FP64 table of omega(q) at the plan's mass (V doubles), built on first
// use by one kernel. If it cannot be allocated the evolution evaluates omega
// per wave-vector instead.
const double* omega_table(qw_plan_t p, hipStream_t st) {
  if (p->d_omega || p->omega_failed) return p->d_omega;
  if (hipMalloc((void**)&p->d_omega, sizeof(double) * p->V) != hipSuccess) {
    p->d_omega = nullptr;
    p->omega_failed = true;
    (void)hipGetLastError();
    return nullptr;
  }
  const int64_t L = contig_len(p);
  PassGeom g = pass_geom(p, L, 1);
  if (launch_omega_table(g, L, p->d_omega, st) != hipSuccess) {
    (void)hipFree(p->d_omega);
    p->d_omega = nullptr;
    p->omega_failed = true;
  }
  return p->d_omega;
}

qw_status evolve_impl(qw_plan_t p, int B, const void* in, void* out, const InstParam* dinst,
                      const InstParam& single, hipStream_t st, const ObsFuse* fuse) {
  const int64_t L = contig_len(p);
  PassGeom g = pass_geom(p, L, B);
  g.single = single;
  g.inst = dinst;
  int mode = MODE_EVOLVE;
  if (p->weyl) {
    // The plan's table at n = 1, m = 0 is the Weyl omega. For complex128 it
    // saves an FP64 atan2 per wave-vector (1.39 -> 1.35 ms per 256^3 jump);
    // for complex64 its 8 bytes per wave-vector, a quarter of the field's,
    // cost more than that (0.64 ms without, 0.66 with).
    g.omega = p->dbl ? omega_table(p, st) : nullptr;
    mode = g.omega ? MODE_WEYL_TAB : MODE_WEYL;
  } else if (!dinst && B == 1) {
    g.omega = omega_table(p, st);
    if (g.omega) mode = MODE_EVOLVE_TAB;
  }
  if (p->dim == 3 && p->slab > 0 && p->slab < p->N[0]) {
    // n1 forward over the whole field; then, slab by slab of n1 planes, the
    // n2 forward, fused n3 and n2 inverse passes (a slab stays in the
    // last-level cache between them); then n1 inverse.
    const int64_t N1 = p->N[0], N2 = p->N[1], N3 = p->N[2];
    const int64_t nc = (int64_t)p->s * B;
    HIP_TRY(launch_fft_strided(p->dbl, 1, N1, out, in, nc, N2 * N3, p->d_tw, st));
    mark();
    g_mark_off = true;
    for (int64_t a = 0; a < N1; a += p->slab) {
      const int64_t k = std::min<int64_t>(p->slab, N1 - a);
      hipError_t e = launch_fft_strided_slab(p->dbl, 1, N2, out, out, nc, k, a, p->V, N3, p->d_tw, st);
      if (e == hipSuccess) {
        PassGeom gs = g;
        gs.pen0 = a * N2;
        gs.ppi = k * N2;
        gs.lg_ppi = lg_pow2(gs.ppi);
        gs.pencils = gs.ppi * B;
        e = launch_fft_contig(p->dbl, mode, L, out, out, gs, p->d_tw, st, p->ce);
      }
      if (e == hipSuccess)
        e = launch_fft_strided_slab(p->dbl, -1, N2, out, out, nc, k, a, p->V, N3, p->d_tw, st);
      if (e != hipSuccess) {
        g_mark_off = false;
        HIP_TRY(e);
      }
    }
    g_mark_off = false;
    mark();
    return last_pass(p, N1, out, out, B, N2 * N3, st, fuse);
  }
  if (has_strided(p)) {
    qw_status r = strided_passes(p, +1, out, in, B, st, nullptr);
    if (r != QW_OK) return r;
    HIP_TRY(launch_fft_contig(p->dbl, mode, L, out, out, g, p->d_tw, st, p->ce));
    mark();
    return strided_passes(p, -1, out, out, B, st, fuse);
  }
  if (fuse) return fail(QW_ERR_INVALID, "no strided pass to fuse the reductions into");
  HIP_TRY(launch_fft_contig(p->dbl, mode, L, out, in, g, p->d_tw, st, p->ce));
  mark();
  return QW_OK;
}

// psi_t = T^-1 [D_q^t a(q)] for B spectra a already in storage order (a
// state prepared in momentum space), in place: the fused pass applies the
// per-instance symbol power and inverts the contiguous axis, then the
// strided inverse passes. Not for the 1D four-step (transposed spectrum).
qw_status evolve_spectrum_impl(qw_plan_t p, int B, void* data, const InstParam* dinst,
                               hipStream_t st, const ObsFuse* fuse) {
  if (p->fourstep) return fail(QW_ERR_UNSUPPORTED, "four-step spectrum layout");
  const int64_t L = contig_len(p);
  PassGeom g = pass_geom(p, L, B);
  g.inst = dinst;
  g.single.m = p->m;
  g.single.n = p->n;
  g.single.t = 0;
  g.inv_scale = 1.0;  // the spectrum is that of the unnormalised inverse
  HIP_TRY(launch_fft_contig(p->dbl, MODE_APPLY_INV, L, data, data, g, p->d_tw, st, 8));
  if (has_strided(p)) return strided_passes(p, -1, data, data, B, st, fuse);
  if (fuse) return fail(QW_ERR_INVALID, "no strided pass to fuse the reductions into");
  return QW_OK;
}

}  // namespace qw

namespace qw {

StateGeom state_geom(qw_plan_t p) {
  StateGeom g;
  memset(&g, 0, sizeof g);
  g.dim = p->dim;
  g.s = p->s;
  g.V = p->V;
  for (int i = 0; i < 3; ++i) {
    g.N[i] = p->N[i];
    g.lg[i] = p->lg[i];
    g.shift[i] = p->shift[i];
  }
  g.Nc = p->Nc;
  g.cs = p->d_cs;
  return g;
}

ObsGeom obs_geom(qw_plan_t p) {
  ObsGeom g;
  memset(&g, 0, sizeof g);
  g.dim = p->dim;
  g.s = p->s;
  g.V = p->V;
  for (int i = 0; i < 3; ++i) {
    g.N[i] = p->N[i];
    g.lg[i] = p->lg[i];
  }
  return g;
}

void finish_obs(qw_plan_t p, const double* R, const double* origin, qw_obs* out) {
  memset(out, 0, sizeof *out);
  out->norm2 = R[0];
  const double inv = R[0] > 0.0 ? 1.0 / R[0] : 0.0;
  for (int i = 0; i < p->dim; ++i) out->mean[i] = origin[i] + R[1 + i] * inv;
  static const int pr[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  for (int k = 0; k < 6; ++k)
    if (pr[k][0] < p->dim && pr[k][1] < p->dim) out->second[k] = R[4 + k] * inv;
  if (p->dim == 1) {
    out->mean_cart[0] = out->mean[0];
  } else if (p->dim == 2) {
    out->mean_cart[0] = out->mean[0] + out->mean[1];
    out->mean_cart[1] = out->mean[0] - out->mean[1];
  } else {
    const double a = out->mean[0], b = out->mean[1], c = out->mean[2];
    out->mean_cart[0] = a + b - c;
    out->mean_cart[1] = a - b + c;
    out->mean_cart[2] = a - b - c;
  }
  out->overlap_re = R[10];
  out->overlap_im = R[11];
  out->ref_norm2 = R[12];
}

StateInst make_state_inst(qw_plan_t p, double m, const double* k0, double sigma,
                          const double* center, double c_plus, double c_minus) {
  StateInst si;
  memset(&si, 0, sizeof si);
  si.order = -1;
  si.m = m;
  si.n = sqrt(1.0 - m * m);
  si.sigma = sigma;
  si.c_plus = c_plus;
  si.c_minus = c_minus;
  double kk[3] = {0, 0, 0}, q0[3];
  for (int i = 0; i < p->dim; ++i) {
    kk[i] = k0[i];
    si.center[i] = center[i];
  }
  q_of_k(p->dim, kk, q0);
  for (int i = 0; i < 3; ++i) si.q0[i] = q0[i];
  // chi_s: normalised column of largest norm of P_s(q0) = (I + s M / sin(omega)) / 2.
  zc M[4][4];
  double cosw, sinw;
  double kq0[3];
  k_of_q(p->dim, q0, kq0);
  dirac_M(p->dim, kq0, m, M, cosw, sinw);
  const int s = p->s;
  for (int sec = 0; sec < 2; ++sec) {
    const double sg = sec == 0 ? 1.0 : -1.0;
    zc P[4][4];
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) {
        const zc mh = sinw >= 1e-12 ? M[a][b] / sinw : zc(0.0);
        P[a][b] = 0.5 * ((a == b ? 1.0 : 0.0) + sg * mh);
      }
    // Column norms of a projector come in exact pairs (P_jj = P_kk): take the
    // lowest index within a relative 1e-12 of the largest norm.
    double nrm[4] = {0.0, 0.0, 0.0, 0.0}, top = 0.0;
    for (int b = 0; b < s; ++b) {
      for (int a = 0; a < s; ++a) nrm[b] += std::norm(P[a][b]);
      nrm[b] = sqrt(nrm[b]);
      top = fmax(top, nrm[b]);
    }
    int best = 0;
    while (best < s - 1 && !(nrm[best] >= top * (1.0 - 1e-12))) ++best;
    const double bn = nrm[best];
    double (*chi)[2] = sec == 0 ? si.chi_p : si.chi_m;
    for (int a = 0; a < s; ++a) {
      chi[a][0] = P[a][best].real() / bn;
      chi[a][1] = P[a][best].imag() / bn;
    }
  }
  return si;
}

qw_status transform_impl(qw_plan_t p, int B, const void* in, void* out, int direction,
                         void* scratch, hipStream_t st) {
  const int64_t L = contig_len(p);
  PassGeom g = pass_geom(p, L, B);
  const int64_t planes = (int64_t)p->s * B;
  if (direction > 0) {
    if (has_strided(p)) {
      qw_status r = strided_passes(p, +1, out, in, B, st, nullptr);
      if (r != QW_OK) return r;
      HIP_TRY(launch_fft_contig(p->dbl, MODE_FWD, L, out, out, g, p->d_tw, st));
    } else {
      HIP_TRY(launch_fft_contig(p->dbl, MODE_FWD, L, out, in, g, p->d_tw, st));
    }
    if (p->fourstep) {
      if (!scratch) return fail(QW_ERR_INVALID, "four-step transform needs scratch");
      // row k1, column k2 holds q index k1 + N1 k2: transpose to natural order.
      HIP_TRY(launch_transpose(p->dbl, scratch, out, planes, p->fs_N1, p->fs_N2, st));
      HIP_TRY(hipMemcpyAsync(out, scratch, p->field_bytes * B, hipMemcpyDeviceToDevice, st));
    }
    return QW_OK;
  }
  const void* src = in;
  if (p->fourstep) {
    if (!scratch) return fail(QW_ERR_INVALID, "four-step transform needs scratch");
    HIP_TRY(launch_transpose(p->dbl, scratch, in, planes, p->fs_N2, p->fs_N1, st));
    src = scratch;
  }
  HIP_TRY(launch_fft_contig(p->dbl, MODE_INV, L, out, src, g, p->d_tw, st));
  if (has_strided(p)) return strided_passes(p, -1, out, out, B, st, nullptr);
  return QW_OK;
}

}  // namespace qw

namespace {

// QW_DEBUG set (to anything but "0"): every entry point waits for its
// stream and reports a failed kernel as its own error (for debugging; slow).
// Read on every call, so that a process can switch it while it runs.
bool debug_mode() {
  const char* v = getenv("QW_DEBUG");
  return v && *v && strcmp(v, "0") != 0;
}

// Runs one entry point inside a named roctx range (visible to rocprofv3
// --marker-trace), and in debug mode synchronises its stream afterwards.
template <typename F>
qw_status traced(const char* name, void* stream, F&& body) {
  roctxRangePush(name);
  qw_status r = body();
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (r == QW_OK && debug_mode() &&
      hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess &&
      cs == hipStreamCaptureStatusNone) {  // a capturing stream cannot be synchronised
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) r = fail(QW_ERR_DEVICE, "%s: %s (QW_DEBUG)", name, hipGetErrorString(e));
  }
  roctxRangePop();
  return r;
}

}  // namespace

extern "C" {

const char* qw_last_error(void) { return g_last_error.c_str(); }

const char* qw_version(void) { return "qw-mi355x 0.1 (gfx950)"; }

static qw_status plan_create(qw_plan_t* out, int dim, const int64_t* N, double m, qw_dtype dtype,
                             void* stream, bool weyl);

qw_status qw_plan(qw_plan_t* out, int dim, const int64_t* N, double m, qw_dtype dtype,
                  void* stream) {
  return plan_create(out, dim, N, m, dtype, stream, false);
}

qw_status qw_plan_weyl(qw_plan_t* out, int dim, const int64_t* N, qw_dtype dtype, void* stream) {
  // d = 1: the Weyl walk diag(e^{-ik}, e^{ik}) is the Dirac walk at m = 0.
  return plan_create(out, dim, N, 0.0, dtype, stream, dim >= 2);
}

static qw_status plan_create(qw_plan_t* out, int dim, const int64_t* N, double m, qw_dtype dtype,
                             void* stream, bool weyl) {
  if (!out) return fail(QW_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (dim < 1 || dim > 3) return fail(QW_ERR_INVALID, "dim must be 1, 2 or 3 (got %d)", dim);
  if (!N) return fail(QW_ERR_INVALID, "N is NULL");
  if (!(m >= 0.0 && m <= 1.0)) return fail(QW_ERR_INVALID, "m must lie in [0, 1]");
  if (dtype != QW_C64 && dtype != QW_C128) return fail(QW_ERR_INVALID, "unknown dtype %d", (int)dtype);
  const int64_t maxN = dim == 1 ? 65536 : (dim == 2 ? 1024 : 512);
  for (int i = 0; i < dim; ++i) {
    if (N[i] < 1) return fail(QW_ERR_INVALID, "N[%d] = %lld is not positive", i, (long long)N[i]);
    if (!is_pow2(N[i]) || N[i] < 2 || N[i] > maxN)
      return fail(QW_ERR_UNSUPPORTED, "N[%d] = %lld: need a power of two in [2, %lld] for dim %d",
                  i, (long long)N[i], (long long)maxN, dim);
  }
  qw_plan_t p = new (std::nothrow) qw_plan_s();
  if (!p) return fail(QW_ERR_NOMEM, "host allocation failed");
  p->dim = dim;
  p->weyl = weyl;
  p->s = (dim == 1 || weyl) ? 2 : 4;
  p->V = 1;
  for (int i = 0; i < dim; ++i) {
    p->N[i] = N[i];
    p->lg[i] = lg2(N[i]);
    p->V *= N[i];
  }
  p->m = m;
  p->n = sqrt(1.0 - m * m);
  p->dtype = dtype;
  p->dbl = dtype == QW_C128;
  p->elem = p->dbl ? 16 : 8;
  p->field_bytes = (size_t)p->s * p->V * p->elem;
  // Fused pass: four elements per thread for complex128 fields of d = 2, 3
  // (eight spill registers there), eight otherwise until tuned.
  if (p->dbl && dim >= 2) p->ce = 4;
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetDevice(&p->device);

  // Transition matrices from the symbol, unitarity checked (Sec. 2).
  const double leak = derive_table(dim, m, p->table);
  const double defect = unitarity_defect(p->table);
  if (leak > 1e-14 || defect > 1e-13) {
    delete p;
    return fail(QW_ERR_DEVICE, "derived transition matrices fail checks (leak %g, unitarity %g)",
                leak, defect);
  }
  std::string why;
  if (!pack_coef<double>(p->table, m, p->coef_d, why) || !pack_coef<float>(p->table, m, p->coef_f, why)) {
    delete p;
    return fail(QW_ERR_DEVICE, "transition matrices: %s", why.c_str());
  }

  // Rank-one pattern of the 3D neighbour blocks (lets the stencil skip zeros).
  if (dim == 3) p->sparse3 = coef_sparse3(p->coef_d);

  // Fourier schedule.
  if (dim == 1 && N[0] > kFourStepL) {
    p->fourstep = true;
    p->fs_N2 = kFourStepL;
    p->fs_N1 = N[0] / kFourStepL;
  }
  int64_t Nc = 1;
  for (int i = 0; i < dim; ++i) Nc = N[i] > Nc ? N[i] : Nc;
  p->Nc = (int)Nc;
  for (int i = 0; i < dim; ++i) p->shift[i] = lg2(Nc / N[i]);

  qw_status r = QW_OK;
  auto upload = [&](void** dst, const void* src, size_t bytes) -> qw_status {
    HIP_TRY(hipMalloc(dst, bytes));
    HIP_TRY(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, st));
    return QW_OK;
  };
  {
    std::vector<double> cs((size_t)4 * Nc);
    for (int64_t j = 0; j < 2 * Nc; ++j) {
      const long double a = 3.14159265358979323846264338327950288L * (long double)j / (long double)Nc;
      double c = (double)cosl(a), sn = (double)sinl(a);
      // exact zeros at multiples of pi/2 (the smallest other |value| is
      // sin(pi / 65536) ~ 5e-5), so that n~ vanishes exactly at the band
      // edge q = pi and sin(omega) = 0 there when m = 0
      if (std::fabs(c) < 1e-15) c = 0.0;
      if (std::fabs(sn) < 1e-15) sn = 0.0;
      cs[(size_t)2 * j] = c;
      cs[(size_t)2 * j + 1] = sn;
    }
    if (p->dbl) {
      auto tw = make_twiddles<double>(TWN);
      r = upload(&p->d_tw, tw.data(), tw.size() * sizeof(tw[0]));
      if (r == QW_OK && p->fourstep) {
        auto t4 = make_twiddles<double>(N[0]);
        r = upload(&p->d_tw4, t4.data(), t4.size() * sizeof(t4[0]));
      }
    } else {
      auto tw = make_twiddles<float>(TWN);
      r = upload(&p->d_tw, tw.data(), tw.size() * sizeof(tw[0]));
      if (r == QW_OK && p->fourstep) {
        auto t4 = make_twiddles<float>(N[0]);
        r = upload(&p->d_tw4, t4.data(), t4.size() * sizeof(t4[0]));
      }
    }
    std::vector<float> csf(cs.begin(), cs.end());
    if (r == QW_OK) r = upload((void**)&p->d_cs, cs.data(), cs.size() * sizeof(double));
    if (r == QW_OK) r = upload((void**)&p->d_csf, csf.data(), csf.size() * sizeof(float));
    if (r == QW_OK) {
      if (p->dbl)
        r = upload(&p->d_coef, &p->coef_d, sizeof(p->coef_d));
      else
        r = upload(&p->d_coef, &p->coef_f, sizeof(p->coef_f));
    }
    if (r == QW_OK) {
      const int64_t nfp = ((int64_t)p->s * fused_obs_blocks(p) + 64) * kObsFields;
      p->partials_len = std::max<int64_t>((int64_t)kObsFields * kObsBlocks, nfp);
      p->partials_len = std::max<int64_t>(p->partials_len, state_scratch_doubles(state_geom(p), 1));
      hipError_t e = hipMalloc(&p->d_partials, sizeof(double) * p->partials_len);
      if (e == hipSuccess) e = hipMalloc(&p->d_result, sizeof(double) * 32);
      if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_result, sizeof(double) * 32, hipHostMallocDefault);
      if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_stage, sizeof(StateInst), hipHostMallocDefault);
      if (e == hipSuccess) e = hipMalloc((void**)&p->d_stage, sizeof(StateInst));
      // the host vectors above are released at scope end: wait for the uploads
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess)
        r = fail(e == hipErrorOutOfMemory ? QW_ERR_NOMEM : QW_ERR_DEVICE, "plan set-up: %s",
                 hipGetErrorString(e));
    } else {
      (void)hipStreamSynchronize(st);
    }
  }
  if (r != QW_OK) {
    delete p;
    return r;
  }
  *out = p;
  return QW_OK;
}

qw_status qw_destroy(qw_plan_t p) {
  if (!p) return QW_OK;
  (void)hipDeviceSynchronize();
  delete p;
  return QW_OK;
}

static StencilGeom stencil_geom(qw_plan_t p) {
  StencilGeom g;
  g.dim = p->dim;
  for (int i = 0; i < 3; ++i) {
    g.N[i] = p->N[i];
    g.lg[i] = p->lg[i];
  }
  g.V = p->V;
  g.sparse3 = p->sparse3 ? 1 : 0;
  g.weyl = p->weyl ? 1 : 0;
  g.nt = 0;
  return g;
}

// Pairs of steps in one launch of the two-step kernel only when switched on
// (qw_set_step_kernel): measured slower than one launch per step at 256^3
// (0.56 against 0.48 ms per pair), its rings of 128 KB of LDS leave one
// workgroup of 8 waves per CU.
static bool g_step2_off = true;

// nsteps steps of B fields in place with device coefficients `coefs`: the
// LDS-resident kernel where a 1D field fits (at most 4096 steps per launch),
// otherwise one launch per step, ping-ponging with `buf` (B fields), or with
// the plan's scratch when buf is null.
static qw_status step_impl(qw_plan_t p, const StencilGeom& g, int B, void* psi,
                           const void* coefs, int64_t nsteps, hipStream_t st,
                           void* buf = nullptr) {
  if (step1d_resident_ok(p->dbl, g)) {
    for (int64_t done = 0; done < nsteps;) {
      const int64_t k = std::min<int64_t>(4096, nsteps - done);
      HIP_TRY(launch_step1d_resident(p->dbl, g, B, psi, coefs, k, st));
      done += k;
    }
    return QW_OK;
  }
  const size_t bytes = p->field_bytes * (size_t)B;
  if (!buf) {
    qw_status r = ensure_scratch(p, bytes);
    if (r != QW_OK) return r;
    buf = p->d_scratch;
  }
  void* a = psi;
  void* b = buf;
  // Pairs of steps in one launch where the two-step kernel applies (it reads
  // and writes the field once per pair), a last odd step alone.
  const bool two = step2_ok(p->dbl, g) && !g_step2_off;
  for (int64_t k = 0; k < nsteps;) {
    if (two && nsteps - k >= 2) {
      HIP_TRY(launch_step2(p->dbl, g, B, b, a, coefs, st));
      k += 2;
    } else {
      HIP_TRY(launch_step(p->dbl, g, B, b, a, coefs, st));
      k += 1;
    }
    void* t = a;
    a = b;
    b = t;
  }
  if (a != psi) HIP_TRY(hipMemcpyAsync(psi, a, bytes, hipMemcpyDeviceToDevice, st));
  return QW_OK;
}

qw_status qw_step(qw_plan_t p, void* psi, int64_t nsteps, void* stream) {
  return traced("qw_step", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    if (!psi) return fail(QW_ERR_INVALID, "psi is NULL");
    if (nsteps < 0) return fail(QW_ERR_INVALID, "nsteps must be >= 0");
    if (nsteps == 0) return QW_OK;
    return step_impl(p, stencil_geom(p), 1, psi, p->d_coef, nsteps, (hipStream_t)stream);
  });
}

}  // extern "C"

// The ping-pong buffer of qw_step_noalloc: a fixed array in device memory,
// one per device (the runtime places it in every device's memory with the
// library's code), kept until the process ends. Host code never uses its
// name as an address: each device's address is looked up once, with that
// device current, and kept in noalloc_ptr.
static __device__ __align__(256) unsigned char scratch[QW_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (null and a message on failure).
void* noalloc_ptr(qw_status* err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *err = fail(QW_ERR_DEVICE, "hipGetDevice: %s (device %d)", hipGetErrorString(e), dev);
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *err = fail(QW_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return nullptr;
    }
    g_noalloc_ptr[dev] = ptr;
  }
  return g_noalloc_ptr[dev];
}
}  // namespace

extern "C" {

qw_status qw_step_noalloc(qw_plan_t p, void* psi, int64_t nsteps, void* stream) {
  return traced("qw_step_noalloc", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    if (!psi) return fail(QW_ERR_INVALID, "psi is NULL");
    if (nsteps < 0) return fail(QW_ERR_INVALID, "nsteps must be >= 0");
    if (p->field_bytes > (size_t)QW_NOALLOC_SCRATCH_BYTES)
      return fail(QW_ERR_UNSUPPORTED,
                  "qw_step_noalloc: the field has %zu bytes, the fixed buffer holds %zu",
                  p->field_bytes, (size_t)QW_NOALLOC_SCRATCH_BYTES);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
      return fail(QW_ERR_INVALID, "qw_step_noalloc: the plan's device (%d) is not current (%d)",
                  p->device, dev);
    if (nsteps == 0) return QW_OK;
    void* buf = noalloc_ptr(&r);
    if (!buf) return r;
    return step_impl(p, stencil_geom(p), 1, psi, p->d_coef, nsteps, (hipStream_t)stream, buf);
  });
}

qw_status qw_step_batched(qw_plan_t p, int B, void* psi, const double* m, int64_t nsteps,
                          void* stream) {
  return traced("qw_step_batched", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    r = dirac_only(p, "qw_step_batched");
    if (r != QW_OK) return r;
    if (B < 0 || B > 65535) return fail(QW_ERR_INVALID, "B must lie in [0, 65535]");
    if (nsteps < 0) return fail(QW_ERR_INVALID, "nsteps must be >= 0");
    if (B == 0 || nsteps == 0) return QW_OK;
    if (!psi || !m) return fail(QW_ERR_INVALID, "NULL argument");
    for (int b = 0; b < B; ++b)
      if (!(m[b] >= 0.0 && m[b] <= 1.0)) return fail(QW_ERR_INVALID, "m[%d] outside [0, 1]", b);
    hipStream_t st = (hipStream_t)stream;
    // Per-instance transition matrices, derived and packed exactly as the
    // plan's own (an instance with the plan's mass gets the plan's numbers).
    StencilGeom g = stencil_geom(p);
    const size_t one = p->dbl ? sizeof(StencilCoef<double>) : sizeof(StencilCoef<float>);
    r = ensure_coefs(p, B);
    if (r != QW_OK) return r;
    // The pinned staging area may still feed an earlier call's copy.
    HIP_TRY(hipStreamSynchronize(st));
    bool sparse = p->dim == 3;
    for (int b = 0; b < B; ++b) {
      Table T;
      const double leak = derive_table(p->dim, m[b], T);
      if (leak > 1e-14 || unitarity_defect(T) > 1e-13)
        return fail(QW_ERR_DEVICE, "derived transition matrices fail checks for m[%d]", b);
      StencilCoef<double> cd;
      StencilCoef<float> cf;
      std::string why;
      if (!pack_coef<double>(T, m[b], cd, why) || !pack_coef<float>(T, m[b], cf, why))
        return fail(QW_ERR_DEVICE, "transition matrices for m[%d]: %s", b, why.c_str());
      if (sparse && !coef_sparse3(cd)) sparse = false;
      if (p->dbl)
        memcpy(p->h_coefs + one * b, &cd, one);
      else
        memcpy(p->h_coefs + one * b, &cf, one);
    }
    g.sparse3 = sparse ? 1 : 0;
    HIP_TRY(hipMemcpyAsync(p->d_coefs, p->h_coefs, one * B, hipMemcpyHostToDevice, st));
    return step_impl(p, g, B, psi, p->d_coefs, nsteps, st);
  });
}

// |t| <= 2^53: every such integer is a double, and the phase omega t is
// reduced exactly (larger t would not be meaningful in FP64 anyway).
static constexpr double kMaxT = 9007199254740992.0;

static qw_status check_time(double t) {
  if (!(fabs(t) <= kMaxT)) return fail(QW_ERR_UNSUPPORTED, "|t| must be finite and at most 2^53");
  return QW_OK;
}
// Integer times are compared as integers: 2^53 + 1 would round to 2^53.
static qw_status check_time(int64_t t) {
  constexpr int64_t kMaxI = int64_t(1) << 53;
  if (t > kMaxI || t < -kMaxI) return fail(QW_ERR_UNSUPPORTED, "|t| must be at most 2^53");
  return QW_OK;
}

qw_status qw_evolve_fft(qw_plan_t p, const void* psi0, void* psi_t, int64_t t, void* stream) {
  return traced("qw_evolve_fft", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    if (!psi0 || !psi_t) return fail(QW_ERR_INVALID, "field pointer is NULL");
    r = check_time(t);
    if (r != QW_OK) return r;
    InstParam ip;
    ip.m = p->m;
    ip.n = p->n;
    ip.t = (double)t;
    return evolve_impl(p, 1, psi0, psi_t, nullptr, ip, (hipStream_t)stream);
  });
}

qw_status qw_evolve_fft_real(qw_plan_t p, const void* psi0, void* psi_t, double t, void* stream) {
  return traced("qw_evolve_fft_real", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    if (!psi0 || !psi_t) return fail(QW_ERR_INVALID, "field pointer is NULL");
    r = check_time(t);
    if (r != QW_OK) return r;
    InstParam ip;
    ip.m = p->m;
    ip.n = p->n;
    ip.t = t;
    return evolve_impl(p, 1, psi0, psi_t, nullptr, ip, (hipStream_t)stream);
  });
}

qw_status qw_set_step_kernel(int two_step, int tile_shape, int chunk) {
  if (two_step != 0 && two_step != 1) return fail(QW_ERR_INVALID, "two_step must be 0 or 1");
  if (tile_shape < 0 || tile_shape > 3) return fail(QW_ERR_INVALID, "tile_shape must lie in [0, 3]");
  if (chunk != 0 && (chunk < 2 || chunk > 256 || (chunk & (chunk - 1))))
    return fail(QW_ERR_INVALID, "chunk must be 0 or a power of two in [2, 256]");
  g_step2_off = two_step == 0;
  set_step2_config(tile_shape, chunk);
  return QW_OK;
}

qw_status qw_set_fft_kernel(int staged) {
  if (staged != 0 && staged != 1) return fail(QW_ERR_INVALID, "staged must be 0 or 1");
  set_fft_staged(staged == 1);
  return QW_OK;
}

qw_status qw_set_schedule(qw_plan_t p, int slab_planes, int contig_elems, int contig_threads,
                          int contig_groups) {
  qw_status r = check_plan(p);
  if (r != QW_OK) return r;
  if (slab_planes < 0) return fail(QW_ERR_INVALID, "slab_planes must be >= 0");
  if (contig_elems != 4 && contig_elems != 8)
    return fail(QW_ERR_INVALID, "contig_elems must be 4 or 8");
  if (contig_threads != 64 && contig_threads != 128 && contig_threads != 256 && contig_threads != 512)
    return fail(QW_ERR_INVALID, "contig_threads must be 64, 128, 256 or 512");
  if (contig_groups < 1 || contig_groups > 64)
    return fail(QW_ERR_INVALID, "contig_groups must lie in [1, 64]");
  p->slab = p->dim == 3 ? slab_planes : 0;
  p->ce = contig_elems;
  p->cb = contig_threads;
  p->gw = contig_groups;
  return QW_OK;
}

qw_status qw_get_schedule(qw_plan_t p, int* slab_planes, int* contig_elems, int* contig_threads,
                          int* contig_groups) {
  qw_status r = check_plan(p);
  if (r != QW_OK) return r;
  if (!slab_planes || !contig_elems || !contig_threads || !contig_groups)
    return fail(QW_ERR_INVALID, "NULL argument");
  *slab_planes = p->slab;
  *contig_elems = p->ce;
  *contig_threads = p->cb;
  *contig_groups = p->gw;
  return QW_OK;
}

qw_status qw_autotune(qw_plan_t p, void* stream, double* best_ms) {
  return traced("qw_autotune", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    // QW_TUNE_CACHE names a text file of earlier results, one line per
    // (device architecture, walk, dimension, lattice, precision): a cached
    // schedule is taken without timing; a new one is appended.
    const char* cache_path = getenv("QW_TUNE_CACHE");
    char key[256] = {0};
    if (cache_path && *cache_path) {
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) prop.gcnArchName[0] = 0;
      snprintf(key, sizeof key, "qw-tune-v1 %s %s d%d %lldx%lldx%lld %s", prop.gcnArchName,
               p->weyl ? "weyl" : "dirac", p->dim, (long long)p->N[0], (long long)p->N[1],
               (long long)p->N[2], p->dbl ? "c128" : "c64");
      for (char* c = key; *c; ++c)
        if (*c == ':' || *c == '\n') *c = '_';  // keep the key one token per field
      if (FILE* f = fopen(cache_path, "r")) {
        char line[512];
        int fs = -1, fc = 0, fb = 0, fg = 0;
        double fms = 0.0;
        const size_t kl = strlen(key);
        while (fgets(line, sizeof line, f)) {
          int a, b, c, d;
          double ms;
          // the last well-formed entry wins; anything else is skipped
          if (strncmp(line, key, kl) == 0 && line[kl] == ' ' &&
              sscanf(line + kl, " %d %d %d %d %lf", &a, &b, &c, &d, &ms) == 5 && a >= 0 &&
              (b == 4 || b == 8) && (c == 64 || c == 128 || c == 256 || c == 512) && d >= 1 &&
              d <= 64 && ms >= 0.0) {
            fs = a; fc = b; fb = c; fg = d; fms = ms;
          }
        }
        fclose(f);
        if (fs >= 0) {
          p->slab = p->dim == 3 ? fs : 0;
          p->ce = fc;
          p->cb = fb;
          p->gw = fg;
          if (best_ms) *best_ms = fms;
          return QW_OK;
        }
      }
    }
    r = ensure_scratch(p, p->field_bytes);
    if (r != QW_OK) return r;
    HIP_TRY(hipMemsetAsync(p->d_scratch, 0, p->field_bytes, st));
    std::vector<int> slabs = {0};
    if (p->dim == 3) {
      const size_t plane = p->field_bytes / (size_t)p->N[0];
      for (size_t target : {size_t(16) << 20, size_t(32) << 20, size_t(64) << 20, size_t(128) << 20}) {
        int64_t k = (int64_t)(target / plane);
        if (k >= 1 && k < p->N[0]) {
          int64_t kk = 1;
          while (kk * 2 <= k) kk *= 2;
          if (std::find(slabs.begin(), slabs.end(), (int)kk) == slabs.end()) slabs.push_back((int)kk);
        }
      }
    }
    // complex128 with eight elements per thread spills registers in the
    // lockstep transform of four components (d = 2, 3): four only.
    const int ces[2] = {8, 4};
    const bool only4 = p->dbl && p->dim >= 2;
    const int cbs[3] = {64, 128, 256};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    InstParam ip;
    ip.m = p->m;
    ip.n = p->n;
    ip.t = 12345;
    // 16 groups per workgroup: about one round of resident workgroups per CU
    // at 256^3, each walking its groups with the loads one ahead.
    const int gws[3] = {1, 4, 16};
    double best = 1e30;
    int bs = 0, bc = 8, bb = 256, bg = 1;
    for (int sl : slabs)
      for (int ce : ces)
        for (int cb : cbs)
          for (int gw : gws) {
        if (ce == 4 && p->dim < 2) continue;
        if (ce == 8 && only4) continue;
        if (gw > 1 && !(p->dim == 3 && ce == 4)) continue;
        p->slab = sl;
        p->ce = ce;
        p->cb = cb;
        p->gw = gw;
        r = evolve_impl(p, 1, p->d_scratch, p->d_scratch, nullptr, ip, st);  // warm-up
        if (r != QW_OK) break;
        (void)hipEventRecord(e0, st);
        const int reps = 3;
        for (int k = 0; k < reps && r == QW_OK; ++k)
          r = evolve_impl(p, 1, p->d_scratch, p->d_scratch, nullptr, ip, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r == QW_OK && ms / reps < best) {
          best = ms / reps;
          bs = sl;
          bc = ce;
          bb = cb;
          bg = gw;
        }
          }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->slab = bs;
    p->ce = bc;
    p->cb = bb;
    p->gw = bg;
    if (r != QW_OK) return r;
    if (best_ms) *best_ms = best;
    if (key[0]) {
      if (FILE* f = fopen(cache_path, "a")) {
        fprintf(f, "%s %d %d %d %d %.6f\n", key, bs, bc, bb, bg, best);
        fclose(f);
      }
    }
    return QW_OK;
  });
}

qw_status qw_evolve_fft_timed(qw_plan_t p, const void* psi0, void* psi_t, int64_t t, void* stream,
                              float* pass_ms, int* npass) {
  return traced("qw_evolve_fft_timed", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    if (!psi0 || !psi_t || !pass_ms || !npass) return fail(QW_ERR_INVALID, "NULL argument");
    r = check_time(t);
    if (r != QW_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    PassTimer tm;
    tm.st = st;
    for (int i = 0; i < 9; ++i) HIP_TRY(hipEventCreate(&tm.ev[i]));
    HIP_TRY(hipEventRecord(tm.ev[tm.n++], st));
    InstParam ip;
    ip.m = p->m;
    ip.n = p->n;
    ip.t = (double)t;
    g_timer = &tm;
    r = evolve_impl(p, 1, psi0, psi_t, nullptr, ip, st);
    g_timer = nullptr;
    hipError_t e = hipEventSynchronize(tm.ev[tm.n - 1]);
    *npass = tm.n - 1;
    for (int i = 0; i + 1 < tm.n && i < 8; ++i) {
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, tm.ev[i], tm.ev[i + 1]);
      pass_ms[i] = ms;
    }
    for (int i = 0; i < 9; ++i) (void)hipEventDestroy(tm.ev[i]);
    if (r != QW_OK) return r;
    if (e != hipSuccess) return fail(QW_ERR_DEVICE, "event timing: %s", hipGetErrorString(e));
    return QW_OK;
  });
}

qw_status qw_evolve_fft_batched(qw_plan_t p, int B, const void* in, void* out, const double* m,
                                const int64_t* t, void* stream) {
  return traced("qw_evolve_fft_batched", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    r = dirac_only(p, "qw_evolve_fft_batched");
    if (r != QW_OK) return r;
    if (B < 0) return fail(QW_ERR_INVALID, "B must be >= 0");
    if (B == 0) return QW_OK;
    if (!in || !out || !m || !t) return fail(QW_ERR_INVALID, "NULL argument");
    for (int b = 0; b < B; ++b) {
      if (!(m[b] >= 0.0 && m[b] <= 1.0)) return fail(QW_ERR_INVALID, "m[%d] outside [0, 1]", b);
      r = check_time(t[b]);
      if (r != QW_OK) return r;
    }
    hipStream_t st = (hipStream_t)stream;
    r = ensure_inst(p, B);
    if (r != QW_OK) return r;
    // The pinned staging area may still feed an earlier batched call's copy.
    HIP_TRY(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b) {
      p->h_inst[b].m = m[b];
      p->h_inst[b].n = sqrt(1.0 - m[b] * m[b]);
      p->h_inst[b].t = (double)t[b];
    }
    HIP_TRY(hipMemcpyAsync(p->d_inst, p->h_inst, sizeof(InstParam) * B, hipMemcpyHostToDevice, st));
    InstParam ip;
    ip.m = p->m;
    ip.n = p->n;
    ip.t = 0;
    return evolve_impl(p, B, in, out, p->d_inst, ip, st);
  });
}

qw_status qw_transform(qw_plan_t p, const void* in, void* out, int direction, void* stream) {
  return traced("qw_transform", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    if (!in || !out) return fail(QW_ERR_INVALID, "field pointer is NULL");
    if (direction != 1 && direction != -1) return fail(QW_ERR_INVALID, "direction must be +1 or -1");
    if (p->fourstep) {
      r = ensure_scratch(p, p->field_bytes);
      if (r != QW_OK) return r;
    }
    return transform_impl(p, 1, in, out, direction, p->d_scratch, (hipStream_t)stream);
  });
}

// Cubic-supercell field [2][s][N1 N2 N3] (Sec. 4, eq:bcc-dft / eq:bcc-idft):
// the strided passes take it as two fields of s components, the pass along n3
// as one pencil of 2s components (combine, per-k powers, recombination).
// omega(kappa) of the cubic supercell at the plan's mass (V doubles), built
// on first use; without it the pass evaluates omega per wave-vector.
static const double* omega_bcc_table(qw_plan_t p, hipStream_t st) {
  if (p->d_omega_bcc || p->omega_bcc_failed) return p->d_omega_bcc;
  if (hipMalloc((void**)&p->d_omega_bcc, sizeof(double) * p->V) != hipSuccess) {
    p->d_omega_bcc = nullptr;
    p->omega_bcc_failed = true;
    (void)hipGetLastError();
    return nullptr;
  }
  PassGeom g = pass_geom(p, p->N[2], 1);
  if (launch_omega_bcc_table(g, p->N[2], p->d_omega_bcc, st) != hipSuccess) {
    (void)hipFree(p->d_omega_bcc);
    p->d_omega_bcc = nullptr;
    p->omega_bcc_failed = true;
  }
  return p->d_omega_bcc;
}

static qw_status bcc_impl(qw_plan_t p, const void* in, void* out, int mode, double t,
                          hipStream_t st) {
  const int64_t L = p->N[2];
  PassGeom g = pass_geom(p, L, 1);
  g.single.t = t;
  g.inv_scale = mode == MODE_BCC ? 0.5 / (double)p->V : 1.0 / sqrt(2.0 * (double)p->V);
  if (mode == MODE_BCC) {
    g.omega = omega_bcc_table(p, st);
    if (g.omega) mode = MODE_BCC_TAB;
  }
  if (mode == MODE_BCC_INV) {
    HIP_TRY(launch_fft_contig(p->dbl, mode, L, out, in, g, p->d_tw, st, 4));
    mark();
    return strided_passes(p, -1, out, out, 2, st, nullptr);
  }
  qw_status r = strided_passes(p, +1, out, in, 2, st, nullptr);
  if (r != QW_OK) return r;
  HIP_TRY(launch_fft_contig(p->dbl, mode, L, out, out, g, p->d_tw, st, 4));
  mark();
  if (mode == MODE_BCC_FWD) return QW_OK;
  return strided_passes(p, -1, out, out, 2, st, nullptr);
}

static qw_status check_bcc(qw_plan_t p, const void* in, const void* out) {
  qw_status r = check_plan(p);
  if (r != QW_OK) return r;
  r = dirac_only(p, "the cubic supercell");
  if (r != QW_OK) return r;
  if (p->dim != 3) return fail(QW_ERR_UNSUPPORTED, "the cubic supercell needs a 3D plan");
  if (!in || !out) return fail(QW_ERR_INVALID, "field pointer is NULL");
  return QW_OK;
}

qw_status qw_bcc_transform(qw_plan_t p, const void* in, void* out, int direction, void* stream) {
  return traced("qw_bcc_transform", stream, [&]() -> qw_status {
    qw_status r = check_bcc(p, in, out);
    if (r != QW_OK) return r;
    if (direction != 1 && direction != -1) return fail(QW_ERR_INVALID, "direction must be +1 or -1");
    return bcc_impl(p, in, out, direction > 0 ? MODE_BCC_FWD : MODE_BCC_INV, 0.0,
                    (hipStream_t)stream);
  });
}

qw_status qw_bcc_step(qw_plan_t p, void* f, int64_t nsteps, void* stream) {
  return traced("qw_bcc_step", stream, [&]() -> qw_status {
    qw_status r = check_bcc(p, f, f);
    if (r != QW_OK) return r;
    if (nsteps < 0) return fail(QW_ERR_INVALID, "nsteps must be >= 0");
    if (nsteps == 0) return QW_OK;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = 2 * p->field_bytes;
    r = ensure_scratch(p, bytes);
    if (r != QW_OK) return r;
    const StencilGeom g = stencil_geom(p);
    void* a = f;
    void* b = p->d_scratch;
    for (int64_t k = 0; k < nsteps; ++k) {
      HIP_TRY(launch_step_bcc(p->dbl, g, b, a, p->d_coef, st));
      void* tmp = a;
      a = b;
      b = tmp;
    }
    if (a != f) HIP_TRY(hipMemcpyAsync(f, a, bytes, hipMemcpyDeviceToDevice, st));
    return QW_OK;
  });
}

qw_status qw_bcc_observables(qw_plan_t p, const void* f, const double* origin, qw_obs* out,
                             void* stream) {
  return traced("qw_bcc_observables", stream, [&]() -> qw_status {
    qw_status r = check_bcc(p, f, f);
    if (r != QW_OK) return r;
    if (!origin || !out) return fail(QW_ERR_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    ObsGeom g = obs_geom(p);
    for (int i = 0; i < 3; ++i) {
      if (!isfinite(origin[i])) return fail(QW_ERR_INVALID, "origin is not finite");
      g.c[i] = origin[i];
    }
    HIP_TRY(launch_bcc_observables(p->dbl, g, f, p->d_partials, p->d_result, st));
    HIP_TRY(hipMemcpyAsync(p->h_result, p->d_result, sizeof(double) * kObsFields,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double* R = p->h_result;
    memset(out, 0, sizeof *out);
    out->norm2 = R[0];
    const double inv = R[0] > 0.0 ? 1.0 / R[0] : 0.0;
    for (int i = 0; i < 3; ++i) {
      out->mean[i] = origin[i] + R[1 + i] * inv;
      out->mean_cart[i] = out->mean[i];  // the coordinates are Cartesian
    }
    for (int k = 0; k < 6; ++k) out->second[k] = R[4 + k] * inv;
    return QW_OK;
  });
}

qw_status qw_bcc_evolve_fft(qw_plan_t p, const void* f0, void* f_t, double t, void* stream) {
  return traced("qw_bcc_evolve_fft", stream, [&]() -> qw_status {
    qw_status r = check_bcc(p, f0, f_t);
    if (r != QW_OK) return r;
    r = check_time(t);
    if (r != QW_OK) return r;
    return bcc_impl(p, f0, f_t, MODE_BCC, t, (hipStream_t)stream);
  });
}

static_assert(kObsFields == QW_OBS_RAW_DOUBLES, "raw reduction record of the public header");

// The jump and its reductions queued on st, the record of kObsFields sums
// left in p->d_result (shared by the waiting and the non-waiting calls).
static qw_status obs_jump_launch(qw_plan_t p, const void* psi0, void* psi_t, int64_t t,
                                 const double* origin, hipStream_t st) {
  qw_status r = check_plan(p);
  if (r != QW_OK) return r;
  if (!psi0 || !origin) return fail(QW_ERR_INVALID, "NULL argument");
  for (int i = 0; i < p->dim; ++i)
    if (!isfinite(origin[i])) return fail(QW_ERR_INVALID, "origin is not finite");
  r = check_time(t);
  if (r != QW_OK) return r;
  void* dst = psi_t;
  if (!dst) {  // intermediate passes need a field; the result is not kept
    r = ensure_scratch(p, p->field_bytes);
    if (r != QW_OK) return r;
    dst = p->d_scratch;
  }
  InstParam ip;
  ip.m = p->m;
  ip.n = p->n;
  ip.t = (double)t;
  const int64_t nb = (int64_t)p->s * fused_obs_blocks(p);
  if (nb > 0) {
    const ObsFuse f = make_fuse(p, origin, nullptr, p->d_partials, psi_t != nullptr);
    r = evolve_impl(p, 1, psi0, dst, nullptr, ip, st, &f);
    if (r != QW_OK) return r;
    HIP_TRY(launch_reduce_partials(1, nb, p->d_partials, p->d_partials + nb * kObsFields,
                                   p->d_result, st));
  } else {
    r = evolve_impl(p, 1, psi0, dst, nullptr, ip, st, nullptr);
    if (r != QW_OK) return r;
    ObsGeom g = obs_geom(p);
    for (int i = 0; i < p->dim; ++i) g.c[i] = origin[i];
    HIP_TRY(launch_observables(p->dbl, g, 1, dst, nullptr, nullptr, p->d_partials, p->d_result,
                               st));
  }
  return QW_OK;
}

qw_status qw_evolve_fft_observables(qw_plan_t p, const void* psi0, void* psi_t, int64_t t,
                                    const double* origin, qw_obs* out, void* stream) {
  return traced("qw_evolve_fft_observables", stream, [&]() -> qw_status {
    if (!out) return fail(QW_ERR_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    qw_status r = obs_jump_launch(p, psi0, psi_t, t, origin, st);
    if (r != QW_OK) return r;
    HIP_TRY(hipMemcpyAsync(p->h_result, p->d_result, sizeof(double) * kObsFields,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    finish_obs(p, p->h_result, origin, out);
    out->overlap_re = out->overlap_im = out->ref_norm2 = 0.0;
    return QW_OK;
  });
}

qw_status qw_evolve_fft_observables_async(qw_plan_t p, const void* psi0, void* psi_t, int64_t t,
                                          const double* origin, double* raw, void* stream) {
  return traced("qw_evolve_fft_observables_async", stream, [&]() -> qw_status {
    if (!raw) return fail(QW_ERR_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    qw_status r = obs_jump_launch(p, psi0, psi_t, t, origin, st);
    if (r != QW_OK) return r;
    HIP_TRY(hipMemcpyAsync(raw, p->d_result, sizeof(double) * kObsFields, hipMemcpyDeviceToHost,
                           st));
    return QW_OK;
  });
}

qw_status qw_obs_from_raw(qw_plan_t p, const double* raw, const double* origin, qw_obs* out) {
  qw_status r = check_plan(p);
  if (r != QW_OK) return r;
  if (!raw || !origin || !out) return fail(QW_ERR_INVALID, "NULL argument");
  for (int i = 0; i < p->dim; ++i)
    if (!isfinite(origin[i])) return fail(QW_ERR_INVALID, "origin is not finite");
  finish_obs(p, raw, origin, out);
  out->overlap_re = out->overlap_im = out->ref_norm2 = 0.0;
  return QW_OK;
}

// Result slots of a time series: grow to n times (replaced buffers are kept
// until qw_destroy, like the plan's other buffers).
static qw_status ensure_series(qw_plan_t p, int64_t n) {
  if (p->series_cap >= n) return QW_OK;
  int64_t cap = 64;
  while (cap < n) cap <<= 1;
  const size_t bytes = sizeof(double) * kObsFields * (size_t)cap;
  double* d = nullptr;
  double* h = nullptr;
  HIP_TRY(hipMalloc((void**)&d, bytes));
  hipError_t e = hipHostMalloc((void**)&h, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(d);
    HIP_TRY(e);
  }
  if (p->d_series) p->retired_dev.push_back(p->d_series);
  if (p->h_series) p->retired_host.push_back(p->h_series);
  p->d_series = d;
  p->h_series = h;
  p->series_cap = cap;
  return QW_OK;
}

// Times of a series whose fused reductions are summed by one launch: their
// partial vectors are kept side by side (at 256^3 complex64, 64 times of
// 8192 partial vectors are 55 MB) and reduced as instances of a batch, each
// in the fixed order of a single reduction.
constexpr int64_t kSeriesChunk = 64;

static qw_status ensure_series_part(qw_plan_t p, int64_t nb) {
  const int64_t len = kSeriesChunk * (nb + 64) * kObsFields;
  if (p->series_part_len >= len) return QW_OK;
  double* d = nullptr;
  HIP_TRY(hipMalloc((void**)&d, sizeof(double) * len));
  if (p->d_series_part) p->retired_dev.push_back(p->d_series_part);
  p->d_series_part = d;
  p->series_part_len = len;
  return QW_OK;
}

qw_status qw_evolve_fft_series(qw_plan_t p, const void* psi0, int64_t n, const int64_t* t,
                               const double* origin, qw_obs* out, void* stream) {
  return traced("qw_evolve_fft_series", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    if (!psi0 || !t || !origin || !out) return fail(QW_ERR_INVALID, "NULL argument");
    if (n < 1 || n > (int64_t(1) << 20)) return fail(QW_ERR_INVALID, "n must lie in [1, 2^20]");
    for (int i = 0; i < p->dim; ++i)
      if (!isfinite(origin[i])) return fail(QW_ERR_INVALID, "origin is not finite");
    for (int64_t i = 0; i < n; ++i) {
      r = check_time(t[i]);
      if (r != QW_OK) return r;
    }
    hipStream_t st = (hipStream_t)stream;
    r = ensure_series(p, n);
    if (r != QW_OK) return r;
    const int64_t nb = (int64_t)p->s * fused_obs_blocks(p);
    if (nb > 0) {
      r = ensure_series_part(p, nb);
      if (r != QW_OK) return r;
    }
    // The spectrum of psi0 once, then per time the apply with the inverse
    // transform; that needs the natural-order spectrum and a strided pass
    // to take the reductions in (d = 2, 3), else each time is a full jump.
    const bool spectral = !p->weyl && !p->fourstep && nb > 0;
    r = ensure_scratch(p, (spectral ? 2 : 1) * p->field_bytes);
    if (r != QW_OK) return r;
    char* spec = (char*)p->d_scratch;
    void* work = spectral ? (void*)(spec + p->field_bytes) : p->d_scratch;
    const int64_t L = contig_len(p);
    const double* omega = nullptr;
    if (spectral) {
      r = transform_impl(p, 1, psi0, spec, +1, nullptr, st);
      if (r != QW_OK) return r;
      omega = omega_table(p, st);
    }
    double* part = p->d_series_part;  // [kSeriesChunk][nb][kObsFields], then the middle sums
    double* mid = part + kSeriesChunk * nb * kObsFields;
    for (int64_t i = 0; i < n; ++i) {
      InstParam ip;
      ip.m = p->m;
      ip.n = p->n;
      ip.t = (double)t[i];
      double* res = p->d_series + (size_t)kObsFields * i;
      double* my_part = part + (i % kSeriesChunk) * nb * kObsFields;
      if (spectral) {
        PassGeom g = pass_geom(p, L, 1);
        g.single = ip;
        g.omega = omega;
        const int mode = omega ? MODE_APPLY_INV_TAB : MODE_APPLY_INV;
        HIP_TRY(launch_fft_contig(p->dbl, mode, L, work, spec, g, p->d_tw, st, p->ce));
        const ObsFuse f = make_fuse(p, origin, nullptr, my_part, false);
        r = strided_passes(p, -1, work, work, 1, st, &f);
        if (r != QW_OK) return r;
      } else if (nb > 0) {
        const ObsFuse f = make_fuse(p, origin, nullptr, my_part, false);
        r = evolve_impl(p, 1, psi0, work, nullptr, ip, st, &f);
        if (r != QW_OK) return r;
      } else {
        r = evolve_impl(p, 1, psi0, work, nullptr, ip, st, nullptr);
        if (r != QW_OK) return r;
        ObsGeom og = obs_geom(p);
        for (int a = 0; a < p->dim; ++a) og.c[a] = origin[a];
        HIP_TRY(launch_observables(p->dbl, og, 1, work, nullptr, nullptr, p->d_partials, res, st));
      }
      // the chunk's reductions, once its last time is in
      if (nb > 0 && (i % kSeriesChunk == kSeriesChunk - 1 || i == n - 1)) {
        const int64_t c0 = i - i % kSeriesChunk;
        HIP_TRY(launch_reduce_partials((int)(i - c0 + 1), nb, part, mid,
                                       p->d_series + (size_t)kObsFields * c0, st));
      }
    }
    HIP_TRY(hipMemcpyAsync(p->h_series, p->d_series, sizeof(double) * kObsFields * (size_t)n,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) {
      finish_obs(p, p->h_series + (size_t)kObsFields * i, origin, &out[i]);
      out[i].overlap_re = out[i].overlap_im = out[i].ref_norm2 = 0.0;
    }
    return QW_OK;
  });
}

qw_status qw_newton_wigner(qw_plan_t p, const void* psi, const double* origin, qw_obs* sectors,
                           double* nw, void* stream) {
  return traced("qw_newton_wigner", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    r = dirac_only(p, "qw_newton_wigner");
    if (r != QW_OK) return r;
    if (!psi || !origin || !sectors || !nw) return fail(QW_ERR_INVALID, "NULL argument");
    for (int i = 0; i < p->dim; ++i)
      if (!isfinite(origin[i])) return fail(QW_ERR_INVALID, "origin is not finite");
    if (p->fourstep)
      return fail(QW_ERR_UNSUPPORTED, "1D lattices above 4096 sites keep a transposed spectrum");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nb = (int64_t)p->s * fused_obs_blocks(p);
    const size_t fb = p->field_bytes;
    const size_t part_bytes =
        sizeof(double) * kObsFields * (size_t)std::max<int64_t>(2 * nb + 2 * 64, 2 * kObsBlocks);
    r = ensure_scratch(p, 2 * fb + part_bytes);
    if (r != QW_OK) return r;
    char* base = (char*)p->d_scratch;
    void* f0 = base;
    void* f1 = base + fb;
    double* part = (double*)(base + 2 * fb);
    // spectrum of psi, twice; sector projector and inverse of instance 0 (+)
    // and 1 (-); reductions of both about the origin
    r = transform_impl(p, 1, psi, f0, +1, nullptr, st);
    if (r != QW_OK) return r;
    HIP_TRY(hipMemcpyAsync(f1, f0, fb, hipMemcpyDeviceToDevice, st));
    const int64_t L = contig_len(p);
    PassGeom g = pass_geom(p, L, 2);
    HIP_TRY(launch_fft_contig(p->dbl, MODE_PROJ_INV, L, f0, f0, g, p->d_tw, st, 8));
    if (nb > 0) {
      const ObsFuse f = make_fuse(p, origin, nullptr, part, false);
      r = strided_passes(p, -1, f0, f0, 2, st, &f);
      if (r != QW_OK) return r;
      HIP_TRY(launch_reduce_partials(2, nb, part, part + 2 * nb * kObsFields, p->d_result, st));
    } else {
      if (has_strided(p)) {
        r = strided_passes(p, -1, f0, f0, 2, st, nullptr);
        if (r != QW_OK) return r;
      }
      ObsGeom og = obs_geom(p);
      for (int i = 0; i < p->dim; ++i) og.c[i] = origin[i];
      HIP_TRY(launch_observables(p->dbl, og, 2, f0, nullptr, nullptr, part, p->d_result, st));
    }
    HIP_TRY(hipMemcpyAsync(p->h_result, p->d_result, sizeof(double) * 2 * kObsFields,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int k = 0; k < 2; ++k) {
      finish_obs(p, p->h_result + k * kObsFields, origin, &sectors[k]);
      sectors[k].overlap_re = sectors[k].overlap_im = sectors[k].ref_norm2 = 0.0;
    }
    const double w0 = sectors[0].norm2, w1 = sectors[1].norm2, ws = w0 + w1;
    for (int i = 0; i < 6; ++i) nw[i] = 0.0;
    if (ws > 0.0)
      for (int i = 0; i < 3; ++i) {
        nw[i] = (w0 * sectors[0].mean[i] + w1 * sectors[1].mean[i]) / ws;
        nw[3 + i] = (w0 * sectors[0].mean_cart[i] + w1 * sectors[1].mean_cart[i]) / ws;
      }
    return QW_OK;
  });
}

qw_status qw_marginals(qw_plan_t p, const void* psi, const int64_t* origin, double* out,
                       int64_t out_len, int64_t* xmin, int64_t* len, void* stream) {
  return traced("qw_marginals", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    if (!xmin || !len) return fail(QW_ERR_INVALID, "NULL argument");
    // Cartesian components of the generators (columns h_j): x = sum_j w_j h_j.
    static const int H1[3][3] = {{1, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    static const int H2[3][3] = {{1, 1, 0}, {1, -1, 0}, {0, 0, 0}};
    static const int H3[3][3] = {{1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
    const int(*H)[3] = p->dim == 1 ? H1 : (p->dim == 2 ? H2 : H3);
    MargGeom g;
    memset(&g, 0, sizeof g);
    g.dim = p->dim;
    g.V = p->V;
    g.s = p->s;
    int total = 0;
    for (int i = 0; i < p->dim; ++i) {
      g.N[i] = p->N[i];
      g.lg[i] = p->lg[i];
      int lo = 0, hi = 0;
      for (int j = 0; j < p->dim; ++j) {
        g.H[i][j] = H[i][j];
        const int half = (int)(p->N[j] / 2);
        if (H[i][j] > 0) {
          lo -= half;
          hi += half - 1;
        } else if (H[i][j] < 0) {
          lo -= half - 1;
          hi += half;
        }
      }
      g.xmin[i] = lo;
      g.off[i] = total;
      xmin[i] = lo;
      len[i] = hi - lo + 1;
      total += hi - lo + 1;
    }
    g.total = total;
    if (!out) return QW_OK;  // layout query
    if (!psi || !origin) return fail(QW_ERR_INVALID, "NULL argument");
    if (out_len < total) return fail(QW_ERR_INVALID, "out holds %lld values, %d needed",
                                     (long long)out_len, total);
    if (p->dim > 1 && (size_t)total * sizeof(double) > 64 * 1024)
      return fail(QW_ERR_UNSUPPORTED, "marginal bins exceed 64 KB of LDS");
    for (int i = 0; i < p->dim; ++i) g.c[i] = (int)(origin[i] & (p->N[i] - 1));
    hipStream_t st = (hipStream_t)stream;
    const int64_t nb = p->dim == 1 ? 0 : marginal_blocks(g);
    const size_t bytes = sizeof(double) * ((size_t)nb * total + total);
    r = ensure_scratch(p, bytes);
    if (r != QW_OK) return r;
    double* part = (double*)p->d_scratch;
    double* dout = part + (size_t)nb * total;
    HIP_TRY(launch_marginals(p->dbl, g, psi, part, dout, st));
    HIP_TRY(hipMemcpyAsync(out, dout, sizeof(double) * total, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return QW_OK;
  });
}

qw_status qw_kspace_drift(qw_plan_t p, const void* psi, qw_drift* out, void* stream) {
  return traced("qw_kspace_drift", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    if (!psi || !out) return fail(QW_ERR_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    r = ensure_scratch(p, p->field_bytes);
    if (r != QW_OK) return r;
    // The spectrum in the storage order of the fused pass (the forward half of
    // the evolution), in the plan's scratch field.
    const int64_t L = contig_len(p);
    PassGeom g = pass_geom(p, L, 1);
    if (has_strided(p)) {
      r = strided_passes(p, +1, p->d_scratch, psi, 1, st, nullptr);
      if (r != QW_OK) return r;
      HIP_TRY(launch_fft_contig(p->dbl, MODE_FWD, L, p->d_scratch, p->d_scratch, g, p->d_tw, st));
    } else {
      HIP_TRY(launch_fft_contig(p->dbl, MODE_FWD, L, p->d_scratch, psi, g, p->d_tw, st));
    }
    HIP_TRY(launch_kdrift(p->dbl, g, L, p->d_scratch, p->d_partials, p->d_result, st));
    HIP_TRY(hipMemcpyAsync(p->h_result, p->d_result, sizeof(double) * 5, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double* R = p->h_result;
    memset(out, 0, sizeof *out);
    const double inv = R[0] > 0.0 ? 1.0 / R[0] : 0.0;
    for (int i = 0; i < p->dim; ++i) out->velocity[i] = -R[2 + i] * inv;
    const double* v = out->velocity;
    if (p->dim == 1) {
      out->velocity_cart[0] = v[0];
    } else if (p->dim == 2) {
      out->velocity_cart[0] = v[0] + v[1];
      out->velocity_cart[1] = v[0] - v[1];
    } else {
      out->velocity_cart[0] = v[0] + v[1] - v[2];
      out->velocity_cart[1] = v[0] - v[1] + v[2];
      out->velocity_cart[2] = v[0] - v[1] - v[2];
    }
    // Parseval: |hat psi|^2 sums to V |psi|^2 with the unnormalised transform.
    const double iv = 1.0 / (double)p->V;
    out->norm2 = R[0] * iv;
    out->sector_norm2[0] = 0.5 * (R[0] + R[1]) * iv;
    out->sector_norm2[1] = 0.5 * (R[0] - R[1]) * iv;
    return QW_OK;
  });
}

qw_status qw_observables(qw_plan_t p, const void* psi, const double* origin, const void* ref,
                         qw_obs* out, void* stream) {
  return traced("qw_observables", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    if (!psi || !origin || !out) return fail(QW_ERR_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    ObsGeom g = obs_geom(p);
    for (int i = 0; i < p->dim; ++i) {
      if (!isfinite(origin[i])) return fail(QW_ERR_INVALID, "origin is not finite");
      g.c[i] = origin[i];
    }
    HIP_TRY(launch_observables(p->dbl, g, 1, psi, ref, nullptr, p->d_partials, p->d_result, st));
    HIP_TRY(hipMemcpyAsync(p->h_result, p->d_result, sizeof(double) * kObsFields,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    finish_obs(p, p->h_result, origin, out);
    if (!ref) out->overlap_re = out->overlap_im = out->ref_norm2 = 0.0;
    return QW_OK;
  });
}

// Taylor coefficients of omega(k) = arccos(n u(k)) at k0 (Cartesian), with
// u the identity component of the Weyl symbol (Sec. 3.1; cos omega = n u,
// Sec. 3.2): 1D cos k, 2D cos kx cos ky, 3D cos kx cos ky cos kz +
// sin kx sin ky sin kz. Derivatives by implicit differentiation of
// cos omega = n u: sin(w) dw_i = -n du_i and
// sin(w) dw_ij = -n du_ij - cos(w) dw_i dw_j.
qw_status qw_dispersion_taylor(int dim, double m, const double* k0, int order, double* c) {
  if (dim < 1 || dim > 3) return fail(QW_ERR_INVALID, "dim must be 1, 2 or 3");
  if (!(m >= 0.0 && m <= 1.0)) return fail(QW_ERR_INVALID, "m must lie in [0, 1]");
  if (order < 0 || order > 2) return fail(QW_ERR_UNSUPPORTED, "order must be 0, 1 or 2");
  if (!k0 || !c) return fail(QW_ERR_INVALID, "NULL argument");
  double k[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < dim; ++i) {
    if (!isfinite(k0[i])) return fail(QW_ERR_INVALID, "k0 not finite");
    k[i] = k0[i];
  }
  const double cx_ = cos(k[0]), sx = sin(k[0]), cy = cos(k[1]), sy = sin(k[1]), cz = cos(k[2]),
               sz = sin(k[2]);
  double u, du[3] = {0, 0, 0}, d2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  if (dim == 1) {
    u = cx_;
    du[0] = -sx;
    d2[0][0] = -cx_;
  } else if (dim == 2) {
    u = cx_ * cy;
    du[0] = -sx * cy;
    du[1] = -cx_ * sy;
    d2[0][0] = d2[1][1] = -cx_ * cy;
    d2[0][1] = d2[1][0] = sx * sy;
  } else {
    u = cx_ * cy * cz + sx * sy * sz;
    du[0] = -sx * cy * cz + cx_ * sy * sz;
    du[1] = -cx_ * sy * cz + sx * cy * sz;
    du[2] = -cx_ * cy * sz + sx * sy * cz;
    d2[0][0] = d2[1][1] = d2[2][2] = -u;
    d2[0][1] = d2[1][0] = sx * sy * cz + cx_ * cy * sz;
    d2[0][2] = d2[2][0] = sx * cy * sz + cx_ * sy * cz;
    d2[1][2] = d2[2][1] = cx_ * sy * sz + sx * cy * cz;
  }
  const double n = sqrt(1.0 - m * m);
  const double cw = n * u;
  const double sw = sqrt(fmax(0.0, 1.0 - cw * cw));
  for (int i = 0; i < 10; ++i) c[i] = 0.0;
  c[0] = atan2(sw, cw);
  if (order >= 1) {
    if (!(sw > 1e-12)) return fail(QW_ERR_INVALID, "omega is not differentiable at k0 (sin omega = 0)");
    double dw[3];
    for (int i = 0; i < 3; ++i) dw[i] = -n * du[i] / sw;
    for (int i = 0; i < dim; ++i) c[1 + i] = dw[i];
    if (order >= 2) {
      auto dd = [&](int i, int j) { return (-n * d2[i][j] - cw * dw[i] * dw[j]) / sw; };
      for (int i = 0; i < dim; ++i) c[4 + i] = 0.5 * dd(i, i);
      if (dim >= 2) c[7] = dd(0, 1);
      if (dim >= 3) {
        c[8] = dd(0, 2);
        c[9] = dd(1, 2);
      }
    }
  }
  return QW_OK;
}

static qw_status check_state_args(qw_plan_t p, void* psi, const double* k0, double sigma,
                                  const double* center, double c_plus, double c_minus) {
  if (p->weyl) return fail(QW_ERR_UNSUPPORTED, "particle states are defined for the Dirac walk");
  if (!psi || !k0 || !center) return fail(QW_ERR_INVALID, "NULL argument");
  if (!(sigma > 0.0) || !isfinite(sigma)) return fail(QW_ERR_INVALID, "sigma must be > 0");
  if (!isfinite(c_plus) || !isfinite(c_minus) || (c_plus == 0.0 && c_minus == 0.0))
    return fail(QW_ERR_INVALID, "c_plus, c_minus must be finite and not both zero");
  for (int i = 0; i < p->dim; ++i)
    if (!isfinite(k0[i]) || !isfinite(center[i])) return fail(QW_ERR_INVALID, "k0/center not finite");
  return QW_OK;
}

// Spectrum of the state `si` (with its dispersive phases, if any) and the
// inverse DFT into psi; waits for the sector norms.
static qw_status prepare_impl(qw_plan_t p, void* psi, const StateInst& si, hipStream_t st) {
  if (p->fourstep) {
    qw_status r = ensure_scratch(p, p->field_bytes);
    if (r != QW_OK) return r;
  }
  // The pinned staging area may still feed an earlier call's copy.
  HIP_TRY(hipStreamSynchronize(st));
  *p->h_stage = si;
  HIP_TRY(hipMemcpyAsync(p->d_stage, p->h_stage, sizeof(StateInst), hipMemcpyHostToDevice, st));
  if (state_scratch_doubles(state_geom(p), 1) > p->partials_len)
    return fail(QW_ERR_DEVICE, "state preparation scratch exceeds the plan's partials");
  HIP_TRY(launch_state_prepare(p->dbl, state_geom(p), 1, p->d_stage, p->d_partials, p->d_result,
                               psi, st));
  HIP_TRY(hipMemcpyAsync(p->h_result, p->d_result, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
  qw_status r = transform_impl(p, 1, psi, psi, -1, p->d_scratch, st);
  if (r != QW_OK) return r;
  HIP_TRY(hipStreamSynchronize(st));
  const double np = p->h_result[0], nm = p->h_result[1];
  if ((si.c_plus != 0.0 && !(np > 0.0)) || (si.c_minus != 0.0 && !(nm > 0.0)))
    return fail(QW_ERR_INVALID, "state has zero weight in a requested sector");
  return QW_OK;
}

qw_status qw_prepare_state(qw_plan_t p, void* psi, const double* k0, double sigma,
                           const double* center, double c_plus, double c_minus, void* stream) {
  return traced("qw_prepare_state", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    r = check_state_args(p, psi, k0, sigma, center, c_plus, c_minus);
    if (r != QW_OK) return r;
    return prepare_impl(p, psi, make_state_inst(p, p->m, k0, sigma, center, c_plus, c_minus),
                        (hipStream_t)stream);
  });
}

qw_status qw_evolve_dispersive(qw_plan_t p, void* psi, const double* k0, double sigma,
                               const double* center, double c_plus, double c_minus, int order,
                               double t, void* stream) {
  return traced("qw_evolve_dispersive", stream, [&]() -> qw_status {
    qw_status r = check_plan(p);
    if (r != QW_OK) return r;
    r = check_state_args(p, psi, k0, sigma, center, c_plus, c_minus);
    if (r != QW_OK) return r;
    if (order < 0 || order > 2) return fail(QW_ERR_UNSUPPORTED, "order must be 0, 1 or 2");
    r = check_time(t);
    if (r != QW_OK) return r;
    StateInst si = make_state_inst(p, p->m, k0, sigma, center, c_plus, c_minus);
    r = qw_dispersion_taylor(p->dim, p->m, k0, order, si.tay);
    if (r != QW_OK) return r;
    si.order = order;
    si.tdisp = t;
    return prepare_impl(p, psi, si, (hipStream_t)stream);
  });
}

}  // extern "C"
