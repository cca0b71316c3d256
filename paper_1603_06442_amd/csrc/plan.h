// Plan object and host-side helpers shared by the C ABI and the server.
#pragma once

#include <math.h>
#include <string.h>

#include <complex>
#include <string>
#include <vector>

#include "qw_internal.h"

namespace qw {
typedef std::complex<double> zc;

// Transition matrices U_h for offsets in {-1,0,1}^d (index sum (o_i+1) 3^(d-1-i)).
struct Table {
  int dim, s;
  zc U[27][4][4];
};

qw_status fail(qw_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::qw::fail(e_ == hipErrorOutOfMemory ? QW_ERR_NOMEM : QW_ERR_DEVICE,           \
                        "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)
}  // namespace qw

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct qw_plan_s {
  using Table = qw::Table;
  int dim = 0, s = 0;
  int64_t N[3] = {1, 1, 1};
  int lg[3] = {0, 0, 0};
  int64_t V = 0;
  double m = 0.0, n = 1.0;
  qw_dtype dtype = QW_C64;
  bool dbl = false;
  size_t elem = 8;        // bytes per complex entry
  size_t field_bytes = 0;
  int device = 0;

  Table table;
  qw::StencilCoef<double> coef_d;
  qw::StencilCoef<float> coef_f;

  // FFT schedule
  int Nc = 1;
  int shift[3] = {0, 0, 0};
  bool fourstep = false;
  bool weyl = false;  // two-component Weyl walk (d = 2, 3; s = 2, m = 0)
  int64_t fs_N1 = 1, fs_N2 = 1;

  // device memory
  void* d_tw = nullptr;     // exp(-2 pi i j / 4096), field precision
  void* d_tw4 = nullptr;    // exp(-2 pi i j / N) for the 1D four-step, field precision
  double* d_cs = nullptr;   // (cos, sin)(pi j / Nc), j < 2 Nc
  float* d_csf = nullptr;   // the same, FP32
  double* d_partials = nullptr;  // partial sums of the reductions (partials_len doubles)
  int64_t partials_len = 0;
  double* d_result = nullptr;
  double* h_result = nullptr;  // pinned
  // Results of a time series (qw_evolve_fft_series): kObsFields doubles per
  // time, on the device and pinned; they only grow.
  double* d_series = nullptr;
  double* h_series = nullptr;
  int64_t series_cap = 0;
  // Partial vectors of the fused reductions of up to kSeriesChunk times,
  // reduced together (series_part_len doubles); it only grows.
  double* d_series_part = nullptr;
  int64_t series_part_len = 0;
  void* d_scratch = nullptr;
  size_t scratch_bytes = 0;
  qw::InstParam* d_inst = nullptr;
  qw::InstParam* h_inst = nullptr;  // pinned
  int inst_cap = 0;
  void* d_coef = nullptr;            // the plan's StencilCoef (field precision), device
  void* d_coefs = nullptr;           // per-instance StencilCoef of qw_step_batched
  unsigned char* h_coefs = nullptr;  // pinned staging for d_coefs
  int coefs_cap = 0;
  qw::StateInst* h_stage = nullptr;  // pinned staging of one state's parameters
  qw::StateInst* d_stage = nullptr;
  double* d_omega = nullptr;    // omega(q) at the plan's mass, built on first use
  bool omega_failed = false;
  double* d_omega_bcc = nullptr;  // omega(kappa) of the cubic supercell, built on first use
  bool omega_bcc_failed = false;

  // Schedule of the 3D Fourier evolution (see qw_set_schedule / qw_autotune).
  int slab = 0;  // n1 planes per slab of the middle passes (0 = whole field)
  int ce = 8;    // elements per thread of the fused contiguous pass (4 or 8)
  int cb = 256;  // target workgroup size of the fused contiguous pass
  int gw = 1;    // pencil groups per workgroup of the fused pass (prefetch when > 1)
  bool sparse3 = false;  // 3D transition matrices have the rank-one block pattern

  // Buffers replaced by a larger one (scratch, per-instance parameters and
  // matrices). Work enqueued earlier, or a graph captured earlier, may still
  // read or write them, so they are released only with the plan.
  std::vector<void*> retired_dev, retired_host;

  ~qw_plan_s() {
    for (void* q : retired_dev) (void)hipFree(q);
    for (void* q : retired_host) (void)hipHostFree(q);
    if (d_tw) (void)hipFree(d_tw);
    if (d_tw4) (void)hipFree(d_tw4);
    if (d_cs) (void)hipFree(d_cs);
    if (d_csf) (void)hipFree(d_csf);
    if (d_partials) (void)hipFree(d_partials);
    if (d_result) (void)hipFree(d_result);
    if (h_result) (void)hipHostFree(h_result);
    if (d_series) (void)hipFree(d_series);
    if (d_series_part) (void)hipFree(d_series_part);
    if (h_series) (void)hipHostFree(h_series);
    if (d_scratch) (void)hipFree(d_scratch);
    if (d_inst) (void)hipFree(d_inst);
    if (h_inst) (void)hipHostFree(h_inst);
    if (d_coef) (void)hipFree(d_coef);
    if (d_coefs) (void)hipFree(d_coefs);
    if (h_coefs) (void)hipHostFree(h_coefs);
    if (d_omega) (void)hipFree(d_omega);
    if (d_omega_bcc) (void)hipFree(d_omega_bcc);
    if (h_stage) (void)hipHostFree(h_stage);
    if (d_stage) (void)hipFree(d_stage);
  }
};


namespace qw {
qw_status check_plan(qw_plan_t p);
qw_status dirac_only(qw_plan_t p, const char* what);
qw_status ensure_scratch(qw_plan_t p, size_t bytes);
qw_status ensure_coefs(qw_plan_t p, int B);
// psi_out = U^t psi_in for B instances back to back; dinst: device per-instance
// (m, n, t), or nullptr to use `single` (B = 1, the plan's mass, omega table).
// With `fuse`, the last inverse pass also writes the reduction partials (and
// writes the field only if fuse->store); an error if the schedule ends
// without a strided pass (1D, N <= 4096).
qw_status evolve_impl(qw_plan_t p, int B, const void* in, void* out, const InstParam* dinst,
                      const InstParam& single, hipStream_t st, const ObsFuse* fuse = nullptr);
// 1D lattices longer than this use the four-step split N = N1 * kFourStepL.
constexpr int64_t kFourStepL = 4096;
// Column blocks per component of the fused last pass (0: no fusion possible),
// for a plan and for a lattice shape without one.
int64_t fused_obs_blocks(qw_plan_t p);
int64_t fused_obs_blocks_of(int dim, const int64_t* N, bool dbl);
ObsFuse make_fuse(qw_plan_t p, const double* origin, const double* origins, double* partials,
                  bool store);
// psi_t = T^-1 [D_q^t a(q)] in place for B spectra in storage order, device
// per-instance (m, n, t); QW_ERR_UNSUPPORTED for the 1D four-step.
qw_status evolve_spectrum_impl(qw_plan_t p, int B, void* data, const InstParam* dinst,
                               hipStream_t st, const ObsFuse* fuse = nullptr);
// Unnormalised DFT of B instances (direction +1 / -1); `scratch` holds B
// fields for the 1D four-step transposes (unused otherwise; may be null then).
qw_status transform_impl(qw_plan_t p, int B, const void* in, void* out, int direction,
                         void* scratch, hipStream_t st);
// Per-instance state parameters (chi_s from the projectors at q' = H^T k0).
StateInst make_state_inst(qw_plan_t p, double m, const double* k0, double sigma,
                          const double* center, double c_plus, double c_minus);
StateGeom state_geom(qw_plan_t p);
ObsGeom obs_geom(qw_plan_t p);
void finish_obs(qw_plan_t p, const double* R, const double* origin, qw_obs* out);
}  // namespace qw
