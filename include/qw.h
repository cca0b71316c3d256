/*
 * qw.h -- C ABI of the MI355X (gfx950) Dirac quantum-walk library (libqw.so).
 *
 * The library evolves the spinor field of the discrete-time Dirac quantum
 * walk of D'Ariano, Mosco, Perinotti and Tosini, "Discrete Time Dirac Quantum
 * Walk in 3+1 Dimensions", on a periodic lattice, in the two ways Sec. 4 of
 * the paper names: step by step in position space, and in one jump through
 * the Fourier representation. It also computes the position and overlap
 * reductions of Sec. 5.
 *
 * Lattices (Sec. 3.1): d = 1 (the line), d = 2 (the square lattice), d = 3
 * (the BCC lattice). Sites are stored in primitive-cell coordinates
 * n = (n_1, .., n_d), 0 <= n_i < N_i, periodic; the Cartesian site is
 * x = sum_j n_j h_j with h_j the generators: 3D h1 = (1,1,1), h2 = (1,-1,-1),
 * h3 = (-1,1,-1); 2D h1 = (1,1), h2 = (1,-1); 1D h = 1.
 *
 * Field layout (all field pointers are DEVICE pointers owned by the caller):
 *   component-major planes, psi[c * V + lin(n)], V = N_1 * .. * N_d,
 *   lin(n) row-major with n_d fastest; each entry is an interleaved complex
 *   number (re, im): two floats for QW_C64, two doubles for QW_C128.
 *   The spinor has s = 2 components for d = 1 and s = 4 for d = 2, 3, in the
 *   row order of the matrix D_k printed in Sec. 3.2.
 *   One field occupies s * V * (8 or 16) bytes and must be 16-byte aligned.
 *
 * Execution: every call is enqueued on `stream` (a hipStream_t; NULL is the
 * null stream) and returns without waiting, except qw_observables,
 * qw_evolve_fft_observables and qw_prepare_state, which wait for their
 * results (qw_evolve_fft_observables_async is the non-waiting form of the
 * second), and the batched calls, which wait for `stream` before staging
 * their per-instance parameters. A plan may be used by one stream at a
 * time; distinct plans are independent.
 *
 * Graph capture: qw_step, qw_evolve_fft, qw_evolve_fft_real, qw_transform,
 * qw_bcc_step, qw_bcc_transform and qw_bcc_evolve_fft enqueue only kernels and
 * device-to-device copies and never synchronise, so a caller may capture them
 * into a HIP graph and replay it. Their first call on a plan may allocate
 * (scratch, the omega tables); make one call outside the capture first.
 * A plan's scratch and parameter buffers only grow: a buffer replaced by a
 * larger one (a later call on more fields, two fields, B instances) is kept
 * until qw_destroy, so work enqueued before and graphs captured before stay
 * valid, and growth never synchronises the device.
 *
 * Errors: every call returns a qw_status; nothing throws across the ABI.
 * qw_last_error() returns a message for the last failing call of the calling
 * thread. Arguments are validated before any work is enqueued, so a call
 * that returns QW_ERR_INVALID or QW_ERR_UNSUPPORTED has changed nothing.
 *
 * Tracing and debugging: each plan-level entry point runs inside a roctx
 * range named after it (rocprofv3 --marker-trace shows them). With the
 * environment variable QW_DEBUG set (to anything but 0; read on every call)
 * an entry point that enqueued work waits for its stream and reports a
 * failed kernel as QW_ERR_DEVICE naming itself, except while the stream is
 * being captured into a graph.
 */
#ifndef QW_H
#define QW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qw_plan_s* qw_plan_t;

typedef enum {
  QW_OK = 0,
  QW_ERR_INVALID = 1,      /* bad argument (null pointer, m outside [0,1], ...) */
  QW_ERR_UNSUPPORTED = 2,  /* valid but not provided (N not a power of two, too large) */
  QW_ERR_NOMEM = 3,        /* device or host allocation failed */
  QW_ERR_DEVICE = 4,       /* a HIP call or kernel launch failed */
  QW_ERR_CANCELLED = 5     /* serving: the request was cancelled before it ran */
} qw_status;

/* The last two enumerators give the type the range of int, so that any value
 * a caller passes is representable and rejected, not undefined behaviour. */
typedef enum {
  QW_C64 = 0,
  QW_C128 = 1,
  QW_DTYPE_INT_MIN_ = -0x7fffffff - 1,
  QW_DTYPE_INT_MAX_ = 0x7fffffff
} qw_dtype;

/* Reductions of one field (Sec. 5.2: position operator X and <psi|X|psi>;
 * Sec. 5.1: the overlap <phi|psi>). Positions are taken about a caller origin
 * c with the minimum image w_i = ((n_i - c_i + N_i/2) mod N_i) - N_i/2 in
 * [-N_i/2, N_i/2) per primitive axis; unused axes are 0. */
typedef struct {
  double norm2;        /* sum over sites and components of |psi|^2 */
  double mean[3];      /* c_i + sum w_i |psi|^2 / norm2 (primitive coordinates) */
  double second[6];    /* sum w_i w_j |psi|^2 / norm2 for ij = 00,11,22,01,02,12 */
  double mean_cart[3]; /* sum_j mean_j h_j (Cartesian) */
  double overlap_re;   /* Re sum conj(ref) psi   (0 if ref is NULL) */
  double overlap_im;   /* Im sum conj(ref) psi   (0 if ref is NULL) */
  double ref_norm2;    /* sum |ref|^2            (0 if ref is NULL) */
} qw_obs;

/* Create a plan for one lattice shape and mass (Sec. 3.2: the Dirac walk
 * D_k = [[n W_k, i m], [i m, n W_k^dag]], n = sqrt(1 - m^2); in 1D the
 * two-component form [[n e^{-ik}, i m], [i m, n e^{ik}]]).
 *   dim    1, 2 or 3.
 *   N      dim entries, each a power of two: 1D 2..65536; 2D 2..1024 per axis;
 *          3D 2..512 per axis. Other values give QW_ERR_UNSUPPORTED.
 *   m      mass, 0 <= m <= 1 (QW_ERR_INVALID otherwise, NaN included).
 *   dtype  arithmetic of the field: QW_C64 (complex FP32; the phase
 *          omega(k) t is still formed and reduced in FP64) or QW_C128.
 *   stream stream for the set-up uploads.
 * The plan derives the transition matrices U_h of the update rule from the
 * symbol (Sec. 2.1, U_k = sum_h e^{-ik.h} U_h) in FP64 and checks the
 * unitarity conditions of Sec. 2 on them; it owns its device tables and
 * scratch memory, released by qw_destroy. */
qw_status qw_plan(qw_plan_t* out, int dim, const int64_t* N, double m, qw_dtype dtype,
                  void* stream);

/* A plan for the two-component Weyl walk of Sec. 3.1 (W_k = u_k I -
 * i sigma.n~_k; 2D on the square lattice, 3D on the BCC lattice, with the
 * same primitive-cell coordinates, sizes and dtype rules as qw_plan). The
 * field has s = 2 components (the layout above with s = 2). Its transition
 * matrices are the upper blocks of the Dirac walk's at m = 0, whose symbol is
 * diag(W_k, W_k^dag). qw_step, qw_evolve_fft, qw_evolve_fft_real (W_k^t =
 * cos(omega t) I - i sin(omega t)/sin(omega) sigma.n~, cos(omega) = u_k; at
 * omega = pi the average cos(pi t) I, as for the Dirac walk),
 * qw_evolve_fft_timed, qw_evolve_fft_observables, qw_transform,
 * qw_observables, qw_marginals, qw_kspace_drift and the schedule calls take
 * such a plan; the
 * batched calls, the particle-state calls, qw_newton_wigner and the
 * cubic-supercell calls return QW_ERR_UNSUPPORTED. dim = 1 gives the Dirac
 * plan at m = 0, which is the 1D Weyl walk diag(e^{-ik}, e^{ik}). */
qw_status qw_plan_weyl(qw_plan_t* out, int dim, const int64_t* N, qw_dtype dtype, void* stream);

/* Release a plan and everything it owns. Waits for the plan's work. NULL is a no-op. */
qw_status qw_destroy(qw_plan_t plan);

/* nsteps >= 0 applications of the update rule psi(x,t+1) = sum_h U_h psi(x+h,t)
 * (Sec. 2, update rule and walk operator), in place on psi. The plan's
 * scratch holds the second buffer of the ping-pong; a 1D field of at most
 * 160 KB (N <= 8192) stays in on-chip memory for up to 4096 steps per launch
 * instead. */
qw_status qw_step(qw_plan_t plan, void* psi, int64_t nsteps, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that must not call hipMalloc):
 * qw_step with its ping-pong buffer in a fixed device array of
 * QW_NOALLOC_SCRATCH_BYTES (64 MiB), which the library holds on every device
 * it runs on until the process ends, instead of the plan's scratch. It
 * allocates nothing, on its first call too, and gives qw_step's result bit
 * for bit. The field (s * V * 8 or 16 bytes) must fit the array, else
 * QW_ERR_UNSUPPORTED (3D up to 128^3 in complex64, 2D up to 1024^2; 1D
 * fields that stay on chip use no buffer); the plan's device must be current
 * (QW_ERR_INVALID). Every call on one device shares that device's array and
 * leaves its last contents there: calls that overlap in time on one device
 * (several streams or threads) race and must be serialised by the caller. */
#define QW_NOALLOC_SCRATCH_BYTES (64u << 20)
qw_status qw_step_noalloc(qw_plan_t plan, void* psi, int64_t nsteps, void* stream);

/* The same for B (0..65535) fields of the plan's shape and precision back to
 * back in psi (DEVICE), instance b with its own mass m[b] (HOST, 0 <= m[b]
 * <= 1): its transition matrices are derived from the symbol exactly as
 * qw_plan derives the plan's. An instance with the plan's mass gets the
 * same result as qw_step, bit for bit. The plan's scratch grows to B fields
 * (none for the on-chip 1D case). Waits for the previous call's parameter
 * upload on `stream` before staging the masses. */
qw_status qw_step_batched(qw_plan_t plan, int B, void* psi, const double* m, int64_t nsteps,
                          void* stream);

/* psi_t = U^t psi0 in one jump through the Fourier representation (Sec. 4):
 * forward DFT with the sign of Sec. 4, per wave-vector the closed form
 * D_q^t = cos(omega t) I - i sin(omega t)/sin(omega) M_q (from
 * D_q = cos(omega) I - i M_q, Sec. 3.2 gamma-matrix form and interpolating
 * Hamiltonian), inverse DFT. |t| <= 2^53 (else QW_ERR_UNSUPPORTED); t < 0
 * gives U^{-|t|}. psi_t may equal psi0 (in place); partial overlap is
 * invalid. */
qw_status qw_evolve_fft(qw_plan_t plan, const void* psi0, void* psi_t, int64_t t, void* stream);

/* The same for real t: the continuous-time evolution exp(-i H t) of Sec. 4
 * that interpolates the walk (H the interpolating Hamiltonian of Sec. 3.2,
 * eigenvalues +-omega(q) in [0, pi]); equal to qw_evolve_fft, bit for bit,
 * at integer t. Where omega = pi (the band edge, reached only for m = 0)
 * the two branches +-pi are averaged, giving cos(pi t) I there. t finite,
 * |t| <= 2^53. */
qw_status qw_evolve_fft_real(qw_plan_t plan, const void* psi0, void* psi_t, double t,
                             void* stream);

/* B independent instances of one plan shape, each with its own mass and time:
 * in and out hold B fields back to back (instance b at byte offset
 * b * s * V * sizeof(complex)); m[b] and t[b] are HOST arrays. out may equal in. */
qw_status qw_evolve_fft_batched(qw_plan_t plan, int B, const void* in, void* out,
                                const double* m, const int64_t* t, void* stream);

/* The unnormalised DFT of every component of a field (Sec. 4):
 * direction +1: out(q) = sum_n e^{+i q.n} psi(n); direction -1:
 * out(n) = sum_q e^{-i q.n} in(q) (no 1/V). q_i = 2 pi j_i / N_i with the
 * unshifted index j_i in [0, N_i). out may equal in. */
qw_status qw_transform(qw_plan_t plan, const void* in, void* out, int direction, void* stream);

/* Cubic-supercell representation of the BCC lattice (Sec. 4, the paragraph
 * on the BCC DFT, eq:bcc-dft and eq:bcc-idft). The BCC vertex set is
 * G = 2Z^3 u (2Z^3 + t), t = (1,1,1) (the Cartesian sites whose coordinates
 * share one parity; Cartesian x here is the x of the header above), taken
 * periodic with period 2 N_i along Cartesian axis i. It is stored as the two
 * sublattice arrays f0_n = f(2n) and f1_n = f(2n + t), n in
 * [0,N1) x [0,N2) x [0,N3), where N1, N2, N3 are the sizes of a 3D plan
 * (its mass and dtype apply; its primitive-cell torus is not used). Layout:
 * f[(j * s + c) * V + lin(n)], sublattice j = 0, 1 first, then the spinor
 * component c, then n as in the field layout above; 2 * s * V complex
 * entries, 16-byte aligned, DEVICE memory owned by the caller. This torus
 * holds 2 N1 N2 N3 sites and differs from the plan's primitive-cell torus
 * of N1 N2 N3 sites; on a state far from both boundaries the two walks
 * agree site by site.
 *
 * qw_bcc_transform: direction +1 writes (hat f0, hat f1) of eq:bcc-dft in
 * the same layout, with F the rectangular DFT of each sublattice array with
 * the sign of Sec. 4, normalised by 1/sqrt(V), unshifted (k_i in [0, N_i))
 * and a_k = e^{i pi sum_i k_i / N_i}: hat f1_k is the spectrum at the
 * Cartesian wave-vector kappa = (pi k_1/N_1, pi k_2/N_2, pi k_3/N_3) and
 * hat f0_k the one at kappa + (pi, 0, 0). The transform is unitary;
 * direction -1 applies eq:bcc-idft, its inverse. out may equal in. A plan of
 * dim != 3 gives QW_ERR_UNSUPPORTED. */
qw_status qw_bcc_transform(qw_plan_t plan, const void* in, void* out, int direction,
                           void* stream);

/* nsteps steps of the update rule of Sec. 2 on the cubic-supercell field f
 * (layout above), in place: psi(x) <- sum_h U_h psi(x + h) with the
 * transition matrices at their Cartesian displacements, the eight
 * neighbours (+-1, +-1, +-1) lying on the other sublattice and the mass term
 * on the site itself. nsteps >= 0. Uses two fields of plan scratch. */
qw_status qw_bcc_step(qw_plan_t plan, void* f, int64_t nsteps, void* stream);

/* Norm and position moments of the cubic-supercell field f (Sec. 5.2, the
 * position expectation; FP64 accumulation): Cartesian minimum-image
 * displacements w of every site x = 2n + j (1,1,1) about the Cartesian point
 * origin (3 HOST doubles) on the torus of period 2 N_i, so that mean = origin
 * + sum w |f|^2 / norm2 and second = sum w_i w_j |f|^2 / norm2 (pairs 00, 11,
 * 22, 01, 02, 12), all Cartesian (mean_cart = mean; overlap fields 0). out:
 * HOST. Waits for the result. */
qw_status qw_bcc_observables(qw_plan_t plan, const void* f, const double* origin, qw_obs* out,
                             void* stream);

/* f_t = U^t f0 on the cubic-supercell torus: eq:bcc-dft, per k the closed
 * form D^t of qw_evolve_fft at kappa applied to hat f1 and at kappa + (pi,0,0)
 * applied to hat f0, eq:bcc-idft; one read and one write of the field per
 * transform axis (the combine, the powers and the recombination are fused
 * into the pass along n3). t real as in qw_evolve_fft_real (exact integer
 * powers up to 2^53). f_t may equal f0. */
qw_status qw_bcc_evolve_fft(qw_plan_t plan, const void* f0, void* f_t, double t, void* stream);

/* The drift law of Sec. 5.1 (drift vector; Sec. 5.2, the classical part of
 * the mean position), from the spectrum of psi: each frequency sector moves
 * along -grad_q omega, so the drift part of the mean position changes by
 *   velocity = -sum_q grad_q omega(q) (|P+ hat psi(q)|^2 - |P- hat psi(q)|^2)
 *              / sum_q |hat psi(q)|^2
 * per step (primitive coordinates; the Zitterbewegung term is left out),
 * with P+- = (I +- M_q / sin(omega)) / 2 the sector projectors and
 * grad_q omega = -n grad_q u / sin(omega). Also the sector weights
 * <psi|P+-|psi> (= ||P+- psi||^2) and ||psi||^2. Wave-vectors with
 * sin(omega) < 1e-12 (only at m = 0), where the two sectors coincide, add
 * nothing to the drift and split their weight evenly between the sectors.
 * Uses the plan's scratch field; waits for the result. Weyl plans:
 * M = sigma . n~. */
typedef struct {
  double velocity[3];      /* primitive coordinates, per step */
  double velocity_cart[3]; /* sum_j velocity_j h_j */
  double sector_norm2[2];  /* <psi|P+|psi>, <psi|P-|psi> */
  double norm2;            /* ||psi||^2 */
} qw_drift;
qw_status qw_kspace_drift(qw_plan_t plan, const void* psi, qw_drift* out, void* stream);

/* Reductions of psi (see qw_obs). origin: dim HOST doubles. ref: NULL or a
 * DEVICE field of the same shape. out: HOST. Waits for the result. */
qw_status qw_observables(qw_plan_t plan, const void* psi, const double* origin, const void* ref,
                         qw_obs* out, void* stream);

/* Mean position without the interference of the two frequency sectors
 * (the Newton-Wigner position of the closing remark of Sec. 5.2, taken
 * gauge-free): psi is split into P_+ psi and P_- psi with the spectral
 * projectors P_s = (I + s M_q / sin omega) / 2 of U_q, and the reductions of
 * each part are taken about origin (as qw_observables). sectors[0], [1]
 * (HOST) receive those of P_+ psi and P_- psi (norm2 = sector weight);
 * nw[0..2] (HOST) the weighted mean in lattice coordinates and nw[3..5] in
 * Cartesian coordinates. For a state of one sector this is the ordinary
 * mean; under the evolution it moves by the drift alone (no
 * Zitterbewegung). The plan's scratch grows to two fields. 1D lattices above
 * 4096 sites: QW_ERR_UNSUPPORTED. Waits for the result. */
qw_status qw_newton_wigner(qw_plan_t plan, const void* psi, const double* origin, qw_obs* sectors,
                           double* nw, void* stream);

/* Probability marginals along the Cartesian axes (the projections shown
 * for the localised state of Sec. 5.2): every site n adds |psi(n)|^2 to the
 * bin X = (H w)_i of axis i, with w the minimum image of n - origin (origin:
 * dim HOST integers, lattice coordinates) and H the generators of the
 * lattice. On return xmin[i] and len[i] (HOST, dim each) give the bins of
 * axis i, X = xmin[i] .. xmin[i] + len[i] - 1; out (HOST, out_len doubles)
 * holds axis 0's len[0] values, then axis 1's, ... With out = NULL only the
 * layout is returned (psi is not read). d = 2, 3 need the bins of all axes
 * within 64 KB (N <= 1024 in 2D, 512 in 3D). Waits for the result; the
 * summation order inside a workgroup is not fixed (results agree to
 * rounding). */
qw_status qw_marginals(qw_plan_t plan, const void* psi, const int64_t* origin, double* out,
                       int64_t out_len, int64_t* xmin, int64_t* len, void* stream);

/* psi_t = U^t psi0 (as qw_evolve_fft) and the reductions of psi_t about
 * origin (as qw_observables with ref = NULL; overlap fields zero), in one
 * pass less: where the Fourier schedule ends with a strided inverse pass
 * (d = 2, 3 and the 1D four-step) the reductions are taken inside it, so
 * psi_t is not read back. psi_t: DEVICE field, may equal psi0, or NULL when
 * only the reductions are wanted (psi_t is then not written; the plan's
 * scratch field holds the intermediate passes). origin: dim HOST doubles;
 * out: HOST. Waits for the result. */
qw_status qw_evolve_fft_observables(qw_plan_t plan, const void* psi0, void* psi_t, int64_t t,
                                    const double* origin, qw_obs* out, void* stream);

/* Doubles of the raw reduction record of qw_evolve_fft_observables_async. */
#define QW_OBS_RAW_DOUBLES 13

/* qw_evolve_fft_observables without the wait (the same jump and Sec. 5.2
 * reductions, queued on `stream`): a copy on the stream leaves the record of
 * the sums in raw[0..QW_OBS_RAW_DOUBLES) once the pass is done, and the call
 * returns as soon as the work is queued. raw: HOST memory, pinned
 * (hipHostMalloc; with pageable memory the copy, and so the call, waits).
 * Once the stream has passed the call (hipStreamSynchronize, or an event
 * recorded after it), qw_obs_from_raw turns the record into the qw_obs that
 * qw_evolve_fft_observables returns, bit for bit. For loops that keep the
 * GPU busy while the host reads an earlier result. The plan's reduction
 * buffers are reused by every such call: calls on one plan must be issued on
 * one stream (on different streams they race). Errors as
 * qw_evolve_fft_observables; raw NULL is QW_ERR_INVALID. */
qw_status qw_evolve_fft_observables_async(qw_plan_t plan, const void* psi0, void* psi_t,
                                          int64_t t, const double* origin, double* raw,
                                          void* stream);

/* The qw_obs of a raw record written by qw_evolve_fft_observables_async
 * (raw: HOST, QW_OBS_RAW_DOUBLES doubles, complete), about the origin passed
 * to that call (dim HOST doubles). Host arithmetic only; no GPU work. */
qw_status qw_obs_from_raw(qw_plan_t plan, const double* raw, const double* origin, qw_obs* out);

/* The reductions of psi(t_i) = U^{t_i} psi0 about origin (as
 * qw_evolve_fft_observables) for n times t[0..n) (HOST int64, |t_i| <= 2^53,
 * any order), out[0..n) (HOST). The series of the position expectation of
 * Sec. 5.2 in one call: the spectrum of psi0 is computed once (Sec. 4: it
 * does not depend on t), and each time costs the per-wave-vector power
 * with the inverse transform, its reductions taken in the last pass, with
 * no wait between times (d = 2, 3 Dirac plans: three field passes per time
 * instead of five; Weyl plans and 1D lattices run a full jump per time).
 * psi0 is not modified; the plan's scratch grows to two fields. The results
 * agree with qw_evolve_fft_observables at each t to rounding (the forward
 * transform is taken by a separate pass). 1 <= n <= 2^20. Waits once, at
 * the end. */
qw_status qw_evolve_fft_series(qw_plan_t plan, const void* psi0, int64_t n, const int64_t* t,
                               const double* origin, qw_obs* out, void* stream);

/* Write a Gaussian particle/antiparticle state into psi (Sec. 5.1,
 * Definition 1; Sec. 5.2, superposition c+ psi+ + c- psi-):
 *   hat psi(q) = c+ a+(q)/|a+| + c- a-(q)/|a-|,
 *   a_s(q) = exp(-sigma^2 |dq|^2 / 2) e^{+i q.c} P_s(q) chi_s,
 * with dq_j = q_j - q'_j wrapped to [-pi, pi), q' = H^T k0 the lattice image
 * of the Cartesian k0, P_+ / P_- the projectors of D_q on its eigenvalues
 * e^{-i omega} / e^{+i omega} (I/2 where sin omega < 1e-12), chi_s the
 * normalised column of P_s(q') of largest norm (the lowest index whose norm
 * is within a relative 1e-12 of the largest: projector columns tie in pairs); then
 * psi = inverse DFT scaled to unit 2-norm.
 *   k0: dim HOST doubles (Cartesian); sigma > 0 in lattice cells;
 *   center: dim HOST doubles; c_plus, c_minus real, not both 0.
 * Waits for completion. */
qw_status qw_prepare_state(qw_plan_t plan, void* psi, const double* k0, double sigma,
                           const double* center, double c_plus, double c_minus, void* stream);

/* qw_evolve_fft with a HIP event recorded on `stream` around every kernel
 * pass; waits, then writes the duration of each pass (ms) to pass_ms and
 * their count to *npass (at most 8; 5 for d = 3). For measurement. */
qw_status qw_evolve_fft_timed(qw_plan_t plan, const void* psi0, void* psi_t, int64_t t,
                              void* stream, float* pass_ms, int* npass);

/* Measurement and tuning of the position-space step (process-wide; not
 * thread-safe against concurrent steps). two_step = 1 runs pairs of steps of
 * the 3D Dirac walk in complex64 (planes that hold one output tile) as one
 * launch that reads and writes the field once per pair (temporal blocking);
 * 0 (the default) runs every step as its own launch, which measured faster.
 * Both give the same bits. tile_shape: 0 = 16 x 32 output tiles, 1 = 8 x 64,
 * 2 = 16 x 16, 3 = 8 x 32;
 * chunk: planes of axis 0 per workgroup (0 = chosen from the lattice, else a
 * power of two in [2, 256]). */
qw_status qw_set_step_kernel(int two_step, int tile_shape, int chunk);

/* Measurement of the strided FFT passes (process-wide). staged = 1 (the
 * default): passes over at least 8192 tiles stage their loads through LDS
 * with the global-to-LDS loads of gfx950, double-buffered, eight tiles per
 * workgroup: complex64 inverse passes of length 256 (tiles of 32 columns; a
 * 256^3 field of 4 components), complex64 passes of length 512 of either
 * direction (tiles of 16 columns; a 512^3 field), complex128 passes of
 * length 256 and 512 of either direction whose rows lie at least 4096
 * elements apart (tiles of 16 and 8 columns; the n1 passes of 256^3 and
 * 512^3 fields); staged = 0:
 * every pass keeps its loads in registers. Both give the same bits (the
 * same tiles and arithmetic). */
qw_status qw_set_fft_kernel(int staged);

/* Schedule of the Fourier evolution. slab_planes = 0 runs the n2 and fused
 * n3 passes over the whole field; slab_planes = k runs the n2 forward, fused
 * n3 and n2 inverse passes on slabs of k planes of n1 in turn, so that a slab
 * stays in the last-level cache between those passes (ignored for d < 3).
 * contig_elems (4 or 8; 4 only for d = 2, 3) is the number of elements per
 * thread and contig_threads (64, 128, 256 or 512) the target workgroup size
 * of the fused contiguous pass; contig_groups (1..64; > 1 only used for
 * d = 3 with contig_elems = 4) lets each of its workgroups transform up to
 * that many pencil groups in turn, loading the next while computing the
 * current one. Every schedule computes the same result. */
qw_status qw_set_schedule(qw_plan_t plan, int slab_planes, int contig_elems, int contig_threads,
                          int contig_groups);
qw_status qw_get_schedule(qw_plan_t plan, int* slab_planes, int* contig_elems,
                          int* contig_threads, int* contig_groups);

/* Time the candidate schedules on the plan's scratch field and keep the
 * fastest; *best_ms (nullable) receives its time per evolution. Waits.
 * With the environment variable QW_TUNE_CACHE naming a text file, a schedule
 * found there for the same (device architecture, walk, d, N, precision) is
 * taken without timing (*best_ms = the time recorded with it; the last such
 * line wins, malformed lines are ignored), and a newly timed one is appended
 * as one line "qw-tune-v1 <arch> <dirac|weyl> d<d> <N1>x<N2>x<N3> <c64|c128>
 * <slab> <elems> <threads> <groups> <ms>". Processes that share the file may
 * append concurrently; each line is written by one fprintf. */
qw_status qw_autotune(qw_plan_t plan, void* stream, double* best_ms);

/* Dispersive approximation of Proposition 1 (Sec. 5.1): the particle /
 * antiparticle state of qw_prepare_state (same arguments) evolved to real t
 * with omega(k) replaced by its Taylor polynomial of the given order about
 * k0: each wave-vector of the + sector is multiplied by e^{-i t T(k - k0)},
 * of the - sector by e^{+i t T(k - k0)} (k - k0 from the wrapped lattice
 * difference, mapped to Cartesian k). order 0 (phase only), 1 (drift
 * vector) or 2 (drift and diffusion tensor, the second-order dispersive
 * equation); else QW_ERR_UNSUPPORTED. QW_ERR_INVALID if omega is not
 * differentiable at k0 (sin omega = 0, only for m = 0). Writes psi (DEVICE);
 * waits for the result. */
qw_status qw_evolve_dispersive(qw_plan_t plan, void* psi, const double* k0, double sigma,
                               const double* center, double c_plus, double c_minus, int order,
                               double t, void* stream);

/* Host only, no device needed: the Taylor coefficients of omega(k) =
 * arccos(n u(k)) at the Cartesian k0 (dim entries) that
 * qw_evolve_dispersive uses, coeffs[10] (HOST): omega(k0); d omega / dk_i
 * (i = x, y, z); (1/2) d^2 omega / dk_i^2; d^2 omega / dk_x dk_y,
 * dk_x dk_z, dk_y dk_z. Entries beyond dim and beyond order are zero. */
qw_status qw_dispersion_taylor(int dim, double m, const double* k0, int order, double* coeffs);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of Fourier evolutions of particle states.
 * A request describes one lattice (dim, N), the mass m, a Gaussian particle /
 * antiparticle state (as in qw_prepare_state: k0, sigma, center, c_plus,
 * c_minus), a time t and the precision. The server prepares the state,
 * evolves it to t (Sec. 4) and returns the reductions of psi(t) about
 * `center` (Sec. 5.2). Requests are admitted in arrival order while the
 * device memory they need (one field, two for the 1D four-step, plus their
 * parameters and partial sums) fits budget_bytes, grouped by (dim, N, dtype) into batches of at most max_batch
 * instances (each with its own m, state and t), and run on nstreams streams;
 * at most 2 * nstreams batches are on the device at once, and requests
 * that arrive meanwhile gather into the next batches, admitted as batches
 * finish and memory frees. A request's result does not depend on what it
 * was batched with.
 * ------------------------------------------------------------------------ */
typedef struct qw_server_s* qw_server_t;

typedef struct {
  int dim;           /* 1, 2, 3 */
  int64_t N[3];      /* dim entries used; powers of two as for qw_plan */
  double m;          /* 0 <= m <= 1 */
  qw_dtype dtype;
  double k0[3];      /* Cartesian central wave-vector (dim entries) */
  double sigma;      /* packet width in cells, > 0 */
  double center[3];  /* packet centre and origin of the reductions */
  double c_plus, c_minus;
  int64_t t;         /* any sign */
} qw_request;

typedef struct {
  int64_t ticket;
  qw_status status;
  int batch_size;          /* instances in the batch that served the request */
  double queue_s;          /* submit -> launch of its batch (host clock) */
  double latency_s;        /* submit -> completion signalled by the stream */
  qw_obs obs;              /* reductions of psi(t) about center (no overlap) */
  double sector_norm2[2];  /* squared norms of the two sector amplitudes before normalisation */
} qw_result;

/* used_bytes: the footprints charged against the budget by the requests on
 * the device (a request's footprint is the device layout of a batch holding
 * it alone: field, transpose buffer, parameters, partial sums, results);
 * laid_out_bytes: the device layouts of the batches on the device, never
 * more than used_bytes. peak_*: the largest value so far. */
typedef struct {
  int64_t submitted, completed, batches, queued;
  int64_t inflight_batches, max_inflight_batches;
  int64_t used_bytes, peak_used_bytes;
  int64_t laid_out_bytes, peak_laid_out_bytes;
  int64_t graphs_captured;  /* batch chains captured into graphs */
  int64_t graph_launches;   /* batches run by replaying a captured graph */
  int64_t slot_bytes;       /* device bytes held by the captured graphs' buffers */
  int64_t launch_host_ns;   /* host time the server spent enqueuing batches */
  int64_t budget_bytes;     /* the budget in force (after resolving 0) */
  int64_t cancelled;        /* requests cancelled while queued */
} qw_server_info;

/* Start a server on the current device. budget_bytes >= 1 MiB, or 0 for
 * the environment variable QW_HBM_BUDGET (bytes, optional K/M/G suffix) or,
 * without it, half of the device memory free at creation; max_batch in
 * [1, 4096], nstreams in [1, 16]. */
qw_status qw_server_create(qw_server_t* out, size_t budget_bytes, int max_batch, int nstreams);
/* Options, before the first submit. use_graphs (default 1): the chain of
 * copies and kernels of a batch is captured into a HIP graph once per
 * (shape, precision, batch size), against buffers kept with the graph, and
 * later batches of that shape and size replay it in one launch with their
 * own parameters (per-instance mass, state, time and centre live in device
 * memory the graph reads); the chain of a (shape, precision, batch size)
 * runs directly until it has been seen twice, and its second direct run
 * records the capture beside it. At most max_graphs graphs are kept (least
 * recently used dropped first; default 256), and their buffers at most the
 * budget; replays give bit for bit the results of the direct chain.
 * autotune (default 1): each shape's schedule is timed once, on a plan of
 * its own whose scratch is released afterwards. */
qw_status qw_server_configure(qw_server_t server, int use_graphs, int autotune, int max_graphs);
/* Queue a request; never blocks on the device. QW_ERR_NOMEM if the request
 * alone exceeds the budget; argument errors as for qw_plan / qw_prepare_state. */
qw_status qw_server_submit(qw_server_t server, const qw_request* req, int64_t* ticket);
/* *done = 1 and *out filled once the request has completed, else *done = 0.
 * A result is handed out once (by poll or wait); the ticket is then unknown
 * (QW_ERR_INVALID): of two callers waiting on one ticket, one gets the
 * result and the other QW_ERR_INVALID. */
qw_status qw_server_poll(qw_server_t server, int64_t ticket, qw_result* out, int* done);
/* Block until the request has completed. */
qw_status qw_server_wait(qw_server_t server, int64_t ticket, qw_result* out);
/* Cancel a request that is still queued (not yet in a batch): its result,
 * with status QW_ERR_CANCELLED, is then collected by poll or wait as usual.
 * *cancelled = 1 if it was cancelled, 0 if it is already on the device or
 * done (it then completes normally). QW_ERR_INVALID for an unknown ticket. */
qw_status qw_server_cancel(qw_server_t server, int64_t ticket, int* cancelled);
/* qw_server_wait for at most timeout_s seconds (>= 0; 1e9 or more waits
 * without limit): *done = 1 and *out filled if the request completed in
 * time, else *done = 0 and it stays pending. */
qw_status qw_server_wait_for(qw_server_t server, int64_t ticket, double timeout_s,
                             qw_result* out, int* done);
/* hold != 0: queue requests but launch none (batches already on the device
 * finish); hold = 0: resume, batching everything queued meanwhile. */
qw_status qw_server_hold(qw_server_t server, int hold);
qw_status qw_server_stats(qw_server_t server, qw_server_info* out);
/* Finish every queued and running request, then release everything. */
qw_status qw_server_destroy(qw_server_t server);

/* Message of the last failing call on this thread ("" if none). */
const char* qw_last_error(void);

/* Library version string. */
const char* qw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QW_H */
