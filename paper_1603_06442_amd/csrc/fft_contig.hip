// FFT pass along the contiguous lattice axis, fused with the per-wave-vector
// evolution of Sec. 4 of the paper.
//
// A team of L/E threads owns one pencil (all s spinor components of one row
// of the lattice), E elements per component per thread. MODE_EVOLVE does, in
// one read and one write of the field:
//   forward FFT along the axis (sign +, Sec. 4)  ->  per q: hat psi(q) <-
//   V^-1 [cos(omega t) I - i sin(omega t)/sin(omega) M_q] hat psi(q)  ->
//   inverse FFT along the axis (sign -).
// The forward transform leaves each thread holding the spectrum at the same
// positions the inverse starts from, so the apply needs no data exchange.
// MODE_FWD / MODE_INV do only the forward / inverse transform; MODE_APPLY_INV
// skips the forward transform (its input is already a spectrum).
//
// Per-q symbol (Sec. 3.1, 3.2): u, n~ of the Weyl walk at the Cartesian k of
// the lattice frequency q (3D: k = ((q1+q2)/2, (q1+q3)/2, -(q2+q3)/2); 2D:
// k = ((q1+q2)/2, (q1-q2)/2); 1D: k = q), cos(omega) = n u,
// sin(omega) = sqrt(n^2 |n~|^2 + m^2), omega = atan2(sin, cos) and
//   M_q = [[n sigma.n~, -m I], [-m I, -n sigma.n~]]   (d = 2, 3),
//   M_q = n sin(q) sigma_z - m sigma_x                 (d = 1),
// so that D_q = cos(omega) I - i M_q and M_q^2 = sin^2(omega) I. omega,
// omega t and its reduction modulo 2 pi are FP64 in both precisions; the
// sine and cosine of the reduced angle are FP32 for complex64 fields.
//
// 1D four-step (N = N1 * L): the strided pass has already transformed along
// n1 (rows k1); here each pencil is one row, pre-multiplied by
// e^{+2 pi i n2 k1 / N} before the forward transform and by the conjugate
// after the inverse. The spectrum sits at row k1, column k2 for q index
// k1 + N1 k2 (never transposed back: the inverse undoes the order).
#include <algorithm>

#include "qw_internal.h"

namespace qw {

// omega t reduced to [-pi, pi] in FP64: the product is split exactly into
// p + pl (FMA remainder), then 2 pi is removed in two parts (Cody-Waite:
// 2 pi = HI + LO with HI the double nearest 2 pi). For |k| < 2^20 the first
// FMA is exact, so the reduced angle keeps the accuracy of omega itself.
// t is any real (integer t are exact up to 2^53).
__device__ __forceinline__ double reduced_phase(double w, double tt) {
  const double p = w * tt;
  const double pl = fma(w, tt, -p);
  const double k = rint(p * 0.15915494309189533577);
  double r = fma(-k, 6.283185307179586232, p);
  r = fma(-k, 2.4492935982947063545e-16, r);
  return r + pl;
}

// omega(q) = atan2(sin(omega), cos(omega)) with cos(omega) = n u and
// sin(omega) = sqrt(n^2 |n~|^2 + m^2), in FP64.
__device__ __forceinline__ double omega_q(int dim, const PassGeom& g, double nn, double m,
                                          int64_t j1, int64_t j2, int64_t j3) {
  double u, n1, n2, n3;
  weyl_un(dim, g.cs, g.Nc, g.shift, j1, j2, j3, u, n1, n2, n3);
  const double sinw = sqrt(nn * nn * (n1 * n1 + n2 * n2 + n3 * n3) + m * m);
  return atan2(sinw, nn * u);
}

// hat psi(q) <- V^-1 [cos(omega t) I - i sin(omega t)/sin(omega) M_q] hat psi(q).
// With TAB, omega comes from the plan's table and everything except the
// phase reduction runs in the field precision.
template <typename T, int DIM, bool TAB>
__device__ __forceinline__ void apply_q(cx<T> (&y)[DIM == 1 ? 2 : 4], const PassGeom& g,
                                        const InstParam& ip, int64_t j1, int64_t j2, int64_t j3,
                                        int64_t qidx) {
  double u, n1, n2, n3;
  weyl_un(DIM, g.cs, g.Nc, g.shift, j1, j2, j3, u, n1, n2, n3);
  const double nn = ip.n, m = ip.m;
  double w;
  T tn1, tn2, tn3, sinw_t;
  if constexpr (TAB) {
    w = g.omega[qidx];
    tn1 = (T)n1;
    tn2 = (T)n2;
    tn3 = (T)n3;
    const T tnn = (T)nn, tm = (T)m;
    sinw_t = sqrt(tnn * tnn * (tn1 * tn1 + tn2 * tn2 + tn3 * tn3) + tm * tm);
  } else {
    const double sinw = sqrt(nn * nn * (n1 * n1 + n2 * n2 + n3 * n3) + m * m);
    w = atan2(sinw, nn * u);
    tn1 = (T)n1;
    tn2 = (T)n2;
    tn3 = (T)n3;
    const T tnn = (T)nn, tm = (T)m;
    sinw_t = sqrt(tnn * tnn * (tn1 * tn1 + tn2 * tn2 + tn3 * tn3) + tm * tm);
  }
  const double r = reduced_phase(w, ip.t);
  T C, S, isw;
  if constexpr (sizeof(T) == 4) {
    sincosf((float)r, &S, &C);
    isw = sinw_t > 1e-30f ? 1.0f / sinw_t : 0.0f;
  } else {
    sincos(r, &S, &C);
    isw = sinw_t > 0.0 ? 1.0 / sinw_t : 0.0;
  }
  const T sc = (T)g.inv_scale;
  const T c = C * sc;
  const T st = S * isw * sc;  // V^-1 sin(omega t) / sin(omega)
  const T tnn = (T)nn;
  if constexpr (DIM == 1) {
    const T a = tnn * tn3 * st;
    const T gg = (T)m * st;
    // z = St M psi
    const cx<T> z0 = mk(a * y[0].x - gg * y[1].x, a * y[0].y - gg * y[1].y);
    const cx<T> z1 = mk(-gg * y[0].x - a * y[1].x, -gg * y[0].y - a * y[1].y);
    // out = C psi - i z
    y[0] = mk(c * y[0].x + z0.y, c * y[0].y - z0.x);
    y[1] = mk(c * y[1].x + z1.y, c * y[1].y - z1.x);
  } else {
    const T a = tnn * tn3 * st;
    const T b = tnn * tn1 * st;
    const T e = tnn * tn2 * st;
    const T gg = (T)m * st;
    const cx<T> p0 = y[0], p1 = y[1], p2 = y[2], p3 = y[3];
    // (b - i e) p = (b p.x + e p.y, b p.y - e p.x); (b + i e) p = (b p.x - e p.y, b p.y + e p.x)
    const cx<T> z0 = mk(a * p0.x + (b * p1.x + e * p1.y) - gg * p2.x,
                        a * p0.y + (b * p1.y - e * p1.x) - gg * p2.y);
    const cx<T> z1 = mk((b * p0.x - e * p0.y) - a * p1.x - gg * p3.x,
                        (b * p0.y + e * p0.x) - a * p1.y - gg * p3.y);
    const cx<T> z2 = mk(-gg * p0.x - a * p2.x - (b * p3.x + e * p3.y),
                        -gg * p0.y - a * p2.y - (b * p3.y - e * p3.x));
    const cx<T> z3 = mk(-gg * p1.x - (b * p2.x - e * p2.y) + a * p3.x,
                        -gg * p1.y - (b * p2.y + e * p2.x) + a * p3.y);
    y[0] = mk(c * p0.x + z0.y, c * p0.y - z0.x);
    y[1] = mk(c * p1.x + z1.y, c * p1.y - z1.x);
    y[2] = mk(c * p2.x + z2.y, c * p2.y - z2.x);
    y[3] = mk(c * p3.x + z3.y, c * p3.y - z3.x);
  }
}


// hat psi(q) <- V^-1 P_s hat psi(q), P_s = (I + s M_q / sin(omega)) / 2: the
// spectral projector on the sector of eigenvalue e^{-s i omega} (Sec. 3.2),
// I/2 where sin(omega) < 1e-12 (as in the state preparation).
template <typename T, int DIM>
__device__ __forceinline__ void apply_proj(cx<T> (&y)[DIM == 1 ? 2 : 4], const PassGeom& g,
                                           double sgn, int64_t j1, int64_t j2, int64_t j3) {
  double u, n1, n2, n3;
  weyl_un(DIM, g.cs, g.Nc, g.shift, j1, j2, j3, u, n1, n2, n3);
  (void)u;
  const double nn = g.single.n, m = g.single.m;
  const double sinw = sqrt(nn * nn * (n1 * n1 + n2 * n2 + n3 * n3) + m * m);
  const double isw = sinw >= 1e-12 ? 1.0 / sinw : 0.0;
  const T h = (T)(0.5 * g.inv_scale);
  const double kk = sgn * 0.5 * g.inv_scale * isw;
  const T a = (T)(nn * n3 * kk), gg = (T)(m * kk);
  if constexpr (DIM == 1) {
    const cx<T> p0 = y[0], p1 = y[1];
    y[0] = mk(h * p0.x + a * p0.x - gg * p1.x, h * p0.y + a * p0.y - gg * p1.y);
    y[1] = mk(h * p1.x - gg * p0.x - a * p1.x, h * p1.y - gg * p0.y - a * p1.y);
  } else {
    const T b = (T)(nn * n1 * kk), e = (T)(nn * n2 * kk);
    const cx<T> p0 = y[0], p1 = y[1], p2 = y[2], p3 = y[3];
    // z = k M p with M = [[n sigma.n~, -m I], [-m I, -n sigma.n~]]
    const cx<T> z0 = mk(a * p0.x + (b * p1.x + e * p1.y) - gg * p2.x,
                        a * p0.y + (b * p1.y - e * p1.x) - gg * p2.y);
    const cx<T> z1 = mk((b * p0.x - e * p0.y) - a * p1.x - gg * p3.x,
                        (b * p0.y + e * p0.x) - a * p1.y - gg * p3.y);
    const cx<T> z2 = mk(-gg * p0.x - a * p2.x - (b * p3.x + e * p3.y),
                        -gg * p0.y - a * p2.y - (b * p3.y - e * p3.x));
    const cx<T> z3 = mk(-gg * p1.x - (b * p2.x - e * p2.y) + a * p3.x,
                        -gg * p1.y - (b * p2.y + e * p2.x) + a * p3.y);
    y[0] = mk(h * p0.x + z0.x, h * p0.y + z0.y);
    y[1] = mk(h * p1.x + z1.x, h * p1.y + z1.y);
    y[2] = mk(h * p2.x + z2.x, h * p2.y + z2.y);
    y[3] = mk(h * p3.x + z3.x, h * p3.y + z3.y);
  }
}

// Two-component Weyl walk (Sec. 3.1): W_q = u I - i sigma.n~ with
// cos(omega) = u, sin(omega) = |n~|, so
//   W_q^t = cos(omega t) I - i sin(omega t)/sin(omega) sigma.n~,
// the Dirac closed form with n = 1, m = 0 restricted to its upper block.
// omega and its phase reduction are FP64; the rest in the field precision.
// With TAB, omega comes from the plan's table (the Dirac table at n = 1,
// m = 0 is the Weyl omega).
template <typename T, int DIM, bool TAB>
__device__ __forceinline__ void apply_weyl(cx<T> (&y)[2], const PassGeom& g, const InstParam& ip,
                                           int64_t j1, int64_t j2, int64_t j3, int64_t qidx) {
  double u, n1, n2, n3;
  weyl_un(DIM, g.cs, g.Nc, g.shift, j1, j2, j3, u, n1, n2, n3);
  const double sinw = sqrt(n1 * n1 + n2 * n2 + n3 * n3);
  const double r = reduced_phase(TAB ? g.omega[qidx] : atan2(sinw, u), ip.t);
  T C, S, isw;
  if constexpr (sizeof(T) == 4) {
    sincosf((float)r, &S, &C);
    const float swf = (float)sinw;
    isw = swf > 1e-30f ? 1.0f / swf : 0.0f;
  } else {
    sincos(r, &S, &C);
    isw = sinw > 0.0 ? 1.0 / sinw : 0.0;
  }
  const T sc = (T)g.inv_scale;
  const T c = C * sc;
  const T st = S * isw * sc;
  const T a = (T)n3 * st, b = (T)n1 * st, e = (T)n2 * st;
  const cx<T> p0 = y[0], p1 = y[1];
  // z = st sigma.n~ p; out = c p - i z
  const cx<T> z0 = mk(a * p0.x + (b * p1.x + e * p1.y), a * p0.y + (b * p1.y - e * p1.x));
  const cx<T> z1 = mk((b * p0.x - e * p0.y) - a * p1.x, (b * p0.y + e * p0.x) - a * p1.y);
  y[0] = mk(c * p0.x + z0.y, c * p0.y - z0.x);
  y[1] = mk(c * p1.x + z1.y, c * p1.y - z1.x);
}

// p <- c p - i Z p for one 4-spinor with Z = [[A, -g I], [-g I, -A]] and
// A = a sigma_z + b sigma_x + e sigma_y (the D^t of Sec. 3.2 with
// c = cos(omega t), (a, b, e) = n n~ sin(omega t)/sin(omega), g = m
// sin(omega t)/sin(omega), all already scaled).
template <typename T>
__device__ __forceinline__ void dirac_mix4(cx<T> (&p)[4], T c, T a, T b, T e, T gg) {
  const cx<T> p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3];
  const cx<T> z0 = mk(a * p0.x + (b * p1.x + e * p1.y) - gg * p2.x,
                      a * p0.y + (b * p1.y - e * p1.x) - gg * p2.y);
  const cx<T> z1 = mk((b * p0.x - e * p0.y) - a * p1.x - gg * p3.x,
                      (b * p0.y + e * p0.x) - a * p1.y - gg * p3.y);
  const cx<T> z2 = mk(-gg * p0.x - a * p2.x - (b * p3.x + e * p3.y),
                      -gg * p0.y - a * p2.y - (b * p3.y - e * p3.x));
  const cx<T> z3 = mk(-gg * p1.x - (b * p2.x - e * p2.y) + a * p3.x,
                      -gg * p1.y - (b * p2.y + e * p2.x) + a * p3.y);
  p[0] = mk(c * p0.x + z0.y, c * p0.y - z0.x);
  p[1] = mk(c * p1.x + z1.y, c * p1.y - z1.x);
  p[2] = mk(c * p2.x + z2.y, c * p2.y - z2.x);
  p[3] = mk(c * p3.x + z3.y, c * p3.y - z3.x);
}

// Cubic-supercell BCC (Sec. 4, eq:bcc-dft / eq:bcc-idft) at the sublattice
// frequency indices (j1, j2, j3). After the forward transforms (sign +,
// unshifted) y[0..4) = F0(k), y[4..8) = F1(k), the rectangular spectra of the
// even and odd sublattice, and with a_k = e^{i pi sum_i j_i / N_i}
//   h1 = F0 + a_k F1   is the BCC spectrum at the Cartesian kappa = pi j / N,
//   h0 = F0 - a_k F1   the one at kappa + pi e_x.
// MODE_BCC applies D^t at kappa to h1 and at kappa + pi e_x to h0 and
// recombines G0 = h0 + h1, G1 = conj(a_k) (h1 - h0) for the inverse
// transforms; the two factors 1/sqrt(2) and the 1/V of the transform pair
// are one factor g.inv_scale = 1/(2V). At kappa + pi e_x the Weyl u and n~
// change sign and the mass term does not. MODE_BCC_FWD stores (h0, h1) and
// MODE_BCC_INV recombines a stored (hat f0, hat f1); both scale by
// g.inv_scale = 1/sqrt(2V). The trig values come from the plan's FP64
// (cos, sin)(pi j / Nc) table: pi j_i / N_i is entry j_i << shift_i.
template <typename T, int MODE>
__device__ __forceinline__ void apply_bcc(cx<T> (&y)[8], const PassGeom& g, int64_t j1,
                                          int64_t j2, int64_t j3, int64_t qidx) {
  const int64_t mask = 2 * (int64_t)g.Nc - 1;
  const int64_t a1 = (j1 << g.shift[0]) & mask;
  const int64_t a2 = (j2 << g.shift[1]) & mask;
  const int64_t a3 = (j3 << g.shift[2]) & mask;
  const int64_t ia = (a1 + a2 + a3) & mask;
  const T ar = (T)g.cs[2 * ia], ai = (T)g.cs[2 * ia + 1];
  const T sc = (T)g.inv_scale;
  if constexpr (MODE == MODE_BCC_INV) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cx<T> h0 = y[c], h1 = y[4 + c];
      const T dx = h1.x - h0.x, dy = h1.y - h0.y;
      y[c] = mk((h0.x + h1.x) * sc, (h0.y + h1.y) * sc);
      y[4 + c] = mk((ar * dx + ai * dy) * sc, (ar * dy - ai * dx) * sc);  // conj(a) d
    }
    return;
  }
  if constexpr (MODE == MODE_BCC_FWD) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cx<T> f1 = y[4 + c];
      const T px = ar * f1.x - ai * f1.y, py = ar * f1.y + ai * f1.x;  // a f1
      const cx<T> f0 = y[c];
      y[c] = mk((f0.x - px) * sc, (f0.y - py) * sc);      // h0
      y[4 + c] = mk((f0.x + px) * sc, (f0.y + py) * sc);  // h1
    }
    return;
  } else if constexpr (MODE == MODE_BCC_TAB) {
    // omega(kappa) from the plan's table, the phase reductions FP64; n~ and
    // sin(omega) in the field precision from the trig table of that
    // precision (they only scale the result).
    T cxf, sxf, cyf, syf, czf, szf;
    if constexpr (sizeof(T) == 4) {
      cxf = g.csf[2 * a1]; sxf = g.csf[2 * a1 + 1];
      cyf = g.csf[2 * a2]; syf = g.csf[2 * a2 + 1];
      czf = g.csf[2 * a3]; szf = g.csf[2 * a3 + 1];
    } else {
      cxf = g.cs[2 * a1]; sxf = g.cs[2 * a1 + 1];
      cyf = g.cs[2 * a2]; syf = g.cs[2 * a2 + 1];
      czf = g.cs[2 * a3]; szf = g.cs[2 * a3 + 1];
    }
    const T n1 = sxf * cyf * czf - cxf * syf * szf;
    const T n2 = cxf * syf * czf + sxf * cyf * szf;
    const T n3 = cxf * cyf * szf - sxf * syf * czf;
    const T tn = (T)g.single.n, tm = (T)g.single.m;
    const T s2 = tn * tn * (n1 * n1 + n2 * n2 + n3 * n3) + tm * tm;
    const double wA = g.omega[qidx];
    const double wB = (3.141592653589793116 - wA) + 1.2246467991473532e-16;
    T CA, SA, CB, SB, isw;
    if constexpr (sizeof(T) == 4) {
      sincosf((float)reduced_phase(wA, g.single.t), &SA, &CA);
      sincosf((float)reduced_phase(wB, g.single.t), &SB, &CB);
      const float sinw = sqrtf(s2);
      isw = sinw > 1e-30f ? 1.0f / sinw : 0.0f;
    } else {
      sincos(reduced_phase(wA, g.single.t), &SA, &CA);
      sincos(reduced_phase(wB, g.single.t), &SB, &CB);
      const double sinw = sqrt(s2);
      isw = sinw > 0.0 ? 1.0 / sinw : 0.0;
    }
    const T a = tn * n3, b = tn * n1, e = tn * n2;
    const T stA = SA * isw * sc, stB = SB * isw * sc;
    cx<T> h0[4], h1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cx<T> f1 = y[4 + c];
      const T px = ar * f1.x - ai * f1.y, py = ar * f1.y + ai * f1.x;  // a f1
      h1[c] = mk(y[c].x + px, y[c].y + py);
      h0[c] = mk(y[c].x - px, y[c].y - py);
    }
    dirac_mix4<T>(h1, (T)CA * sc, a * stA, b * stA, e * stA, (T)tm * stA);
    dirac_mix4<T>(h0, (T)CB * sc, -a * stB, -b * stB, -e * stB, (T)tm * stB);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const T dx = h1[c].x - h0[c].x, dy = h1[c].y - h0[c].y;
      y[c] = mk(h0[c].x + h1[c].x, h0[c].y + h1[c].y);
      y[4 + c] = mk(ar * dx + ai * dy, ar * dy - ai * dx);  // conj(a) (h1 - h0)
    }
  } else {
    // The scalar coefficients first (FP64 omega and phase reduction), so the
    // spinor values are combined only once they are needed.
    const double cxd = g.cs[2 * a1], sxd = g.cs[2 * a1 + 1];
    const double cyd = g.cs[2 * a2], syd = g.cs[2 * a2 + 1];
    const double czd = g.cs[2 * a3], szd = g.cs[2 * a3 + 1];
    const double u = cxd * cyd * czd + sxd * syd * szd;
    const double n1 = sxd * cyd * czd - cxd * syd * szd;
    const double n2 = cxd * syd * czd + sxd * cyd * szd;
    const double n3 = cxd * cyd * szd - sxd * syd * czd;
    const double nn = g.single.n, m = g.single.m;
    const double sinw = sqrt(nn * nn * (n1 * n1 + n2 * n2 + n3 * n3) + m * m);
    const double wA = atan2(sinw, nn * u);
    // omega at kappa + pi e_x: atan2(sin, -cos) = pi - omega, with pi in two
    // parts (the double nearest pi and its remainder).
    const double wB = (3.141592653589793116 - wA) + 1.2246467991473532e-16;
    const double rA = reduced_phase(wA, g.single.t);
    const double rB = reduced_phase(wB, g.single.t);
    T CA, SA, CB, SB, isw;
    if constexpr (sizeof(T) == 4) {
      sincosf((float)rA, &SA, &CA);
      sincosf((float)rB, &SB, &CB);
      const float swf = (float)sinw;
      isw = swf > 1e-30f ? 1.0f / swf : 0.0f;
    } else {
      sincos(rA, &SA, &CA);
      sincos(rB, &SB, &CB);
      isw = sinw > 0.0 ? 1.0 / sinw : 0.0;
    }
    const T tn = (T)nn, tm = (T)m;
    const T a = tn * (T)n3, b = tn * (T)n1, e = tn * (T)n2;
    const T stA = SA * isw * sc, stB = SB * isw * sc;
    cx<T> h0[4], h1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const cx<T> f1 = y[4 + c];
      const T px = ar * f1.x - ai * f1.y, py = ar * f1.y + ai * f1.x;  // a f1
      h1[c] = mk(y[c].x + px, y[c].y + py);
      h0[c] = mk(y[c].x - px, y[c].y - py);
    }
    dirac_mix4<T>(h1, CA * sc, a * stA, b * stA, e * stA, tm * stA);
    dirac_mix4<T>(h0, CB * sc, -a * stB, -b * stB, -e * stB, tm * stB);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const T dx = h1[c].x - h0[c].x, dy = h1[c].y - h0[c].y;
      y[c] = mk(h0[c].x + h1[c].x, h0[c].y + h1[c].y);
      y[4 + c] = mk(ar * dx + ai * dy, ar * dy - ai * dx);  // conj(a) (h1 - h0)
    }
  }
}

// complex64 with the plan's omega table: omega and the phase reduction stay
// FP64; n~, sin(omega) and M_q are FP32 (they only scale the result), read
// from the FP32 (cos, sin)(pi j / Nc) table; the sine and cosine of the
// reduced angle use the hardware FP32 units.
struct PencilTrig {  // cos/sin of the pencil's fixed Cartesian component(s)
  float c, s;
  int a1, a2;
};

template <int DIM>
__device__ __forceinline__ PencilTrig pencil_trig(const PassGeom& g, int64_t pen) {
  PencilTrig pt;
  pt.c = 1.0f;
  pt.s = 0.0f;
  pt.a1 = pt.a2 = 0;
  if constexpr (DIM == 3) {
    const int j1 = (int)(pen >> g.lgN1), j2 = (int)(pen & (g.N[1] - 1));
    pt.a1 = j1 << g.shift[0];
    pt.a2 = j2 << g.shift[1];
    const int jx = (pt.a1 + pt.a2) & (2 * g.Nc - 1);  // k_x = (q1 + q2) / 2
    pt.c = g.csf[2 * jx];
    pt.s = g.csf[2 * jx + 1];
  } else if constexpr (DIM == 2) {
    pt.a1 = (int)pen << g.shift[0];
  }
  return pt;
}

template <int DIM>
__device__ __forceinline__ void apply_q_f32(cx<float> (&y)[DIM == 1 ? 2 : 4], const PassGeom& g,
                                            const InstParam& ip, const PencilTrig& pt, int64_t pen,
                                            int z, int64_t qidx) {
  const int twoNc1 = 2 * g.Nc - 1;
  float n1, n2, n3;
  if constexpr (DIM == 3) {
    const int a3 = z << g.shift[2];
    const int jy = (pt.a1 + a3) & twoNc1;  // k_y = (q1 + q3) / 2
    const int jz = (pt.a2 + a3) & twoNc1;  // k_z = -(q2 + q3) / 2
    const float2 ty = *reinterpret_cast<const float2*>(g.csf + 2 * jy);
    const float2 tz = *reinterpret_cast<const float2*>(g.csf + 2 * jz);
    const float cx_ = pt.c, sx = pt.s, cy = ty.x, sy = ty.y, cz = tz.x, sz = -tz.y;
    const float cycz = cy * cz, sysz = sy * sz, sycz = sy * cz, cysz = cy * sz;
    n1 = sx * cycz - cx_ * sysz;
    n2 = cx_ * sycz + sx * cysz;
    n3 = cx_ * cysz - sx * sycz;
  } else if constexpr (DIM == 2) {
    const int a2 = z << g.shift[1];
    const int jx = (pt.a1 + a2) & twoNc1, jy = (pt.a1 - a2 + 2 * g.Nc) & twoNc1;
    const float2 tx = *reinterpret_cast<const float2*>(g.csf + 2 * jx);
    const float2 ty = *reinterpret_cast<const float2*>(g.csf + 2 * jy);
    n1 = tx.y * ty.x;
    n2 = tx.x * ty.y;
    n3 = tx.y * ty.y;
  } else {
    const int64_t j1 = g.fourstep ? pen + g.N1 * z : z;
    const int jj = (int)((2 * (j1 << g.shift[0])) & twoNc1);
    n1 = 0.0f;
    n2 = 0.0f;
    n3 = g.csf[2 * jj + 1];
  }
  const float nn = (float)ip.n, m = (float)ip.m;
  const float sinw2 = nn * nn * (n1 * n1 + n2 * n2 + n3 * n3) + m * m;
  const float r = (float)reduced_phase(g.omega[qidx], ip.t);
  float S, C;
  __sincosf(r, &S, &C);
  const float sc = (float)g.inv_scale;
  const float c = C * sc;
  // V^-1 sin(omega t) / sin(omega), with the hardware reciprocal square root
  const float st = sinw2 > 1e-30f ? S * sc * __frsqrt_rn(sinw2) : 0.0f;
  if constexpr (DIM == 1) {
    const float a = nn * n3 * st, gg = m * st;
    const cx<float> z0 = mk(a * y[0].x - gg * y[1].x, a * y[0].y - gg * y[1].y);
    const cx<float> z1 = mk(-gg * y[0].x - a * y[1].x, -gg * y[0].y - a * y[1].y);
    y[0] = mk(c * y[0].x + z0.y, c * y[0].y - z0.x);
    y[1] = mk(c * y[1].x + z1.y, c * y[1].y - z1.x);
  } else {
    const float a = nn * n3 * st, b = nn * n1 * st, e = nn * n2 * st, gg = m * st;
    const cx<float> p0 = y[0], p1 = y[1], p2 = y[2], p3 = y[3];
    const cx<float> z0 = mk(a * p0.x + (b * p1.x + e * p1.y) - gg * p2.x,
                            a * p0.y + (b * p1.y - e * p1.x) - gg * p2.y);
    const cx<float> z1 = mk((b * p0.x - e * p0.y) - a * p1.x - gg * p3.x,
                            (b * p0.y + e * p0.x) - a * p1.y - gg * p3.y);
    const cx<float> z2 = mk(-gg * p0.x - a * p2.x - (b * p3.x + e * p3.y),
                            -gg * p0.y - a * p2.y - (b * p3.y - e * p3.x));
    const cx<float> z3 = mk(-gg * p1.x - (b * p2.x - e * p2.y) + a * p3.x,
                            -gg * p1.y - (b * p2.y + e * p2.x) + a * p3.y);
    y[0] = mk(c * p0.x + z0.y, c * p0.y - z0.x);
    y[1] = mk(c * p1.x + z1.y, c * p1.y - z1.x);
    y[2] = mk(c * p2.x + z2.y, c * p2.y - z2.x);
    y[3] = mk(c * p3.x + z3.y, c * p3.y - z3.x);
  }
}


// Pencil groups: group r holds the P pencils r*P .. r*P+P-1 of the launch.
// A workgroup walks the groups blockIdx.x, blockIdx.x + gridDim.x, ... and
// issues the global loads of its next group before transforming the current
// one, so that memory traffic of one group overlaps the arithmetic of the
// previous one.
template <typename T, int S, int E, int L>
__device__ __forceinline__ void load_group(cx<T> (&dst)[S][E], const cx<T>* __restrict__ in,
                                           const PassGeom& g, int64_t grp, int P, int p, int t) {
  constexpr int TT = L / E;
  const int64_t gp = grp * P + p;
  const bool valid = gp < g.pencils;
  const int64_t gpc = valid ? gp : 0;
  const int64_t b = g.lg_ppi >= 0 ? gpc >> g.lg_ppi : gpc / g.ppi;
  const int64_t pen = g.pen0 + (gpc - b * g.ppi);
  const int64_t base = b * S * g.V + pen * L;
  // Lanes past the last pencil read pencil 0 (in bounds) and never store:
  // unconditional loads keep the whole group's loads in flight together.
  (void)valid;
#pragma unroll
  for (int c = 0; c < S; ++c)
#pragma unroll
    for (int e = 0; e < E; ++e) dst[c][e] = in[base + c * g.V + t + TT * e];
}

template <typename T, int L, int E, int DIM, int MODE, bool PIPE>
__global__ __launch_bounds__(512) void k_fft_contig(cx<T>* __restrict__ out,
                                                    const cx<T>* __restrict__ in, PassGeom g,
                                                    const cx<T>* __restrict__ tw) {
  constexpr int S = contig_components(DIM, MODE);
  constexpr int TT = L / E;
  // omega(q) from the plan's table, one instance (the time in g.single)
  constexpr bool kTabApply = MODE == MODE_EVOLVE_TAB || MODE == MODE_APPLY_INV_TAB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int t = tid & (TT - 1);
  const int p = tid / TT;
  const int P = blockDim.x / TT;
  constexpr int LP = L;                 // component stride (swizzled slots)
  cx<T>* my = lds + p * (S * L + TT);  // team region (see fft_team_multi)
  const int64_t ngroups = (g.pencils + P - 1) / P;
  const cx<T>* tw4 = (const cx<T>*)g.tw4;
  const int64_t N = g.N[0];

  // complex64 transforms of four elements per thread (at most 16 twiddles
  // per thread) keep their twiddles in registers for every pencil group and
  // both directions.
  constexpr int TWC = team_twiddle_count<L, E>();
  constexpr bool kTwCache = sizeof(T) == 4 && E == 4 && TWC > 0 && TWC <= 16;
  cx<T> twc[kTwCache ? TWC : 1];
  if constexpr (kTwCache) load_team_twiddles<T, L, E>(twc, t, tw);

  // With PIPE the next group's loads are issued into nx before the current
  // group is transformed; without it each workgroup loads its group straight
  // into v (nx would otherwise stay live through the whole transform).
  cx<T> nx[S][E];
  int64_t grp = blockIdx.x;
  if constexpr (PIPE) {
    if (grp < ngroups) load_group<T, S, E, L>(nx, in, g, grp, P, p, t);
  }
  for (; grp < ngroups; grp += gridDim.x) {
    cx<T> v[S][E];
    if constexpr (PIPE) {
#pragma unroll
      for (int c = 0; c < S; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) v[c][e] = nx[c][e];
      if (grp + gridDim.x < ngroups) load_group<T, S, E, L>(nx, in, g, grp + gridDim.x, P, p, t);
    } else {
      load_group<T, S, E, L>(v, in, g, grp, P, p, t);
    }

    const int64_t gp = grp * P + p;
    const bool valid = gp < g.pencils;
    const int64_t gpc = valid ? gp : 0;
    const int64_t b = g.lg_ppi >= 0 ? gpc >> g.lg_ppi : gpc / g.ppi;
    const int64_t pen = g.pen0 + (gpc - b * g.ppi);
    const int64_t base = b * S * g.V + pen * L;

    if constexpr (MODE != MODE_INV && MODE != MODE_APPLY_INV && MODE != MODE_APPLY_INV_TAB &&
                  MODE != MODE_PROJ_INV && MODE != MODE_BCC_INV) {
      if (DIM == 1 && g.fourstep) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const cx<T> w = tw4[((int64_t)(t + TT * e) * pen) & (N - 1)];
#pragma unroll
          for (int c = 0; c < S; ++c) v[c][e] = cmulc(v[c][e], w);  // times e^{+2 pi i n2 k1 / N}
        }
      }
      if constexpr (kTwCache)
        fft_team_multi_c<T, L, E, 1, S>(v, my, LP, t, twc);
      else
        fft_team_multi<T, L, E, 1, S>(v, my, LP, t, tw);
    }
    if constexpr (MODE == MODE_WEYL || MODE == MODE_WEYL_TAB) {
      const InstParam ip = g.single;
#pragma unroll 1
      for (int e = 0; e < E; ++e) {
        const int64_t z = t + TT * e;
        int64_t j1, j2, j3;
        q_index<DIM>(g, pen, z, j1, j2, j3);
        cx<T> y[S];
#pragma unroll
        for (int c = 0; c < S; ++c) y[c] = v[c][0];
        apply_weyl<T, DIM, MODE == MODE_WEYL_TAB>(y, g, ip, j1, j2, j3, pen * L + z);
#pragma unroll
        for (int c = 0; c < S; ++c) {
#pragma unroll
          for (int k = 0; k + 1 < E; ++k) v[c][k] = v[c][k + 1];
          v[c][E - 1] = y[c];
        }
      }
    } else if constexpr (is_bcc_mode(MODE)) {
      // One wave-vector per iteration with the register rotation below.
#pragma unroll 1
      for (int e = 0; e < E; ++e) {
        const int64_t z = t + TT * e;
        int64_t j1, j2, j3;
        q_index<3>(g, pen, z, j1, j2, j3);
        cx<T> y[S];
#pragma unroll
        for (int c = 0; c < S; ++c) y[c] = v[c][0];
        apply_bcc<T, MODE>(y, g, j1, j2, j3, pen * L + z);
#pragma unroll
        for (int c = 0; c < S; ++c) {
#pragma unroll
          for (int k = 0; k + 1 < E; ++k) v[c][k] = v[c][k + 1];
          v[c][E - 1] = y[c];
        }
      }
    } else if constexpr (kTabApply && sizeof(T) == 4 && E <= 4) {
      // Four wave-vectors per thread: unrolled (independent chains, no
      // register rotation).
      const InstParam ip = g.single;
      const PencilTrig pt = pencil_trig<DIM>(g, pen);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int z = t + TT * e;
        cx<T> y[S];
#pragma unroll
        for (int c = 0; c < S; ++c) y[c] = v[c][e];
        apply_q_f32<DIM>(y, g, ip, pt, pen, z, pen * L + z);
#pragma unroll
        for (int c = 0; c < S; ++c) v[c][e] = y[c];
      }
    } else if constexpr (kTabApply && sizeof(T) == 4) {
      const InstParam ip = g.single;
      const PencilTrig pt = pencil_trig<DIM>(g, pen);
#pragma unroll 1
      for (int e = 0; e < E; ++e) {
        const int z = t + TT * e;
        cx<T> y[S];
#pragma unroll
        for (int c = 0; c < S; ++c) y[c] = v[c][0];
        apply_q_f32<DIM>(y, g, ip, pt, pen, z, pen * L + z);
#pragma unroll
        for (int c = 0; c < S; ++c) {
#pragma unroll
          for (int k = 0; k + 1 < E; ++k) v[c][k] = v[c][k + 1];
          v[c][E - 1] = y[c];
        }
      }
    } else if constexpr (MODE == MODE_PROJ_INV) {
      const double sgn = (b & 1) ? -1.0 : 1.0;
#pragma unroll 1
      for (int e = 0; e < E; ++e) {
        const int64_t z = t + TT * e;
        int64_t j1, j2, j3;
        q_index<DIM>(g, pen, z, j1, j2, j3);
        cx<T> y[S];
#pragma unroll
        for (int c = 0; c < S; ++c) y[c] = v[c][0];
        apply_proj<T, DIM>(y, g, sgn, j1, j2, j3);
#pragma unroll
        for (int c = 0; c < S; ++c) {
#pragma unroll
          for (int k = 0; k + 1 < E; ++k) v[c][k] = v[c][k + 1];
          v[c][E - 1] = y[c];
        }
      }
    } else if constexpr (MODE == MODE_EVOLVE || MODE == MODE_APPLY_INV || kTabApply) {
      const InstParam ip = g.inst ? g.inst[b] : g.single;
      // One wave-vector per iteration, deliberately not unrolled (an unrolled
      // loop lets the compiler hoist every element's table reads and keep
      // them live across the transforms). The register array is rotated by
      // one position per iteration so the body only uses static indices;
      // after E iterations every element is back in place.
#pragma unroll 1
      for (int e = 0; e < E; ++e) {
        const int64_t z = t + TT * e;
        int64_t j1, j2, j3;
        q_index<DIM>(g, pen, z, j1, j2, j3);
        cx<T> y[S];
#pragma unroll
        for (int c = 0; c < S; ++c) y[c] = v[c][0];
        apply_q<T, DIM, kTabApply>(y, g, ip, j1, j2, j3, pen * L + z);
#pragma unroll
        for (int c = 0; c < S; ++c) {
#pragma unroll
          for (int k = 0; k + 1 < E; ++k) v[c][k] = v[c][k + 1];
          v[c][E - 1] = y[c];
        }
      }
    }
    if constexpr (MODE != MODE_FWD && MODE != MODE_BCC_FWD) {
      if constexpr (kTwCache)
        fft_team_multi_c<T, L, E, -1, S>(v, my, LP, t, twc);
      else
        fft_team_multi<T, L, E, -1, S>(v, my, LP, t, tw);
      if (DIM == 1 && g.fourstep) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const cx<T> w = tw4[((int64_t)(t + TT * e) * pen) & (N - 1)];
#pragma unroll
          for (int c = 0; c < S; ++c) v[c][e] = cmul(v[c][e], w);  // times e^{-2 pi i n2 k1 / N}
        }
      }
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < S; ++c)
#pragma unroll
        for (int e = 0; e < E; ++e) out[base + c * g.V + t + TT * e] = v[c][e];
    }
  }
}

template <typename T, int L, int DIM, int MODE, int EE, bool PIPE>
static hipError_t run_contig_k(cx<T>* out, const cx<T>* in, const PassGeom& g, const cx<T>* tw,
                               hipStream_t st);

template <typename T, int L, int DIM, int MODE, int EE>
static hipError_t run_contig(cx<T>* out, const cx<T>* in, const PassGeom& g, const cx<T>* tw,
                             hipStream_t st) {
  // The prefetching variant is built for the complex64 3D evolution with
  // four elements per thread only (the autotuner's candidate; in complex128
  // it spills registers); elsewhere one group per workgroup.
  constexpr bool kPipe = DIM == 3 && EE == 4 && MODE == MODE_EVOLVE_TAB && sizeof(T) == 4;
  if constexpr (kPipe) {
    if (g.groups_per_wg > 1) return run_contig_k<T, L, DIM, MODE, EE, true>(out, in, g, tw, st);
  }
  return run_contig_k<T, L, DIM, MODE, EE, false>(out, in, g, tw, st);
}

template <typename T, int L, int DIM, int MODE, int EE, bool PIPE>
static hipError_t run_contig_k(cx<T>* out, const cx<T>* in, const PassGeom& g, const cx<T>* tw,
                               hipStream_t st) {
  constexpr int E = L < EE ? L : EE;
  constexpr int TT = L / E;
  int P = (g.block_threads > 0 ? g.block_threads : 256) / TT;
  if (P < 1) P = 1;
  if ((int64_t)P > g.pencils) {
    int q = 1;
    while ((int64_t)q < g.pencils) q <<= 1;
    P = q;
  }
  const int threads = TT * P;
  if (threads > 512) return hipErrorInvalidValue;
  const size_t lds = (size_t)P * (contig_components(DIM, MODE) * L + TT) * sizeof(cx<T>);
  auto kern = k_fft_contig<T, L, E, DIM, MODE, PIPE>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t ngroups = (g.pencils + P - 1) / P;
  // Enough workgroups to fill the chip g.groups_per_wg times over at most;
  // each then walks ngroups / nblk pencil groups with its loads one ahead.
  int64_t nblk = ngroups;
  if (PIPE && g.groups_per_wg > 1) {
    static int occ[2][8] = {};  // cached occupancy per (precision, log2 threads)
    int& o = occ[sizeof(T) == 8][ilog2(threads) & 7];
    if (o == 0) {
      int v = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, (const void*)kern, threads, lds) !=
              hipSuccess ||
          v < 1)
        v = 1;
      o = v;
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus < 1) cus = 1;
    const int64_t resident = (int64_t)o * cus;
    const int64_t want = (ngroups + g.groups_per_wg - 1) / g.groups_per_wg;
    nblk = std::max<int64_t>(resident, want);
    if (nblk > ngroups) nblk = ngroups;
  }
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(threads), lds, st, out, in, g, tw);
  return hipGetLastError();
}

template <typename T, int DIM, int MODE, int EE>
static hipError_t dispatch_contig(int64_t L, cx<T>* out, const cx<T>* in, const PassGeom& g,
                                  const cx<T>* tw, hipStream_t st) {
  switch (L) {
    case 2: return run_contig<T, 2, DIM, MODE, EE>(out, in, g, tw, st);
    case 4: return run_contig<T, 4, DIM, MODE, EE>(out, in, g, tw, st);
    case 8: return run_contig<T, 8, DIM, MODE, EE>(out, in, g, tw, st);
    case 16: return run_contig<T, 16, DIM, MODE, EE>(out, in, g, tw, st);
    case 32: return run_contig<T, 32, DIM, MODE, EE>(out, in, g, tw, st);
    case 64: return run_contig<T, 64, DIM, MODE, EE>(out, in, g, tw, st);
    case 128: return run_contig<T, 128, DIM, MODE, EE>(out, in, g, tw, st);
    case 256: return run_contig<T, 256, DIM, MODE, EE>(out, in, g, tw, st);
    case 512: return run_contig<T, 512, DIM, MODE, EE>(out, in, g, tw, st);
    case 1024:
      if constexpr (DIM <= 2) return run_contig<T, 1024, DIM, MODE, EE>(out, in, g, tw, st);
      return hipErrorInvalidValue;
    case 2048:
      if constexpr (DIM == 1) return run_contig<T, 2048, DIM, MODE, EE>(out, in, g, tw, st);
      return hipErrorInvalidValue;
    case 4096:
      if constexpr (DIM == 1 && EE >= 8) return run_contig<T, 4096, DIM, MODE, EE>(out, in, g, tw, st);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int MODE, int EE>
static hipError_t dispatch_dim(int64_t L, cx<T>* out, const cx<T>* in, const PassGeom& g,
                               const cx<T>* tw, hipStream_t st) {
  switch (g.dim) {
    case 1: return dispatch_contig<T, 1, MODE, EE>(L, out, in, g, tw, st);
    case 2: return dispatch_contig<T, 2, MODE, EE>(L, out, in, g, tw, st);
    case 3: return dispatch_contig<T, 3, MODE, EE>(L, out, in, g, tw, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t dispatch_mode(int mode, int64_t L, cx<T>* out, const cx<T>* in,
                                const PassGeom& g, const cx<T>* tw, hipStream_t st, int E) {
  // Four elements per thread for the table evolution of d = 2, 3 when the
  // autotuner picks it. The per-instance modes evaluate omega(q) in FP64 in
  // the kernel and run out of registers with eight (scratch spills), so they
  // take four wherever the team fits a workgroup (L <= 2048), except the
  // complex64 line, which fits eight.
  const bool e4 = E == 4 && g.dim >= 2;
  // Four elements per thread for complex64, two for complex128 (whose 32
  // values of eight components would not fit the register file).
  constexpr int kBccE = sizeof(T) == 8 ? 2 : 4;
  const bool e4i = L <= 2048 && (g.dim >= 2 || sizeof(T) == 8);
  // Two-component fields of d = 2, 3 (Weyl walks): the transforms alone are
  // the one-dimensional kernels (two components per pencil, no apply).
  if (g.s == 2 && g.dim >= 2) {
    switch (mode) {
      case MODE_FWD: return dispatch_contig<T, 1, MODE_FWD, 8>(L, out, in, g, tw, st);
      case MODE_INV: return dispatch_contig<T, 1, MODE_INV, 8>(L, out, in, g, tw, st);
      case MODE_WEYL:
        return g.dim == 2 ? dispatch_contig<T, 2, MODE_WEYL, 8>(L, out, in, g, tw, st)
                          : dispatch_contig<T, 3, MODE_WEYL, 8>(L, out, in, g, tw, st);
      case MODE_WEYL_TAB:
        if (!g.omega) return hipErrorInvalidValue;
        return g.dim == 2 ? dispatch_contig<T, 2, MODE_WEYL_TAB, 8>(L, out, in, g, tw, st)
                          : dispatch_contig<T, 3, MODE_WEYL_TAB, 8>(L, out, in, g, tw, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (mode) {
    case MODE_EVOLVE:
      return e4i ? dispatch_dim<T, MODE_EVOLVE, 4>(L, out, in, g, tw, st)
                 : dispatch_dim<T, MODE_EVOLVE, 8>(L, out, in, g, tw, st);
    // complex128 transforms alone take four elements per thread wherever
    // the team fits a workgroup (eight spill registers at L = 512).
    case MODE_FWD:
      return (sizeof(T) == 8 && e4i) ? dispatch_dim<T, MODE_FWD, 4>(L, out, in, g, tw, st)
                                     : dispatch_dim<T, MODE_FWD, 8>(L, out, in, g, tw, st);
    case MODE_INV:
      return (sizeof(T) == 8 && e4i) ? dispatch_dim<T, MODE_INV, 4>(L, out, in, g, tw, st)
                                     : dispatch_dim<T, MODE_INV, 8>(L, out, in, g, tw, st);
    case MODE_APPLY_INV:
      return e4i ? dispatch_dim<T, MODE_APPLY_INV, 4>(L, out, in, g, tw, st)
                 : dispatch_dim<T, MODE_APPLY_INV, 8>(L, out, in, g, tw, st);
    case MODE_PROJ_INV:
      return e4i ? dispatch_dim<T, MODE_PROJ_INV, 4>(L, out, in, g, tw, st)
                 : dispatch_dim<T, MODE_PROJ_INV, 8>(L, out, in, g, tw, st);
    case MODE_EVOLVE_TAB:
      return e4 ? dispatch_dim<T, MODE_EVOLVE_TAB, 4>(L, out, in, g, tw, st)
                : dispatch_dim<T, MODE_EVOLVE_TAB, 8>(L, out, in, g, tw, st);
    case MODE_APPLY_INV_TAB:
      if (!g.omega || g.inst) return hipErrorInvalidValue;
      return e4 ? dispatch_dim<T, MODE_APPLY_INV_TAB, 4>(L, out, in, g, tw, st)
                : dispatch_dim<T, MODE_APPLY_INV_TAB, 8>(L, out, in, g, tw, st);
    // Cubic-supercell field: eight components per pencil, kBccE elements each.
    case MODE_BCC:
      if (g.dim != 3) return hipErrorInvalidValue;
      return dispatch_contig<T, 3, MODE_BCC, kBccE>(L, out, in, g, tw, st);
    case MODE_BCC_FWD:
      if (g.dim != 3) return hipErrorInvalidValue;
      return dispatch_contig<T, 3, MODE_BCC_FWD, kBccE>(L, out, in, g, tw, st);
    case MODE_BCC_INV:
      if (g.dim != 3) return hipErrorInvalidValue;
      return dispatch_contig<T, 3, MODE_BCC_INV, kBccE>(L, out, in, g, tw, st);
    case MODE_BCC_TAB:
      if (g.dim != 3 || !g.omega) return hipErrorInvalidValue;
      return dispatch_contig<T, 3, MODE_BCC_TAB, kBccE>(L, out, in, g, tw, st);
    default: return hipErrorInvalidValue;
  }
}

// omega(q) for every wave-vector, in the storage order of the contiguous pass
// (pencil-major; for the 1D four-step the order k1 + N1 k2 of its rows).
template <int DIM>
__global__ __launch_bounds__(256) void k_omega_table(PassGeom g, int64_t L, double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.V) return;
  const int64_t pen = idx / L, z = idx - pen * L;
  int64_t j1, j2, j3;
  q_index<DIM>(g, pen, z, j1, j2, j3);
  out[idx] = omega_q(DIM, g, g.single.n, g.single.m, j1, j2, j3);
}

hipError_t launch_omega_table(const PassGeom& g, int64_t L, double* omega, hipStream_t st) {
  const unsigned nblk = (unsigned)((g.V + 255) / 256);
  if (g.dim == 1) hipLaunchKernelGGL(k_omega_table<1>, dim3(nblk), dim3(256), 0, st, g, L, omega);
  else if (g.dim == 2) hipLaunchKernelGGL(k_omega_table<2>, dim3(nblk), dim3(256), 0, st, g, L, omega);
  else hipLaunchKernelGGL(k_omega_table<3>, dim3(nblk), dim3(256), 0, st, g, L, omega);
  return hipGetLastError();
}

// omega(kappa), kappa = pi j / N, for the cubic-supercell pass (the Weyl u
// and n~ at the Cartesian kappa, from the FP64 trig table).
__global__ __launch_bounds__(256) void k_omega_bcc_table(PassGeom g, int64_t L,
                                                         double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.V) return;
  const int64_t pen = idx / L, z = idx - pen * L;
  int64_t j1, j2, j3;
  q_index<3>(g, pen, z, j1, j2, j3);
  const int64_t mask = 2 * (int64_t)g.Nc - 1;
  const int64_t a1 = (j1 << g.shift[0]) & mask;
  const int64_t a2 = (j2 << g.shift[1]) & mask;
  const int64_t a3 = (j3 << g.shift[2]) & mask;
  const double cx_ = g.cs[2 * a1], sx = g.cs[2 * a1 + 1];
  const double cy = g.cs[2 * a2], sy = g.cs[2 * a2 + 1];
  const double cz = g.cs[2 * a3], sz = g.cs[2 * a3 + 1];
  const double u = cx_ * cy * cz + sx * sy * sz;
  const double n1 = sx * cy * cz - cx_ * sy * sz;
  const double n2 = cx_ * sy * cz + sx * cy * sz;
  const double n3 = cx_ * cy * sz - sx * sy * cz;
  const double nn = g.single.n, m = g.single.m;
  out[idx] = atan2(sqrt(nn * nn * (n1 * n1 + n2 * n2 + n3 * n3) + m * m), nn * u);
}

hipError_t launch_omega_bcc_table(const PassGeom& g, int64_t L, double* omega, hipStream_t st) {
  if (g.dim != 3) return hipErrorInvalidValue;
  const unsigned nblk = (unsigned)((g.V + 255) / 256);
  hipLaunchKernelGGL(k_omega_bcc_table, dim3(nblk), dim3(256), 0, st, g, L, omega);
  return hipGetLastError();
}

hipError_t launch_fft_contig(bool dbl, int mode, int64_t L, void* out, const void* in,
                             const PassGeom& g, const void* tw, hipStream_t st, int E) {
  if (dbl)
    return dispatch_mode<double>(mode, L, (cx<double>*)out, (const cx<double>*)in, g,
                                 (const cx<double>*)tw, st, E);
  return dispatch_mode<float>(mode, L, (cx<float>*)out, (const cx<float>*)in, g,
                              (const cx<float>*)tw, st, E);
}

}  // namespace qw
