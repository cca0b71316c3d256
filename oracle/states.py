"""Initial states (test infrastructure).

* Particle states, Sec. 5.1 Definition 1: a wave-packet g(k)|k>|u(k)> that is
  smooth and concentrated around a central wave-vector k', built on one
  frequency sector of the walk. Sec. 5.2 superposes a particle and an
  antiparticle packet c+ psi+ + c- psi- with |c+|^2 + |c-|^2 = 1.
* Perfectly localised states |x>|zeta> (Sec. 5.2).

Readings (listed in the design notes):
* g is the amplitude Gaussian exp(-sigma^2 |dq|^2 / 2) in lattice
  coordinates q, with dq_j = q_j - q'_j wrapped to [-pi, pi) per axis,
  sigma in lattice cells (the paper quotes the k-space width 1/sigma), times
  the carrier e^{+i q.c} that centres the packet at site c.
* "Projected on the eigenvector" is taken gauge-free: the sector projector
  P_s(q) applied to a fixed spinor chi_s, the normalised column of P_s(q')
  with the largest 2-norm. The column norms of a projector come in exact
  structural pairs (P_jj = P_kk), so the tie rule takes the lowest index
  whose norm is within a relative 1e-12 of the largest. P_+ is the spectral
  projector of U_q on its eigenvalue e^{-i omega} (positive frequency,
  particle), P_- the one on e^{+i omega}.
"""
import numpy as np

from . import fourier, walk

SINGULAR_SIN_OMEGA = 1e-12


def sector_projectors(D):
    """Spectral projectors (P+, P-) of the unitary stack D[..., s, s].

    For every walk of Sec. 3 the symbol has the form cos(omega) I - i M with
    M Hermitian, trace-free and M^2 = sin^2(omega) I (the eigenvalues are
    e^{-+i omega}). So cos(omega) = Re tr(D)/s, M = i(D - cos(omega) I), every
    column of M has norm sin(omega), and P+- = (I +- M / sin(omega)) / 2.
    Where sin(omega) < 1e-12 the two eigenvalues coincide and I/2 is used.
    """
    s = D.shape[-1]
    eye = np.eye(s, dtype=np.complex128)
    cosw = np.real(np.trace(D, axis1=-2, axis2=-1)) / s
    M = 1j * (D - cosw[..., None, None] * eye)
    sinw = np.sqrt(np.sum(np.abs(M[..., :, 0]) ** 2, axis=-1))
    safe = sinw >= SINGULAR_SIN_OMEGA
    Mh = np.where(safe[..., None, None], M / np.where(safe, sinw, 1.0)[..., None, None], 0.0)
    return 0.5 * (eye + Mh), 0.5 * (eye - Mh)


CHI_TIE = 1e-12


def _chi(P0):
    norms = np.sqrt(np.sum(np.abs(P0) ** 2, axis=0))
    top = norms.max()
    j = int(np.flatnonzero(norms >= top * (1.0 - CHI_TIE))[0])
    return P0[:, j] / norms[j]


def particle_spectra(d, N, m, k0_cart, sigma, center, c_plus=1.0, c_minus=0.0):
    """The two sector spectra c+ hat psi+(q) and c- hat psi-(q) of the
    Gaussian particle/antiparticle state, component-first [s, q_1..q_d],
    scaled so that their sum has the unit-norm position state as its
    inverse DFT. A sector with a zero coefficient is all zeros."""
    table = walk.stencil_table(d, m)
    q = walk.lattice_q(N, d)
    q0 = walk.q_of_k(d, np.asarray(k0_cart, dtype=np.float64).reshape(d))
    c = np.asarray(center, dtype=np.float64).reshape(d)
    dq = np.mod(q - q0 + np.pi, 2.0 * np.pi) - np.pi
    g = np.exp(-0.5 * sigma * sigma * np.sum(dq * dq, axis=-1)) * np.exp(1j * (q @ c))
    Dq = walk.symbol_from_table(table, q)
    Pp, Pm = sector_projectors(Dq)
    P0p, P0m = sector_projectors(walk.symbol_from_table(table, q0))
    out = []
    for coef, P, P0 in ((c_plus, Pp, P0p), (c_minus, Pm, P0m)):
        if coef == 0:
            out.append(np.zeros((Dq.shape[-1],) + tuple(g.shape), dtype=np.complex128))
            continue
        sec = g[..., None] * (P @ _chi(P0))            # [..., s]
        sec = sec / np.sqrt(np.sum(np.abs(sec) ** 2))
        out.append(np.moveaxis(coef * sec, -1, 0))
    # the sectors are orthogonal at every q: |psi|^2 = |c+|^2 + |c-|^2 before
    # the inverse DFT, whose norm is that over sqrt(V)
    V = int(np.prod(g.shape))
    scale = np.sqrt(V) / np.sqrt(abs(c_plus) ** 2 + abs(c_minus) ** 2)
    return out[0] * scale, out[1] * scale


def particle_state(d, N, m, k0_cart, sigma, center, c_plus=1.0, c_minus=0.0):
    """Gaussian particle/antiparticle state on the N^d torus, unit 2-norm.
    Returns psi[c, n_1..n_d] (complex128).
    """
    sp, sm = particle_spectra(d, N, m, k0_cart, sigma, center, c_plus, c_minus)
    psi = fourier.idft(sp + sm)
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2))


def localized_state(d, N, center, zeta):
    """|x>|zeta> with x = center (Sec. 5.2, perfectly localised states)."""
    zeta = np.asarray(zeta, dtype=np.complex128)
    psi = np.zeros((zeta.size,) + (N,) * d, dtype=np.complex128)
    psi[(slice(None),) + tuple(int(x) for x in center)] = zeta
    return psi
