"""Fourier evaluation of U^t (test infrastructure).

Sec. 4: psi(t) = U^t psi(0) is evaluated in the Fourier representation of
Sec. 2.1, where U acts at each wave-vector as the s x s matrix U_q. The DFT
carries the paper's sign: hat psi(q) = sum_n e^{+i q.n} psi(n), with inverse
psi(n) = V^-1 sum_q e^{-i q.n} hat psi(q) (the 1/sqrt(V) of each direction
and the half-band index shift are folded into one 1/V and dropped; neither
changes the result). With this sign a plane wave e^{-iq.n} v is the pure
frequency q, and one step multiplies hat psi(q) by U_q = sum_h e^{-iq.h} U_h.

U_q is summed directly from the transition-matrix table (not from any closed
form), and U_q^t is formed by binary powering (U_q^dag for t < 0); for real
t (the continuous-time interpolation of Sec. 4, psi(t) with e^{-i H(k) t})
by diagonalising U_q.
"""
import numpy as np

from . import walk


def dft(psi):
    """hat psi(q) = sum_n e^{+i q.n} psi(n) over the lattice axes."""
    axes = tuple(range(1, psi.ndim))
    V = int(np.prod(psi.shape[1:]))
    return np.fft.ifftn(psi, axes=axes) * V


def idft(phat):
    """psi(n) = V^-1 sum_q e^{-i q.n} hat psi(q)."""
    axes = tuple(range(1, phat.ndim))
    V = int(np.prod(phat.shape[1:]))
    return np.fft.fftn(phat, axes=axes) / V


def symbol_grid(table, N, d):
    """U_q[N_1,...,N_d, s, s] on the DFT grid, by direct summation."""
    return walk.symbol_from_table(table, walk.lattice_q(N, d))


def matpow(D, t):
    """D^t for a stack D[..., s, s] by binary powering; D^dag^|t| if t < 0."""
    t = int(t)
    if t < 0:
        D = np.conj(np.swapaxes(D, -1, -2))
        t = -t
    s = D.shape[-1]
    R = np.broadcast_to(np.eye(s, dtype=np.complex128), D.shape).copy()
    B = D.copy()
    while t:
        if t & 1:
            R = R @ B
        t >>= 1
        if t:
            B = B @ B
    return R


def apply_symbol(Dt, phat):
    """out(q) = Dt(q) hat psi(q), with phat[c, q...] component-first."""
    ph = np.moveaxis(phat, 0, -1)[..., None]
    return np.moveaxis((Dt @ ph)[..., 0], -1, 0)


def evolve_fourier(psi, table, t):
    """U^t psi by DFT, per-q binary powering of U_q, inverse DFT."""
    d = psi.ndim - 1
    Dt = matpow(symbol_grid(table, psi.shape[1:], d), t)
    return idft(apply_symbol(Dt, dft(psi)))


def matpow_real(D, t):
    """D^t for real t and a stack of unitary D[..., s, s]: exp(-i t H) with
    D = exp(-i H) and the spectrum of H in [-pi, pi] (the continuous-time
    interpolation of Sec. 4, exact at integer t). D is diagonalised in an
    orthonormal basis through the commuting Hermitian parts A = (D + D^dag)/2,
    B = (D - D^dag)/2i: the eigenvectors of A + c B for a generic c are
    eigenvectors of D. An eigenvalue -1 (phase pi, reached only at the band
    edge when m = 0) has two one-sided limits e^{+-i pi t}; their average
    cos(pi t) is taken."""
    t = float(t)
    Dh = np.conj(np.swapaxes(D, -1, -2))
    A = (D + Dh) / 2
    B = (D - Dh) / 2j
    _, V = np.linalg.eigh(A + 0.7390851332151607 * B)
    lam = np.einsum("...ji,...jk,...ki->...i", np.conj(V), D, V)
    theta = np.angle(lam)
    f = np.exp(1j * t * theta)
    edge = np.abs(lam + 1.0) < 1e-12
    f = np.where(edge, np.cos(np.pi * t), f)
    return V @ (f[..., :, None] * np.conj(np.swapaxes(V, -1, -2)))


def evolve_fourier_real(psi, table, t):
    """U^t psi for real t: DFT, per-q exp(-i t H_q) by diagonalisation,
    inverse DFT."""
    d = psi.ndim - 1
    Dt = matpow_real(symbol_grid(table, psi.shape[1:], d), t)
    return idft(apply_symbol(Dt, dft(psi)))
