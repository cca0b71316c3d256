"""Proposition 1 (Sec. 5.1): the dispersive approximation of the evolution
of a particle state (test infrastructure).

A particle state evolves exactly as hat psi(k, t) = e^{-i omega_k t} hat
psi(k, 0) in its sector (e^{+i omega_k t} in the antiparticle sector).
Truncating the expansion of omega_k about the central wave-vector k' at
order n (the dispersive differential equation of Proposition 1; order 2
gives the drift vector and the diffusion tensor) replaces omega_k by its
Taylor polynomial T_n(k - k'). The overlap of the approximate and the exact
state obeys the bound of the proof of Proposition 1,
|<psi~(t)|psi(t)>| >= 1 - epsilon - gamma Sigma^{n+1} t (up to higher
orders in Sigma), with epsilon and Sigma from Definition 1.

omega_k = arccos(n u(k)) with u the identity component of the Weyl symbol
of Sec. 3.1 (cos omega = n u, the dispersion of Sec. 3.2), differentiated
symbolically in the Cartesian k. On the lattice k - k' is taken from the
per-axis wrapped q - q' (as for the Gaussian itself).
"""
import itertools
import math

import numpy as np
import sympy as sp

from . import fourier, states, walk


def u_expr(d, k):
    """u(k) of the Weyl walks of Sec. 3.1 in Cartesian k (1D: cos k; 2D,
    reading of the square lattice: cos kx cos ky; 3D BCC:
    cos kx cos ky cos kz + sin kx sin ky sin kz)."""
    if d == 1:
        return sp.cos(k[0])
    if d == 2:
        return sp.cos(k[0]) * sp.cos(k[1])
    return (sp.cos(k[0]) * sp.cos(k[1]) * sp.cos(k[2]) +
            sp.sin(k[0]) * sp.sin(k[1]) * sp.sin(k[2]))


def multi_indices(d, order):
    """All alpha in N^d with |alpha| = order."""
    return [a for a in itertools.product(range(order + 1), repeat=d) if sum(a) == order]


def derivatives(d, m, k0, order):
    """{alpha: d^alpha omega / dk^alpha at k0} for |alpha| <= order, from the
    symbolic omega = acos(n u(k)), evaluated with 30 digits."""
    k = sp.symbols("k0:%d" % d, real=True)
    mm = sp.Rational(float(m))
    n = sp.sqrt(1 - mm * mm)
    w = sp.acos(n * u_expr(d, k))
    at = {k[i]: sp.Rational(float(k0[i])) for i in range(d)}
    out = {}
    for o in range(order + 1):
        for a in multi_indices(d, o):
            e = w
            for i in range(d):
                if a[i]:
                    e = sp.diff(e, k[i], a[i])
            out[a] = float(sp.N(e.subs(at), 30))
    return out


def taylor_coefficients(d, m, k0, order):
    """{alpha: omega^(alpha)(k0) / alpha!} for |alpha| <= order."""
    der = derivatives(d, m, k0, order)
    return {a: v / math.prod(math.factorial(x) for x in a) for a, v in der.items()}


def delta_k(d, N, k0):
    """k - k' on the DFT grid [..., d]: per-axis wrapped q - q', mapped to
    Cartesian k (the linear map k(q) of the lattice)."""
    q = walk.lattice_q(N, d)
    q0 = walk.q_of_k(d, np.asarray(k0, dtype=np.float64).reshape(d))
    dq = np.mod(q - q0 + np.pi, 2.0 * np.pi) - np.pi
    return walk.k_of_q(d, dq)


def taylor_grid(d, N, k0, coeffs):
    """T_n(k - k') on the DFT grid."""
    dk = delta_k(d, N, k0)
    T = np.zeros(dk.shape[:-1])
    for a, c in coeffs.items():
        term = np.full(dk.shape[:-1], c)
        for i in range(d):
            if a[i]:
                term = term * dk[..., i] ** a[i]
        T = T + term
    return T


def evolve_dispersive(d, N, m, k0, sigma, center, c_plus, c_minus, order, t):
    """The order-n approximation psi~(t) of the evolved particle state."""
    sp_, sm_ = states.particle_spectra(d, N, m, k0, sigma, center, c_plus, c_minus)
    T = taylor_grid(d, N, k0, taylor_coefficients(d, m, k0, order))
    phat = sp_ * np.exp(-1j * t * T) + sm_ * np.exp(1j * t * T)
    psi = fourier.idft(phat)
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2))


def overlap_bound(d, N, m, k0, sigma, center, order, t, box):
    """1 - epsilon - gamma Sigma^{n+1} t for the particle state (c+ = 1) with
    the box |k_i - k'_i| <= box of Definition 1 (Sigma = box): epsilon is
    the weight of |g|^2 outside the box and gamma = (n+1) sum over
    |alpha| = n+1 of |omega^(alpha)| / alpha! times the weight inside."""
    sp_, _ = states.particle_spectra(d, N, m, k0, sigma, center, 1.0, 0.0)
    w = np.sum(np.abs(sp_) ** 2, axis=0)
    w = w / np.sum(w)
    inside = np.all(np.abs(delta_k(d, N, k0)) <= box, axis=-1)
    W = float(np.sum(w[inside]))
    eps = 1.0 - W
    der = derivatives(d, m, k0, order + 1)
    s = sum(abs(v) / math.prod(math.factorial(x) for x in a)
            for a, v in der.items() if sum(a) == order + 1)
    gamma = (order + 1) * s * W
    return 1.0 - eps - gamma * box ** (order + 1) * t, eps, gamma
