"""Position-space stepping: the ground truth (test infrastructure).

Sec. 2, update rule: psi(x,t+1) = sum_y E(y,x) psi(y,t). For the homogeneous
walk U = sum_h T_h (x) U_h with T_y|x> = |x-y> (Sec. 2.1) this reads
psi(x,t+1) = sum_h U_h psi(x+h,t) on the periodic N^d torus. The inverse step
is the adjoint walk, psi(x,t-1) = sum_h U_h^dag psi(x-h,t).

Fields are complex128 arrays psi[c, n_1, ..., n_d] (component first, then
the lattice axes in primitive coordinates, last axis fastest).
"""
import numpy as np


def _shifted(psi, off):
    """Return a with a[c, n] = psi[c, n + off] (periodic)."""
    d = psi.ndim - 1
    return np.roll(psi, shift=[-o for o in off], axis=tuple(range(1, d + 1)))


def step(psi, table):
    """One walk step psi(x) <- sum_h U_h psi(x+h)."""
    out = np.zeros_like(psi)
    for off, U in table.items():
        out += np.tensordot(U, _shifted(psi, off), axes=(1, 0))
    return out


def step_back(psi, table):
    """One inverse step psi(x) <- sum_h U_h^dag psi(x-h)."""
    out = np.zeros_like(psi)
    for off, U in table.items():
        neg = tuple(-o for o in off)
        out += np.tensordot(U.conj().T, _shifted(psi, neg), axes=(1, 0))
    return out


def evolve_steps(psi, table, t):
    """U^t psi by |t| successive (inverse, if t < 0) steps."""
    psi = np.array(psi, dtype=np.complex128, copy=True)
    f = step if t >= 0 else step_back
    for _ in range(abs(int(t))):
        psi = f(psi, table)
    return psi
