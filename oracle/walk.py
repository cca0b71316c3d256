"""Walk definitions (test infrastructure; see the package header).

Sources in the paper:
* Sec. 2: update rule psi(x,t+1) = sum_y E(y,x) psi(y,t); walk operator
  U = sum_h T_h (x) U_h; unitarity conditions on the transition matrices.
* Sec. 2.1: translations T_y|x> = |x-y>, plane waves |k> ~ sum_x e^{-ik.x}|x>,
  Fourier symbol U_k = sum_h e^{-ik.h} U_h.
* Sec. 3.1: Weyl symbols W_k = u_k I - i sigma . n~_k for d = 3 (BCC), d = 2
  (square lattice) and d = 1; BCC generators h1..h4.
* Sec. 3.2: Dirac coupling D_k = [[n W_k, i m], [i m, n W_k^dag]], n^2+m^2=1,
  and the two-component 1D form D_k = [[n e^{-ik}, i m], [i m, n e^{ik}]].

Readings taken here (each also listed in the design notes):
* The lattice is stored in primitive-cell coordinates n in Z_N^d; the
  Cartesian site is x = H n where the columns of H are the generators h_j.
  A wave-vector q in lattice coordinates is q_j = k . h_j, i.e. q = H^T k.
* 3D: h1 = (1,1,1), h2 = (1,-1,-1), h3 = (-1,1,-1) (Sec. 3.1); h4 = -(h1+h2+h3)
  is the lattice offset (-1,-1,-1).
* 2D: the paper's definition of k_x, k_y in terms of k_1, k_2 is read as the
  primitive generators h1 = (1,1), h2 = (1,-1), so k_x = (q1+q2)/2 and
  k_y = (q1-q2)/2. With this reading the symbol has support on the four
  nearest neighbours +-e1, +-e2 only.
* 1D uses the two-component Dirac walk of Sec. 3.2 (the four-component one
  decouples into two copies of it).
* The spinor component order is the matrix index of D_k as printed.
"""
import itertools

import numpy as np

SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)
I2 = np.eye(2, dtype=np.complex128)


def spinor_dim(d):
    """Coin dimension s: 2 for the 1D Dirac walk, 4 for d = 2, 3 (Sec. 3.2)."""
    if d == 1:
        return 2
    if d in (2, 3):
        return 4
    raise ValueError("dimension must be 1, 2 or 3")


def mass_n(m):
    """n = sqrt(1 - m^2), the coupling constraint n^2 + m^2 = 1 (Sec. 3.2)."""
    m = float(m)
    if not (0.0 <= m <= 1.0):
        raise ValueError("m must lie in [0, 1]")
    return float(np.sqrt(1.0 - m * m))


def generators(d):
    """Matrix H whose columns are the primitive generators h_j (Cartesian).

    3D: the BCC generators h1, h2, h3 of Sec. 3.1. 2D: h1 = (1,1), h2 = (1,-1)
    (reading of the 2D k_x, k_y definition). 1D: h = 1.
    """
    if d == 1:
        return np.array([[1.0]])
    if d == 2:
        return np.array([[1.0, 1.0], [1.0, -1.0]])
    if d == 3:
        h1 = [1.0, 1.0, 1.0]
        h2 = [1.0, -1.0, -1.0]
        h3 = [-1.0, 1.0, -1.0]
        return np.array([h1, h2, h3]).T
    raise ValueError("dimension must be 1, 2 or 3")


def q_of_k(d, k):
    """Lattice wave-vector q = H^T k (q_j = k . h_j) for Cartesian k[..., d]."""
    return np.asarray(k, dtype=np.float64) @ generators(d)


def k_of_q(d, q):
    """Cartesian wave-vector k = H^{-T} q for lattice q[..., d]."""
    H = generators(d)
    return np.asarray(q, dtype=np.float64) @ np.linalg.inv(H)


def weyl_u_n(d, k):
    """u_k and n~_k of the Weyl walk at Cartesian k[..., d] (Sec. 3.1).

    Returns (u, nt) with u[...] and nt[..., 3].
    """
    k = np.asarray(k, dtype=np.float64)
    c = np.cos(k)
    s = np.sin(k)
    if d == 3:
        cx, cy, cz = c[..., 0], c[..., 1], c[..., 2]
        sx, sy, sz = s[..., 0], s[..., 1], s[..., 2]
        u = cx * cy * cz + sx * sy * sz
        nt = np.stack([sx * cy * cz - cx * sy * sz,
                       cx * sy * cz + sx * cy * sz,
                       cx * cy * sz - sx * sy * cz], axis=-1)
    elif d == 2:
        cx, cy = c[..., 0], c[..., 1]
        sx, sy = s[..., 0], s[..., 1]
        u = cx * cy
        nt = np.stack([sx * cy, cx * sy, sx * sy], axis=-1)
    elif d == 1:
        u = c[..., 0]
        nt = np.stack([np.zeros_like(u), np.zeros_like(u), s[..., 0]], axis=-1)
    else:
        raise ValueError("dimension must be 1, 2 or 3")
    return u, nt


def weyl_symbol(d, k):
    """W_k = u_k I - i sigma . n~_k (Sec. 3.1, general Weyl form)."""
    u, nt = weyl_u_n(d, k)
    W = u[..., None, None] * I2
    for a in range(3):
        W = W - 1j * nt[..., a, None, None] * SIGMA[a]
    return W


def dirac_symbol(d, q, m):
    """Dirac walk symbol D(q)[..., s, s] at lattice wave-vector q[..., d].

    d = 2, 3: the block coupling of two Weyl walks [[nW, im], [im, nW^dag]]
    (Sec. 3.2), W evaluated at the Cartesian k = H^{-T} q.
    d = 1: [[n e^{-iq}, im], [im, n e^{iq}]] (Sec. 3.2, one space dimension).
    """
    q = np.asarray(q, dtype=np.float64)
    n = mass_n(m)
    if d == 1:
        qq = q[..., 0]
        D = np.zeros(qq.shape + (2, 2), dtype=np.complex128)
        D[..., 0, 0] = n * np.exp(-1j * qq)
        D[..., 1, 1] = n * np.exp(1j * qq)
        D[..., 0, 1] = 1j * m
        D[..., 1, 0] = 1j * m
        return D
    W = weyl_symbol(d, k_of_q(d, q))
    D = np.zeros(W.shape[:-2] + (4, 4), dtype=np.complex128)
    D[..., :2, :2] = n * W
    D[..., 2:, 2:] = n * np.conj(np.swapaxes(W, -1, -2))
    D[..., :2, 2:] = 1j * m * I2
    D[..., 2:, :2] = 1j * m * I2
    return D


def stencil_table(d, m, L=4, tol=1e-13):
    """Transition matrices U_h of the walk, from its symbol (Sec. 2.1).

    The symbol is U(q) = sum_h e^{-iq.h} U_h, so U_h is the inverse DFT
    U_h = L^-d sum_q e^{+iq.h} U(q) over the L^d grid q = 2 pi j / L. With
    L = 4 the offsets -1, 0, 1, 2 are distinct mod L; a coefficient at offset
    2 (or a mismatch of the symbol off the grid, checked by the tests) would
    mean the support is wider than one cell. Returns {offset tuple: U_h}
    holding the entries whose largest magnitude exceeds ``tol``.
    """
    s = spinor_dim(d)
    grid = np.stack(np.meshgrid(*([np.arange(L)] * d), indexing="ij"), axis=-1)
    q = 2.0 * np.pi * grid.reshape(-1, d) / L
    Dq = dirac_symbol(d, q, m)
    table = {}
    for off in itertools.product((-1, 0, 1, 2), repeat=d):
        phase = np.exp(1j * (q @ np.array(off, dtype=np.float64)))
        U = np.tensordot(phase, Dq, axes=(0, 0)) / q.shape[0]
        if np.abs(U).max() > tol:
            if max(abs(o) for o in off) > 1:
                raise AssertionError("symbol support wider than one cell at %r" % (off,))
            table[off] = U.reshape(s, s)
    return table


def weyl_table(d, L=4, tol=1e-13):
    """Transition matrices of the two-component Weyl walk (Sec. 3.1): the
    inverse DFT over the L^d grid of W at the Cartesian k = H^{-T} q, exactly
    as for the Dirac walk in ``stencil_table``. The 1D Weyl walk is
    W = diag(e^{-ik}, e^{ik}) (the Dirac walk at m = 0)."""
    grid = np.stack(np.meshgrid(*([np.arange(L)] * d), indexing="ij"), axis=-1)
    q = 2.0 * np.pi * grid.reshape(-1, d) / L
    if d == 1:
        Wq = dirac_symbol(1, q, 0.0)
    else:
        Wq = weyl_symbol(d, k_of_q(d, q))
    table = {}
    for off in itertools.product((-1, 0, 1, 2), repeat=d):
        phase = np.exp(1j * (q @ np.array(off, dtype=np.float64)))
        U = np.tensordot(phase, Wq, axes=(0, 0)) / q.shape[0]
        if np.abs(U).max() > tol:
            if max(abs(o) for o in off) > 1:
                raise AssertionError("symbol support wider than one cell at %r" % (off,))
            table[off] = U.reshape(2, 2)
    return table


def symbol_from_table(table, q):
    """U(q) = sum_h e^{-iq.h} U_h by direct summation (Sec. 2.1)."""
    q = np.asarray(q, dtype=np.float64)
    s = next(iter(table.values())).shape[0]
    out = np.zeros(q.shape[:-1] + (s, s), dtype=np.complex128)
    for off, U in table.items():
        ph = np.exp(-1j * (q @ np.array(off, dtype=np.float64)))
        out = out + ph[..., None, None] * U
    return out


def unitarity_defect(table):
    """Largest violation of the unitarity conditions on the U_h (Sec. 2).

    sum_h U_h^dag U_h = sum_h U_h U_h^dag = I, and for every non-zero offset
    h'' the sums of U_h^dag U_h' over h' - h = h'' and of U_h' U_h^dag over
    h' - h = h'' vanish.
    """
    offs = list(table)
    s = table[offs[0]].shape[0]
    eye = np.eye(s)
    worst = 0.0
    worst = max(worst, np.abs(sum(U.conj().T @ U for U in table.values()) - eye).max())
    worst = max(worst, np.abs(sum(U @ U.conj().T for U in table.values()) - eye).max())
    diffs = {}
    for h in offs:
        for hp in offs:
            dd = tuple(a - b for a, b in zip(hp, h))
            if any(dd):
                diffs.setdefault(dd, []).append((h, hp))
    for dd, pairs in diffs.items():
        a = sum(table[h].conj().T @ table[hp] for h, hp in pairs)
        b = sum(table[hp] @ table[h].conj().T for h, hp in pairs)
        worst = max(worst, np.abs(a).max(), np.abs(b).max())
    return float(worst)


def lattice_q(N, d):
    """DFT frequencies q[N_1,...,N_d, d] = 2 pi j_i / N_i on the unshifted
    index set (N an int for a cubic torus, or a tuple of d sizes).

    The paper shifts the index set by floor(N/2) so frequencies lie in
    [-pi, pi) (Sec. 4); the symbol is 2 pi periodic, so the unshifted set
    describes the same samples.
    """
    Ns = (int(N),) * d if np.isscalar(N) else tuple(int(x) for x in N)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in Ns], indexing="ij"), axis=-1)
    return 2.0 * np.pi * j.astype(np.float64) / np.array(Ns, dtype=np.float64)
