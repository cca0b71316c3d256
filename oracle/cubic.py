"""Cubic-supercell representation of the BCC lattice (test infrastructure).

Sec. 4 (the BCC paragraph, eq:bcc-dft and eq:bcc-idft): the BCC vertex set is
G = 2Z^3 u (2Z^3 + t), t = (1,1,1), i.e. the Cartesian sites whose three
coordinates share one parity. It is truncated to B = 2N u (2N + t), with
N = [0,N1) x [0,N2) x [0,N3), and extended periodically (period 2 N_i along
Cartesian axis i), then split into the sublattice sequences
f0_n = f_{2n} and f1_n = f_{2n+t}, n in N, each periodic with matrix
diag(N1, N2, N3). Its Fourier transform over the index set
K = [-N1,N1) x [-N2,N2) x [-N3,N3) is
    hat f_k = (2 sqrt|B|)^-1 sum_{n in B} f_n e^{2 pi i k.(2N)^-1 n},
and reduces to two rectangular DFTs of the sublattice arrays combined with
a_k = e^{i pi k.N^-1 t} (eq:bcc-dft), with the inverse of eq:bcc-idft.

Fields are complex128 arrays f[2, s, N1, N2, N3]: sublattice first (0: even
sites 2n, 1: odd sites 2n + t), then the spinor component, then the three
sublattice indices (last fastest). A Cartesian field is fc[s, 2N1, 2N2, 2N3]
with zeros on the mixed-parity sites.

Readings taken here (each also listed in the design notes):
* The rectangular F of eq:bcc-dft is the DFT of eq:dft with the paper's sign
  (e^{+2 pi i k.N^-1 n}), normalised by 1/sqrt(N1 N2 N3), without the
  half-band shift p (the BCC transform above has none), on k in N. With it,
  hat f1_k = 2 hat f_k and hat f0_k = 2 hat f_{k + N1 e1}: hat f1 samples the
  BCC spectrum at the Cartesian wave-vector kappa = pi k / N (per axis),
  hat f0 at kappa + pi e_x; the other points of K repeat these (the spectrum
  is periodic under the reciprocal FCC lattice).
* The walk on this torus is the update rule of Sec. 2 with the Cartesian
  offsets of the transition matrices (the primitive offset o is the Cartesian
  displacement H o, H the matrix of the generators h1, h2, h3 of Sec. 3.1).
  Its symbol at Cartesian kappa is U(kappa) = sum_h e^{-i kappa.h} U_h.
"""
import numpy as np

from . import fourier, walk


def split(fc):
    """Sublattice arrays f[2, s, N1, N2, N3] of a Cartesian field
    fc[s, 2N1, 2N2, 2N3]: f0_n = f_{2n}, f1_n = f_{2n+t}."""
    f0 = fc[:, 0::2, 0::2, 0::2]
    f1 = fc[:, 1::2, 1::2, 1::2]
    return np.stack([f0, f1]).astype(np.complex128)


def embed(f):
    """Cartesian field fc[s, 2N1, 2N2, 2N3] holding f0 on the even sites and
    f1 on the odd sites, zero on the mixed-parity sites."""
    _, s, N1, N2, N3 = f.shape
    fc = np.zeros((s, 2 * N1, 2 * N2, 2 * N3), dtype=np.complex128)
    fc[:, 0::2, 0::2, 0::2] = f[0]
    fc[:, 1::2, 1::2, 1::2] = f[1]
    return fc


def bcc_dft_direct(f):
    """hat f_k over all of K by the direct sum of the definition (tiny tori
    only). Returns hat[s, 2N1, 2N2, 2N3] indexed by k + N (k from -N to N-1)."""
    _, s, N1, N2, N3 = f.shape
    Ns = np.array([N1, N2, N3], dtype=np.float64)
    n = np.stack(np.meshgrid(np.arange(N1), np.arange(N2), np.arange(N3), indexing="ij"),
                 axis=-1).reshape(-1, 3)
    sites = np.concatenate([2 * n, 2 * n + 1])                       # B, Cartesian
    vals = np.concatenate([f[0].reshape(s, -1), f[1].reshape(s, -1)], axis=1)
    k = np.stack(np.meshgrid(np.arange(-N1, N1), np.arange(-N2, N2), np.arange(-N3, N3),
                             indexing="ij"), axis=-1).reshape(-1, 3)
    ph = np.exp(2j * np.pi * ((k / (2 * Ns)) @ sites.T.astype(np.float64)))
    card = 2 * N1 * N2 * N3
    hat = (vals @ ph.T) / (2.0 * np.sqrt(card))
    return hat.reshape(s, 2 * N1, 2 * N2, 2 * N3)


def rect_dft(g):
    """F(g)(k) = (N1 N2 N3)^-1/2 sum_n g_n e^{+2 pi i k.N^-1 n} over the last
    three axes (eq:dft with the sign of Sec. 4, unshifted)."""
    V = int(np.prod(g.shape[-3:]))
    return np.fft.ifftn(g, axes=(-3, -2, -1)) * np.sqrt(V)


def rect_idft(g):
    """F^-1(g)(n) = (N1 N2 N3)^-1/2 sum_k g_k e^{-2 pi i k.N^-1 n} (eq:idft)."""
    V = int(np.prod(g.shape[-3:]))
    return np.fft.fftn(g, axes=(-3, -2, -1)) / np.sqrt(V)


def phase_a(N1, N2, N3):
    """a_k = e^{i pi k.N^-1 t} on k in N (eq:bcc-dft)."""
    k = np.meshgrid(np.arange(N1) / N1, np.arange(N2) / N2, np.arange(N3) / N3, indexing="ij")
    return np.exp(1j * np.pi * (k[0] + k[1] + k[2]))


def bcc_dft(f):
    """(hat f0, hat f1) of eq:bcc-dft as hat[2, s, N1, N2, N3]."""
    a = phase_a(*f.shape[-3:])
    F0 = rect_dft(f[0])
    F1 = rect_dft(f[1])
    return np.stack([(F0 - a * F1) / np.sqrt(2.0), (F0 + a * F1) / np.sqrt(2.0)])


def bcc_idft(h):
    """(f0, f1) of eq:bcc-idft from hat[2, s, N1, N2, N3]."""
    a = phase_a(*h.shape[-3:])
    f0 = rect_idft(h[0] + h[1]) / np.sqrt(2.0)
    f1 = rect_idft(np.conj(a) * (h[1] - h[0])) / np.sqrt(2.0)
    return np.stack([f0, f1])


def cartesian_table(m):
    """{Cartesian offset h: U_h} of the 3D Dirac walk: the transition
    matrices of the primitive-cell table at their Cartesian displacements."""
    H = walk.generators(3).astype(np.int64)
    out = {}
    for off, U in walk.stencil_table(3, m).items():
        h = tuple(int(v) for v in H @ np.array(off, dtype=np.int64))
        out[h] = U
    return out


def step_cartesian(fc, ctable):
    """One step psi(x) <- sum_h U_h psi(x+h) on the Cartesian (2N)^3 torus."""
    out = np.zeros_like(fc)
    for h, U in ctable.items():
        sh = np.roll(fc, shift=[-v for v in h], axis=(1, 2, 3))
        out += np.tensordot(U, sh, axes=(1, 0))
    return out


def symbol_cartesian(ctable, kappa):
    """U(kappa) = sum_h e^{-i kappa.h} U_h at Cartesian kappa[..., 3]."""
    kappa = np.asarray(kappa, dtype=np.float64)
    s = next(iter(ctable.values())).shape[0]
    out = np.zeros(kappa.shape[:-1] + (s, s), dtype=np.complex128)
    for h, U in ctable.items():
        ph = np.exp(-1j * (kappa @ np.array(h, dtype=np.float64)))
        out = out + ph[..., None, None] * U
    return out


def _power(D, t):
    if float(t) == int(t):
        return fourier.matpow(D, int(t))
    return fourier.matpow_real(D, t)


def evolve_cubic(f, m, t):
    """U^t f in the cubic-supercell representation, through the Cartesian
    embedding: DFT over the whole (2N)^3 Cartesian torus with the sign of
    Sec. 4, U(kappa)^t per wave-vector kappa = pi j / N (binary powering for
    integer t, the principal-logarithm interpolation of Sec. 4 for real t),
    inverse DFT, then the two sublattices. Independent of the two-sublattice
    reduction (mixed-parity sites stay zero because every offset h lies in G)."""
    fc = embed(f)
    Nc = fc.shape[1:]
    j = np.stack(np.meshgrid(*[np.arange(n) for n in Nc], indexing="ij"), axis=-1)
    kappa = 2.0 * np.pi * j / np.array(Nc, dtype=np.float64)
    Dt = _power(symbol_cartesian(cartesian_table(m), kappa), t)
    hat = np.fft.ifftn(fc, axes=(1, 2, 3)) * fc[0].size
    hat = fourier.apply_symbol(Dt, hat)
    return split(np.fft.fftn(hat, axes=(1, 2, 3)) / fc[0].size)


def evolve_two_sublattice(f, m, t):
    """U^t f by the paper's route: eq:bcc-dft, U(kappa)^t on hat f1 and
    U(kappa + pi e_x)^t on hat f0 (kappa = pi k / N), eq:bcc-idft."""
    N1, N2, N3 = f.shape[-3:]
    j = np.stack(np.meshgrid(np.arange(N1), np.arange(N2), np.arange(N3), indexing="ij"),
                 axis=-1)
    kappa = np.pi * j / np.array([N1, N2, N3], dtype=np.float64)
    ct = cartesian_table(m)
    D1 = _power(symbol_cartesian(ct, kappa), t)
    D0 = _power(symbol_cartesian(ct, kappa + np.array([np.pi, 0.0, 0.0])), t)
    h = bcc_dft(f)
    h = np.stack([fourier.apply_symbol(D0, h[0]), fourier.apply_symbol(D1, h[1])])
    return bcc_idft(h)


def observables_cubic(f, center):
    """Norm and Cartesian position moments of a cubic-supercell field about
    the Cartesian point c (Sec. 5.2 position expectation, minimum image on the
    torus of period 2 N_i): the plain reductions of the Cartesian embedding,
    whose grid indices are the Cartesian coordinates. Returns norm2, mean[3]
    (Cartesian) and second[6] (pairs 00, 11, 22, 01, 02, 12 about c)."""
    from . import observables as ob
    o = ob.observables(embed(f), center)
    return {"norm2": o["norm2"], "mean": o["mean"], "second": o["second"]}
