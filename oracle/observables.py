"""Reductions on a field (test infrastructure).

* Position: X = sum_x x |x><x| (x) I and <psi|X|psi> (Sec. 5.2). On the N^d
  torus X is taken about a caller origin c with the minimum image
  w = ((n - c + N/2) mod N) - N/2 in [-N/2, N/2) per primitive axis
  (reading: valid while the support stays within c +- N/2).
* Overlap <phi|psi> and fidelity |<phi|psi>| / (|phi| |psi|), as in the
  overlap bound of Sec. 5.1.
* The drift law of Sec. 5.1 (second-order equation, drift v = grad omega)
  and the mean-position decomposition of Sec. 5.2 (classical drift of each
  sector plus the particle/antiparticle interference term), evaluated
  exactly in k-space.
"""
import numpy as np

from . import fourier, states, walk

PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def min_image(N, d, center):
    """w[d, N_1..N_d]: per-axis minimum-image displacement of every site from c."""
    Ns = (int(N),) * d if np.isscalar(N) else tuple(int(x) for x in N)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in Ns], indexing="ij")
    c = np.asarray(center, dtype=np.float64).reshape(d)
    return np.stack([np.mod(g - c[i] + Ns[i] / 2.0, Ns[i]) - Ns[i] / 2.0
                     for i, g in enumerate(grids)])


def observables(psi, center, ref=None):
    """Norm, position moments about c (primitive and Cartesian), overlap."""
    d = psi.ndim - 1
    p = np.sum(np.abs(psi) ** 2, axis=0)
    norm2 = float(np.sum(p))
    w = min_image(psi.shape[1:], d, center)
    c = np.asarray(center, dtype=np.float64).reshape(d)
    mean = np.zeros(3)
    second = np.zeros(6)
    for i in range(d):
        mean[i] = c[i] + float(np.sum(w[i] * p)) / norm2
    for k, (i, j) in enumerate(PAIRS):
        if i < d and j < d:
            second[k] = float(np.sum(w[i] * w[j] * p)) / norm2
    mean_cart = np.zeros(3)
    mean_cart[:d] = walk.generators(d) @ mean[:d]
    out = {"norm2": norm2, "mean": mean, "second": second, "mean_cart": mean_cart,
           "overlap": 0j, "ref_norm2": 0.0}
    if ref is not None:
        out["overlap"] = complex(np.vdot(ref.reshape(-1), psi.reshape(-1)))
        out["ref_norm2"] = float(np.sum(np.abs(ref) ** 2))
    return out


def fidelity(phi, psi):
    return abs(np.vdot(phi.reshape(-1), psi.reshape(-1))) / np.sqrt(
        np.sum(np.abs(phi) ** 2) * np.sum(np.abs(psi) ** 2))


def rel_l2(a, b):
    """|a - b|_2 / |b|_2 over all entries (no phase alignment)."""
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))


def omega_and_grad(table, N, d):
    """omega(q) and grad_q omega(q) on the DFT grid from the U_h table.

    cos(omega) = Re tr(U_q)/s and d cos(omega)/dq_j = Re tr(dU_q/dq_j)/s with
    dU_q/dq_j = sum_h (-i h_j) e^{-iq.h} U_h; sin(omega) is the column norm of
    M = i(U_q - cos(omega) I). Returns (omega[N..N], grad[N..N, d]).
    """
    q = walk.lattice_q(N, d)
    s = next(iter(table.values())).shape[0]
    D = walk.symbol_from_table(table, q)
    cosw = np.real(np.trace(D, axis1=-2, axis2=-1)) / s
    M = 1j * (D - cosw[..., None, None] * np.eye(s))
    sinw = np.sqrt(np.sum(np.abs(M[..., :, 0]) ** 2, axis=-1))
    omega = np.arctan2(sinw, cosw)
    grad = np.zeros(q.shape, dtype=np.float64)
    for off, U in table.items():
        ph = np.exp(-1j * (q @ np.array(off, dtype=np.float64)))
        trU = np.trace(U)
        for j in range(d):
            grad[..., j] += np.real(-1j * off[j] * ph * trU) / s
    grad = -grad / sinw[..., None]
    return omega, grad


def drift_prediction(psi, table, t):
    """<n>(t) - <n>(0) = -t sum_q grad omega (|P+ psi^|^2 - |P- psi^|^2)/|psi^|^2.

    The drift term of the mean position for each frequency sector (Sec. 5.1,
    drift vector; Sec. 5.2, classical part of the mean position). Packets
    drift along -grad omega with the Fourier sign of Sec. 2.1 and Sec. 4.
    Returns a length-d vector in primitive coordinates.
    """
    d = psi.ndim - 1
    N = psi.shape[1:]
    _, grad = omega_and_grad(table, N, d)
    phat = fourier.dft(psi)
    Pp, Pm = states.sector_projectors(walk.symbol_from_table(table, walk.lattice_q(N, d)))
    pp = fourier.apply_symbol(Pp, phat)
    pm = fourier.apply_symbol(Pm, phat)
    wgt = np.sum(np.abs(pp) ** 2, axis=0) - np.sum(np.abs(pm) ** 2, axis=0)
    tot = np.sum(np.abs(phat) ** 2)
    return -t * np.array([np.sum(grad[..., j] * wgt) for j in range(d)]) / tot


def mean_position_kspace(psi, table, center, times, parts=False):
    """<n>(t) for a two-sector state, exactly in k-space (Sec. 5.2).

    With hat psi_+- = P_+- hat psi at t = 0 the evolved field is
    e^{-i omega t} hat psi_+ + e^{+i omega t} hat psi_-. The mean position
    about c splits into <n>(0), the drift -t sum grad omega (|psi_+|^2 -
    |psi_-|^2), and the interference term x_int(t) - x_int(0) with
    x_int(t) = 2 Re sum_q e^{2 i omega t} hat psi_+^dag (-i grad hat psi_-),
    where -i grad hat psi_- is the DFT of w(n) psi_-(n). Exact on the torus up
    to the weight the packet has near the wrap (reading of Sec. 5.2 on a
    torus). Returns <n>(t)[len(times), d] in primitive coordinates; with
    ``parts`` also the drift per step and x_int(t)[len(times), d].
    """
    d = psi.ndim - 1
    N = psi.shape[1:]
    V = int(np.prod(N))
    omega, grad = omega_and_grad(table, N, d)
    phat = fourier.dft(psi)
    Pp, Pm = states.sector_projectors(walk.symbol_from_table(table, walk.lattice_q(N, d)))
    pp = fourier.apply_symbol(Pp, phat)
    pm = fourier.apply_symbol(Pm, phat)
    psim = fourier.idft(pm)
    w = min_image(N, d, center)
    norm2 = float(np.sum(np.abs(psi) ** 2))
    base = observables(psi, center)["mean"][:d]
    wdiff = np.sum(np.abs(pp) ** 2, axis=0) - np.sum(np.abs(pm) ** 2, axis=0)
    drift = np.array([np.sum(grad[..., j] * wdiff) for j in range(d)]) / V / norm2
    xg = [np.sum(np.conj(pp) * fourier.dft(w[j][None] * psim), axis=0) for j in range(d)]

    def xint(t):
        ph = np.exp(2j * omega * t)
        return np.array([2.0 * np.real(np.sum(ph * xg[j])) for j in range(d)]) / V / norm2

    x0 = xint(0)
    mean = np.array([base - t * drift + xint(t) - x0 for t in times])
    if parts:
        return mean, drift, np.array([xint(t) for t in times])
    return mean


def newton_wigner(psi, table, center):
    """Mean position without the interference of the two frequency sectors
    (the Newton-Wigner position of the closing remark of Sec. 5.2, read
    gauge-free): psi is split into its sector parts P+- psi (spectral
    projectors of U_q applied to hat psi), each part's reductions are taken
    about c as in ``observables``, and the means are combined with the
    sector weights. Returns (mean[3], mean_cart[3], (obs_plus, obs_minus))."""
    d = psi.ndim - 1
    N = psi.shape[1:]
    Pp, Pm = states.sector_projectors(walk.symbol_from_table(table, walk.lattice_q(N, d)))
    phat = fourier.dft(psi)
    parts = [observables(fourier.idft(fourier.apply_symbol(P, phat)), center) for P in (Pp, Pm)]
    wsum = parts[0]["norm2"] + parts[1]["norm2"]
    mean = (parts[0]["norm2"] * np.asarray(parts[0]["mean"]) +
            parts[1]["norm2"] * np.asarray(parts[1]["mean"])) / wsum
    H = walk.generators(d)
    mean_cart = np.zeros(3)
    mean_cart[:d] = H @ mean[:d]
    return mean, mean_cart, parts


def marginals(psi, center):
    """Probability marginals along the Cartesian axes (the projections of
    the figures of Sec. 5.2): every site n contributes |psi(n)|^2 to bin
    X_i = (H w)_i of axis i, w the minimum image of n - c (integer c).
    Returns a list of d (xmin, values) pairs, values[b] at X_i = xmin + b."""
    d = psi.ndim - 1
    N = psi.shape[1:]
    p = np.sum(np.abs(psi) ** 2, axis=0)
    w = np.rint(min_image(N, d, center)).astype(np.int64)  # [d, N...]
    H = walk.generators(d).astype(np.int64)
    out = []
    for i in range(d):
        X = np.tensordot(H[i], w, axes=(0, 0))
        lo = sum(-(N[j] // 2) if H[i, j] > 0 else -(N[j] // 2 - 1) for j in range(d) if H[i, j] != 0)
        hi = sum(N[j] // 2 - 1 if H[i, j] > 0 else N[j] // 2 for j in range(d) if H[i, j] != 0)
        vals = np.bincount((X - lo).ravel(), weights=p.ravel(), minlength=hi - lo + 1)
        out.append((lo, vals))
    return out
