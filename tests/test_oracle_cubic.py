"""Pins of the cubic-supercell oracle (Sec. 4, eq:bcc-dft and eq:bcc-idft).

The two-sublattice transform is checked against the direct sum of the BCC
DFT's definition over the whole index set K; the Fourier evolution through
the Cartesian embedding against brute-force stepping on the Cartesian torus;
the paper's two-sublattice route against the embedding; and the cubic torus
against the primitive-cell torus on a localised state, inside the light cone
where neither torus wraps. No GPU.
"""
import numpy as np
import pytest

from oracle import cubic, observables as ob, stepper, walk


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return x / np.linalg.norm(x)


@pytest.mark.parametrize("N", [(2, 2, 2), (2, 4, 2), (4, 2, 4)])
def test_two_sublattice_dft_matches_the_definition_on_all_of_K(N):
    """eq:bcc-dft against the direct sum over B: for k in K write
    k = kk + N r with kk in N; then hat f_k is hat f1_kk / 2 when sum(r) is
    even and hat f0_kk / 2 when it is odd."""
    f = _rand((2, 4) + N, 11 + sum(N))
    direct = cubic.bcc_dft_direct(f)
    h = cubic.bcc_dft(f)
    N1, N2, N3 = N
    worst = 0.0
    for k1 in range(-N1, N1):
        for k2 in range(-N2, N2):
            for k3 in range(-N3, N3):
                r = [k1 // N1, k2 // N2, k3 // N3]
                kk = (k1 - r[0] * N1, k2 - r[1] * N2, k3 - r[2] * N3)
                sub = 1 if sum(r) % 2 == 0 else 0
                want = h[sub][(slice(None),) + kk] / 2.0
                got = direct[:, k1 + N1, k2 + N2, k3 + N3]
                worst = max(worst, np.abs(got - want).max())
    assert worst < 1e-13


@pytest.mark.parametrize("N", [(2, 4, 8), (8, 4, 2)])
def test_two_sublattice_dft_is_unitary_and_inverted_by_eq_bcc_idft(N):
    f = _rand((2, 4) + N, 21)
    h = cubic.bcc_dft(f)
    assert abs(np.linalg.norm(h) - 1.0) < 1e-13
    assert np.abs(cubic.bcc_idft(h) - f).max() < 1e-14


def test_sublattice_split_and_embedding():
    fc = np.zeros((4, 4, 8, 6), dtype=np.complex128)
    rng = np.random.default_rng(3)
    for x in np.ndindex(4, 8, 6):
        if x[0] % 2 == x[1] % 2 == x[2] % 2:
            fc[(slice(None),) + x] = rng.standard_normal(4)
    f = cubic.split(fc)
    assert f.shape == (2, 4, 2, 4, 3)
    assert f[1, 2, 1, 3, 2] == fc[2, 3, 7, 5]
    assert np.array_equal(cubic.embed(f), fc)


def test_cartesian_offsets_are_bcc_neighbours():
    """The walk connects each site to itself (mass term) and to the eight
    Cartesian neighbours (+-1, +-1, +-1) (Sec. 3.1 generators and h4)."""
    ct = cubic.cartesian_table(0.3)
    want = {(0, 0, 0)} | {(a, b, c) for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)}
    assert set(ct) <= want
    assert {h for h in want if h != (0, 0, 0)} <= set(ct)
    assert set(cubic.cartesian_table(0.0)) == {h for h in want if h != (0, 0, 0)}


@pytest.mark.parametrize("m", [0.0, 0.3, 1.0])
def test_embedding_evolution_equals_cartesian_steps(m):
    """Fourier evolution on the (2N)^3 Cartesian torus against t steps of the
    update rule with the Cartesian offsets (brute force)."""
    f = _rand((2, 4, 2, 4, 4), 31)
    ct = cubic.cartesian_table(m)
    fc = cubic.embed(f)
    for t in range(4):
        got = cubic.evolve_cubic(f, m, t)
        assert np.abs(got - cubic.split(fc)).max() < 1e-13, t
        fc = cubic.step_cartesian(fc, ct)
        # the walk never populates mixed-parity sites
        assert np.abs(fc - cubic.embed(cubic.split(fc))).max() == 0.0


@pytest.mark.parametrize("m,t", [(0.0, 3), (0.2, 5), (0.2, -4), (1.0, 2), (0.37, 2.6),
                                 (0.0, 0.5)])
def test_two_sublattice_route_equals_the_embedding(m, t):
    """The paper's route (eq:bcc-dft, per-frequency powers at kappa and
    kappa + pi e_x, eq:bcc-idft) against the embedding, integer and real t."""
    f = _rand((2, 4, 4, 2, 8), 41)
    a = cubic.evolve_two_sublattice(f, m, t)
    b = cubic.evolve_cubic(f, m, t)
    assert np.abs(a - b).max() < 1e-12
    if m > 0 or float(t) == int(t):
        # (at m = 0 the band edge takes the average cos(pi t), not unitary)
        assert abs(np.linalg.norm(a) - 1.0) < 1e-12


@pytest.mark.parametrize("m", [0.0, 0.4])
def test_cubic_and_primitive_tori_agree_inside_the_light_cone(m):
    """A state localised at the origin, stepped t times on the primitive-cell
    torus and on the cubic torus: the two agree site by site (Cartesian
    x = H n) while the support stays clear of both periodic boundaries."""
    t = 3
    Np = 16
    zeta = np.array([0.6, 0.2j, -0.5, 0.3 + 0.4j]) / np.linalg.norm([0.6, 0.2j, -0.5, 0.3 + 0.4j])
    prim = np.zeros((4, Np, Np, Np), dtype=np.complex128)
    prim[:, 0, 0, 0] = zeta
    prim = stepper.evolve_steps(prim, walk.stencil_table(3, m), t)
    fc = np.zeros((4, 16, 16, 16), dtype=np.complex128)
    fc[:, 0, 0, 0] = zeta
    ct = cubic.cartesian_table(m)
    for _ in range(t):
        fc = cubic.step_cartesian(fc, ct)
    H = walk.generators(3).astype(np.int64)
    mapped = np.zeros_like(fc)
    for n in np.ndindex(Np, Np, Np):
        v = prim[(slice(None),) + n]
        if not np.any(v):
            continue
        nc = np.array([(a + Np // 2) % Np - Np // 2 for a in n])
        x = H @ nc
        assert np.all(np.abs(x) <= t)
        mapped[(slice(None),) + tuple(x % 16)] = v
    assert np.abs(mapped - fc).max() < 1e-14
    assert abs(np.linalg.norm(fc) - 1.0) < 1e-13


def test_cubic_observables_by_brute_force():
    """Norm and moments summed site by site over both sublattices."""
    N = (2, 4, 4)
    f = _rand((2, 4) + N, 91)
    c = np.array([1.3, 6.0, 2.5])
    got = cubic.observables_cubic(f, c)
    L = 2 * np.array(N)
    tot, s1, s2 = 0.0, np.zeros(3), np.zeros((3, 3))
    for j in (0, 1):
        for m in np.ndindex(*N):
            x = 2 * np.array(m) + j
            w = np.mod(x - c + L / 2, L) - L / 2
            p = float(np.sum(np.abs(f[(j, slice(None)) + m]) ** 2))
            tot += p
            s1 += w * p
            s2 += np.outer(w, w) * p
    assert abs(got["norm2"] - tot) < 1e-13
    assert np.allclose(got["mean"], c + s1 / tot, atol=1e-12)
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    assert np.allclose(got["second"], [s2[i, j] / tot for i, j in pairs], atol=1e-12)


def test_cubic_observables_equal_the_primitive_torus_ones_inside_the_light_cone():
    """A localised state stepped on both tori: the Cartesian mean and the
    Cartesian second moments (H S H^T of the primitive ones) agree."""
    t, Np, m = 3, 16, 0.3
    zeta = np.array([0.6, 0.2j, -0.5, 0.3 + 0.4j])
    zeta = zeta / np.linalg.norm(zeta)
    prim = np.zeros((4, Np, Np, Np), dtype=np.complex128)
    prim[:, 8, 8, 8] = zeta
    prim = stepper.evolve_steps(prim, walk.stencil_table(3, m), t)
    op = ob.observables(prim, [8, 8, 8])
    fc = np.zeros((4, 16, 16, 16), dtype=np.complex128)
    fc[:, 0, 0, 0] = zeta
    ct = cubic.cartesian_table(m)
    for _ in range(t):
        fc = cubic.step_cartesian(fc, ct)
    oc = cubic.observables_cubic(cubic.split(fc), [0.0, 0.0, 0.0])
    H = walk.generators(3)
    assert np.allclose(oc["mean"], H @ (op["mean"] - 8.0), atol=1e-12)
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    S = np.zeros((3, 3))
    for k, (i, j) in enumerate(pairs):
        S[i, j] = S[j, i] = op["second"][k]
    Sc = H @ S @ H.T
    assert np.allclose(oc["second"], [Sc[i, j] for i, j in pairs], atol=1e-12)
