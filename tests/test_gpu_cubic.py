"""GPU parity of the cubic-supercell BCC path (Sec. 4, eq:bcc-dft and
eq:bcc-idft) through the C ABI: qw_bcc_transform against the oracle's
two-sublattice DFT, qw_bcc_evolve_fft against the oracle's evolution through
the Cartesian embedding (which does not use the two-sublattice reduction),
and the cubic torus against the primitive-cell torus, both on the GPU, on a
localised state inside the light cone."""
import numpy as np
import pytest
import torch

from oracle import cubic, observables as ob, walk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1603_06442_amd import qw as mod
    return mod


def to_dev(x, plan):
    return torch.from_numpy(np.ascontiguousarray(x)).to(plan.torch_dtype).cuda()


def to_np(x):
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.complex128)


def tol_fft(dtype, t):
    return 2e-5 if dtype == "c64" else max(1e-12, 1e-15 * abs(t))


def rand_sub(N, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((2, 4) + N) + 1j * rng.standard_normal((2, 4) + N)
    return f / np.linalg.norm(f)


SHAPES = [(2, 2, 2), (4, 8, 16), (16, 16, 16), (8, 4, 32), (2, 16, 4), (4, 4, 128), (2, 2, 512)]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("N", SHAPES)
def test_bcc_transform_matches_oracle(qw, N, dtype):
    f = rand_sub(N, 5 + sum(N))
    plan = qw.Plan(3, list(N), 0.2, dtype)
    x = to_dev(f, plan)
    h = plan.bcc_transform(x, +1)
    tol = 1e-6 if dtype == "c64" else 1e-13
    assert ob.rel_l2(to_np(h), cubic.bcc_dft(f)) < tol
    back = plan.bcc_transform(h, -1)
    assert ob.rel_l2(to_np(back), f) < tol
    # the inverse alone, on a spectrum from the oracle
    g = rand_sub(N, 77)
    inv = plan.bcc_transform(to_dev(g, plan), -1)
    assert ob.rel_l2(to_np(inv), cubic.bcc_idft(g)) < tol


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("N", [(2, 2, 2), (4, 4, 8), (8, 8, 8), (16, 8, 32), (4, 2, 64),
                               (2, 2, 512)])
@pytest.mark.parametrize("t", [0, 1, 5, -3, 1000, 100000])
def test_bcc_evolve_matches_oracle(qw, N, t, dtype):
    m = 0.21
    f = rand_sub(N, 300 + sum(N))
    plan = qw.Plan(3, list(N), m, dtype)
    out = plan.bcc_evolve_fft(to_dev(f, plan), t)
    ref = cubic.evolve_cubic(f, m, t)
    assert ob.rel_l2(to_np(out), ref) < tol_fft(dtype, t)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("m,t", [(0.0, 7), (1.0, 3), (0.0, 0.5), (0.37, 2.6), (0.05, -11.25)])
def test_bcc_evolve_degenerate_masses_and_real_t(qw, m, t, dtype):
    """m = 0 (massless, with the band edge at kappa = 0 + pi e_x), m = 1 (no
    hopping) and real t (the principal-logarithm interpolation of Sec. 4)."""
    N = (8, 4, 16)
    f = rand_sub(N, 41)
    plan = qw.Plan(3, list(N), m, dtype)
    out = plan.bcc_evolve_fft(to_dev(f, plan), t)
    ref = cubic.evolve_cubic(f, m, t)
    assert ob.rel_l2(to_np(out), ref) < tol_fft(dtype, t)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_bcc_evolve_in_place_and_reversible(qw, dtype):
    N = (16, 16, 32)
    f = rand_sub(N, 9)
    plan = qw.Plan(3, list(N), 0.3, dtype)
    x = to_dev(f, plan)
    plan.bcc_evolve_fft(x, 123, out=x)
    norm = torch.linalg.vector_norm(x).item()
    assert abs(norm - 1.0) < (1e-5 if dtype == "c64" else 1e-13)
    plan.bcc_evolve_fft(x, -123, out=x)
    assert ob.rel_l2(to_np(x), f) < (4e-6 if dtype == "c64" else 1e-13)


def _delta_pair(qw, Np, Nc, t, m, dtype):
    """Evolve the same localised state on the primitive-cell torus (Np^3) and
    on the cubic torus (sublattice arrays Nc^3) on the GPU; return the
    Cartesian window |x_i| <= t of both, and the norm each holds there."""
    zeta = np.array([0.6, 0.2j, -0.5, 0.3 + 0.4j])
    zeta = zeta / np.linalg.norm(zeta)
    pp = qw.Plan(3, [Np] * 3, m, dtype)
    prim = torch.zeros((4, Np, Np, Np), dtype=pp.torch_dtype, device="cuda")
    prim[:, 0, 0, 0] = torch.from_numpy(zeta).to(pp.torch_dtype)
    prim = pp.evolve_fft(prim, t)
    cp = qw.Plan(3, [Nc] * 3, m, dtype)
    cub = torch.zeros((2, 4, Nc, Nc, Nc), dtype=cp.torch_dtype, device="cuda")
    cub[0, :, 0, 0, 0] = torch.from_numpy(zeta).to(cp.torch_dtype)
    cub = cp.bcc_evolve_fft(cub, t)
    # Cartesian sites of G in the window, and their indices on both tori
    r = np.arange(-t, t + 1)
    X = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    X = X[(X[:, 0] % 2 == X[:, 1] % 2) & (X[:, 1] % 2 == X[:, 2] % 2)]
    Hinv = np.linalg.inv(walk.generators(3))
    n = np.rint(X @ Hinv.T).astype(np.int64) % Np
    sub = X[:, 0] % 2
    mm = ((X - sub[:, None]) // 2) % Nc
    dev = lambda a: torch.from_numpy(a).cuda()
    pv = prim[:, dev(n[:, 0]), dev(n[:, 1]), dev(n[:, 2])]
    cv = cub[dev(sub), :, dev(mm[:, 0]), dev(mm[:, 1]), dev(mm[:, 2])].T
    return to_np(pv), to_np(cv)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("m", [0.0, 0.4])
def test_cubic_and_primitive_tori_agree_on_the_gpu(qw, m, dtype):
    """Two independent GPU paths on one localised state: the window holds the
    whole state on both tori and the values agree site by site."""
    t = 20
    pv, cv = _delta_pair(qw, 64, 32, t, m, dtype)
    tol = 2e-5 if dtype == "c64" else 1e-12
    assert abs(np.linalg.norm(pv) - 1.0) < tol
    assert abs(np.linalg.norm(cv) - 1.0) < tol
    assert ob.rel_l2(cv, pv) < tol


def test_bcc_rejects_other_dimensions(qw):
    plan = qw.Plan(2, [8, 8], 0.2, "c64")
    x = torch.zeros((2, 4, 8, 8), dtype=torch.complex64, device="cuda")
    import ctypes
    p = ctypes.c_void_p(x.data_ptr())
    assert qw.LIB.qw_bcc_transform(plan._h, p, p, 1, None) == qw.QW_ERR_UNSUPPORTED
    assert qw.LIB.qw_bcc_evolve_fft(plan._h, p, p, 1.0, None) == qw.QW_ERR_UNSUPPORTED
    plan3 = qw.Plan(3, [4, 4, 4], 0.2, "c64")
    y = torch.zeros((2, 4, 4, 4, 4), dtype=torch.complex64, device="cuda")
    q = ctypes.c_void_p(y.data_ptr())
    assert qw.LIB.qw_bcc_transform(plan3._h, q, q, 0, None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_bcc_evolve_fft(plan3._h, q, q, float("inf"), None) == qw.QW_ERR_UNSUPPORTED


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_bcc_capture_into_a_graph(qw, dtype):
    """qw_bcc_evolve_fft, qw_bcc_transform and qw_bcc_step, called once
    beforehand (the plan builds its omega table and stepping scratch then),
    captured into a HIP graph: every replay, with eager work and
    synchronisations between replays, gives bitwise the eager result (the
    steps run the LDS-tiled kernel at complex64, the marching one at
    complex128)."""
    N = (16, 8, 64)
    plan = qw.Plan(3, list(N), 0.11, dtype)
    f0 = to_dev(rand_sub(N, 13), plan)
    a = plan.bcc_evolve_fft(f0, 29)
    h = plan.bcc_transform(a, +1)
    st = f0.clone()
    plan.bcc_step(st, 3)
    torch.cuda.synchronize()
    want_a, want_h, want_s = a.clone(), h.clone(), st.clone()
    ga, gh, gs = torch.empty_like(f0), torch.empty_like(f0), f0.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.bcc_evolve_fft(f0, 29, out=ga, stream=side)
        plan.bcc_transform(ga, +1, out=gh, stream=side)
        plan.bcc_step(f0.clone(), 3, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        s = torch.cuda.current_stream()
        plan.bcc_evolve_fft(f0, 29, out=ga, stream=s)
        plan.bcc_transform(ga, +1, out=gh, stream=s)
        plan.bcc_step(gs, 3, stream=s)
    for r in range(3):
        ga.zero_()
        gh.zero_()
        gs.copy_(f0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ga, want_a), r
        assert torch.equal(gh, want_h), r
        assert torch.equal(gs, want_s), r
        e = plan.bcc_evolve_fft(f0, 3)  # eager work between replays
        torch.cuda.synchronize()
        del e


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("threads", [64, 128, 256, 512])
def test_bcc_evolve_under_every_schedule(qw, dtype, threads):
    """The cubic-supercell passes follow the plan's workgroup size (the
    autotuner picks 64, 128 or 256 threads, a caller may set 512; a team
    wider than that runs one pencil per workgroup); the slab schedule of the
    primitive path does not apply to them. Same results as the oracle under
    each."""
    N = (16, 8, 64)
    m, t = 0.13, 77
    f = rand_sub(N, 61)
    plan = qw.Plan(3, list(N), m, dtype)
    plan.set_schedule(4, 8, threads, 1)
    out = plan.bcc_evolve_fft(to_dev(f, plan), t)
    ref = cubic.evolve_cubic(f, m, t)
    assert ob.rel_l2(to_np(out), ref) < tol_fft(dtype, t)
    plan.autotune()
    out2 = plan.bcc_evolve_fft(to_dev(f, plan), t)
    assert ob.rel_l2(to_np(out2), ref) < tol_fft(dtype, t)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("N", [(2, 2, 2), (4, 8, 16), (8, 4, 32), (2, 4, 64), (4, 4, 64),
                               (16, 4, 64), (8, 8, 128)])
@pytest.mark.parametrize("m", [0.0, 0.3, 1.0])
def test_bcc_step_matches_oracle(qw, N, m, dtype):
    """Position-space steps on the two sublattice arrays against the oracle's
    Cartesian stepping of the embedded field (odd and even step counts). The
    shapes with at least 4 x 64 sites per plane of axis 0 take the LDS-tiled
    kernel at complex64 (one tile per plane at 2 x 4 x 64, so its halos wrap
    onto the tile itself; several chunks of planes at 16 x 4 x 64)."""
    f = rand_sub(N, 71 + sum(N))
    plan = qw.Plan(3, list(N), m, dtype)
    x = to_dev(f, plan)
    ct = cubic.cartesian_table(m)
    fc = cubic.embed(f)
    done = 0
    for k in (1, 4):
        plan.bcc_step(x, k)
        for _ in range(k):
            fc = cubic.step_cartesian(fc, ct)
        done += k
        tol = max(2e-5, 4 * done * 2.0 ** -24) if dtype == "c64" else 1e-12
        assert ob.rel_l2(to_np(x), cubic.split(fc)) < tol


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_bcc_jump_equals_steps_on_the_gpu(qw, dtype):
    """Sec. 4's two routes on the cubic supercell agree on the GPU: t
    position-space steps and one Fourier jump to t."""
    N = (16, 8, 32)
    f = rand_sub(N, 83)
    plan = qw.Plan(3, list(N), 0.17, dtype)
    x = to_dev(f, plan)
    jump = plan.bcc_evolve_fft(x, 9)
    plan.bcc_step(x, 9)
    tol = 4e-5 if dtype == "c64" else 1e-12
    assert ob.rel_l2(to_np(x), to_np(jump)) < tol


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("N", [(2, 2, 2), (4, 8, 16), (8, 4, 32), (2, 2, 512)])
@pytest.mark.parametrize("origin", [(0.0, 0.0, 0.0), (3.0, 5.5, 1.25)])
def test_bcc_observables_match_oracle(qw, N, origin, dtype):
    """Norm and Cartesian moments about a Cartesian origin (integer and not)
    on the period-2N torus, against the oracle's reductions of the Cartesian
    embedding."""
    f = rand_sub(N, 101 + sum(N))
    plan = qw.Plan(3, list(N), 0.2, dtype)
    got = plan.bcc_observables(to_dev(f, plan), origin)
    if dtype == "c64":
        f = f.astype(np.complex64).astype(np.complex128)
    want = cubic.observables_cubic(f, origin)
    assert abs(got["norm2"] - want["norm2"]) < 1e-12
    assert np.allclose(got["mean"], want["mean"], atol=1e-10)
    assert np.allclose(got["second"], want["second"], atol=1e-9)
