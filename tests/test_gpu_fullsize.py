"""Parity at the full sizes of the timed workloads, in the launch
configuration the benchmark uses (the autotuned Fourier schedule).

256^3 complex64 (the headline workload): the GPU stencil and the GPU Fourier
jump are compared with the FP64 oracle's position-space steps on the whole
field (two steps: about 16 s of host time), the fused reductions with the
oracle's reductions of that field, and the evolution is checked to be
reversible at t = 1e5. 512^3 (the large workload): complex64 against
complex128 at t = 1e6 and the Fourier jump against a stencil step, on the
whole field. The Weyl walk on the 256^3 lattice and the cubic supercell of
two 256^3 sublattice arrays: a localised state against the oracle on a small
torus that holds the whole light cone."""
import numpy as np
import pytest
import torch

from oracle import observables as ob, stepper, walk
from paper_1603_06442_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1603_06442_amd import qw as mod
    return mod


def rel(a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def test_bcc256_c64_against_oracle_steps(qw):
    w = inputs.workload(2)
    plan = qw.Plan(3, w["N"], w["m"], "c64")
    x = plan.empty()
    plan.prepare_state(x, w["k0"], w["sigma"], w["center"], w["c_plus"], w["c_minus"])
    plan.autotune()
    torch.cuda.synchronize()
    psi0 = x.cpu().numpy().astype(np.complex128)
    ref = stepper.evolve_steps(psi0, walk.stencil_table(3, w["m"]), 2)
    # stencil
    y = x.clone()
    plan.step(y, 2)
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.complex128)
    assert ob.rel_l2(got, ref) < 2e-5
    del got, y
    # Fourier jump with the fused reductions
    z = plan.empty()
    o = plan.evolve_fft_observables(x, 2, w["center"], out=z)
    torch.cuda.synchronize()
    got = z.cpu().numpy().astype(np.complex128)
    assert ob.rel_l2(got, ref) < 2e-5
    want = ob.observables(ref, w["center"])
    assert abs(o["norm2"] - want["norm2"]) < 1e-5
    assert np.allclose(o["mean"], want["mean"], rtol=0, atol=1e-4)
    assert np.allclose(o["mean_cart"], want["mean_cart"], rtol=0, atol=1e-4)
    assert np.allclose(o["second"], want["second"], rtol=1e-4, atol=1e-3)


def test_bcc256_c64_reversible_at_large_t(qw):
    w = inputs.workload(2)
    plan = qw.Plan(3, w["N"], w["m"], "c64")
    x = plan.empty()
    plan.prepare_state(x, w["k0"], w["sigma"], w["center"], w["c_plus"], w["c_minus"])
    plan.autotune()
    t = 100000
    y = plan.evolve_fft(x, t)
    back = plan.evolve_fft(y, -t)
    assert rel(back, x) < 2e-5
    o = plan.evolve_fft_observables(x, t, w["center"])
    assert abs(o["norm2"] - 1.0) < 2e-5


def test_bcc128_jump_at_t_1e5_against_oracle(qw):
    """The headline workload's state on the 128^3 torus (width scaled to 10
    cells) jumped to the last time of its schedule, t = 1e5, in both
    precisions, against the oracle's binary powering of the summed symbol
    (about 15 s of host time), with the fused reductions."""
    from oracle import fourier, states
    w = inputs.workload(2)
    N, t = 128, w["times"][-1]
    c = [N // 2] * 3
    psi0 = states.particle_state(3, N, w["m"], w["k0"], w["sigma"] * N / w["N"], c,
                                 w["c_plus"], w["c_minus"])
    ref = fourier.evolve_fourier(psi0, walk.stencil_table(3, w["m"]), t)
    want = ob.observables(ref, c)
    for dtype, tol in (("c64", 2e-5), ("c128", 1e-15 * t)):
        plan = qw.Plan(3, N, w["m"], dtype)
        plan.autotune()
        x = torch.from_numpy(np.ascontiguousarray(psi0)).to(plan.torch_dtype).cuda()
        y = plan.empty()
        o = plan.evolve_fft_observables(x, t, c, out=y)
        torch.cuda.synchronize()
        e = ob.rel_l2(y.cpu().numpy().astype(np.complex128), ref)
        print("128^3 %s at t = %d: rel-L2 %.3e" % (dtype, t, e))
        assert e < tol
        assert np.allclose(o["mean"], want["mean"], rtol=0, atol=N * tol)
        assert abs(o["norm2"] - 1.0) < (1e-5 if dtype == "c64" else 1e-12)
        del plan, x, y


def test_bcc512_c64_vs_c128_and_jump_vs_step(qw):
    w = inputs.workload(4)
    N = w["N"]
    p64 = qw.Plan(3, N, w["m"], "c64")
    p128 = qw.Plan(3, N, w["m"], "c128")
    x128 = p128.empty()
    p128.prepare_state(x128, w["k0"], w["sigma"], w["center"], w["c_plus"], w["c_minus"])
    x64 = x128.to(torch.complex64)
    t = w["t"]
    y128 = p128.evolve_fft(x128, t)
    y64 = p64.evolve_fft(x64, t)
    assert rel(y64.to(torch.complex128), y128) < 2e-5
    assert abs(float(torch.linalg.vector_norm(y128)) ** 2 - 1.0) < 1e-9
    del y128, y64
    # one Fourier jump t = 1 against one stencil step (independent kernels)
    s = x128.clone()
    p128.step(s, 1)
    j = p128.evolve_fft(x128, 1)
    assert rel(j, s) < 1e-12


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_max_1d_lattice_against_oracle(qw, dtype):
    """The largest 1D lattice (N = 65536: four-step transform with the
    reductions fused into its strided pass) at t = 1e5 against the oracle."""
    from oracle import fourier, states
    N, m = 65536, 0.1
    psi = states.particle_state(1, N, m, [0.3], 200.0, [N // 2], 1 / np.sqrt(2), 1 / np.sqrt(2))
    plan = qw.Plan(1, N, m, dtype)
    x = torch.from_numpy(np.ascontiguousarray(psi)).to(plan.torch_dtype).cuda()
    t = 100000
    y = plan.empty()
    o = plan.evolve_fft_observables(x, t, [N // 2], out=y)
    torch.cuda.synchronize()
    ref = fourier.evolve_fourier(psi, walk.stencil_table(1, m), t)
    got = y.cpu().numpy().astype(np.complex128)
    tol = 2e-5 if dtype == "c64" else 1e-10
    assert ob.rel_l2(got, ref) < tol
    want = ob.observables(ref, [N // 2])
    assert abs(o["mean"][0] - want["mean"][0]) < tol * N


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_max_2d_lattice_against_oracle(qw, dtype):
    """The largest 2D lattice (1024 x 1024; the first axis is too long for
    the fused reduction): Fourier jump and three stencil steps against the
    oracle."""
    from oracle import fourier, states
    N, m = 1024, 0.2
    psi = states.particle_state(2, N, m, [0.2, -0.1], 30.0, [N // 2] * 2)
    tab = walk.stencil_table(2, m)
    plan = qw.Plan(2, N, m, dtype)
    x = torch.from_numpy(np.ascontiguousarray(psi)).to(plan.torch_dtype).cuda()
    tol = 2e-5 if dtype == "c64" else 1e-11
    y = plan.evolve_fft(x, 1000)
    assert ob.rel_l2(y.cpu().numpy().astype(np.complex128), fourier.evolve_fourier(psi, tab, 1000)) < tol
    s = x.clone()
    plan.step(s, 3)
    assert ob.rel_l2(s.cpu().numpy().astype(np.complex128), stepper.evolve_steps(psi, tab, 3)) < tol


def test_weyl256_c64_localised_state_against_oracle(qw):
    """The Weyl walk on the 256^3 workload lattice (complex64), stencil and
    Fourier jump: a state localised at the centre, after 12 steps, against
    the oracle's steps on a 32^3 torus (the light cone fits); the rest of
    the 256^3 field stays zero up to rounding."""
    N, t, c = 256, 12, 128
    zeta = np.array([0.8, 0.6j])
    plan = qw.Plan(3, N, 0.0, "c64", weyl=True)
    x = torch.zeros((2, N, N, N), dtype=torch.complex64, device="cuda")
    x[:, c, c, c] = torch.from_numpy(zeta).to(torch.complex64)
    y = plan.evolve_fft(x, t)
    plan.step(x, t)
    small = np.zeros((2, 32, 32, 32), dtype=np.complex128)
    small[:, 0, 0, 0] = zeta
    ref = stepper.evolve_steps(small, walk.weyl_table(3), t)
    for field in (x, y):
        torch.cuda.synchronize()
        win = field[:, c - t:c + t + 1, c - t:c + t + 1, c - t:c + t + 1].cpu().numpy()
        r = np.arange(-t, t + 1) % 32
        want = ref[np.ix_([0, 1], r, r, r)]
        assert ob.rel_l2(win.astype(np.complex128), want) < 2e-5
        assert abs(float(torch.linalg.vector_norm(field)) - 1.0) < 2e-5


def test_cubic256_c64_localised_state_against_oracle(qw):
    """The cubic supercell at the timed size (two 256^3 sublattice arrays,
    complex64): a state localised on the even sublattice, evolved by one
    jump to t = 6 and by 6 position-space steps, against the oracle's
    Cartesian steps on a 16^3 Cartesian torus (the light cone fits); norm kept
    on the whole field."""
    from oracle import cubic
    N, t, m = 256, 6, 0.02
    zeta = np.array([0.6, 0.2j, -0.5, 0.3 + 0.4j])
    zeta = zeta / np.linalg.norm(zeta)
    plan = qw.Plan(3, N, m, "c64")
    f = torch.zeros((2, 4, N, N, N), dtype=torch.complex64, device="cuda")
    f[0, :, 64, 64, 64] = torch.from_numpy(zeta).to(torch.complex64)
    g = plan.bcc_evolve_fft(f, t)
    h = plan.bcc_step(f.clone(), t)
    fc = np.zeros((4, 16, 16, 16), dtype=np.complex128)
    fc[:, 0, 0, 0] = zeta
    ct = cubic.cartesian_table(m)
    for _ in range(t):
        fc = cubic.step_cartesian(fc, ct)
    # Cartesian site x = 2*64 + w (|w_i| <= t) of the big torus: sublattice
    # parity of w, index 64 + floor(w/2)
    r = np.arange(-t, t + 1)
    W = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    W = W[(W[:, 0] % 2 == W[:, 1] % 2) & (W[:, 1] % 2 == W[:, 2] % 2)]
    sub = W[:, 0] % 2
    mm = 64 + (W - sub[:, None]) // 2
    dev = lambda a: torch.from_numpy(a).cuda()
    want = fc[:, W[:, 0] % 16, W[:, 1] % 16, W[:, 2] % 16]
    for field in (g, h):
        got = field[dev(sub), :, dev(mm[:, 0]), dev(mm[:, 1]), dev(mm[:, 2])].T
        torch.cuda.synchronize()
        got = got.cpu().numpy().astype(np.complex128)
        assert ob.rel_l2(got, want) < 2e-5
        assert abs(float(torch.linalg.vector_norm(field)) - 1.0) < 2e-5


def test_c128_tiled_step_batched_against_oracle(qw):
    """complex128 batches whose fields together reach 256 MiB take the LDS
    tile kernel (the rule counts the whole batch): two 128^3 fields with
    their own masses, and 32 fields of 512 x 4 x 64, whose planes are one
    tile high and wide so that the halo of every tile wraps onto itself.
    Three steps (odd: the result is copied back from scratch)."""
    rng = np.random.default_rng(91)
    for shape, ms in (((128, 128, 128), [0.05, 0.4]),
                      ((512, 4, 64), [0.0, 0.1, 0.3, 1.0] * 8)):
        B = len(ms)
        plan = qw.Plan(3, list(shape), 0.1, "c128")
        assert B * 4 * int(np.prod(shape)) * 16 >= 256 << 20
        psis = []
        for b in range(B):
            z = rng.standard_normal((4,) + shape) + 1j * rng.standard_normal((4,) + shape)
            psis.append(z / np.linalg.norm(z))
        x = torch.from_numpy(np.stack(psis)).cuda()
        plan.step_batched(x, ms, 3)
        torch.cuda.synchronize()
        got = x.cpu().numpy()
        del x
        for b in sorted(set(range(B)) & {0, 1, 2, 3, B - 1}):
            ref = stepper.evolve_steps(psis[b], walk.stencil_table(3, ms[b]), 3)
            assert ob.rel_l2(got[b], ref) < 1e-12, (shape, b)


def test_c128_tiled_step_against_oracle(qw):
    """complex128 fields of at least 256 MiB take the LDS tile kernel of the
    3D step: 256 x 128 x 128 (exactly 256 MiB; 64 tiles of 4 x 64 per plane,
    chunks of 8 planes), two steps against the oracle's stepping."""
    shape, m = (256, 128, 128), 0.3
    rng = np.random.default_rng(77)
    psi = rng.standard_normal((4,) + shape) + 1j * rng.standard_normal((4,) + shape)
    psi /= np.linalg.norm(psi)
    plan = qw.Plan(3, list(shape), m, "c128")
    x = torch.from_numpy(psi).cuda()
    plan.step(x, 2)
    ref = stepper.evolve_steps(psi, walk.stencil_table(3, m), 2)
    assert ob.rel_l2(x.cpu().numpy(), ref) < 1e-12


def test_c128_weyl_tiled_step_against_oracle(qw):
    """complex128 Weyl fields of at least 256 MiB take the LDS tile kernel
    (tiles of 8 x 64): 128 x 256 x 256 (exactly 256 MiB), two steps against
    the oracle's stepping."""
    shape = (128, 256, 256)
    rng = np.random.default_rng(78)
    psi = rng.standard_normal((2,) + shape) + 1j * rng.standard_normal((2,) + shape)
    psi /= np.linalg.norm(psi)
    plan = qw.Plan(3, list(shape), 0.0, "c128", weyl=True)
    x = torch.from_numpy(psi).cuda()
    plan.step(x, 2)
    ref = stepper.evolve_steps(psi, walk.weyl_table(3), 2)
    assert ob.rel_l2(x.cpu().numpy(), ref) < 1e-12
