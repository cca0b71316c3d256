"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Inputs come from the seeded generators or from the oracle; nothing the oracle
sees comes from the GPU. Tolerances (relative L2 over all entries, no phase
alignment):
* complex128: 1e-12 for t <= 1e3 and 1e-15 t beyond (the phase omega t
  carries an absolute error ~ t * eps64);
* complex64: 2e-5 for the Fourier jump (FP32 transforms, FP64 phase); the
  FP32 stencil's transition matrices are rounded to FP32, so each step is
  off the unitary one by O(2^-24) and the error grows linearly in the number
  of steps: max(2e-5, 4 steps 2^-24), which is 2e-5 up to 83 steps; the
  128-step 64^3 workload is held to 2e-5 itself.
"""
import math

import numpy as np
import pytest
import torch

from oracle import fourier, observables as ob, states, stepper, walk
from paper_1603_06442_amd import inputs

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


def tol_step(dtype, steps):
    # complex64: the transition matrices are rounded to FP32, so each step is
    # off by O(2^-24) from the unitary one and the error grows linearly in t.
    return max(2e-5, 4 * steps * 2.0 ** -24) if dtype == "c64" else 1e-12


def table(d, m):
    return walk.stencil_table(d, m)


SHAPES = [(1, (64,)), (1, (256,)), (2, (8, 16)), (2, (32, 32)), (3, (4, 8, 16)), (3, (16, 16, 16))]


def rand_field(d, shape, seed):
    rng = np.random.default_rng(seed)
    s = walk.spinor_dim(d)
    psi = rng.standard_normal((s,) + shape) + 1j * rng.standard_normal((s,) + shape)
    return psi / np.linalg.norm(psi)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,shape", SHAPES)
@pytest.mark.parametrize("m", [0.0, 0.13, 1.0])
def test_step_matches_oracle(qw, d, shape, m, dtype):
    psi0 = rand_field(d, shape, 100 + d)
    plan = qw.Plan(d, list(shape), m, dtype)
    x = to_dev(psi0, plan)
    plan.step(x, 7)
    ref = stepper.evolve_steps(psi0, table(d, m), 7)
    assert ob.rel_l2(to_np(x), ref) < tol_step(dtype, 7)


TWO_STEP_TILES = {0: (16, 32), 1: (8, 64), 2: (16, 16), 3: (8, 32)}


@pytest.mark.parametrize("tile", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", [(2, 16, 64), (4, 16, 32), (16, 16, 64), (8, 32, 128),
                                   (64, 16, 32), (4, 8, 64), (4, 16, 16), (2, 8, 32)])
@pytest.mark.parametrize("m", [0.0, 0.3, 1.0])
def test_two_step_kernel_matches_oracle_and_single_steps(qw, shape, m, tile):
    """Pairs of complex64 3D steps run as one launch (both rings in LDS):
    against the oracle over 2 and 5 steps (a pair, two pairs and a single
    step), and bitwise equal to the same steps one launch each. Shapes whose
    planes are one tile (16 x 32, or 8 x 64) so that every halo wraps onto
    the tile itself, N1 = 2 (the whole axis in one chunk), several tiles and
    chunks; every tile shape."""
    t2, t3 = TWO_STEP_TILES[tile]
    if shape[1] < t2 or shape[2] < t3:
        pytest.skip("plane smaller than the tile")
    psi0 = rand_field(3, shape, 33)
    plan = qw.Plan(3, list(shape), m, "c64")
    try:
        qw.set_step_kernel(True, tile)
        for n in (2, 5):
            x = to_dev(psi0, plan)
            plan.step(x, n)
            ref = stepper.evolve_steps(psi0, table(3, m), n)
            assert ob.rel_l2(to_np(x), ref) < tol_step("c64", n), n
            qw.set_step_kernel(False)
            y = to_dev(psi0, plan)
            plan.step(y, n)
            torch.cuda.synchronize()
            assert torch.equal(x, y), n
            qw.set_step_kernel(True, tile)
    finally:
        qw.set_step_kernel(False, 0, 0)


def test_two_step_kernel_batched_and_chunks(qw):
    """Batched pairs of steps with per-instance masses, and every number of
    planes per workgroup, against one launch per step (bitwise) and the
    oracle."""
    shape = (32, 16, 64)
    ms = [0.0, 0.05, 0.3]
    psis = [rand_field(3, shape, 60 + b) for b in range(3)]
    plan = qw.Plan(3, list(shape), 0.1, "c64")
    try:
        qw.set_step_kernel(False)
        want = torch.stack([to_dev(p, plan) for p in psis]).contiguous()
        plan.step_batched(want, ms, 4)
        for tile in (0, 2):
            for chunk in (2, 4, 8, 16, 32):
                qw.set_step_kernel(True, tile, chunk)
                x = torch.stack([to_dev(p, plan) for p in psis]).contiguous()
                plan.step_batched(x, ms, 4)
                torch.cuda.synchronize()
                assert torch.equal(x, want), (tile, chunk)
    finally:
        qw.set_step_kernel(False, 0, 0)
    for b in range(3):
        ref = stepper.evolve_steps(psis[b], table(3, ms[b]), 4)
        assert ob.rel_l2(to_np(want[b]), ref) < tol_step("c64", 4)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("shape", [(8, 8, 64), (4, 16, 128), (32, 8, 64)])
@pytest.mark.parametrize("m", [0.0, 0.3])
def test_step_3d_plane_ring_matches_oracle(qw, shape, m, dtype):
    """complex64 lattices with N1 >= 4, N2 >= 8 and N3 >= 64 take the LDS
    plane-ring kernel (tiles of 8 x 64, chunks along n1, periodic wrap in all
    three axes); complex128 takes one thread per site here (its LDS tile
    kernel serves fields of at least 256 MiB: the full-size tests)."""
    psi0 = rand_field(3, shape, 31)
    plan = qw.Plan(3, list(shape), m, dtype)
    x = to_dev(psi0, plan)
    plan.step(x, 5)
    ref = stepper.evolve_steps(psi0, table(3, m), 5)
    assert ob.rel_l2(to_np(x), ref) < tol_step(dtype, 5)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,shape", SHAPES + [(1, (8192,)), (1, (65536,)), (1, (2,)), (3, (2, 2, 2))])
def test_transform_matches_dft(qw, d, shape, dtype):
    psi0 = rand_field(d, shape, 7)
    plan = qw.Plan(d, list(shape), 0.2, dtype)
    x = to_dev(psi0, plan)
    fw = plan.transform(x, +1)
    ref = fourier.dft(psi0)
    tol = 1e-6 if dtype == "c64" else 1e-13
    assert ob.rel_l2(to_np(fw), ref) < tol
    back = plan.transform(fw, -1)
    assert ob.rel_l2(to_np(back) / np.prod(shape), psi0) < tol


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,shape", SHAPES + [(1, (8192,))])
@pytest.mark.parametrize("t", [0, 1, 5, -3, 1000, 100000])
def test_evolve_fft_matches_oracle(qw, d, shape, t, dtype):
    m = 0.21
    psi0 = rand_field(d, shape, 200 + d)
    plan = qw.Plan(d, list(shape), m, dtype)
    out = plan.evolve_fft(to_dev(psi0, plan), t)
    ref = fourier.evolve_fourier(psi0, table(d, m), t)
    assert ob.rel_l2(to_np(out), ref) < tol_fft(dtype, t)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,shape", [(1, (128,)), (2, (16, 16)), (3, (8, 8, 8))])
@pytest.mark.parametrize("m", [0.0, 1.0])
def test_evolve_fft_degenerate_masses(qw, d, shape, m, dtype):
    """m = 0 (sin omega = 0 at the band centre) and m = 1 (n = 0)."""
    psi0 = rand_field(d, shape, 5)
    plan = qw.Plan(d, list(shape), m, dtype)
    for t in (1, 2, 7, 64):
        out = plan.evolve_fft(to_dev(psi0, plan), t)
        ref = fourier.evolve_fourier(psi0, table(d, m), t)
        assert ob.rel_l2(to_np(out), ref) < tol_fft(dtype, t)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_evolve_in_place_and_reversible(qw, dtype):
    d, shape, m = 3, (16, 16, 16), 0.3
    psi0 = rand_field(d, shape, 9)
    plan = qw.Plan(d, list(shape), m, dtype)
    x = to_dev(psi0, plan)
    plan.evolve_fft(x, 12345, out=x)
    plan.evolve_fft(x, -12345, out=x)
    assert ob.rel_l2(to_np(x), psi0) < (4e-5 if dtype == "c64" else 1e-11)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_fft_jump_equals_steps_on_gpu(qw, dtype):
    d, shape, m = 3, (16, 16, 16), 0.05
    psi0 = rand_field(d, shape, 3)
    plan = qw.Plan(d, list(shape), m, dtype)
    a = to_dev(psi0, plan)
    plan.step(a, 20)
    b = plan.evolve_fft(to_dev(psi0, plan), 20)
    assert ob.rel_l2(to_np(a), to_np(b)) < (4e-5 if dtype == "c64" else 1e-12)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,shape", [(1, (512,)), (2, (32, 16)), (3, (16, 16, 16))])
def test_observables_match_oracle(qw, d, shape, dtype):
    psi = rand_field(d, shape, 11)
    refp = rand_field(d, shape, 12)
    plan = qw.Plan(d, list(shape), 0.1, dtype)
    _check_observables(plan, psi, refp, [n // 3 + 0.0 for n in shape], dtype)
    _check_observables(plan, psi, refp, [n / 3 + 0.37 for n in shape], dtype)
    _check_observables(plan, psi, None, [n - 1.5 for n in shape], dtype)


def _check_observables(plan, psi, refp, c, dtype):
    got = plan.observables(to_dev(psi, plan), c,
                           ref=to_dev(refp, plan) if refp is not None else None)
    # the oracle sees the field rounded to the GPU's precision
    if dtype == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)
        if refp is not None:
            refp = refp.astype(np.complex64).astype(np.complex128)
    want = ob.observables(psi, c, refp)
    assert abs(got["norm2"] - want["norm2"]) < 1e-12
    assert np.allclose(got["mean"][:plan.dim], want["mean"][:plan.dim], atol=1e-10)
    assert np.allclose(got["second"], want["second"], atol=1e-9)
    assert np.allclose(got["mean_cart"], want["mean_cart"], atol=1e-10)
    assert abs(got["overlap"] - want["overlap"]) < 1e-12
    assert abs(got["ref_norm2"] - want["ref_norm2"]) < 1e-12


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,N,k0,sigma,cp,cm", [
    (1, 1024, [0.3], 10.0, 1.0, 0.0),
    (1, 8192, [-0.2], 40.0, 0.6, 0.8),
    (2, 64, [0.2, -0.1], 4.0, 1 / math.sqrt(2), 1 / math.sqrt(2)),
    (3, 32, [0.1, 0.1, 0.1], 3.0, 1 / math.sqrt(2), 1 / math.sqrt(2)),
    (3, 32, [0.3, -0.2, 0.1], 2.5, 0.0, 1.0),
])
def test_prepare_state_matches_oracle(qw, d, N, k0, sigma, cp, cm, dtype):
    m = 0.1
    c = [N // 2] * d
    plan = qw.Plan(d, N, m, dtype)
    x = plan.empty()
    plan.prepare_state(x, k0, sigma, c, cp, cm)
    want = states.particle_state(d, N, m, k0, sigma, c, cp, cm)
    assert ob.rel_l2(to_np(x), want) < (2e-6 if dtype == "c64" else 1e-12)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batched_matches_single_and_oracle(qw, dtype):
    d, shape = 3, (8, 8, 16)
    plan = qw.Plan(d, list(shape), 0.1, dtype)
    B = 5
    ms = [0.0, 0.05, 0.1, 0.3, 1.0]
    ts = [1, 17, -4, 100000, 3]
    xs = np.stack([rand_field(d, shape, 50 + b) for b in range(B)])
    x = to_dev(xs, plan)
    out = plan.evolve_fft_batched(x, ms, ts)
    outn = to_np(out)
    for b in range(B):
        single = qw.Plan(d, list(shape), ms[b], dtype)
        one = single.evolve_fft(to_dev(xs[b], single), ts[b])
        # same arithmetic, except that the single call reads omega from the
        # plan's table: equal up to rounding of the FP64 phase
        assert ob.rel_l2(outn[b], to_np(one)) < (1e-6 if dtype == "c64" else tol_fft(dtype, ts[b]))
        ref = fourier.evolve_fourier(xs[b], table(d, ms[b]), ts[b])
        assert ob.rel_l2(outn[b], ref) < tol_fft(dtype, ts[b])


def test_workload_line_4096_c128(qw):
    """The 1D workload: N = 4096, complex128, m = 0.1, packet at k0 = 0.3,
    width 40: 1000 steps and the t = 1000 jump vs the oracle, drift law."""
    w = inputs.workload(0)
    psi0 = states.particle_state(1, w["N"], w["m"], w["k0"], w["sigma"], w["center"])
    plan = qw.Plan(1, w["N"], w["m"], "c128")
    ref = stepper.evolve_steps(psi0, table(1, w["m"]), w["steps"])
    x = to_dev(psi0, plan)
    plan.step(x, w["steps"])
    assert ob.rel_l2(to_np(x), ref) < 1e-12
    y = plan.evolve_fft(to_dev(psi0, plan), w["t"])
    assert ob.rel_l2(to_np(y), ref) < 1e-12
    o0 = plan.observables(to_dev(psi0, plan), w["center"])
    o1 = plan.observables(y, w["center"])
    drift = ob.drift_prediction(psi0, table(1, w["m"]), w["t"])[0]
    assert abs((o1["mean"][0] - o0["mean"][0]) - drift) < 1e-8
    assert abs(o1["norm2"] - 1.0) < 1e-12


def test_workload_bcc_64_c64(qw):
    """The 64^3 BCC workload (complex64 on the GPU vs complex128 oracle):
    t = 128 by the stencil and by one Fourier jump."""
    w = inputs.workload(1)
    psi0 = states.particle_state(3, w["N"], w["m"], w["k0"], w["sigma"], w["center"])
    ref = fourier.evolve_fourier(psi0, table(3, w["m"]), w["t"])
    plan = qw.Plan(3, w["N"], w["m"], "c64")
    x = to_dev(psi0, plan)
    plan.step(x, w["steps"])
    e_step = ob.rel_l2(to_np(x), ref)
    y = plan.evolve_fft(to_dev(psi0, plan), w["t"])
    e_fft = ob.rel_l2(to_np(y), ref)
    o = plan.observables(y, w["center"])
    os_ = plan.observables(x, w["center"])
    print("64^3 complex64, t = %d: stencil rel-L2 %.3e (norm drift %.2e), "
          "Fourier jump rel-L2 %.3e (norm drift %.2e)"
          % (w["t"], e_step, abs(os_["norm2"] - 1.0), e_fft, abs(o["norm2"] - 1.0)))
    # the FP32-path bound, for the 128 stencil steps as for the jump
    assert e_step < 2e-5
    assert e_fft < 2e-5
    assert abs(o["norm2"] - 1.0) < 1e-5
    assert abs(os_["norm2"] - 1.0) < 1e-5


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_every_schedule_gives_the_same_evolution(qw, dtype):
    """Slabbed middle passes and both fused-pass widths vs the oracle, on a
    non-cubic torus, including a slab size that does not divide N1."""
    d, shape, m, t = 3, (16, 8, 32), 0.07, 777
    psi0 = rand_field(d, shape, 21)
    ref = fourier.evolve_fourier(psi0, table(d, m), t)
    plan = qw.Plan(d, list(shape), m, dtype)
    for slab in (0, 1, 3, 4, 16):
        for ce in (4, 8):
            for cb, gw in ((64, 1), (256, 1), (64, 4), (128, 3)):
                plan.set_schedule(slab, ce, cb, gw)
                out = plan.evolve_fft(to_dev(psi0, plan), t)
                assert ob.rel_l2(to_np(out), ref) < tol_fft(dtype, t), (slab, ce, cb, gw)
    ms = plan.autotune()
    assert ms > 0 and plan.schedule()[1] in (4, 8) and plan.schedule()[3] >= 1
    out = plan.evolve_fft(to_dev(psi0, plan), t)
    assert ob.rel_l2(to_np(out), ref) < tol_fft(dtype, t)


def test_batched_with_slabs(qw):
    d, shape = 3, (8, 8, 16)
    plan = qw.Plan(d, list(shape), 0.1, "c64")
    plan.set_schedule(2, 4, 128, 2)
    ms, ts = [0.02, 0.2, 0.5], [3, 999, -70]
    xs = np.stack([rand_field(d, shape, 70 + b) for b in range(3)])
    outn = to_np(plan.evolve_fft_batched(to_dev(xs, plan), ms, ts))
    for b in range(3):
        ref = fourier.evolve_fourier(xs[b], table(d, ms[b]), ts[b])
        assert ob.rel_l2(outn[b], ref) < 2e-5


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_workload_512_subcase_t_1e6(qw, dtype):
    """The 512^3 workload's oracle sub-case: 32^3, m = 0.1, k0 from the
    workload's seed, width 2.5 cells, t = 1e6 by one Fourier jump vs the
    oracle's binary powering (complex128 bound 1e-15 t = 1e-9)."""
    w = inputs.workload(4)
    N, t = w["sub_N"], w["t"]
    psi0 = states.particle_state(3, N, w["m"], w["k0"], w["sub_sigma"], [N // 2] * 3)
    ref = fourier.evolve_fourier(psi0, table(3, w["m"]), t)
    plan = qw.Plan(3, N, w["m"], dtype)
    out = plan.evolve_fft(to_dev(psi0, plan), t)
    assert ob.rel_l2(to_np(out), ref) < tol_fft(dtype, t)
    assert abs(plan.observables(out, [N // 2] * 3)["norm2"] - 1.0) < (1e-5 if dtype == "c64" else 1e-12)


def test_fp32_path_vs_fp64_path_large_t(qw):
    """complex64 (FP32 transforms, FP64 phase) vs complex128 on the GPU, 64^3,
    at t = 1e6: within the FP32 tolerance."""
    N, m = 64, 0.1
    psi0 = rand_field(3, (N, N, N), 41)
    p64 = qw.Plan(3, N, m, "c64")
    p128 = qw.Plan(3, N, m, "c128")
    for t in (1, 999999, 1000000):
        a = to_np(p64.evolve_fft(to_dev(psi0, p64), t))
        b = to_np(p128.evolve_fft(to_dev(psi0, p128), t))
        assert ob.rel_l2(a, b) < 2e-5


def _obs_close(a, b, dim, rt):
    assert abs(a["norm2"] - b["norm2"]) <= rt * max(1.0, abs(b["norm2"]))
    for x, y in zip(a["mean"][:dim], b["mean"][:dim]):
        assert abs(x - y) <= rt * max(1.0, abs(y))
    for x, y in zip(a["second"], b["second"]):
        assert abs(x - y) <= rt * max(1.0, abs(y))
    for x, y in zip(a["mean_cart"], b["mean_cart"]):
        assert abs(x - y) <= rt * max(1.0, abs(y))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,shape,slab", [
    (3, (16, 16, 16), 0), (3, (8, 16, 64), 0), (3, (32, 16, 64), 8), (2, (32, 64), 0),
    (2, (256, 16), 0), (1, (8192,), 0), (1, (1024,), 0),
    (2, (1024, 16), 0), (3, (512, 4, 8), 0)])  # long first axes: reduction not fused
def test_evolve_fft_observables_fused(qw, d, shape, slab, dtype):
    """The reductions taken inside the last inverse pass equal evolve_fft
    followed by observables; the field it writes is evolve_fft's, bitwise."""
    psi = rand_field(d, shape, 21)
    plan = qw.Plan(d, list(shape), 0.15, dtype)
    if slab:
        plan.set_schedule(slab, 8, 256, 1)
    x = to_dev(psi, plan)
    t = 777
    ref_t = plan.evolve_fft(x, t)
    for origin in ([n // 2 for n in shape], [n / 3 + 0.37 for n in shape]):
        want = plan.observables(ref_t, origin)
        out = plan.empty()
        got = plan.evolve_fft_observables(x, t, origin, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_t)
        _obs_close(got, want, d, 1e-12)
        got2 = plan.evolve_fft_observables(x, t, origin)  # result not kept
        assert got2 == got
    # against the oracle
    ref = fourier.evolve_fourier(psi, table(d, 0.15), t)
    want = ob.observables(ref, [n // 2 for n in shape])
    got = plan.evolve_fft_observables(x, t, [n // 2 for n in shape])
    rt = 1e-4 if dtype == "c64" else 1e-10
    _obs_close(got, {"norm2": want["norm2"], "mean": list(want["mean"]),
                     "second": list(want["second"]), "mean_cart": list(want["mean_cart"])}, d, rt)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,shape", [(1, (4096,)), (1, (64,)), (1, (16384,)), (2, (32, 64)),
                                     (3, (16, 16, 16)), (3, (8, 8, 64))])
def test_step_batched_matches_single_and_oracle(qw, d, shape, dtype):
    """Batched stepping, one mass per instance: bitwise equal to qw_step on a
    plan of that mass, and equal to the oracle (1D fields of at most 160 KB
    run on-chip, larger ones and 2D/3D stream)."""
    ms = [0.0, 0.1, 0.37, 1.0]
    psis = [rand_field(d, shape, 40 + b) for b in range(len(ms))]
    plan = qw.Plan(d, list(shape), 0.1, dtype)
    x = torch.stack([to_dev(p, plan) for p in psis]).contiguous()
    nsteps = 7
    plan.step_batched(x, ms, nsteps)
    for b, m in enumerate(ms):
        pb = qw.Plan(d, list(shape), m, dtype)
        y = to_dev(psis[b], pb)
        pb.step(y, nsteps)
        torch.cuda.synchronize()
        assert torch.equal(x[b], y), m
        ref = stepper.evolve_steps(psis[b], table(d, m), nsteps)
        assert ob.rel_l2(to_np(x[b]), ref) < tol_step(dtype, nsteps)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_step_1d_on_chip_long_runs(qw, dtype):
    """More steps than one on-chip launch takes (4096): the field goes back
    to memory between launches without changing the result; m = 0 stays a
    pure shift, bit for bit."""
    N, nsteps = 64, 5000
    psi0 = rand_field(1, (N,), 77)
    plan = qw.Plan(1, N, 0.2, dtype)
    x = to_dev(psi0, plan)
    plan.step(x, nsteps)
    ref = stepper.evolve_steps(psi0, table(1, 0.2), nsteps)
    assert ob.rel_l2(to_np(x), ref) < tol_step(dtype, nsteps)
    p0 = qw.Plan(1, N, 0.0, dtype)
    x = to_dev(psi0, p0)
    p0.step(x, nsteps)
    got = to_np(x)
    want = to_np(to_dev(psi0, p0))
    assert np.array_equal(got[0], np.roll(want[0], -nsteps))
    assert np.array_equal(got[1], np.roll(want[1], nsteps))


@pytest.mark.parametrize("d,shape,dtype", [(3, (64, 64, 64), "c64"), (3, (16, 16, 16), "c128"),
                                           (1, (8192,), "c64"), (2, (64, 32), "c64"),
                                           (3, (256, 128, 128), "c128")])
def test_capture_into_a_graph(qw, d, shape, dtype):
    """qw_step and qw_evolve_fft, called once beforehand (so the plan has its
    scratch and tables), can be captured into a HIP graph by the caller.
    Each replay, with eager work and synchronisations between replays,
    gives bitwise the eager result. The 256 MiB complex128 field steps
    through the LDS tile kernel, whose launch sets its LDS size attribute."""
    plan = qw.Plan(d, list(shape), 0.07, dtype)
    x0 = to_dev(rand_field(d, shape, 5), plan)
    a = x0.clone()
    b = plan.empty()
    plan.step(a, 3)
    plan.evolve_fft(a, 41, out=b)
    torch.cuda.synchronize()
    want_a, want_b = a.clone(), b.clone()
    ga, gb = x0.clone(), plan.empty()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.step(ga.clone(), 3, stream=side)
        plan.evolve_fft(ga, 41, out=gb, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        s = torch.cuda.current_stream()
        plan.step(ga, 3, stream=s)
        plan.evolve_fft(ga, 41, out=gb, stream=s)
    for r in range(3):
        ga.copy_(x0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ga, want_a), r
        assert torch.equal(gb, want_b), r
        e = x0.clone()  # eager work between replays
        plan.step(e, 1)
        torch.cuda.synchronize()


def test_captured_step_survives_scratch_growth(qw):
    """A graph that captured qw_step (whose ping-pong buffer is the plan's
    scratch) is replayed after qw_bcc_step (two fields of scratch) and
    qw_step_batched (three) have grown that scratch: the plan keeps the
    buffer the graph holds until it is destroyed, so every replay still
    gives the eager result bitwise. A call refused for its time leaves the
    scratch as it was."""
    shape = (16, 16, 64)
    plan = qw.Plan(3, list(shape), 0.2, "c64")
    x0 = to_dev(rand_field(3, shape, 17), plan)
    want = x0.clone()
    plan.step(want, 3)
    torch.cuda.synchronize()
    ga = x0.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.step(ga, 3, stream=torch.cuda.current_stream())
    f = torch.from_numpy(rand_field(3, shape, 18)[None].repeat(2, 0)).to(torch.complex64).cuda()
    plan.bcc_step(f, 2)
    xb = torch.stack([x0.clone() for _ in range(3)]).contiguous()
    plan.step_batched(xb, [0.2, 0.1, 0.0], 1)
    with pytest.raises(qw.QwError):
        plan.evolve_fft_observables(x0, 1 << 60, [8, 8, 32])
    torch.cuda.synchronize()
    for r in range(3):
        ga.copy_(x0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ga, want), r
        plan.step(x0.clone(), 1)  # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,shape", [(1, (256,)), (1, (8192,)), (2, (16, 32)), (3, (8, 16, 16))])
def test_evolve_fft_real_t(qw, d, shape, dtype):
    """Real t against the oracle's diagonalised exp(-i t H_q); integer t
    through the real entry equals qw_evolve_fft bit for bit."""
    m = 0.17
    psi = rand_field(d, shape, 61)
    plan = qw.Plan(d, list(shape), m, dtype)
    x = to_dev(psi, plan)
    for t in (0.5, -1.25, 2.75, 1000.37):
        out = plan.evolve_fft_real(x, t)
        ref = fourier.evolve_fourier_real(psi, table(d, m), t)
        assert ob.rel_l2(to_np(out), ref) < tol_fft(dtype, t), t
    for t in (3, -7, 1000):
        a = plan.evolve_fft_real(x, float(t))
        b = plan.evolve_fft(x, t)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    # half steps compose to a stencil step
    h = plan.evolve_fft_real(plan.evolve_fft_real(x, 0.5), 0.5)
    s = x.clone()
    plan.step(s, 1)
    assert ob.rel_l2(to_np(h), to_np(s)) < (2e-5 if dtype == "c64" else 1e-12)


def test_evolve_fft_real_t_band_edge_convention(qw):
    """m = 0: at omega = pi (q = pi on an even 1D lattice) the two branches
    are averaged, as in the oracle."""
    psi = rand_field(1, (64,), 62)
    plan = qw.Plan(1, 64, 0.0, "c128")
    out = plan.evolve_fft_real(to_dev(psi, plan), 0.5)
    ref = fourier.evolve_fourier_real(psi, table(1, 0.0), 0.5)
    assert ob.rel_l2(to_np(out), ref) < 1e-12


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,N,k0,sigma,cp,cm", [
    (1, 4096, [0.3], 40.0, 1.0, 0.0),
    (2, 64, [0.2, -0.1], 5.0, 1 / math.sqrt(2), 1 / math.sqrt(2)),
    (3, 32, [0.1, 0.1, 0.1], 3.0, 1.0, 0.0),
])
def test_evolve_dispersive_matches_oracle(qw, d, N, k0, sigma, cp, cm, dtype):
    from oracle import dispersive
    m = 0.1
    c = [N // 2] * d
    plan = qw.Plan(d, N, m, dtype)
    x = plan.empty()
    for order in (0, 1, 2):
        for t in (0.0, 7.5, 100.0):
            plan.evolve_dispersive(x, k0, sigma, c, cp, cm, order, t)
            ref = dispersive.evolve_dispersive(d, (N,) * d, m, k0, sigma, c, cp, cm, order, t)
            assert ob.rel_l2(to_np(x), ref) < (2e-5 if dtype == "c64" else tol_fft(dtype, t)), (order, t)


def test_evolve_dispersive_overlap_bound_on_the_gpu(qw):
    """3D, 64^3: the GPU's order-2 approximation against the GPU's exact
    Fourier evolution satisfies the overlap bound of Proposition 1, with
    parameters where the bound is informative (m = 0.5, sigma = 20 cells,
    box 3 / sigma: the bound is 0.93, 0.83, 0.67 at t = 2, 5, 10)."""
    from oracle import dispersive
    d, N, m, k0, sigma = 3, 64, 0.5, [0.3, 0.2, 0.1], 20.0
    c = [32] * d
    plan = qw.Plan(d, N, m, "c128")
    x0 = plan.empty()
    plan.prepare_state(x0, k0, sigma, c, 1.0, 0.0)
    approx = plan.empty()
    bounds = []
    for t in (2, 5, 10):
        exact = plan.evolve_fft(x0, t)
        plan.evolve_dispersive(approx, k0, sigma, c, 1.0, 0.0, 2, float(t))
        fid = abs(plan.observables(exact, c, ref=approx)["overlap"])
        bound, eps, gamma = dispersive.overlap_bound(d, (N,) * d, m, k0, sigma, c, 2, t, 3.0 / sigma)
        assert fid >= bound, (t, fid, bound, eps, gamma)
        bounds.append(bound)
    assert bounds[0] > 0.9  # the bound is informative at these parameters


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,shape", [(1, (1024,)), (2, (32, 64)), (3, (16, 16, 32)), (3, (32, 32, 32))])
def test_newton_wigner_matches_oracle(qw, d, shape, dtype):
    m = 0.15
    plan = qw.Plan(d, list(shape), m, dtype)
    c = [n / 2 for n in shape]
    psi = rand_field(d, shape, 71)
    for field in (psi, states.particle_state(d, shape, m, [0.2, 0.1, -0.1][:d], 3.0, c,
                                             1 / math.sqrt(2), 1 / math.sqrt(2))):
        got = plan.newton_wigner(to_dev(field, plan), c)
        if dtype == "c64":
            field = field.astype(np.complex64).astype(np.complex128)
        mean, mean_cart, parts = ob.newton_wigner(field, table(d, m), c)
        tol = 2e-5 if dtype == "c64" else 1e-10
        assert np.allclose(got["mean"][:d], mean[:d], atol=tol * max(shape)), (got, mean)
        assert np.allclose(got["mean_cart"][:d], mean_cart[:d], atol=tol * max(shape))
        for k in range(2):
            assert abs(got["sectors"][k]["norm2"] - parts[k]["norm2"]) < tol


def test_newton_wigner_moves_with_the_drift_on_the_gpu(qw):
    """Particle + antiparticle packet in 3D: the GPU's sector-projected mean
    after t jumps equals its value at t = 0 plus the drift term, while the
    ordinary mean jitters."""
    d, N, m = 3, 32, 0.3
    c = [16, 16, 16]
    plan = qw.Plan(d, N, m, "c128")
    x0 = plan.empty()
    plan.prepare_state(x0, [0.2, 0.1, 0.0], 2.5, c, 1 / math.sqrt(2), 1 / math.sqrt(2))
    psi0 = to_np(x0)
    nw0 = np.array(plan.newton_wigner(x0, c)["mean"][:d])
    jit = []
    for t in (2, 5, 9):
        xt = plan.evolve_fft(x0, t)
        nw = np.array(plan.newton_wigner(xt, c)["mean"][:d])
        want = nw0 + ob.drift_prediction(psi0, table(d, m), t)
        assert np.allclose(nw, want, atol=1e-8), t
        jit.append(abs(plan.observables(xt, c)["mean"][0] - nw[0]))
    assert max(jit) > 1e-3


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("d,shape,c", [(1, (1024,), [300]), (2, (32, 64), [5, 60]),
                                       (3, (16, 32, 8), [15, 0, 3]), (3, (64, 64, 64), [32, 32, 32])])
def test_marginals_match_oracle(qw, d, shape, c, dtype):
    plan = qw.Plan(d, list(shape), 0.1, dtype)
    psi = rand_field(d, shape, 81)
    got = plan.marginals(to_dev(psi, plan), c)
    if dtype == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)
    want = ob.marginals(psi, c)
    for (lo, vals), (wlo, wvals) in zip(got, want):
        assert lo == wlo and len(vals) == len(wvals)
        assert np.allclose(vals, wvals, rtol=1e-12, atol=1e-15)


def test_marginals_of_the_localised_state_on_the_gpu(qw):
    """Localised state after 28 steps (the 3D walk of the paper's projection
    figure, m = 0.03): zero beyond |X| = 28, equal to the oracle's."""
    d, N, m, t = 3, 64, 0.03, 28
    plan = qw.Plan(d, N, m, "c128")
    psi0 = states.localized_state(d, N, [32, 32, 32], [1, 0, 0, 0])
    x = to_dev(psi0, plan)
    plan.step(x, t)
    got = plan.marginals(x, [32, 32, 32])
    want = ob.marginals(stepper.evolve_steps(psi0, table(d, m), t), [32, 32, 32])
    for (lo, vals), (_, wvals) in zip(got, want):
        X = np.arange(lo, lo + len(vals))
        assert np.all(np.asarray(vals)[np.abs(X) > t] == 0.0)
        assert np.allclose(vals, wvals, rtol=1e-11, atol=1e-15)
