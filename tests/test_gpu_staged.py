"""Strided FFT passes staged through LDS (global-to-LDS loads, double
buffered) against the register kernels they replace, bit for bit.

The staged kernels take the passes of at least 8192 tiles: at complex64 the
length-256 inverse ones (32-column tiles; a 256^3 field of four components)
and the length-512 ones of both directions (16-column tiles), at complex128
the length-256 and -512 ones whose rows are at least 4096 elements apart,
both directions (16- and 8-column tiles; the n1 passes at 256^3 and 512^3);
with qw_set_fft_kernel(0) every pass keeps its loads in registers. Both run the
same tiles through the same arithmetic, so every result must have the same
bits: the field of a jump (Sec. 4: the Fourier evaluation of U^t), the
reductions fused into its last pass (Sec. 5.2), the transforms, the time
series, a batched jump whose instances together cross the size threshold,
the slab schedule (its n1 pass staged, its slab passes not) and a graph
replay of a staged jump."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1603_06442_amd import qw as mod
    yield mod
    mod.set_fft_kernel(True)


def _field(plan, seed, B=1):
    g = torch.Generator(device="cuda").manual_seed(seed)
    shape = plan.empty().shape
    x = torch.randn((B,) + tuple(shape) if B > 1 else shape, dtype=plan.torch_dtype,
                    generator=g, device="cuda")
    return x / torch.linalg.vector_norm(x)


def _both(qw, fn):
    """fn() with the staged kernels (the default), then with register kernels."""
    try:
        qw.set_fft_kernel(True)
        a = fn()
        torch.cuda.synchronize()
        qw.set_fft_kernel(False)
        b = fn()
        torch.cuda.synchronize()
    finally:
        qw.set_fft_kernel(True)
    return a, b


def test_full_size_jump_and_reductions(qw):
    n = 256
    plan = qw.Plan(3, n, 0.1, "c64")
    x = _field(plan, 5)
    origin = [n / 2 - 0.5, n / 3, 17.25]
    print("256^3 complex64: jump, fused reductions, inverse transform, series", flush=True)
    a, b = _both(qw, lambda: plan.evolve_fft(x, 777))
    assert torch.equal(a, b)
    del a, b
    out = [plan.empty(), plan.empty()]
    k = iter(range(2))

    def fused():
        i = next(k)
        return plan.evolve_fft_observables(x, -12345, origin, out=out[i])
    oa, ob = _both(qw, fused)
    assert oa == ob
    assert torch.equal(out[0], out[1])
    want = plan.observables(out[0], origin)
    assert abs(oa["norm2"] - want["norm2"]) < 1e-12
    assert np.abs(np.array(oa["mean"]) - np.array(want["mean"])).max() < 1e-9
    del out
    na, nb = _both(qw, lambda: plan.evolve_fft_observables(x, 99, origin))  # no field written
    assert na == nb
    ta, tb = _both(qw, lambda: plan.transform(x, -1))
    assert torch.equal(ta, tb)
    del ta, tb
    sa, sb = _both(qw, lambda: plan.evolve_fft_series(x, [1, 64, 4096, 100000], origin))
    assert sa == sb


@pytest.mark.parametrize("B", [2, 3])
def test_batched_instances_cross_the_threshold(qw, B):
    """256 x 128 x 256: one instance is 4096 tiles (register kernel), two
    are 8192 and three 12288 (staged; tiles of one workgroup may belong to
    two instances); per-instance masses and times."""
    plan = qw.Plan(3, [256, 128, 256], 0.2, "c64")
    x = _field(plan, 9, B=B)
    print("batched %d x 256x128x256 complex64" % B, flush=True)
    m = [0.2, 0.05, 0.31][:B]
    t = [333, -70, 100001][:B]
    a, b = _both(qw, lambda: plan.evolve_fft_batched(x, m, t))
    assert torch.equal(a, b)
    # each instance as a single jump at its own mass gives the same field to rounding
    for i in range(B):
        p1 = qw.Plan(3, [256, 128, 256], m[i], "c64")
        one = p1.evolve_fft(x[i].contiguous(), t[i])
        rel = (torch.linalg.vector_norm(one - a[i]) / torch.linalg.vector_norm(one)).item()
        assert rel < 2e-5, (i, rel)
        del one, p1


@pytest.mark.parametrize("weyl,shape", [(True, [256, 512, 256]), (False, [256, 512, 128])])
def test_other_shapes(qw, weyl, shape):
    """The n1 inverse pass over 4096-column rows (Weyl, two components) and
    2048-column rows of a non-cubic lattice (the n2 passes have length 512
    there and keep the register kernel): field and fused reductions."""
    plan = qw.Plan(3, shape, 0.0 if weyl else 0.15, "c64", weyl=weyl)
    x = _field(plan, 17)
    origin = [shape[0] / 2 + 0.25, shape[1] / 3, shape[2] - 5.5]
    print("staged n1 pass: %s %s" % ("Weyl" if weyl else "Dirac", shape), flush=True)
    a, b = _both(qw, lambda: plan.evolve_fft(x, 2024))
    assert torch.equal(a, b)
    del a, b
    oa, ob = _both(qw, lambda: plan.evolve_fft_observables(x, -31, origin))
    assert oa == ob


def test_complex128_n1_passes(qw):
    """256^3 complex128: the n1 passes of both directions staged."""
    n = 256
    plan = qw.Plan(3, n, 0.1, "c128")
    x = _field(plan, 23)
    origin = [n / 2 + 0.5, 100.0, 31.75]
    print("256^3 complex128: jump, transforms, fused reductions", flush=True)
    a, b = _both(qw, lambda: plan.evolve_fft(x, 4321))
    assert torch.equal(a, b)
    del a, b
    for d in (1, -1):
        ta, tb = _both(qw, lambda: plan.transform(x, d))
        assert torch.equal(ta, tb), d
        del ta, tb
    oa, ob = _both(qw, lambda: plan.evolve_fft_observables(x, 777, origin))
    assert oa == ob
    ra, rb = _both(qw, lambda: plan.evolve_fft_real(x, 0.5))
    assert torch.equal(ra, rb)


def test_complex128_batched(qw):
    plan = qw.Plan(3, [256, 128, 256], 0.2, "c128")
    x = _field(plan, 29, B=2)
    print("batched 2 x 256x128x256 complex128", flush=True)
    a, b = _both(qw, lambda: plan.evolve_fft_batched(x, [0.2, 0.05], [333, -70]))
    assert torch.equal(a, b)


@pytest.mark.parametrize("shape", [[512, 128, 256], [256, 512, 128]])
def test_length_512_passes(qw, shape):
    """complex64 passes of length 512 (the n1 pass over 32768-column rows,
    then the n2 pass over 128-column rows), both directions."""
    plan = qw.Plan(3, shape, 0.1, "c64")
    x = _field(plan, 31)
    print("length-512 passes: %s" % shape, flush=True)
    for d in (1, -1):
        ta, tb = _both(qw, lambda: plan.transform(x, d))
        assert torch.equal(ta, tb), d
        del ta, tb
    a, b = _both(qw, lambda: plan.evolve_fft(x, -999))
    assert torch.equal(a, b)


def test_complex128_length_512(qw):
    """512 x 128 x 128 complex128: the n1 pass (length 512, 16384-column rows)
    staged, both directions."""
    plan = qw.Plan(3, [512, 128, 128], 0.25, "c128")
    x = _field(plan, 37)
    print("complex128 length-512 n1 pass", flush=True)
    for d in (1, -1):
        ta, tb = _both(qw, lambda: plan.transform(x, d))
        assert torch.equal(ta, tb), d
        del ta, tb
    a, b = _both(qw, lambda: plan.evolve_fft(x, 12))
    assert torch.equal(a, b)


def test_slab_schedule(qw):
    plan = qw.Plan(3, 256, 0.3, "c64")
    plan.set_schedule(32, 8, 256, 1)
    x = _field(plan, 13)
    print("256^3 complex64, slab schedule", flush=True)
    a, b = _both(qw, lambda: plan.evolve_fft(x, 4242))
    assert torch.equal(a, b)


def test_switch_arguments(qw):
    assert qw.LIB.qw_set_fft_kernel(2) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_set_fft_kernel(-1) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_set_fft_kernel(1) == qw.QW_OK


def test_staged_passes_in_a_graph(qw):
    """qw_evolve_fft at 256^3 complex64 (its inverse passes staged) captured
    into a HIP graph: each replay, with eager work and synchronisations
    between replays, gives bitwise the eager result."""
    plan = qw.Plan(3, 256, 0.05, "c64")
    x0 = _field(plan, 41)
    want = plan.evolve_fft(x0, 99)
    torch.cuda.synchronize()
    out = plan.empty()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.evolve_fft(x0, 99, out=out, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    print("capturing the 256^3 jump", flush=True)
    with torch.cuda.graph(g):
        plan.evolve_fft(x0, 99, out=out, stream=torch.cuda.current_stream())
    for r in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), r
        e = plan.evolve_fft(x0, 7)  # eager work between replays
        torch.cuda.synchronize()
        del e


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_full_size_series_matches_fused_jumps(qw, dtype):
    """256^3: the series (staged reduction pass without a store, after the
    staged n2 inverse pass) against the fused jump at each time (staged
    reduction pass with a store), the same quantity to rounding."""
    n = 256
    plan = qw.Plan(3, n, 0.02, dtype)
    x = plan.empty()
    plan.prepare_state(x, [0.1, 0.1, 0.1], 20.0, [n // 2] * 3, 1 / np.sqrt(2), 1 / np.sqrt(2))
    origin = [n / 2, n / 2, n / 2]
    times = [1, 100, 4096, 100000]
    print("256^3 %s series against fused jumps" % dtype, flush=True)
    ser = plan.evolve_fft_series(x, times, origin)
    tol = 4e-5 * n if dtype == "c64" else 1e-11 * n
    for t, s in zip(times, ser):
        o = plan.evolve_fft_observables(x, t, origin)
        assert abs(s["norm2"] - o["norm2"]) < (2e-6 if dtype == "c64" else 1e-12), t
        assert np.abs(np.array(s["mean"]) - np.array(o["mean"])).max() < tol, t
