"""qw_evolve_fft_series: the reductions of U^t psi0 for many times in one
call (Sec. 4: the spectrum of psi0 does not depend on t; Sec. 5.2: the
position expectation over time).

Checked against qw_evolve_fft_observables at every time (the same quantity
through the fused jump, to rounding) on every lattice dimension, both
precisions, the 1D four-step split and the Weyl walk; against the oracle's
exact torus evolution on a 3D state; and for its argument handling."""
import math

import numpy as np
import pytest
import torch

from oracle import fourier, observables as ob, states, walk

pytestmark = pytest.mark.gpu

TIMES = [0, 1, 2, 7, -5, 64, 1000, 12345, 99999, 100000, 1 << 40, 7]


@pytest.fixture(scope="module")
def qw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1603_06442_amd import qw as mod
    return mod


def _atol(dtype, n):
    # minimum-image means of fields within 2e-5 (complex64) / 1e-12
    # (complex128) of each other in 2-norm differ by at most n times that
    return n * (4e-5 if dtype == "c64" else 1e-11)


def _state(qw, plan, n):
    x = plan.empty()
    k0 = [0.3, -0.2, 0.1][:plan.dim]
    plan.prepare_state(x, k0, max(1.5, n / 12.0), [n / 2] * plan.dim, 0.6, 0.8)
    return x


CASES = [(1, 512), (1, 8192), (2, 64), (3, 32), (3, 16)]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("dim,n", CASES)
def test_series_matches_fused_jumps(qw, dim, n, dtype):
    plan = qw.Plan(dim, n, 0.15, dtype)
    x = _state(qw, plan, n)
    keep = x.clone()
    origin = [n / 2 - 1.5] * dim
    ser = plan.evolve_fft_series(x, TIMES, origin)
    assert torch.equal(x, keep)  # psi0 untouched
    assert len(ser) == len(TIMES)
    tol = _atol(dtype, n)
    for t, s in zip(TIMES, ser):
        o = plan.evolve_fft_observables(x, t, origin)
        assert abs(s["norm2"] - o["norm2"]) < (2e-6 if dtype == "c64" else 1e-12), t
        assert np.abs(np.array(s["mean"]) - np.array(o["mean"])).max() < tol, t
        assert np.abs(np.array(s["mean_cart"]) - np.array(o["mean_cart"])).max() < 2 * tol, t
        assert np.allclose(s["second"], o["second"], rtol=1e-4 if dtype == "c64" else 1e-9,
                           atol=tol * n), t
    # a repeated time gives the same bits
    assert ser[3] == ser[-1]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_series_matches_the_oracle(qw, dtype):
    """3D, 16^3, particle/antiparticle state: the oracle's exact torus
    evolution (DFT, binary powering of the summed symbol, inverse DFT)."""
    n, m = 16, 0.2
    center = [8, 8, 8]
    k0 = [0.2, -0.1, 0.3]
    psi0 = states.particle_state(3, n, m, k0, 2.0, center, 1 / math.sqrt(2), 1 / math.sqrt(2))
    table = walk.stencil_table(3, m)
    plan = qw.Plan(3, n, m, dtype)
    x = torch.from_numpy(np.ascontiguousarray(psi0)).to(plan.torch_dtype).cuda()
    times = [1, 10, 333, 4096, 100000]
    ser = plan.evolve_fft_series(x, times, center)
    for t, s in zip(times, ser):
        want = ob.observables(fourier.evolve_fourier(psi0, table, t), center)
        # complex64: the field bound 2e-5; complex128: the oracle's binary
        # powering itself drifts with t (its norm at t = 1e5 is 1 - 3e-12),
        # so max(1e-12, 1e-15 t) as in the Zitterbewegung tests
        e = 2e-5 if dtype == "c64" else max(1e-12, 1e-15 * t)
        assert abs(s["norm2"] - want["norm2"]) < e, t
        assert np.abs(np.array(s["mean"]) - np.array(want["mean"][:3])).max() < 2 * n * e, t


def test_weyl_series(qw):
    plan = qw.Plan(3, 16, 0.0, "c64", weyl=True)
    x = plan.empty()
    x.copy_(torch.randn(x.shape, dtype=torch.complex64,
                        generator=torch.Generator(device="cuda").manual_seed(3), device="cuda"))
    times = [3, 40, 500]
    ser = plan.evolve_fft_series(x, times, [8, 8, 8])
    for t, s in zip(times, ser):
        o = plan.evolve_fft_observables(x, t, [8, 8, 8])
        assert abs(s["norm2"] - o["norm2"]) <= 1e-6 * o["norm2"]
        assert np.abs(np.array(s["mean"]) - np.array(o["mean"])).max() < _atol("c64", 16)


def test_series_arguments(qw):
    plan = qw.Plan(3, 16, 0.1, "c64")
    x = _state(qw, plan, 16)
    with pytest.raises(ValueError):
        plan.evolve_fft_series(x, [], [8, 8, 8])
    with pytest.raises(qw.QwError) as e:
        plan.evolve_fft_series(x, [1, (1 << 53) + 1], [8, 8, 8])
    assert e.value.status == qw.QW_ERR_UNSUPPORTED
    with pytest.raises(qw.QwError) as e:
        plan.evolve_fft_series(x, [1, 2], [8, float("nan"), 8])
    assert e.value.status == qw.QW_ERR_INVALID
    import ctypes
    o = (qw.QwObs * 1)()
    t = (ctypes.c_int64 * 1)(5)
    assert qw.LIB.qw_evolve_fft_series(plan._h, None, 1, t, (ctypes.c_double * 3)(8, 8, 8), o,
                                       None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_evolve_fft_series(plan._h, ctypes.c_void_p(x.data_ptr()), 0, t,
                                       (ctypes.c_double * 3)(8, 8, 8), o,
                                       None) == qw.QW_ERR_INVALID
    # a larger series after a smaller one (the result slots grow)
    big = plan.evolve_fft_series(x, list(range(200)), [8, 8, 8])
    assert len(big) == 200 and all(abs(b["norm2"] - 1) < 2e-5 for b in big)
