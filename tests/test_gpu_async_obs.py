"""qw_evolve_fft_observables_async + qw_obs_from_raw against the waiting
qw_evolve_fft_observables, through the C ABI: the same jump and Sec. 5.2
reductions, so the same qw_obs bit for bit, with several calls queued on one
stream before a single wait (each into its own pinned record), with and
without the evolved field written, for plans whose reductions are fused
into the last strided pass (2D, 3D) and for one whose reductions take a
separate read (1D)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1603_06442_amd import qw as mod
    return mod


CASES = [(3, 64, "c64"), (3, [32, 64, 16], "c128"), (2, 128, "c64"), (1, 1024, "c128")]


def _prepared(qw, dim, N, dtype):
    plan = qw.Plan(dim, N, 0.15, dtype)
    x = plan.empty()
    n = [N] * dim if isinstance(N, int) else N
    plan.prepare_state(x, [0.2] * dim, 3.0, [v // 2 for v in n], 1.0, 0.0)
    origin = [v / 2 - 0.25 for v in n]
    return plan, x, origin


@pytest.mark.parametrize("dim,N,dtype", CASES)
def test_async_records_match_waiting_call(qw, dim, N, dtype):
    plan, x, origin = _prepared(qw, dim, N, dtype)
    times = [7, 1000, 99999]
    print("async reductions: %dD %s %s" % (dim, N, dtype), flush=True)
    want = [plan.evolve_fft_observables(x, t, origin) for t in times]
    raws = [torch.full((qw.OBS_RAW_DOUBLES,), float("nan"), dtype=torch.float64,
                       pin_memory=True) for _ in times]
    outs = [plan.empty() for _ in times]
    for t, raw, out in zip(times, raws, outs):
        plan.evolve_fft_observables_async(x, t, origin, raw, out=out)
    torch.cuda.synchronize()
    for t, raw, out, w in zip(times, raws, outs, want):
        got = plan.obs_from_raw(raw, origin)
        assert got == w, t
        assert torch.equal(out, plan.evolve_fft(x, t)), t
    # the record alone (no field written), reused by a second call
    raw = raws[0]
    for t, w in zip(times, want):
        plan.evolve_fft_observables_async(x, t, origin, raw)
        torch.cuda.synchronize()
        assert plan.obs_from_raw(raw, origin) == w, t
    assert abs(want[0]["norm2"] - 1.0) < (1e-5 if dtype == "c64" else 1e-12)


def test_async_argument_checks(qw):
    import ctypes
    plan, x, origin = _prepared(qw, 3, 32, "c64")
    with pytest.raises(ValueError):
        plan.evolve_fft_observables_async(x, 5, origin, torch.zeros(qw.OBS_RAW_DOUBLES,
                                                                     dtype=torch.float64))
    with pytest.raises(ValueError):
        plan.evolve_fft_observables_async(x, 5, origin, torch.zeros(4, dtype=torch.float64,
                                                                     pin_memory=True))
    org = (ctypes.c_double * 3)(*origin)
    assert qw.LIB.qw_evolve_fft_observables_async(plan._h, ctypes.c_void_p(x.data_ptr()), None, 5,
                                                  org, None, None) == qw.QW_ERR_INVALID
    raw = torch.zeros(qw.OBS_RAW_DOUBLES, dtype=torch.float64, pin_memory=True)
    bad = (ctypes.c_double * 3)(float("nan"), 0.0, 0.0)
    assert qw.LIB.qw_evolve_fft_observables_async(plan._h, ctypes.c_void_p(x.data_ptr()), None, 5,
                                                  bad, ctypes.c_void_p(raw.data_ptr()),
                                                  None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_evolve_fft_observables_async(plan._h, ctypes.c_void_p(x.data_ptr()), None,
                                                  2 ** 60, org, ctypes.c_void_p(raw.data_ptr()),
                                                  None) == qw.QW_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert np.all(raw.numpy() == 0.0)  # rejected calls queue nothing
