"""CPU-side checks of the C-ABI library: it loads, and exports every entry
point that include/qw.h declares. No compute calls (no GPU here)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qw.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qw_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("qw_plan", "qw_step", "qw_evolve_fft", "qw_observables", "qw_destroy"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_1603_06442_amd import qw
    out = subprocess.run(["nm", "-D", "--defined-only", qw.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    assert set(qw.EXPORTS) <= exported


def test_library_loads_and_reports_version():
    from paper_1603_06442_amd import qw
    assert "gfx950" in qw.version()


def test_binding_validates_before_the_library():
    from paper_1603_06442_amd import qw
    with pytest.raises(ValueError):
        qw.Plan(3, [8, 8], 0.1)
    with pytest.raises(ValueError):
        qw.Plan(1, 16, 0.1, dtype="f16")


@pytest.mark.parametrize("dim,N,m,status", [
    (4, [8], 0.1, 1),            # dimension
    (0, [8], 0.1, 1),
    (1, [8], -0.1, 1),           # mass outside [0, 1]
    (1, [8], 1.5, 1),
    (1, [8], float("nan"), 1),
    (1, [12], 0.1, 2),           # not a power of two
    (1, [131072], 0.1, 2),       # beyond the 1D limit
    (2, [2048, 2048], 0.1, 2),   # beyond the 2D limit
    (3, [8, 8, 1024], 0.1, 2),   # beyond the 3D limit
    (3, [8, 0, 8], 0.1, 1),      # non-positive size
])
def test_plan_rejects_bad_arguments_on_the_host(dim, N, m, status):
    """Argument validation happens on the host, before any device call."""
    import ctypes
    from paper_1603_06442_amd import qw
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * len(N))(*N)
    got = qw.LIB.qw_plan(ctypes.byref(h), dim, arr, m, 0, None)
    assert got == status
    assert h.value is None
    assert qw.LIB.qw_last_error().decode()


def test_calls_reject_null_plan():
    import ctypes
    from paper_1603_06442_amd import qw
    assert qw.LIB.qw_step(None, ctypes.c_void_p(1), 1, None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_evolve_fft(None, None, None, 1, None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_evolve_fft_observables(None, None, None, 1, None, None, None) == \
        qw.QW_ERR_INVALID
    assert qw.LIB.qw_evolve_fft_observables_async(None, None, None, 1, None, None, None) == \
        qw.QW_ERR_INVALID
    assert qw.LIB.qw_obs_from_raw(None, None, None, None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_kspace_drift(None, None, None, None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_bcc_step(None, None, 1, None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_bcc_observables(None, None, None, None, None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_bcc_transform(None, None, None, 1, None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_bcc_evolve_fft(None, None, None, 1.0, None) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_destroy(None) == qw.QW_OK


def test_server_rejects_bad_arguments_on_the_host():
    import ctypes
    from paper_1603_06442_amd import qw
    h = ctypes.c_void_p()
    for budget, mb, ns in [(1000, 4, 1), (1 << 30, 0, 1), (1 << 30, 4, 0), (1 << 30, 5000, 1),
                           (1 << 30, 4, 17)]:
        assert qw.LIB.qw_server_create(ctypes.byref(h), budget, mb, ns) == qw.QW_ERR_INVALID
        assert h.value is None
    tk = ctypes.c_int64()
    assert qw.LIB.qw_server_submit(None, None, ctypes.byref(tk)) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_server_hold(None, 1) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_server_destroy(None) == qw.QW_OK


@pytest.mark.parametrize("d", [1, 2, 3])
def test_dispersion_taylor_matches_symbolic_derivatives(d):
    """The library's analytic Taylor coefficients of omega (host code, no
    GPU) against the oracle's symbolic differentiation."""
    from oracle import dispersive
    from paper_1603_06442_amd import qw
    m = 0.07
    k0 = [0.31, -0.22, 0.17][:d]
    got = qw.dispersion_taylor(d, m, k0, 2)
    want = dispersive.taylor_coefficients(d, m, k0, 2)
    names = {(0,) * d: 0}
    for i in range(d):
        a = [0] * d
        a[i] = 1
        names[tuple(a)] = 1 + i
        a[i] = 2
        names[tuple(a)] = 4 + i
    mixed = [(0, 1, 7), (0, 2, 8), (1, 2, 9)]
    for i, j, slot in mixed:
        if j < d:
            a = [0] * d
            a[i] = a[j] = 1
            names[tuple(a)] = slot
    for a, slot in names.items():
        assert abs(got[slot] - want[a]) < 1e-13 * max(1.0, abs(want[a])), (a, got[slot], want[a])
    for slot in range(10):
        if slot not in names.values():
            assert got[slot] == 0.0


def test_dispersion_taylor_rejects_bad_arguments():
    import ctypes
    from paper_1603_06442_amd import qw
    out = (ctypes.c_double * 10)()
    k = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    assert qw.LIB.qw_dispersion_taylor(4, 0.1, k, 1, out) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_dispersion_taylor(1, 1.5, k, 1, out) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_dispersion_taylor(1, 0.1, k, 3, out) == qw.QW_ERR_UNSUPPORTED
    # m = 0 at k0 = 0: sin omega = 0, omega not differentiable
    assert qw.LIB.qw_dispersion_taylor(3, 0.0, k, 1, out) == qw.QW_ERR_INVALID
    assert qw.LIB.qw_dispersion_taylor(3, 0.0, k, 0, out) == qw.QW_OK
