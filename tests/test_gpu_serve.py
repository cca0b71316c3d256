"""Serving tier through the C ABI (qw_server_*): results against the FP64
oracle, bitwise independence of a request's result from what it was batched
with, admission under the byte budget, and argument errors."""
import math

import numpy as np
import pytest
import torch

from oracle import fourier, observables as ob, states, walk

pytestmark = pytest.mark.gpu

MiB = 1 << 20


@pytest.fixture(scope="module")
def qw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1603_06442_amd import qw as mod
    return mod


def req(d, N, m, k0, sigma, t, cp=1.0, cm=0.0, dtype="c64", center=None):
    return dict(dim=d, N=N, m=m, k0=k0, sigma=sigma,
                center=center if center is not None else [N // 2] * d,
                c_plus=cp, c_minus=cm, t=t, dtype=dtype)


def oracle_obs(r):
    d, N = r["dim"], r["N"]
    psi = states.particle_state(d, N, r["m"], r["k0"], r["sigma"], r["center"], r["c_plus"],
                                r["c_minus"])
    psit = fourier.evolve_fourier(psi, walk.stencil_table(d, r["m"]), r["t"])
    return ob.observables(psit, r["center"])


def run_all(server, reqs, hold=True):
    if hold:
        server.hold(True)
    tickets = [server.submit(**r) for r in reqs]
    if hold:
        server.hold(False)
    return [server.wait(tk) for tk in tickets]


MIX = [
    req(1, 1024, 0.1, [0.3], 10.0, 1000),
    req(1, 8192, 0.05, [-0.2], 40.0, 12345, 0.6, 0.8),          # four-step length
    req(2, 64, 0.2, [0.2, -0.1], 4.0, 77, 1 / math.sqrt(2), 1 / math.sqrt(2)),
    req(3, 16, 0.3, [0.1, 0.1, 0.1], 2.5, -40),
    req(3, 32, 0.1, [0.3, -0.2, 0.1], 3.0, 100000, 0.0, 1.0),
    req(1, 1024, 0.0, [0.1], 20.0, 333),                         # massless
    req(2, 64, 1.0, [0.0, 0.3], 6.0, 5),                         # m = 1: no hopping
    req(3, 16, 0.05, [-0.3, 0.0, 0.2], 2.0, 999, 1 / math.sqrt(2), 1 / math.sqrt(2)),
]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_server_results_match_oracle(qw, dtype):
    reqs = [dict(r, dtype=dtype) for r in MIX]
    srv = qw.Server(1 << 30, max_batch=4, nstreams=2)
    try:
        got = run_all(srv, reqs)
    finally:
        srv.close()
    for r, g in zip(reqs, got):
        assert g["status"] == qw.QW_OK
        want = oracle_obs(r)
        d = r["dim"]
        rt = 2e-4 if dtype == "c64" else 1e-9
        assert abs(g["obs"]["norm2"] - 1.0) < (5e-5 if dtype == "c64" else 1e-11)
        assert np.allclose(g["obs"]["mean"], want["mean"][:d], rtol=0, atol=rt * r["N"]), r
        assert np.allclose(g["obs"]["second"], want["second"], rtol=rt,
                           atol=rt * r["N"] ** 2 * 1e-2), r
        assert np.allclose(g["obs"]["mean_cart"], want["mean_cart"], rtol=0,
                           atol=rt * r["N"] * 2), r


def test_result_does_not_depend_on_the_batch_mix(qw):
    rng = np.random.default_rng(1234)
    reqs = []
    for i in range(24):
        d, N = [(3, 16), (3, 32), (1, 1024), (2, 64)][i % 4]
        reqs.append(req(d, N, float(rng.uniform(0, 0.3)), list(rng.uniform(-0.3, 0.3, d)),
                        float(rng.uniform(2.0, 4.0)), int(rng.integers(-5000, 5000)),
                        dtype="c64" if i % 3 else "c128"))
    alone_srv = qw.Server(1 << 30, max_batch=1, nstreams=1)
    try:
        alone = [run_all(alone_srv, [r], hold=False)[0] for r in reqs]
    finally:
        alone_srv.close()
    mix_srv = qw.Server(1 << 30, max_batch=8, nstreams=3)
    try:
        mixed = run_all(mix_srv, reqs)
        st = mix_srv.stats()
    finally:
        mix_srv.close()
    assert max(m["batch_size"] for m in mixed) > 1
    assert st["batches"] < len(reqs)
    # a batch's device layout never exceeds the footprints charged for it
    assert 0 < st["peak_laid_out_bytes"] <= st["peak_used_bytes"]
    assert st["laid_out_bytes"] == 0 and st["used_bytes"] == 0
    for a, m in zip(alone, mixed):
        assert a["status"] == m["status"] == qw.QW_OK
        assert a["batch_size"] == 1
        assert a["obs"] == m["obs"]                    # bitwise
        assert a["sector_norm2"] == m["sector_norm2"]


def test_admission_respects_the_budget(qw):
    # one 32^3 complex128 field is 2 MiB: a 3 MiB budget admits one at a time
    srv = qw.Server(3 * MiB, max_batch=8, nstreams=2)
    try:
        reqs = [req(3, 32, 0.1, [0.1, 0.0, -0.1], 3.0, 10 * i + 1, dtype="c128") for i in range(6)]
        got = run_all(srv, reqs)
        st = srv.stats()
        with pytest.raises(qw.QwError) as e:
            srv.submit(**req(3, 64, 0.1, [0.1, 0.0, -0.1], 3.0, 5, dtype="c128"))
        assert e.value.status == qw.QW_ERR_NOMEM
    finally:
        srv.close()
    assert all(g["status"] == qw.QW_OK for g in got)
    assert all(g["batch_size"] == 1 for g in got)
    assert st["batches"] == 6 and st["completed"] == 6
    assert 0 < st["peak_used_bytes"] <= 3 * MiB
    assert 0 < st["peak_laid_out_bytes"] <= st["peak_used_bytes"]
    assert st["used_bytes"] == 0 and st["queued"] == 0
    # queued behind memory: later requests wait for earlier ones
    lat = [g["latency_s"] for g in got]
    assert lat[-1] >= lat[0]


def test_requests_are_collected_once_and_bad_requests_rejected(qw):
    srv = qw.Server(64 * MiB, max_batch=4, nstreams=1)
    try:
        tk = srv.submit(**req(1, 1024, 0.1, [0.3], 10.0, 100))
        r = srv.wait(tk)
        assert r["status"] == qw.QW_OK and r["ticket"] == tk
        with pytest.raises(qw.QwError):
            srv.wait(tk)
        with pytest.raises(qw.QwError):
            srv.poll(tk + 100)
        bad = [
            (dict(N=48), qw.QW_ERR_UNSUPPORTED),
            (dict(sigma=0.0), qw.QW_ERR_INVALID),
            (dict(c_plus=0.0, c_minus=0.0), qw.QW_ERR_INVALID),
            (dict(m=1.5), qw.QW_ERR_INVALID),
        ]
        for change, status in bad:
            r = dict(req(1, 1024, 0.1, [0.3], 10.0, 100), **change)
            if "N" in change:
                r["center"] = [24]
            with pytest.raises(qw.QwError) as e:
                srv.submit(**r)
            assert e.value.status == status, change
        # a poll loop sees the request complete
        tk = srv.submit(**req(2, 64, 0.1, [0.1, 0.1], 5.0, 50))
        res = None
        for _ in range(100000):
            res = srv.poll(tk)
            if res is not None:
                break
        if res is None:
            res = srv.wait(tk)
        assert res["status"] == qw.QW_OK
    finally:
        srv.close()


def _mixed_requests(n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        d, N = [(3, 16), (3, 32), (1, 1024), (2, 64), (1, 8192)][i % 5]
        reqs.append(req(d, N, float(rng.uniform(0, 0.3)), list(rng.uniform(-0.3, 0.3, d)),
                        float(rng.uniform(2.0, 4.0)), int(rng.integers(-5000, 5000)),
                        dtype="c64" if i % 3 else "c128"))
    return reqs


def test_graph_replays_equal_the_direct_chain(qw):
    """With graphs, a (shape, precision, size) runs its chain directly until
    its second run, which captures it; later batches replay the capture with
    their own parameters. One request per batch, so every later request of a
    shape is a replay: 30 requests over five shapes (the 1D four-step among
    them) in both precisions, one at a time with eager GPU work and a
    synchronisation between them, then all at once on two streams. Every
    result is bitwise that of a server without graphs."""
    reqs = _mixed_requests(30, 4321)
    eager = qw.Server(1 << 30, max_batch=1, nstreams=1, graphs=False)
    try:
        want = [run_all(eager, [r], hold=False)[0] for r in reqs]
        st_e = eager.stats()
    finally:
        eager.close()
    assert st_e["graphs_captured"] == 0 and st_e["graph_launches"] == 0
    srv = qw.Server(1 << 30, max_batch=1, nstreams=2, graphs=True)
    try:
        one = []
        for r in reqs:
            one.append(run_all(srv, [r], hold=False)[0])
            x = torch.randn(4096, device="cuda")
            (x * 2.0).sum().item()
            torch.cuda.synchronize()
        burst = run_all(srv, reqs)
        st = srv.stats()
    finally:
        srv.close()
    shapes = {(r["dim"], r["N"], r["dtype"]) for r in reqs}
    # one at a time: each shape runs directly twice (capturing on the
    # second run), then replays; in the burst the first request of each shape
    # finds its graph idle (others may capture a second graph while it is busy)
    assert st["graphs_captured"] >= len(shapes)
    assert st["graph_launches"] >= len(reqs) - len(shapes)
    for w, a, b in zip(want, one, burst):
        assert w["status"] == a["status"] == b["status"] == qw.QW_OK
        assert a["obs"] == w["obs"] and b["obs"] == w["obs"]  # bitwise
        assert a["sector_norm2"] == w["sector_norm2"] == b["sector_norm2"]


def test_graph_slots_stay_within_their_limits(qw):
    """At most max_graphs captured graphs are kept, the least recently used
    dropped first, and their buffers stay within the budget."""
    reqs = _mixed_requests(40, 99)
    srv = qw.Server(64 * MiB, max_batch=1, nstreams=1, graphs=True, max_graphs=2)
    try:
        got = [run_all(srv, [r], hold=False)[0] for r in reqs]
        st = srv.stats()
    finally:
        srv.close()
    assert all(g["status"] == qw.QW_OK for g in got)
    assert 0 < st["slot_bytes"] <= 64 * MiB
    # ten (shape, precision) pairs in turn through two graphs: each recaptured
    assert st["graphs_captured"] >= 10
