#!/usr/bin/env python3
"""Benchmark of the Dirac quantum-walk hot path on one MI355X.

Workload: the 3D walk on the BCC lattice stored as a 256^3 primitive-cell
torus, 4-component complex64 spinor (FP32 transforms and stencil, FP64
phase), m = 0.02, an equal-weight particle/antiparticle Gaussian state at
k0 = (0.1, 0.1, 0.1) with width 20 cells, prepared on the GPU. One timed
step is one pass over the whole hot path:
  * one Fourier jump psi_t = U^t psi_0 (t cycling through the 64 times
    log-spaced in [1, 1e5]) with the position/norm reduction of psi_t (the
    Zitterbewegung observable) taken inside its last inverse pass,
  * two position-space steps of a second field.
Each step's reductions reach the host through a pinned record
(qw_evolve_fft_observables_async) that is read while the next step runs, so
the GPU is not left idle during the read; the same steps with the host
waiting for each jump are timed beside them (ms_per_step_waiting).
`value` is steps per second, i.e. Fourier evolutions per second with the
reduction and the two stencil steps included in each. The JSON line also
carries the stencil's own site-steps/s, the roofline of the dominant kernel
measured with HIP events on the launch stream, and the FP64 CPU oracle timed
on a bounded sample.

The serving tier is measured beside it: 512 mixed requests through the
continuous-batching server (saturation throughput batched and unbatched,
p50/p99 latency under Poisson arrivals).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-serving] [--record RUNS.jsonl]
       python bench.py --copy-calib     (a plain copy of one field, for counters)
       python bench.py --counter-pass   (the hot kernels only, for counters)
--record (or QW_RUN_RECORD) appends the JSON line, with host, device, library
version and time, to a JSONL file: one record per run.
"""
import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_bcc256_c64.json")


def _source_hash(rel):
    """sha256 of a committed kernel source (to tell stale counter data)."""
    import hashlib
    if not rel:
        return None
    path = os.path.join(ROOT, rel)
    if not os.path.exists(path):
        return None
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def cpu_baseline(w, budget_s=15.0):
    """The FP64 oracle's Fourier evaluation as it stands (numpy DFT, per-q
    binary powering of the symbol summed from the transition matrices,
    inverse DFT; single-threaded numpy) on the workload's state on the 128^3
    torus (width scaled by 128/256), at times from the 1..1e5 schedule,
    timed on the host and scaled by (128/256)^3 to the 256^3 unit (the
    powering, which dominates, is linear in the volume; the FFT's log factor
    is left out). Beside it, as context: a forward + inverse FFT of the 256^3
    four-component field in complex128 with scipy.fft on all host cores,
    the least any host evaluation of one evolution must spend."""
    import numpy as np
    from oracle import fourier, states, walk
    Ns = 128
    table = walk.stencil_table(3, w["m"])
    psi = states.particle_state(3, Ns, w["m"], w["k0"], w["sigma"] * Ns / 256.0, [Ns // 2] * 3,
                                w["c_plus"], w["c_minus"])
    times = w["times"]
    done = 0
    t0 = time.perf_counter()
    while True:
        fourier.evolve_fourier(psi, table, times[(7 * done + 40) % len(times)])
        done += 1
        el = time.perf_counter() - t0
        if el > budget_s or done >= 16:
            break
    scale = (Ns / 256.0) ** 3
    out = {"value": done / el * scale, "unit": "evolutions/s", "cores": 1, "kind": "oracle",
           "sample": "%d oracle Fourier evolutions (numpy FFT + binary powering, complex128, "
                     "single thread) of the workload's state on the 128^3 torus at t from the "
                     "1..1e5 schedule in %.1f s, scaled by (128/256)^3 to the 256^3 unit"
                     % (done, el),
           "host_threads_available": os.cpu_count(), "cpu_model": _cpu_model()}
    # The oracle's position-space stepping (np.roll over the transition
    # matrices, complex128, one thread) on the 64^3 torus, as context for
    # the stencil's site-steps/s.
    from oracle import stepper
    from paper_1603_06442_amd.inputs import random_field
    f64 = random_field(np.random.default_rng(3), 3, 64, 4)
    t0 = time.perf_counter()
    nst = 0
    while nst < 64 and time.perf_counter() - t0 < 3.0:
        f64 = stepper.evolve_steps(f64, table, 2)
        nst += 2
    el = time.perf_counter() - t0
    out["context_stencil_oracle_64"] = {
        "site_steps_per_s": round(nst * 64 ** 3 / el, 1), "steps": nst, "seconds": round(el, 3),
        "cores": 1, "what": "oracle stepping (np.roll over the transition matrices, complex128, "
                            "single thread) on the 64^3 torus"}
    try:
        import scipy.fft as sfft
        nw = os.cpu_count() or 1
        x = (np.random.default_rng(0).standard_normal((4, 256, 256, 256)) + 0j)
        sfft.ifftn(x, axes=(1, 2, 3), workers=nw, overwrite_x=False)
        t0 = time.perf_counter()
        y = sfft.ifftn(x, axes=(1, 2, 3), workers=nw)
        sfft.fftn(y, axes=(1, 2, 3), workers=nw, overwrite_x=True)
        ft = time.perf_counter() - t0
        out["context_fft_roundtrip_256_c128"] = {
            "seconds": round(ft, 3), "workers": nw,
            "what": "scipy.fft forward + inverse of the 4 x 256^3 complex128 field on all "
                    "host cores (no apply): a lower bound for a host evolution"}
        del x, y
    except ImportError:
        pass
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def copy_calib(steps):
    import torch
    n = 4 * 256 ** 3
    x = torch.ones(n, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(steps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calib_bytes_read": 8 * n, "copy_calib_bytes_written": 8 * n,
                      "launches": steps}))


def counter_pass():
    """A short run of the hot kernels for hardware-counter passes: three
    Fourier jumps of the 256^3 workload with the fused reduction at the
    five-pass schedule (no slab grouping, so every pass is one whole-field
    launch), two single stencil steps and one two-step launch."""
    import torch
    from paper_1603_06442_amd import inputs, qw
    w = inputs.workload(2)
    plan = qw.Plan(3, w["N"], w["m"], "c64")
    plan.set_schedule(0, 4, 128, 4)
    x = plan.empty()
    plan.prepare_state(x, w["k0"], w["sigma"], w["center"], w["c_plus"], w["c_minus"])
    y = plan.empty()
    for i in range(3):
        plan.evolve_fft_observables(x, 1000 + i, w["center"], out=y)
        print("jump", i, flush=True)
    plan.step(y, 2)
    qw.set_step_kernel(True)
    try:
        plan.step(y, 2)
    finally:
        qw.set_step_kernel(False)
    torch.cuda.synchronize()
    print(json.dumps({"counter_pass": "done"}))


def _submit(srv, r):
    return srv.submit(dim=r["d"], N=r["N"], m=r["m"], k0=r["k0"], sigma=r["sigma"],
                      center=r["center"], c_plus=r["c_plus"], c_minus=r["c_minus"], t=r["t"],
                      dtype=r.get("dtype", "c64"))


def _burst(srv, reqs):
    """Submit everything while held, release, wait: makespan and results."""
    srv.hold(True)
    t0 = time.perf_counter()
    tks = [_submit(srv, r) for r in reqs]
    srv.hold(False)
    res = [srv.wait(tk) for tk in tks]
    return time.perf_counter() - t0, res


def _pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(math.ceil(q * len(xs))) - 1)]


def stencil_line(qw):
    """The 1D workload (N = 4096, two components, complex128, m = 0.1, 1000
    steps): one field alone, and 1024 instances with masses drawn in
    [0, 0.3] batched. Each field is 128 KB and is stepped on-chip."""
    import torch
    from paper_1603_06442_amd import inputs
    w = inputs.workload(0)
    N, steps, B = w["N"], w["steps"], 1024
    plan = qw.Plan(1, N, w["m"], "c128")
    x = plan.empty()
    plan.prepare_state(x, w["k0"], w["sigma"], w["center"], w["c_plus"], w["c_minus"])
    xb = x.unsqueeze(0).repeat(B, 1, 1).contiguous()
    rng = inputs.rng_for(0)
    ms = [float(v) for v in rng.uniform(0.0, 0.3, B)]
    plan.step(x.clone(), 10)
    plan.step_batched(xb, ms, 10)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    y = x.clone()
    e0.record(st)
    plan.step(y, steps)
    e1.record(st)
    e1.synchronize()
    one_ms = e0.elapsed_time(e1)
    e0.record(st)
    plan.step_batched(xb, ms, steps)
    e1.record(st)
    e1.synchronize()
    b_ms = e0.elapsed_time(e1)
    return {"workload": "1D N=4096 complex128 m=0.1, %d steps" % steps,
            "single_ms": round(one_ms, 4),
            "single_site_steps_per_s": round(N * steps / (one_ms * 1e-3), 1),
            "batched_instances": B, "batched_ms": round(b_ms, 4),
            "batched_site_steps_per_s": round(B * N * steps / (b_ms * 1e-3), 1)}


def _poisson(srv, reqs, gaps):
    """Open-loop arrivals: request i is submitted at sum(gaps[:i+1]) seconds
    (host clock); returns the results."""
    tks = []
    t0 = time.perf_counter()
    due = 0.0
    for r, gap in zip(reqs, gaps):
        due += gap
        while time.perf_counter() - t0 < due:
            pass
        tks.append(_submit(srv, r))
    return [srv.wait(tk) for tk in tks]


def _lat(res):
    lat = [1e3 * x["latency_s"] for x in res]
    return {"p50_latency_ms": round(_pct(lat, 0.50), 3), "p99_latency_ms": round(_pct(lat, 0.99), 3),
            "mean_batch": round(sum(x["batch_size"] for x in res) / len(res), 2)}


def serving(qw, budget_gib=16):
    """The mixed request stream (512 requests: 1D/2D/3D lattices, masses,
    states and times drawn per request) through the continuous-batching
    server, in three forms: batched complex64 with the batch chains replayed
    from captured HIP graphs (the serving form), the same without graphs,
    and the plain single-instance complex128 form (one request per batch, one
    stream, no graphs). Each form: saturation throughput of a burst of the
    512 requests (after a warm-up burst that builds and tunes the plans and
    captures the graphs), then open-loop Poisson arrivals at 70% of the
    serving form's saturation rate, the same arrival times for every form,
    for p50/p99 latency (submit to completion signalled by the stream), the
    stream run once unmeasured first so that the server is in its steady
    state; the plain form also at 70% of its own saturation rate. Last, the serving form
    under a 256 MiB budget, which makes requests wait for memory."""
    from paper_1603_06442_amd import inputs
    reqs = inputs.workload(3)["requests"]
    reqs128 = [dict(r, dtype="c128") for r in reqs]
    budget = budget_gib << 30
    forms = {"batched_c64_graphs": (reqs, 32, 4, True),
             "batched_c64_direct": (reqs, 32, 4, False),
             "single_c128_plain": (reqs128, 1, 1, False)}
    out = {"requests": len(reqs), "budget_bytes": budget}
    servers = {}
    bad = 0
    drift = 0.0
    try:
        sat = {}
        for name, (rq, mb, ns, gr) in forms.items():
            srv = qw.Server(budget, max_batch=mb, nstreams=ns, graphs=gr)
            servers[name] = srv
            _burst(srv, rq)  # plans, tuning, graphs
            st0 = srv.stats()
            el, res = _burst(srv, rq)
            st = srv.stats()
            nb = st["batches"] - st0["batches"]
            sat[name] = len(rq) / el
            bad += sum(1 for x in res if x["status"] != qw.QW_OK)
            drift = max(drift, max(abs(x["obs"]["norm2"] - 1.0) for x in res))
            out[name] = {"max_batch": mb, "streams": ns, "graphs": gr,
                         "saturation_requests_per_s": round(sat[name], 1),
                         "saturation_batches": nb,
                         "saturation_mean_batch": round(len(rq) / max(1, nb), 2),
                         "graph_launches": st["graph_launches"] - st0["graph_launches"],
                         "graphs_captured": st["graphs_captured"],
                         "peak_used_bytes": st["peak_used_bytes"]}
        rate = 0.7 * sat["batched_c64_graphs"]
        gaps = inputs.rng_for(3).exponential(1.0 / rate, len(reqs))
        out["poisson_rate_per_s"] = round(rate, 1)
        for name, (rq, mb, ns, gr) in forms.items():
            # one pass of the stream to reach the steady state (the batch sizes
            # Poisson arrivals form differ from a burst's: their chains are
            # captured here), then the measured pass
            st0 = servers[name].stats()
            _poisson(servers[name], rq, gaps)
            st1 = servers[name].stats()
            res = _poisson(servers[name], rq, gaps)
            st2 = servers[name].stats()
            bad += sum(1 for x in res if x["status"] != qw.QW_OK)
            nb = st2["batches"] - st1["batches"]
            out[name]["poisson"] = dict(
                _lat(res), batches=nb,
                graph_launches=st2["graph_launches"] - st1["graph_launches"],
                graphs_captured_warmup=st1["graphs_captured"] - st0["graphs_captured"],
                host_us_per_batch=round((st2["launch_host_ns"] - st1["launch_host_ns"]) / max(1, nb) / 1e3, 1))
        own = 0.7 * sat["single_c128_plain"]
        gaps128 = inputs.rng_for(3).exponential(1.0 / own, len(reqs))
        res = _poisson(servers["single_c128_plain"], reqs128, gaps128)
        bad += sum(1 for x in res if x["status"] != qw.QW_OK)
        out["single_c128_plain"]["poisson_own_rate"] = dict(_lat(res), rate_per_s=round(own, 1))
        small = qw.Server(256 << 20, max_batch=32, nstreams=4)
        try:
            _burst(small, reqs)
            els, ress = _burst(small, reqs)
            sst = small.stats()
        finally:
            small.close()
        bad += sum(1 for x in ress if x["status"] != qw.QW_OK)
        out["small_budget"] = {"budget_bytes": 256 << 20,
                               "requests_per_s": round(len(reqs) / els, 1),
                               "peak_used_bytes": sst["peak_used_bytes"],
                               "slot_bytes": sst["slot_bytes"]}
        out["failed"] = bad
        out["max_norm_drift"] = drift
        # the serving form's figures at the top level of the section
        out["p50_latency_ms"] = out["batched_c64_graphs"]["poisson"]["p50_latency_ms"]
        out["p99_latency_ms"] = out["batched_c64_graphs"]["poisson"]["p99_latency_ms"]
        out["saturation_requests_per_s"] = out["batched_c64_graphs"]["saturation_requests_per_s"]
        return out
    finally:
        for srv in servers.values():
            srv.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--record", default=os.environ.get("QW_RUN_RECORD"),
                    help="append the JSON line with host/device/time to this JSONL file")
    ap.add_argument("--counter-pass", action="store_true",
                    help="short run of the hot kernels only, for rocprofv3 --pmc")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calib:
        copy_calib(max(1, args.steps))
        return
    if args.counter_pass:
        counter_pass()
        return
    from paper_1603_06442_amd import inputs, qw

    w = inputs.workload(2)
    N = w["N"]
    torch.cuda.set_device(0)
    plan = qw.Plan(3, N, w["m"], "c64")
    psi0 = plan.empty()
    plan.prepare_state(psi0, w["k0"], w["sigma"], w["center"], w["c_plus"], w["c_minus"])
    psit = plan.empty()
    psis = psi0.clone()
    tuned_ms = plan.autotune()
    schedule = plan.schedule()
    times = w["times"]
    V = N ** 3
    field_bytes = psi0.numel() * psi0.element_size()

    # Each step queues its jump, whose reductions a copy leaves in a pinned
    # record (qw_evolve_fft_observables_async), and its two stencil steps,
    # then reads the previous step's record, complete by then: the GPU is
    # not left idle while the host waits for a result.
    raws = [torch.empty(qw.OBS_RAW_DOUBLES, dtype=torch.float64, pin_memory=True)
            for _ in range(2)]
    done = [torch.cuda.Event() for _ in range(2)]

    def step(i):
        k = i & 1
        plan.evolve_fft_observables_async(psi0, times[i % len(times)], w["center"], raws[k],
                                          out=psit)
        done[k].record()
        plan.step(psis, 2)
        if i == 0:
            return None
        done[k ^ 1].synchronize()
        return plan.obs_from_raw(raws[k ^ 1], w["center"])

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    obs = plan.obs_from_raw(raws[(args.steps - 1) & 1], w["center"])  # the last step's
    el = time.perf_counter() - t0
    ms_per_step = 1e3 * el / args.steps

    # The same steps with the host waiting for each jump's reductions.
    def step_waiting(i):
        o = plan.evolve_fft_observables(psi0, times[i % len(times)], w["center"], out=psit)
        plan.step(psis, 2)
        return o

    if step_waiting(args.steps - 1) != obs:
        raise RuntimeError("reductions read back late differ from the waiting call's")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step_waiting(i)
    torch.cuda.synchronize()
    ms_per_step_waiting = 1e3 * (time.perf_counter() - t0) / args.steps

    # Per-kernel durations, HIP events on the launch stream.
    reps = 10
    acc = None
    for r in range(reps):
        _, ms = plan.evolve_fft_timed(psi0, times[(5 * r) % len(times)], out=psit)
        acc = ms if acc is None else [a + b for a, b in zip(acc, ms)]
    pass_ms = [a / reps for a in acc]
    if len(pass_ms) == 5:
        names = ["fft_strided n1 fwd", "fft_strided n2 fwd", "fft_contig n3 fwd+apply+inv",
                 "fft_strided n2 inv", "fft_strided n1 inv"]
        launches = [1, 1, 1, 1, 1]
    else:
        nslab = -(-N // schedule[0])
        names = ["fft_strided n1 fwd",
                 "slabs: fft_strided n2 fwd + fft_contig n3 fwd+apply+inv + fft_strided n2 inv",
                 "fft_strided n1 inv"]
        launches = [1, 3 * nslab, 1]
    # Each pass against HBM peak: algorithmic bytes = the field read and
    # written once (2 s V b), plus the 8 V bytes of the omega table that the
    # fused n3 pass reads.
    pass_roofline = {}
    if len(pass_ms) == 5:
        for n, v in zip(names, pass_ms):
            nbytes = 2 * field_bytes + (8 * V if n.startswith("fft_contig") else 0)
            gbs = nbytes / (v * 1e-3) / 1e9
            pass_roofline[n] = {"bytes": nbytes, "GB/s": round(gbs, 1),
                                "frac": round(gbs / PEAK_HBM_GBS, 4)}
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def stencil_pair_ms():
        """Time of plan.step(psis, 2) on the launch stream (HIP events)."""
        plan.step(psis, 2)
        e0.record(st)
        for _ in range(reps):
            plan.step(psis, 2)
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    # The two steps of a timed step, one launch each (the default); the
    # two-step kernel (psi read and written once per pair) beside it.
    single_ms = stencil_pair_ms() / 2
    qw.set_step_kernel(True)
    pair_ms = stencil_pair_ms()
    qw.set_step_kernel(False)
    e0.record(st)
    for _ in range(reps):
        plan.observables(psit, w["center"])
    e1.record(st)
    e1.synchronize()
    obs_ms = e0.elapsed_time(e1) / reps  # includes the small D2H copy and host wait
    evo_ms = sum(pass_ms)

    # Dominant kernel of a step: the one with the largest time per step among
    # single kernels (the slab group is several kernels and is not a
    # candidate). Algorithmic bytes per launch: 2 s b per site-step, i.e. one
    # read and one write of the field per Fourier pass and per stencil step
    # (two per launch of the two-step kernel).
    cands = [("k_step3d_ring (stencil step)", single_ms, 2, 2 * field_bytes)]
    for n, v, k in zip(names, pass_ms, launches):
        if k == 1:
            cands.append((n, v, 1, 2 * field_bytes))
    dom_name, dom_ms, dom_launches, alg_bytes = max(cands, key=lambda c: c[1] * c[2])
    achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        ent = tr.get("kernels", {}).get(dom_name)
        if ent and ent.get("source_sha256") == _source_hash(ent.get("source")):
            traffic = ent.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                "kernel": dom_name, "kernel_ms": round(dom_ms, 4), "launches_per_step": dom_launches,
                "algorithmic_bytes_per_launch": alg_bytes}

    line = {
        "metric": "lattice site-steps/s and FFT evolutions/s at 256^3 4-spinor; p99 request latency",
        "value": round(1e3 / ms_per_step, 3),
        "unit": "hot-path steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": "bcc256_zb: 3D Dirac walk, 256^3 BCC primitive-cell torus, "
                               "4-spinor complex64, m=0.02, particle+antiparticle Gaussian "
                               "k0=(0.1,0.1,0.1) sigma=20, t over 64 log-spaced times in [1,1e5]",
                   "step": "one hot-path step = 1 Fourier jump psi_t = U^t psi_0 with the "
                           "<x>/norm reduction fused into its last pass + 2 stencil steps of a "
                           "second field, each step's reductions read by the host while the next "
                           "step runs (qw_evolve_fft_observables_async; ms_per_step_waiting: "
                           "the host waiting for each jump's); value = such steps per second "
                           "(wall clock)",
                   "lattice": [N, N, N], "spinor": 4, "global_batch": 1},
        "ms_per_step_waiting": round(ms_per_step_waiting, 4),
        "fft_evolutions_per_s_kernels": round(1e3 / evo_ms, 2),
        "schedule": {"slab_planes": schedule[0], "contig_elems": schedule[1],
                     "contig_threads": schedule[2], "contig_groups": schedule[3],
                     "autotune_ms_per_evolution": round(tuned_ms, 4)},
        "fft_pass_ms": {n: round(v, 4) for n, v in zip(names, pass_ms)},
        "fft_pass_roofline": pass_roofline,
        "stencil_site_steps_per_s": round(V / (single_ms * 1e-3), 1),
        "stencil_ms_per_step": round(single_ms, 4),
        "stencil_gbs": round(2 * field_bytes / (single_ms * 1e-3) / 1e9, 1),
        "stencil_two_step_kernel": {"ms_per_launch": round(pair_ms, 4),
                                    "site_steps_per_s": round(2 * V / (pair_ms * 1e-3), 1),
                                    "used": False},
        "observables_ms": round(obs_ms, 4),
        "roofline": roofline,
        "last_obs": {"norm2": obs["norm2"], "mean_cart": obs["mean_cart"]},
    }
    # Accuracy beside the speed: the complex64 path (FP32 transforms, FP64
    # phase) against the complex128 GPU path on the same state, at the
    # largest time of the schedule; norm drift of both.
    p128 = qw.Plan(3, N, w["m"], "c128")
    p128.autotune()
    x128 = p128.empty()
    p128.prepare_state(x128, w["k0"], w["sigma"], w["center"], w["c_plus"], w["c_minus"])
    tmax = times[-1]
    y128 = p128.evolve_fft(x128, tmax)
    y64 = plan.evolve_fft(psi0, tmax, out=psit)
    _, ms128 = p128.evolve_fft_timed(x128, tmax, out=y128)
    diff = (y64.to(torch.complex128) - y128)
    rel = float(torch.linalg.vector_norm(diff) / torch.linalg.vector_norm(y128))
    line["accuracy"] = {
        "t": tmax, "c64_vs_c128_rel_l2": rel,
        "c128_ms_per_evolution": round(sum(ms128), 4),
        "c128_fused_pass_ms": round(ms128[2], 4) if len(ms128) == 5 else None,
        "norm_drift_c64": abs(plan.observables(y64, w["center"])["norm2"] - 1.0),
        "norm_drift_c128": abs(p128.observables(y128, w["center"])["norm2"] - 1.0)}
    # The whole <x>(t) series of the workload in one call (the spectrum of
    # psi0 taken once, three passes per time), in both precisions, against
    # the per-time fused jumps at a few times.
    line["zb_series"] = {}
    for name, pl, xs in (("c64", plan, psi0), ("c128", p128, x128)):
        pl.evolve_fft_series(xs, times[:4], w["center"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ser = pl.evolve_fft_series(xs, times, w["center"])
        el = time.perf_counter() - t0
        dev = 0.0
        for i in (0, len(times) // 2, len(times) - 1):
            o = pl.evolve_fft_observables(xs, times[i], w["center"])
            dev = max(dev, max(abs(a - b) for a, b in zip(ser[i]["mean"], o["mean"])))
        line["zb_series"][name] = {
            "times": len(times), "ms_per_series": round(1e3 * el, 3),
            "ms_per_time": round(1e3 * el / len(times), 4),
            "evolutions_per_s": round(len(times) / el, 1),
            "max_mean_dev_vs_fused_jump": dev}
    del p128, x128, y128, diff
    # Proposition 1 beside the exact jump: the order-2 dispersive state at
    # t = 100 (one state preparation with the phases and one inverse
    # transform) and its overlap with the exact evolution of the same state.
    tdisp = 100
    approx = plan.empty()
    plan.evolve_dispersive(approx, w["k0"], w["sigma"], w["center"], w["c_plus"], w["c_minus"],
                           2, float(tdisp))
    exact = plan.evolve_fft(psi0, tdisp, out=psit)
    fid = abs(plan.observables(exact, w["center"], ref=approx)["overlap"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        plan.evolve_dispersive(approx, w["k0"], w["sigma"], w["center"], w["c_plus"],
                               w["c_minus"], 2, float(tdisp))
    disp_ms = 1e3 * (time.perf_counter() - t0) / 5
    line["dispersive"] = {"order": 2, "t": tdisp, "ms_per_state": round(disp_ms, 4),
                          "overlap_with_exact": fid}
    del approx, exact

    # The other widened operations on the same field (wall time per call,
    # including the host wait of the calls that return values).
    def wall(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return round(1e3 * (time.perf_counter() - t0) / reps, 4)

    line["more_ops_ms"] = {
        "evolve_fft_real_t_1000.5": wall(lambda: plan.evolve_fft_real(psi0, 1000.5, out=psit)),
        "newton_wigner": wall(lambda: plan.newton_wigner(psi0, w["center"])),
        "marginals": wall(lambda: plan.marginals(psi0, [int(x) for x in w["center"]])),
        "kspace_drift": wall(lambda: plan.kspace_drift(psi0)),
        "evolve_fft_observables": wall(lambda: plan.evolve_fft_observables(
            psi0, 1000, w["center"], out=psit)),
    }
    line["workload_512"] = workload512_line(qw)
    line["cubic_supercell"] = cubic_line(qw, [N, N, N], w["m"], wall)
    line["weyl"] = weyl_line(qw, [N, N, N], wall)
    line["stencil_1d"] = stencil_line(qw)
    if not args.no_serving:
        line["serving"] = serving(qw)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line))
    if args.record:
        # one JSON record per run, appended: the line plus where and when it ran
        rec = dict(line)
        rec["record"] = {"unix_time": round(time.time(), 1), "host": platform.node(),
                         "device": torch.cuda.get_device_name(0),
                         "library": qw.version(), "argv": sys.argv[1:]}
        with open(args.record, "a") as f:
            f.write(json.dumps(rec) + "\n")


def workload512_line(qw):
    """The 512^3 workload (m = 0.1, particle state of width 40 cells about
    the centre, k0 from its seed, t = 1e6): one Fourier jump in complex64
    (FP32 transforms, FP64 phase; 4.3 GB per field) and one in complex128
    (8.6 GB) of the same state, with the time of each (HIP events), the
    complex64 result's relative L2 distance and infidelity 1 - |<psi64|psi128>|
    against the complex128 one, and both norm drifts."""
    import torch
    from paper_1603_06442_amd import inputs
    w = inputs.workload(4)
    N, t = w["N"], w["t"]
    out = {"lattice": [N, N, N], "t": t, "m": w["m"], "sigma": w["sigma"]}
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    res = {}
    for dtype in ("c64", "c128"):
        plan = qw.Plan(3, N, w["m"], dtype)
        # the schedules the autotuner picks at 256^3 (tuning at 512^3 would
        # launch several thousand candidate passes)
        plan.set_schedule(0, 4, 128 if dtype == "c64" else 64, 4 if dtype == "c64" else 1)
        x = plan.empty()
        plan.prepare_state(x, w["k0"], w["sigma"], w["center"], w["c_plus"], w["c_minus"])
        y = plan.empty()
        plan.evolve_fft(x, t, out=y)
        e0.record(st)
        for _ in range(3):
            plan.evolve_fft(x, t, out=y)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 3
        drift = abs(plan.observables(y, w["center"])["norm2"] - 1.0)
        out[dtype] = {"ms_per_evolution": round(ms, 4), "norm_drift": drift,
                      "field_bytes": y.numel() * y.element_size()}
        res[dtype] = (plan, y)
        del x
    p128, y128 = res["c128"]
    y64 = res["c64"][1].to(torch.complex128)
    rel = float(torch.linalg.vector_norm(y64 - y128) / torch.linalg.vector_norm(y128))
    o = p128.observables(y64, w["center"], ref=y128)
    fid = abs(o["overlap"]) / math.sqrt(o["norm2"] * o["ref_norm2"])
    out["c64_vs_c128_rel_l2"] = rel
    out["c64_infidelity"] = 1.0 - fid
    del res, p128, y128, y64
    torch.cuda.empty_cache()
    return out


def cubic_line(qw, N, m, wall):
    """The paper's cubic-supercell representation of the BCC lattice: two
    sublattice arrays of the workload's size (2 N^3 sites, Cartesian torus of
    period 2N), one Fourier jump (three passes of the two arrays as eight
    planes, the a_k combine, both frequencies and the recombination fused into
    the pass along n3), the two-sublattice transform alone, the time per
    position-space step and the Cartesian position moments."""
    import torch
    plan = qw.Plan(3, N, m, "c64")
    f = torch.randn((2, 4) + tuple(N), dtype=torch.complex64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(5))
    f /= torch.linalg.vector_norm(f)
    g = torch.empty_like(f)
    sites = 2 * N[0] * N[1] * N[2]
    ev = wall(lambda: plan.bcc_evolve_fft(f, 1000, out=g), reps=10)
    out = {"sublattice": list(N), "sites": sites, "t": 1000,
           "ms_per_evolution": ev,
           "site_evolutions_per_s": round(sites / (ev * 1e-3), 1),
           "transform_ms": wall(lambda: plan.bcc_transform(f, 1, out=g), reps=10),
           # two steps per call: an even count ends in the caller's buffer
           "ms_per_step": round(wall(lambda: plan.bcc_step(g, 2), reps=10) / 2, 4),
           "observables_ms": wall(lambda: plan.bcc_observables(f, [256.0, 256.0, 256.0]), reps=10),
           "norm_after": float(torch.linalg.vector_norm(plan.bcc_evolve_fft(f, 1000, out=g)))}
    del f, g, plan
    return out


def weyl_line(qw, N, wall):
    """The two-component Weyl walk on the workload's lattice (complex64):
    one Fourier jump and the time per position-space step."""
    import torch
    plan = qw.Plan(3, N, 0.0, "c64", weyl=True)
    x = torch.randn((2,) + tuple(N), dtype=torch.complex64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(6))
    x /= torch.linalg.vector_norm(x)
    y = torch.empty_like(x)
    V = N[0] * N[1] * N[2]
    ev = wall(lambda: plan.evolve_fft(x, 1000, out=y), reps=10)
    # two steps per call: an even count ends in the caller's buffer (no copy back)
    st = round(wall(lambda: plan.step(y, 2), reps=10) / 2, 4)
    out = {"lattice": list(N), "spinor": 2, "ms_per_evolution": ev, "ms_per_step": st,
           "step_gbs": round(2 * 2 * 8 * V / (st * 1e-3) / 1e9, 1)}
    del x, y, plan
    return out


if __name__ == "__main__":
    main()
