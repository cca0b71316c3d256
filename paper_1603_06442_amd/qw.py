"""Python binding of libqw (ctypes). Argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory
and the current stream. The names mirror the C ABI of include/qw.h:
``Plan`` wraps qw_plan / qw_destroy, and its methods call qw_step,
qw_evolve_fft, qw_evolve_fft_batched, qw_transform, qw_observables and
qw_prepare_state. ``Server`` wraps the continuous-batching server
(qw_server_create / submit / poll / wait / stats / destroy).

Importing this module loads libqw.so and fails loudly if it is missing.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqw.so")

QW_OK, QW_ERR_INVALID, QW_ERR_UNSUPPORTED, QW_ERR_NOMEM, QW_ERR_DEVICE, QW_ERR_CANCELLED = range(6)
QW_C64, QW_C128 = 0, 1
OBS_RAW_DOUBLES = 13  # QW_OBS_RAW_DOUBLES
DTYPES = {"c64": (QW_C64, torch.complex64), "c128": (QW_C128, torch.complex128)}
EXPORTS = ("qw_plan", "qw_plan_weyl", "qw_destroy", "qw_step", "qw_step_noalloc",
           "qw_step_batched", "qw_evolve_fft", "qw_evolve_fft_real", "qw_evolve_fft_batched",
           "qw_evolve_fft_timed", "qw_transform", "qw_observables", "qw_evolve_fft_observables",
           "qw_evolve_fft_observables_async", "qw_obs_from_raw", "qw_evolve_fft_series", "qw_newton_wigner",
           "qw_marginals", "qw_bcc_transform", "qw_bcc_evolve_fft", "qw_bcc_step", "qw_bcc_observables",
           "qw_kspace_drift",
           "qw_prepare_state", "qw_evolve_dispersive", "qw_dispersion_taylor",
           "qw_set_schedule", "qw_get_schedule", "qw_set_step_kernel", "qw_set_fft_kernel",
           "qw_autotune",
           "qw_last_error", "qw_version",
           "qw_server_create", "qw_server_configure", "qw_server_submit", "qw_server_poll", "qw_server_wait",
           "qw_server_cancel", "qw_server_wait_for",
           "qw_server_hold", "qw_server_stats", "qw_server_destroy")


class QwError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("qw status %d: %s" % (status, message))
        self.status = status


class QwDrift(ctypes.Structure):
    _fields_ = [("velocity", ctypes.c_double * 3), ("velocity_cart", ctypes.c_double * 3),
                ("sector_norm2", ctypes.c_double * 2), ("norm2", ctypes.c_double)]


class QwObs(ctypes.Structure):
    _fields_ = [("norm2", ctypes.c_double), ("mean", ctypes.c_double * 3),
                ("second", ctypes.c_double * 6), ("mean_cart", ctypes.c_double * 3),
                ("overlap_re", ctypes.c_double), ("overlap_im", ctypes.c_double),
                ("ref_norm2", ctypes.c_double)]


class QwRequest(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("N", ctypes.c_int64 * 3), ("m", ctypes.c_double),
                ("dtype", ctypes.c_int), ("k0", ctypes.c_double * 3), ("sigma", ctypes.c_double),
                ("center", ctypes.c_double * 3), ("c_plus", ctypes.c_double),
                ("c_minus", ctypes.c_double), ("t", ctypes.c_int64)]


class QwResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int), ("batch_size", ctypes.c_int),
                ("queue_s", ctypes.c_double), ("latency_s", ctypes.c_double), ("obs", QwObs),
                ("sector_norm2", ctypes.c_double * 2)]


class QwServerInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted", "completed", "batches", "queued", "inflight_batches",
        "max_inflight_batches", "used_bytes", "peak_used_bytes", "laid_out_bytes",
        "peak_laid_out_bytes", "graphs_captured", "graph_launches", "slot_bytes",
        "launch_host_ns", "budget_bytes", "cancelled")]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqw.so is not built (%s): run "
                          "python -m paper_1603_06442_amd.build" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, cint = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    sig = {
        "qw_plan": [ctypes.POINTER(vp), cint, ctypes.POINTER(i64), dbl, cint, vp],
        "qw_plan_weyl": [ctypes.POINTER(vp), cint, ctypes.POINTER(i64), cint, vp],
        "qw_destroy": [vp],
        "qw_step": [vp, vp, i64, vp],
        "qw_step_batched": [vp, cint, vp, ctypes.POINTER(dbl), i64, vp],
        "qw_step_noalloc": [vp, vp, i64, vp],
        "qw_evolve_fft": [vp, vp, vp, i64, vp],
        "qw_evolve_fft_real": [vp, vp, vp, dbl, vp],
        "qw_evolve_fft_timed": [vp, vp, vp, i64, vp, ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(cint)],
        "qw_evolve_fft_batched": [vp, cint, vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), vp],
        "qw_transform": [vp, vp, vp, cint, vp],
        "qw_bcc_transform": [vp, vp, vp, cint, vp],
        "qw_bcc_evolve_fft": [vp, vp, vp, dbl, vp],
        "qw_bcc_step": [vp, vp, i64, vp],
        "qw_bcc_observables": [vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(QwObs), vp],
        "qw_kspace_drift": [vp, vp, ctypes.POINTER(QwDrift), vp],
        "qw_observables": [vp, vp, ctypes.POINTER(dbl), vp, ctypes.POINTER(QwObs), vp],
        "qw_newton_wigner": [vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(QwObs), ctypes.POINTER(dbl),
                             vp],
        "qw_marginals": [vp, vp, ctypes.POINTER(i64), ctypes.POINTER(dbl), i64,
                         ctypes.POINTER(i64), ctypes.POINTER(i64), vp],
        "qw_evolve_fft_observables": [vp, vp, vp, i64, ctypes.POINTER(dbl),
                                      ctypes.POINTER(QwObs), vp],
        "qw_evolve_fft_observables_async": [vp, vp, vp, i64, ctypes.POINTER(dbl), vp, vp],
        "qw_obs_from_raw": [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(QwObs)],
        "qw_prepare_state": [vp, vp, ctypes.POINTER(dbl), dbl, ctypes.POINTER(dbl), dbl, dbl, vp],
        "qw_evolve_dispersive": [vp, vp, ctypes.POINTER(dbl), dbl, ctypes.POINTER(dbl), dbl, dbl,
                                 cint, dbl, vp],
        "qw_dispersion_taylor": [cint, dbl, ctypes.POINTER(dbl), cint, ctypes.POINTER(dbl)],
        "qw_set_schedule": [vp, cint, cint, cint, cint],
        "qw_set_step_kernel": [cint, cint, cint],
        "qw_set_fft_kernel": [cint],
        "qw_get_schedule": [vp, ctypes.POINTER(cint), ctypes.POINTER(cint), ctypes.POINTER(cint),
                            ctypes.POINTER(cint)],
        "qw_autotune": [vp, vp, ctypes.POINTER(dbl)],
        "qw_server_create": [ctypes.POINTER(vp), ctypes.c_size_t, cint, cint],
        "qw_server_configure": [vp, cint, cint, cint],
        "qw_server_submit": [vp, ctypes.POINTER(QwRequest), ctypes.POINTER(i64)],
        "qw_server_poll": [vp, i64, ctypes.POINTER(QwResult), ctypes.POINTER(cint)],
        "qw_server_wait": [vp, i64, ctypes.POINTER(QwResult)],
        "qw_server_cancel": [vp, i64, ctypes.POINTER(cint)],
        "qw_evolve_fft_series": [vp, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                 ctypes.POINTER(QwObs), vp],
        "qw_server_wait_for": [vp, i64, dbl, ctypes.POINTER(QwResult), ctypes.POINTER(cint)],
        "qw_server_hold": [vp, cint],
        "qw_server_stats": [vp, ctypes.POINTER(QwServerInfo)],
        "qw_server_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = cint
    lib.qw_last_error.restype = ctypes.c_char_p
    lib.qw_last_error.argtypes = []
    lib.qw_version.restype = ctypes.c_char_p
    lib.qw_version.argtypes = []
    return lib


LIB = _load()


def _check(status):
    if status != QW_OK:
        raise QwError(status, LIB.qw_last_error().decode())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _darr(vals, n):
    vals = [float(v) for v in vals]
    if len(vals) != n:
        raise ValueError("expected %d values, got %d" % (n, len(vals)))
    return (ctypes.c_double * n)(*vals)


class Plan:
    """A lattice shape, mass and precision (qw_plan)."""

    def __init__(self, dim, N, m, dtype="c64", stream=None, weyl=False):
        """weyl=True: the two-component Weyl walk (qw_plan_weyl; m must be 0)."""
        if weyl and float(m) != 0.0:
            raise ValueError("the Weyl walk is massless (m = 0)")
        if dtype not in DTYPES:
            raise ValueError("dtype must be 'c64' or 'c128'")
        self.dim = int(dim)
        Ns = [int(N)] * self.dim if isinstance(N, int) else [int(x) for x in N]
        if len(Ns) != self.dim:
            raise ValueError("need %d lattice sizes" % self.dim)
        self.N = tuple(Ns)
        self.m = float(m)
        self.dtype = dtype
        self.weyl = bool(weyl)
        self.s = 2 if (self.dim == 1 or self.weyl) else 4
        self.torch_dtype = DTYPES[dtype][1]
        self.shape = (self.s,) + self.N
        self._h = ctypes.c_void_p()
        arr = (ctypes.c_int64 * self.dim)(*Ns)
        if self.weyl:
            _check(LIB.qw_plan_weyl(ctypes.byref(self._h), self.dim, arr, DTYPES[dtype][0],
                                    _stream(stream)))
        else:
            _check(LIB.qw_plan(ctypes.byref(self._h), self.dim, arr, self.m, DTYPES[dtype][0],
                               _stream(stream)))

    def close(self):
        if self._h is not None and self._h.value:
            LIB.qw_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------
    def empty(self, batch=None, device="cuda"):
        shape = self.shape if batch is None else (batch,) + self.shape
        return torch.empty(shape, dtype=self.torch_dtype, device=device)

    def _field(self, x, batch=1, name="field"):
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError("%s must be a CUDA (HIP) tensor" % name)
        if x.dtype != self.torch_dtype:
            raise TypeError("%s has dtype %s, plan needs %s" % (name, x.dtype, self.torch_dtype))
        if not x.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        want = batch * self.s
        for n in self.N:
            want *= n
        if x.numel() != want:
            raise ValueError("%s has %d elements, expected %d" % (name, x.numel(), want))
        return ctypes.c_void_p(x.data_ptr())

    # -- C ABI calls ----------------------------------------------------------
    def step(self, psi, nsteps, stream=None):
        """qw_step: nsteps position-space steps, in place."""
        _check(LIB.qw_step(self._h, self._field(psi, name="psi"), int(nsteps), _stream(stream)))
        return psi

    def step_noalloc(self, psi, nsteps, stream=None):
        """qw_step_noalloc: qw_step with the library's fixed per-device
        buffer (allocates nothing; fields up to 64 MiB)."""
        _check(LIB.qw_step_noalloc(self._h, self._field(psi, name="psi"), int(nsteps),
                                   _stream(stream)))
        return psi

    def step_batched(self, psi, m, nsteps, stream=None):
        """qw_step_batched: nsteps steps of B = len(m) fields (shape (B,) +
        self.shape, contiguous) in place, instance b with mass m[b]."""
        B = len(m)
        _check(LIB.qw_step_batched(self._h, B, self._field(psi, batch=B, name="psi"),
                                   _darr(m, B), int(nsteps), _stream(stream)))
        return psi

    def evolve_fft(self, psi0, t, out=None, stream=None):
        """qw_evolve_fft: U^t psi0 by one Fourier jump (out may be psi0)."""
        if out is None:
            out = torch.empty_like(psi0)
        _check(LIB.qw_evolve_fft(self._h, self._field(psi0, name="psi0"),
                                 self._field(out, name="out"), int(t), _stream(stream)))
        return out

    def evolve_fft_timed(self, psi0, t, out=None, stream=None):
        """qw_evolve_fft_timed: the jump plus the duration (ms) of each pass."""
        if out is None:
            out = torch.empty_like(psi0)
        ms = (ctypes.c_float * 8)()
        n = ctypes.c_int(0)
        _check(LIB.qw_evolve_fft_timed(self._h, self._field(psi0, name="psi0"),
                                       self._field(out, name="out"), int(t), _stream(stream), ms,
                                       ctypes.byref(n)))
        return out, [ms[i] for i in range(n.value)]

    def evolve_fft_batched(self, x, m, t, out=None, stream=None):
        """qw_evolve_fft_batched over x[B, s, N..]: per-instance mass and time."""
        B = int(x.shape[0])
        if out is None:
            out = torch.empty_like(x)
        ma = (ctypes.c_double * B)(*[float(v) for v in m])
        ta = (ctypes.c_int64 * B)(*[int(v) for v in t])
        _check(LIB.qw_evolve_fft_batched(self._h, B, self._field(x, B, "x"),
                                         self._field(out, B, "out"), ma, ta, _stream(stream)))
        return out

    def transform(self, x, direction, out=None, stream=None):
        """qw_transform: unnormalised DFT, +1 = e^{+iq.n} forward, -1 inverse."""
        if out is None:
            out = torch.empty_like(x)
        _check(LIB.qw_transform(self._h, self._field(x, name="x"), self._field(out, name="out"),
                                int(direction), _stream(stream)))
        return out

    # -- cubic-supercell BCC field (3D plans): shape (2, s, N1, N2, N3) --------
    def bcc_transform(self, f, direction, out=None, stream=None):
        """qw_bcc_transform: +1 = (hat f0, hat f1) of the two-sublattice DFT,
        -1 = its inverse; f holds the two sublattice arrays back to back."""
        if out is None:
            out = torch.empty_like(f)
        _check(LIB.qw_bcc_transform(self._h, self._field(f, 2, "f"), self._field(out, 2, "out"),
                                    int(direction), _stream(stream)))
        return out

    def bcc_step(self, f, nsteps, stream=None):
        """qw_bcc_step: nsteps position-space steps on the cubic supercell, in place."""
        _check(LIB.qw_bcc_step(self._h, self._field(f, 2, "f"), int(nsteps), _stream(stream)))
        return f

    def bcc_observables(self, f, origin, stream=None):
        """qw_bcc_observables: norm, Cartesian mean and second moments of a
        cubic-supercell field about a Cartesian origin."""
        o = QwObs()
        _check(LIB.qw_bcc_observables(self._h, self._field(f, 2, "f"), _darr(origin, 3),
                                      ctypes.byref(o), _stream(stream)))
        return {"norm2": o.norm2, "mean": list(o.mean), "second": list(o.second)}

    def bcc_evolve_fft(self, f0, t, out=None, stream=None):
        """qw_bcc_evolve_fft: U^t on the cubic-supercell torus (real t)."""
        if out is None:
            out = torch.empty_like(f0)
        _check(LIB.qw_bcc_evolve_fft(self._h, self._field(f0, 2, "f0"),
                                     self._field(out, 2, "out"), float(t), _stream(stream)))
        return out

    def kspace_drift(self, psi, stream=None):
        """qw_kspace_drift: drift velocity per step (primitive and Cartesian)
        and the sector norms of psi."""
        o = QwDrift()
        _check(LIB.qw_kspace_drift(self._h, self._field(psi, name="psi"), ctypes.byref(o),
                                   _stream(stream)))
        return {"velocity": list(o.velocity)[:self.dim], "velocity_cart": list(o.velocity_cart),
                "sector_norm2": list(o.sector_norm2), "norm2": o.norm2}

    def observables(self, psi, origin, ref=None, stream=None):
        """qw_observables: norm, positions about origin, overlap with ref."""
        o = QwObs()
        refp = self._field(ref, name="ref") if ref is not None else ctypes.c_void_p(0)
        _check(LIB.qw_observables(self._h, self._field(psi, name="psi"),
                                  _darr(origin, self.dim), refp, ctypes.byref(o), _stream(stream)))
        return {"norm2": o.norm2, "mean": list(o.mean), "second": list(o.second),
                "mean_cart": list(o.mean_cart),
                "overlap": complex(o.overlap_re, o.overlap_im), "ref_norm2": o.ref_norm2}

    def evolve_fft_real(self, psi0, t, out=None, stream=None):
        """qw_evolve_fft_real: the continuous-time evolution to real t."""
        if out is None:
            out = torch.empty_like(psi0)
        _check(LIB.qw_evolve_fft_real(self._h, self._field(psi0, name="psi0"),
                                      self._field(out, name="out"), float(t), _stream(stream)))
        return out

    def evolve_fft_observables(self, psi0, t, origin, out=None, stream=None):
        """qw_evolve_fft_observables: psi_t = U^t psi0 into ``out`` (not kept
        when out is None) and the reductions of psi_t about origin."""
        o = QwObs()
        outp = self._field(out, name="out") if out is not None else ctypes.c_void_p(0)
        _check(LIB.qw_evolve_fft_observables(self._h, self._field(psi0, name="psi0"), outp,
                                             int(t), _darr(origin, self.dim), ctypes.byref(o),
                                             _stream(stream)))
        return {"norm2": o.norm2, "mean": list(o.mean), "second": list(o.second),
                "mean_cart": list(o.mean_cart)}

    def evolve_fft_observables_async(self, psi0, t, origin, raw, out=None, stream=None):
        """qw_evolve_fft_observables_async: queues psi_t = U^t psi0 (into
        ``out``, not kept when out is None) and its reductions about origin,
        whose raw record a copy on the stream leaves in ``raw`` (a pinned CPU
        float64 tensor of at least OBS_RAW_DOUBLES elements). Returns without
        waiting; read the record with obs_from_raw once the stream has passed
        the call."""
        if (not isinstance(raw, torch.Tensor) or raw.device.type != "cpu" or
                raw.dtype != torch.float64 or not raw.is_contiguous() or
                raw.numel() < OBS_RAW_DOUBLES or not raw.is_pinned()):
            raise ValueError("raw must be a pinned, contiguous CPU float64 tensor of at least "
                             "%d elements" % OBS_RAW_DOUBLES)
        outp = self._field(out, name="out") if out is not None else ctypes.c_void_p(0)
        _check(LIB.qw_evolve_fft_observables_async(self._h, self._field(psi0, name="psi0"), outp,
                                                   int(t), _darr(origin, self.dim),
                                                   ctypes.c_void_p(raw.data_ptr()),
                                                   _stream(stream)))

    def obs_from_raw(self, raw, origin):
        """qw_obs_from_raw: the dict evolve_fft_observables returns, from a
        complete raw record (a CPU float64 tensor)."""
        if raw.device.type != "cpu" or raw.dtype != torch.float64 or raw.numel() < OBS_RAW_DOUBLES:
            raise ValueError("raw must be a CPU float64 tensor of at least %d elements"
                             % OBS_RAW_DOUBLES)
        r = raw.contiguous()
        o = QwObs()
        _check(LIB.qw_obs_from_raw(self._h, ctypes.cast(r.data_ptr(), ctypes.POINTER(ctypes.c_double)),
                                   _darr(origin, self.dim), ctypes.byref(o)))
        return {"norm2": o.norm2, "mean": list(o.mean), "second": list(o.second),
                "mean_cart": list(o.mean_cart)}

    def evolve_fft_series(self, psi0, times, origin, stream=None):
        """qw_evolve_fft_series: the reductions of U^t psi0 about origin for
        every t in times (one call, one wait); a list of dicts as
        evolve_fft_observables returns."""
        times = [int(x) for x in times]
        n = len(times)
        if n < 1:
            raise ValueError("need at least one time")
        tarr = (ctypes.c_int64 * n)(*times)
        outs = (QwObs * n)()
        _check(LIB.qw_evolve_fft_series(self._h, self._field(psi0, name="psi0"), n, tarr,
                                        _darr(origin, self.dim), outs, _stream(stream)))
        return [{"norm2": o.norm2, "mean": list(o.mean), "second": list(o.second),
                 "mean_cart": list(o.mean_cart)} for o in outs]

    def newton_wigner(self, psi, origin, stream=None):
        """qw_newton_wigner: sector-projected mean position; returns
        {"mean", "mean_cart", "sectors": [obs+, obs-]}."""
        sec = (QwObs * 2)()
        nw = (ctypes.c_double * 6)()
        _check(LIB.qw_newton_wigner(self._h, self._field(psi, name="psi"), _darr(origin, self.dim),
                                    sec, nw, _stream(stream)))
        return {"mean": list(nw[0:3]), "mean_cart": list(nw[3:6]),
                "sectors": [_obs_dict(sec[k], 3) for k in range(2)]}

    def marginals(self, psi, origin, stream=None):
        """qw_marginals: [(xmin, values), ...] per Cartesian axis."""
        xmin = (ctypes.c_int64 * 3)()
        ln = (ctypes.c_int64 * 3)()
        _check(LIB.qw_marginals(self._h, None, None, None, 0, xmin, ln, None))
        total = sum(ln[i] for i in range(self.dim))
        out = (ctypes.c_double * total)()
        org = (ctypes.c_int64 * self.dim)(*[int(x) for x in origin])
        _check(LIB.qw_marginals(self._h, self._field(psi, name="psi"), org, out, total, xmin, ln,
                                _stream(stream)))
        res, o = [], 0
        for i in range(self.dim):
            res.append((xmin[i], list(out[o:o + ln[i]])))
            o += ln[i]
        return res

    def set_schedule(self, slab_planes, contig_elems=8, contig_threads=256, contig_groups=1):
        """qw_set_schedule: slab size (n1 planes, 0 = whole field), the fused
        pass's elements per thread (4 or 8), workgroup size and pencil groups
        per workgroup."""
        _check(LIB.qw_set_schedule(self._h, int(slab_planes), int(contig_elems),
                                   int(contig_threads), int(contig_groups)))

    def schedule(self):
        """qw_get_schedule: (slab_planes, contig_elems, contig_threads, contig_groups)."""
        a, b, c, d = (ctypes.c_int(0) for _ in range(4))
        _check(LIB.qw_get_schedule(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                   ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def autotune(self, stream=None):
        """qw_autotune: time the candidate schedules, keep the fastest.
        Returns the best time per evolution in ms."""
        ms = ctypes.c_double(0.0)
        _check(LIB.qw_autotune(self._h, _stream(stream), ctypes.byref(ms)))
        return ms.value

    def prepare_state(self, psi, k0, sigma, center, c_plus=1.0, c_minus=0.0, stream=None):
        """qw_prepare_state: Gaussian particle/antiparticle state, unit norm."""
        _check(LIB.qw_prepare_state(self._h, self._field(psi, name="psi"), _darr(k0, self.dim),
                                    float(sigma), _darr(center, self.dim), float(c_plus),
                                    float(c_minus), _stream(stream)))
        return psi

    def evolve_dispersive(self, psi, k0, sigma, center, c_plus, c_minus, order, t, stream=None):
        """qw_evolve_dispersive: the particle state evolved to real t with the
        order-n Taylor polynomial of omega (Proposition 1)."""
        _check(LIB.qw_evolve_dispersive(self._h, self._field(psi, name="psi"), _darr(k0, self.dim),
                                        float(sigma), _darr(center, self.dim), float(c_plus),
                                        float(c_minus), int(order), float(t), _stream(stream)))
        return psi


def dispersion_taylor(dim, m, k0, order):
    """qw_dispersion_taylor: the 10 Taylor coefficients of omega at k0."""
    out = (ctypes.c_double * 10)()
    _check(LIB.qw_dispersion_taylor(int(dim), float(m), _darr(k0, int(dim)), int(order), out))
    return list(out)


def set_step_kernel(two_step=False, tile_shape=0, chunk=0):
    """qw_set_step_kernel (measurement): pairs of 3D complex64 steps in one
    launch (two_step) or one launch per step (the default); tile shape
    0 = 16 x 32, 1 = 8 x 64, 2 = 16 x 16, 3 = 8 x 32; planes per workgroup
    (0 = automatic)."""
    _check(LIB.qw_set_step_kernel(1 if two_step else 0, int(tile_shape), int(chunk)))


def set_fft_kernel(staged=True):
    """qw_set_fft_kernel (measurement): strided passes of large fields
    (complex64 length-256 inverse and length-512, complex128 length-256 with
    far-apart rows) staged through LDS (the default) or with their loads in
    registers; the same bits either way."""
    _check(LIB.qw_set_fft_kernel(1 if staged else 0))


def version():
    return LIB.qw_version().decode()


def _obs_dict(o, dim):
    return {"norm2": o.norm2, "mean": list(o.mean)[:dim], "second": list(o.second),
            "mean_cart": list(o.mean_cart)}


class Server:
    """Continuous-batching server (qw_server_*): requests are Gaussian
    particle states evolved to their own time with their own mass; results
    are the reductions of psi(t) about the request's centre. budget_bytes = 0
    takes QW_HBM_BUDGET, else half of the free device memory."""

    def __init__(self, budget_bytes=0, max_batch=16, nstreams=2, graphs=True, autotune=True,
                 max_graphs=256):
        self._h = ctypes.c_void_p()
        _check(LIB.qw_server_create(ctypes.byref(self._h), int(budget_bytes), int(max_batch),
                                    int(nstreams)))
        try:
            _check(LIB.qw_server_configure(self._h, 1 if graphs else 0, 1 if autotune else 0,
                                           int(max_graphs)))
        except QwError:
            LIB.qw_server_destroy(self._h)
            self._h = None
            raise
        self._dims = {}

    def submit(self, dim, N, m, k0, sigma, center, c_plus, c_minus, t, dtype="c64"):
        r = QwRequest()
        r.dim = int(dim)
        Ns = [int(N)] * r.dim if isinstance(N, int) else [int(x) for x in N]
        if len(Ns) != r.dim:
            raise ValueError("need %d lattice sizes" % r.dim)
        for i in range(3):
            r.N[i] = Ns[i] if i < r.dim else 1
        r.m = float(m)
        if dtype not in DTYPES:
            raise ValueError("dtype must be 'c64' or 'c128'")
        r.dtype = DTYPES[dtype][0]
        k0 = [float(x) for x in k0]
        center = [float(x) for x in center]
        if len(k0) != r.dim or len(center) != r.dim:
            raise ValueError("k0 and center need %d entries" % r.dim)
        for i in range(r.dim):
            r.k0[i] = k0[i]
            r.center[i] = center[i]
        r.sigma = float(sigma)
        r.c_plus = float(c_plus)
        r.c_minus = float(c_minus)
        r.t = int(t)
        tk = ctypes.c_int64()
        _check(LIB.qw_server_submit(self._h, ctypes.byref(r), ctypes.byref(tk)))
        self._dims[tk.value] = r.dim
        return tk.value

    def _convert(self, res):
        dim = self._dims.get(res.ticket, 3)
        return {"ticket": res.ticket, "status": res.status, "batch_size": res.batch_size,
                "queue_s": res.queue_s, "latency_s": res.latency_s,
                "obs": _obs_dict(res.obs, dim), "sector_norm2": list(res.sector_norm2)}

    def poll(self, ticket):
        res = QwResult()
        done = ctypes.c_int()
        _check(LIB.qw_server_poll(self._h, int(ticket), ctypes.byref(res), ctypes.byref(done)))
        return self._convert(res) if done.value else None

    def wait(self, ticket):
        res = QwResult()
        _check(LIB.qw_server_wait(self._h, int(ticket), ctypes.byref(res)))
        return self._convert(res)

    def wait_for(self, ticket, timeout_s):
        """qw_server_wait_for: the result, or None if the request has not
        completed within timeout_s seconds (it then stays pending)."""
        res = QwResult()
        done = ctypes.c_int()
        _check(LIB.qw_server_wait_for(self._h, int(ticket), float(timeout_s), ctypes.byref(res),
                                      ctypes.byref(done)))
        return self._convert(res) if done.value else None

    def cancel(self, ticket):
        """qw_server_cancel: True if the request was still queued and is now
        cancelled (its result carries status QW_ERR_CANCELLED)."""
        c = ctypes.c_int()
        _check(LIB.qw_server_cancel(self._h, int(ticket), ctypes.byref(c)))
        return bool(c.value)

    def hold(self, on=True):
        """qw_server_hold: queue without launching (on) or resume (off)."""
        _check(LIB.qw_server_hold(self._h, 1 if on else 0))

    def stats(self):
        info = QwServerInfo()
        _check(LIB.qw_server_stats(self._h, ctypes.byref(info)))
        return {n: getattr(info, n) for n, _ in QwServerInfo._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            LIB.qw_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
