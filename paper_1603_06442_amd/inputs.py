"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module draws random numbers and builds parameter sets; it holds none of
the walk's arithmetic (no symbols, projectors, transforms or steps), so the
HIP path and the oracle can both take their inputs from it without sharing
any of the method.

Workloads (shapes, sizes and distributions of the paper's experiments):
* the 1D line of 4096 sites, m = 0.1, packet at k0 = 0.3 with width 40 sites;
* the 3D BCC lattice as a 64^3 primitive-cell torus, m = 0.05, k0 drawn
  uniformly in the Cartesian ball |k| < 0.5, width 6 cells;
* the 3D 256^3 torus, m = 0.02, k0 = (0.1, 0.1, 0.1), width 20 cells, equal
  particle/antiparticle weights, 64 times log-spaced in [1, 1e5];
* a stream of 512 mixed-shape requests for the serving loop;
* the 3D 512^3 torus, m = 0.1, width 40 cells, t = 1e6.
"""
import math

import numpy as np


def rng_for(config_index):
    """The generator for a workload: numpy default_rng(1000 + index)."""
    return np.random.default_rng(1000 + int(config_index))


def random_field(rng, d, N, s, complex_dtype=np.complex128):
    """Complex Gaussian field psi[s, N..N] with unit 2-norm."""
    shape = (s,) + (N,) * d
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    psi /= np.sqrt(np.sum(np.abs(psi) ** 2))
    return psi.astype(complex_dtype)


def random_spinor(rng, s):
    z = rng.standard_normal(s) + 1j * rng.standard_normal(s)
    return z / np.linalg.norm(z)


def k0_in_ball(rng, d, radius=0.5):
    """Cartesian k0 uniform in the ball |k| < radius (direction ~ N(0, I))."""
    v = rng.standard_normal(d)
    v /= np.linalg.norm(v)
    return v * radius * rng.uniform() ** (1.0 / d)


def zb_times(count=64, t_max=1e5):
    """t_i = max(t_{i-1} + 1, round(t_max^(i/(count-1)))), i = 0..count-1."""
    out = []
    prev = 0
    for i in range(count):
        t = max(prev + 1, int(round(t_max ** (i / (count - 1)))))
        out.append(t)
        prev = t
    return out


def workload(index):
    """Parameter dictionary of one of the five workloads (index 0..4)."""
    rng = rng_for(index)
    if index == 0:
        return dict(d=1, N=4096, m=0.1, k0=[0.3], sigma=40.0, center=[2048],
                    c_plus=1.0, c_minus=0.0, steps=1000, t=1000, dtype="c128")
    if index == 1:
        return dict(d=3, N=64, m=0.05, k0=list(k0_in_ball(rng, 3)), sigma=6.0,
                    center=[32, 32, 32], c_plus=1.0, c_minus=0.0, steps=128, t=128,
                    dtype="c64")
    if index == 2:
        r = 1.0 / math.sqrt(2.0)
        return dict(d=3, N=256, m=0.02, k0=[0.1, 0.1, 0.1], sigma=20.0,
                    center=[128, 128, 128], c_plus=r, c_minus=r, times=zb_times(),
                    dtype="c64")
    if index == 3:
        return dict(requests=serving_requests(rng, 512))
    if index == 4:
        return dict(d=3, N=512, m=0.1, k0=list(k0_in_ball(rng, 3)), sigma=40.0,
                    center=[256, 256, 256], c_plus=1.0, c_minus=0.0, t=1000000,
                    dtype="c64", sub_N=32, sub_sigma=2.5)
    raise ValueError("workload index must be 0..4")


def serving_requests(rng, count, rate=None):
    """Mixed requests: d uniform in {1,2,3}, N a power of two (1D 2^10..2^16,
    2D 2^6..2^10, 3D 2^5..2^7, log-uniform), m ~ U[0, 0.3], k0 uniform in the
    ball |k| < 0.5, sigma log-uniform in [4, N/8], (c+, c-) = (1, 0) or
    (1/sqrt2, 1/sqrt2) with probability 1/2, t log-uniform integer in
    [1, 1e6]. ``rate`` (requests/s) adds Poisson arrival offsets."""
    lo_hi = {1: (10, 16), 2: (6, 10), 3: (5, 7)}
    reqs = []
    at = 0.0
    for i in range(count):
        d = int(rng.integers(1, 4))
        lo, hi = lo_hi[d]
        N = 1 << int(rng.integers(lo, hi + 1))
        m = float(rng.uniform(0.0, 0.3))
        k0 = k0_in_ball(rng, d)
        sigma = float(math.exp(rng.uniform(math.log(4.0), math.log(N / 8.0))))
        two = bool(rng.integers(0, 2))
        cp, cm = (1.0 / math.sqrt(2.0), 1.0 / math.sqrt(2.0)) if two else (1.0, 0.0)
        t = int(round(math.exp(rng.uniform(0.0, math.log(1e6)))))
        if rate:
            at += float(rng.exponential(1.0 / rate))
        reqs.append(dict(id=i, d=d, N=N, m=m, k0=list(k0), sigma=sigma,
                         center=[N // 2] * d, c_plus=cp, c_minus=cm, t=t, arrival=at))
    return reqs
