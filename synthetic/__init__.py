"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and shapes them into canonical arrays. It holds
none of the solver's arithmetic (no Dirac operator, no clover term, no Schwarz or Krylov
step), so that the CPU oracle and the HIP path can both consume its output without
sharing any code of the method.

Canonical layouts (all complex128, x fastest):
  links   U[t, z, y, x, mu, a, b]   mu = 0..3 for x, y, z, t; (a, b) colour row, column
  spinor  psi[t, z, y, x, s, a]     s = spin 0..3, a = colour 0..2
  batch   psi[rhs, t, z, y, x, s, a]

Gauge fields follow the recipe of the benchmark configurations: every link is
U = exp(i * eps * H) with H a traceless Hermitian 3x3 matrix whose underlying complex
entries are i.i.d. standard normal; the exponential is taken through the eigen
decomposition of H. Random numbers come from numpy's default_rng in fixed site chunks of
CHUNK sites: chunk k of a field draws from the k-th child of SeedSequence(seed) (sites
ascending, then mu = 0..3, inside the chunk), so any chunk can be drawn on its own and
the result does not depend on how many worker processes draw the chunks. Gaussian
sources do the same per right-hand side: source r draws from the r-th child of
SeedSequence(seed), chunk k of it from that child's k-th child.
"""
from __future__ import annotations

import concurrent.futures as cf
import multiprocessing as mp
import os

import numpy as np

__all__ = [
    "CHUNK",
    "CONFIGS",
    "gauge_field",
    "gaussian_source",
    "point_sources",
    "random_su3",
    "serving_requests",
]

CHUNK = 1 << 16  # sites per random-number chunk


def _exp_i_eps_h(g: np.ndarray, eps: float) -> np.ndarray:
    """Turn Gaussian 3x3 complex matrices g[..., 3, 3] into SU(3) links exp(i eps H)."""
    h = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    lam, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * lam)
    return (v * ph[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def _link_chunk(seq, n: int, eps: float) -> np.ndarray:
    g = np.random.default_rng(seq).standard_normal((n, 4, 3, 3, 2))
    return _exp_i_eps_h(g[..., 0] + 1j * g[..., 1], eps)


def _normal_chunk(seq, n: int) -> np.ndarray:
    g = np.random.default_rng(seq).standard_normal((n, 4, 3, 2))
    return g[..., 0] + 1j * g[..., 1]


def _workers(vol: int, workers):
    if workers is not None:
        return max(1, int(workers))
    if vol < (1 << 20):
        return 1
    # forked workers only draw random numbers; eight at most keeps the process count of a
    # GPU job low even when the parent already holds the device
    return max(1, min(8, len(os.sched_getaffinity(0))))


def _fill(out: np.ndarray, jobs, fn, workers: int, progress=None, total: int = 0):
    """out[s0:s0 + n] = fn(*args) for every (s0, n, args) job, in worker processes if
    workers > 1 (fork: the children only compute and send back their chunk)."""
    done = 0
    if workers == 1:
        for s0, n, args in jobs:
            out[s0:s0 + n] = fn(*args)
            done += n
            if progress is not None:
                progress(done, total)
        return
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        futs = {ex.submit(fn, *args): (s0, n) for s0, n, args in jobs}
        for f in cf.as_completed(futs):
            s0, n = futs[f]
            out[s0:s0 + n] = f.result()
            done += n
            if progress is not None:
                progress(done, total)


def gauge_field(dims, eps: float, seed: int, workers=None, progress=None) -> np.ndarray:
    """Random SU(3) gauge field U[t,z,y,x,mu,3,3] for lattice dims = (Lx, Ly, Lz, Lt).

    `workers` processes draw the chunks (default: one below 2^20 sites, else up to eight);
    the field is the same for every worker count. `progress(done_sites, total_sites)` is
    called after every chunk if given.
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    vol = lx * ly * lz * lt
    kids = np.random.SeedSequence(seed).spawn((vol + CHUNK - 1) // CHUNK)
    out = np.empty((vol, 4, 3, 3), dtype=np.complex128)
    jobs = [(k * CHUNK, min(CHUNK, vol - k * CHUNK), (kid, min(CHUNK, vol - k * CHUNK), eps))
            for k, kid in enumerate(kids)]
    _fill(out, jobs, _link_chunk, _workers(vol, workers), progress, vol)
    return out.reshape(lt, lz, ly, lx, 4, 3, 3)


def gaussian_source(dims, nrhs: int, seed: int, rhs=None, workers=None) -> np.ndarray:
    """Gaussian spinors psi[rhs,t,z,y,x,4,3], Re and Im i.i.d. N(0,1) per component.

    `rhs` (a list of indices) draws only those right-hand sides of the nrhs, equal to the
    same entries of the full set."""
    lx, ly, lz, lt = (int(d) for d in dims)
    vol = lx * ly * lz * lt
    which = list(range(nrhs)) if rhs is None else [int(r) for r in rhs]
    kids = np.random.SeedSequence(seed).spawn(nrhs)
    out = np.empty((len(which) * vol, 4, 3), dtype=np.complex128)
    jobs = []
    for i, r in enumerate(which):
        for k, kid in enumerate(kids[r].spawn((vol + CHUNK - 1) // CHUNK)):
            n = min(CHUNK, vol - k * CHUNK)
            jobs.append((i * vol + k * CHUNK, n, (kid, n)))
    _fill(out, jobs, _normal_chunk, _workers(vol * len(which), workers))
    return out.reshape(len(which), lt, lz, ly, lx, 4, 3)


def point_sources(dims, origin=(0, 0, 0, 0)) -> np.ndarray:
    """Twelve unit point sources psi[12,t,z,y,x,4,3], one per (spin, colour) at origin."""
    lx, ly, lz, lt = (int(d) for d in dims)
    ox, oy, oz, ot = origin
    out = np.zeros((12, lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    for s in range(4):
        for a in range(3):
            out[3 * s + a, ot, oz, oy, ox, s, a] = 1.0
    return out


def random_su3(shape, seed: int) -> np.ndarray:
    """Haar-ish random SU(3) matrices of the given leading shape (QR of a Gaussian)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(tuple(shape) + (3, 3, 2))
    z = g[..., 0] + 1j * g[..., 1]
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[..., None, None]


# Benchmark configurations: lattice (Lx, Ly, Lz, Lt), SAP block, kappa, c_sw, eps,
# right-hand sides, storage precision of the preconditioner, seeds.
CONFIGS = {
    "c1_4x4x4x4_f64": dict(dims=(4, 4, 4, 4), block=(2, 2, 2, 2), kappa=0.12, csw=1.0,
                           eps=0.3, nrhs=1, source="gaussian", prec="f64",
                           gauge_seed=11, source_seed=21),
    "c2_16x16x16x32_f32": dict(dims=(16, 16, 16, 32), block=(8, 4, 4, 4), kappa=0.125,
                               csw=1.0, eps=0.3, nrhs=1, source="gaussian", prec="f32",
                               gauge_seed=12, source_seed=22),
    "c3_32x32x32x64_f16": dict(dims=(32, 32, 32, 64), block=(4, 4, 4, 4), kappa=0.126,
                               csw=1.0, eps=0.25, nrhs=12, source="point", prec="f16",
                               gauge_seed=13, source_seed=23),
    "c5_48x48x48x96_f16": dict(dims=(48, 48, 48, 96), block=(8, 4, 4, 4), kappa=0.1265,
                               csw=1.0, eps=0.2, nrhs=12, source="gaussian", prec="f16",
                               gauge_seed=15, source_seed=25),
}

SERVING_VOLUMES = ((16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64))


def serving_requests(n: int, rate: float, seed: int = 31, volumes=SERVING_VOLUMES,
                     kappa_range=(0.120, 0.126), max_rhs: int = 12):
    """Poisson request stream: list of dicts with arrival time, volume, kappa, nrhs, seed.

    Inter-arrival times are exponential with the given rate (requests per second); the
    volume is drawn uniformly from `volumes`, kappa uniformly from kappa_range and the
    number of right-hand sides uniformly from 1..max_rhs.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        out.append(dict(id=i, t_arrival=t, vol=int(rng.integers(len(volumes))),
                        kappa=float(rng.uniform(*kappa_range)),
                        nrhs=int(rng.integers(1, max_rhs + 1)),
                        seed=int(rng.integers(1 << 30))))
    return out
