"""Seeded synthetic spectra for the correlation workloads.

This module only draws inputs: band profiles, time-varying band amplitudes
and noise.  It holds none of the correlation method's arithmetic, and both
the HIP path's tests/benchmark and the CPU oracle's tests take their inputs
from it.

Recipe (band generator).  Spectral axis nu = 0..n-1; perturbation steps
t = 0..m-1 (equidistant, as the discrete equations require, Sec. 2).  Each
band k has a profile L_k(nu) -- Lorentzian g^2/((nu-c)^2+g^2) or Gaussian
exp(-ln2 (nu-c)^2/g^2), g the half width at half maximum -- with centre
c ~ U[50/512 n, 460/512 n] and half width g ~ U[3, 12] sqrt(n/512).  Its
amplitude varies along the perturbation as
    a_k + b_k sin(2 pi t / T + phi_k) [+ d_k t/(m-1)],   T = 1.5 (m-1),
phi_k ~ U[0, pi].  Spectra are S[t, nu] = sum_k amp_k(t) L_k(nu) plus
Gaussian noise of standard deviation sigma.  These seeded inputs stand in for
the paper's simulated and measured data (its sim2ddata() parameters and the
FuranMale dataset are not given in the paper).

Seeds: BASE_SEED + k for workload k (1..4); BASE_SEED + 1000 + i for the i-th
dataset of the batched workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 180800685


def _profiles(rng, n, nbands, kinds):
    nu = np.arange(n, dtype=np.float64)
    c = rng.uniform(50.0 / 512.0 * n, 460.0 / 512.0 * n, size=nbands)
    g = rng.uniform(3.0, 12.0, size=nbands) * math.sqrt(n / 512.0)
    P = np.empty((nbands, n))
    for k in range(nbands):
        d2 = (nu - c[k]) ** 2
        if kinds[k] == "L":
            P[k] = g[k] ** 2 / (d2 + g[k] ** 2)
        else:
            P[k] = np.exp(-math.log(2.0) * d2 / g[k] ** 2)
    return P, c, g


def bands(m, n, nbands, seed, a_range=(0.5, 2.0), b_range=(0.1, 1.0), drift=None,
          sigma=1e-3, kinds=None, log_amplitude=False, relative_b=False):
    """Generic band generator; returns (S, meta) with S of shape (m, n), float64."""
    rng = np.random.default_rng(seed)
    if kinds is None:
        kinds = ["L"] * nbands
    P, c, g = _profiles(rng, n, nbands, kinds)
    if log_amplitude:
        a = np.exp(rng.uniform(math.log(a_range[0]), math.log(a_range[1]), size=nbands))
    else:
        a = rng.uniform(a_range[0], a_range[1], size=nbands)
    b = rng.uniform(b_range[0], b_range[1], size=nbands)
    if relative_b:
        b = b * a
    phase = rng.uniform(0.0, math.pi, size=nbands)
    d = np.zeros(nbands)
    if drift is not None:
        d = rng.uniform(drift[0], drift[1], size=nbands)
        if relative_b:
            d = d * a
    t = np.arange(m, dtype=np.float64)
    T = 1.5 * (m - 1)
    amp = (a[None, :] + b[None, :] * np.sin(2.0 * math.pi * t[:, None] / T + phase[None, :])
           + d[None, :] * t[:, None] / max(m - 1, 1))
    S = amp @ P + rng.normal(0.0, sigma, size=(m, n))
    meta = dict(centers=c, hwhm=g, a=a, b=b, phase=phase, drift=d, period=T)
    return S, meta


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------
def workload_small(seed=BASE_SEED + 1):
    """m=11 steps x n=512 points, 4 Lorentzian bands, noise sigma 1e-3."""
    return bands(11, 512, 4, seed, a_range=(0.5, 2.0), b_range=(0.1, 1.0), sigma=1e-3)


def workload_medium(seed=BASE_SEED + 2):
    """m=64 x n=4096, 32 Lorentzians with linear-plus-sinusoidal drift."""
    return bands(64, 4096, 32, seed, a_range=(0.5, 2.0), b_range=(0.1, 1.0),
                 drift=(-0.5, 0.5), sigma=1e-3)


def workload_large(seed=BASE_SEED + 3, m=256, n=16384):
    """m=256 x n=16384, 128 bands (even k Lorentzian, odd k Gaussian),
    amplitudes log-uniform in [1e-3, 1e2], b = U[0.05,0.5] a, drift U[-0.3,0.3] a,
    noise sigma 1e-4."""
    kinds = ["L" if k % 2 == 0 else "G" for k in range(128)]
    return bands(m, n, 128, seed, a_range=(1e-3, 1e2), b_range=(0.05, 0.5), drift=(-0.3, 0.3),
                 sigma=1e-4, kinds=kinds, log_amplitude=True, relative_b=True)


def workload_hetero(seed=BASE_SEED + 4, m=128, n1=8192, n2=2048, drivers=16):
    """Two spectra sets sharing m=128 steps: n1=8192 (64 bands) and n2=2048
    (24 bands).  Band k of either set follows latent driver d = k mod 16,
    g_d(t) = sin(2 pi t/T + phi_d), phi_d ~ U[0, pi]; its amplitude is
    base_k (1 + 0.3 w_k g_d(t)) with base log-uniform in [1e-2, 1e2] and
    w_k ~ U[0.2, 1].  Noise sigma 1e-4.  meta carries each band's driver and
    the driver phases, which fix the expected sign of the asynchronous
    spectrum between coupled bands."""
    rng = np.random.default_rng(seed)
    t = np.arange(m, dtype=np.float64)
    T = 1.5 * (m - 1)
    dphase = rng.uniform(0.0, math.pi, size=drivers)
    G = np.sin(2.0 * math.pi * t[:, None] / T + dphase[None, :])  # (m, drivers)

    def one(n, nb):
        P, c, g = _profiles(rng, n, nb, ["L"] * nb)
        base = np.exp(rng.uniform(math.log(1e-2), math.log(1e2), size=nb))
        w = rng.uniform(0.2, 1.0, size=nb)
        drv = np.arange(nb) % drivers
        amp = base[None, :] * (1.0 + 0.3 * w[None, :] * G[:, drv])
        S = amp @ P + rng.normal(0.0, 1e-4, size=(m, n))
        return S, dict(centers=c, hwhm=g, base=base, weight=w, driver=drv)

    S1, m1 = one(n1, 64)
    S2, m2 = one(n2, 24)
    return S1, S2, dict(set1=m1, set2=m2, driver_phase=dphase, period=T)


@dataclass
class BatchItem:
    m: int
    n: int
    nbands: int
    seed: int


@dataclass
class Batch:
    items: list = field(default_factory=list)


def batch_spec(count=256, seed=BASE_SEED + 5, m_range=(8, 200), n_range=(256, 8192),
               band_range=(4, 64)):
    """Sizes of the batched workload: m ~ U{8..200}, n ~ U{256..8192},
    bands ~ U{4..64}; dataset i is drawn with seed BASE_SEED + 1000 + i."""
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_range[0], m_range[1] + 1, size=count)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    bs = rng.integers(band_range[0], band_range[1] + 1, size=count)
    return [BatchItem(int(ms[i]), int(ns[i]), int(bs[i]), BASE_SEED + 1000 + i)
            for i in range(count)]


def batch_item_data(item: BatchItem):
    """Spectra of one batched dataset (the medium workload's generator)."""
    S, _ = bands(item.m, item.n, item.nbands, item.seed, a_range=(0.5, 2.0),
                 b_range=(0.1, 1.0), drift=(-0.5, 0.5), sigma=1e-3)
    return S
