"""Seeded synthetic de-dispersed time series for the acceleration search.

This module only *generates inputs*: white Gaussian noise plus sinusoids whose
frequency drifts linearly in time (the constant-acceleration signal model of
Sec. 1 and Sec. 2 of Dimoudi & Armour, arXiv:1511.07343).  It holds none of the
search's arithmetic (no transforms, templates, normalisation, sums or
thresholds), so both the GPU path and the CPU oracle can consume its output
without sharing any of the method's code.

Signal model.  Over an observation of N samples, u = n / N in [0, 1), a
sinusoid with mean Fourier frequency r (in bins) and frequency derivative z
(the total drift in bins over the observation, z = fdot * T^2 with T the
observation length, Sec. 2) has phase

    phi(u) = phi0 + 2 pi [ (r - z/2) u + z u^2 / 2 ]

so its instantaneous frequency is r + z (u - 1/2) bins.  A pulsar with
``nharm`` phase-locked harmonics adds amp * cos(h * phi(u)) for h = 1..nharm;
harmonic h therefore sits at mean frequency h r with drift h z.  A harmonic is
left out when its swept band reaches the Nyquist edge: h r + |h z| / 2 >= N/2 - h.

All draws use numpy's PCG64 ``default_rng``.  Noise is drawn first, in float64;
pulsar parameters are drawn after it from the same generator; the sum is cast
to float32 last, so every consumer sees the same float32 series.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

__all__ = [
    "Pulsar",
    "Trial",
    "add_pulsar",
    "make_series",
    "single_tone_series",
    "draw_pulsars",
    "ska_trial",
    "Dispersed",
    "make_filterbank",
    "batch_trials",
    "served_trace",
    "precision_trials",
]


@dataclass(frozen=True)
class Pulsar:
    """One injected accelerated pulsar (fundamental parameters)."""

    r: float  # mean Fourier frequency of the fundamental, in bins
    z: float  # drift of the fundamental over the observation, in bins
    amp: float  # amplitude of every harmonic
    phi0: float = 0.0
    nharm: int = 1


@dataclass
class Trial:
    """A synthetic DM trial: the float32 series and what was injected."""

    x: np.ndarray
    seed: int
    pulsars: List[Pulsar] = field(default_factory=list)

    @property
    def nsamp(self) -> int:
        return int(self.x.shape[0])


def add_pulsar(x64: np.ndarray, p: Pulsar) -> None:
    """Add ``p`` in place to the float64 series ``x64``."""
    n = x64.shape[0]
    nb = n // 2
    keep = [h for h in range(1, p.nharm + 1) if h * p.r + abs(h * p.z) / 2.0 < nb - h]
    if not keep:
        return
    u = np.arange(n, dtype=np.float64) / n
    # cycles of the fundamental, reduced mod 1 before scaling to radians so the
    # phase stays accurate for large r
    cyc = (p.r - p.z / 2.0) * u + (p.z / 2.0) * u * u
    cyc -= np.floor(cyc)
    c1 = np.cos(p.phi0 + 2.0 * np.pi * cyc)
    # cos(h theta) by the Chebyshev recurrence T_h = 2 c1 T_{h-1} - T_{h-2}
    prev, cur = np.ones(n), c1
    for h in range(1, max(keep) + 1):
        if h > 1:
            prev, cur = cur, 2.0 * c1 * cur - prev
        if h in keep:
            x64 += p.amp * cur


def make_series(n: int, seed: int, pulsars=(), noise_sigma: float = 1.0) -> Trial:
    """White Gaussian noise (mean 0, std ``noise_sigma``) plus ``pulsars``."""
    rng = np.random.default_rng(seed)
    x64 = rng.standard_normal(n) * noise_sigma if noise_sigma > 0 else np.zeros(n)
    for p in pulsars:
        add_pulsar(x64, p)
    return Trial(x=x64.astype(np.float32), seed=seed, pulsars=list(pulsars))


def single_tone_series(n: int = 1 << 17, seed: int = 1, r: float = 20000.3, z: float = 40.0,
                       amp: float = 0.05, noise_sigma: float = 1.0) -> Trial:
    """Plain one-series workload: noise plus one accelerated sinusoid.

    Defaults are the small plain configuration: 2^17 samples, r0 = 20000.3 bins
    (mean frequency), z0 = +40 bins, amplitude 0.05, phi0 = 0, seed 1.
    """
    return make_series(n, seed, [Pulsar(r=r, z=z, amp=amp, phi0=0.0, nharm=1)], noise_sigma)


def draw_pulsars(rng: np.random.Generator, count: int, nharm: int = 8,
                 r_range=(1.0e4, 1.0e6), z_range=(-180.0, 180.0),
                 amp_range=(0.01, 0.05)) -> List[Pulsar]:
    """Draw ``count`` pulsars: r, z, amp uniform on their ranges, phi0 uniform on [0, 2 pi)."""
    out = []
    for _ in range(count):
        r = rng.uniform(*r_range)
        z = rng.uniform(*z_range)
        a = rng.uniform(*amp_range)
        phi0 = rng.uniform(0.0, 2.0 * np.pi)
        out.append(Pulsar(r=float(r), z=float(z), amp=float(a), phi0=float(phi0), nharm=nharm))
    return out


def _trial_with_random_pulsars(n: int, seed: int, count: int | None, max_count: int = 3,
                               r_range=(1.0e4, 1.0e6)) -> Trial:
    rng = np.random.default_rng(seed)
    x64 = rng.standard_normal(n)
    if count is None:
        count = int(rng.integers(0, max_count + 1))
    # keep the fundamental's whole band inside the spectrum for short series
    hi = min(r_range[1], n / 2 - 200.0)
    pulsars = draw_pulsars(rng, count, r_range=(r_range[0], hi))
    for p in pulsars:
        add_pulsar(x64, p)
    return Trial(x=x64.astype(np.float32), seed=seed, pulsars=pulsars)


def ska_trial(n: int = 1 << 23, seed: int = 2, npulsars: int = 4) -> Trial:
    """SKA-shaped single trial: 2^23 samples, 4 pulsars of 8 harmonics each."""
    return _trial_with_random_pulsars(n, seed, npulsars)


def batch_trials(count: int = 64, n: int = 1 << 23, seed0: int = 1000) -> List[Trial]:
    """Independent trials, seeds seed0 + i, each with 0-3 pulsars."""
    return [_trial_with_random_pulsars(n, seed0 + i, None) for i in range(count)]


def precision_trials(count: int = 16, n: int = 1 << 22, seed0: int = 5000) -> List[Trial]:
    """Trials for the reduced-precision comparison: seeds seed0 + i, 0-3 pulsars."""
    return [_trial_with_random_pulsars(n, seed0 + i, None) for i in range(count)]


def served_trace(count: int = 6000, seed: int = 4, duration_s: float = 530.0,
                 lengths=(1 << 21, 1 << 22, 1 << 23), probs=(0.2, 0.3, 0.5),
                 pulsar_fraction: float = 0.05):
    """Arrival trace of DM-trial requests for the serving loop.

    Returns a list of dicts {t_arrival, nsamp, seed, has_pulsar}; request i's
    series is ``served_request(entry)``.  Arrivals are Poisson with rate
    count / duration_s (exponential gaps).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(duration_s / count, size=count)
    t = np.cumsum(gaps)
    lens = rng.choice(np.asarray(lengths), size=count, p=np.asarray(probs))
    has = rng.uniform(size=count) < pulsar_fraction
    return [dict(t_arrival=float(t[i]), nsamp=int(lens[i]), seed=40000 + i, has_pulsar=bool(has[i]))
            for i in range(count)]


def served_request(entry) -> Trial:
    """The series of one request from ``served_trace``."""
    return _trial_with_random_pulsars(entry["nsamp"], entry["seed"], 1 if entry["has_pulsar"] else 0)


@dataclass(frozen=True)
class Dispersed:
    """A periodic pulsar injected into a filterbank: pulses of Gaussian shape
    (width in seconds) every ``period`` seconds, dispersed by ``dm``
    (pc cm^-3) with the cold-plasma delay of each channel."""

    period: float
    dm: float
    width: float
    amp: float  # peak height in the 8-bit units of the noise (sigma 16)
    phase0: float = 0.0  # arrival time of the first pulse at the top of the band, s


# cold-plasma dispersion delay constant, s MHz^2 pc^-1 cm^3 (signal model of the injection)
_DISPERSION_S = 4.148808e3


def make_filterbank(nchan: int, nsamp: int, f_top: float, foff: float, tsamp: float, seed: int,
                    pulsars=(), mean: float = 128.0, sigma: float = 16.0) -> np.ndarray:
    """Channel-major 8-bit filterbank (nchan x nsamp): Gaussian noise of the
    given mean and sigma, plus dispersed periodic pulses (continuous delays),
    rounded to the nearest integer and clipped to [0, 255].  Channel c has
    frequency f_top - c foff MHz."""
    rng = np.random.default_rng(seed)
    fil = np.empty((nchan, nsamp), dtype=np.uint8)
    t = np.arange(nsamp, dtype=np.float64) * tsamp
    for c in range(nchan):
        row = mean + sigma * rng.standard_normal(nsamp)
        f = f_top - foff * c
        for p in pulsars:
            delay = _DISPERSION_S * p.dm * (1.0 / (f * f) - 1.0 / (f_top * f_top))
            ph = (t - p.phase0 - delay) / p.period
            dt = (ph - np.round(ph)) * p.period  # time from the nearest pulse
            row += p.amp * np.exp(-0.5 * (dt / p.width) ** 2)
        fil[c] = np.clip(np.rint(row), 0, 255).astype(np.uint8)
    return fil
