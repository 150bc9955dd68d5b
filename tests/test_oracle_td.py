"""Pins of the oracle's time-domain resampling search (the other acceleration
search of Sec. 1): the resampling map against the phase law it inverts, the
linear interpolation on a ramp, a drifting tone turned into a pure tone, and
the harmonic sums against brute force."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _tone(N, rbar, z, amps, phase0=0.3):
    u = np.arange(N, dtype=np.float64) / N
    x = np.zeros(N)
    for j, a in enumerate(amps, 1):
        x += a * np.cos(phase0 * j + 2 * np.pi * ((j * rbar - j * z / 2) * u + j * z * u * u / 2))
    return x


def test_zero_acceleration_is_the_series():
    x = np.random.default_rng(1).standard_normal(4096)
    assert np.array_equal(O.td_resample(x, 0.0), x)


@pytest.mark.parametrize("alpha", [1e-3, -2.5e-3, 0.02])
def test_resampling_inverts_the_phase_law(alpha):
    # a ramp x[n] = n is interpolated exactly, so the resampled ramp is the
    # source position s_m; v = s_m / N - 1/2 must satisfy tau_m = v + alpha v^2 / 2
    N = 8192
    y = O.td_resample(np.arange(N, dtype=np.float64), alpha)
    tau = np.arange(N) / N - 0.5
    v = y / N - 0.5
    # positions between the first and the last sample (where both
    # interpolation neighbours are samples of the ramp)
    inside = (y > 0) & (y < N - 1)
    inside[1:] &= np.diff(y) > 0
    assert inside.sum() > 0.97 * N
    assert np.max(np.abs(v[inside] + alpha * v[inside] ** 2 / 2 - tau[inside])) < 1e-12
    # past the end of the series the resampled value is zero
    spos = N * (2 * tau / (1 + np.sqrt(1 + 2 * alpha * tau)) + 0.5)
    assert np.all(y[spos >= N] == 0.0)


def test_matched_resampling_makes_a_pure_tone():
    # a tone of mean frequency 100.3 bins drifting by 3.3 bins, resampled with
    # alpha = 3.3 / 100.3: (1) it equals the tone evaluated at the exact
    # positions, found by Newton's method on the phase law tau = v + alpha v^2 / 2,
    # up to the linear interpolation's error; (2) the power gathers in the
    # tone's bin like that of a constant tone (sinc^2(0.3) = 0.737, less the
    # alpha/8 of the new axis that runs before the data); (3) without the
    # matched resampling it does not.
    N, rbar, z = 1 << 14, 100.3, 3.3
    alpha = z / rbar
    x = _tone(N, rbar, z, [1.0])
    y = O.td_resample(x, alpha)
    tau = np.arange(N) / N - 0.5
    v = tau.copy()
    for _ in range(30):
        v -= (v + alpha * v * v / 2 - tau) / (1 + alpha * v)
    u = v + 0.5
    ideal = np.where((u >= 0) & (u < 1), np.cos(
        0.3 + 2 * np.pi * ((rbar - z / 2) * u + z * u * u / 2)), 0.0)
    inside = (u >= 0) & (u * N < N - 1)
    assert np.max(np.abs(y[inside] - ideal[inside])) < 2e-3  # (pi f)^2 / 8 at f = 0.006
    Y = O.real_spectrum(y) / (N / 2)
    assert abs(Y[100]) ** 2 > (1 - alpha / 8) ** 2 * 0.99 * np.sinc(0.3) ** 2
    for a in (0.0, -alpha):
        Y0 = O.real_spectrum(O.td_resample(x, a)) / (N / 2)
        assert np.max(np.abs(Y0[90:111]) ** 2) < 0.65 * np.sinc(0.3) ** 2


def test_harmonic_sum_brute_force():
    rng = np.random.default_rng(4)
    P = rng.random((3, 50))
    for nh in (2, 4, 8):
        S = O.td_harmonic_sum(P, nh)
        for i in range(3):
            for k in range(50):
                want = 0.0
                for j in range(1, nh + 1):
                    q = Fraction(j * k, nh)
                    kj = int(q + Fraction(1, 2)) if q >= 0 else -int(-q + Fraction(1, 2))
                    want += P[i, kj]
                assert S[i, k] == pytest.approx(want, rel=1e-14)


def test_search_finds_accelerated_pulsar():
    # 4 phase-locked harmonics drifting by 6.2 bins at 700.4: the strongest
    # 4-harmonic candidate sits at the trial nearest alpha = 6.2 / 700.4 and
    # at a top-harmonic bin next to 4 x 700.4 = 2801.6 (2801 gathers the
    # harmonics at 700, 1401, 2101, 2801, nearer the true 700.4, 1400.8,
    # 2101.2 than 2802 does), with r, z of the fundamental
    N = 1 << 14
    rng = np.random.default_rng(9)
    x = rng.standard_normal(N) + _tone(N, 700.4, 6.2, [0.12, 0.12, 0.12, 0.12])
    alpha_max, nalpha = 0.02, 21
    res = O.td_search(x, alpha_max=alpha_max, nalpha=nalpha, sigma=6.0, nharm_max=4, W=256)
    alphas = O.td_alphas(alpha_max, nalpha)
    best = max((c for c in res.candidates if c.nharm == 4), key=lambda c: c.power)
    assert best.iz == int(np.argmin(np.abs(alphas - 6.2 / 700.4)))
    assert best.k == 2801 and best.r == 700.25
    assert best.z == pytest.approx(alphas[best.iz] * 700.25, rel=1e-12)
