"""Pins of the oracle's Fourier interpolation and candidate refinement (the
extension past the paper's method that evaluates the Sec. 2 response off the
(k, z) grid) against results fixed by other means: the plane of Eq. (1) at
grid points, the sinc interpolation identity at zero drift, the matched
response of a synthesised drifting tone, and the exponential law of noise."""
import math

import numpy as np
import pytest
from scipy import special, stats

import oracle as O


def _chirp(N, rbar, zbar, amps, phase0=0.4):
    """Phase-locked harmonics of a tone of mean frequency rbar bins whose
    frequency drifts by zbar bins over the series (harmonic j at j rbar, j zbar)."""
    u = np.arange(N, dtype=np.float64) / N
    x = np.zeros(N)
    for j, a in enumerate(amps, 1):
        x += a * np.cos(phase0 * j + 2 * np.pi * ((j * rbar - j * zbar / 2) * u + j * zbar * u * u / 2))
    return x


def _captured(r, z, h):
    """sum_{|r - k| <= h} |A(r - k, z)|^2 from the closed form."""
    k = np.arange(math.ceil(r - h), math.floor(r + h) + 1)
    return float(np.sum(np.abs(O.template_response(r - k, z)) ** 2))


def test_grid_points_are_the_plane():
    # At integer r and a bank drift the interpolated power is the plane cell
    # of the direct correlation (including the zero-padded spectrum ends).
    rng = np.random.default_rng(3)
    N = 1 << 12
    x = rng.standard_normal(N) + _chirp(N, 600.4, 9.0, [0.2])
    Xh = O.normalise(O.real_spectrum(x), 256)
    taps, zs, h = O.template_taps(20.0, 2.0)
    P = O.correlate(Xh, taps)
    nb = Xh.shape[0]
    cells = [(0, 0), (3, 5), (10, 600), (15, 601), (20, nb - 1), (7, nb - 20), (12, h), (18, 1)]
    cells += [(int(i), int(k)) for i, k in zip(rng.integers(0, zs.size, 12), rng.integers(0, nb, 12))]
    for iz, k in cells:
        got = O.interp_power(Xh, float(k), float(zs[iz]), h)
        assert abs(got - P[iz, k]) <= 1e-11 * max(P[iz, k], 1.0), (iz, k, got, P[iz, k])


@pytest.mark.parametrize("delta", [0.5, 0.25, -0.3, 0.125])
def test_zero_drift_is_sinc_interpolation(delta):
    # A spectrum with one non-zero bin k0: P(k0 + delta, 0) = sinc^2(delta) / D
    # with D the sum of sinc^2(delta - m) over |delta - m| <= h.  Since
    # sum over all m of 1 / (delta - m)^2 = pi^2 / sin^2(pi delta), D is 1
    # minus the two tails, and each tail is a trigamma value:
    #   sum_{m >= M} 1 / (m - delta)^2 = psi_1(M - delta).
    h, nb, k0 = 20, 400, 200
    Xh = np.zeros(nb, dtype=np.complex128)
    Xh[k0] = 1.0
    hi = math.floor(delta + h) + 1      # first m with m - delta > h
    lo = math.ceil(delta - h) - 1       # last m with delta - m > h
    tails = special.polygamma(1, hi - delta) + special.polygamma(1, delta - lo)
    D = 1.0 - (math.sin(math.pi * delta) / math.pi) ** 2 * tails
    want = np.sinc(delta) ** 2 / D
    got = O.interp_power(Xh, k0 + delta, 0.0, h)
    assert abs(got - want) <= 1e-12 * want


@pytest.mark.parametrize("amps", [[1.0], [1.0, 0.7, 0.5, 0.3]])
def test_refine_recovers_drifting_tone(amps):
    # A noiseless tone at rbar = 1000.3 drifting by zbar = 7.4 bins (both off
    # the grid).  The matched response gives S(rbar, zbar) = sum_j a_j^2
    # sum_k |A(j rbar - k, j zbar)|^2 for the spectrum scaled by 2 / N, to
    # the accuracy of the continuous-time model of the sampled DFT; the
    # search must end within its resolution of (rbar, zbar), recovering the
    # power that the grid cell loses to the fractional offsets.
    N, rbar, zbar = 1 << 14, 1000.3, 7.4
    nh = len(amps)
    zmax, dz, levels = 40.0, 2.0, 7
    h = O.halfwidth(zmax)
    Xh = O.real_spectrum(_chirp(N, rbar, zbar, amps)) / (N / 2)
    want = sum(a * a * _captured(j * rbar, j * zbar, h) for j, a in enumerate(amps, 1))
    assert abs(O.interp_sum(Xh, rbar, zbar, nh, h) / want - 1.0) < 3e-4
    izc = int(round(zmax / dz))
    k = int(round(nh * rbar))
    iz = izc + int(round(nh * zbar / dz))
    r, z, S, sg = O.refine(Xh, k, iz, nh, zmax=zmax, dz=dz, h=h, levels=levels)
    assert abs(r - rbar) <= 2.0 ** -levels
    assert abs(z - zbar) <= 2.0 * dz * 2.0 ** -levels
    assert S >= (1.0 - 5e-4) * want
    grid = O.interp_sum(Xh, *O.refine_start(k, iz, nh, dz, izc), nh, h)
    assert S > grid
    if nh == 1:
        # scalloping at a 0.3-bin offset (sinc^2(0.3) = 0.737) is recovered
        assert S / grid > 1.3
    assert sg == pytest.approx(O.sigma_of(S, nh), rel=1e-12)


def test_noise_power_is_exponential_off_grid():
    # For white noise of unit mean power the interpolated power is Exp(1) at
    # any (r, z): the template is a unit-norm combination of independent
    # complex Gaussian bins.
    rng = np.random.default_rng(11)
    nb = 1 << 15
    Xh = (rng.standard_normal(nb) + 1j * rng.standard_normal(nb)) / math.sqrt(2.0)
    h = O.halfwidth(30.0)
    rs = rng.uniform(200.0, nb - 200.0, 1500)
    zs = rng.uniform(-30.0, 30.0, 1500)
    p = np.array([O.interp_power(Xh, float(r), float(z), h) for r, z in zip(rs, zs)])
    assert abs(p.mean() - 1.0) < 0.1
    assert stats.kstest(p, "expon").pvalue > 1e-3


def test_refine_endpoints_without_ties_is_the_search():
    rng = np.random.default_rng(5)
    N = 1 << 13
    x = rng.standard_normal(N) + _chirp(N, 700.6, -5.3, [0.3, 0.2])
    Xh = O.normalise(O.real_spectrum(x), 256)
    zmax, dz, levels = 20.0, 2.0, 5
    h = O.halfwidth(zmax)
    izc = int(round(zmax / dz))
    for nh, k, iz in [(1, 701, izc - 3), (2, 1401, izc - 5)]:
        r, z, S, _ = O.refine(Xh, k, iz, nh, zmax=zmax, dz=dz, h=h, levels=levels)
        ends = O.refine_endpoints(Xh, k, iz, nh, zmax=zmax, dz=dz, h=h, levels=levels, tol=lambda s: 0.0)
        assert ends == {(r, z): S}


def test_refine_respects_the_bank_edge():
    # A candidate at the largest drift: no point with |nh z| > zmax is taken.
    rng = np.random.default_rng(8)
    N = 1 << 12
    x = rng.standard_normal(N) + _chirp(N, 500.2, 21.0, [0.5])
    Xh = O.normalise(O.real_spectrum(x), 256)
    zmax, dz = 20.0, 2.0
    h = O.halfwidth(zmax)
    izc = 10
    r, z, S, _ = O.refine(Xh, 500, 2 * izc, 1, zmax=zmax, dz=dz, h=h, levels=6)
    assert abs(z) <= zmax
    assert S >= O.interp_power(Xh, 500.0, 20.0, h)


def test_half_bin_columns_are_interpolated_power():
    # The half-bin plane interleaves the plane (even columns) with the
    # correlation at k + 1/2 (odd columns), which must equal the interpolated
    # power there, ends included.
    rng = np.random.default_rng(21)
    N = 1 << 12
    x = rng.standard_normal(N) + _chirp(N, 300.5, -6.0, [0.3])
    res = O.search(x, zmax=10.0, dz=2.0, sigma=3.0, nharm_max=2, W=256, interbin=True)
    P2, Xh, h = res.plane, res.spectrum, res.h
    taps, zs, _ = O.template_taps(10.0, 2.0)
    assert P2.shape == (zs.size, N)
    assert np.array_equal(P2[:, 0::2], O.correlate(Xh, taps))
    nb = Xh.shape[0]
    cells = [(0, 0), (2, 300), (3, 299), (5, nb - 1), (10, nb - 2), (7, h - 1)]
    cells += [(int(i), int(k)) for i, k in zip(rng.integers(0, zs.size, 10), rng.integers(0, nb, 10))]
    for iz, k in cells:
        want = O.interp_power(Xh, k + 0.5, float(zs[iz]), h)
        assert abs(P2[iz, 2 * k + 1] - want) <= 1e-11 * max(want, 1.0), (iz, k)
    assert all(abs(c.r * 2 * c.nharm - c.k) < 1e-9 for c in res.candidates)


def test_half_bin_plane_recovers_tone_between_bins():
    # A noiseless tone halfway between bins 700 and 701 at a bank drift: the
    # plane keeps sinc^2(1/2) = 0.405 of its matched power, the half-bin
    # column all of it (the captured energy), and the strongest candidate sits
    # exactly at r = 700.5.
    N, rbar, zbar, a = 1 << 13, 700.5, 4.0, 10.0
    Xh = O.real_spectrum(a * _chirp(N, rbar, zbar, [1.0])) / (N / 2)
    zmax, dz = 10.0, 2.0
    res = O.search(spectrum=Xh, normalised=True, zmax=zmax, dz=dz, sigma=6.0, nharm_max=1, interbin=True)
    h = res.h
    full = a * a * _captured(rbar, zbar, h)
    iz = int(round((zbar + zmax) / dz))
    assert abs(res.plane[iz, 1401] / full - 1.0) < 1e-3
    assert res.plane[iz, 1400] / full == pytest.approx(np.sinc(0.5) ** 2, rel=2e-2)
    best = max(res.candidates, key=lambda c: c.power)
    assert (best.k, best.iz, best.r, best.z) == (1401, iz, 700.5, zbar)
