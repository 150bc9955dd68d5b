"""Pins of the oracle's spectrum, normalisation, correlation, harmonic sum,
thresholds and peak rule against brute force, closed forms and library
routines that the oracle itself does not call."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- spectrum
def test_real_spectrum_vs_naive_dft():
    rng = np.random.default_rng(11)
    n = 512
    x = rng.standard_normal(n)
    X = O.real_spectrum(x)
    nn = np.arange(n)
    naive = np.array([np.sum(x * np.exp(-2j * np.pi * k * nn / n)) for k in range(n // 2)])
    naive[0] = 0.0
    assert X.shape == (n // 2,)
    assert np.max(np.abs(X - naive)) < 1e-10


def test_real_spectrum_parseval():
    rng = np.random.default_rng(12)
    n = 4096
    x = rng.standard_normal(n) + 0.3
    X = O.real_spectrum(x)
    full = np.fft.fft(x)
    # sum x^2 = (|F0|^2 + 2 sum_{0<k<N/2} |Fk|^2 + |F_{N/2}|^2) / N
    lhs = np.sum(x * x)
    rhs = (abs(full[0]) ** 2 + 2 * np.sum(np.abs(X[1:]) ** 2) + abs(full[n // 2]) ** 2) / n
    assert abs(lhs - rhs) < 1e-9 * lhs
    assert X[0] == 0


# ---------------------------------------------------------------- normalisation
def test_block_medians_are_order_statistics():
    rng = np.random.default_rng(13)
    p = rng.exponential(size=5000)
    med, cen = O.block_medians(p, 1024)
    assert med.shape == (5,)
    for b in range(5):
        blk = np.sort(p[b * 1024:(b + 1) * 1024])
        w = blk.shape[0]
        want = blk[w // 2] if w % 2 else 0.5 * (blk[w // 2 - 1] + blk[w // 2])
        assert med[b] == want
    assert cen[0] == 511.5 and cen[4] == 4096 + (904 - 1) / 2


def test_median_curve_interpolates_between_centres():
    # blocks of W = 4 with constant powers 1, 3, 7: medians 1, 3, 7 at
    # centres 1.5, 5.5, 9.5; linear in between, flat outside.
    p = np.array([1.0] * 4 + [3.0] * 4 + [7.0] * 4)
    m = O.median_curve(p, 4)
    assert m[0] == 1.0 and m[1] == 1.0
    assert m[2] == pytest.approx(1.0 + 2.0 * 0.5 / 4)
    assert m[5] == pytest.approx(3.0 - 2.0 * 0.5 / 4)
    assert m[6] == pytest.approx(3.0 + 4.0 * 0.5 / 4)
    assert m[10] == 7.0 and m[11] == 7.0


def test_normalised_white_noise_is_unit_exponential():
    t = synth.make_series(1 << 17, seed=21)
    X = O.normalise(O.real_spectrum(t.x), 1024)
    p = np.abs(X[1:]) ** 2
    assert abs(p.mean() - 1.0) < 0.02
    assert stats.kstest(p, "expon").pvalue > 1e-3
    # the median of the raw power is N ln 2 per bin for unit-variance noise
    raw = np.abs(O.real_spectrum(t.x)[1:]) ** 2
    assert abs(np.median(raw) / ((1 << 17) * math.log(2)) - 1.0) < 0.02


def test_zero_spectrum_normalises_to_zero():
    X = np.zeros(4096, dtype=complex)
    assert np.all(O.normalise(X, 1024) == 0)


# ---------------------------------------------------------------- correlation
def test_direct_correlation_equals_convolution_theorem():
    # Independent route: zero-padded linear convolution through numpy's FFT.
    rng = np.random.default_rng(31)
    nb, h = 300, 7
    X = rng.standard_normal(nb) + 1j * rng.standard_normal(nb)
    taps = rng.standard_normal((3, 2 * h + 1)) + 1j * rng.standard_normal((3, 2 * h + 1))
    P = O.correlate(X, taps)
    L = nb + 2 * h + 1
    for iz in range(3):
        full = np.fft.ifft(np.fft.fft(X, 2 * L) * np.fft.fft(taps[iz], 2 * L))[: nb + 2 * h]
        # taps index 0 is q = -h, so output k sits at position k + h
        y = full[h: h + nb]
        assert np.max(np.abs(P[iz] - np.abs(y) ** 2)) < 1e-9 * np.max(np.abs(y) ** 2)


def test_direct_correlation_bruteforce_tiny():
    # Python loop over the definition on a tiny case, asymmetric taps so that
    # a reversed or shifted tap index cannot pass.
    X = np.array([1 + 2j, -0.5j, 3.0, 0.25 - 1j, 2 + 2j], dtype=complex)
    taps = np.array([[0.1 + 0.2j, -1.0, 0.5j]])  # q = -1, 0, +1
    P = O.correlate(X, taps)
    for k in range(5):
        y = 0
        for q in (-1, 0, 1):
            if 0 <= k - q < 5:
                y += X[k - q] * taps[0, q + 1]
        assert abs(P[0, k] - abs(y) ** 2) < 1e-13
    cells = O.correlate_cells(X, taps, [0, 0], [0, 4])
    assert np.allclose(cells, P[0, [0, 4]], rtol=0, atol=0)


def test_zero_drift_row_is_power_spectrum():
    t = synth.make_series(1 << 14, seed=32)
    r = O.search(t.x, zmax=20.0, dz=2.0, nharm_max=1, W=256)
    iz0 = int(np.nonzero(r.zs == 0.0)[0][0])
    assert np.max(np.abs(r.plane[iz0] - np.abs(r.spectrum) ** 2)) < 1e-12 * np.max(r.plane[iz0])


def test_noiseless_tone_recovered_in_one_cell():
    # Sec. 2: the conjugate filter returns a drifting tone's leaked power to the
    # single cell at its (r0, z0); off-peak cells follow |A(r0 - k, z0 - z)|^2.
    g = json.load(open(os.path.join(GOLDEN, "single_tone_peak.json")))
    n, a = g["nsamp"], 0.05
    t = synth.single_tone_series(n=n, r=g["r0"], z=g["z0"], amp=a, noise_sigma=0.0)
    X = O.real_spectrum(t.x.astype(np.float64)) / (a * n / 2)
    taps, zs, h = O.template_taps(100.0, 2.0)
    iz = np.arange(zs.shape[0])
    ks = np.arange(19900, 20100)
    P = np.stack([O.correlate_cells(X, taps, np.full(ks.shape, i), ks) for i in iz])
    i_pk, k_pk = np.unravel_index(np.argmax(P), P.shape)
    assert ks[k_pk] == g["expected_peak_k"] and zs[i_pk] == g["expected_peak_z"]
    for dz_off in (0.0, 2.0, -2.0, 10.0):
        z = g["z0"] + dz_off
        i = int(np.nonzero(zs == z)[0][0])
        kept = np.sum(np.abs(O.template_response(np.arange(-h, h + 1.0), z)) ** 2)
        for k in (19995, 20000, 20001, 20010):
            want = abs(O.template_response(np.array([g["r0"] - k]), g["z0"] - z)[0]) ** 2 / kept
            got = P[i, k - ks[0]]
            assert abs(got - want) < 2e-3 * max(want, 0.05), (z, k, got, want)
    i0 = int(np.nonzero(zs == g["z0"])[0][0])
    assert P[i0, 20000 - ks[0]] == pytest.approx(g["sinc2_0p3"], rel=3e-3)


def test_single_tone_workload_peak():
    g = json.load(open(os.path.join(GOLDEN, "single_tone_peak.json")))
    t = synth.single_tone_series()
    r = O.search(t.x, zmax=100.0, dz=2.0, sigma=6.0, nharm_max=1)
    top = max(r.candidates, key=lambda c: c.power)
    assert top.k == g["expected_peak_k"] and top.z == g["expected_peak_z"] and top.nharm == 1
    assert r.plane.shape == (101, 65536)
    assert abs(r.plane.mean() - 1.0) < 0.01


# ---------------------------------------------------------------- harmonic sum
def _round_half_away(fr: Fraction) -> int:
    s = 1 if fr >= 0 else -1
    a = abs(fr)
    return s * int(math.floor(a + Fraction(1, 2)))


def _harm_bruteforce(P, nh, izc):
    nz, nb = P.shape
    S = np.zeros_like(P)
    for iz in range(nz):
        for k in range(nb):
            for j in range(1, nh + 1):
                kj = _round_half_away(Fraction(j * k, nh))
                izj = izc + _round_half_away(Fraction(j * (iz - izc), nh))
                S[iz, k] += P[izj, kj]
    return S


@pytest.mark.parametrize("nh", [1, 2, 4, 8, 16])
def test_harmonic_sum_bruteforce(nh):
    rng = np.random.default_rng(40 + nh)
    P = rng.exponential(size=(9, 70))
    S = O.harmonic_sum(P, nh, izc=4)
    assert np.max(np.abs(S - _harm_bruteforce(P, nh, 4))) < 1e-12


def test_harmonic_sum_closed_form_on_ramp():
    # P[iz, k] = k: S_nh(k) = sum_j round(j k / nh), independent of iz
    nb, nz, izc = 400, 5, 2
    P = np.tile(np.arange(nb, dtype=float), (nz, 1))
    for nh in (2, 4, 8, 16):
        S = O.harmonic_sum(P, nh, izc)
        for k in (0, 1, 7, 8, 15, 16, 17, 399):
            want = sum(_round_half_away(Fraction(j * k, nh)) for j in range(1, nh + 1))
            assert np.all(S[:, k] == want)
    # harmonic nh of the sum is the cell itself; all reads stay in range
    kj, izj = O.harmonic_indices(np.arange(nb), np.arange(nz), 16, 16, izc)
    assert np.all(kj == np.arange(nb)) and np.all(izj == np.arange(nz))


def test_harmonic_sum_cells_matches_plane():
    rng = np.random.default_rng(44)
    P = rng.exponential(size=(11, 300))
    S = O.harmonic_sum(P, 8, 5)
    iz = rng.integers(0, 11, 50)
    k = rng.integers(0, 300, 50)
    got = O.harmonic_sum_cells(lambda a, b: P[a, b], iz, k, 8, 5)
    assert np.max(np.abs(got - S[iz, k])) < 1e-12


# ---------------------------------------------------------------- thresholds
def test_thresholds_closed_forms():
    sig = 6.0
    thr = O.thresholds(sig, [1, 2, 4, 8, 16])
    tail = stats.norm.sf(sig)
    # one harmonic: P(exp(1) >= t) = e^-t
    assert thr[1] == pytest.approx(-math.log(tail), rel=1e-12)
    # 2 x (sum of nh unit exponentials) is chi-square with 2 nh degrees of freedom
    for nh in (2, 4, 8, 16):
        assert thr[nh] == pytest.approx(stats.chi2.isf(tail, 2 * nh) / 2.0, rel=1e-9)
    for nh, want in zip((1, 2, 4, 8, 16), (20.737, 23.954, 29.169, 37.844, 52.606)):
        assert thr[nh] == pytest.approx(want, abs=6e-4)


def test_sigma_round_trip():
    for sig in (3.0, 6.0, 9.5):
        thr = O.thresholds(sig, [1, 4, 16])
        for nh, t in thr.items():
            assert O.sigma_of(t, nh) == pytest.approx(sig, abs=1e-9)
    # deep tail (no underflow): one harmonic, S = 2000 -> Phi_c(sigma) = e^-2000
    s = O.sigma_of(2000.0, 1)
    assert stats.norm.logsf(s) == pytest.approx(-2000.0, rel=1e-9)


# ---------------------------------------------------------------- peaks
def test_peak_rule_handmade():
    S = np.zeros((4, 6))
    S[1, 2] = 10.0           # clean peak
    S[3, 5] = 8.0            # peak on the corner
    S[0, 0] = S[0, 1] = 7.0  # plateau along k: only the earlier cell
    S[2, 4] = 9.0            # beaten by nothing (neighbour (3,5) = 8 is smaller)
    S[2, 2] = 9.5            # below its neighbour (1,2) = 10
    pk = O.find_peaks(S, 5.0)
    got = {tuple(v) for v in pk}
    assert got == {(1, 2), (0, 0), (2, 4)}
    # (3,5) = 8 is a neighbour of (2,4) = 9, so it is not a peak
    assert O.find_peaks(S, 9.8).tolist() == [[1, 2]]
    # a plateau across rows: the earlier row wins
    T = np.zeros((3, 3))
    T[0, 1] = T[1, 1] = 4.0
    assert O.find_peaks(T, 1.0).tolist() == [[0, 1]]
    # threshold is inclusive
    assert O.find_peaks(np.array([[2.0]]), 2.0).tolist() == [[0, 0]]


def test_peaks_bruteforce_random():
    rng = np.random.default_rng(50)
    S = rng.integers(0, 4, size=(7, 9)).astype(float)  # many ties
    pk = {tuple(v) for v in O.find_peaks(S, 2.0)}
    want = set()
    for i in range(7):
        for k in range(9):
            if S[i, k] < 2.0:
                continue
            ok = True
            for di in (-1, 0, 1):
                for dk in (-1, 0, 1):
                    if (di, dk) == (0, 0) or not (0 <= i + di < 7 and 0 <= k + dk < 9):
                        continue
                    n = S[i + di, k + dk]
                    before = (i + di) * 9 + (k + dk) < i * 9 + k
                    ok &= (S[i, k] > n) if before else (S[i, k] >= n)
            if ok:
                want.add((i, k))
    assert pk == want


def test_noise_candidate_rate_one_harmonic():
    # On pure noise the number of above-threshold local maxima is a small
    # fraction of cells * e^-thr; at sigma = 3 there are enough to count.
    t = synth.make_series(1 << 15, seed=60)
    r = O.search(t.x, zmax=10.0, dz=2.0, sigma=3.0, nharm_max=1, W=512)
    n_above = int(np.sum(r.plane >= r.thresholds[1]))
    expect = r.plane.size * stats.norm.sf(3.0)
    assert 0.6 * expect < n_above < 1.4 * expect
    assert 0 < len(r.candidates) <= n_above
