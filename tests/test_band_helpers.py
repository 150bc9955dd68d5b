"""The banded full-size checks (tests/parity.py) against the oracle's whole-
plane harmonic sums and peaks on a small case, and their sensitivity to a
dropped or an added candidate (CPU)."""
import numpy as np

import oracle as O
import synth
from parity import band_sums, compare_band


def _small():
    t = synth.make_series(1 << 14, seed=41, pulsars=[synth.Pulsar(r=700.3, z=9.0, amp=0.12, nharm=6)])
    Xh = O.normalise(O.real_spectrum(t.x), 256)
    taps, zs, h = O.template_taps(20.0, 2.0)
    return Xh, taps, (zs.shape[0] - 1) // 2


def _oracle_cands(P, izc, thr, nhs):
    rec = []
    for nh in nhs:
        S = P if nh == 1 else O.harmonic_sum(P, nh, izc)
        for iz, k in O.find_peaks(S, thr[nh]):
            rec.append((int(k), int(iz), nh, float(S[iz, k])))
    out = np.zeros(len(rec), dtype=[("k", "<i8"), ("iz", "<i4"), ("nharm", "<i4"), ("power", "<f4")])
    for i, (k, iz, nh, s) in enumerate(rec):
        out[i] = (k, iz, nh, s)
    return out


def test_band_sums_equal_whole_plane_sums():
    Xh, taps, izc = _small()
    P = O.correlate(Xh, taps)
    nb = Xh.shape[0]
    nhs = [1, 2, 4, 8, 16]
    for k0, k1 in ((0, 300), (1000, 1400), (nb - 257, nb), (4000, 4001)):
        a, sums = band_sums(Xh, taps, izc, k0, k1, nhs)
        assert a == max(k0 - 1, 0)
        for nh in nhs:
            full = P if nh == 1 else O.harmonic_sum(P, nh, izc)
            want = full[:, a:a + sums[nh].shape[1]]
            assert np.max(np.abs(sums[nh] - want)) <= 1e-9 * max(1.0, np.max(want))


def test_compare_band_accepts_the_oracle_and_catches_changes():
    Xh, taps, izc = _small()
    P = O.correlate(Xh, taps)
    nhs = [1, 2, 4, 8, 16]
    thr = O.thresholds(4.5, nhs)
    cands = _oracle_cands(P, izc, thr, nhs)
    k0, k1 = 600, 1500
    a, sums = band_sums(Xh, taps, izc, k0, k1, nhs)
    rep = compare_band(cands, sums, thr, a, k0, k1)
    assert rep["ok"] and rep["n_orc"] > 20 and rep["common"] == rep["n_orc"], rep
    inside = np.nonzero((cands["k"] >= k0) & (cands["k"] < k1))[0]
    # a dropped candidate is missing
    drop = np.delete(cands, inside[len(inside) // 2])
    rep = compare_band(drop, sums, thr, a, k0, k1)
    assert not rep["ok"] and len(rep["missing"]) == 1
    # a candidate moved by one bin is both missing and extra
    moved = cands.copy()
    moved["k"][inside[0]] += 1
    rep = compare_band(moved, sums, thr, a, k0, k1)
    assert not rep["ok"] and rep["missing"] and rep["extra"]
    # a power off by 1e-3 relative fails the 1e-4 bound
    off = cands.copy()
    off["power"][inside[1]] *= 1.001
    rep = compare_band(off, sums, thr, a, k0, k1)
    assert not rep["ok"] and rep["max_err_fraction"] > 1.0
    # candidates outside the band are ignored
    rep = compare_band(cands[cands["k"] < k0], sums, thr, a, k0, k1)
    assert not rep["ok"] and len(rep["missing"]) == rep["n_orc"]
