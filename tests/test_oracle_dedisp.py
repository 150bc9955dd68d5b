"""Pins of the oracle's de-dispersion (the step before the search, Sec. 1):
the dispersion constant against physical constants, the delays' shape, the
sums against a brute-force loop, and a dispersed pulse brought back to one
sample."""
import math

import numpy as np
import pytest
from scipy import constants as C

import oracle as O
import synth


def test_dispersion_constant_from_physical_constants():
    # delay = e^2 / (8 pi^2 eps0 m_e c) DM / f^2 in SI units, DM in
    # electrons per m^2 (1 pc cm^-3 = parsec x 1e6 m^-2), f in Hz
    k = C.e ** 2 / (8 * math.pi ** 2 * C.epsilon_0 * C.m_e * C.c) * C.parsec * 1e6 / 1e12
    assert O.KDM == pytest.approx(k, rel=1e-5)
    # 100 pc cm^-3 delays 1400 MHz by 0.2117 s against infinite frequency
    assert O.KDM * 100 / 1400.0 ** 2 == pytest.approx(0.21167, rel=1e-4)


def test_delays_are_zero_at_dm_zero_and_grow_down_the_band():
    d = O.dm_delays(64, 1500.0, 4.0, 5e-4, [0.0, 10.0, 300.0])
    assert np.all(d[0] == 0)
    assert np.all(d[:, 0] == 0)
    assert np.all(np.diff(d[1:], axis=1) >= 0)
    assert np.all(d[2] >= d[1])
    # rounding to the nearest sample
    f = 1500.0 - 4.0 * 63
    exact = O.KDM * 300.0 * (1 / f ** 2 - 1 / 1500.0 ** 2) / 5e-4
    assert abs(d[2, 63] - exact) <= 0.5


def test_dedisperse_brute_force():
    rng = np.random.default_rng(3)
    fil = rng.integers(0, 256, size=(6, 300), dtype=np.uint8)
    dms = [0.0, 40.0, 95.5]
    d = O.dm_delays(6, 1400.0, 20.0, 1e-3, dms)
    nout = 300 - int(d.max())
    y = O.dedisperse(fil, 1400.0, 20.0, 1e-3, dms, nout)
    for i in range(len(dms)):
        for t in range(nout):
            assert y[i, t] == sum(int(fil[c, t + d[i, c]]) for c in range(6))
    assert np.array_equal(y[0], fil[:, :nout].astype(np.int64).sum(axis=0).astype(np.float64))
    with pytest.raises(ValueError):
        O.dedisperse(fil, 1400.0, 20.0, 1e-3, dms, nout + 1)


def test_dispersed_pulse_comes_back_to_one_sample():
    # an impulse in every channel at the delay of DM 60 adds up to nchan x 100
    # at that DM and spreads at others
    nchan, nsamp, dm0, t0 = 32, 2048, 60.0, 100
    d = O.dm_delays(nchan, 1500.0, 8.0, 1e-3, [dm0])[0]
    fil = np.zeros((nchan, nsamp), dtype=np.uint8)
    fil[np.arange(nchan), t0 + d] = 100
    y = O.dedisperse(fil, 1500.0, 8.0, 1e-3, [dm0, 0.0, 2 * dm0], nsamp - 2 * int(d.max()) - 1)
    assert y[0, t0] == nchan * 100 and y[0].sum() == nchan * 100
    assert y[1].max() < nchan * 100 / 4 and y[2].max() < nchan * 100 / 4


def test_synthetic_pulsar_peaks_at_its_dm():
    fil = synth.make_filterbank(64, 1 << 13, 1500.0, 5.0, 5e-4, seed=7,
                                pulsars=[synth.Dispersed(period=0.05, dm=80.0, width=1e-3, amp=12.0)])
    dms = np.arange(0.0, 161.0, 10.0)
    d = O.dm_delays(64, 1500.0, 5.0, 5e-4, dms)
    y = O.dedisperse(fil, 1500.0, 5.0, 5e-4, dms, (1 << 13) - int(d.max()))
    # folded at the period, the pulse is sharpest at the injected DM
    per = int(round(0.05 / 5e-4))
    n = (y.shape[1] // per) * per
    prof = y[:, :n].reshape(len(dms), -1, per).mean(axis=1)
    contrast = prof.max(axis=1) - np.median(prof, axis=1)
    assert dms[int(np.argmax(contrast))] == 80.0
