"""De-dispersion (fdas_dedisperse) on the GPU against the oracle, through the
C ABI: integer sums, so bit-exact; the argument checks; and the front end
feeding the search (a dispersed pulsar found in the series of its DM)."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("nchan,nsamp,f_top,foff,tsamp,dms", [
    (16, 4099, 1500.0, 12.5, 1e-3, [0.0, 17.3, 50.0, 133.7]),            # ragged nout
    (1, 2048, 800.0, 0.0, 5e-4, [0.0, 100.0]),                           # one channel: all delays 0
    (257, 1 << 14, 1450.0, 1.171875, 2.56e-4, list(np.arange(0.0, 96.0, 3.0))),
    (64, 20000, 400.0, 1.5, 1e-4, [7.0]),                                # low band, long delays
    (8, 40000, 400.0, 10.0, 1e-4, [0.0, 200.0, 3.0]),                    # 24,300-sample delays, unsorted DMs
])
def test_dedisperse_bit_exact(gpu_lib, nchan, nsamp, f_top, foff, tsamp, dms):
    fil = synth.make_filterbank(nchan, nsamp, f_top, foff, tsamp, seed=nchan,
                                pulsars=[synth.Dispersed(period=0.031, dm=40.0, width=5e-4, amp=30.0)])
    d = O.dm_delays(nchan, f_top, foff, tsamp, dms)
    nout = nsamp - int(d.max())
    assert nout > 0
    got = gpu_lib.dedisperse(_dev(fil), f_top, foff, tsamp, dms, nout).cpu().numpy()
    want = O.dedisperse(fil, f_top, foff, tsamp, dms, nout)
    assert np.array_equal(got.astype(np.float64), want)


def test_dedisperse_rejects_bad_arguments(gpu_lib):
    fil = _dev(synth.make_filterbank(8, 1024, 1500.0, 10.0, 1e-3, seed=1))
    d = O.dm_delays(8, 1500.0, 10.0, 1e-3, [100.0])
    with pytest.raises(gpu_lib.FdasError):  # one sample past what the channels supply
        gpu_lib.dedisperse(fil, 1500.0, 10.0, 1e-3, [100.0], 1024 - int(d.max()) + 1)
    with pytest.raises(gpu_lib.FdasError):  # a channel at or below 0 MHz
        gpu_lib.dedisperse(fil, 60.0, 10.0, 1e-3, [0.0], 100)
    with pytest.raises(gpu_lib.FdasError):
        gpu_lib.dedisperse(fil, 1500.0, 10.0, 1e-3, [-1.0], 100)
    with pytest.raises(gpu_lib.FdasError):
        gpu_lib.dedisperse(fil, 1500.0, 10.0, 0.0, [0.0], 100)


def test_front_end_feeds_the_search(gpu_lib):
    # a dispersed pulsar of period P in a 64-channel filterbank: de-dispersed
    # at its DM the series holds harmonics at k = T / P (T = 2^15 samples), and
    # the search of that series reports its fundamental there; the GPU series
    # equals the oracle's, so the oracle's search of it is the reference
    nchan, f_top, foff, tsamp = 64, 1500.0, 4.0, 5e-4
    nout = 1 << 15
    dms = [0.0, 45.0, 90.0, 135.0]
    d = O.dm_delays(nchan, f_top, foff, tsamp, dms)
    nsamp = nout + int(d.max())
    period = 0.0413
    fil = synth.make_filterbank(nchan, nsamp, f_top, foff, tsamp, seed=5,
                                pulsars=[synth.Dispersed(period=period, dm=90.0, width=8e-4, amp=6.0)])
    series = gpu_lib.dedisperse(_dev(fil), f_top, foff, tsamp, dms, nout)
    assert np.array_equal(series.cpu().numpy().astype(np.float64), O.dedisperse(fil, f_top, foff, tsamp, dms, nout))
    bank = gpu_lib.make_templates(10.0, 2.0)
    plan = gpu_lib.Plan(bank, nout, 256, nharm_max=8, sigma=8.0, median_window=512)
    r0 = nout * tsamp / period  # fundamental in bins
    best = []
    for i in range(len(dms)):
        c, _ = plan.search(series[i].contiguous())
        best.append(float(c["power"].max()) if len(c) else 0.0)
        if dms[i] == 90.0:
            top = c[np.argmax(c["power"])]
            assert abs(top["r"] - r0) <= 0.51 and abs(top["z"]) <= 1.0
    assert int(np.argmax(best)) == 2
    plan.close()
    bank.close()
