"""Served results against the FP64 oracle: requests of uneven lengths (the
served mix's 2^21 / 2^22 / 2^23 classes, scaled to 2^19 / 2^20 / 2^21 so the
oracle finishes in seconds) submitted to one server while others run; the
candidates of every request with a pulsar are compared, in both directions,
with the oracle's complete candidate set on bands of top-harmonic columns
around the pulsar's harmonics and in the noise (Sec. 2 Eq. (1), Sec. 4)."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import band_sums, compare_band

pytestmark = pytest.mark.gpu

ZMAX, DZ, SEG, NHARM, SIGMA = 200.0, 2.0, 8192, 16, 6.0
B = 1024


def test_served_requests_match_oracle(gpu_lib):
    lens = [1 << 21, 1 << 19, 1 << 20, 1 << 21, 1 << 19, 1 << 20]
    reqs = []
    for i, n in enumerate(lens):
        ps = [synth.Pulsar(r=n / 11.3 + 37.25 * i, z=60.0 - 25.0 * i, amp=0.03, nharm=8)] if i % 2 == 0 else []
        reqs.append(synth.make_series(n, seed=700 + i, pulsars=ps))
    bank = gpu_lib.make_templates(ZMAX, DZ)
    srv = gpu_lib.Server(bank, SEG, max(lens), hbm_budget=0, max_slots=3, nharm_max=NHARM, sigma=SIGMA)
    for i, t in enumerate(reqs):
        srv.submit(t.x, tag=i)
    got = {}
    for _ in reqs:
        tag, c, n, lat = srv.poll(timeout_ms=120000, cap=1 << 20)
        assert n == len(c)
        got[tag] = c
    srv.close()
    taps, zs, h = O.template_taps(ZMAX, DZ)
    izc = (zs.shape[0] - 1) // 2
    nhs = O.harmonic_list(NHARM)
    thr = O.thresholds(SIGMA, nhs)
    checked = 0
    for i, t in enumerate(reqs):
        if not t.pulsars:
            continue
        nb = t.nsamp // 2
        Xh = O.normalise(O.real_spectrum(t.x), 1024)
        p = t.pulsars[0]
        bands = [(nb // 2, nb // 2 + B)]
        for hm in range(1, p.nharm + 1):
            c = int(round(hm * p.r))
            if B // 2 <= c < nb - B // 2:
                bands.append((c - B // 2, c + B // 2))
        print(f"request {i}: {t.nsamp} samples, {len(got[i])} candidates, {len(bands)} bands", flush=True)
        for k0, k1 in bands:
            a, sums = band_sums(Xh, taps, izc, k0, k1, nhs)
            rep = compare_band(got[i], sums, thr, a, k0, k1)
            assert rep["ok"], (i, k0, k1, {k: (v[:10] if isinstance(v, list) else v) for k, v in rep.items()})
            checked += rep["n_orc"]
    assert checked > 200
    bank.close()
