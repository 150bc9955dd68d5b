"""The allocation-free refinement entry point (fdas_refine_noalloc) against
fdas_refine, through the C ABI: identical records on two calls in a row, the
second with fewer records, and its size limit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_refine_noalloc_matches_refine(gpu_lib):
    import torch
    n = 1 << 17
    t = synth.make_series(n, seed=90, pulsars=[synth.Pulsar(r=20000.3, z=40.0, amp=0.06, nharm=4),
                                                synth.Pulsar(r=9000.7, z=-22.0, amp=0.05, nharm=2)])
    bank = gpu_lib.make_templates(100.0, 2.0)
    plan = gpu_lib.Plan(bank, n, 2048, nharm_max=4, sigma=4.5)
    cands, nf = plan.search(torch.from_numpy(t.x).cuda())
    assert nf == len(cands) >= 120
    order = np.argsort(-cands["sigma"], kind="stable")
    first, second = cands[order[:120]], cands[order[200:237]]
    for recs in (first, second):  # two calls in a row, the second smaller
        want = plan.refine(recs, 5)
        got = plan.refine_noalloc(recs, 5)
        assert np.array_equal(got, want)
        assert np.any(got["power"] != recs["power"])  # the records were refined
    # the larger first call's records do not leak into the smaller second's
    again = plan.refine_noalloc(second, 5)
    assert np.array_equal(again, plan.refine(second, 5))
    # beyond the fixed array: a clear INVAL, nothing refined
    big = np.repeat(first[:1], plan.REFINE_NOALLOC_MAX + 1)
    with pytest.raises(gpu_lib.FdasError) as e:
        plan.refine_noalloc(big, 2)
    assert e.value.status == -1 and "FDAS_REFINE_NOALLOC_MAX" in e.value.message
    # an empty call is a no-op
    assert plan.refine_noalloc(first[:0], 2).size == 0
    plan.close()
    bank.close()
