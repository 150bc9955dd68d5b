"""Host-memory input with the transfer overlapped (fdas_search_host), and the
isolation of fdas_search's state from batches, through the C ABI."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _series(n, seeds):
    return [synth.make_series(n, seed=s, pulsars=[synth.Pulsar(r=900.2 + 50 * s, z=6.0, amp=0.15, nharm=3)]).x
            for s in seeds]


def test_search_host_equals_device_search(gpu_lib):
    import torch
    n = 1 << 16
    xs = _series(n, [70, 71, 72, 73])
    bank = gpu_lib.make_templates(20.0, 2.0)
    opts = dict(nharm_max=4, sigma=5.0, median_window=256)
    plan = gpu_lib.Plan(bank, n, 512, **opts)
    ref = [plan.search(torch.from_numpy(x).cuda()) for x in xs]
    pinned = [torch.from_numpy(x).pin_memory() for x in xs]
    plane = torch.empty((bank.nz, n // 2), dtype=torch.float32, device="cuda")
    # a chain of prefetches: call i searches series i and starts copying i + 1
    for i in range(len(xs)):
        nxt = pinned[i + 1] if i + 1 < len(xs) else None
        got, nf = plan.search_host(pinned[i], next=nxt, plane=plane if i == 2 else None)
        assert nf == ref[i][1] and np.array_equal(got, ref[i][0]), i
        if i == 2:
            want = torch.empty_like(plane)
            plan.search(torch.from_numpy(xs[2]).cuda(), plane=want)
            assert torch.equal(plane, want)
    # a staged series that is not the one searched next is dropped, not used
    plan.search_host(pinned[0], next=pinned[1])
    got, nf = plan.search_host(pinned[3], next=pinned[1])
    assert nf == ref[3][1] and np.array_equal(got, ref[3][0])
    got, nf = plan.search_host(pinned[1])
    assert nf == ref[1][1] and np.array_equal(got, ref[1][0])
    # pageable numpy input and the same pointer as current and next
    for _ in range(2):
        got, nf = plan.search_host(xs[2], next=xs[2])
        assert nf == ref[2][1] and np.array_equal(got, ref[2][0])
    with pytest.raises(ValueError):
        plan.search_host(xs[0][: n // 2])
    plan.close()
    bank.close()


def test_batch_leaves_single_search_state(gpu_lib):
    """Refinement, interpolation, work counts and the spectrum hook describe
    the last fdas_search even after a batch ran on the same plan."""
    import torch
    n = 1 << 15
    xs = _series(n, [80, 81, 82])
    bank = gpu_lib.make_templates(20.0, 2.0)
    plan = gpu_lib.Plan(bank, n, 512, nharm_max=4, sigma=5.0, median_window=256)
    cands, nf = plan.search(torch.from_numpy(xs[0]).cuda())
    assert nf > 0
    top = cands[np.argsort(-cands["sigma"], kind="stable")[:8]]
    ref_refined = plan.refine(top, 4)
    ref_counts = plan.search_counts()
    spec0 = torch.empty(n // 2, dtype=torch.complex64, device="cuda")
    plan.fetch_spectrum(spectrum=spec0)
    r = top["r"].astype(np.float64)
    z = top["z"].astype(np.float64)
    ref_interp = plan.interp_power(r, z, top["nharm"])
    plan.search_batch([torch.from_numpy(x).cuda() for x in xs[1:]], caps=[1 << 16] * 2)
    torch.cuda.synchronize()
    assert np.array_equal(plan.refine(top, 4), ref_refined)
    assert plan.search_counts() == ref_counts
    assert np.array_equal(plan.interp_power(r, z, top["nharm"]), ref_interp)
    spec1 = torch.empty_like(spec0)
    plan.fetch_spectrum(spectrum=spec1)
    assert torch.equal(spec0, spec1)
    plan.close()
    bank.close()
