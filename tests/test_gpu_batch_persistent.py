"""The persistent batch launch (segment lengths 4096 and 8192): many trials
of uneven lengths through one launch of the persistent kernel, whose work
queue runs every trial's segment DFTs, correlation tiles, harmonic-sum screen,
exact sums and neighbour tests.  Each trial's records must be bit-identical
to the same trial searched alone, whatever the batch around it (more trials
than plane slots, two launches past 64 trials); one batched trial is checked
against the FP64 oracle (Sec. 2, Eq. (1); Sec. 4 steps 2-7)."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import compare_candidates

pytestmark = pytest.mark.gpu

ZMAX, DZ = 100.0, 2.0
OPTS = dict(nharm_max=16, sigma=5.0)
PERSISTENT = dict(OPTS, batch_launch="persistent")


def _dev(x):
    import torch
    return torch.from_numpy(x).cuda()


def _trials(lens, seed0):
    out = []
    for i, n in enumerate(lens):
        ps = [] if i % 3 == 1 else [synth.Pulsar(r=n / 7.3 + 11.5 * i, z=9.0 - 4.0 * i, amp=0.07, nharm=4)]
        out.append(synth.make_series(n, seed=seed0 + i, pulsars=ps))
    return out


def _alone(gpu_lib, bank, seg, trials, cap):
    want = []
    for t in trials:
        p = gpu_lib.Plan(bank, t.nsamp, seg, **OPTS)
        want.append(p.search(_dev(t.x), cap=cap)[0])
        p.close()
    return want


@pytest.mark.parametrize("seg", [4096, 8192])
def test_persistent_batch_equals_alone(gpu_lib, seg):
    # 9 trials of uneven lengths: more than the 4 plane slots, so slots are reused
    lens = [1 << 18, 1 << 16, 1 << 17, 1 << 18, 1 << 15, 1 << 18, 1 << 17, 1 << 16, 1 << 18]
    trials = _trials(lens, 300)
    bank = gpu_lib.make_templates(ZMAX, DZ)
    plan = gpu_lib.Plan(bank, 1 << 18, seg, **PERSISTENT)
    xs = [_dev(t.x) for t in trials]
    print(f"persistent batch: seg {seg}, {len(xs)} trials", flush=True)
    got = plan.search_batch(xs, caps=[200000] * len(xs))
    again = plan.search_batch(xs[::-1], caps=[200000] * len(xs))[::-1]  # another order, other slots
    want = _alone(gpu_lib, bank, seg, trials, 200000)
    levels = set()
    for i, (a, b, w) in enumerate(zip(got, again, want)):
        assert np.array_equal(a, w), (i, len(a), len(w))
        assert np.array_equal(b, w), i
        levels |= set(int(v) for v in np.unique(a["nharm"]))
    assert levels == {1, 2, 4, 8, 16}
    plan.close()
    bank.close()


def test_persistent_batch_trial_matches_oracle(gpu_lib):
    lens = [1 << 16, 1 << 17, 1 << 16, 1 << 15, 1 << 17]
    trials = _trials(lens, 400)
    bank = gpu_lib.make_templates(ZMAX, DZ)
    plan = gpu_lib.Plan(bank, 1 << 17, 4096, **PERSISTENT)
    got = plan.search_batch([_dev(t.x) for t in trials], caps=[100000] * len(trials))
    plan.close()
    bank.close()
    t = trials[2]  # 2^16 samples with a 4-harmonic pulsar
    orc = O.search(t.x, zmax=ZMAX, dz=DZ, sigma=OPTS["sigma"], nharm_max=OPTS["nharm_max"], W=1024, keep_sums=True)
    rep = compare_candidates(got[2], orc)
    assert rep["ok"], rep
    assert rep["n_orc"] > 20


def test_persistent_batch_two_launches(gpu_lib):
    # 67 short trials: two launches of the persistent kernel (64 + 3)
    lens = [1 << 14 if i % 2 else 1 << 15 for i in range(67)]
    trials = _trials(lens, 500)
    bank = gpu_lib.make_templates(ZMAX, DZ)
    plan = gpu_lib.Plan(bank, 1 << 15, 4096, **PERSISTENT)
    got = plan.search_batch([_dev(t.x) for t in trials], caps=[50000] * len(trials))
    want = _alone(gpu_lib, bank, 4096, trials, 50000)
    for i, (a, w) in enumerate(zip(got, want)):
        assert np.array_equal(a, w), i
    assert sum(len(a) for a in got) > 0
    plan.close()
    bank.close()


def test_persistent_batch_overflow_reports_counts(gpu_lib):
    trials = _trials([1 << 16, 1 << 16], 600)
    bank = gpu_lib.make_templates(ZMAX, DZ)
    plan = gpu_lib.Plan(bank, 1 << 16, 4096, **PERSISTENT)
    xs = [_dev(t.x) for t in trials]
    full = plan.search_batch(xs, caps=[100000, 100000])
    assert len(full[0]) > 3
    with pytest.raises(gpu_lib.FdasError) as e:
        plan.search_batch(xs, caps=[3, 100000])
    assert e.value.status == -4
    plan.close()
    bank.close()


def test_stream_launch_equals_persistent(gpu_lib):
    # the other launch form of fdas_search_batch (per-trial graphs on two
    # streams) on the same trials gives the same records
    lens = [1 << 17, 1 << 16, 1 << 17, 1 << 15, 1 << 17, 1 << 16]
    trials = _trials(lens, 800)
    bank = gpu_lib.make_templates(ZMAX, DZ)
    xs = [_dev(t.x) for t in trials]
    a = gpu_lib.Plan(bank, 1 << 17, 4096, **PERSISTENT)
    b = gpu_lib.Plan(bank, 1 << 17, 4096, batch_launch="streams", **OPTS)
    got_a = a.search_batch(xs, caps=[100000] * len(xs))
    got_b = b.search_batch(xs, caps=[100000] * len(xs))
    for i, (x, y) in enumerate(zip(got_a, got_b)):
        assert np.array_equal(x, y), i
    with pytest.raises(ValueError):
        gpu_lib.Plan(bank, 1 << 17, 4096, batch_launch="both", **OPTS)
    a.close()
    b.close()
    bank.close()


def test_stream_batch_into_page_locked_buffer(gpu_lib):
    # the default launch form with a page-locked record buffer returns what it
    # copies into pageable memory; a capacity below a trial's count reports
    # OVERFLOW
    lens = [1 << 16, 1 << 15, 1 << 16, 1 << 16, 1 << 15]
    trials = _trials(lens, 900)
    bank = gpu_lib.make_templates(ZMAX, DZ)
    xs = [_dev(t.x) for t in trials]
    plan = gpu_lib.Plan(bank, 1 << 16, 4096, **OPTS)
    caps = [100000] * len(xs)
    ref = plan.search_batch(xs, caps=caps)
    assert len(ref[0]) > 3
    got = plan.search_batch(xs, caps=caps, out=gpu_lib.pinned_candidates(sum(caps)))
    for i, (a, b) in enumerate(zip(got, ref)):
        assert np.array_equal(a, b), i
    small = [3] + caps[1:]
    with pytest.raises(gpu_lib.FdasError) as e:
        plan.search_batch(xs, caps=small, out=gpu_lib.pinned_candidates(sum(small)))
    assert e.value.status == -4
    plan.close()
    bank.close()
