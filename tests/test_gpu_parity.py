"""GPU path vs the FP64 oracle, through the C ABI, on seeded synthetic inputs.

Small cases compare the whole plane element by element and the whole
candidate list; the full SKA-shaped trial (2^23 samples, 201 templates,
8192-bin segments, 16 harmonics) compares sampled cells and checks every GPU
candidate against the oracle's sums at that cell and its neighbours.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth
from parity import REL, compare_candidates, plane_errors

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run(fdas, x, zmax, dz, seg, kind=0, cap=1 << 22, **opts):
    import torch
    bank = fdas.make_templates(zmax, dz)
    nsamp = x.shape[0] if kind == 0 else 2 * x.shape[0]
    plan = fdas.Plan(bank, nsamp, seg, **opts)
    if kind == 0:
        inp = _dev(x.astype(np.float32))
    else:
        inp = _dev(x.astype(np.complex64))
    plane = torch.empty((bank.nz, nsamp // 2), dtype=torch.float32, device="cuda")
    cands, n = plan.search(inp, kind=kind, plane=plane, cap=cap)
    torch.cuda.synchronize()
    P = plane.cpu().numpy()
    plan.close()
    bank.close()
    return P, cands, n


# ------------------------------------------------------------------ DFT
@pytest.mark.parametrize("log2n", list(range(6, 14)))
def test_workgroup_dft_matches_numpy(gpu_lib, log2n):
    import torch
    n = 1 << log2n
    rng = np.random.default_rng(log2n)
    x = (rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))).astype(np.complex64)
    xd = torch.from_numpy(x).cuda()
    for inverse in (False, True):
        y = gpu_lib.dft_c64(xd, inverse=inverse).cpu().numpy()
        ref = np.fft.ifft(x.astype(np.complex128), axis=-1) * n if inverse else np.fft.fft(x.astype(np.complex128), axis=-1)
        rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        assert rel < 3e-7 * log2n, (log2n, inverse, rel)


# ------------------------------------------------------ spectrum, medians
@pytest.mark.parametrize("log2n", [12, 16, 17, 23])
def test_spectrum_and_medians(gpu_lib, log2n):
    import torch
    n = 1 << log2n
    t = synth.make_series(n, seed=100 + log2n, pulsars=[synth.Pulsar(r=n / 11.3, z=7.0, amp=0.2)])
    W = 1024 if n >= 1 << 16 else 256
    bank = gpu_lib.make_templates(10.0, 2.0)
    plan = gpu_lib.Plan(bank, n, 256 if n < 1 << 16 else 2048, median_window=W, nharm_max=1)
    plan.search(_dev(t.x), cap=100000, allow_overflow=True)
    nb = n // 2
    Xg = torch.empty(nb, dtype=torch.complex64, device="cuda")
    medg = torch.empty((nb + W - 1) // W, dtype=torch.float64, device="cuda")
    plan.fetch_spectrum(Xg, medg)
    X = O.real_spectrum(t.x)
    med, _ = O.block_medians(np.abs(X) ** 2, W)
    Xh = O.normalise(X, W)
    mg = medg.cpu().numpy()
    assert np.max(np.abs(mg - med) / med) < 2e-5
    xg = Xg.cpu().numpy().astype(np.complex128)
    # normalised bins have unit mean power; FP32 DFT error is relative to that scale
    err = np.abs(xg - Xh)
    assert np.max(err / np.maximum(np.abs(Xh), 1.0)) < 2e-5
    assert xg[0] == 0
    plan.close()
    bank.close()


# ------------------------------------------------------------ whole plane
@pytest.mark.parametrize("seg", [256, 1024])
def test_plane_parity_small(gpu_lib, seg):
    # 2^16 samples, 21 templates (h = 26): with seg 256 there are 161 segments
    # of 204 valid bins (the last one ragged); with 1024, 35 of 972.
    t = synth.make_series(1 << 16, seed=7, pulsars=[synth.Pulsar(r=9000.4, z=-13.0, amp=0.08, nharm=3)])
    P, cands, n = _run(gpu_lib, t.x, 20.0, 2.0, seg, nharm_max=4, sigma=5.0)
    orc = O.search(t.x, zmax=20.0, dz=2.0, sigma=5.0, nharm_max=4, keep_sums=True)
    worst, rel_max, rel_rms = plane_errors(P, orc.plane)
    assert worst <= REL, (worst, rel_max, rel_rms)
    rep = compare_candidates(cands, orc)
    assert rep["ok"], rep
    assert rep["n_orc"] > 0


def test_single_tone_config(gpu_lib):
    """2^17 samples, one drifting tone, 101 templates, 2048-bin segments, one
    harmonic, 6 sigma: whole plane and candidate list."""
    g = json.load(open(os.path.join(GOLDEN, "single_tone_peak.json")))
    t = synth.single_tone_series()
    P, cands, n = _run(gpu_lib, t.x, 100.0, 2.0, 2048, nharm_max=1, sigma=6.0)
    assert P.shape == (101, 65536)
    orc = O.search(t.x, zmax=100.0, dz=2.0, sigma=6.0, nharm_max=1)
    worst, rel_max, rel_rms = plane_errors(P, orc.plane)
    assert worst <= REL, (worst, rel_max, rel_rms)
    rep = compare_candidates(cands, orc)
    assert rep["ok"], rep
    top = cands[np.argmax(cands["power"])]
    assert top["k"] == g["expected_peak_k"] and top["z"] == g["expected_peak_z"]


def test_harmonic_sum_candidates(gpu_lib):
    # low threshold so that hundreds of noise candidates exercise every level
    t = synth.make_series(1 << 16, seed=8, pulsars=[synth.Pulsar(r=2100.7, z=6.0, amp=0.05, nharm=8)])
    P, cands, n = _run(gpu_lib, t.x, 50.0, 2.0, 1024, nharm_max=16, sigma=4.0)
    orc = O.search(t.x, zmax=50.0, dz=2.0, sigma=4.0, nharm_max=16, keep_sums=True)
    rep = compare_candidates(cands, orc)
    assert rep["ok"], {k: (v if not isinstance(v, list) else v[:10]) for k, v in rep.items()}
    assert all(np.sum(cands["nharm"] == nh) > 5 for nh in (1, 2, 4, 8, 16))


def test_many_candidates_sorted_on_device(gpu_lib):
    # a low threshold gives thousands of candidates at every level: exercises
    # the device radix sort and the FP64 significance against the oracle
    t = synth.make_series(1 << 15, seed=12)
    P, cands, n = _run(gpu_lib, t.x, 10.0, 2.0, 256, nharm_max=16, sigma=2.5, median_window=256)
    orc = O.search(t.x, zmax=10.0, dz=2.0, sigma=2.5, nharm_max=16, W=256, keep_sums=True)
    rep = compare_candidates(cands, orc)
    assert rep["ok"], {k: (v if not isinstance(v, list) else v[:10]) for k, v in rep.items()}
    assert n > 3000
    o = {(c.nharm, c.k, c.iz): c for c in orc.candidates}
    for c in cands[:: max(1, len(cands) // 300)]:
        ref = o.get((int(c["nharm"]), int(c["k"]), int(c["iz"])))
        if ref is None:
            continue
        assert c["r"] == ref.r and c["z"] == pytest.approx(ref.z, abs=1e-12)
        # sigma from the FP32 sum: d sigma ~ dS / sigma
        assert abs(c["sigma"] - ref.sigma) <= 1e-4 * ref.power / max(ref.sigma, 1.0) + 1e-5


@pytest.mark.parametrize("kind", [1, 2])
def test_spectrum_inputs(gpu_lib, kind):
    t = synth.make_series(1 << 15, seed=9, pulsars=[synth.Pulsar(r=3000.2, z=10.0, amp=0.1)])
    X = O.real_spectrum(t.x)
    if kind == 2:
        X = O.normalise(X, 512)
    P, cands, n = _run(gpu_lib, X, 30.0, 2.0, 512, kind=kind, nharm_max=2, sigma=5.0, median_window=512)
    orc = O.search(spectrum=X, normalised=(kind == 2), zmax=30.0, dz=2.0, sigma=5.0, nharm_max=2, W=512,
                   keep_sums=True)
    worst, _, _ = plane_errors(P, orc.plane)
    assert worst <= REL
    assert compare_candidates(cands, orc)["ok"]


# -------------------------------------------------------------- edge cases
def test_zero_series(gpu_lib):
    x = np.zeros(1 << 14, dtype=np.float32)
    P, cands, n = _run(gpu_lib, x, 10.0, 2.0, 256, nharm_max=16)
    assert n == 0 and np.all(P == 0)


def test_candidate_overflow_reports_true_count(gpu_lib):
    import torch
    t = synth.make_series(1 << 14, seed=10)
    bank = gpu_lib.make_templates(10.0, 2.0)
    plan = gpu_lib.Plan(bank, 1 << 14, 256, nharm_max=1, sigma=2.0, median_window=256)
    x = _dev(t.x)
    cands, n = plan.search(x, cap=100000)
    assert n > 10
    with pytest.raises(gpu_lib.FdasError) as e:
        plan.search(x, cap=3)
    assert e.value.status == -4
    c3, n3 = plan.search(x, cap=3, allow_overflow=True)
    assert n3 == n and len(c3) == 3
    assert np.array_equal(c3, cands[:3])
    plan.close()
    bank.close()


def test_hit_list_overflow_is_reported(gpu_lib):
    # a tiny capacity makes the internal list of threshold-passing cells
    # overflow; the search must say so rather than return a silent subset
    t = synth.make_series(1 << 15, seed=13)
    bank = gpu_lib.make_templates(10.0, 2.0)
    plan = gpu_lib.Plan(bank, 1 << 15, 256, nharm_max=4, sigma=2.0, median_window=256, cand_capacity=16)
    with pytest.raises(gpu_lib.FdasError) as e:
        plan.search(_dev(t.x), cap=1000)
    assert e.value.status == -4
    plan.close()
    bank.close()


def test_repeat_is_bit_identical(gpu_lib):
    t = synth.make_series(1 << 16, seed=11)
    a = _run(gpu_lib, t.x, 20.0, 2.0, 512, nharm_max=16, sigma=4.0)
    b = _run(gpu_lib, t.x, 20.0, 2.0, 512, nharm_max=16, sigma=4.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------- batch and server
def test_batch_equals_single(gpu_lib):
    lens = [1 << 15, 1 << 16, 1 << 14, 1 << 16]
    trials = [synth.make_series(n, seed=20 + i, pulsars=[synth.Pulsar(r=n / 7.1, z=4.0, amp=0.1, nharm=2)])
              for i, n in enumerate(lens)]
    bank = gpu_lib.make_templates(20.0, 2.0)
    opts = dict(nharm_max=8, sigma=4.5, median_window=256)
    plan = gpu_lib.Plan(bank, 1 << 16, 512, **opts)
    xs = [_dev(t.x) for t in trials]
    got = plan.search_batch(xs, caps=[20000] * len(xs))
    # the captured graphs are replayed with other inputs in between
    again = plan.search_batch(xs[::-1], caps=[20000] * len(xs))[::-1]
    for a, b in zip(got, again):
        assert np.array_equal(a, b)
    for t, x, g in zip(trials, xs, got):
        single = gpu_lib.Plan(bank, t.nsamp, 512, **opts)
        want, n = single.search(x, cap=20000)
        single.close()
        assert np.array_equal(g, want)
        assert n > 0
    plan.close()
    bank.close()


def test_server_alone_vs_mix(gpu_lib):
    lens = [1 << 16, 1 << 15, 1 << 16, 1 << 14, 1 << 15, 1 << 16, 1 << 16]
    trials = [synth.make_series(n, seed=40 + i, pulsars=[synth.Pulsar(r=n / 9.3, z=-6.0, amp=0.1, nharm=2)])
              for i, n in enumerate(lens)]
    bank = gpu_lib.make_templates(20.0, 2.0)
    opts = dict(nharm_max=8, sigma=4.5, median_window=256)
    alone = []
    for t in trials:
        p = gpu_lib.Plan(bank, t.nsamp, 512, **opts)
        alone.append(p.search(_dev(t.x), cap=20000)[0])
        p.close()
    srv = gpu_lib.Server(bank, 512, 1 << 16, hbm_budget=0, max_slots=3, **opts)
    for i, t in enumerate(trials):
        srv.submit(t.x, tag=1000 + i)
    seen = {}
    for _ in trials:
        tag, c, n, lat = srv.poll(timeout_ms=60000, cap=20000)
        seen[tag] = c
        assert lat > 0
    assert srv.outstanding == 0
    srv.close()
    for i in range(len(trials)):
        assert np.array_equal(seen[1000 + i], alone[i])


def test_autotune_and_cache(gpu_lib, tmp_path):
    bank = gpu_lib.make_templates(50.0, 2.0)  # h = 41: every segment length is valid
    cache = str(tmp_path / "tune.txt")
    seg, tpb, ms = gpu_lib.autotune(bank, 1 << 16, cache_path=cache, nharm_max=4)
    assert seg in (1024, 2048, 4096, 8192) and tpb in (7, 13, 26) and ms > 0
    assert len(open(cache).read().splitlines()) == 1
    assert gpu_lib.autotune(bank, 1 << 16, cache_path=cache, nharm_max=4) == (seg, tpb, ms)
    # the persistent launch form tunes over its own segment lengths, in a line of its own
    seg_p, tpb_p, ms_p = gpu_lib.autotune(bank, 1 << 16, cache_path=cache, nharm_max=4, batch_launch="persistent")
    assert seg_p in (4096, 8192) and tpb_p in (7, 13, 26) and ms_p > 0
    assert len(open(cache).read().splitlines()) == 2
    assert gpu_lib.autotune(bank, 1 << 16, cache_path=cache, nharm_max=4) == (seg, tpb, ms)
    # a plan with the tuned shape gives the same candidates as the default one
    t = synth.make_series(1 << 16, seed=70, pulsars=[synth.Pulsar(r=4000.2, z=9.0, amp=0.1, nharm=2)])
    x = _dev(t.x)
    a = gpu_lib.Plan(bank, 1 << 16, seg, nharm_max=4, templates_per_block=tpb).search(x)[0]
    b = gpu_lib.Plan(bank, 1 << 16, 1024, nharm_max=4).search(x)[0]
    assert np.array_equal(a[["nharm", "k", "iz"]], b[["nharm", "k", "iz"]])
    bank.close()


def test_pinned_output_buffer(gpu_lib):
    # records written into page-locked memory by the device (straight from the
    # finishing kernel, or by the copy kernel after refinement) equal the ones
    # copied into pageable memory; a capacity below the count reports
    # OVERFLOW with the true count and the first records in order
    t = synth.make_series(1 << 15, seed=71)
    bank = gpu_lib.make_templates(10.0, 2.0)
    x = _dev(t.x)
    for levels in (0, 2):
        plan = gpu_lib.Plan(bank, 1 << 15, 256, nharm_max=4, sigma=3.0, median_window=256, refine_levels=levels)
        ref, n = plan.search(x)
        assert n > 8
        out = gpu_lib.pinned_candidates(1 << 16)
        got, n2 = plan.search(x, out=out)
        assert n2 == n and np.array_equal(got, ref)
        small = gpu_lib.pinned_candidates(5)
        with pytest.raises(gpu_lib.FdasError) as e:
            plan.search(x, out=small, cap=5)
        assert e.value.status == -4
        got, n3 = plan.search(x, out=small, cap=5, allow_overflow=True)
        assert n3 == n and np.array_equal(got, ref[:5])
        plan.close()
    bank.close()


def test_server_small_budget_queues(gpu_lib):
    # a budget that holds one 2^16 request at a time still completes everything
    t = [synth.make_series(1 << 16, seed=60 + i) for i in range(3)]
    bank = gpu_lib.make_templates(20.0, 2.0)
    opts = dict(nharm_max=4, sigma=5.0, median_window=256)
    p = gpu_lib.Plan(bank, 1 << 16, 512, **opts)
    one = p.device_bytes  # bank + one series' buffers, candidate buffers included
    p.close()
    srv = gpu_lib.Server(bank, 512, 1 << 16, hbm_budget=int(one * 1.5), max_slots=3, **opts)
    for i, tr in enumerate(t):
        srv.submit(tr.x, tag=i)
    tags = sorted(srv.poll(timeout_ms=60000)[0] for _ in t)
    assert tags == [0, 1, 2]
    srv.close()


# ----------------------------------------------------- full-size SKA shape
def test_ska_trial_sampled(gpu_lib):
    import torch
    tr = synth.ska_trial()
    n = tr.nsamp
    zmax, dz, seg = 200.0, 2.0, 8192
    bank = gpu_lib.make_templates(zmax, dz)
    plan = gpu_lib.Plan(bank, n, seg, nharm_max=16, sigma=6.0)
    plane = torch.empty((bank.nz, n // 2), dtype=torch.float32, device="cuda")
    cands, nf = plan.search(_dev(tr.x), plane=plane)
    torch.cuda.synchronize()
    Xh = O.normalise(O.real_spectrum(tr.x), 1024)
    taps, zs, h = O.template_taps(zmax, dz)
    rng = np.random.default_rng(5)
    iz = rng.integers(0, bank.nz, 3000)
    k = rng.integers(0, n // 2, 3000)
    # plus segment edges and the ragged end of the spectrum
    L = (seg - 2 * h) & ~3  # valid bins per segment (a multiple of 4)
    edge_k = np.concatenate([np.arange(0, 3), L - 1 + np.arange(3), 77 * L + np.arange(-2, 2), n // 2 - 3 + np.arange(3)])
    iz = np.concatenate([iz, rng.integers(0, bank.nz, edge_k.shape[0])])
    k = np.concatenate([k, edge_k])
    Pg = plane[torch.from_numpy(iz).cuda(), torch.from_numpy(k).cuda()].cpu().numpy().astype(np.float64)
    Po = O.correlate_cells(Xh, taps, iz, k)
    assert np.max(np.abs(Pg - Po) / np.maximum(Po, 1.0)) <= REL
    # every GPU candidate is a threshold-passing local maximum of the oracle's sums
    thr = O.thresholds(6.0, [1, 2, 4, 8, 16])
    izc = (bank.nz - 1) // 2
    cell = lambda a, b: O.correlate_cells(Xh, taps, a, b)  # noqa: E731
    assert 0 < nf == len(cands)
    pick = cands if len(cands) <= 150 else cands[rng.choice(len(cands), 150, replace=False)]
    for c in pick:
        nh, kk, ii = int(c["nharm"]), int(c["k"]), int(c["iz"])
        s0 = O.harmonic_sum_cells(cell, [ii], [kk], nh, izc)[0]
        assert abs(c["power"] - s0) <= REL * max(s0, nh)
        tau = lambda x: REL * max(abs(x), nh)  # noqa: E731
        assert s0 >= thr[nh] - 2 * tau(thr[nh])
        for di in (-1, 0, 1):
            for dk in (-1, 0, 1):
                if (di, dk) == (0, 0) or not (0 <= ii + di < bank.nz and 0 <= kk + dk < n // 2):
                    continue
                sn = O.harmonic_sum_cells(cell, [ii + di], [kk + dk], nh, izc)[0]
                earlier = di < 0 or (di == 0 and dk < 0)
                ok = (s0 > sn) if earlier else (s0 >= sn)
                assert ok or abs(s0 - sn) <= 2 * tau(s0)
    # each injected pulsar shows up at its fundamental (one harmonic)
    one = cands[cands["nharm"] == 1]
    for p in tr.pulsars:
        near = one[(np.abs(one["k"] - p.r) <= 2) & (np.abs(one["z"] - p.z) <= 2 * dz)]
        assert len(near) > 0, p
    plan.close()
    bank.close()


def test_segment_length_invariance(gpu_lib):
    """The overlap-save segment length changes only the rounding: S = 2048,
    4096 and 8192 give the same plane (to 1e-4) and the same candidates as the
    oracle's direct sum, and so as each other (2^17 samples, 101 templates,
    16 harmonics)."""
    t = synth.make_series(1 << 17, seed=31, pulsars=[synth.Pulsar(r=12000.2, z=-30.0, amp=0.06, nharm=6)])
    orc = O.search(t.x, zmax=100.0, dz=2.0, sigma=5.5, nharm_max=16, keep_sums=True)
    sets = []
    for seg in (2048, 4096, 8192):
        P, cands, n = _run(gpu_lib, t.x, 100.0, 2.0, seg, nharm_max=16, sigma=5.5)
        worst, _, _ = plane_errors(P, orc.plane)
        assert worst <= REL, (seg, worst)
        rep = compare_candidates(cands, orc)
        assert rep["ok"], (seg, {k: (v if not isinstance(v, list) else v[:10]) for k, v in rep.items()})
        sets.append({(int(c["nharm"]), int(c["k"]), int(c["iz"])) for c in cands})
    assert len(sets[0]) > 10
    # each length matched the oracle up to its borderline cells, so the three
    # sets can differ only there
    o_keys = {(c.nharm, c.k, c.iz) for c in orc.candidates}
    for a in sets[1:]:
        assert len(a ^ sets[0]) <= len(a ^ o_keys) + len(sets[0] ^ o_keys)


@pytest.mark.parametrize("case", range(6))
def test_random_configurations(gpu_lib, case):
    """Seeded random shapes: length, segment, template range and step,
    harmonics, threshold and median window, against the oracle."""
    rng = np.random.default_rng(100 + case)
    log2n = int(rng.integers(12, 17))
    n = 1 << log2n
    dz = float(rng.choice([0.5, 1.0, 2.0]))
    zmax = dz * int(rng.integers(1, 21))
    h = O.halfwidth(zmax)
    segs = [s for s in (256, 512, 1024, 2048, 4096) if s >= 4 * h and s <= n // 2]
    seg = int(rng.choice(segs))
    nharm = int(rng.choice([1, 2, 4, 8, 16]))
    sigma = float(rng.uniform(3.5, 6.0))
    W = int(rng.choice([w for w in (64, 128, 256, 512) if w <= n // 2]))
    p = synth.Pulsar(r=float(rng.uniform(100, n / 2 - 200)), z=float(rng.uniform(-zmax, zmax)),
                     amp=float(rng.uniform(0.05, 0.2)), nharm=int(rng.integers(1, 4)))
    t = synth.make_series(n, seed=200 + case, pulsars=[p])
    P, cands, nf = _run(gpu_lib, t.x, zmax, dz, seg, nharm_max=nharm, sigma=sigma, median_window=W)
    orc = O.search(t.x, zmax=zmax, dz=dz, sigma=sigma, nharm_max=nharm, W=W, keep_sums=True)
    worst, _, _ = plane_errors(P, orc.plane)
    cfg = dict(n=n, seg=seg, zmax=zmax, dz=dz, nharm=nharm, sigma=sigma, W=W)
    assert worst <= REL, (cfg, worst)
    rep = compare_candidates(cands, orc)
    assert rep["ok"], (cfg, {k: (v if not isinstance(v, list) else v[:10]) for k, v in rep.items()})


def test_device_memory_exhaustion_is_nomem(gpu_lib):
    """A plan whose buffers cannot fit in device memory fails with NOMEM (and
    leaves nothing allocated), rather than faulting later."""
    bank = gpu_lib.make_templates(1200.0, 0.5)  # 4801 templates
    with pytest.raises(gpu_lib.FdasError) as e:
        gpu_lib.Plan(bank, 1 << 26, 8192)  # plane alone: 4801 x 2^25 x 4 B = 644 GB
    assert e.value.status == -2
    bank.close()
    # the failed allocation leaves no error behind for the next plan's launches
    t = synth.make_series(1 << 14, seed=3)
    bank = gpu_lib.make_templates(10.0, 2.0)
    plan = gpu_lib.Plan(bank, 1 << 14, 256, nharm_max=1)
    cands, n = plan.search(_dev(t.x))
    assert n == len(cands)
    plan.close()
    bank.close()
