"""Candidate refinement and Fourier interpolation on the GPU (FP64 on the
FP32 spectrum of the search) against the FP64 oracle, through the C ABI.

The interpolated powers are compared point by point; the refined candidates
are compared with every end point the oracle's search can reach when values
within the tolerance of a level's best count as ties (the GPU reads an FP32
spectrum, so near-equal neighbours may be ordered either way).  The
tolerance is the plane's, 1e-4 max(S, nharm).
"""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

REL = 1e-4


def _tol(s, nh):
    return REL * max(abs(s), nh)


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _plan_search(fdas, x, zmax, dz, seg, kind=0, **opts):
    bank = fdas.make_templates(zmax, dz)
    nsamp = x.shape[0] if kind == 0 else 2 * x.shape[0]
    plan = fdas.Plan(bank, nsamp, seg, **opts)
    inp = _dev(x.astype(np.float32) if kind == 0 else x.astype(np.complex64))
    cands, n = plan.search(inp, kind=kind, cap=1 << 20)
    return bank, plan, cands, inp


def _check_refined(cands, Xh, zmax, dz, h, levels, limit=None):
    """Each refined record ends on a point the oracle's search can reach, with
    the oracle's S there; returns the number of records checked."""
    order = np.argsort(-cands["power"], kind="stable")
    if limit is not None:
        order = order[:limit]
    for i in order:
        c = cands[i]
        nh = int(c["nharm"])
        ends = O.refine_endpoints(Xh, int(c["k"]), int(c["iz"]), nh, zmax=zmax, dz=dz, h=h, levels=levels,
                                  tol=lambda s: 2.0 * _tol(s, nh))
        key = (float(c["r"]), float(c["z"]))
        assert key in ends, (c, sorted(ends))
        S = ends[key]
        assert abs(float(c["power"]) - S) <= _tol(S, nh) + 1e-7 * abs(S), (c, S)
        assert float(c["sigma"]) == pytest.approx(O.sigma_of(float(c["power"]), nh), rel=1e-5, abs=1e-5)
    return len(order)


def test_interp_power_matches_oracle(gpu_lib):
    # 2^15 samples, a drifting pulsar with 4 harmonics; points on and off the
    # grid, near both spectrum ends, at the drift limits, for 1..16 harmonics.
    t = synth.make_series(1 << 15, seed=41, pulsars=[synth.Pulsar(r=1234.37, z=-11.3, amp=0.08, nharm=4)])
    zmax, dz, W = 30.0, 2.0, 512
    bank, plan, cands, _ = _plan_search(gpu_lib, t.x, zmax, dz, 512, nharm_max=4, median_window=W, sigma=5.0)
    Xh = O.normalise(O.real_spectrum(t.x), W)
    h = bank.h
    nb = Xh.shape[0]
    rng = np.random.default_rng(7)
    r = np.concatenate([rng.uniform(0.0, nb - 1.0, 40), [0.0, 0.25, nb - 1.0, nb - 0.5, 1234.37, 1234.0, 617.185],
                        np.arange(5, dtype=np.float64) + 2468.74])
    z = np.concatenate([rng.uniform(-zmax, zmax, 40), [0.0, zmax, -zmax, 3.7, -11.3, -12.0, -5.65],
                        np.full(5, -22.6)])
    nh = np.concatenate([rng.choice([1, 2, 4, 8, 16], 40), [1, 1, 1, 2, 1, 1, 2], [1, 2, 4, 8, 16]]).astype(np.int32)
    got = plan.interp_power(r, z, nh)
    for i in range(r.size):
        want = O.interp_sum(Xh, float(r[i]), float(z[i]), int(nh[i]), h)
        assert abs(got[i] - want) <= _tol(want, nh[i]), (i, r[i], z[i], nh[i], got[i], want)
    bad = plan.interp_power(np.array([5.0, 6.0]), np.array([0.0, 0.0]), np.array([0, 17], dtype=np.int32))
    assert np.all(np.isnan(bad))
    plan.close()
    bank.close()


@pytest.mark.parametrize("levels", [1, 6])
def test_refined_candidates_match_oracle(gpu_lib, levels):
    # Two pulsars (one with 8 harmonics) in noise; harmonic sums to 8.  The
    # detection itself (k, iz, nharm) does not change with refinement.
    t = synth.make_series(1 << 15, seed=43, pulsars=[
        synth.Pulsar(r=2100.55, z=13.7, amp=0.09, nharm=8), synth.Pulsar(r=5003.2, z=-4.4, amp=0.12, nharm=1)])
    zmax, dz, W = 40.0, 2.0, 512
    opts = dict(nharm_max=8, median_window=W, sigma=6.0)
    bank, plan, plain, _ = _plan_search(gpu_lib, t.x, zmax, dz, 512, **opts)
    plan.close()
    bank.close()
    bank, plan, cands, _ = _plan_search(gpu_lib, t.x, zmax, dz, 512, refine_levels=levels, **opts)
    for f in ("k", "iz", "nharm"):
        assert np.array_equal(plain[f], cands[f])
    assert len(cands) > 10
    Xh = O.normalise(O.real_spectrum(t.x), W)
    # refined powers never fall below the cell's own harmonic sum at the start
    izc = int(round(zmax / dz))
    start = plan.interp_power(cands["k"] / cands["nharm"],
                              ((cands["iz"] - izc) * dz) / cands["nharm"], cands["nharm"])
    assert np.all(cands["power"] >= start.astype(np.float32) * (1 - 1e-6))
    assert _check_refined(cands, Xh, zmax, dz, bank.h, levels, limit=30) > 10
    plan.close()
    bank.close()


def test_refine_on_normalised_spectrum_and_matrix_correlator(gpu_lib):
    # The refinement reads the spectrum the search read: the caller's
    # normalised spectrum (no medians), or the series' spectrum whatever the
    # correlator (it always works in FP64).
    t = synth.make_series(1 << 14, seed=44, pulsars=[synth.Pulsar(r=3001.7, z=6.1, amp=0.15, nharm=2)])
    zmax, dz, W = 20.0, 1.0, 256
    Xh = O.normalise(O.real_spectrum(t.x), W)
    opts = dict(nharm_max=2, median_window=W, sigma=6.0, refine_levels=5)
    bank, plan, cands, _ = _plan_search(gpu_lib, Xh, zmax, dz, 256, kind=2, **opts)
    assert len(cands) > 0
    _check_refined(cands, Xh, zmax, dz, bank.h, 5)
    plan.close()
    bank.close()
    bank, plan, cands, _ = _plan_search(gpu_lib, t.x, zmax, dz, 256, correlator="bf16", **opts)
    assert len(cands) > 0
    _check_refined(cands, Xh, zmax, dz, bank.h, 5, limit=10)
    plan.close()
    bank.close()


def test_refine_finds_noiseless_tone(gpu_lib):
    # Normalised-spectrum input holding the DFT of a noiseless drifting tone
    # (scaled by 2 / N plus a unit-power floor so that nothing is below the
    # float range): the refined fundamental lies within the search's
    # resolution of the true (r, z).
    N, rbar, zbar = 1 << 14, 2000.3, 7.4
    u = np.arange(N) / N
    x = np.cos(0.3 + 2 * np.pi * ((rbar - zbar / 2) * u + zbar * u * u / 2))
    X = O.real_spectrum(x) / (N / 2) * 20.0
    rng = np.random.default_rng(9)
    X = X + (rng.standard_normal(X.size) + 1j * rng.standard_normal(X.size)) * 1e-3
    zmax, dz, levels = 20.0, 2.0, 8
    bank, plan, cands, _ = _plan_search(gpu_lib, X, zmax, dz, 256, kind=2, nharm_max=1, sigma=8.0,
                                        refine_levels=levels)
    best = cands[np.argmax(cands["power"])]
    assert abs(best["r"] - rbar) <= 2.0 ** -levels
    assert abs(best["z"] - zbar) <= 2.0 * dz * 2.0 ** -levels
    plan.close()
    bank.close()


def test_refine_in_batch_equals_single(gpu_lib):
    trials = [synth.make_series(1 << 14, seed=50 + i, pulsars=[synth.Pulsar(r=1500.4 + 300 * i, z=3.3, amp=0.15)])
              for i in range(3)]
    bank = gpu_lib.make_templates(10.0, 2.0)
    plan = gpu_lib.Plan(bank, 1 << 14, 256, nharm_max=4, sigma=5.0, median_window=256, refine_levels=4)
    xs = [_dev(t.x) for t in trials]
    alone = [plan.search(x, cap=20000)[0] for x in xs]
    batch = plan.search_batch(xs, caps=[20000] * len(xs))
    for a, b in zip(alone, batch):
        assert np.array_equal(a, b)
    assert all(len(a) > 0 for a in alone)
    plan.close()
    bank.close()


def test_refine_stage_is_timed(gpu_lib):
    t = synth.make_series(1 << 14, seed=45, pulsars=[synth.Pulsar(r=900.2, z=2.0, amp=0.2)])
    bank = gpu_lib.make_templates(10.0, 2.0)
    plan = gpu_lib.Plan(bank, 1 << 14, 256, nharm_max=1, median_window=256, refine_levels=3)
    plan.enable_timing(True)
    plan.search(_dev(t.x))
    st, n = plan.stage_times()
    assert n == 1 and st["refine"] > 0.0
    plan.close()
    bank.close()


def test_refine_levels_validation(gpu_lib):
    bank = gpu_lib.make_templates(10.0, 2.0)
    with pytest.raises(gpu_lib.FdasError):
        gpu_lib.Plan(bank, 1 << 14, 256, refine_levels=21)
    with pytest.raises(gpu_lib.FdasError):
        gpu_lib.Plan(bank, 1 << 14, 256, refine_levels=-1)
    bank.close()


def test_refine_chosen_records(gpu_lib):
    # fdas_refine on the most significant records of a plain search equals the
    # refinement inside the search for those records, and matches the oracle.
    t = synth.make_series(1 << 15, seed=46, pulsars=[synth.Pulsar(r=4100.8, z=-17.9, amp=0.1, nharm=4)])
    zmax, dz, W = 30.0, 2.0, 512
    opts = dict(nharm_max=4, median_window=W, sigma=5.5)
    bank, plan, plain, x = _plan_search(gpu_lib, t.x, zmax, dz, 512, **opts)
    top = plain[np.argsort(-plain["sigma"], kind="stable")[:12]]
    got = plan.refine(top, levels=6)
    for f in ("k", "iz", "nharm"):
        assert np.array_equal(got[f], top[f])
    Xh = O.normalise(O.real_spectrum(t.x), W)
    assert _check_refined(got, Xh, zmax, dz, bank.h, 6) == len(top)
    assert len(plan.refine(top[:0])) == 0
    bad = top[:1].copy()
    bad["nharm"] = 3
    with pytest.raises(gpu_lib.FdasError):
        plan.refine(bad)
    with pytest.raises(gpu_lib.FdasError):
        plan.refine(top, levels=0)
    plan.close()
    bank.close()
    bank, plan, full, _ = _plan_search(gpu_lib, t.x, zmax, dz, 512, refine_levels=6, **opts)
    idx = {(int(c["k"]), int(c["iz"]), int(c["nharm"])): c for c in full}
    for c in got:
        assert c.tobytes() == idx[(int(c["k"]), int(c["iz"]), int(c["nharm"]))].tobytes()
    plan.close()
    bank.close()


def test_refine_needs_a_search(gpu_lib):
    bank = gpu_lib.make_templates(10.0, 2.0)
    plan = gpu_lib.Plan(bank, 1 << 14, 256)
    rec = np.zeros(1, dtype=gpu_lib.CAND_DTYPE)
    rec["nharm"] = 1
    with pytest.raises(gpu_lib.FdasError):
        plan.refine(rec)
    with pytest.raises(gpu_lib.FdasError):
        plan.interp_power(np.array([1.0]), np.array([0.0]), 1)
    plan.close()
    bank.close()


def test_response_accuracy_two_bins(gpu_lib):
    # A normalised spectrum with two exactly representable non-zero bins
    # isolates the FP64 response evaluation (Fresnel series, continued
    # fraction, drift-sign and phase handling):
    #   P(r, z) = |conj A(r - k0, z) + (i / 2) conj A(r - k0 - 3, z)|^2 / D.
    nb, k0 = 4096, 2000
    X = np.zeros(nb, dtype=np.complex128)
    X[k0] = 1.0
    X[k0 + 3] = 0.5j
    zmax, dz = 200.0, 4.0
    bank, plan, _, x = _plan_search(gpu_lib, X, zmax, dz, 512, kind=2, nharm_max=1, sigma=30.0)
    h = bank.h
    rng = np.random.default_rng(12)
    dr = np.concatenate([[0.0, 0.5, -0.25, 3.0, 1.7, -40.3, 60.9, 116.0, -116.5],
                         rng.uniform(-120.0, 120.0, 40)])
    zz = np.concatenate([[0.0, 0.0, 0.3, -0.3, 7.7, -150.2, 150.2, 199.9, -2.0],
                         rng.uniform(-zmax, zmax, 40)])
    got = plan.interp_power(k0 + dr, zz, 1)
    for i in range(dr.size):
        want = O.interp_power(X, k0 + float(dr[i]), float(zz[i]), h)
        # the oracle reduces the phase pi p^2 / z (p = q - z/2) modulo 2 pi in
        # FP64: up to 2^-52 pi p^2 / z of error, 2e-10 at p = 120, z = 0.05
        assert abs(got[i] - want) <= 1e-9 * want + 1e-13, (dr[i], zz[i], got[i], want)
    plan.close()
    bank.close()
