"""Half-bin plane (fdas_opts.interbin) on the GPU against the FP64 oracle,
through the C ABI: the plane element by element (1e-4 rule; the library
stores row iz as the Nb bins then the Nb half-bin points, the oracle's
plane interleaves them),
the candidates (indices exact except at borderline cells), batches equal to
single searches, and refinement starting from half-bin cells."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import compare_candidates, plane_errors

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _split(P2):
    """Library layout of an interleaved half-bin plane: bins, then half-bin points."""
    return np.concatenate([P2[:, 0::2], P2[:, 1::2]], axis=1)


def _run(fdas, x, zmax, dz, seg, kind=0, **opts):
    import torch
    bank = fdas.make_templates(zmax, dz)
    nsamp = x.shape[0] if kind == 0 else 2 * x.shape[0]
    plan = fdas.Plan(bank, nsamp, seg, interbin=True, **opts)
    assert plan.plane_columns == nsamp
    plane = torch.empty((bank.nz, nsamp), dtype=torch.float32, device="cuda")
    inp = _dev(x.astype(np.float32) if kind == 0 else x.astype(np.complex64))
    cands, n = plan.search(inp, kind=kind, plane=plane, cap=1 << 20)
    torch.cuda.synchronize()
    return bank, plan, plane.cpu().numpy(), cands, n


@pytest.mark.parametrize("n,seg,zmax,dz,nharm,W", [
    (1 << 14, 256, 20.0, 2.0, 4, 256),     # h = 26: 204-bin segments, ragged last one
    (1 << 15, 512, 30.0, 1.0, 8, 512),
    (1 << 16, 2048, 60.0, 4.0, 16, 1024),
])
def test_half_bin_plane_matches_oracle(gpu_lib, n, seg, zmax, dz, nharm, W):
    t = synth.make_series(n, seed=60 + nharm, pulsars=[
        synth.Pulsar(r=n / 9.7 + 0.5, z=zmax / 3.1, amp=0.1, nharm=4),
        synth.Pulsar(r=n / 5.3 + 0.25, z=-zmax / 2.3, amp=0.15, nharm=1)])
    bank, plan, P, cands, nfound = _run(gpu_lib, t.x, zmax, dz, seg, nharm_max=nharm, median_window=W, sigma=5.0)
    orc = O.search(t.x, zmax=zmax, dz=dz, sigma=5.0, nharm_max=nharm, W=W, keep_sums=True, interbin=True)
    assert P.shape == orc.plane.shape
    scaled, rel_max, rel_rms = plane_errors(P, _split(orc.plane))
    assert scaled <= 1e-4, (scaled, rel_max, rel_rms)
    rep = compare_candidates(cands, orc)
    assert rep["ok"], {k: (v if not isinstance(v, list) else v[:10]) for k, v in rep.items()}
    assert rep["n_orc"] > 5
    for c in cands:
        assert c["r"] == c["k"] / (2.0 * c["nharm"])
    plan.close()
    bank.close()


def test_half_bin_plane_finds_tone_between_bins(gpu_lib):
    # normalised-spectrum input: a strong noiseless tone at 700.5 bins drifting
    # by a bank z; the strongest record is the half-bin cell itself
    N, rbar, zbar, a = 1 << 13, 700.5, 4.0, 10.0
    u = np.arange(N) / N
    x = a * np.cos(0.4 + 2 * np.pi * ((rbar - zbar / 2) * u + zbar * u * u / 2))
    X = O.real_spectrum(x) / (N / 2)
    zmax, dz = 10.0, 2.0
    bank, plan, P, cands, n = _run(gpu_lib, X, zmax, dz, 256, kind=2, nharm_max=1, sigma=6.0)
    iz = int(round((zbar + zmax) / dz))
    best = cands[np.argmax(cands["power"])]
    assert (int(best["k"]), int(best["iz"]), float(best["r"]), float(best["z"])) == (1401, iz, 700.5, zbar)
    assert P[iz, 700] / P[iz, (N // 2) + 700] == pytest.approx(np.sinc(0.5) ** 2, rel=3e-2)
    plan.close()
    bank.close()


def test_half_bin_batch_equals_single(gpu_lib):
    trials = [synth.make_series(1 << 14, seed=70 + i, pulsars=[synth.Pulsar(r=1200.5 + 333 * i, z=2.7, amp=0.15)])
              for i in range(3)]
    bank = gpu_lib.make_templates(10.0, 2.0)
    plan = gpu_lib.Plan(bank, 1 << 14, 256, nharm_max=4, sigma=5.0, median_window=256, interbin=True)
    xs = [_dev(t.x) for t in trials]
    alone = [plan.search(x, cap=20000)[0] for x in xs]
    batch = plan.search_batch(xs, caps=[20000] * len(xs))
    for a, b in zip(alone, batch):
        assert np.array_equal(a, b)
    assert all(len(a) > 0 for a in alone)
    plan.close()
    bank.close()


def test_half_bin_refinement_matches_oracle(gpu_lib):
    t = synth.make_series(1 << 14, seed=75, pulsars=[synth.Pulsar(r=2500.6, z=-7.3, amp=0.12, nharm=2)])
    zmax, dz, W = 20.0, 2.0, 256
    bank, plan, P, cands, n = _run(gpu_lib, t.x, zmax, dz, 256, nharm_max=2, median_window=W, sigma=6.0,
                                   refine_levels=5)
    Xh = O.normalise(O.real_spectrum(t.x), W)
    assert len(cands) > 0
    for c in cands[np.argsort(-cands["power"], kind="stable")[:8]]:
        nh = int(c["nharm"])
        ends = O.refine_endpoints(Xh, int(c["k"]), int(c["iz"]), nh, zmax=zmax, dz=dz, h=bank.h, levels=5,
                                  tol=lambda s: 2e-4 * max(s, nh), cpb=2)
        key = (float(c["r"]), float(c["z"]))
        assert key in ends, (c, sorted(ends))
        assert abs(float(c["power"]) - ends[key]) <= 1e-4 * max(ends[key], nh) + 1e-7 * ends[key]
    plan.close()
    bank.close()


def test_half_bin_options_and_plane_size(gpu_lib):
    import torch
    bank = gpu_lib.make_templates(10.0, 2.0)
    with pytest.raises(gpu_lib.FdasError):
        gpu_lib.Plan(bank, 1 << 14, 256, interbin=True, correlator="bf16")
    plan = gpu_lib.Plan(bank, 1 << 14, 256, interbin=True, nharm_max=1)
    small = torch.empty((bank.nz, 1 << 13), dtype=torch.float32, device="cuda")  # Nb columns, not 2 Nb
    with pytest.raises(ValueError):
        plan.search(_dev(synth.make_series(1 << 14, seed=1).x), plane=small)
    plan.close()
    bank.close()


def test_server_with_half_bins_and_refinement(gpu_lib):
    # the served path carries the plan options: each result equals the search
    # of the same series alone with the half-bin plane and refinement on
    lens = [1 << 15, 1 << 14, 1 << 15, 1 << 15]
    trials = [synth.make_series(n, seed=90 + i, pulsars=[synth.Pulsar(r=n / 7.1 + 0.5, z=3.1, amp=0.12, nharm=2)])
              for i, n in enumerate(lens)]
    bank = gpu_lib.make_templates(10.0, 2.0)
    opts = dict(nharm_max=4, sigma=5.5, median_window=256, interbin=True, refine_levels=3)
    alone = []
    for t in trials:
        p = gpu_lib.Plan(bank, t.nsamp, 256, **opts)
        alone.append(p.search(_dev(t.x), cap=20000)[0])
        p.close()
    srv = gpu_lib.Server(bank, 256, 1 << 15, hbm_budget=0, max_slots=2, **opts)
    for i, t in enumerate(trials):
        srv.submit(t.x, tag=500 + i)
    seen = {}
    for _ in trials:
        tag, c, n, lat = srv.poll(timeout_ms=60000, cap=20000)
        seen[tag] = c
    srv.close()
    for i in range(len(trials)):
        assert np.array_equal(seen[500 + i], alone[i])
    assert sum(len(a) for a in alone) > 0
    bank.close()
