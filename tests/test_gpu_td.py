"""Time-domain resampling search (fdas_td_plan) on the GPU against the FP64
oracle, through the C ABI: the plane of per-trial powers element by element
(1e-4 rule), the candidates (indices exact except at borderline cells), and
the options and entry points such a plan refuses."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import compare_candidates, plane_errors

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("n,nalpha,alpha_max,nharm,W", [
    (1 << 13, 11, 0.02, 4, 256),
    (1 << 14, 21, 0.01, 8, 512),
    (1 << 15, 1, 0.0, 2, 1024),
])
def test_td_plane_and_candidates_match_oracle(gpu_lib, n, nalpha, alpha_max, nharm, W):
    import torch
    rbar = n / 13.1 + 0.3
    z = 0.6 * alpha_max * rbar  # drift between two trials
    t = synth.make_series(n, seed=80 + nharm, pulsars=[synth.Pulsar(r=rbar, z=z, amp=0.15, nharm=4),
                                                        synth.Pulsar(r=n / 5.7, z=0.0, amp=0.1, nharm=1)])
    plan = gpu_lib.TdPlan(n, alpha_max, nalpha, nharm_max=nharm, median_window=W, sigma=5.0)
    plane = torch.empty((nalpha, n // 2), dtype=torch.float32, device="cuda")
    cands, nfound = plan.search(_dev(t.x), plane=plane, cap=1 << 20)
    torch.cuda.synchronize()
    P = plane.cpu().numpy()
    orc = O.td_search(t.x, alpha_max=alpha_max, nalpha=nalpha, sigma=5.0, nharm_max=nharm, W=W, keep_sums=True)
    assert np.allclose(plan.alphas, O.td_alphas(alpha_max, nalpha), rtol=0, atol=0)
    scaled, rel_max, rel_rms = plane_errors(P, orc.plane)
    assert scaled <= 1e-4, (scaled, rel_max, rel_rms)
    rep = compare_candidates(cands, orc)
    assert rep["ok"], {k: (v if not isinstance(v, list) else v[:10]) for k, v in rep.items()}
    assert rep["n_orc"] > 3
    alphas = O.td_alphas(alpha_max, nalpha)
    for c in cands:
        assert c["r"] == c["k"] / c["nharm"]
        assert c["z"] == alphas[c["iz"]] * c["r"]
    plan.close()


def test_td_finds_accelerated_pulsar(gpu_lib):
    n, nalpha, alpha_max = 1 << 15, 41, 0.02
    rbar = 2000.3
    z = 0.012 * rbar  # alpha = 0.012: trial 32
    t = synth.make_series(n, seed=85, pulsars=[synth.Pulsar(r=rbar, z=z, amp=0.08, nharm=4)])
    plan = gpu_lib.TdPlan(n, alpha_max, nalpha, nharm_max=4, median_window=512, sigma=6.0)
    cands, _ = plan.search(_dev(t.x))
    best = cands[cands["nharm"] == 4][np.argmax(cands[cands["nharm"] == 4]["power"])]
    assert int(best["iz"]) == int(np.argmin(np.abs(plan.alphas - z / rbar)))
    assert abs(best["r"] - rbar) <= 0.25
    assert abs(best["z"] - z) <= 0.6
    plan.enable_timing(True)
    plan.search(_dev(t.x))
    st, nt = plan.stage_times()
    assert nt == 1 and st["r2c"] > 0 and st["harmonic_sum"] > 0
    plan.close()


def test_td_plan_refuses(gpu_lib):
    with pytest.raises(gpu_lib.FdasError):
        gpu_lib.TdPlan(1 << 14, 0.6, 11)
    with pytest.raises(gpu_lib.FdasError):
        gpu_lib.TdPlan(1 << 14, 0.01, 0)
    with pytest.raises(gpu_lib.FdasError):
        gpu_lib.TdPlan(1 << 14, 0.01, 11, interbin=True)
    with pytest.raises(gpu_lib.FdasError):
        gpu_lib.TdPlan(1 << 14, 0.01, 11, refine_levels=3)
    plan = gpu_lib.TdPlan(1 << 14, 0.01, 11, nharm_max=2)
    x = _dev(synth.make_series(1 << 14, seed=2).x)
    plan.search(x)
    rec = np.zeros(1, dtype=gpu_lib.CAND_DTYPE)
    rec["nharm"] = 1
    with pytest.raises(gpu_lib.FdasError):
        plan.refine(rec)
    with pytest.raises(gpu_lib.FdasError):
        plan.interp_power(np.array([10.0]), np.array([0.0]), 1)
    with pytest.raises(gpu_lib.FdasError):
        plan.search_batch([x], caps=[100])
    import torch
    with pytest.raises(gpu_lib.FdasError):
        plan.search(torch.zeros(1 << 13, dtype=torch.complex64, device="cuda"), kind=1)
    plan.close()
