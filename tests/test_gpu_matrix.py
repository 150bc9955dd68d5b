"""The matrix-core correlators (Eq. (1) of Sec. 2 as a BF16 / FP16 matrix
product with FP32 accumulation) against the FP64 oracle.

A 1e-4 tolerance does not apply: the operands are rounded to 16 bits.  The
test derives the bound from that rounding instead.  With x = Xhat[k - q],
t = T_z[q], unit roundoff u of the format and B_k = sum_q |x| |t|, the
correlation Y_z[k] = sum_q x t is off by at most
    E = (2u + u^2 + 1e-4) B_k + s_k,
where 1e-4 covers the FP32 accumulation and the FP32 spectrum the GPU
normalises, and s_k the absolute rounding of subnormal operands.  The power
is then off by at most 2 sqrt(P) E + E^2.  Candidates may differ only where
the oracle's value lies within that bound of the threshold or of a
neighbour's.
"""
import numpy as np
import pytest

import oracle as O
import synth
from parity import compare_candidates

pytestmark = pytest.mark.gpu

# unit roundoff, and the smallest normal (subnormal operands are rounded to an
# absolute spacing of 2^-24 times it)
FORMATS = {"bf16": (2.0 ** -8, 2.0 ** -126), "f16": (2.0 ** -11, 2.0 ** -14)}
TAP_SCALE = 16.0  # the library scales taps by 16 before rounding (exactly undone)


def _bound(x, zmax, dz, W, fmt):
    """Per-cell bound of |P_gemm - P_oracle| (nz x nb) and the oracle plane."""
    u, tiny = FORMATS[fmt]
    Xh = O.normalise(O.real_spectrum(x), W)
    taps, zs, h = O.template_taps(zmax, dz)
    nb = Xh.shape[0]
    ax = np.abs(Xh)
    ones = np.ones(2 * h + 1)
    sub_x = 2.0 ** -24 * tiny  # absolute rounding of a subnormal spectrum value
    sub_t = 2.0 ** -24 * tiny / TAP_SCALE
    sum_x = np.convolve(ax, ones)[h:h + nb]
    E = np.empty((taps.shape[0], nb))
    for iz in range(taps.shape[0]):
        at = np.abs(taps[iz])
        B = np.convolve(ax, at)[h:h + nb]
        E[iz] = (2 * u + u * u + 1e-4) * B + sub_t * sum_x + sub_x * at.sum()
    return E


def _run(fdas, x, zmax, dz, W, corr, **opts):
    import torch
    bank = fdas.make_templates(zmax, dz)
    plan = fdas.Plan(bank, x.shape[0], 256, correlator=corr, median_window=W, **opts)
    plane = torch.empty((bank.nz, x.shape[0] // 2), dtype=torch.float32, device="cuda")
    cands, n = plan.search(torch.from_numpy(x.astype(np.float32)).cuda(), plane=plane)
    torch.cuda.synchronize()
    P = plane.cpu().numpy()
    plan.close()
    bank.close()
    return P, cands, n


@pytest.mark.parametrize("corr", ["bf16", "f16"])
def test_matrix_correlator_within_rounding_bound(gpu_lib, corr):
    # 2^15 samples, 21 templates (h = 26, K = 106 padded to 128): 32 row
    # blocks of 512 bins over one slice of 32 templates (11 of them padding)
    t = synth.make_series(1 << 15, seed=21, pulsars=[synth.Pulsar(r=3000.3, z=7.0, amp=0.1, nharm=2)])
    zmax, dz, W = 20.0, 2.0, 256
    P, cands, n = _run(gpu_lib, t.x, zmax, dz, W, corr, nharm_max=1, sigma=4.0)
    orc = O.search(t.x, zmax=zmax, dz=dz, sigma=4.0, nharm_max=1, W=W)
    E = _bound(t.x, zmax, dz, W, corr)
    dP = 2.0 * np.sqrt(orc.plane) * E + E * E
    err = np.abs(P.astype(np.float64) - orc.plane)
    assert np.all(err <= dP), float((err / dP).max())
    # the error is of the order of the rounding, not far below it (the
    # 16-bit path really ran)
    big = orc.plane >= 1.0
    rel = err[big] / orc.plane[big]
    u = FORMATS[corr][0]
    assert 0.02 * u < np.sqrt(np.mean(rel ** 2)) < 4 * u
    rep = compare_candidates(cands, orc, tol={1: dP})
    assert rep["ok"], {k: (v if not isinstance(v, list) else v[:10]) for k, v in rep.items()}
    assert rep["n_orc"] > 20


@pytest.mark.parametrize("corr", ["bf16", "f16"])
def test_matrix_correlator_harmonic_sums(gpu_lib, corr):
    # several slices (nz = 81 -> 3 slices of 32) and ragged template padding;
    # harmonic sums to 8: per-level bounds are sums of the cells' bounds
    t = synth.make_series(1 << 15, seed=22, pulsars=[synth.Pulsar(r=1500.6, z=-9.0, amp=0.07, nharm=6)])
    zmax, dz, W = 40.0, 1.0, 512
    P, cands, n = _run(gpu_lib, t.x, zmax, dz, W, corr, nharm_max=8, sigma=5.0)
    orc = O.search(t.x, zmax=zmax, dz=dz, sigma=5.0, nharm_max=8, W=W, keep_sums=True)
    E = _bound(t.x, zmax, dz, W, corr)
    dP = 2.0 * np.sqrt(orc.plane) * E + E * E
    assert np.all(np.abs(P.astype(np.float64) - orc.plane) <= dP)
    izc = (orc.plane.shape[0] - 1) // 2
    tol = {1: dP}
    for nh in (2, 4, 8):
        # FP32 summation of nh terms adds at most nh * 2^-24 of the sum
        tol[nh] = O.harmonic_sum(dP, nh, izc) + nh * 2.0 ** -24 * orc.sums[nh]
    rep = compare_candidates(cands, orc, tol=tol)
    assert rep["ok"], {k: (v if not isinstance(v, list) else v[:10]) for k, v in rep.items()}
    assert rep["n_orc"] > 5


def test_matrix_correlator_batch_equals_single(gpu_lib):
    import torch
    trials = [synth.make_series(1 << 14, seed=30 + i) for i in range(3)]
    bank = gpu_lib.make_templates(10.0, 2.0)
    opts = dict(nharm_max=4, sigma=4.0, median_window=256, correlator="bf16")
    plan = gpu_lib.Plan(bank, 1 << 14, 256, **opts)
    xs = [torch.from_numpy(t.x).cuda() for t in trials]
    alone = [plan.search(x, cap=20000)[0] for x in xs]
    batch = plan.search_batch(xs, caps=[20000] * len(xs))
    for a, b in zip(alone, batch):
        assert np.array_equal(a, b)
    assert sum(len(a) for a in alone) > 0
    plan.close()
    bank.close()
