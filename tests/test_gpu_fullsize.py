"""Sampled parity at full size for the shapes the measurements run besides
the SKA trial: the precision-variant trials (2^22 samples, 801 templates
z in [-400, 400] step 1, h = 216, 8192-bin segments, one harmonic) through
the FP32 FFT correlator and the BF16 / FP16 matrix correlators, and the two
shorter lengths of the served mix (2^21 and 2^22 samples, 201 templates).

The plane is checked on sampled cells (random, segment edges and the ragged
end of the spectrum), each against the FP64 oracle's direct correlation
(Eq. (1) of Sec. 2) at that cell: the 1e-4 rule for the FFT path, the
16-bit rounding bound of the matrix correlators otherwise (the bound is the
one derived in test_gpu_matrix.py, taken per cell).  Sampled candidates must
be threshold-passing 3x3 local maxima of the oracle's powers within that
tolerance."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import REL

pytestmark = pytest.mark.gpu

FORMATS = {"bf16": (2.0 ** -8, 2.0 ** -126), "f16": (2.0 ** -11, 2.0 ** -14)}
TAP_SCALE = 16.0


def _cells(rng, nz, nb, L, nrand):
    iz = rng.integers(0, nz, nrand)
    k = rng.integers(0, nb, nrand)
    edge_k = np.concatenate([np.arange(0, 3), L - 2 + np.arange(4), 41 * L + np.arange(-2, 2),
                             (nb // L) * L + np.arange(-1, 2), nb - 3 + np.arange(3)])
    edge_k = edge_k[(edge_k >= 0) & (edge_k < nb)]
    iz = np.concatenate([iz, rng.integers(0, nz, edge_k.shape[0]), np.zeros(3, int), np.full(3, nz - 1)])
    k = np.concatenate([k, edge_k, rng.integers(0, nb, 6)])
    return iz, k


def _bound_cells(Xh, taps, iz, k, fmt):
    """Per-cell bound of |P_gpu - P_oracle| for a 16-bit matrix correlator."""
    u, tiny = FORMATS[fmt]
    h = (taps.shape[1] - 1) // 2
    ax = np.abs(np.pad(Xh, h))
    win = ax[k[:, None] + 2 * h - np.arange(2 * h + 1)[None, :]]  # |Xh[k - q]|, q = -h..h
    at = np.abs(taps[iz])
    B = np.sum(win * at, axis=1)
    E = (2 * u + u * u + 1e-4) * B + 2.0 ** -24 * tiny / TAP_SCALE * win.sum(axis=1) \
        + 2.0 ** -24 * tiny * at.sum(axis=1)
    P = O.correlate_cells(Xh, taps, iz, k)
    return 2.0 * np.sqrt(P) * E + E * E


def _check(gpu_lib, x, zmax, dz, seg, corr, nrand, seed):
    import torch
    n = x.shape[0]
    nb = n // 2
    bank = gpu_lib.make_templates(zmax, dz)
    plan = gpu_lib.Plan(bank, n, seg, nharm_max=1, sigma=6.0, correlator=corr)
    plane = torch.empty((bank.nz, nb), dtype=torch.float32, device="cuda")
    cands, nf = plan.search(torch.from_numpy(x).cuda(), plane=plane)
    torch.cuda.synchronize()
    Xh = O.normalise(O.real_spectrum(x), 1024)
    taps, zs, h = O.template_taps(zmax, dz)
    assert taps.shape[0] == bank.nz and h == bank.h
    L = (seg - 2 * h) & ~3
    rng = np.random.default_rng(seed)
    iz, k = _cells(rng, bank.nz, nb, L, nrand)
    Pg = plane[torch.from_numpy(iz).cuda(), torch.from_numpy(k).cuda()].cpu().numpy().astype(np.float64)
    Po = O.correlate_cells(Xh, taps, iz, k)
    if corr == "fft":
        tol = REL * np.maximum(Po, 1.0)
    else:
        tol = _bound_cells(Xh, taps, iz, k, corr)
    err = np.abs(Pg - Po)
    assert np.all(err <= tol), float(np.max(err / tol))
    # sampled candidates: oracle value near the GPU's, above threshold and a
    # local maximum (strict against earlier neighbours), within tolerance
    thr = O.thresholds(6.0, [1])[1]
    assert nf == len(cands) and np.all(cands["nharm"] == 1)
    pick = cands if len(cands) <= 60 else cands[rng.choice(len(cands), 60, replace=False)]
    for c in pick:
        kk, ii = int(c["k"]), int(c["iz"])
        nbr = [(ii + di, kk + dk) for di in (-1, 0, 1) for dk in (-1, 0, 1)
               if 0 <= ii + di < bank.nz and 0 <= kk + dk < nb]
        ai = np.array([a for a, _ in nbr])
        ak = np.array([b for _, b in nbr])
        Pn = O.correlate_cells(Xh, taps, ai, ak)
        if corr == "fft":
            tn = REL * np.maximum(Pn, 1.0)
        else:
            tn = _bound_cells(Xh, taps, ai, ak, corr)
        me = nbr.index((ii, kk))
        s0, t0 = Pn[me], tn[me]
        assert abs(c["power"] - s0) <= t0
        assert s0 >= thr - 2 * t0
        for j, (a, b) in enumerate(nbr):
            if j == me:
                continue
            earlier = a < ii or (a == ii and b < kk)
            ok = (s0 > Pn[j]) if earlier else (s0 >= Pn[j])
            assert ok or abs(s0 - Pn[j]) <= 2 * (t0 + tn[j])
    plan.close()
    bank.close()
    return len(cands)


@pytest.mark.parametrize("corr", ["fft", "bf16", "f16"])
def test_precision_shape_sampled(gpu_lib, corr):
    tr = next(t for t in synth.precision_trials(4) if t.pulsars)
    n = _check(gpu_lib, tr.x, 400.0, 1.0, 8192, corr, 1500, 11)
    assert n > 0


@pytest.mark.parametrize("nsamp", [1 << 21, 1 << 22])
def test_served_lengths_sampled(gpu_lib, nsamp):
    tr = synth.served_request({"nsamp": nsamp, "seed": 40007, "has_pulsar": True})
    n = _check(gpu_lib, tr.x, 200.0, 2.0, 8192, "fft", 1500, 12)
    assert n > 0


def test_longest_series_sampled(gpu_lib):
    # the longest series a plan takes (2^26 samples, 2^25 bins: the real DFT's
    # largest four-step split) with a small bank
    t = synth.make_series(1 << 26, seed=35, pulsars=[synth.Pulsar(r=12345678.4, z=9.0, amp=0.004, nharm=1)])
    n = _check(gpu_lib, t.x, 20.0, 2.0, 8192, "fft", 1500, 13)
    assert n > 0
