"""Sampled full-size parity of the extension rows, in the configurations the
measurements run: the half-bin plane and the time-domain resampling search on
the SKA-shaped trial (2^23 samples), refinement of the trial's most
significant records, and de-dispersion of a 64-channel filterbank into 256
series of 2^23 samples.  Each compares the GPU with the FP64 oracle on
sampled outputs the oracle computes one by one (cells, whole rows, records):
the 1e-4 rule for powers and sums, bit-exact integer sums for
de-dispersion."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import REL

pytestmark = pytest.mark.gpu

N = 1 << 23


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _tol(s, nh):
    return REL * max(abs(s), nh)


def _check_peak(S, tolf, nbr, me, thr):
    """Cell me of the neighbourhood nbr (list of (iz, k)) with oracle sums S:
    above threshold and a 3x3 local maximum (strict against earlier cells),
    up to the tolerance."""
    s0 = S[me]
    assert s0 >= thr - 2 * tolf(thr)
    ii, kk = nbr[me]
    for j, (a, b) in enumerate(nbr):
        if j == me:
            continue
        earlier = a < ii or (a == ii and b < kk)
        ok = (s0 > S[j]) if earlier else (s0 >= S[j])
        assert ok or abs(s0 - S[j]) <= 2 * tolf(s0), (nbr[me], nbr[j], s0, S[j])


def test_half_bin_plane_full_size_sampled(gpu_lib):
    import torch
    tr = synth.ska_trial()
    zmax, dz, seg = 200.0, 2.0, 8192
    bank = gpu_lib.make_templates(zmax, dz)
    plan = gpu_lib.Plan(bank, N, seg, nharm_max=16, sigma=6.0, interbin=True)
    nb = N // 2
    plane = torch.empty((bank.nz, 2 * nb), dtype=torch.float32, device="cuda")
    cands, nf = plan.search(_dev(tr.x), plane=plane)
    torch.cuda.synchronize()
    Xh = O.normalise(O.real_spectrum(tr.x), 1024)
    taps, _, h = O.template_taps(zmax, dz)
    half, _, _ = O.template_taps_half(zmax, dz)

    def cell(iz, c):  # oracle power at half-bin column c (bin c/2 or half point (c-1)/2)
        iz = np.asarray(iz)
        c = np.asarray(c)
        out = np.empty(c.shape[0])
        ev = c % 2 == 0
        if ev.any():
            out[ev] = O.correlate_cells(Xh, taps, iz[ev], c[ev] // 2)
        if (~ev).any():
            out[~ev] = O.correlate_cells(Xh, half, iz[~ev], c[~ev] // 2)
        return out

    rng = np.random.default_rng(31)
    L = (seg - 2 * h) & ~3
    k = np.concatenate([rng.integers(0, nb, 1500), np.arange(3), L - 1 + np.arange(3), nb - 2 + np.arange(2)])
    iz = rng.integers(0, bank.nz, k.shape[0])
    ti, tk = torch.from_numpy(iz).cuda(), torch.from_numpy(k).cuda()
    got_bin = plane[ti, tk].cpu().numpy().astype(np.float64)  # library row: Nb bins, then Nb half points
    got_half = plane[ti, tk + nb].cpu().numpy().astype(np.float64)
    want_bin = cell(iz, 2 * k)
    want_half = cell(iz, 2 * k + 1)
    assert np.all(np.abs(got_bin - want_bin) <= REL * np.maximum(want_bin, 1.0))
    assert np.all(np.abs(got_half - want_half) <= REL * np.maximum(want_half, 1.0))
    # sampled candidates on the half-bin grid (2 Nb columns, harmonics in half bins)
    thr = O.thresholds(6.0, [1, 2, 4, 8, 16])
    izc = (bank.nz - 1) // 2
    assert nf == len(cands) > 0
    pick = cands[rng.choice(len(cands), min(40, len(cands)), replace=False)]
    for c in pick:
        nh, kk, ii = int(c["nharm"]), int(c["k"]), int(c["iz"])
        assert c["r"] == kk / (2.0 * nh)
        nbr = [(ii + di, kk + dk) for di in (-1, 0, 1) for dk in (-1, 0, 1)
               if 0 <= ii + di < bank.nz and 0 <= kk + dk < 2 * nb]
        S = np.array([O.harmonic_sum_cells(cell, [a], [b], nh, izc)[0] for a, b in nbr])
        me = nbr.index((ii, kk))
        assert abs(c["power"] - S[me]) <= _tol(S[me], nh)
        _check_peak(S, lambda s: _tol(s, nh), nbr, me, thr[nh])
    plan.close()
    bank.close()


def test_time_domain_full_size_sampled(gpu_lib):
    import torch
    tr = synth.ska_trial()
    amax, nal = 0.02, 201
    plan = gpu_lib.TdPlan(N, amax, nal, nharm_max=16, sigma=6.0)
    nb = N // 2
    plane = torch.empty((nal, nb), dtype=torch.float32, device="cuda")
    cands, nf = plan.search(_dev(tr.x), plane=plane, cap=1 << 22)
    torch.cuda.synchronize()
    alphas = O.td_alphas(amax, nal)
    assert np.array_equal(plan.alphas, alphas)
    # the row of the strongest candidate and its two neighbours, whole, plus
    # the first and last trials
    assert nf == len(cands) > 0
    top = cands[np.argmax(cands["sigma"])]
    i0 = int(top["iz"])
    rows = sorted({0, nal - 1, max(i0 - 1, 0), i0, min(i0 + 1, nal - 1)})
    P = {}
    for i in rows:
        P[i] = np.abs(O.normalise(O.real_spectrum(O.td_resample(tr.x, float(alphas[i]))), 1024)) ** 2
        got = plane[i].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - P[i]) <= REL * np.maximum(P[i], 1.0)), i
    # every candidate of row i0 whose neighbourhood lies in the computed rows
    thr = O.thresholds(6.0, [1, 2, 4, 8, 16])
    S = {nh: {i: O.td_harmonic_sum(P[i][None, :], nh)[0] for i in P} for nh in (1, 2, 4, 8, 16)}
    mine = cands[cands["iz"] == i0]
    assert len(mine) > 0
    for c in mine[:200]:
        nh, kk = int(c["nharm"]), int(c["k"])
        nbr = [(i0 + di, kk + dk) for di in (-1, 0, 1) for dk in (-1, 0, 1)
               if 0 <= i0 + di < nal and 0 <= kk + dk < nb]
        Sv = np.array([S[nh][a][b] for a, b in nbr])
        me = nbr.index((i0, kk))
        assert abs(c["power"] - Sv[me]) <= _tol(Sv[me], nh)
        assert c["z"] == alphas[i0] * c["r"]
        _check_peak(Sv, lambda s: _tol(s, nh), nbr, me, thr[nh])
    plan.close()


def test_refine_full_size(gpu_lib):
    tr = synth.ska_trial()
    zmax, dz = 200.0, 2.0
    bank = gpu_lib.make_templates(zmax, dz)
    plan = gpu_lib.Plan(bank, N, 8192, nharm_max=16, sigma=6.0)
    cands, nf = plan.search(_dev(tr.x))
    rng = np.random.default_rng(33)
    order = np.argsort(-cands["sigma"], kind="stable")
    sel = cands[np.concatenate([order[:10], rng.choice(order[10:], 10, replace=False)])]
    ref = plan.refine(sel, 6)
    Xh = O.normalise(O.real_spectrum(tr.x), 1024)
    for c0, c in zip(sel, ref):
        nh = int(c["nharm"])
        assert (c["k"], c["iz"], c["nharm"]) == (c0["k"], c0["iz"], c0["nharm"])
        ends = O.refine_endpoints(Xh, int(c["k"]), int(c["iz"]), nh, zmax=zmax, dz=dz, h=bank.h, levels=6,
                                  tol=lambda s: 2.0 * _tol(s, nh))
        key = (float(c["r"]), float(c["z"]))
        assert key in ends, (c, sorted(ends)[:5])
        assert abs(float(c["power"]) - ends[key]) <= _tol(ends[key], nh) + 1e-7 * ends[key]
    plan.close()
    bank.close()


def test_dedisperse_full_size_rows(gpu_lib):
    import torch
    nchan, f_top, foff, tsamp = 64, 1500.0, 4.0, 64e-6
    dms = np.linspace(0.0, 500.0, 256)
    d = O.dm_delays(nchan, f_top, foff, tsamp, dms)
    nsamp = N + int(d.max())
    fil = synth.make_filterbank(nchan, nsamp, f_top, foff, tsamp, seed=34)
    out = gpu_lib.dedisperse(_dev(fil), f_top, foff, tsamp, dms, N)
    torch.cuda.synchronize()
    for i in (0, 97, 255):
        want = O.dedisperse(fil, f_top, foff, tsamp, [dms[i]], N)[0]
        assert np.array_equal(out[i].cpu().numpy().astype(np.float64), want), i
