"""Comparison rules between the GPU path and the FP64 oracle.

Powers: |P_gpu - P_orc| <= 1e-4 max(P_orc, 1) per plane cell; harmonic sums
<= 1e-4 max(S_orc, nh).  Candidate indices must match exactly, except at
cells where FP32 and FP64 may legitimately decide differently ("borderline"):
an oracle cell is borderline for nh when its sum is within 2 tau(thr) of the
threshold, or within 2 tau(S) of one of its in-plane neighbours, with
tau(x) = 1e-4 max(|x|, nh).
"""
from __future__ import annotations

import numpy as np

REL = 1e-4


def plane_errors(P_gpu: np.ndarray, P_orc: np.ndarray):
    """(max scaled error, max rel error over P >= 1, rms rel error over P >= 1)."""
    P_gpu = np.asarray(P_gpu, dtype=np.float64)
    err = np.abs(P_gpu - P_orc)
    scaled = err / np.maximum(P_orc, 1.0)
    big = P_orc >= 1.0
    rel = err[big] / P_orc[big] if np.any(big) else np.zeros(1)
    return float(scaled.max()), float(rel.max()), float(np.sqrt(np.mean(rel ** 2)))


def _tau(x, nh):
    return REL * max(abs(x), nh)


def is_borderline(S: np.ndarray, thr: float, nh: int, iz: int, k: int, tol: np.ndarray | None = None) -> bool:
    """With tol (per-cell absolute error bounds of S) a decision may differ
    where the oracle's sum is within tol of the threshold, or where the
    bounds of two neighbours overlap; else the 2 tau rule above."""
    s = S[iz, k]
    if tol is None:
        if abs(s - thr) <= 2 * _tau(thr, nh):
            return True
    elif abs(s - thr) <= tol[iz, k]:
        return True
    nz, nb = S.shape
    for di in (-1, 0, 1):
        for dk in (-1, 0, 1):
            if (di, dk) == (0, 0):
                continue
            i, j = iz + di, k + dk
            if not (0 <= i < nz and 0 <= j < nb):
                continue
            lim = 2 * _tau(s, nh) if tol is None else tol[iz, k] + tol[i, j]
            if abs(s - S[i, j]) <= lim:
                return True
    return False


def compare_candidates(gpu: np.ndarray, orc, tol: dict | None = None) -> dict:
    """gpu: structured array (CAND_DTYPE); orc: oracle SearchResult with sums
    kept (or nharm_max 1).  tol: optional {nh: per-cell absolute error bound
    of the GPU's sums}, replacing the 1e-4 rule (for the 16-bit correlators).
    Returns a report; report['ok'] says whether the two sets agree."""
    sums = dict(orc.sums)
    sums.setdefault(1, orc.plane)
    tol = tol or {}
    o = {(c.nharm, c.k, c.iz): c.power for c in orc.candidates}
    g = {(int(c["nharm"]), int(c["k"]), int(c["iz"])): float(c["power"]) for c in gpu}
    missing, extra, border = [], [], 0
    for key in set(o) - set(g):
        nh, k, iz = key
        if is_borderline(sums[nh], orc.thresholds[nh], nh, iz, k, tol.get(nh)):
            border += 1
        else:
            missing.append(key)
    for key in set(g) - set(o):
        nh, k, iz = key
        if is_borderline(sums[nh], orc.thresholds[nh], nh, iz, k, tol.get(nh)):
            border += 1
        else:
            extra.append(key)
    worst = 0.0  # max error as a fraction of the allowed error
    for key in set(g) & set(o):
        nh, k, iz = key
        allowed = tol[nh][iz, k] if nh in tol else REL * max(o[key], nh)
        worst = max(worst, abs(g[key] - o[key]) / allowed)
    # sorted order (nharm, k, iz)
    keys = [(int(c["nharm"]), int(c["k"]), int(c["iz"])) for c in gpu]
    return dict(ok=not missing and not extra and worst <= 1.0 and keys == sorted(keys),
                missing=missing, extra=extra, borderline=border, n_gpu=len(g), n_orc=len(o),
                max_power_err=worst * (REL if not tol else 1.0), max_err_fraction=worst,
                sorted=keys == sorted(keys))


# ------------------------------------------------ banded full-size checks
def band_sums(Xh: np.ndarray, taps: np.ndarray, izc: int, k0: int, k1: int, nhs):
    """The oracle's harmonic sums S_nh over every plane row for the columns
    [a, b) = [k0 - 1, k1 + 1) clipped to the plane (one column of margin for
    the 3x3 neighbours of [k0, k1)).

    Each sum needs fraction m/16 (m = 16 j / nh) of every column: the
    columns floor((m k + 8) / 16), k in [a, b), of all rows.  Those are
    correlated directly by the oracle (Eq. (1), FP64) on a zero-padded slice
    of the normalised spectrum, and the sums are taken with the oracle's own
    harmonic index maps.  Returns (a, {nh: S[nz, b - a]})."""
    import oracle as O
    nb = Xh.shape[0]
    nz, ntap = taps.shape
    h = (ntap - 1) // 2
    a, b = max(k0 - 1, 0), min(k1 + 1, nb)
    ks = np.arange(a, b, dtype=np.int64)
    cache = {}

    def cols(m):
        if m not in cache:
            c0 = (m * a + 8) // 16
            c1 = (m * (b - 1) + 8) // 16 + 1
            lo, hi = c0 - h, c1 + h
            seg = np.zeros(hi - lo, dtype=np.complex128)
            s0, s1 = max(lo, 0), min(hi, nb)
            seg[s0 - lo:s1 - lo] = Xh[s0:s1]
            cache[m] = (c0, O.correlate(seg, taps)[:, h:h + (c1 - c0)])
        return cache[m]

    rows = np.arange(nz, dtype=np.int64)
    out = {}
    for nh in nhs:
        if 16 % nh:
            raise ValueError("nh must divide 16")
        S = np.zeros((nz, b - a), dtype=np.float64)
        for j in range(1, nh + 1):
            c0, P = cols(16 * j // nh)
            kj, _ = O.harmonic_indices(ks, izc, j, nh, izc)
            _, izj = O.harmonic_indices(0, rows, j, nh, izc)
            S += P[np.ix_(izj, kj - c0)]
        out[nh] = S
    return a, out


def compare_band(gpu: np.ndarray, sums: dict, thr: dict, a: int, k0: int, k1: int) -> dict:
    """Both directions of the candidate comparison restricted to the columns
    [k0, k1): every oracle candidate there (threshold and 3x3 maximum of the
    band's sums) must be a GPU candidate and every GPU candidate there an
    oracle candidate, except at borderline cells; common candidates' sums
    agree to 1e-4 max(S, nh).  sums: band_sums output starting at column a."""
    import oracle as O
    o = {}
    for nh, S in sums.items():
        for iz, kl in O.find_peaks(S, thr[nh]):
            k = int(kl) + a
            if k0 <= k < k1:
                o[(nh, k, int(iz))] = float(S[iz, kl])
    sel = (gpu["k"] >= k0) & (gpu["k"] < k1)
    g = {(int(c["nharm"]), int(c["k"]), int(c["iz"])): float(c["power"]) for c in gpu[sel]}
    missing, extra, border = [], [], 0
    for key in set(o) ^ set(g):
        nh, k, iz = key
        if nh in sums and is_borderline(sums[nh], thr[nh], nh, iz, k - a):
            border += 1
        elif key in o:
            missing.append(key)
        else:
            extra.append(key)
    worst = 0.0
    for key in set(g) & set(o):
        worst = max(worst, abs(g[key] - o[key]) / (REL * max(o[key], key[0])))
    return dict(ok=not missing and not extra and worst <= 1.0, missing=missing, extra=extra,
                borderline=border, n_gpu=len(g), n_orc=len(o), common=len(set(g) & set(o)),
                max_err_fraction=worst)
