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


def is_borderline(S: np.ndarray, thr: float, nh: int, iz: int, k: int) -> bool:
    s = S[iz, k]
    if abs(s - thr) <= 2 * _tau(thr, nh):
        return True
    nz, nb = S.shape
    for di in (-1, 0, 1):
        for dk in (-1, 0, 1):
            if (di, dk) == (0, 0):
                continue
            i, j = iz + di, k + dk
            if 0 <= i < nz and 0 <= j < nb and abs(s - S[i, j]) <= 2 * _tau(s, nh):
                return True
    return False


def compare_candidates(gpu: np.ndarray, orc) -> dict:
    """gpu: structured array (CAND_DTYPE); orc: oracle SearchResult with sums
    kept (or nharm_max 1).  Returns a report; report['ok'] is the verdict."""
    sums = dict(orc.sums)
    sums.setdefault(1, orc.plane)
    o = {(c.nharm, c.k, c.iz): c.power for c in orc.candidates}
    g = {(int(c["nharm"]), int(c["k"]), int(c["iz"])): float(c["power"]) for c in gpu}
    missing, extra, border = [], [], 0
    for key in set(o) - set(g):
        nh, k, iz = key
        if is_borderline(sums[nh], orc.thresholds[nh], nh, iz, k):
            border += 1
        else:
            missing.append(key)
    for key in set(g) - set(o):
        nh, k, iz = key
        if is_borderline(sums[nh], orc.thresholds[nh], nh, iz, k):
            border += 1
        else:
            extra.append(key)
    worst = 0.0
    for key in set(g) & set(o):
        nh = key[0]
        worst = max(worst, abs(g[key] - o[key]) / max(o[key], nh))
    # sorted order (nharm, k, iz)
    keys = [(int(c["nharm"]), int(c["k"]), int(c["iz"])) for c in gpu]
    return dict(ok=not missing and not extra and worst <= REL and keys == sorted(keys),
                missing=missing, extra=extra, borderline=border, n_gpu=len(g), n_orc=len(o),
                max_power_err=worst, sorted=keys == sorted(keys))
