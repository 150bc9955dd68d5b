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
