"""Plain, slow, FP64 CPU oracle of the FDAS hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may use this module.  It shares no code with the GPU library.

Source: S. Dimoudi and W. Armour, "Pulsar Acceleration Searches on the GPU for
the Square Kilometre Array" (arXiv:1511.07343).  Each function names the part
of the paper it follows.  The paper leaves several points open (normalisation,
template width, harmonic summing, thresholds, peak rule); the readings taken
here are stated where they are used.

Every step is the plain definition, with no FFT-based correlation, no
segmentation, no blocking:

1. ``real_spectrum``   real-to-complex DFT of the series (Sec. 4, step 2).
2. ``normalise``       block-median power normalisation (reading; paper silent).
3. ``template_taps``   constant-acceleration response and its conjugate, which
                        undoes the drift's spreading (Sec. 2, after Ransom et al.).
4. ``correlate``       Eq. (1) summed directly (plain C, FP64).
5. ``harmonic_sum``    incoherent sums over 1/2/4/8/16 harmonics (reading).
6. ``thresholds``      single-trial sigma threshold per harmonic count (reading).
7. ``find_peaks``      threshold plus 3x3 local maximum (reading).
8. ``interp_power``, ``refine``  Fourier interpolation of the correlation at
                        fractional (r, z) and a pattern search around each
                        candidate (an extension past the paper's method).
9. ``td_search``       the time-domain resampling search the paper names as
                        the other method (Sec. 1): resample per acceleration,
                        one long DFT each, harmonic sums along each spectrum.
10. ``dedisperse``     the de-dispersion that produces the series (Sec. 1:
                        one series per dispersion-measure trial).

Parity pins for each function live in tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np
from scipy import optimize, special

from . import build as _build

__all__ = [
    "LN2",
    "real_spectrum",
    "block_medians",
    "median_curve",
    "normalise",
    "template_response",
    "halfwidth",
    "z_values",
    "template_taps",
    "template_taps_half",
    "interbin_plane",
    "correlate",
    "correlate_cells",
    "harmonic_list",
    "harmonic_indices",
    "harmonic_sum",
    "harmonic_sum_cells",
    "thresholds",
    "log_survival",
    "sigma_of",
    "find_peaks",
    "Candidate",
    "SearchResult",
    "search",
    "interp_power",
    "interp_sum",
    "refine_start",
    "refine",
    "refine_endpoints",
    "td_alphas",
    "td_resample",
    "td_harmonic_sum",
    "td_search",
    "KDM",
    "dm_delays",
    "dedisperse",
]

LN2 = math.log(2.0)


# --------------------------------------------------------------------------
# 1. Real-to-complex DFT (Sec. 4, step 2)
# --------------------------------------------------------------------------
def real_spectrum(x) -> np.ndarray:
    """X_k = sum_n x_n exp(-2 pi i k n / N) for k in [0, N/2), in FP64.

    The Nyquist bin k = N/2 is dropped and the DC bin is set to zero, so the
    plane has N/2 frequency columns (reading: DC carries no periodic signal and
    the configurations quote N/2 columns).
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    if n % 2:
        raise ValueError("series length must be even")
    X = np.fft.rfft(x)[: n // 2].copy()
    if X.shape[0]:
        X[0] = 0.0
    return X


# --------------------------------------------------------------------------
# 2. Normalisation by block medians (reading; the paper is silent)
# --------------------------------------------------------------------------
def block_medians(power: np.ndarray, W: int):
    """Median of each block of W consecutive powers (last block may be short).

    For an even count the median is the mean of the two middle order
    statistics.  Returns (medians, centres) with centre_b = b W + (w_b - 1)/2.
    """
    power = np.asarray(power, dtype=np.float64)
    nb = power.shape[0]
    nblk = (nb + W - 1) // W
    med = np.empty(nblk)
    cen = np.empty(nblk)
    for b in range(nblk):
        blk = power[b * W: min(nb, (b + 1) * W)]
        med[b] = np.median(blk)
        cen[b] = b * W + (blk.shape[0] - 1) / 2.0
    return med, cen


def median_curve(power: np.ndarray, W: int) -> np.ndarray:
    """m(k): block medians joined linearly between block centres, held flat
    beyond the first and last centre."""
    med, cen = block_medians(power, W)
    k = np.arange(power.shape[0], dtype=np.float64)
    return np.interp(k, cen, med)


def normalise(X: np.ndarray, W: int = 1024) -> np.ndarray:
    """Xhat_k = X_k sqrt(ln 2 / m(k)).

    The median of an exponential distribution of mean mu is mu ln 2, so for
    white noise |Xhat|^2 is exponential with unit mean.  Bins whose local
    median m(k) is not positive (a spectrum that is zero over half a block)
    are set to zero.
    """
    X = np.asarray(X, dtype=np.complex128)
    p = X.real ** 2 + X.imag ** 2
    m = median_curve(p, W)
    scale = np.zeros_like(m)
    pos = m > 0
    scale[pos] = np.sqrt(LN2 / m[pos])
    return X * scale


# --------------------------------------------------------------------------
# 3. Templates (Sec. 2: the conjugate constant-acceleration response)
# --------------------------------------------------------------------------
def template_response(q, z: float) -> np.ndarray:
    """A(q, z): Fourier response at offset q = r - k bins of a unit sinusoid
    whose frequency drifts linearly by z bins over the observation.

        A(q, z) = int_0^1 exp(2 pi i [ (q - z/2) u + z u^2 / 2 ]) du

    Closed form through the Fresnel integrals C, S (normalised so that
    C(x) = int_0^x cos(pi t^2 / 2) dt):
      z = 0:  exp(i pi q) sin(pi q) / (pi q)  (1 at q = 0, 0 at other integers)
      z > 0:  with p = q - z/2, Y = p sqrt(2/z), Z = (p + z) sqrt(2/z),
              exp(-i pi p^2 / z) / sqrt(2 z) * ([C(Z) - C(Y)] + i [S(Z) - S(Y)])
      z < 0:  conj(A(-q, -z))
    """
    q = np.asarray(q, dtype=np.float64)
    if z == 0.0:
        out = np.exp(1j * np.pi * q) * np.sinc(q)
        integer = q == np.round(q)
        out = np.where(integer, np.where(q == 0.0, 1.0 + 0.0j, 0.0j), out)
        return out
    if z < 0.0:
        return np.conj(template_response(-q, -z))
    p = q - z / 2.0
    s = math.sqrt(2.0 / z)
    SY, CY = special.fresnel(p * s)
    SZ, CZ = special.fresnel((p + z) * s)
    # exp(-i pi p^2 / z) with the argument reduced mod 2 (in units of pi)
    ph = np.mod(p * p / z, 2.0)
    rot = np.exp(-1j * np.pi * ph)
    return rot / math.sqrt(2.0 * z) * ((CZ - CY) + 1j * (SZ - SY))


def halfwidth(zmax: float) -> int:
    """Template half-width h = ceil(zmax / 2) + 16 bins (reading).

    A drifting tone sweeps |z| bins centred on its mean frequency, so its
    response is spread over about +-|z|/2 bins plus sinc-like wings; 16 extra
    bins on each side keep more than 99.7 % of the response energy at
    |z| = zmax for the configurations used here.  m = 2h in Eq. (1).
    """
    return int(math.ceil(zmax / 2.0)) + 16


def z_values(zmax: float, dz: float) -> np.ndarray:
    """z grid -zmax + iz dz, iz = 0 .. 2 zmax / dz (inclusive)."""
    nz = int(round(2.0 * zmax / dz)) + 1
    return -zmax + dz * np.arange(nz, dtype=np.float64)


def template_taps(zmax: float, dz: float, h: int | None = None):
    """Inverse-filter taps T[iz, q + h] = conj(A(q, z_iz)) / ||A(., z_iz)||.

    The norm is taken over the 2h + 1 kept taps, which makes the correlated
    power of white unit-mean-power noise have unit mean (reading; the paper
    does not state a normalisation).  Returns (taps, zs, h).
    """
    if h is None:
        h = halfwidth(zmax)
    zs = z_values(zmax, dz)
    q = np.arange(-h, h + 1, dtype=np.float64)
    taps = np.empty((zs.shape[0], 2 * h + 1), dtype=np.complex128)
    for i, z in enumerate(zs):
        a = template_response(q, float(z))
        taps[i] = np.conj(a) / np.sqrt(np.sum(np.abs(a) ** 2))
    return taps, zs, h


def template_taps_half(zmax: float, dz: float, h: int | None = None):
    """Half-bin taps T'[iz, q + h] = conj(A(q + 1/2, z_iz)) / norm for
    q = -h .. h-1 and 0 at q = h: the template of the correlation at the
    point halfway between bins k and k + 1 (the offsets r - k' of the bins k'
    within h of r = k + 1/2), normalised over those 2h taps (reading; an
    extension past the paper's method).  Returns (taps, zs, h)."""
    if h is None:
        h = halfwidth(zmax)
    zs = z_values(zmax, dz)
    q = np.arange(-h, h, dtype=np.float64) + 0.5
    taps = np.zeros((zs.shape[0], 2 * h + 1), dtype=np.complex128)
    for i, z in enumerate(zs):
        a = template_response(q, float(z))
        taps[i, :2 * h] = np.conj(a) / np.sqrt(np.sum(np.abs(a) ** 2))
    return taps, zs, h


def interbin_plane(P: np.ndarray, P_half: np.ndarray) -> np.ndarray:
    """Half-bin plane on the half-bin grid: column 2k = P[:, k] (bin k),
    2k + 1 = P_half[:, k] (k + 1/2); the harmonic sums index it in half bins."""
    out = np.empty((P.shape[0], 2 * P.shape[1]), dtype=np.float64)
    out[:, 0::2] = P
    out[:, 1::2] = P_half
    return out


# --------------------------------------------------------------------------
# 4. Eq. (1), summed directly (plain C, FP64)
# --------------------------------------------------------------------------
_lib = None


def _clib():
    global _lib
    if _lib is None:
        path = _build.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_correlate_plane.argtypes = [dp, ctypes.c_int64, dp, ctypes.c_int32, ctypes.c_int32, dp]
        lib.oracle_correlate_plane.restype = None
        lib.oracle_correlate_cells.argtypes = [dp, ctypes.c_int64, dp, ctypes.c_int32, ctypes.c_int64,
                                               ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_int64), dp, dp]
        lib.oracle_correlate_cells.restype = None
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def correlate(Xhat: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """P[iz, k] = |sum_{q=-h}^{h} Xhat[k - q] T[iz, q]|^2, Xhat = 0 outside [0, nb).

    This is Eq. (1) with the output bin k as reference frequency r0, m = 2h,
    and the spectrum zero-padded (not wrapped) at both ends.
    """
    X = np.ascontiguousarray(Xhat, dtype=np.complex128)
    T = np.ascontiguousarray(taps, dtype=np.complex128)
    nz, ntap = T.shape
    h = (ntap - 1) // 2
    nb = X.shape[0]
    P = np.empty((nz, nb), dtype=np.float64)
    _clib().oracle_correlate_plane(_dptr(X.view(np.float64)), nb, _dptr(T.view(np.float64)),
                                   nz, h, _dptr(P))
    return P


def correlate_cells(Xhat: np.ndarray, taps: np.ndarray, iz, k, return_complex: bool = False):
    """Eq. (1) at the listed cells only (same definition as ``correlate``)."""
    X = np.ascontiguousarray(Xhat, dtype=np.complex128)
    T = np.ascontiguousarray(taps, dtype=np.complex128)
    iz = np.ascontiguousarray(iz, dtype=np.int32)
    k = np.ascontiguousarray(k, dtype=np.int64)
    n = iz.shape[0]
    h = (T.shape[1] - 1) // 2
    P = np.empty(n, dtype=np.float64)
    Y = np.empty(n, dtype=np.complex128) if return_complex else None
    _clib().oracle_correlate_cells(
        _dptr(X.view(np.float64)), X.shape[0], _dptr(T.view(np.float64)), h, n,
        iz.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(P),
        _dptr(Y.view(np.float64)) if Y is not None else ctypes.POINTER(ctypes.c_double)())
    return (P, Y) if return_complex else P


# --------------------------------------------------------------------------
# 5. Harmonic summing (reading; the paper is silent)
# --------------------------------------------------------------------------
def harmonic_list(nharm_max: int) -> List[int]:
    """Harmonic counts searched: 1, 2, 4, ... up to nharm_max (a power of two <= 16)."""
    if nharm_max not in (1, 2, 4, 8, 16):
        raise ValueError("nharm_max must be 1, 2, 4, 8 or 16")
    out, nh = [], 1
    while nh <= nharm_max:
        out.append(nh)
        nh *= 2
    return out


def harmonic_indices(k, iz, j: int, nh: int, izc: int):
    """Cell read for harmonic j of an nh-harmonic sum whose top harmonic is at (iz, k).

    Harmonic j of a fundamental (r, z) lies at (j r, j z); with the top
    harmonic nh at bin k and drift index iz (offset d = iz - izc from z = 0)
    harmonic j sits at k j / nh and d j / nh, rounded to the nearest cell with
    halves rounded away from zero:
        k_j  = floor((2 j k + nh) / (2 nh))
        iz_j = izc + sign(d) floor((2 |d| j + nh) / (2 nh))
    """
    k = np.asarray(k, dtype=np.int64)
    d = np.asarray(iz, dtype=np.int64) - izc
    kj = (2 * j * k + nh) // (2 * nh)
    izj = izc + np.sign(d) * ((2 * np.abs(d) * j + nh) // (2 * nh))
    return kj, izj


def harmonic_sum(P: np.ndarray, nh: int, izc: int) -> np.ndarray:
    """S_nh[iz, k] = sum_{j=1}^{nh} P[iz_j, k_j] over the whole plane (FP64)."""
    nz, nb = P.shape
    k = np.arange(nb, dtype=np.int64)
    iz = np.arange(nz, dtype=np.int64)
    S = np.zeros((nz, nb), dtype=np.float64)
    for j in range(1, nh + 1):
        kj, _ = harmonic_indices(k, izc, j, nh, izc)
        _, izj = harmonic_indices(0, iz, j, nh, izc)
        S += P[np.ix_(izj, kj)]
    return S


def harmonic_sum_cells(cell_power, iz, k, nh: int, izc: int) -> np.ndarray:
    """S_nh at listed cells; ``cell_power(iz_array, k_array)`` returns P there."""
    iz = np.asarray(iz, dtype=np.int64)
    k = np.asarray(k, dtype=np.int64)
    S = np.zeros(iz.shape[0], dtype=np.float64)
    for j in range(1, nh + 1):
        kj, izj = harmonic_indices(k, iz, j, nh, izc)
        S += cell_power(izj, kj)
    return S


# --------------------------------------------------------------------------
# 6. Thresholds and significance (reading of "n-sigma")
# --------------------------------------------------------------------------
def log_survival(S, nh: int):
    """log Q(nh, S), Q = exp(-S) sum_{i<nh} S^i / i!: the probability that a
    sum of nh independent unit-mean exponential powers reaches S."""
    S = np.atleast_1d(np.asarray(S, dtype=np.float64))
    out = np.empty_like(S)
    for n, s in enumerate(S):
        if s <= 0.0:
            out[n] = 0.0
            continue
        terms = [i * math.log(s) - math.lgamma(i + 1) for i in range(nh)]
        mx = max(terms)
        out[n] = -s + mx + math.log(sum(math.exp(t - mx) for t in terms))
    return out


def thresholds(sigma: float, nhs) -> Dict[int, float]:
    """thr(nh): the power sum whose null survival Q(nh, thr) equals the
    one-sided Gaussian tail probability Phi_c(sigma) (single-trial sigma)."""
    target = special.log_ndtr(-sigma)
    out = {}
    for nh in nhs:
        f = lambda P, nh=nh: log_survival(P, nh)[0] - target  # noqa: E731
        hi = 10.0
        while f(hi) > 0:
            hi *= 2.0
        out[nh] = optimize.brentq(f, 0.0, hi, xtol=1e-13, rtol=1e-15, maxiter=500)
    return out


def sigma_of(S: float, nh: int) -> float:
    """Gaussian-equivalent single-trial significance of a sum S of nh powers:
    the sigma with Phi_c(sigma) = Q(nh, S)."""
    lq = float(log_survival(S, nh)[0])
    f = lambda s: special.log_ndtr(-s) - lq  # noqa: E731
    lo, hi = -40.0, 40.0
    while f(hi) > 0:
        hi *= 2.0
    if f(lo) < 0:
        return lo
    return optimize.brentq(f, lo, hi, xtol=1e-12, maxiter=500)


# --------------------------------------------------------------------------
# 7. Peaks (reading)
# --------------------------------------------------------------------------
def find_peaks(S: np.ndarray, thr: float):
    """Cells (iz, k) with S >= thr that are local maxima of S over their 3x3
    neighbourhood (neighbours outside the plane ignored).

    Ties: a cell must be strictly greater than the neighbours that come before
    it in row-major (iz, k) order and at least equal to those after it.
    Returns an (n, 2) int64 array of (iz, k), sorted by k then iz.
    """
    nz, nb = S.shape
    pad = np.full((nz + 2, nb + 2), -np.inf)
    pad[1:-1, 1:-1] = S
    c = pad[1:-1, 1:-1]
    ok = c >= thr
    for di in (-1, 0, 1):
        for dk in (-1, 0, 1):
            if di == 0 and dk == 0:
                continue
            nbr = pad[1 + di: 1 + di + nz, 1 + dk: 1 + dk + nb]
            earlier = di < 0 or (di == 0 and dk < 0)
            ok &= (c > nbr) if earlier else (c >= nbr)
    iz, k = np.nonzero(ok)
    order = np.lexsort((iz, k))
    return np.stack([iz[order], k[order]], axis=1).astype(np.int64)


# --------------------------------------------------------------------------
# Whole path
# --------------------------------------------------------------------------
@dataclass
class Candidate:
    k: int
    iz: int
    nharm: int
    r: float
    z: float
    power: float
    sigma: float


@dataclass
class SearchResult:
    plane: np.ndarray
    candidates: List[Candidate]
    thresholds: Dict[int, float]
    spectrum: np.ndarray
    zs: np.ndarray
    h: int
    sums: Dict[int, np.ndarray] = field(default_factory=dict)


def search(x=None, *, spectrum=None, normalised: bool = False, zmax: float, dz: float,
           sigma: float = 6.0, nharm_max: int = 16, W: int = 1024,
           keep_sums: bool = False, interbin: bool = False) -> SearchResult:
    """The whole hot path on one series (or spectrum), every step in FP64.

    Candidates are reported per harmonic count, sorted by (nharm, k, iz); r and
    z describe the fundamental: r = k / nharm, z = z(iz) / nharm.  With
    interbin the plane has 2 nb columns (``interbin_plane``), k counts half
    bins and r = k / (2 nharm).
    """
    if x is not None:
        X = real_spectrum(x)
    else:
        X = np.asarray(spectrum, dtype=np.complex128)
    Xhat = X if normalised else normalise(X, W)
    taps, zs, h = template_taps(zmax, dz)
    P = correlate(Xhat, taps)
    cpb = 1
    if interbin:
        P = interbin_plane(P, correlate(Xhat, template_taps_half(zmax, dz, h)[0]))
        cpb = 2
    izc = int(round(zmax / dz))
    nhs = harmonic_list(nharm_max)
    thr = thresholds(sigma, nhs)
    cands: List[Candidate] = []
    sums = {}
    for nh in nhs:
        S = P if nh == 1 else harmonic_sum(P, nh, izc)
        if keep_sums:
            sums[nh] = S
        for iz, k in find_peaks(S, thr[nh]):
            s = float(S[iz, k])
            cands.append(Candidate(k=int(k), iz=int(iz), nharm=nh, r=k / (nh * cpb), z=float(zs[iz]) / nh,
                                   power=s, sigma=sigma_of(s, nh)))
    return SearchResult(plane=P, candidates=cands, thresholds=thr, spectrum=Xhat, zs=zs, h=h,
                        sums=sums)


# --------------------------------------------------------------------------
# 8. Fourier interpolation and candidate refinement (an extension past the
#    paper's method: the response of Sec. 2 evaluated off the (k, z) grid)
# --------------------------------------------------------------------------
def interp_power(Xhat: np.ndarray, r: float, z: float, h: int) -> float:
    """P(r, z): the correlation of Eq. (1) at a fractional frequency r (bins)
    and any drift z, with the template built for that exact offset (reading).

    The bins used are those within h of r, K(r) = {k : |r - k| <= h}; the
    template is the conjugate response at offsets r - k, normalised over K(r):
        Y = sum_{k in K(r)} Xhat[k] conj(A(r - k, z)) / sqrt(sum_{k in K(r)} |A(r - k, z)|^2)
    with Xhat = 0 outside [0, nb), and P = |Y|^2.  At an integer r and a grid
    z this is the plane cell of ``correlate``; for white unit-mean-power
    noise P is unit-mean exponential at every (r, z).
    """
    nb = Xhat.shape[0]
    k = np.arange(math.ceil(r - h), math.floor(r + h) + 1, dtype=np.int64)
    a = template_response(r - k.astype(np.float64), float(z))
    inside = (k >= 0) & (k < nb)
    y = np.sum(Xhat[k[inside]] * np.conj(a[inside]))
    return float(abs(y) ** 2 / np.sum(np.abs(a) ** 2))


def interp_sum(Xhat: np.ndarray, r: float, z: float, nh: int, h: int) -> float:
    """S(r, z) = sum_{j=1}^{nh} P(j r, j z): harmonic j of the fundamental
    (r, z) taken at its exact frequency and drift (no rounding to cells)."""
    return float(sum(interp_power(Xhat, j * r, j * z, h) for j in range(1, nh + 1)))


def refine_start(k: int, iz: int, nh: int, dz: float, izc: int, cpb: int = 1):
    """Fundamental of a candidate cell: r = k / (nh cpb), z = ((iz - izc) dz) / nh
    (cpb = 2 plane columns per bin on a half-bin plane)."""
    return k / (nh * cpb), (float(iz - izc) * dz) / nh


def _refine_level(Xhat, r, z, level, nh, dz, zmax, h):
    """Values of the 8 neighbours of (r, z) at one level, in search order:
    steps sr = 2^-level / nh, sz = (dz 2^-level) / nh; z-offset major, then
    r-offset, each in -1, 0, +1 (the centre itself skipped).  Points whose top
    harmonic drifts beyond the bank (|nh z| > zmax) are not candidates."""
    sr = 2.0 ** -level / nh
    sz = (dz * 2.0 ** -level) / nh
    out = []
    for b in (-1, 0, 1):
        for a in (-1, 0, 1):
            if a == 0 and b == 0:
                continue
            rr = r + a * sr
            zz = z + b * sz
            if abs(nh * zz) > zmax:
                continue
            out.append((rr, zz, interp_sum(Xhat, rr, zz, nh, h)))
    return out


def refine(Xhat: np.ndarray, k: int, iz: int, nh: int, *, zmax: float, dz: float, h: int,
           levels: int, cpb: int = 1):
    """Pattern search for the largest S(r, z) around a candidate (reading).

    Start at the candidate's fundamental; at each level l = 1 .. levels look
    at the 8 neighbours at steps (2^-l / nh, dz 2^-l / nh) in the order of
    ``_refine_level`` and move to the first one whose S is strictly larger
    than every value seen before it on this level (the centre's included).
    The steps halve per level, so the search can move up to one grid cell
    of the fundamental and ends on a (2^-levels)-fraction of it.  Returns
    (r, z, S, sigma) of the final point.
    """
    izc = int(round(zmax / dz))
    r, z = refine_start(k, iz, nh, dz, izc, cpb)
    best = interp_sum(Xhat, r, z, nh, h)
    for level in range(1, levels + 1):
        br, bz = r, z
        for rr, zz, s in _refine_level(Xhat, r, z, level, nh, dz, zmax, h):
            if s > best:
                best, br, bz = s, rr, zz
        r, z = br, bz
    return r, z, best, sigma_of(best, nh)


def refine_endpoints(Xhat: np.ndarray, k: int, iz: int, nh: int, *, zmax: float, dz: float, h: int,
                     levels: int, tol, max_paths: int = 1024, cpb: int = 1):
    """Every end point the search of ``refine`` can reach when values within
    tol(S) of a level's best count as ties (either may win in a different
    rounding): a dict {(r, z): S}.  Used to check a result computed in lower
    precision, where near-equal neighbours may be ordered differently."""
    izc = int(round(zmax / dz))
    r0, z0 = refine_start(k, iz, nh, dz, izc, cpb)
    paths = [(r0, z0, interp_sum(Xhat, r0, z0, nh, h))]
    for level in range(1, levels + 1):
        nxt = {}
        for r, z, s0 in paths:
            pts = [(r, z, s0)] + _refine_level(Xhat, r, z, level, nh, dz, zmax, h)
            top = max(p[2] for p in pts)
            for rr, zz, s in pts:
                if s >= top - tol(top):
                    nxt[(rr, zz)] = s
        if len(nxt) > max_paths:
            raise RuntimeError("refine_endpoints: too many near-tied paths")
        paths = [(rr, zz, s) for (rr, zz), s in nxt.items()]
    return {(r, z): s for r, z, s in paths}


# --------------------------------------------------------------------------
# 9. Time-domain resampling search (Sec. 1: the other acceleration search,
#    resampling the series per acceleration, then one long DFT per trial)
# --------------------------------------------------------------------------
def td_alphas(alpha_max: float, nalpha: int) -> np.ndarray:
    """Acceleration trials alpha_i = -alpha_max + i d, d = 2 alpha_max / (nalpha - 1)
    (one trial, alpha = 0, when nalpha is 1).  alpha is the frequency drift
    over the observation relative to the mean frequency: a tone of mean
    frequency r bins drifts by z = alpha r bins (reading)."""
    if nalpha == 1:
        return np.zeros(1)
    d = 2.0 * alpha_max / (nalpha - 1)
    return -alpha_max + d * np.arange(nalpha, dtype=np.float64)


def td_resample(x: np.ndarray, alpha: float) -> np.ndarray:
    """The series on a time axis along which a tone drifting by alpha (relative
    to its mean frequency) has constant frequency (reading).

    With u = n / N, v = u - 1/2, a tone of mean frequency rbar has phase
    2 pi rbar (v + alpha v^2 / 2) + const; the new axis is tau = v + alpha v^2 / 2,
    sampled at tau_m = m / N - 1/2, so sample m is x at
        v_m = 2 tau_m / (1 + sqrt(1 + 2 alpha tau_m))    (the root with v -> tau as alpha -> 0),
    position s_m = N (v_m + 1/2) samples, linearly interpolated between the two
    neighbouring samples (zero outside the series).
    """
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    tau = np.arange(N, dtype=np.float64) / N - 0.5
    v = 2.0 * tau / (1.0 + np.sqrt(1.0 + 2.0 * alpha * tau))
    spos = N * (v + 0.5)
    i = np.floor(spos).astype(np.int64)
    f = spos - i
    xp = np.concatenate([x, [0.0]])  # x[N] = 0
    ok = (i >= 0) & (i <= N - 1)
    ic = np.clip(i, 0, N - 1)
    return np.where(ok, xp[ic] * (1.0 - f) + xp[ic + 1] * f, 0.0)


def td_harmonic_sum(P: np.ndarray, nh: int) -> np.ndarray:
    """S_nh[i, k] = sum_{j=1}^{nh} P[i, k_j], k_j the rounding (half away from
    zero) of j k / nh: resampling removes the drift of every harmonic at once,
    so all harmonics of a trial lie in its own spectrum (reading)."""
    nb = P.shape[1]
    k = np.arange(nb, dtype=np.int64)
    S = np.zeros_like(P, dtype=np.float64)
    for j in range(1, nh + 1):
        S += P[:, (2 * j * k + nh) // (2 * nh)]
    return S


def td_search(x, *, alpha_max: float, nalpha: int, sigma: float = 6.0, nharm_max: int = 16,
              W: int = 1024, keep_sums: bool = False) -> SearchResult:
    """The time-domain resampling search on one series, every step in FP64:
    resample per trial (``td_resample``), real DFT (Sec. 4 step 2),
    normalisation (``normalise``), powers, harmonic sums along each trial's
    spectrum, thresholds and 3x3 local maxima over (trial, bin) as in
    ``find_peaks``.  Candidates: iz is the trial, r = k / nharm the
    fundamental's mean frequency, z = alpha r its drift over the
    observation."""
    alphas = td_alphas(alpha_max, nalpha)
    rows = []
    for a in alphas:
        X = real_spectrum(td_resample(x, float(a)))
        rows.append(np.abs(normalise(X, W)) ** 2)
    P = np.array(rows)
    nhs = harmonic_list(nharm_max)
    thr = thresholds(sigma, nhs)
    cands: List[Candidate] = []
    sums = {}
    for nh in nhs:
        S = P if nh == 1 else td_harmonic_sum(P, nh)
        if keep_sums:
            sums[nh] = S
        for iz, k in find_peaks(S, thr[nh]):
            s = float(S[iz, k])
            r = k / nh
            cands.append(Candidate(k=int(k), iz=int(iz), nharm=nh, r=r, z=float(alphas[iz]) * r, power=s,
                                   sigma=sigma_of(s, nh)))
    return SearchResult(plane=P, candidates=cands, thresholds=thr, spectrum=None, zs=alphas, h=0, sums=sums)


# --------------------------------------------------------------------------
# 10. De-dispersion (Sec. 1: the step before the search, one series per DM)
# --------------------------------------------------------------------------
KDM = 4.148808e3  # dispersion constant, s MHz^2 pc^-1 cm^3 (cold-plasma delay)


def dm_delays(nchan: int, f_top: float, foff: float, tsamp: float, dms) -> np.ndarray:
    """Integer sample delays d[i, c] = floor(KDM DM_i (f_c^-2 - f_top^-2) / tsamp + 1/2)
    of channel c (frequency f_c = f_top - c foff MHz) relative to the top of the
    band, for each DM (pc cm^-3): the cold-plasma dispersion delay rounded to
    the nearest sample (reading: the paper only names de-dispersion)."""
    f = f_top - foff * np.arange(nchan, dtype=np.float64)
    dms = np.asarray(dms, dtype=np.float64)
    raw = KDM * dms[:, None] * (1.0 / (f[None, :] * f[None, :]) - 1.0 / (f_top * f_top)) / tsamp
    return np.floor(raw + 0.5).astype(np.int64)


def dedisperse(fil: np.ndarray, f_top: float, foff: float, tsamp: float, dms, nout: int) -> np.ndarray:
    """y[i, t] = sum_c fil[c, t + d[i, c]] for t < nout: the channels of a
    channel-major filterbank (nchan x nsamp samples, 8-bit) shifted by their
    delays and added, in exact integer arithmetic (returned as float64)."""
    fil = np.asarray(fil)
    nchan, nsamp = fil.shape
    d = dm_delays(nchan, f_top, foff, tsamp, dms)
    if nout > nsamp - int(d.max(initial=0)):
        raise ValueError("nout exceeds the samples every channel can supply")
    out = np.zeros((d.shape[0], nout), dtype=np.int64)
    for i in range(d.shape[0]):
        for c in range(nchan):
            out[i] += fil[c, d[i, c]:d[i, c] + nout].astype(np.int64)
    return out.astype(np.float64)
