"""Pins of the oracle's templates (Sec. 2) against mathematics that does not
go through the oracle's own closed form."""
import math

import mpmath
import numpy as np
import pytest

import oracle as O


def _quad_response(q, z, dps=30):
    """A(q, z) by adaptive quadrature of its defining integral (mpmath)."""
    mpmath.mp.dps = dps
    q = mpmath.mpf(q)
    z = mpmath.mpf(z)
    f = lambda u: mpmath.expj(2 * mpmath.pi * ((q - z / 2) * u + z * u * u / 2))  # noqa: E731
    # split [0, 1] finely enough for the oscillation (|phase'| <= 2 pi (|q| + |z|))
    npieces = int(4 * (abs(float(q)) + abs(float(z)))) + 8
    pts = [mpmath.mpf(i) / npieces for i in range(npieces + 1)]
    v = mpmath.quad(f, pts)
    return complex(v)


@pytest.mark.parametrize("q,z", [(3.7, 40.0), (-12.2, -40.0), (0.0, 2.0), (55.0, 100.0),
                                 (-101.5, 200.0), (0.3, 1.0), (7.0, -3.0), (-60.0, 116.0)])
def test_closed_form_matches_quadrature(q, z):
    got = complex(O.template_response(np.array([q]), z)[0])
    ref = _quad_response(q, z)
    assert abs(got - ref) < 1e-12, (got, ref)


def test_zero_drift_is_fourier_bin_response():
    # z = 0: the standard response of an unaccelerated tone, exp(i pi q) sinc(q);
    # a Kronecker delta at integer offsets.
    q = np.arange(-50, 51, dtype=float)
    a = O.template_response(q, 0.0)
    delta = (q == 0).astype(float)
    assert np.max(np.abs(a - delta)) == 0.0
    qf = np.array([0.5, -0.25, 3.3])
    ref = np.exp(1j * np.pi * qf) * np.sin(np.pi * qf) / (np.pi * qf)
    assert np.max(np.abs(O.template_response(qf, 0.0) - ref)) < 1e-15
    # and the z = 0 taps of a bank are exactly the identity filter
    taps, zs, h = O.template_taps(100.0, 2.0)
    iz0 = int(np.nonzero(zs == 0.0)[0][0])
    row = taps[iz0]
    assert row[h] == 1.0 and np.count_nonzero(row) == 1


def test_time_reversal_identity():
    # u -> 1 - u in the defining integral: A(q, z) = exp(2 pi i q) A(-q, z).
    q = np.linspace(-80.3, 80.3, 97)
    for z in (1.0, 17.0, 40.0, 200.0):
        a = O.template_response(q, z)
        b = np.exp(2j * np.pi * q) * O.template_response(-q, z)
        assert np.max(np.abs(a - b)) < 1e-12


def test_drift_sign_symmetry():
    # complex conjugation of the integrand: A(q, -z) = conj(A(-q, z)),
    # hence T_{-z}[q] = conj(T_z[-q]) for the taps.
    taps, zs, h = O.template_taps(100.0, 2.0)
    nz = zs.shape[0]
    for iz in range(nz):
        assert np.max(np.abs(taps[nz - 1 - iz] - np.conj(taps[iz][::-1]))) < 1e-13


def test_energy_parseval():
    # The tone exp(2 pi i phi(u)) has unit modulus on [0, 1), so by Parseval its
    # Fourier coefficients at integer offsets carry total energy 1.
    for z in (3.0, 40.0, 200.0):
        q = np.arange(-4000, 4001, dtype=float)
        e = np.sum(np.abs(O.template_response(q, z)) ** 2)
        assert abs(e - 1.0) < 2e-4
        h = O.halfwidth(max(z, 2.0))
        qq = np.arange(-h, h + 1, dtype=float)
        kept = np.sum(np.abs(O.template_response(qq, z)) ** 2)
        assert kept > 0.997
    taps, _, _ = O.template_taps(200.0, 2.0)
    assert np.allclose(np.sum(np.abs(taps) ** 2, axis=1), 1.0, atol=1e-13)


def test_matched_filter_identity():
    # sum_j A(alpha - j, z1) conj(A(beta - j, z2)) = A(alpha - beta, z1 - z2)
    # (Poisson summation); this is why correlating with the conjugate template
    # gathers a drifting tone into one cell.
    j = np.arange(-6000, 6001, dtype=float)
    for (alpha, beta, z1, z2) in [(0.3, 0.0, 40.0, 40.0), (10.7, 2.0, 30.0, -12.0),
                                 (-5.2, 3.1, 100.0, 90.0)]:
        lhs = np.sum(O.template_response(alpha - j, z1) * np.conj(O.template_response(beta - j, z2)))
        rhs = O.template_response(np.array([alpha - beta]), z1 - z2)[0]
        assert abs(lhs - rhs) < 2e-3, (lhs, rhs)


def test_halfwidth_and_grid():
    assert O.halfwidth(100.0) == 66 and O.halfwidth(200.0) == 116 and O.halfwidth(400.0) == 216
    zs = O.z_values(200.0, 2.0)
    assert zs.shape[0] == 201 and zs[0] == -200.0 and zs[-1] == 200.0 and zs[100] == 0.0
    assert O.z_values(400.0, 1.0).shape[0] == 801
