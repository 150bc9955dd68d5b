"""The C-ABI library: it loads, exports every symbol include/fdas.h declares,
its host-side FP64 template and threshold code agrees with the oracle, and it
rejects bad arguments before touching the device.  No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1511_07343_amd as fdas

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdas.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(fdas_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = fdas.load()
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_cand_struct_layout():
    assert fdas.CAND_DTYPE.itemsize == 40
    assert fdas.CAND_DTYPE.fields["power"][1] == 32 and fdas.CAND_DTYPE.fields["sigma"][1] == 36


@pytest.mark.parametrize("zmax,dz", [(100.0, 2.0), (200.0, 2.0), (20.0, 1.0), (400.0, 8.0), (0.0, 1.0)])
def test_bank_taps_match_oracle(zmax, dz):
    bank = fdas.make_templates(zmax, dz)
    taps, zs, h = O.template_taps(zmax, dz)
    assert bank.nz == zs.shape[0] and bank.h == h
    for iz in range(bank.nz):
        assert bank.z(iz) == pytest.approx(zs[iz], abs=1e-12)
        assert np.max(np.abs(bank.taps(iz) - taps[iz])) < 1e-12
    bank.close()


def test_thresholds_and_significance_match_oracle():
    for sig in (3.0, 6.0, 8.5):
        thr = O.thresholds(sig, [1, 2, 4, 8, 16])
        for nh, t in thr.items():
            assert fdas.threshold(sig, nh) == pytest.approx(t, rel=1e-12)
    for s, nh in [(25.0, 1), (60.0, 16), (400.0, 4), (3000.0, 2)]:
        assert fdas.significance(s, nh) == pytest.approx(O.sigma_of(s, nh), abs=1e-8)


def test_bad_template_arguments():
    lib = fdas.load()
    h = ctypes.c_void_p()
    for zmax, dz in [(-1.0, 2.0), (100.0, 0.0), (100.0, 3.0), (1e6, 1.0)]:
        assert lib.fdas_make_templates(zmax, dz, ctypes.byref(h)) == -1
        assert h.value is None
    with pytest.raises(fdas.FdasError) as e:
        fdas.make_templates(10.0, 3.0)
    assert "integer" in e.value.message


def test_bad_plan_arguments_rejected_before_device():
    lib = fdas.load()
    bank = fdas.make_templates(100.0, 2.0)  # h = 66, so seg >= 264
    h = ctypes.c_void_p()
    o = fdas._opts()
    for nsamp, seg in [(3000, 2048), (1 << 17, 1000), (1 << 17, 256), (1 << 27, 2048), (512, 2048)]:
        assert lib.fdas_plan(bank.handle, nsamp, seg, ctypes.byref(o), ctypes.byref(h)) == -1
    bad = fdas._opts(nharm_max=3)
    assert lib.fdas_plan(bank.handle, 1 << 17, 2048, ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = fdas._opts(median_window=1000)
    assert lib.fdas_plan(bank.handle, 1 << 17, 2048, ctypes.byref(bad), ctypes.byref(h)) == -1
    assert lib.fdas_plan(None, 1 << 17, 2048, ctypes.byref(o), ctypes.byref(h)) == -1
    assert lib.fdas_search(None, 0, None, None, None, 0, None, None) == -1
    assert lib.fdas_dft_c64(5, 0, 1, None, None, None) == -1
    assert lib.fdas_strerror(-4) == b"candidate capacity exceeded"
    bank.close()


def test_matrix_correlator_option_validation():
    """Plan options are checked before any device work: an unknown correlator,
    or a matrix correlator with a bank wider than h = 271, is INVAL."""
    import paper_1511_07343_amd as fdas

    narrow = fdas.make_templates(20.0, 2.0)
    wide = fdas.make_templates(600.0, 2.0)
    try:
        lib = fdas.load()
        o = fdas._opts(correlator="bf16")
        o.correlator = 7
        h = ctypes.c_void_p()
        assert lib.fdas_plan(narrow._h, 1 << 14, 256, ctypes.byref(o), ctypes.byref(h)) == -1
        o = fdas._opts(correlator="f16")
        assert lib.fdas_plan(wide._h, 1 << 14, 4096, ctypes.byref(o), ctypes.byref(h)) == -1
        assert b"h <= 271" in lib.fdas_last_error()
        with pytest.raises(ValueError):
            fdas._opts(correlator="tf32")
    finally:
        narrow.close()
        wide.close()
