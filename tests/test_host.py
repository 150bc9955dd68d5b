"""Host-side behaviour that needs no GPU: the binding refuses to run without
the built library (no CPU fallback), the bench refuses more than one GPU, and
the bench's algorithmic byte and flop counts equal their closed forms at the
SKA shape."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    import paper_1511_07343_amd as fdas
    monkeypatch.setattr(fdas, "_lib", None)
    monkeypatch.setattr(fdas, "_LIB_PATH", str(tmp_path / "libfdas.so"))
    with pytest.raises(ImportError):
        fdas.load()
    with pytest.raises(ImportError):
        fdas.make_templates(10.0, 2.0)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_bench_counts_at_the_ska_shape():
    sys.path.insert(0, ROOT)
    import bench
    n, nz, S, h = 1 << 23, 201, 8192, 116
    nb = n // 2
    # series in 4 N, spectrum 2 x 8 Nb, plane 2 x 4 nz Nb
    assert bench.path_bytes(n, nz) == 4 * n + 16 * nb + 8 * nz * nb == 6_845_104_128
    L = (S - 2 * h) & ~3
    nseg = -(-nb // L)
    assert (L, nseg) == (7960, 527)
    # per (segment, template): 5 S log2 S + 6 S + 3 L
    assert bench.correlate_flops(nseg, nz, S, L) == nseg * nz * (5 * S * 13 + 6 * S + 3 * L)
    assert bench.correlate_bytes(nseg, nz, S, nb) == 4.5 * nz * nb + 8 * nseg * S + 8 * nz * S
    rl = bench.path_roofline(bench.path_bytes(n, nz), 100.0)
    assert rl["frac"] == pytest.approx(6.845104128e9 * 100 / 8e12, abs=1e-4)
