"""Host-side checks of bench.py (no GPU): the one-GPU refusal, the flop
count its roofline uses, and the format of the committed traffic record."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bulk_flop_count_of_the_benchmark():
    """2 (multiply-add) x 2 n_w rows x 2 (Re, Im) x (upper-triangle pairs
    without the G = 0 row) x N_T, for N_G = 113, 400 w, 8^3 k, 4 + 16 bands."""
    import bench
    from synth import make_si_ng113

    wl = make_si_ng113(n_q=1)
    pairs = 113 * 114 // 2 - 113
    assert pairs == 6328 and wl.n_t == 2 * 4 * 16 * 512
    assert bench.bulk_flops_per_launch(wl) == pytest.approx(2.0 * 800 * 2 * pairs * 65536)
    assert bench.bulk_flops_per_launch(wl) == pytest.approx(1.327077785600e12)


def test_traffic_record_format():
    """The committed counter summary names a 16-hex source hash and bytes per
    launch no smaller than the algorithmic operands (R, weights, partials)."""
    import bench

    txt = open(bench.TRAFFIC_FILE).read()
    m_h = re.search(r"source_sha256_16:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    assert m_h and len(m_h.group(1)) == 16
    algorithmic = 113 * 65536 * 8 + 800 * 65536 * 4 + 8 * 800 * 12800 * 4
    assert float(m_b.group(1)) >= algorithmic
    assert len(bench.kernel_source_hash()) == 16
