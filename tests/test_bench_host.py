"""Host logic of bench.py (no GPU): the one-GPU guard, the comment-insensitive hash
that ties the committed HBM-traffic counters to the GEMM code, the lookup of those
counters, and the far-rule pair fraction against the oracle's classification."""
import os
import subprocess
import sys

import numpy as np

import synth
from oracle import efie, rwg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_gemm_hash_ignores_comments_and_whitespace(tmp_path):
    src = open(bench.GEMM_SOURCE).read()
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    a.write_text(src)
    b.write_text("// a new comment line\n" + src.replace("\n", "\n  "))
    assert bench.gemm_code_sha256(str(a)) == bench.gemm_code_sha256(str(b)) == bench.gemm_code_sha256()
    c = tmp_path / "c.hip"
    c.write_text(src.replace("constexpr int AS = KC + 2;", "constexpr int AS = KC + 3;", 1))
    assert bench.gemm_code_sha256(str(c)) != bench.gemm_code_sha256()


def test_committed_traffic_matches_the_current_gemm():
    """The committed counters belong to the current GEMM code (else the bench line
    would report traffic null): one entry for the FP64-flush tile the tuner picks."""
    t, src = bench.measured_traffic([64, 32, 32], True, 30720, 512, "calderon")
    assert src is not None and 7.9e9 < t < 1e12
    assert bench.measured_traffic([64, 128, 16], True, 30720, 512, "calderon") == (None, None)
    assert bench.measured_traffic([64, 32, 32], True, 7680, 512, "calderon") == (None, None)


def test_committed_assembly_traffic_matches_the_current_tiles():
    """The committed assembly counters belong to the current tile code and the bench
    workload (the level-5 sphere at k = 10, complex64, no far rule), and show Z
    written once with at most three times its bytes in all."""
    t, src = bench.assembly_traffic(30720, 10.0, "c64", 0.0)
    z = 30720 * 30720 * 8
    assert src is not None and z <= t <= 3 * z
    assert bench.assembly_traffic(7680, 10.0, "c64", 0.0) == (None, None)
    assert bench.assembly_traffic(30720, 10.0, "c64", 4.0) == (None, None)
    # the same entry's shader counters: the kernel issues VALU instructions most of its time
    assert 0.5 < bench.assembly_valu_issue(30720, 10.0, "c64", 0.0) <= 1.0
    assert bench.assembly_valu_issue(30720, 10.0, "c128", 0.0) is None


def test_far3_fraction_matches_oracle_classification():
    v, f = synth.icosphere(2)
    m = rwg.build(v, f)
    n3 = nfar = 0
    for p in range(m.t):
        d = m.centroid - m.centroid[p]
        d2 = (d * d).sum(-1)
        hm = np.maximum(m.hmax, m.hmax[p])
        n3 += int(efie.far3_row(m, p, 3.0).sum())
        nfar += int(np.count_nonzero(d2 >= (2.0 * hm) ** 2))
    got = bench.far3_fraction(np.asarray(v, dtype=np.float64), np.asarray(f), 3.0)
    assert abs(got - n3 / nfar) < 1e-12


def test_assembly_alu_bound_is_the_cost_model():
    """The assembly's ALU bound is the algorithmic model (49 T^2/N^2 evaluations per
    entry, 46 FP32 or 110 FP64 issue slots each, no credit for the symmetry), not a
    count taken from the compiled kernel: about 39 Gentries/s (complex64) and 16
    Gentries/s (complex128) at 256 CUs x 64 lanes x 2.4 GHz on the level-5 sphere."""
    n, t = 30720, 20480
    assert abs(bench.assembly_alu_peak(n, t, "c64") - 3.93216e13 / (49 * 4 / 9 * 46) / 1e6) < 1e-6
    assert 39000 < bench.assembly_alu_peak(n, t, "c64") < 39500
    assert 16000 < bench.assembly_alu_peak(n, t, "c128") < 16500
