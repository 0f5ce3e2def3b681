"""Host logic of bench.py that needs no GPU: the counter-measured traffic is
reported only for the workload and kernel source it was measured on, and a
request for more than one GPU is refused before anything touches a device."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _entry(source, sha, nbytes=123.0):
    return {"source": source, "sha256": sha, "bytes": nbytes}


def _sha(source):
    path = os.path.join(ROOT, "paper_2109_13655_amd", "csrc", source)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def test_traffic_only_for_the_profiled_source_and_workload():
    for source in ("k_bspmm.hip", "k_block.hip"):
        good = _entry(source, _sha(source))
        assert bench.profiled_traffic("c2", good) == 123.0
        assert bench.profiled_traffic("c3", good) is None
        assert bench.profiled_traffic("c2", _entry(source, "0" * 64)) is None
    assert bench.profiled_traffic("c2", _entry("no_such_file.hip", "0" * 64)) is None


def test_stored_entries_name_existing_sources():
    for e in (bench.SPMM_TRAFFIC_C2, bench.MOMENTS_TRAFFIC_C2):
        assert os.path.exists(os.path.join(ROOT, "paper_2109_13655_amd", "csrc", e["source"]))
        assert len(e["sha256"]) == 64 and e["bytes"] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_experiment1_filter_values_match_the_oracle():
    """The filter curves of the Experiment I harness (from the library's
    quadrature) equal the oracle's filter functions f and f_g."""
    import numpy as np
    import paper_2109_13655_amd as cs
    from oracle import quadrature as Q
    for a, b in ((0.8, 1.2), (1e-3, 1e-1)):
        s = np.logspace(-4, 0.2, 37)
        for tr, qt in ((cs.CSVD_PLAIN, Q.PLAIN), (cs.CSVD_EXP, Q.EXP)):
            got = bench.filter_values(cs, a, b, s, tr)
            ref = Q.filter_f(s, a, b, 32, alpha=0.1, transform=qt)
            np.testing.assert_allclose(got, ref.real, rtol=1e-10, atol=1e-13)
