"""Host-side parts of bench.py that run without a GPU: the single-GPU guard,
the oracle timing leg and its host record, and the traffic summaries' source
digest."""
import os
import subprocess
import sys

import numpy as np

import oracle
from paper_1907_08607_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_host_info():
    h = bench.host_info()
    assert h["host_nproc"] >= 1
    assert isinstance(h["host_cpu"], str) and h["host_cpu"]


def test_cpu_baseline_record():
    g = gg.workload_er_1k_planted()
    w = oracle.wedges(g, oracle.rank(g, "degree"))
    cb = bench.cpu_baseline(g, w, 0.2)
    for k in ("value", "unit", "cores", "kind", "sample", "host_nproc", "host_cpu"):
        assert k in cb
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["unit"] == "wedges/s"
    assert np.isfinite(cb["value"]) and cb["value"] > 0


def test_traffic_summaries_name_their_sources():
    """Each committed traffic summary records the digest of the counting
    sources it was measured on, in the form bench.py compares."""
    prof = os.path.join(ROOT, "profiles")
    found = 0
    for name in os.listdir(prof):
        if not name.endswith("_traffic.txt"):
            continue
        fields = dict(line.split(": ", 1) for line in open(os.path.join(prof, name)).read().splitlines()
                      if ": " in line and not line.startswith("#"))
        assert len(fields["source_sha256"]) == 64
        assert float(fields["traffic_bytes_per_launch"]) > 0
        found += 1
    assert found >= 1


def test_source_digest_ignores_comments_only():
    """The digest covers code, not comments: a comment edit keeps a traffic
    summary valid, a code edit voids it; string literals count as code."""
    a = 'int f(int x) {  // one\n    /* two\n       lines */ return x + 1;\n}\nconst char *s = "a // b";\n'
    b = 'int f(int x) {\n    return x + 1;  // changed comment\n}\n\nconst char *s = "a // b";\n'
    c = 'int f(int x) {\n    return x + 2;\n}\nconst char *s = "a // b";\n'
    d = 'int f(int x) {\n    return x + 1;\n}\nconst char *s = "a // c";\n'
    assert bench.code_only(a) == bench.code_only(b)
    assert bench.code_only(a) != bench.code_only(c)
    assert bench.code_only(a) != bench.code_only(d)
    assert "return x + 1;" in bench.code_only(a) and "one" not in bench.code_only(a)
