"""The GPU queue balancer's pass routine (csrc/pq_pass.h) built for the host
with AddressSanitizer and run pass by pass on the oracle's pin cases of the
queue balancer (paper Sec. 5.3 "Balancing"): every array is allocated at its
exact size, so an access outside one fails the run, and the result (part,
block weights, passes) must equal the oracle's O9b.  No GPU is needed."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen
from tests.test_oracle_pins_pq import _case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC) or shutil.which("g++") is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("pq") / "pq_host")
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
           "-I", os.path.join(ROOT, "paper_2105_02022_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "pq_host_harness.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def _run(exe, g, level, seed, part, wt, cap):
    n, m, nb = g.n, int(g.xadj[-1]), len(wt)
    buf = b"".join([np.array([n, m, nb, level], np.int32).tobytes(), np.array([seed], np.uint64).tobytes(),
                    np.array([g.vwgt is not None, g.adjwgt is not None], np.int32).tobytes(),
                    np.asarray(g.xadj, np.int32).tobytes(), np.asarray(g.adjncy, np.int32).tobytes(),
                    b"" if g.vwgt is None else np.asarray(g.vwgt, np.int32).tobytes(),
                    b"" if g.adjwgt is None else np.asarray(g.adjwgt, np.int32).tobytes(),
                    np.asarray(part, np.int32).tobytes(), np.asarray(wt, np.int64).tobytes(),
                    np.asarray(cap, np.int64).tobytes()])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    r = subprocess.run([exe], input=buf, capture_output=True, env=env)
    assert r.returncode == 0, r.stderr.decode()[-3000:]
    o = r.stdout
    passes, full = np.frombuffer(o[:8], np.int32)
    got_part = np.frombuffer(o[8:8 + 4 * n], np.int32)
    got_wt = np.frombuffer(o[8 + 4 * n:8 + 4 * n + 8 * nb], np.int64)
    return int(passes), int(full), got_part, got_wt


@pytest.mark.parametrize("seed", list(range(12)) + [33, 54, 66, 81, 144, 151, 160, 166, 175, 223])
def test_pass_routine_equals_oracle(harness, seed):
    g, part, wt, cap = _case(seed, max_vw=1 + seed % 4)
    exp_part, exp_wt, exp_p = oracle.balance_pq(g, seed % 3, 900 + seed, part, wt, cap)
    p, full, got_part, got_wt = _run(harness, g, seed % 3, 900 + seed, part, wt, cap)
    assert full == 0
    assert p == exp_p
    assert np.array_equal(got_part, exp_part)
    assert np.array_equal(got_wt, exp_wt)


@pytest.mark.parametrize("seed", range(3))
def test_pass_routine_larger_cases(harness, seed):
    g, part, wt, cap = _case(100 + seed, n=3000, nb=9, max_vw=5, iso=0.05)
    exp_part, exp_wt, exp_p = oracle.balance_pq(g, 1, seed, part, wt, cap)
    p, full, got_part, got_wt = _run(harness, g, 1, seed, part, wt, cap)
    assert full == 0 and p == exp_p
    assert np.array_equal(got_part, exp_part) and np.array_equal(got_wt, exp_wt)


def test_pass_routine_heavy_nodes_and_unit_weights(harness):
    """Weighted nodes on a random graph and a grid with unit weights, several blocks overloaded."""
    rng = np.random.default_rng(5)
    for g, nb in ((gen.random_graph(800, 6.0, 17, max_vw=30, max_ew=5), 7), (gen.grid(30, 40), 6)):
        c = np.ones(g.n, np.int64) if g.vwgt is None else np.asarray(g.vwgt, np.int64)
        part = rng.integers(0, nb, g.n).astype(np.int32)
        part[: g.n // 2] = rng.integers(0, 2, g.n // 2)
        wt = np.bincount(part, weights=c, minlength=nb).astype(np.int64)
        cap = np.full(nb, int(c.sum()) // nb + 3, np.int64)
        exp_part, exp_wt, exp_p = oracle.balance_pq(g, 2, 77, part, wt, cap)
        p, full, got_part, got_wt = _run(harness, g, 2, 77, part, wt, cap)
        assert full == 0 and p == exp_p and p >= 1
        assert np.array_equal(got_part, exp_part) and np.array_equal(got_wt, exp_wt)
