"""GPU: the serving loop (kmp_server_*).  Jobs of mixed type, size and k are
submitted over time from a separate thread; every result must equal the
oracle's partition of that job alone (bit-exact), and the same job run alone
through kmp_partition_ex must give the same output as in the mix."""
import ctypes
import sys
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2105_02022_amd import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kmp():
    import paper_2105_02022_amd as k
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    k.library()
    return k


def small_serving_jobs(count, seed):
    """The serving recipe at small sizes: n log-uniform in [2^9, 2^13], k over {2, 8, 64, 512, 4096}."""
    jobs = []
    for typ, n, k, s in gen.serving_jobs(count, seed=seed, lo=9, hi=13):
        if typ == "rmat":
            g = gen.rmat(max(9, int(round(np.log2(n)))), 8 << max(9, int(round(np.log2(n)))), seed=s)
        elif typ == "grid":
            a = int(np.sqrt(n))
            g = gen.grid(a, n // a)
        else:
            g = gen.rgg(n, 8.0, seed=s)
        jobs.append((f"{typ}{g.n}_k{k}_s{s}", g, k, s))
    return jobs


def _device_jobs(kmp, specs):
    out = []
    for name, g, k, s in specs:
        xadj, adjncy, vwgt, adjwgt = kmp.to_device(g, "cuda")
        out.append(dict(name=name, g=g, xadj=xadj, adjncy=adjncy, vwgt=vwgt, adjwgt=adjwgt, k=k, epsilon=0.03,
                        seed=s, out=torch.full((g.n,), -5, dtype=torch.int32, device="cuda")))
    return out


def _check(job, res):
    ref = oracle.partition(job["g"], job["k"], job["epsilon"], job["seed"])
    assert res["status"] == ref.status, job["name"]
    assert np.array_equal(job["out"].cpu().numpy(), ref.part), job["name"]
    assert res["cut"] == ref.stats["cut"], job["name"]
    assert res["level_n"] == ref.stats["level_n"], job["name"]


def test_server_jobs_over_time_match_oracle(kmp):
    jobs = _device_jobs(kmp, small_serving_jobs(30, seed=7))
    say(f"[server] {len(jobs)} jobs, sum n = {sum(j['g'].n for j in jobs)}")
    ids = [None] * len(jobs)
    with kmp.Server(8 << 30, workers=2) as srv:
        def submitter():
            rng = np.random.default_rng(3)
            for i, j in enumerate(jobs):
                time.sleep(float(rng.exponential(0.002)))
                ids[i] = srv.submit(j)
        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
    say(f"  batches {st['batches']}, largest {st['max_batch_jobs']}, p50 latency "
        f"{np.percentile([r['latency_ms'] for r in res], 50):.1f} ms")
    assert st["jobs_done"] == len(jobs) and st["jobs_submitted"] == len(jobs)
    assert all(r["latency_ms"] > 0 for r in res)
    for j, r in zip(jobs, res):
        _check(j, r)
    # the same jobs alone give the same outputs
    for j in jobs[::5]:
        rc, alone, _ = kmp.kmp_partition_ex(j["xadj"], j["adjncy"], j["vwgt"], j["adjwgt"], j["k"], j["epsilon"],
                                            j["seed"])
        assert torch.equal(alone, j["out"]), j["name"]


def test_server_budget_admission_and_polling(kmp):
    """A budget below every job's footprint runs the jobs one at a time; poll reports pending / done."""
    jobs = _device_jobs(kmp, small_serving_jobs(8, seed=11))
    with kmp.Server(1, workers=2) as srv:
        ids = [srv.submit(j) for j in jobs]
        res = {}
        t_end = time.time() + 120
        while len(res) < len(ids) and time.time() < t_end:
            for i in ids:
                if i not in res:
                    r = srv.poll(i)
                    if r is not None:
                        res[i] = r
            time.sleep(0.001)
        st = srv.stats()
        with pytest.raises(KeyError):
            srv.poll(ids[0])  # results are taken once
    assert len(res) == len(ids)
    assert st["max_batch_jobs"] == 1 and st["batches"] == len(jobs)
    for j, i in zip(jobs, ids):
        _check(j, res[i])


def test_server_destroy_finishes_submitted_jobs(kmp):
    jobs = _device_jobs(kmp, small_serving_jobs(10, seed=5))
    srv = kmp.Server(8 << 30, workers=3)
    for j in jobs:
        srv.submit(j)
    srv.close()  # returns once every submitted job is done
    for j in jobs:
        ref = oracle.partition(j["g"], j["k"], j["epsilon"], j["seed"])
        assert np.array_equal(j["out"].cpu().numpy(), ref.part), j["name"]


def test_server_with_ip_options_matches_oracle(kmp):
    """kmp_server_set_options: served jobs get 2-way FM and the IP pool, as in the oracle."""
    jobs = _device_jobs(kmp, small_serving_jobs(8, seed=11))
    say(f"[server options] {len(jobs)} jobs, fm_passes=2, ip_pool=1")
    with kmp.Server(8 << 30, workers=2) as srv:
        o = kmp.KmpOptions()
        o.fm_passes = 17
        assert kmp.library().kmp_server_set_options(srv._h, ctypes.byref(o)) == kmp.KMP_EINVAL
        assert srv.set_options(fm_passes=2, ip_pool=True) == kmp.KMP_OK
        ids = [srv.submit(j) for j in jobs]
        res = [srv.wait(i) for i in ids]
    for j, r in zip(jobs, res):
        ref = oracle.partition(j["g"], j["k"], j["epsilon"], j["seed"], fm_passes=2, pool=True)
        assert r["status"] == ref.status, j["name"]
        assert np.array_equal(j["out"].cpu().numpy(), ref.part), j["name"]
        assert r["cut"] == ref.stats["cut"], j["name"]


def test_server_options_bound_at_submission(kmp):
    """Options changed while earlier jobs still wait apply only to jobs submitted after the change: each
    result equals the oracle's with the options that were current when that job was submitted."""
    specs = small_serving_jobs(12, seed=13)
    jobs = _device_jobs(kmp, specs)
    with kmp.Server(8 << 30, workers=1) as srv:
        ids, opts = [], []
        for i, j in enumerate(jobs):
            if i % 4 == 0:
                o = [(0, False), (2, True), (1, False)][(i // 4) % 3]
                assert srv.set_options(fm_passes=o[0], ip_pool=o[1]) == kmp.KMP_OK
            ids.append(srv.submit(j))
            opts.append(o)
        res = [srv.wait(i) for i in ids]
    for j, r, (p, q) in zip(jobs, res, opts):
        ref = oracle.partition(j["g"], j["k"], j["epsilon"], j["seed"], fm_passes=p, pool=q)
        assert r["status"] == ref.status, j["name"]
        assert np.array_equal(j["out"].cpu().numpy(), ref.part), (j["name"], p, q)
        assert r["cut"] == ref.stats["cut"], j["name"]


def test_server_two_waiters_on_one_job(kmp):
    """Two threads wait on the same job: one receives the result, the other an error, and nothing
    crashes."""
    jobs = _device_jobs(kmp, small_serving_jobs(3, seed=17))
    with kmp.Server(8 << 30, workers=1) as srv:
        ids = [srv.submit(j) for j in jobs]
        got, errs = [], []

        def waiter():
            try:
                got.append(srv.wait(ids[-1]))
            except KeyError:
                errs.append(1)

        ths = [threading.Thread(target=waiter) for _ in range(2)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        for i in ids[:-1]:
            srv.wait(i)
    assert len(got) == 1 and len(errs) == 1
    _check(jobs[-1], got[0])
