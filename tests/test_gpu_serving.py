"""Serving (continuous batching) through the C ABI.

Every request's result in a mixed, overlapping request stream must equal the
same extraction run alone (frw_extract) up to fp32 summation order, and the
admitted device footprint must stay within the memory budget.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_09730_amd as lib
    lib.mw_init(0)
    return lib


def _requests():
    rng = np.random.Generator(np.random.PCG64(11))
    reqs = []
    c2 = W.c2_structure()
    for i in range(6):
        reqs.append((c2, i % 4, int(rng.integers(100000, 600000)), 100 + i))
    for K in (6, 12, 24, 48):
        st = W.request_structure(K, rng)
        reqs.append((st, int(rng.integers(0, st.n_nets)), int(rng.integers(100000, 900000)), 200 + K))
    return reqs


def _same(a, b):
    scale = np.abs(b["row"]).max()
    return np.all(np.abs(a["row"] - b["row"]) <= 1e-6 * np.abs(b["row"]) + 1e-9 * scale)


def test_mix_equals_alone(mw):
    reqs = _requests()
    srv = mw.Server(4 << 30)
    tickets = [srv.submit(st, m, b, seed) for st, m, b, seed in reqs]
    results = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    print("server stats", stats)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["max_concurrent"] > 1  # requests overlapped on the device
    assert stats["max_resident_bytes"] <= 4 << 30
    for (st, m, b, seed), r in zip(reqs, results):
        alone = mw.frw_extract(st, m, b, seed=seed)
        assert r["walks"] == b
        assert _same(r, alone), (r["row"], alone["row"])
        assert np.allclose(r["se"], alone["se"], rtol=1e-4, atol=1e-12)
        assert r["latency"] > 0


def test_admission_respects_budget(mw):
    reqs = _requests()[:6]
    # footprint of one of these requests (all on the same structure)
    srv = mw.Server(1 << 30)
    srv.wait(srv.submit(*reqs[0]))
    one = srv.stats()["max_resident_bytes"]
    srv.close()
    # room for two requests at a time
    budget = int(2.5 * one)
    srv = mw.Server(budget)
    tickets = [srv.submit(st, m, b, seed) for st, m, b, seed in reqs]
    results = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    print("small-budget stats", stats, "one", one)
    assert stats["completed"] == len(reqs)
    assert stats["max_resident_bytes"] <= budget
    assert stats["max_concurrent"] == 2
    for (st, m, b, seed), r in zip(reqs, results):
        alone = mw.frw_extract(st, m, b, seed=seed)
        assert _same(r, alone)


def test_oversized_request_is_rejected(mw):
    srv = mw.Server(16 << 10)
    t = srv.submit(W.c2_structure(), 0, 100000, 1)
    with pytest.raises(mw.MWError) as e:
        srv.wait(t, timeout=60)
    assert e.value.status == mw.MW_ELIMIT
    srv.close()


def test_target_stops_early(mw):
    srv = mw.Server(2 << 30, target_rel_3sigma=0.05)
    t = srv.submit(W.c2_structure(), 0, 50000000, 7)
    r = srv.wait(t)
    srv.close()
    assert r["walks"] < 50000000
    assert 3 * r["se"][0] / r["row"][0] <= 0.05
