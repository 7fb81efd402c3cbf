"""Serving loop (plu_server_*): requests of uneven shapes arrive while
others run, are admitted by HBM footprint and batched continuously; each
result must be bit-identical to the same request solved alone (a single
call on the same data with the same seed)."""

import time

import numpy as np
import pytest

from tests.gpu_common import torch, have_gpu, handle, dev, host
from synth import lowrank_plus_noise, spectrum

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


def _requests(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m, n = (int(x) for x in rng.integers(400, 3000, 2))
        r = int(rng.integers(16, 100))
        A = lowrank_plus_noise(m, n, spectrum("exp", r, tau=r / 4), 7 * i + 1, 7 * i + 2,
                               1e-4 / np.sqrt(max(m, n)), 7 * i + 3)
        v = int(rng.integers(2, 6))
        if i % 2:
            b = 8
            l = min(16 * b, b * ((min(m, n) - 1) // b))
            out.append(dict(A=A, mode=1, eps=1e-3, b=b, l=l, v=v, seed=50 + i))
        else:
            out.append(dict(A=A, mode=0, k=r // 2, p_over=10, v=v, seed=50 + i))
    return out


def _alone(h, rq):
    A = dev(rq["A"])
    prec = rq.get("prec", 0)
    if rq["mode"] == 0:
        f = h.fixed_rank(A, rq["k"], rq["p_over"], rq["v"], seed=rq["seed"], prec=prec)
    else:
        f = h.fixed_precision(A, rq["eps"], rq["b"], l=rq["l"], v=rq["v"], seed=rq["seed"],
                              prec=prec)
    return f


def _footprint(h, rq):
    """Device bytes the server holds for a request: A, p, q, L and U at its
    capacity, and the workspace of its shape (each rounded to 256 bytes)."""
    m, n = rq["A"].shape
    l = rq["k"] + rq["p_over"] if rq["mode"] == 0 else rq["l"]
    cap = rq["k"] if rq["mode"] == 0 else l
    a = lambda x: (x + 255) // 256 * 256
    return (a(4 * m * n) + a(4 * m) + a(4 * n) + a(4 * m * cap) + a(4 * cap * n)
            + a(h.workspace_size(m, n, l)))


def _submit(srv, rq):
    kw = {k: v for k, v in rq.items() if k != "A"}
    return srv.submit(rq["A"], **kw)


def _check_same(res, f):
    assert res["status"] in (0, 1, 2)
    assert res["rank"] == f.rank
    assert np.array_equal(res["p"], host(f.p)) and np.array_equal(res["q"], host(f.q))
    assert np.array_equal(res["L"], host(f.L)) and np.array_equal(res["U"], host(f.U))


def test_server_mix_equals_alone():
    import paper_2002_07138_amd as plu
    reqs = _requests(11, 12)
    h = handle()
    alone = [_alone(h, rq) for rq in reqs]
    h.close()
    srv = plu.Server(0, hbm_budget_bytes=4 << 30, max_slots=16)
    tickets = []
    for i, rq in enumerate(reqs):
        tickets.append(_submit(srv, rq))
        if i % 4 == 3:
            time.sleep(0.002)      # later requests arrive while earlier ones run
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for res, f in zip(results, alone):
        _check_same(res, f)
    # latencies are measured from submission
    assert all(r["t_done"] >= r["t_admit"] >= r["t_submit"] for r in results)


def test_server_precision_forms_equal_alone():
    """Requests in the precision forms (BF16 / FP8 passes, with and without
    exact trailing passes) mixed with FP32 ones: a rounded-form request is
    issued whole on its lane (not merged), and every result equals the
    single call in the same form, bit for bit."""
    import paper_2002_07138_amd as plu
    forms = [1, 0, 2, 1 | 16, 2 | 32, 0, 1, 2]
    reqs = _requests(14, len(forms))
    for rq, f in zip(reqs, forms):
        rq["prec"] = f
    h = handle()
    alone = [_alone(h, rq) for rq in reqs]
    h.close()
    srv = plu.Server(0, hbm_budget_bytes=4 << 30, max_slots=16)
    tickets = []
    for i, rq in enumerate(reqs):
        tickets.append(_submit(srv, rq))
        if i % 3 == 2:
            time.sleep(0.002)
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for res, f in zip(results, alone):
        _check_same(res, f)


def test_server_rejects_fp64_indicator():
    import paper_2002_07138_amd as plu
    rq = _requests(15, 2)[1]
    srv = plu.Server(0, hbm_budget_bytes=1 << 30, max_slots=2)
    with pytest.raises(plu.PowerLUError) as e:
        _submit(srv, dict(rq, prec=128))
    srv.close()
    assert e.value.code == plu.PLU_ERR_NOT_IMPLEMENTED


def test_server_admission_by_budget():
    """A budget too small for all requests at once: some are admitted only
    after others completed and freed their memory; results are unchanged."""
    import paper_2002_07138_amd as plu
    reqs = _requests(12, 6)
    h = handle()
    alone = [_alone(h, rq) for rq in reqs]
    foot = [_footprint(h, rq) for rq in reqs]
    h.close()
    # room for the largest request and a tenth of it: never for all of them
    budget = int(1.1 * max(foot))
    assert sum(foot) > 2 * budget
    srv = plu.Server(0, hbm_budget_bytes=budget, max_slots=16)
    tickets = [_submit(srv, rq) for rq in reqs]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for res, f in zip(results, alone):
        _check_same(res, f)
    first_done = min(r["t_done"] for r in results)
    assert any(r["t_admit"] >= first_done for r in results)


def test_server_one_slot_serializes():
    import paper_2002_07138_amd as plu
    reqs = _requests(13, 3)
    h = handle()
    alone = [_alone(h, rq) for rq in reqs]
    h.close()
    srv = plu.Server(0, hbm_budget_bytes=2 << 30, max_slots=1)
    tickets = [_submit(srv, rq) for rq in reqs]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for res, f in zip(results, alone):
        _check_same(res, f)
    for a, b in zip(results, results[1:]):
        assert b["t_admit"] >= a["t_done"]


def test_server_strided_host_blocks():
    """Requests that are blocks of a larger host matrix (row stride above the
    block width): a stride up to 3x the width goes up as one contiguous span
    kept with its stride on the device, a wider one as a 2-D copy; either way
    each result equals the single call on a packed device copy, bit for bit."""
    import paper_2002_07138_amd as plu
    rng = np.random.default_rng(21)
    big = lowrank_plus_noise(2600, 3000, spectrum("exp", 60, tau=15.0), 31, 32, 1e-5, 33)
    reqs = []
    for i, (r0, c0, m, n) in enumerate([(10, 20, 1500, 1400),     # stride 3000 / 1400: span
                                        (500, 100, 900, 2600),     # span
                                        (0, 0, 2000, 700),         # 3000 / 700 > 3: 2-D copy
                                        (300, 2000, 1200, 900)]):  # span
        blk = big[r0:r0 + m, c0:c0 + n]
        if i % 2:
            b = 8
            l = min(16 * b, b * ((min(m, n) - 1) // b))
            reqs.append(dict(A=blk, mode=1, eps=1e-3, b=b, l=l, v=4, seed=90 + i))
        else:
            reqs.append(dict(A=blk, mode=0, k=20, p_over=10, v=3, seed=90 + i))
    h = handle()
    alone = [_alone(h, rq) for rq in reqs]
    h.close()
    srv = plu.Server(0, hbm_budget_bytes=2 << 30, max_slots=8)
    tickets = [_submit(srv, rq) for rq in reqs]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for res, f in zip(results, alone):
        _check_same(res, f)
