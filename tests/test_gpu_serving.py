"""Serving form: requests submitted through the overlapping server give, for
every search, exactly the result of running the same request sequence one
call at a time (and the oracle's); the final membership matches too."""
import numpy as np
import pytest
import torch

import oracle
import paper_2601_11808_amd as sivf
import workloads
from tests.gpu_common import compare_results, say
from tests.invariants import check_dump, membership_of, same_membership

pytestmark = pytest.mark.gpu


def _requests(w, rng, n_req, n_base):
    """A mixed stream: searches (varied sizes and nprobe), inserts of fresh
    ids, removes of live ids (oldest or random)."""
    live = list(range(n_base))
    next_id = n_base
    reqs = []
    for _ in range(n_req):
        r = rng.random()
        if r < 0.5:
            nq = int(rng.integers(1, 65))
            reqs.append(("search", w.queries(nq, tag=int(rng.integers(1 << 30))), int(rng.integers(1, 17))))
        elif r < 0.8:
            n = int(rng.integers(1, 400))
            xb, _ = w.stream_batch(int(rng.integers(1, 1 << 20)), n)
            reqs.append(("add", xb, np.arange(next_id, next_id + n, dtype=np.int64)))
            live += list(range(next_id, next_id + n))
            next_id += n
        else:
            n = min(int(rng.integers(1, 500)), len(live))
            if rng.random() < 0.5:
                gone = sorted(live)[:n]
            else:
                gone = list(rng.choice(np.asarray(live), size=n, replace=False))
            s = set(gone)
            live = [u for u in live if u not in s]
            reqs.append(("remove", np.asarray(gone, np.int64)))
    return reqs, next_id


@pytest.mark.parametrize("storage", [0, 1])
def test_server_mix_equals_serial(storage):
    w = workloads.tiny()
    x, ids = w.base()
    rng = np.random.default_rng(77)
    reqs, cap = _requests(w, rng, 120, x.shape[0])
    kw = dict(metric=w.metric, slab_capacity=w.slab, num_slabs=1200, id_capacity=cap + 16, max_batch=4096,
              max_queries=64, max_k=16, max_nprobe=16, storage=storage, rerank_factor=4 if storage else 0)
    a = sivf.Index(w.dim, w.nlist, w.centroids, **kw)   # served
    b = sivf.Index(w.dim, w.nlist, w.centroids, **kw)   # one call at a time
    ref = oracle.OracleIndex(w.dim, w.nlist, w.centroids, w.metric, w.slab, 1200, cap + 16)
    for ix in (a, b):
        ix.add(x, ids)
        assert ix.sync() == 0
    assert ref.add(x, ids) == 0
    srv = sivf.Server(a)
    tickets = []
    for r in reqs:                      # submit everything at once: maximum overlap
        if r[0] == "search":
            t, d, l = srv.search(r[1], 10, r[2])
            waited = 0
            while t is None:            # search slots full: let earlier requests finish, then resubmit
                assert waited < len(tickets), "search refused with nothing in flight"
                srv.wait(tickets[waited][0])
                waited += 1
                t, d, l = srv.search(r[1], 10, r[2], out=(d, l))
            tickets.append((t, d, l))
        elif r[0] == "add":
            t = srv.add(r[1], r[2])
            waited = 0
            while t is None:            # refused: let earlier requests finish, then resubmit
                assert waited < len(tickets), "admission refused with nothing in flight"
                srv.wait(tickets[waited][0])
                waited += 1
                t = srv.add(r[1], r[2])
            tickets.append((t,))
        else:
            t, nrem = srv.remove(r[1])
            tickets.append((t, nrem))
    for tk in tickets:
        srv.wait(tk[0])
    nb, nreq = srv.batches()
    srv.close()
    assert a.sync() == 0
    nsearch = 0
    for r, tk in zip(reqs, tickets):
        if r[0] == "search":
            gd, gl = b.search(r[1], 10, r[2])
            assert b.sync() == 0
            np.testing.assert_array_equal(tk[2].cpu().numpy(), gl.cpu().numpy())
            np.testing.assert_array_equal(tk[1].cpu().numpy(), gd.cpu().numpy())
            if storage == 0:
                st, rd, rl = ref.search(r[1], 10, r[2])
                compare_results(tk[1].cpu().numpy(), tk[2].cpu().numpy(), rd, rl)
            nsearch += 1
        elif r[0] == "add":
            b.add(r[1], r[2])
            assert b.sync() == 0
            assert ref.add(r[1], r[2]) == 0
        else:
            nr = b.remove(r[1])
            assert b.sync() == 0
            st, rn = ref.remove(r[1])
            assert int(tk[1].item()) == int(nr.item()) == rn
    da, db = a.dump(), b.dump()
    check_dump(da, w.slab, 1200)
    assert same_membership(membership_of(da), membership_of(db))
    assert same_membership(membership_of(da), ref.membership())
    assert nreq == nsearch and nb <= nsearch
    say(f"  {len(reqs)} requests ({nsearch} searches in {nb} batches) identical in the mix and one at a time")


@pytest.mark.parametrize("storage", [0, 1])
def test_server_coalesces_searches(storage):
    """Searches submitted while a search batch is in flight join one batch:
    a run of 60 searches (sizes 1..40, k 1..16, nprobe 1..16) goes out in
    fewer launches than requests, rows past the batch slots start a new batch,
    and every result equals the same search run alone (and the oracle)."""
    w = workloads.tiny()
    x, ids = w.base()
    rng = np.random.default_rng(78)
    kw = dict(metric=w.metric, slab_capacity=w.slab, num_slabs=400, id_capacity=8192, max_batch=4096,
              max_queries=128, max_k=16, max_nprobe=16, storage=storage, rerank_factor=4 if storage else 0)
    a = sivf.Index(w.dim, w.nlist, w.centroids, **kw)
    a.add(x, ids)
    assert a.sync() == 0
    ref = oracle.OracleIndex(w.dim, w.nlist, w.centroids, w.metric, w.slab, 400, 8192)
    assert ref.add(x, ids) == 0
    reqs = [(w.queries(int(rng.integers(1, 41)), tag=1000 + i), int(rng.integers(1, 17)), int(rng.integers(1, 17)))
            for i in range(60)]
    srv = sivf.Server(a)
    out = []
    for q, k, npb in reqs:
        t, d, l = srv.search(q, k, npb)
        while t is None:
            srv.wait(out[0][0] if out else 0)
            for o in out:
                srv.poll(o[0])
            t, d, l = srv.search(q, k, npb, out=(d, l))
        out.append((t, d, l))
    for o in out:
        srv.wait(o[0])
    nb, nreq = srv.batches()
    srv.close()
    assert a.sync() == 0
    assert nreq == 60 and nb < 60, (nb, nreq)
    for (q, k, npb), (t, d, l) in zip(reqs, out):
        gd, gl = a.search(q, k, npb)
        assert a.sync() == 0
        np.testing.assert_array_equal(l.cpu().numpy(), gl.cpu().numpy())
        np.testing.assert_array_equal(d.cpu().numpy(), gd.cpu().numpy())
        if storage == 0:
            st, rd, rl = ref.search(q, k, npb)
            compare_results(d.cpu().numpy(), l.cpu().numpy(), rd, rl)
    say(f"  60 searches in {nb} batches, each identical to its alone result")


def test_server_admission_and_live_ids():
    w = workloads.tiny()
    x, ids = w.base()
    a = sivf.Index(w.dim, w.nlist, w.centroids, metric=0, slab_capacity=32, num_slabs=160, id_capacity=9000,
                   max_batch=4096, max_queries=64, max_k=16, max_nprobe=16)
    a.add(x, ids)
    assert a.sync() == 0
    srv = sivf.Server(a)
    free, res = srv.free_slabs()
    assert free == 160 - a.stats()["used_slabs"] and res == 0
    # an insert too large for the free slabs is refused on the host
    xb, idb = w.stream_batch(1, 3000)
    assert srv.add(xb, idb + 1000) is None
    # a live id fails the call on the device and changes nothing
    before = membership_of(a.dump())
    t = srv.add(x[:3], np.array([0, 1, 2]))
    srv.wait(t)
    srv.close()
    assert a.sync() == sivf.ERR_LIVE_ID
    assert same_membership(membership_of(a.dump()), before)
    # ... and leaves no partial counts behind: later calls still match the oracle
    ref = oracle.OracleIndex(w.dim, w.nlist, w.centroids, 0, 32, 160, 9000)
    assert ref.add(x, ids) == 0
    xb, idb = w.stream_batch(2, 300)
    a.add(xb, idb)
    assert a.sync() == 0
    assert ref.add(xb, idb) == 0
    check_dump(a.dump(), 32, 160)
    assert same_membership(membership_of(a.dump()), ref.membership())
    q = w.queries()
    gd, gl = a.search(q, 10, 4)
    assert a.sync() == 0
    st, rd, rl = ref.search(q, 10, 4)
    compare_results(gd.cpu().numpy(), gl.cpu().numpy(), rd, rl)


def test_non_finite_vector_rejects_batch():
    w = workloads.tiny()
    x, ids = w.base()
    a = sivf.Index(w.dim, w.nlist, w.centroids, metric=0, slab_capacity=32, num_slabs=400, id_capacity=9000,
                   max_batch=4096, max_queries=64, max_k=16, max_nprobe=16)
    a.add(x, ids)
    assert a.sync() == 0
    before = membership_of(a.dump())
    xb, idb = w.stream_batch(1, 100)
    for bad in (np.nan, np.inf, -np.inf):
        xx = xb.copy()
        xx[37, 5] = bad
        a.add(xx, idb)
        assert a.sync() == sivf.ERR_ARG
        assert same_membership(membership_of(a.dump()), before)
    a.add(xb, idb)
    assert a.sync() == 0
    ref = oracle.OracleIndex(w.dim, w.nlist, w.centroids, 0, 32, 400, 9000)
    assert ref.add(x, ids) == 0 and ref.add(xb, idb) == 0
    check_dump(a.dump(), 32, 400)
    assert same_membership(membership_of(a.dump()), ref.membership())
