"""Precision form: bf16 / fp16 slabs scanned on MFMA with an exact fp32
re-rank of the best R * k candidates.

There is no bit parity for the approximate stage; what is checked:
  - membership and device invariants stay bit-exact (the coarse assignment is
    the exact FP32/FP64 path);
  - get_rows returns the exact fp32 rows (the shadow copy);
  - every returned distance equals the oracle's canonical FP32 distance of
    the returned id (the re-rank is exact), results are ordered by
    (distance, id) and never contain a deleted id;
  - recall@10 against the oracle's FP32 search at the same nprobe and against
    exact FP64 kNN, with stated thresholds (reported in the log).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_common import say
from tests.invariants import check_dump, membership_of, same_membership

pytestmark = pytest.mark.gpu


def _vmf(n, d, nlist, seed, kappa=50.0):
    rng = np.random.default_rng(seed)
    mu = rng.standard_normal((nlist, d))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    comp = rng.integers(0, nlist, n)
    x = mu[comp] + rng.standard_normal((n, d)) / np.sqrt(kappa)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return mu.astype(np.float32), x.astype(np.float32)


def _check_results(ref, q, gd, gl, k, nprobe, metric, removed=()):
    st, rd, rl = ref.search(q, k, nprobe)
    assert st == 0
    rec = []
    for i in range(q.shape[0]):
        ids = gl[i][gl[i] >= 0]
        for j, u in enumerate(ids):
            row = ref.row_of(int(u))
            assert row is not None, "returned id is not live"
            want = oracle.fine_dist(q[i], row, metric)
            assert gd[i, j].view(np.uint32) == np.float32(want).view(np.uint32), (i, j)
        # ordered by (distance, id): ascending L2, descending IP
        keys = [(float(gd[i, j]) if metric == 0 else -float(gd[i, j]), int(gl[i, j])) for j in range(len(ids))]
        assert keys == sorted(keys)
        assert not np.isin(ids, np.asarray(removed, np.int64)).any()
        rec.append(len(set(ids.tolist()) & set(rl[i][rl[i] >= 0].tolist())) / max(1, (rl[i] >= 0).sum()))
    return float(np.mean(rec))


@pytest.mark.parametrize("storage", [1, 2])
def test_precision_ip_vmf(storage):
    """Deep-like workload (d=96, unit vectors, inner product), slab 128."""
    import paper_2601_11808_amd as sivf
    d, nlist, n, k, R = 96, 64, 30000, 10, 4
    cent, x = _vmf(n + 4000, d, nlist, seed=[3, storage])
    q = x[n:n + 300]
    xb = x[:n]
    ix = sivf.Index(d, nlist, cent, metric=1, slab_capacity=128, num_slabs=600, id_capacity=n + 4000,
                    max_batch=8192, max_queries=512, max_k=16, max_nprobe=64, storage=storage, rerank_factor=R)
    ref = oracle.OracleIndex(d, nlist, cent, 1, 128, 600, n + 4000)
    for s in range(0, n, 8192):
        ix.add(xb[s:s + 8192], np.arange(s, min(n, s + 8192)))
    assert ix.sync() == 0
    assert ref.add(xb, np.arange(n)) == 0
    dmp = ix.dump()
    check_dump(dmp, 128, 600)
    assert same_membership(membership_of(dmp), ref.membership())
    rows = ix.get_rows(np.arange(0, n, 997)).cpu().numpy()
    np.testing.assert_array_equal(rows, xb[::997])
    for nprobe in (4, 16):
        gd, gl = ix.search(q, k, nprobe)
        r = _check_results(ref, q, gd.cpu().numpy(), gl.cpu().numpy(), k, nprobe, 1)
        say(f"  storage {storage} nprobe {nprobe}: recall@10 vs fp32 oracle search = {r:.4f}")
        assert r >= 0.95
    # window step: delete 3000, insert 3000 fresh
    rm = np.arange(0, 3000)
    ix.remove(rm)
    ix.add(x[n:n + 3000], np.arange(n, n + 3000))
    assert ix.sync() == 0
    ref.remove(rm)
    assert ref.add(x[n:n + 3000], np.arange(n, n + 3000)) == 0
    dmp = ix.dump()
    check_dump(dmp, 128, 600)
    assert same_membership(membership_of(dmp), ref.membership())
    gd, gl = ix.search(q, k, 16)
    r = _check_results(ref, q, gd.cpu().numpy(), gl.cpu().numpy(), k, 16, 1, removed=rm)
    kd, ki = ref.knn_exact(q, k)
    r64 = float(np.mean([len(set(gl.cpu().numpy()[i]) & set(ki[i])) / k for i in range(q.shape[0])]))
    say(f"  after a step: recall@10 vs fp32 oracle {r:.4f}, vs exact fp64 kNN {r64:.4f}")
    assert r >= 0.95


def test_precision_l2_tiny_bf16():
    """L2 with bf16 slabs on the tiny workload (slab 32, d=32)."""
    import paper_2601_11808_amd as sivf
    w = workloads.tiny()
    x, ids = w.base()
    q = w.queries()
    ix = sivf.Index(w.dim, w.nlist, w.centroids, metric=0, slab_capacity=32, num_slabs=400, id_capacity=8192,
                    max_batch=4096, max_queries=64, max_k=16, max_nprobe=16, storage=1, rerank_factor=4)
    ref = oracle.OracleIndex(w.dim, w.nlist, w.centroids, 0, 32, 400, 8192)
    ix.add(x, ids)
    assert ix.sync() == 0
    assert ref.add(x, ids) == 0
    for t in range(1, 4):
        xb, idb = w.stream_batch(t)
        ix.add(xb, idb)
        ref.add(xb, idb)
        gd, gl = ix.search(q, 10, 4)
        assert ix.sync() == 0
        r = _check_results(ref, q, gd.cpu().numpy(), gl.cpu().numpy(), 10, 4, 0)
        say(f"  step {t}: recall@10 vs fp32 oracle {r:.4f}")
        assert r >= 0.95
        ix.remove(w.oldest_ids(t))
        ref.remove(w.oldest_ids(t))
        assert ix.sync() == 0
        dmp = ix.dump()
        check_dump(dmp, 32, 400)
        assert same_membership(membership_of(dmp), ref.membership())
    # per-query k
    kpq = np.array([0, 1, 5, 10] * 16, np.int32)
    gd, gl = ix.search(q, 10, 4, k_per_query=kpq)
    gl = gl.cpu().numpy()
    for i in range(q.shape[0]):
        assert (gl[i, kpq[i]:] == -1).all() and (gl[i, :kpq[i]] >= 0).all()
