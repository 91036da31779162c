"""Lazy deletes (SIVF_DELETE_LAZY, the paper's validity-bitmap eviction): a
delete clears a bit and moves nothing, inserts publish their slots, searches
skip dead slots, and compaction reclaims them later.  Membership and every
search equal the oracle's at all times (the oracle deletes at once); a search
that starts after a delete has completed never returns the deleted id, also
when searches and deletes run at the same time on two streams (Theorem 3)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2601_11808_amd as sivf
from tests.gpu_common import compare_results, say
from tests.invariants import check_dump, membership_of, same_membership

pytestmark = pytest.mark.gpu


def _pair(d, nlist, cent, metric, C, num_slabs, cap, **kw):
    ix = sivf.Index(d, nlist, cent, metric=metric, slab_capacity=C, num_slabs=num_slabs, id_capacity=cap,
                    delete_mode=sivf.DELETE_LAZY, **kw)
    ref = oracle.OracleIndex(d, nlist, cent, metric, C, num_slabs, cap)
    return ix, ref


def _check(ix, ref, C, num_slabs, q, k, nprobe, lazy=True):
    d = ix.dump()
    check_dump(d, C, num_slabs, lazy=lazy)
    assert same_membership(membership_of(d), ref.membership())
    assert ix.stats()["live"] == ref.live()
    for tile in ((8, 16) if ix.cfg.storage == 0 and ix.cfg.dim <= 256 and ix.cfg.max_k <= 64 else (8,)):
        ix.set_search_schedule(tile, 14, 0)
        gd, gl = ix.search(q, k, nprobe)
        assert ix.sync() == 0
        st, rd, rl = ref.search(q, k, nprobe)
        compare_results(gd.cpu().numpy(), gl.cpu().numpy(), rd, rl)


@pytest.mark.parametrize("C,d,metric,seed", [(64, 32, 0, 1), (32, 17, 1, 2), (128, 24, 0, 3), (16, 40, 0, 4)])
def test_lazy_random_ops_vs_oracle(C, d, metric, seed):
    rng = np.random.default_rng([seed, 51])
    nlist, cap = 11, 4000
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    num_slabs = 4000   # room for every dead slot between compactions
    ix, ref = _pair(d, nlist, cent, metric, C, num_slabs, cap, max_batch=1024, max_queries=64, max_k=40,
                    max_nprobe=16)
    q = rng.standard_normal((50, d)).astype(np.float32)
    for step in range(30):
        n = int(rng.integers(0, 700))
        ids = rng.integers(0, cap, n)
        x = rng.standard_normal((n, d)).astype(np.float32)
        if n > 10:
            x[:5] = x[5:10]
        ix.add(x, ids)
        assert ix.sync() == 0
        assert ref.add(x, ids) == 0
        rm = rng.integers(0, cap, int(rng.integers(0, 600)))
        nr = ix.remove(rm)
        assert ix.sync() == 0
        st, rn = ref.remove(rm)
        assert int(nr.item()) == rn
        _check(ix, ref, C, num_slabs, q, int(rng.integers(1, 41)), int(rng.integers(1, 12)))
        if step % 7 == 6:
            frac = float(rng.choice([0.0, 0.2, 0.6]))
            ix.compact(frac)
            assert ix.sync() == 0
            _check(ix, ref, C, num_slabs, q, 10, 5)
    while int(ix.compact(0.0).item()) > 0:
        pass
    assert ix.sync() == 0
    _check(ix, ref, C, num_slabs, q, 10, 11, lazy=False)   # fully compacted: dense lists again
    assert ix.stats()["used_slabs"] == ref.used_slabs()
    say(f"  C={C} d={d} metric={metric}: 30 rounds identical to the oracle; compacted to dense")


def test_lazy_compaction_budget_and_space():
    """A compaction call reclaims at most max_batch dead slots (one list may be
    compacted in part); dead slots hold their space until then."""
    rng = np.random.default_rng(52)
    d, nlist, C = 16, 3, 32
    cent = (rng.standard_normal((nlist, d)) * 5).astype(np.float32)
    num_slabs = 900
    ix, ref = _pair(d, nlist, cent, 0, C, num_slabs, 30000, max_batch=1000, max_queries=32, max_k=16,
                    max_nprobe=3)
    x = (cent[rng.integers(0, nlist, 20000)] + rng.standard_normal((20000, d))).astype(np.float32)
    for s in range(0, 20000, 1000):
        ix.add(x[s:s + 1000], np.arange(s, s + 1000))
        assert ref.add(x[s:s + 1000], np.arange(s, s + 1000)) == 0
    assert ix.sync() == 0
    used0 = ix.stats()["used_slabs"]
    rm = rng.permutation(20000)[:9000]
    for s in range(0, 9000, 1000):
        ix.remove(rm[s:s + 1000])
        assert ref.remove(rm[s:s + 1000])[0] == 0
    assert ix.sync() == 0
    st = ix.stats()
    assert st["live"] == 11000 and st["used_slabs"] == used0   # nothing reclaimed yet
    q = rng.standard_normal((32, d)).astype(np.float32)
    _check(ix, ref, C, num_slabs, q, 16, 3)
    calls = 0
    while True:
        n = int(ix.compact(0.0).item())
        assert ix.sync() == 0
        if n == 0:
            break
        assert n <= 1000
        calls += 1
        _check(ix, ref, C, num_slabs, q, 16, 3)
    assert calls == 9
    _check(ix, ref, C, num_slabs, q, 16, 3, lazy=False)
    assert ix.stats()["used_slabs"] == ref.used_slabs()
    say(f"  9,000 dead slots reclaimed in {calls} calls of at most 1,000; slabs {used0} -> {ref.used_slabs()}")


def test_lazy_concurrent_searches_never_return_deleted():
    """Searches on one stream and lazy deletes on another run at the same
    time.  A search enqueued after a delete completed (stream wait on the
    delete's event) equals the oracle after the delete; a search running
    alongside returns only ids live when it started, and where neither its
    result nor the oracle's involves the ids being deleted, it equals the
    oracle exactly (Theorem 3: deleted ids are never returned afterwards)."""
    rng = np.random.default_rng(53)
    d, nlist, C, n = 32, 64, 64, 200_000
    cent = (rng.standard_normal((nlist, d)) * 4).astype(np.float32)
    ix, ref = _pair(d, nlist, cent, 0, C, n // C + 2 * nlist + 64, n, max_batch=65536, max_queries=2048,
                    max_k=16, max_nprobe=16)
    x = (cent[rng.integers(0, nlist, n)] + rng.standard_normal((n, d))).astype(np.float32)
    for s in range(0, n, 65536):
        ix.add(x[s:s + 65536], np.arange(s, min(n, s + 65536)))
    assert ix.sync() == 0
    assert ref.add(x, np.arange(n)) == 0
    live = np.ones(n, bool)
    dev = ix.device
    s_search, s_del = torch.cuda.Stream(dev), torch.cuda.Stream(dev)
    qh = (cent[rng.integers(0, nlist, 2048)] + rng.standard_normal((2048, d))).astype(np.float32)
    q = torch.from_numpy(qh).to(dev)
    torch.cuda.synchronize()
    overlapped = 0
    for r in range(8):
        gone = rng.choice(np.flatnonzero(live), 3000, replace=False)
        gone_d = torch.from_numpy(gone).to(dev)
        torch.cuda.synchronize()
        st0, rd0, rl0 = ref.search(qh, 10, 8)
        with torch.cuda.stream(s_search):
            da, la = ix.search(q, 10, 8, stream=s_search)      # runs alongside the delete
        with torch.cuda.stream(s_del):
            nrem = ix.remove(gone_d, stream=s_del)
            ev = torch.cuda.Event()
            ev.record(s_del)
        with torch.cuda.stream(s_search):
            s_search.wait_event(ev)
            db, lb = ix.search(q, 10, 8, stream=s_search)      # starts after the delete completed
        torch.cuda.synchronize()
        assert ix.sync() == 0
        assert int(nrem.item()) == 3000
        assert ref.remove(gone)[0] == 0
        st1, rd1, rl1 = ref.search(qh, 10, 8)
        compare_results(db.cpu().numpy(), lb.cpu().numpy(), rd1, rl1)
        la = la.cpu().numpy()
        ok = la[la >= 0]
        assert live[ok].all(), "a concurrent search returned an id deleted before it started"
        gs = set(gone.tolist())
        touched = np.array([bool(gs & set(a.tolist())) or bool(gs & set(b.tolist())) for a, b in zip(la, rl0)])
        overlapped += int(touched.sum())
        compare_results(da.cpu().numpy()[~touched], la[~touched], rd0[~touched], rl0[~touched])
        live[gone] = False
    _check(ix, ref, C, ix.cfg.num_slabs, qh[:64], 10, 8)
    say(f"  8 rounds of 3,000 concurrent deletes; {overlapped} query results touched by a concurrent delete")


def test_lazy_reduced_precision_and_checkpoint(tmp_path):
    """bf16 slabs with lazy deletes: results never hold a deleted id and their
    distances are the exact FP32 ones; a checkpoint keeps only live entries."""
    rng = np.random.default_rng(54)
    d, nlist, C, n = 48, 16, 64, 20000
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    ix, ref = _pair(d, nlist, cent, 0, C, 2 * n // C + 4 * nlist, n, max_batch=8192, max_queries=256, max_k=10,
                    max_nprobe=16, storage=sivf.BF16, rerank_factor=4)
    x = rng.standard_normal((n, d)).astype(np.float32)
    for s in range(0, n, 8192):
        ix.add(x[s:s + 8192], np.arange(s, min(n, s + 8192)))
    assert ref.add(x, np.arange(n)) == 0
    gone = rng.permutation(n)[:7000]
    ix.remove(gone)
    assert ix.sync() == 0
    assert ref.remove(gone)[0] == 0
    q = rng.standard_normal((256, d)).astype(np.float32)
    gd, gl = ix.search(q, 10, 6)
    assert ix.sync() == 0
    gl, gd = gl.cpu().numpy(), gd.cpu().numpy()
    assert not np.isin(gl, gone).any()
    st, rd, rl = ref.search(q, 10, 6)
    hit = np.mean([len(set(a) & set(b)) / 10 for a, b in zip(gl, rl)])
    assert hit >= 0.95, hit
    path = tmp_path / "lazy.sivf"
    ix.save(path)
    cfg, live = sivf.checkpoint_config(path)
    assert live == n - 7000
    jx = sivf.Index.load(path)
    assert same_membership(jx.membership(), ref.membership())
    jd, jl = jx.search(q, 10, 6)
    assert jx.sync() == 0
    np.testing.assert_array_equal(jl.cpu().numpy(), gl)
    say(f"  bf16 lazy: recall {hit:.3f} against the FP32 oracle; checkpoint holds {live} live entries")
