"""Host tier: whole lists offloaded to pinned host memory (the paper's planned
hierarchical storage, Sec. 6).  Searches, deletes, upserts, row reads and
checkpoints see cold entries exactly as device ones: membership and every
search equal the oracle's (which has no tiers) at all times, while lists move
to the tier, are deleted from there, refilled on the device and released."""
import numpy as np
import pytest

import oracle
import paper_2601_11808_amd as sivf
from tests.gpu_common import compare_results, say
from tests.invariants import check_dump, same_membership

pytestmark = pytest.mark.gpu


def _pair(d, nlist, cent, metric, C, num_slabs, cap, host_slabs, **kw):
    ix = sivf.Index(d, nlist, cent, metric=metric, slab_capacity=C, num_slabs=num_slabs, id_capacity=cap,
                    delete_mode=sivf.DELETE_LAZY, **kw)
    ix.tier_attach(host_slabs)
    ref = oracle.OracleIndex(d, nlist, cent, metric, C, 1 << 20, cap)
    return ix, ref


def _check(ix, ref, q, k, nprobe, tiles=(8, 16), kpq=None, npq=None):
    check_dump(ix.dump(), ix.C, ix.cfg.num_slabs, lazy=True, cold_ids=ix.tier_dump()["cold_ids"])
    assert same_membership(ix.membership(), ref.membership())
    assert ix.stats()["live"] == ref.live()
    st, rd, rl = ref.search(q, k, nprobe, k_per_query=kpq, nprobe_per_query=npq)
    for tile in tiles:
        ix.set_search_schedule(tile, 12, tile == 16)
        gd, gl = ix.search(q, k, nprobe, k_per_query=kpq, nprobe_per_query=npq)
        assert ix.sync() == 0
        compare_results(gd.cpu().numpy(), gl.cpu().numpy(), rd, rl)


@pytest.mark.parametrize("C,d,metric,seed", [(64, 32, 0, 1), (32, 17, 1, 2), (16, 40, 0, 3)])
def test_tier_random_ops_vs_oracle(C, d, metric, seed):
    rng = np.random.default_rng([seed, 61])
    nlist, cap = 13, 5000
    cent = (rng.standard_normal((nlist, d)) * 2).astype(np.float32)
    ix, ref = _pair(d, nlist, cent, metric, C, 3000, cap, 3000, max_batch=1024, max_queries=64, max_k=40,
                    max_nprobe=13)
    q = rng.standard_normal((60, d)).astype(np.float32)
    rows = {}
    for step in range(24):
        n = int(rng.integers(0, 600))
        ids = rng.integers(0, cap, n)                 # fresh ids and upserts, cold ones included
        x = rng.standard_normal((n, d)).astype(np.float32)
        if n > 10:
            x[:5] = x[5:10]                           # equal rows: exact distance ties
        ix.add(x, ids)
        assert ix.sync() == 0
        assert ref.add(x, ids) == 0
        for i, u in enumerate(ids.tolist()):
            rows[u] = x[i]
        rm = rng.integers(0, cap, int(rng.integers(0, 500)))
        nr = ix.remove(rm)
        assert ix.sync() == 0
        st, rn = ref.remove(rm)
        assert int(nr.item()) == rn
        for u in rm.tolist():
            rows.pop(u, None)
        if step % 3 == 1:                             # offload some lists (again, for some)
            lists = rng.choice(nlist, int(rng.integers(1, 6)), replace=False)
            ix.tier_offload(lists)
        if step % 5 == 4:
            ix.tier_reclaim()
        if step % 7 == 6:
            ix.compact(0.0)
            assert ix.sync() == 0
        _check(ix, ref, q, int(rng.integers(1, 41)), int(rng.integers(1, 14)))
        live = np.array(sorted(rows), np.int64)
        if live.shape[0]:
            pick = rng.choice(live, min(100, live.shape[0]), replace=False)
            got = ix.get_rows(pick).cpu().numpy()
            np.testing.assert_array_equal(got, np.stack([rows[u] for u in pick.tolist()]))
    ts = ix.tier_stats()
    assert ts["cold_positions"] > 0
    say(f"  C={C} d={d} metric={metric}: 24 rounds with offloads identical to the oracle; tier {ts}")


def test_tier_two_pass_k128_and_reclaim():
    """max_k 128 with per-query k across 64: the cold pass feeds both passes of
    the certified search.  Deleting every entry of the offloaded lists lets a
    reclaim release their cold segments."""
    rng = np.random.default_rng(62)
    d, nlist, C = 48, 9, 32
    cent = (rng.standard_normal((nlist, d)) * 5).astype(np.float32)
    ix, ref = _pair(d, nlist, cent, 0, C, 1200, 20000, 1200, max_batch=8192, max_queries=200, max_k=128,
                    max_nprobe=9)
    n = 16000
    x = (cent[rng.integers(0, nlist, n)] + rng.standard_normal((n, d))).astype(np.float32)
    x[100:150] = x[:50]
    for s in range(0, n, 8192):
        ix.add(x[s:s + 8192], np.arange(s, min(n, s + 8192)))
    assert ix.sync() == 0
    assert ref.add(x, np.arange(n)) == 0
    off = [0, 3, 4, 7]
    moved = ix.tier_offload(off)
    assert moved > 0 and ix.stats()["used_slabs"] < 1200
    q = (cent[rng.integers(0, nlist, 200)] + rng.standard_normal((200, d))).astype(np.float32)
    kpq = rng.choice([0, 1, 10, 64, 65, 100, 128], 200).astype(np.int32)
    npq = rng.integers(1, 10, 200).astype(np.int32)
    _check(ix, ref, q, 128, 9, tiles=(4, 8, 16), kpq=kpq, npq=npq)
    # more inserts land on the device part of the offloaded lists
    y = (cent[rng.integers(0, nlist, 3000)] + rng.standard_normal((3000, d))).astype(np.float32)
    ix.add(y, np.arange(n, n + 3000))
    assert ix.sync() == 0 and ref.add(y, np.arange(n, n + 3000)) == 0
    _check(ix, ref, q, 128, 9, tiles=(8, 16), kpq=kpq, npq=npq)
    # delete every cold entry: the cold segments die and are released
    cold = ix.tier_dump()["cold_ids"]
    cold = cold[cold >= 0]
    ix.remove(cold)
    assert ix.sync() == 0
    assert ref.remove(cold)[0] == 0
    assert ix.tier_stats()["cold_live"] == 0
    released = ix.tier_reclaim()
    ts = ix.tier_stats()
    assert released == moved and ts["cold_positions"] == 0 and ts["cold_used_slabs"] == 0
    _check(ix, ref, q, 100, 9, tiles=(8, 16))
    say(f"  {moved} positions offloaded, searched with k up to 128, deleted and released")


def test_tier_errors_and_checkpoint(tmp_path):
    rng = np.random.default_rng(63)
    d, nlist, C = 16, 5, 16
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    dense = sivf.Index(d, nlist, cent, slab_capacity=C, num_slabs=64, id_capacity=256, max_batch=256,
                       max_queries=8, max_k=8, max_nprobe=5)
    with pytest.raises(sivf.SivfError):
        dense.tier_attach(16)                         # compacting deletes: no tier
    ix, ref = _pair(d, nlist, cent, 0, C, 200, 3000, 40, max_batch=2048, max_queries=32, max_k=10, max_nprobe=5)
    with pytest.raises(sivf.SivfError):
        ix.tier_attach(40)                            # one tier per index
    x = rng.standard_normal((2000, d)).astype(np.float32)
    ix.add(x, np.arange(2000))
    assert ix.sync() == 0 and ref.add(x, np.arange(2000)) == 0
    with pytest.raises(sivf.SivfError):
        ix.tier_offload([0, 0])                       # repeated list
    with pytest.raises(sivf.SivfError):
        ix.tier_offload([nlist])                      # no such list
    before = ix.membership()
    with pytest.raises(sivf.SivfError) as e:
        ix.tier_offload(list(range(nlist)))           # 2000 positions need > 40 cold slabs
    assert e.value.status == sivf.ERR_NOSPACE
    assert same_membership(ix.membership(), before) and ix.tier_stats()["cold_positions"] == 0
    small = [int(np.argmin([len(before.get(l, [])) for l in range(nlist)]))]
    assert 0 < len(before[small[0]]) <= 40 * C
    assert ix.tier_offload(small) > 0
    ix.remove(np.arange(0, 2000, 3))
    assert ix.sync() == 0 and ref.remove(np.arange(0, 2000, 3))[0] == 0
    q = rng.standard_normal((32, d)).astype(np.float32)
    _check(ix, ref, q, 10, 5)
    ix.save(tmp_path / "tier.sivf")
    cfg, live = sivf.checkpoint_config(tmp_path / "tier.sivf")
    assert live == ref.live()
    jx = sivf.Index.load(tmp_path / "tier.sivf")
    assert same_membership(jx.membership(), ref.membership())
    st, rd, rl = ref.search(q, 10, 5)
    gd, gl = jx.search(q, 10, 5)
    assert jx.sync() == 0
    compare_results(gd.cpu().numpy(), gl.cpu().numpy(), rd, rl)
    say("  dense index refused, NOSPACE leaves the index unchanged, checkpoint keeps cold entries")


def test_tier_maintain_policy():
    """Below the free-slab mark, maintain offloads the least probed lists
    first; results stay exact; a later maintain reclaims dead segments."""
    rng = np.random.default_rng(64)
    d, nlist, C = 24, 12, 32
    cent = (rng.standard_normal((nlist, d)) * 6).astype(np.float32)
    ix, ref = _pair(d, nlist, cent, 0, C, 400, 12000, 600, max_batch=4096, max_queries=256, max_k=16,
                    max_nprobe=3)
    lab = rng.integers(0, nlist, 10000)
    x = (cent[lab] + rng.standard_normal((10000, d))).astype(np.float32)
    for s in range(0, 10000, 4096):
        ix.add(x[s:s + 4096], np.arange(s, min(10000, s + 4096)))
    assert ix.sync() == 0 and ref.add(x, np.arange(10000)) == 0
    hot = [0, 1, 2, 3, 4, 5]
    qh = (cent[rng.choice(hot, 256)] + 0.1 * rng.standard_normal((256, d))).astype(np.float32)
    for _ in range(4):
        ix.search(qh, 16, 3)                          # only lists near the hot centroids get probed
    assert ix.sync() == 0
    heat = ix.list_heat()
    free0 = ix.stats()["free_slabs"]
    rep = ix.maintain(0.0, free0 + 60, 4)
    assert 1 <= rep["offloaded_lists"] <= 4 and rep["offloaded_positions"] > 0
    cold_lists = np.flatnonzero(ix.tier_dump()["cold_len"] > 0)
    assert heat[cold_lists].max() <= np.sort(heat)[len(cold_lists) - 1]   # the least probed went first
    _check(ix, ref, qh[:64], 16, 3)
    # the offloaded entries all leave (a window slides past them); maintain releases their segments
    cold = ix.tier_dump()["cold_ids"]
    cold = cold[cold >= 0]
    ix.remove(cold)
    assert ix.sync() == 0 and ref.remove(cold)[0] == 0
    rep2 = ix.maintain(0.0, 0, 0)
    assert rep2["reclaimed"] == rep["offloaded_positions"] and ix.tier_stats()["cold_positions"] == 0
    _check(ix, ref, qh[:64], 16, 3)
    say(f"  maintain: {rep}; then {rep2}")
