"""Checkpoint round trip (sivf_save / sivf_load): the loaded index holds the
same lists as the saved one -- membership bit-exact, every search identical --
also when it is loaded into a different pool (slab size, pool size, id range),
and it keeps matching the oracle under further mutation."""
import numpy as np
import pytest

import oracle
import paper_2601_11808_amd as sivf
from tests.gpu_common import compare_results, say
from tests.invariants import check_dump, membership_of, same_membership

pytestmark = pytest.mark.gpu


def _build(rng, d, nlist, metric, storage, C, n=6000, cap=10000):
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    kw = dict(metric=metric, slab_capacity=C, num_slabs=n // C + 2 * nlist + 16, id_capacity=cap, max_batch=4096,
              max_queries=256, max_k=16, max_nprobe=nlist, storage=storage, rerank_factor=4 if storage else 0)
    ix = sivf.Index(d, nlist, cent, **kw)
    ref = oracle.OracleIndex(d, nlist, cent, metric, C, kw["num_slabs"], cap)
    x = rng.standard_normal((n, d)).astype(np.float32)
    ids = rng.permutation(cap)[:n].astype(np.int64)
    for s in range(0, n, 4096):
        ix.add(x[s:s + 4096], ids[s:s + 4096])
        assert ref.add(x[s:s + 4096], ids[s:s + 4096]) == 0
    # deletes and upserts scramble positions inside the lists
    rm = ids[rng.random(n) < 0.3]
    ix.remove(rm)
    assert ref.remove(rm)[0] == 0
    up = ids[rng.random(n) < 0.1]
    xu = rng.standard_normal((up.shape[0], d)).astype(np.float32)
    ix.add(xu, up)
    assert ref.add(xu, up) == 0
    assert ix.sync() == 0
    return ix, ref, cent, kw


@pytest.mark.parametrize("metric,storage", [(0, 0), (1, 0), (0, 1)])
def test_checkpoint_round_trip(tmp_path, metric, storage):
    rng = np.random.default_rng([31, metric, storage])
    d, nlist = 40, 23
    ix, ref, cent, kw = _build(rng, d, nlist, metric, storage, 64)
    path = tmp_path / "index.sivf"
    ix.save(path)
    cfg, live = sivf.checkpoint_config(path)
    assert live == ref.live() and cfg.dim == d and cfg.nlist == nlist
    q = rng.standard_normal((200, d)).astype(np.float32)
    d0, l0 = ix.search(q, 16, 5)
    assert ix.sync() == 0
    d0, l0 = d0.cpu().numpy(), l0.cpu().numpy()
    m0 = membership_of(ix.dump())
    for over in ({}, {"slab_capacity": 32, "num_slabs": kw["num_slabs"] * 2, "id_capacity": 20000},
                 {"slab_capacity": 128, "max_batch": 1000}):
        jx = sivf.Index.load(path, **over)
        C = over.get("slab_capacity", 64)
        dj = jx.dump()
        check_dump(dj, C, over.get("num_slabs", kw["num_slabs"]))
        assert same_membership(membership_of(dj), m0)
        d1, l1 = jx.search(q, 16, 5)
        assert jx.sync() == 0
        np.testing.assert_array_equal(l1.cpu().numpy(), l0)
        np.testing.assert_array_equal(d1.cpu().numpy().view(np.uint32), d0.view(np.uint32))
        # the loaded index stays consistent under further mutation
        x = rng.standard_normal((500, d)).astype(np.float32)
        nid = rng.integers(0, 10000, 500)
        jx.add(x, nid)
        assert jx.sync() == 0
        jx.remove(nid[:100])
        assert jx.sync() == 0
        check_dump(jx.dump(), C, over.get("num_slabs", kw["num_slabs"]))
        del jx
    if storage == 0:
        st, rd, rl = ref.search(q, 16, 5)
        compare_results(d0, l0, rd, rl)
    say(f"  metric={metric} storage={storage}: {live} entries; identical after load into three pools")


def test_checkpoint_continues_like_oracle(tmp_path):
    """After a load, the same operation sequence on the loaded index and on the
    oracle (which never saved) gives the same membership and searches."""
    rng = np.random.default_rng(32)
    d, nlist = 24, 11
    ix, ref, cent, kw = _build(rng, d, nlist, 0, 0, 32, n=3000, cap=5000)
    path = tmp_path / "index.sivf"
    ix.save(path)
    jx = sivf.Index.load(path, num_slabs=kw["num_slabs"] + 100)
    q = rng.standard_normal((64, d)).astype(np.float32)
    for step in range(5):
        x = rng.standard_normal((400, d)).astype(np.float32)
        nid = rng.integers(0, 5000, 400)
        jx.add(x, nid)
        assert jx.sync() == 0
        assert ref.add(x, nid) == 0
        rm = rng.integers(0, 5000, 300)
        jx.remove(rm)
        assert jx.sync() == 0
        assert ref.remove(rm)[0] == 0
        assert same_membership(membership_of(jx.dump()), ref.membership())
        gd, gl = jx.search(q, 10, 4)
        assert jx.sync() == 0
        st, rd, rl = ref.search(q, 10, 4)
        compare_results(gd.cpu().numpy(), gl.cpu().numpy(), rd, rl)


def test_checkpoint_errors(tmp_path):
    rng = np.random.default_rng(33)
    ix, ref, cent, kw = _build(rng, 16, 7, 0, 0, 32, n=2000, cap=3000)
    path = tmp_path / "index.sivf"
    ix.save(path)
    with pytest.raises(sivf.SivfError) as e:      # the pool cannot hold the entries
        sivf.Index.load(path, num_slabs=20)
    assert e.value.status == sivf.ERR_NOSPACE
    with pytest.raises(sivf.SivfError) as e:      # ids beyond the new id range
        sivf.Index.load(path, id_capacity=100)
    assert e.value.status == sivf.ERR_ID_RANGE
    with pytest.raises(sivf.SivfError) as e:      # not a checkpoint
        bad = tmp_path / "bad.sivf"
        bad.write_bytes(b"not a checkpoint" * 10)
        sivf.Index.load(bad)
    assert e.value.status == sivf.ERR_ARG
    # an empty index round-trips too
    ex = sivf.Index(16, 7, cent, metric=0, slab_capacity=32, num_slabs=64, id_capacity=100, max_batch=64,
                    max_queries=8, max_k=8, max_nprobe=7)
    ex.save(tmp_path / "empty.sivf")
    ey = sivf.Index.load(tmp_path / "empty.sivf")
    assert ey.stats()["live"] == 0
    gd, gl = ey.search(rng.standard_normal((3, 16)).astype(np.float32), 4, 7)
    assert ey.sync() == 0 and (gl.cpu().numpy() == -1).all()
