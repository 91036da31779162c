"""External 64-bit id registry (sivf_registry_*): arbitrary int64 keys mapped
onto the dense internal ids on the device.  Checked against the oracle run on
the internal ids the registry reports (so even exact ties resolve the same
way), with upserts, duplicate keys in a batch, absent and repeated removes,
id-space exhaustion (a failed add maps nothing), table rebuilds after many
tombstones, and a save / load round trip."""
import numpy as np
import pytest

import oracle
import paper_2601_11808_amd as sivf
from tests.gpu_common import compare_results, say
from tests.invariants import check_dump, membership_of, same_membership

pytestmark = pytest.mark.gpu

INT64_MIN = np.iinfo(np.int64).min


def _keys(rng, n):
    """n distinct keys over the whole int64 range, small and negative ones included."""
    k = rng.integers(INT64_MIN + 2, np.iinfo(np.int64).max, n, dtype=np.int64)
    k[: n // 8] = rng.choice(np.arange(-500, 500), n // 8, replace=False)
    assert np.unique(k).shape[0] == n
    return k


class Mirror:
    """A registry over a GPU index, and the oracle fed the internal ids the
    registry reports."""

    def __init__(self, d, nlist, cent, cap, C=32, num_slabs=600):
        self.ix = sivf.Index(d, nlist, cent, metric=0, slab_capacity=C, num_slabs=num_slabs, id_capacity=cap,
                             max_batch=2048, max_queries=128, max_k=16, max_nprobe=nlist)
        self.reg = sivf.Registry(self.ix)
        self.ref = oracle.OracleIndex(d, nlist, cent, 0, C, num_slabs, cap)
        self.held = {}            # external -> internal, as the test expects it
        self.C, self.num_slabs = C, num_slabs

    def add(self, x, keys, expect=0):
        self.reg.add(x, keys)
        st = self.reg.sync()
        assert st == expect, (st, expect)
        if st != 0:
            return
        internal = self.reg.lookup(keys).cpu().numpy()
        assert (internal >= 0).all()
        # equal keys share one internal id; different keys never do
        for k, v in zip(keys.tolist(), internal.tolist()):
            assert self.held.setdefault(k, v) == v
        assert len(set(self.held.values())) == len(self.held)
        assert self.ref.add(x, internal) == 0

    def remove(self, keys):
        internal = self.reg.lookup(keys).cpu().numpy()
        nrem = self.reg.remove(keys)
        assert self.reg.sync() == 0
        st, rn = self.ref.remove(internal[internal >= 0])
        assert st == 0 and int(nrem.item()) == rn
        for k in keys.tolist():
            self.held.pop(k, None)
        assert (self.reg.lookup(keys).cpu().numpy() == -1).all()

    def check(self, q, k=10, nprobe=4):
        d = self.ix.dump()
        check_dump(d, self.C, self.num_slabs)
        assert same_membership(membership_of(d), self.ref.membership())
        gd, gl = self.reg.search(q, k, nprobe)
        assert self.reg.sync() == 0
        st, rd, rl = self.ref.search(q, k, nprobe)
        inv = {v: kk for kk, v in self.held.items()}
        want = np.vectorize(lambda v: inv[v] if v >= 0 else -1, otypes=[np.int64])(rl)
        compare_results(gd.cpu().numpy(), gl.cpu().numpy(), rd, want)


def test_registry_matches_oracle():
    rng = np.random.default_rng(41)
    d, nlist, cap = 16, 9, 5000
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    m = Mirror(d, nlist, cent, cap)
    q = rng.standard_normal((50, d)).astype(np.float32)
    pool = _keys(rng, 6000)
    live = []
    for step in range(20):
        n = int(rng.integers(1, 600))
        keys = pool[rng.integers(0, pool.shape[0], n)]       # repeats within the batch and upserts
        x = rng.integers(-2, 3, (n, d)).astype(np.float32)     # small integers: exact ties on distance
        if len(set(m.held) | set(keys.tolist())) > cap:
            continue
        m.add(x, keys)
        live = list(m.held)
        rm = np.concatenate([np.asarray(live, np.int64)[rng.integers(0, len(live), int(rng.integers(0, 300)))],
                             _keys(rng, 20)])                # live, repeated and absent keys
        m.remove(rm)
        m.check(q)
    say(f"  {len(m.held)} keys held after 20 rounds; identical to the oracle")


def test_registry_exhaustion_rebuild_and_reserved_keys():
    rng = np.random.default_rng(42)
    d, nlist, cap = 8, 5, 300
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    m = Mirror(d, nlist, cent, cap, num_slabs=200)
    q = rng.standard_normal((20, d)).astype(np.float32)
    keys = _keys(rng, 301)
    m.add(rng.standard_normal((250, d)).astype(np.float32), keys[:250])
    # 51 new keys with only 50 internal ids free: the whole batch fails and maps nothing
    m.add(rng.standard_normal((51, d)).astype(np.float32), keys[250:], expect=sivf.ERR_NOSPACE)
    assert (m.reg.lookup(keys[250:]).cpu().numpy() == -1).all()
    m.check(q)
    m.add(rng.standard_normal((50, d)).astype(np.float32), keys[250:300])
    assert len(m.held) == 300
    m.check(q)
    # reserved markers are refused
    m.reg.add(rng.standard_normal((2, d)).astype(np.float32), np.array([INT64_MIN, 5], np.int64))
    assert m.reg.sync() == sivf.ERR_ARG
    m.check(q)
    # many add / remove rounds leave tombstones: the table is rebuilt and keeps answering
    for r in range(40):
        old = np.asarray(list(m.held), np.int64)[:100]
        m.remove(old)
        fresh = _keys(rng, 100)
        m.add(rng.standard_normal((100, d)).astype(np.float32), fresh)
    m.check(q)
    say(f"  exhaustion refused and rolled back; 4,000 fresh keys through a 2,048-slot table")


def test_registry_save_load(tmp_path):
    rng = np.random.default_rng(43)
    d, nlist, cap = 12, 7, 3000
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    m = Mirror(d, nlist, cent, cap)
    keys = _keys(rng, 2500)
    m.add(rng.standard_normal((2000, d)).astype(np.float32), keys[:2000])
    m.remove(keys[:500])
    q = rng.standard_normal((40, d)).astype(np.float32)
    d0, l0 = m.reg.search(q, 10, 3)
    assert m.reg.sync() == 0
    m.ix.save(tmp_path / "ix.sivf")
    m.reg.save(tmp_path / "reg.sivf")
    jx = sivf.Index.load(tmp_path / "ix.sivf")
    jr = sivf.Registry(jx)
    jr.load(tmp_path / "reg.sivf")
    d1, l1 = jr.search(q, 10, 3)
    assert jr.sync() == 0
    np.testing.assert_array_equal(l1.cpu().numpy(), l0.cpu().numpy())
    np.testing.assert_array_equal(d1.cpu().numpy(), d0.cpu().numpy())
    np.testing.assert_array_equal(jr.lookup(keys).cpu().numpy(), m.reg.lookup(keys).cpu().numpy())
    # the loaded registry hands out only free internal ids
    jr.add(rng.standard_normal((500, d)).astype(np.float32), keys[2000:])
    assert jr.sync() == 0
    internal = jr.lookup(keys[500:]).cpu().numpy()
    assert (internal >= 0).all() and np.unique(internal).shape[0] == 2000
