"""Certified FP32 MFMA scan (search tile 16 on fp32 slabs): the matrix-core
values only decide which slots get their canonical FP32 distance recomputed,
so results must be bit-identical to the VALU scan's and match the oracle
(identical ids, distances within 1e-5 relative).  Cases that stress the
error bound: near-ties, large common offsets (cancellation in
|x|^2 + |q|^2 - 2 x.q), tiny magnitudes (underflow), equal rows."""
import numpy as np
import pytest

import oracle
import paper_2601_11808_amd as sivf
from tests.gpu_common import Pair, compare_results, say
from tests.invariants import membership_of, same_membership

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    say(f"\n[gpu] {request.node.name}")
    yield


def _both(ix, q, k, nprobe, kpq=None, npq=None, sched=(16, 14, 0)):
    """Search with the VALU scan (tile 8) and the certified scan; assert bit-identical results."""
    ix.set_search_schedule(8, 14, 0)
    d0, l0 = ix.search(q, k, nprobe, k_per_query=kpq, nprobe_per_query=npq)
    assert ix.sync() == 0
    ix.set_search_schedule(*sched)
    d1, l1 = ix.search(q, k, nprobe, k_per_query=kpq, nprobe_per_query=npq)
    assert ix.sync() == 0
    d0, l0, d1, l1 = d0.cpu().numpy(), l0.cpu().numpy(), d1.cpu().numpy(), l1.cpu().numpy()
    np.testing.assert_array_equal(l1, l0)
    np.testing.assert_array_equal(d1.view(np.uint32), d0.view(np.uint32))
    return d1, l1


KINDS = ["normal", "offset", "tiny", "grid"]


def _data(kind, rng, n, d):
    if kind == "normal":
        return rng.standard_normal((n, d)).astype(np.float32)
    if kind == "offset":      # common offset 300 per dimension, unit noise: |x|^2 >> distances
        return (300.0 + rng.standard_normal((n, d))).astype(np.float32)
    if kind == "tiny":        # magnitudes near 1e-19: squared terms near the bottom of fp32's range
        return (1e-19 * rng.standard_normal((n, d))).astype(np.float32)
    if kind == "grid":        # small integers: many exact ties
        return rng.integers(-2, 3, (n, d)).astype(np.float32)
    raise ValueError(kind)


@pytest.mark.parametrize("kind,d,metric,C,mk", [("normal", 128, 0, 64, 64), ("normal", 100, 1, 32, 64),
                                                ("offset", 64, 0, 64, 64), ("offset", 32, 1, 16, 16),
                                                ("tiny", 48, 0, 64, 64), ("grid", 17, 0, 8, 64), ("grid", 24, 1, 4, 16),
                                                ("normal", 256, 0, 128, 64), ("normal", 5, 1, 64, 64),
                                                ("normal", 128, 0, 64, 16), ("tiny", 40, 1, 32, 16),
                                                ("grid", 33, 0, 64, 32)])
def test_cert_scan_matches_valu_and_oracle(kind, d, metric, C, mk):
    """mk = max_k: 16 keeps four queries' lists per register, 32 and 64 one."""
    rng = np.random.default_rng([KINDS.index(kind), d, metric, C, mk])
    nlist, n = 13, 6000
    cent = _data(kind, rng, nlist, d)
    x = _data(kind, rng, n, d)
    x[100:200] = x[:100]                       # equal rows under different ids
    x[200:300] = np.nextafter(x[:100], np.float32(np.inf))   # one-ulp neighbours
    ids = rng.permutation(n).astype(np.int64)
    q = np.concatenate([_data(kind, rng, 150, d), x[:50]]).astype(np.float32)   # some queries on data rows
    p = Pair(d, nlist, cent, metric, C, num_slabs=n // C + 4 * nlist + 8, id_capacity=n, max_batch=n,
             max_queries=q.shape[0], max_k=mk, max_nprobe=nlist)
    assert p.add(x, ids) == 0
    for k, nprobe in [(10, 3), (mk, 13), (1, 1)]:
        gd, gl = _both(p.gpu, q, k, nprobe)
        st, rd, rl = p.ref.search(q, k, nprobe)
        assert st == 0
        compare_results(gd, gl, rd, rl)
    kpq = rng.integers(0, mk + 1, q.shape[0]).astype(np.int32)
    npq = rng.integers(1, nlist + 1, q.shape[0]).astype(np.int32)
    gd, gl = _both(p.gpu, q, mk, nlist, kpq, npq)
    st, rd, rl = p.ref.search(q, mk, nlist, k_per_query=kpq, nprobe_per_query=npq)
    compare_results(gd, gl, rd, rl)
    # after deletes (tail-swap moves rows and their norms) and upserts
    assert p.remove(ids[::4]) == 0
    assert p.add(x[1::7] * np.float32(0.5), ids[1::7]) == 0
    gd, gl = _both(p.gpu, q, min(32, mk), 5, sched=(16, 10, 1))
    st, rd, rl = p.ref.search(q, min(32, mk), 5)
    compare_results(gd, gl, rd, rl)
    say(f"  {kind} d={d} metric={metric} C={C} max_k={mk}: identical to the VALU scan and the oracle")


@pytest.mark.parametrize("metric,mk", [(0, 64), (1, 64), (0, 16)])
def test_cert_scan_split_lists(metric, mk):
    """Long lists split into chunks, both schedules, ragged tails."""
    rng = np.random.default_rng([77, metric, mk])
    sizes = [30001, 12000, 999, 65, 3, 0]
    d = 64
    cent = (rng.standard_normal((len(sizes), d)) * 8).astype(np.float32)
    x = np.concatenate([cent[l] + rng.standard_normal((s, d)) for l, s in enumerate(sizes) if s]).astype(np.float32)
    ids = rng.permutation(x.shape[0]).astype(np.int64)
    q = (cent[rng.integers(0, len(sizes), 400)] + rng.standard_normal((400, d))).astype(np.float32)
    ix = sivf.Index(d, len(sizes), cent, metric=metric, slab_capacity=64, num_slabs=800, id_capacity=x.shape[0],
                    max_batch=1 << 16, max_queries=400, max_k=mk, max_nprobe=4)
    ref = oracle.OracleIndex(d, len(sizes), cent, metric, 64, 800, x.shape[0])
    ix.add(x, ids)
    assert ix.sync() == 0
    assert ref.add(x, ids) == 0
    k = min(50, mk)
    st, rd, rl = ref.search(q, k, 4)
    for sched in [(16, 10, 0), (16, 10, 1), (16, 12, 0), (16, 17, 1)]:
        gd, gl = _both(ix, q, k, 4, sched=sched)
        compare_results(gd, gl, rd, rl)
    t, sh, pm = ix.tune_search(q, k, 4)
    assert ix.sync() == 0
    gd, gl = ix.search(q, k, 4)
    assert ix.sync() == 0
    compare_results(gd.cpu().numpy(), gl.cpu().numpy(), rd, rl)
    say(f"  split lists: identical on 4 schedules; tuner chose tile {t}, 2^{sh}, persistent={pm}")


def test_cert_schedule_limits():
    """Tile 16 on fp32 slabs needs d <= 256 and slabs of >= 4 slots (any max_k up to 128)."""
    rng = np.random.default_rng(5)

    def mk(d, max_k, C):
        cent = rng.standard_normal((4, d)).astype(np.float32)
        return sivf.Index(d, 4, cent, slab_capacity=C, num_slabs=64, id_capacity=1024, max_batch=1024,
                          max_queries=16, max_k=max_k, max_nprobe=4)

    mk(256, 64, 4).set_search_schedule(16, 14, 0)
    mk(64, 128, 64).set_search_schedule(16, 14, 0)
    for d, max_k, C in [(257, 16, 64), (64, 16, 2)]:
        with pytest.raises(sivf.SivfError):
            mk(d, max_k, C).set_search_schedule(16, 14, 0)


@pytest.mark.parametrize("metric", [0, 1])
def test_cert_scan_k128_split_lists(metric):
    """Lists of 128 keys (k = 100 and 128, per-query k): work items of 8 queries,
    two registers per list; long lists split into chunks, both schedules; bit for
    bit equal to the VALU scan and equal to the oracle."""
    rng = np.random.default_rng([78, metric])
    sizes = [20001, 9000, 999, 130, 3, 0]
    d = 48
    cent = (rng.standard_normal((len(sizes), d)) * 8).astype(np.float32)
    x = np.concatenate([cent[l] + rng.standard_normal((s, d)) for l, s in enumerate(sizes) if s]).astype(np.float32)
    x[500:600] = x[:100]                       # equal rows: ties on distance
    ids = rng.permutation(x.shape[0]).astype(np.int64)
    q = np.concatenate([(cent[rng.integers(0, len(sizes), 300)] + rng.standard_normal((300, d))),
                        x[rng.integers(0, x.shape[0], 50)]]).astype(np.float32)
    ix = sivf.Index(d, len(sizes), cent, metric=metric, slab_capacity=64, num_slabs=700, id_capacity=x.shape[0],
                    max_batch=1 << 16, max_queries=q.shape[0], max_k=128, max_nprobe=6)
    ref = oracle.OracleIndex(d, len(sizes), cent, metric, 64, 700, x.shape[0])
    ix.add(x, ids)
    assert ix.sync() == 0
    assert ref.add(x, ids) == 0
    for k, nprobe in [(100, 3), (128, 6), (65, 1)]:
        st, rd, rl = ref.search(q, k, nprobe)
        for sched in [(16, 10, 0), (16, 12, 1), (16, 17, 0)]:
            gd, gl = _both(ix, q, k, nprobe, sched=sched)
            compare_results(gd, gl, rd, rl)
    kpq = rng.integers(0, 129, q.shape[0]).astype(np.int32)
    npq = rng.integers(1, 7, q.shape[0]).astype(np.int32)
    gd, gl = _both(ix, q, 128, 6, kpq, npq, sched=(16, 11, 1))
    st, rd, rl = ref.search(q, 128, 6, k_per_query=kpq, nprobe_per_query=npq)
    compare_results(gd, gl, rd, rl)
    # after deletes (tail moves) the lists are read again
    assert ix.remove(ids[::3]) is not None and ix.sync() == 0
    assert ref.remove(ids[::3])[0] == 0
    gd, gl = _both(ix, q, 100, 4, sched=(16, 12, 0))
    st, rd, rl = ref.search(q, 100, 4)
    compare_results(gd, gl, rd, rl)
    say("  k = 100/128 certified scan: identical to the VALU scan and the oracle on split lists")


@pytest.mark.parametrize("metric", [0, 1])
def test_cert_ties_across_work_items(metric):
    """Equal keys spread over every chunk of a split list: 300 distinct integer
    rows, each stored 80 times at random positions under random ids, so a
    query's k-th distance is shared by dozens of rows in different work items.
    A work item may take another item's published k-th value as its threshold;
    rows equal to it must still pass, so the k smallest ids of the tied rows
    come out (the oracle's order), for k up to 64 and above 64, split and
    whole-list schedules."""
    rng = np.random.default_rng([81, metric])
    d = 24
    base = np.concatenate([rng.integers(-2, 3, (200, d)), 3 + rng.integers(-1, 2, (100, d))]).astype(np.float32)
    x = np.repeat(base, 80, axis=0)[rng.permutation(base.shape[0] * 80)]
    ids = rng.permutation(x.shape[0]).astype(np.int64)
    cent = np.stack([np.zeros(d), np.full(d, 3.0), np.full(d, -3.0)]).astype(np.float32)
    q = np.concatenate([rng.integers(-2, 4, (100, d)).astype(np.float32), base[rng.integers(0, 300, 50)]])
    ix = sivf.Index(d, 3, cent, metric=metric, slab_capacity=64, num_slabs=420, id_capacity=x.shape[0],
                    max_batch=1 << 15, max_queries=q.shape[0], max_k=128, max_nprobe=3)
    ref = oracle.OracleIndex(d, 3, cent, metric, 64, 420, x.shape[0])
    ix.add(x, ids)
    assert ix.sync() == 0
    assert ref.add(x, ids) == 0
    for k, nprobe in [(10, 1), (64, 3), (100, 2), (128, 3)]:
        st, rd, rl = ref.search(q, k, nprobe)
        assert st == 0
        for sched in [(16, 10, 0), (16, 10, 1), (16, 17, 0)]:
            if k > 64:
                ix.set_deep_schedule(*sched)
            gd, gl = _both(ix, q, k, nprobe, sched=sched)
            compare_results(gd, gl, rd, rl)
    say(f"  metric={metric}: tied keys across work items resolved as the oracle does")


@pytest.mark.parametrize("deep", [(4, 12, 1), (8, 10, 0), (16, 13, 1), (16, 11, 0)])
def test_cert_two_pass_mixed_k(deep):
    """A certified-scan search whose per-query k straddles 64 runs two passes
    (k <= 64 certified, k > 64 on the deep schedule) over one snapshot: equal
    to the oracle and to the single-pass VALU scan, for every deep schedule,
    with k = 0 queries, k exactly 64 and 65, and lists split into chunks; the
    profile counts each search once."""
    rng = np.random.default_rng([79, deep[0], deep[1]])
    sizes = [12000, 5000, 700, 65, 1, 0, 3000]
    d = 40
    cent = (rng.standard_normal((len(sizes), d)) * 6).astype(np.float32)
    x = np.concatenate([cent[l] + rng.standard_normal((s, d)) for l, s in enumerate(sizes) if s]).astype(np.float32)
    x[200:260] = x[:60]
    ids = rng.permutation(x.shape[0]).astype(np.int64)
    q = (cent[rng.integers(0, len(sizes), 400)] + rng.standard_normal((400, d))).astype(np.float32)
    ix = sivf.Index(d, len(sizes), cent, metric=0, slab_capacity=32, num_slabs=900, id_capacity=x.shape[0],
                    max_batch=1 << 15, max_queries=q.shape[0], max_k=128, max_nprobe=7)
    ref = oracle.OracleIndex(d, len(sizes), cent, 0, 32, 900, x.shape[0])
    ix.add(x, ids)
    assert ix.sync() == 0
    assert ref.add(x, ids) == 0
    kpq = rng.choice([0, 1, 7, 16, 33, 64, 65, 100, 128], q.shape[0]).astype(np.int32)
    npq = rng.integers(1, 8, q.shape[0]).astype(np.int32)
    ix.set_deep_schedule(*deep)
    assert ix.search_schedule()[1] == deep
    st, rd, rl = ref.search(q, 128, 7, k_per_query=kpq, nprobe_per_query=npq)
    gd, gl = _both(ix, q, 128, 7, kpq, npq, sched=(16, 12, 1))
    compare_results(gd, gl, rd, rl)
    # one k for all: k > 64 runs the deep pass alone, k <= 64 the certified scan alone
    for k in (100, 40):
        st, rd, rl = ref.search(q, k, 5)
        gd, gl = _both(ix, q, k, 5, sched=(16, 10, 0))
        compare_results(gd, gl, rd, rl)
    ix.set_search_schedule(16, 12, 1)
    ix.profile(True)
    for _ in range(3):
        ix.search(q, 128, 7, k_per_query=kpq, nprobe_per_query=npq)
    assert ix.sync() == 0
    prof = ix.profile_read()
    ix.profile(False)
    assert prof["search"][1] == 3 and prof["scan"][1] == 3 and prof["merge"][1] == 3, prof
    assert prof["scan_deep"][1] == 3 and prof["scan_deep"][0] > 0, prof
    say(f"  deep schedule {deep}: two-pass search identical to the oracle and the VALU scan")


def test_deep_schedule_args():
    rng = np.random.default_rng(80)
    cent = rng.standard_normal((4, 32)).astype(np.float32)
    ix = sivf.Index(32, 4, cent, slab_capacity=16, num_slabs=64, id_capacity=256, max_batch=256, max_queries=16,
                    max_k=100, max_nprobe=4)
    for bad in [(5, 12, 1), (16, 5, 0), (4, 12, 2)]:
        with pytest.raises(sivf.SivfError):
            ix.set_deep_schedule(*bad)
    ix.set_deep_schedule(8, 14, 0)
    assert ix.search_schedule()[1] == (8, 14, 0)
    bx = sivf.Index(32, 4, cent, slab_capacity=16, num_slabs=64, id_capacity=256, max_batch=256, max_queries=16,
                    max_k=10, max_nprobe=4, storage=sivf.BF16, rerank_factor=2)
    with pytest.raises(sivf.SivfError):
        bx.set_deep_schedule(4, 12, 1)


def test_cert_random_configs():
    """150 seeded random configurations (d 1..256, C 4..128, L2/IP, max_k 16/32/64, data from 1e-25 to 1e18
    in scale, repeated rows and one-ulp neighbours, random schedules): tile 16 and tile 8 agree bit for bit,
    and both equal the oracle (same ids, distances within 1e-5 relative)."""
    rng = np.random.default_rng(2026)
    for it in range(150):
        d = int(rng.integers(1, 257))
        C = int(rng.choice([4, 8, 16, 32, 64, 128]))
        metric = int(rng.integers(0, 2))
        mk = int(rng.choice([16, 32, 64]))
        nlist = int(rng.integers(1, 30))
        n = int(rng.integers(1, 6000))
        kind = ["normal", "offset", "tiny", "grid", "mixed", "huge"][it % 6]
        if kind == "normal":
            x = rng.standard_normal((n, d))
        elif kind == "offset":
            x = float(10 ** rng.uniform(0, 4)) + rng.standard_normal((n, d))
        elif kind == "tiny":
            x = 10 ** rng.uniform(-25, -15) * rng.standard_normal((n, d))
        elif kind == "grid":
            x = rng.integers(-3, 4, (n, d)).astype(np.float64)
        elif kind == "mixed":
            x = rng.standard_normal((n, d)) * (10 ** rng.uniform(-3, 3, (n, 1)))
        else:
            x = 10 ** rng.uniform(10, 18) * rng.standard_normal((n, d))
        x = x.astype(np.float32)
        if n > 40:
            x[n // 2:n // 2 + 10] = x[:10]
            x[n // 2 + 10:n // 2 + 20] = np.nextafter(x[:10], np.float32(np.inf))
        nq = int(rng.integers(1, 200))
        q = np.concatenate([x[rng.integers(0, n, nq // 2)],
                            x[rng.integers(0, n, nq - nq // 2)] +
                            (np.float32(1e-3) * rng.standard_normal((nq - nq // 2, d))).astype(np.float32)])
        q = q.astype(np.float32)
        cent = (x[rng.integers(0, n, nlist)] + np.float32(0.1) * rng.standard_normal((nlist, d))).astype(np.float32)
        ix = sivf.Index(d, nlist, cent, metric=metric, slab_capacity=C, num_slabs=n // C + 2 * nlist + 8,
                        id_capacity=n, max_batch=n, max_queries=nq, max_k=mk, max_nprobe=nlist)
        ref = oracle.OracleIndex(d, nlist, cent, metric, C, n // C + 2 * nlist + 8, n)
        ids = rng.permutation(n).astype(np.int64)
        ix.add(x, ids)
        assert ix.sync() == 0
        assert ref.add(x, ids) == 0
        k, nprobe = int(rng.integers(1, mk + 1)), int(rng.integers(1, nlist + 1))
        gd, gl = _both(ix, q, k, nprobe, sched=(16, int(rng.integers(6, 18)), int(rng.integers(0, 2))))
        st, rd, rl = ref.search(q, k, nprobe)
        assert st == 0
        try:
            compare_results(gd, gl, rd, rl)
        except AssertionError:
            gp, rp = ix.probe(q, nprobe).cpu().numpy(), oracle.probe(q, cent, nprobe, metric)
            same_m = same_membership(membership_of(ix.dump()), ref.membership())
            say(f"  config {it}: kind={kind} d={d} C={C} metric={metric} max_k={mk} nlist={nlist} n={n} nq={nq} "
                f"k={k} nprobe={nprobe}; probes equal: {np.array_equal(gp, rp)}; membership equal: {same_m}")
            raise
        del ix, ref
    say("  150 random configurations: identical to each other and to the oracle")
