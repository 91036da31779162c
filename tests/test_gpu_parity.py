"""GPU parity: the HIP library against the CPU oracle on seeded inputs.

Membership after every operation must be bit-exact (same ids in the same
lists), device-state invariants must hold, and FP32 search must return the
oracle's ids with distances within 1e-5 relative.
"""
import json
import os

import numpy as np
import pytest

import oracle
import paper_2601_11808_amd as sivf
import workloads
from tests.gpu_common import Pair, compare_results, say
from tests.invariants import check_dump

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(autouse=True)
def _announce(request):
    say(f"\n[gpu] {request.node.name}")
    yield


# ------------------------------------------------------------ coarse stage

@pytest.mark.parametrize("kind,d,nlist", [("normal", 32, 16), ("int", 128, 1024), ("scaled", 96, 300),
                                          ("unit", 96, 256), ("odd", 30, 77)])
def test_coarse_mfma_error_bound(kind, d, nlist):
    """The approximate FP32-MFMA distances stay inside the bound the exact
    re-check assumes: |approx - exact| <= (4d+16) 2^-24 (|x|+|c|)^2."""
    rng = np.random.default_rng([7, d, nlist])
    if kind == "int":
        cent = rng.uniform(0, 255, (nlist, d)).astype(np.float32)
        x = rng.integers(0, 256, (3000, d)).astype(np.float32)
    elif kind == "scaled":
        cent = (rng.standard_normal((nlist, d)) * 1e3).astype(np.float32)
        x = (rng.standard_normal((3000, d)) * 1e3 + 5e3).astype(np.float32)
    elif kind == "unit":
        cent = rng.standard_normal((nlist, d))
        cent = (cent / np.linalg.norm(cent, axis=1, keepdims=True)).astype(np.float32)
        x = rng.standard_normal((3000, d))
        x = (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)
    else:
        cent = rng.standard_normal((nlist, d)).astype(np.float32)
        x = rng.standard_normal((3000, d)).astype(np.float32)
    for storage, metric in ((0, 0), (0, 1), (1, 0), (1, 1)):
        if storage == 1 and d > 256:
            continue
        ix = sivf.Index(d, nlist, cent, metric=metric, slab_capacity=64, num_slabs=64, id_capacity=64,
                        max_batch=4096, max_queries=64, max_k=16, max_nprobe=16, storage=storage,
                        rerank_factor=4 if storage else 0)
        s = ix.coarse_scores(x).cpu().numpy().astype(np.float64)
        xd, cd = x.astype(np.float64), cent.astype(np.float64)
        nx, nc = np.linalg.norm(xd, axis=1), np.linalg.norm(cd, axis=1)
        coef = (4 * d + 16) * 2.0 ** -24
        u = 2.0 ** -8     # bf16 operands on reduced-storage indexes: |x.c - x~.c~| <= (2u + u^2)|x||c|
        if metric == 0:
            exact = ((xd[:, None, :] - cd[None]) ** 2).sum(-1)
            bound = coef * (nx[:, None] + nc[None]) ** 2 + storage * 2 * (2 * u + u * u) * nx[:, None] * nc[None]
        else:
            exact = -(xd @ cd.T)
            bound = coef * nx[:, None] * nc[None] + storage * (2 * u + u * u) * nx[:, None] * nc[None]
        ratio = np.abs(s - exact) / bound
        say(f"  storage {storage} metric {metric}: max |approx-exact|/bound = {ratio.max():.3e}")
        assert ratio.max() <= (0.5 if storage == 0 else 1.0)


def _tie_data(seed, d, nlist, n):
    rng = np.random.default_rng(seed)
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    cent[5] = cent[2]                       # exact duplicates: ties -> lower id
    cent[nlist - 1] = cent[0]
    x = rng.standard_normal((n, d)).astype(np.float32)
    a = rng.integers(0, nlist, n // 3)
    b = rng.integers(0, nlist, n // 3)
    x[: n // 3] = (cent[a] + cent[b]) * np.float32(0.5)   # near-equidistant points
    x[n // 3: n // 3 + 8] = cent[[0, 2, 5, 7, 9, nlist - 1, 3, 4]]
    return cent, x


@pytest.mark.parametrize("metric", [0, 1])
def test_assign_and_probe_exact(metric):
    """Coarse decisions equal the oracle's (FP64 canonical distance, ties to
    the smaller list id) on inputs full of near-ties and exact ties."""
    # one-wave selection with 32 (up to 2,048 lists) and 64 (up to 4,096) distances per lane; 4,100 lists
    # take the block selection
    for d, nlist in [(16, 64), (128, 1024), (7, 13), (24, 3000), (40, 4096), (20, 4100)]:
        cent, x = _tie_data(d * 1000 + nlist, d, nlist, 6000)
        p = Pair(d, nlist, cent, metric=metric, max_batch=8192, max_nprobe=64)
        ga = p.gpu.assign(x).cpu().numpy()
        ra = oracle.assign(x, cent, metric)
        np.testing.assert_array_equal(ga, ra)
        for m in (1, 5, 32, 64):
            gp = p.gpu.probe(x[:1500], m).cpu().numpy()
            rp = oracle.probe(x[:1500], cent, m, metric)
            np.testing.assert_array_equal(gp, rp)


@pytest.mark.parametrize("metric", [0, 1])
def test_assign_and_probe_exact_bf16_coarse(metric):
    """Reduced-storage indexes run the coarse GEMM on bf16 MFMA; with the
    wider certified bound the decisions still equal the oracle's exactly."""
    for d, nlist in [(16, 64), (128, 1024), (7, 13), (96, 4100)]:
        cent, x = _tie_data(d * 1000 + nlist + 7, d, nlist, 4000)
        ix = sivf.Index(d, nlist, cent, metric=metric, slab_capacity=64, num_slabs=64, id_capacity=64,
                        max_batch=4096, max_queries=4096, max_k=16, max_nprobe=64, storage=1, rerank_factor=4)
        np.testing.assert_array_equal(ix.assign(x).cpu().numpy(), oracle.assign(x, cent, metric))
        for m in (1, 7, 64):
            gp = ix.probe(x[:1000], m).cpu().numpy()
            np.testing.assert_array_equal(gp, oracle.probe(x[:1000], cent, m, metric))
    w = workloads.serving(n_base=0)
    rng = np.random.default_rng([12, metric])
    x = (w.means[rng.integers(0, 16384, 3000)] + 48 * rng.standard_normal((3000, 128))).astype(np.float32)
    ix = sivf.Index(128, 16384, w.centroids, metric=metric, slab_capacity=128, num_slabs=64, id_capacity=64,
                    max_batch=4096, max_queries=4096, max_k=16, max_nprobe=64, storage=2, rerank_factor=4)
    np.testing.assert_array_equal(ix.assign(x).cpu().numpy(), oracle.assign(x, w.centroids, metric))
    np.testing.assert_array_equal(ix.probe(x[:300], 64).cpu().numpy(), oracle.probe(x[:300], w.centroids, 64, metric))


@pytest.mark.parametrize("metric", [0, 1])
def test_assign_bf16_large_batches(metric):
    """Large insert batches on bf16-coarse indexes: blocks sweep many centroid
    tiles (up to 16, double-buffered) and segments end on a ragged tile; sampled
    rows equal the oracle's nearest list (the rows are independent)."""
    w = workloads.serving(n_base=0)
    rng = np.random.default_rng([13, metric])
    for nlist, cent, n in [(16384, w.centroids, 40000), (4100, None, 30000)]:
        if cent is None:
            cent = (rng.standard_normal((nlist, 96)) * 3).astype(np.float32)
            x = (cent[rng.integers(0, nlist, n)] + rng.standard_normal((n, 96))).astype(np.float32)
            x[:50] = cent[:50]                              # exact centroid copies
        else:
            x = (w.means[rng.integers(0, nlist, n)] + 48 * rng.standard_normal((n, 128))).astype(np.float32)
        ix = sivf.Index(x.shape[1], nlist, cent, metric=metric, slab_capacity=64, num_slabs=64, id_capacity=64,
                        max_batch=n, max_queries=64, max_k=16, max_nprobe=8, storage=2, rerank_factor=4)
        got = ix.assign(x).cpu().numpy()
        sub = np.concatenate([np.arange(50), rng.choice(n, 1500, replace=False), np.arange(n - 50, n)])
        np.testing.assert_array_equal(got[sub], oracle.assign(x[sub], cent, metric))
        say(f"  bf16 coarse, {n} rows x {nlist} lists: {sub.shape[0]} sampled rows equal the oracle")


@pytest.mark.parametrize("metric", [0, 1])
def test_assign_decided_in_sweep(metric):
    """Batches of 65,536 rows or more over at most 2,048 lists: the bf16 sweep
    sees every list of its rows, decides the rows whose nearest list is
    separated by the certified bound and leaves the others to the FP64
    re-check.  Exact ties (duplicate centroids), near-equidistant points,
    centroid copies and rows too large for fp32 squares all equal the oracle,
    as does a random sample of the rest; fp32 and bf16 storage."""
    for d, nlist, n, storage in [(128, 1024, 70000, 0), (96, 2048, 66000, 0), (40, 1500, 80000, 1)]:
        cent, x = _tie_data(d * 7 + nlist + metric, d, nlist, n)
        x[-20:] = cent[:20] * np.float32(3e18)          # |x|^2 overflows fp32: every list re-checked
        rng = np.random.default_rng([d, nlist, metric])
        ix = sivf.Index(d, nlist, cent, metric=metric, slab_capacity=64, num_slabs=64, id_capacity=64,
                        max_batch=n, max_queries=64, max_k=16, max_nprobe=8, storage=storage,
                        rerank_factor=4 if storage else 0)
        got = ix.assign(x).cpu().numpy()
        sub = np.concatenate([np.arange(3000), np.arange(n // 3, n // 3 + 8),
                              rng.choice(n, 2000, replace=False), np.arange(n - 20, n)])
        np.testing.assert_array_equal(got[sub], oracle.assign(x[sub], cent, metric))
        say(f"  {n} rows x {nlist} lists (d={d}, storage {storage}): {sub.shape[0]} rows equal the oracle")


@pytest.mark.parametrize("metric", [0, 1])
def test_assign_many_lists_and_extremes(metric):
    """Nearest-list decisions at the serving shape (d=128, 16,384 lists), with
    a ragged last group of lists (4,100 lists), and at magnitudes where fp32
    squares overflow (every list is then re-checked in FP64)."""
    w = workloads.serving(n_base=0)
    rng = np.random.default_rng([11, metric])
    x = (w.means[rng.integers(0, 16384, 3000)] + 48 * rng.standard_normal((3000, 128))).astype(np.float32)
    p = Pair(128, 16384, w.centroids, metric=metric, max_batch=4096, max_nprobe=64)
    np.testing.assert_array_equal(p.gpu.assign(x).cpu().numpy(), oracle.assign(x, w.centroids, metric))
    gp = p.gpu.probe(x[:500], 64).cpu().numpy()
    np.testing.assert_array_equal(gp, oracle.probe(x[:500], w.centroids, 64, metric))
    cent, xt = _tie_data(4100 + metric, 128, 4100, 3000)
    p = Pair(128, 4100, cent, metric=metric, max_batch=4096, max_nprobe=64)
    np.testing.assert_array_equal(p.gpu.assign(xt).cpu().numpy(), oracle.assign(xt, cent, metric))
    big_c = (rng.standard_normal((300, 33)) * 1e19).astype(np.float32)
    big_x = (big_c[rng.integers(0, 300, 2000)] * np.float32(1.0001)
             + (rng.standard_normal((2000, 33)) * 1e17).astype(np.float32)).astype(np.float32)
    assert np.isfinite(big_x).all()
    p = Pair(33, 300, big_c, metric=metric, max_batch=4096, max_nprobe=64)
    np.testing.assert_array_equal(p.gpu.assign(big_x).cpu().numpy(), oracle.assign(big_x, big_c, metric))


@pytest.mark.parametrize("metric", [0, 1])
def test_probe_and_search_at_overflow_magnitudes(metric):
    """Probe sets and searches equal the oracle's where fp32 squares, norm sums or
    dot products of the coarse GEMM overflow (approximations become inf or NaN):
    such rows must be re-checked against every list, not dropped.  Vector norms
    from about 1e17 up to 1e19 (either side of the re-check-everything threshold
    |x| + max|c| = 2^60), nprobe 2, 7 and 64, k 10.  IP coordinates stay below
    1.5e19, so every fp32 product of the fine distance is finite."""
    rng = np.random.default_rng([13, metric])
    # the hand-made case: x equal to a centroid whose fp32 |c|^2 + |x|^2 and 2 x.c
    # both overflow (approximation inf - inf = NaN), next to finite competitors
    cent = np.array([[7e18] * 4, [0.0] * 4, [1e18] * 4, [-3e18, 1e18, 2e18, 0.0]], np.float32)
    x = np.concatenate([cent, cent * np.float32(0.999), cent[:1] * np.float32(1.001)]).astype(np.float32)
    p = Pair(4, 4, cent, metric=metric, C=4, num_slabs=64, id_capacity=64, max_batch=64, max_queries=64,
             max_k=16, max_nprobe=4)
    assert p.add(x, np.arange(x.shape[0])) == 0
    p.check_state()
    for m in (1, 2, 3, 4):
        np.testing.assert_array_equal(p.gpu.probe(x, m).cpu().numpy(), oracle.probe(x, cent, m, metric))
        p.check_search(x, 5, m)
    for d, scale in [(8, 3e17), (16, 2e18), (33, 7e18), (128, 1e18)]:
        nlist = 96
        c = rng.standard_normal((nlist, d)) * scale
        pts = c[rng.integers(0, nlist, 3000)] * 1.0001 + rng.standard_normal((3000, d)) * scale * 0.02
        if metric == 1:
            c, pts = np.clip(c, -1.5e19, 1.5e19), np.clip(pts, -1.5e19, 1.5e19)
        c, pts = c.astype(np.float32), pts.astype(np.float32)
        assert np.isfinite(pts).all()
        pts[:8] = c[:8]                      # rows equal to centroids
        q = np.concatenate([pts[rng.integers(0, 3000, 150)], c[8:58]]).astype(np.float32)
        p = Pair(d, nlist, c, metric=metric, C=64, num_slabs=3000 // 64 + nlist + 8, id_capacity=3000,
                 max_batch=3000, max_queries=q.shape[0], max_k=16, max_nprobe=64)
        assert p.add(pts, rng.permutation(3000).astype(np.int64)) == 0
        p.check_state()
        for m in (2, 7, 64):
            np.testing.assert_array_equal(p.gpu.probe(q, m).cpu().numpy(), oracle.probe(q, c, m, metric))
            p.check_search(q, 10, m)
        say(f"  d={d} scale={scale:.0e}: probes and searches equal the oracle")


def test_ip_signed_zero_scores_tie_on_id():
    """IP scores that round to -0 and to +0 are the same score: the results are
    ordered by id among them, on the VALU scan (tile 8), the certified scan
    (tile 16) and the reduced-precision scan with its exact re-rank."""
    rng = np.random.default_rng(47)
    n, d = 3000, 8
    x = (rng.choice([-1.0, 1.0], (n, d)) * 1e-30).astype(np.float32)
    cent = np.zeros((2, d), np.float32)
    cent[1, 0] = 1.0
    q = np.concatenate([np.full((8, d), 1e-30), rng.choice([-1.0, 1.0], (8, d)) * 1e-30]).astype(np.float32)
    p = Pair(d, 2, cent, metric=1, C=64, num_slabs=200, id_capacity=n, max_batch=n, max_queries=16, max_k=32,
             max_nprobe=2)
    assert p.add(x, rng.permutation(n).astype(np.int64)) == 0
    for tile in (8, 16):
        p.gpu.set_search_schedule(tile, 14, 0)
        p.check_search(q, 32, 2)
        p.check_search(q, 5, 1)
    ix = sivf.Index(d, 2, cent, metric=1, slab_capacity=64, num_slabs=200, id_capacity=n, max_batch=n,
                    max_queries=16, max_k=16, max_nprobe=2, storage=1, rerank_factor=4)
    ix.add(x, np.arange(n))
    assert ix.sync() == 0
    gd, gl = ix.search(q, 10, 2)
    gl = gl.cpu().numpy()
    assert (gd.cpu().numpy() == 0).all()
    # every candidate scores 0 exactly, so the re-ranked top 10 of the 40 candidates
    # are the 10 smallest candidate ids: ascending, and never a deleted or missing id
    assert (np.diff(gl, axis=1) > 0).all() and (gl >= 0).all()


# --------------------------------------------------------- golden sequence

def test_golden_mutation_sequence_gpu():
    g = json.load(open(os.path.join(GOLD, "mutation_small.json")))
    cent = np.array(g["centroids"], np.float32)
    p = Pair(g["dim"], len(cent), cent, g["metric"], g["slab_capacity"], g["num_slabs"], g["id_capacity"],
             max_batch=64, max_queries=8, max_k=8, max_nprobe=4)
    for n, st in enumerate(g["steps"]):
        if st["op"] == "add":
            status = p.add(np.array(st["x"], np.float32), np.array(st["ids"], np.int64))
        else:
            status = p.remove(np.array(st["ids"], np.int64))
        assert status == st["status"], n
        d = p.check_state()
        mem = {str(l): v.tolist() for l, v in p.ref.membership().items()}
        assert mem == {k: sorted(v) for k, v in st["lists"].items()}, n
        assert int(((d["list_len"] + 1) // 2).sum()) == st["used_slabs"]
        for idk, row in st.get("rows", {}).items():
            got = p.gpu.get_rows(np.array([int(idk)])).cpu().numpy()[0]
            np.testing.assert_array_equal(got, np.array(row, np.float32))
    s = g["searches_after_last_step"]
    for case in s["cases"]:
        gd, gl = p.gpu.search(np.array([s["query"]], np.float32), case["k"], case["nprobe"])
        assert gl.cpu().numpy()[0].tolist() == case["ids"]
        assert gd.cpu().numpy()[0].tolist() == [float(v) for v in case["dist"]]


def test_golden_search_ip_gpu():
    g = json.load(open(os.path.join(GOLD, "search_ip_small.json")))
    cent = np.array(g["centroids"], np.float32)
    p = Pair(g["dim"], len(cent), cent, g["metric"], g["slab_capacity"], g["num_slabs"], g["id_capacity"],
             max_batch=16, max_queries=4, max_k=8, max_nprobe=4)
    assert p.add(np.array(g["add"]["x"], np.float32), np.array(g["add"]["ids"])) == 0
    p.check_state()
    for case in g["cases"]:
        gd, gl = p.gpu.search(np.array([g["query"]], np.float32), case["k"], case["nprobe"])
        assert gl.cpu().numpy()[0].tolist() == case["ids"]
        assert gd.cpu().numpy()[0].tolist() == [float(v) for v in case["dist"]]


# -------------------------------------------------------- tiny workload

def test_tiny_window_workload():
    """Tiny plain FP32 workload: 4,096 base vectors, d=32, 16 lists, slab 32,
    four window steps of +256 / -256 oldest, 64 queries, nprobe 4, k 10."""
    w = workloads.tiny()
    x, ids = w.base()
    q = w.queries()
    p = Pair(w.dim, w.nlist, w.centroids, w.metric, w.slab, num_slabs=400, id_capacity=8192,
             max_batch=4096, max_queries=64, max_k=16, max_nprobe=16)
    assert p.add(x, ids) == 0
    p.check_state()
    nbit = p.check_search(q, w.k, w.nprobe)
    for t in range(1, 5):
        xb, idb = w.stream_batch(t)
        assert p.add(xb, idb) == 0
        nbit += p.check_search(q, w.k, w.nprobe)
        assert p.remove(w.oldest_ids(t)) == 0
        p.check_state()
        nbit += p.check_search(q, 10, 16)       # all lists
    say(f"  distances differing in any bit: {nbit}")


def test_step_call_matches_separate_calls():
    w = workloads.tiny()
    x, ids = w.base()
    q = w.queries()
    p = Pair(w.dim, w.nlist, w.centroids, w.metric, w.slab, num_slabs=400, id_capacity=8192,
             max_batch=4096, max_queries=64, max_k=16, max_nprobe=16)
    assert p.add(x, ids) == 0
    for t in range(1, 4):
        xb, idb = w.stream_batch(t)
        old = w.oldest_ids(t)
        gd, gl, nrem = p.gpu.step(xb, idb, q, w.k, w.nprobe, old)
        assert p.gpu.sync() == 0
        assert p.ref.add(xb, idb) == 0
        st, rd, rl = p.ref.search(q, w.k, w.nprobe)
        st, rn = p.ref.remove(old)
        compare_results(gd.cpu().numpy(), gl.cpu().numpy(), rd, rl)
        assert int(nrem.item()) == rn
        p.check_state()


# -------------------------------------------------------- random op stress

@pytest.mark.parametrize("C,d,metric,seed", [(32, 5, 0, 1), (64, 32, 0, 2), (128, 17, 0, 3), (64, 24, 1, 4),
                                             (32, 64, 1, 5)])
def test_random_ops_vs_oracle(C, d, metric, seed):
    """Random batches of adds (fresh, upserts, duplicates within a batch) and
    removes (live, absent, repeated) on a small id space; state and search
    compared after every operation."""
    rng = np.random.default_rng([seed, 99])
    nlist = 11
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    cap = 3000
    p = Pair(d, nlist, cent, metric, C, num_slabs=2000, id_capacity=cap, max_batch=1024, max_queries=64,
             max_k=40, max_nprobe=16)
    q = rng.standard_normal((50, d)).astype(np.float32)
    for step in range(25):
        n = int(rng.integers(0, 700))
        ids = rng.integers(0, cap, n)
        x = rng.standard_normal((n, d)).astype(np.float32)
        if n > 10:
            x[:5] = x[5:10]                     # equal rows, different ids: equal distances
        assert p.add(x, ids) == 0
        p.check_state()
        rm = rng.integers(0, cap, int(rng.integers(0, 600)))
        assert p.remove(rm) == 0
        p.check_state()
        k = int(rng.integers(1, 41))
        p.check_search(q, k, int(rng.integers(1, 16)))
    kpq = rng.integers(0, 41, 50).astype(np.int32)
    npq = rng.integers(1, 17, 50).astype(np.int32)
    p.check_search(q, 40, 0, kpq=kpq, npq=npq)


def test_single_list_contention_and_drain():
    """Every vector lands in one list (maximum contention on one list's
    counters), then the list is drained to empty and refilled."""
    d, nlist = 16, 8
    rng = np.random.default_rng(5)
    cent = rng.standard_normal((nlist, d)).astype(np.float32) * 10
    p = Pair(d, nlist, cent, 0, 64, num_slabs=600, id_capacity=40000, max_batch=20000, max_queries=16,
             max_k=16, max_nprobe=8)
    x = np.tile(cent[3], (20000, 1)) + rng.standard_normal((20000, d)).astype(np.float32) * 0.01
    assert p.add(x, np.arange(20000)) == 0
    d0 = p.check_state()
    assert d0["list_len"][3] == 20000
    q = x[:16]
    p.check_search(q, 16, 2)
    order = rng.permutation(20000)
    for part in np.array_split(order, 5):
        assert p.remove(part) == 0
        p.check_state()
    assert p.gpu.stats()["live"] == 0 and p.gpu.stats()["used_slabs"] == 0
    assert p.add(x[:5000], np.arange(20000, 25000)) == 0
    p.check_state()
    p.check_search(q, 16, 8)


def test_errors_leave_state_unchanged():
    d, nlist = 8, 4
    rng = np.random.default_rng(6)
    cent = (np.eye(4, 8) * 10).astype(np.float32)
    p = Pair(d, nlist, cent, 0, 32, num_slabs=10, id_capacity=1000, max_batch=512, max_queries=8,
             max_k=8, max_nprobe=4)
    x = np.tile(cent[0], (330, 1)) + rng.standard_normal((330, 8)).astype(np.float32) * 0.1
    assert p.add(x[:320], np.arange(320)) == 0         # list 0: 10 full slabs = whole pool
    before = p.check_state()
    assert p.add(x[320:321], np.array([320])) == -2    # one more vector: NOSPACE
    assert p.add(x[:2], np.array([5, 1000])) == -3      # id out of range
    assert p.remove(np.array([1, -1])) == -3
    after = p.check_state()
    for k in ("list_len", "ids_by_list", "att"):
        np.testing.assert_array_equal(before[k], after[k])
    assert p.remove(np.array([7, 7, 7, 999, 998])) == 0   # duplicates and absent ids
    assert p.add(x[320:321], np.array([320])) == 0     # room again after the delete
    p.check_state()


def test_empty_and_padding_cases():
    d, nlist = 12, 6
    rng = np.random.default_rng(7)
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    for metric in (0, 1):
        p = Pair(d, nlist, cent, metric, 64, num_slabs=64, id_capacity=100, max_batch=100, max_queries=16,
                 max_k=64, max_nprobe=64)
        q = rng.standard_normal((5, d)).astype(np.float32)
        p.check_search(q, 10, 3)                         # empty index: all padding
        x = rng.standard_normal((7, d)).astype(np.float32)
        assert p.add(x, np.arange(7)) == 0
        p.check_search(q, 64, 64)                         # k > live, nprobe > nlist
        p.check_search(q, 1, 1)
        assert p.remove(np.arange(7)) == 0
        p.check_search(q, 5, 6)
        p.check_state()


def test_graph_replay_matches_oracle():
    """A window step captured once as a HIP graph and replayed on refilled
    buffers gives the oracle's results on every replay, with eager calls of
    the program between replays."""
    import torch
    w = workloads.tiny()
    x, ids = w.base()
    q = w.queries()
    p = Pair(w.dim, w.nlist, w.centroids, w.metric, w.slab, num_slabs=400, id_capacity=8192,
             max_batch=4096, max_queries=64, max_k=16, max_nprobe=16)
    assert p.add(x, ids) == 0
    dev = torch.device("cuda:0")
    xb = torch.empty((w.batch, w.dim), dtype=torch.float32, device=dev)
    ib = torch.empty(w.batch, dtype=torch.int64, device=dev)
    rb = torch.empty(w.batch, dtype=torch.int64, device=dev)
    qb = torch.from_numpy(q).to(dev)
    dist = torch.empty((q.shape[0], w.k), dtype=torch.float32, device=dev)
    lab = torch.empty((q.shape[0], w.k), dtype=torch.int64, device=dev)
    nrem = torch.zeros(1, dtype=torch.int64, device=dev)
    g = p.gpu.step_graph(xb, ib, qb, w.k, w.nprobe, rb, dist, lab, nrem)
    for t in range(1, 6):
        xt, it = w.stream_batch(t)
        xb.copy_(torch.from_numpy(xt))
        ib.copy_(torch.from_numpy(it))
        rb.copy_(torch.from_numpy(w.oldest_ids(t)))
        g.launch()
        assert p.gpu.sync() == 0
        assert p.ref.add(xt, it) == 0
        st, rd, rl = p.ref.search(q, w.k, w.nprobe)
        st, rn = p.ref.remove(w.oldest_ids(t))
        compare_results(dist.cpu().numpy(), lab.cpu().numpy(), rd, rl)
        assert int(nrem.item()) == rn
        p.check_state()
        p.check_search(q[:7], 12, 3)            # eager work between replays
    g.close()
