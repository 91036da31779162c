"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: exact rational IEEE
models of its distance definitions, integer-valued inputs whose distances are
exact in any summation order (so numpy brute force is an independent
reference), hand-derived golden sequences, and invariants.  Each test names
the mistake it is there to catch.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests.ieee_model import F, r32, r64

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- distances

def _model_fine_l2(q, x):
    r = Fraction(0)
    for a, b in zip(q, x):
        t = r32(F(a) - F(b))
        r = r32(t * t + r)           # one rounding: fused multiply-add
    return r


def _model_fine_ip(q, x):
    r = Fraction(0)
    for a, b in zip(q, x):
        r = r32(F(a) * F(b) + r)
    return r


def _model_coarse_l2(x, c):
    r = Fraction(0)
    for a, b in zip(x, c):
        t = r64(F(a) - F(b))
        r = r64(t * t + r)
    return r


def _model_coarse_ip(x, c):
    r = Fraction(0)
    for a, b in zip(x, c):
        r = r64(F(a) * F(b) + r)
    return -r


def _unfused_l2(q, x):
    r = Fraction(0)
    for a, b in zip(q, x):
        t = r32(F(a) - F(b))
        r = r32(r32(t * t) + r)
    return r


def _reversed_l2(q, x):
    return _model_fine_l2(q[::-1], x[::-1])


def test_fine_distance_matches_exact_ieee_model():
    """Catches: a non-fused multiply-add, a different summation order, a
    dropped term, or IP/L2 mixed up in the FP32 fine distance."""
    rng = np.random.default_rng(11)
    differs_unfused = differs_order = 0
    for trial in range(60):
        d = int(rng.integers(1, 24))
        q = rng.standard_normal(d).astype(np.float32) * np.float32(3.0)
        x = rng.standard_normal(d).astype(np.float32) * np.float32(3.0)
        want = _model_fine_l2(q, x)
        got = oracle.fine_dist(q, x, oracle.L2)
        assert Fraction(float(got)) == want, (trial, d)
        differs_unfused += _unfused_l2(q, x) != want
        differs_order += _reversed_l2(q, x) != want
        want_ip = _model_fine_ip(q, x)
        assert Fraction(float(oracle.fine_dist(q, x, oracle.IP))) == want_ip
    # the model is sharp enough to tell the variants apart on these inputs
    assert differs_unfused > 5 and differs_order > 5


def test_coarse_distance_matches_exact_ieee_model():
    """Catches: FP32 instead of FP64 accumulation, unfused updates, wrong sign
    convention for IP (smaller must mean closer)."""
    rng = np.random.default_rng(12)
    for trial in range(40):
        d = int(rng.integers(1, 20))
        x = rng.standard_normal(d).astype(np.float32)
        c = rng.standard_normal(d).astype(np.float32)
        assert Fraction(oracle.coarse_dist(x, c, oracle.L2)) == _model_coarse_l2(x, c)
        assert Fraction(oracle.coarse_dist(x, c, oracle.IP)) == _model_coarse_ip(x, c)


def test_distances_integer_data_exact():
    """Integer-valued rows (the window workload's 0..255 values, d=128): every
    partial sum is an integer below 2^24, so FP32 and FP64 are exact in any
    order and must equal the integer distance."""
    rng = np.random.default_rng(13)
    for _ in range(50):
        q = rng.integers(0, 256, 128)
        x = rng.integers(0, 256, 128)
        exact = int(((q - x) ** 2).sum())
        assert float(oracle.fine_dist(q, x, oracle.L2)) == exact
        assert oracle.coarse_dist(q, x, oracle.L2) == exact
        dot = int((q * x).sum())
        assert oracle.coarse_dist(q, x, oracle.IP) == -dot


# ---------------------------------------------------------- coarse quantizer

def _int_case(seed, n, nlist, d, dup=True):
    rng = np.random.default_rng(seed)
    cent = rng.integers(0, 16, (nlist, d)).astype(np.float32)
    if dup:
        cent[nlist // 2] = cent[1]           # exact duplicate: ties
        cent[nlist - 1] = cent[0]
    x = rng.integers(0, 16, (n, d)).astype(np.float32)
    x[:4] = cent[[0, 1, 3, nlist - 1]]       # points equal to a centroid
    return x, cent


def test_assign_equals_integer_bruteforce_with_ties():
    """Catches: argmax instead of argmin, a tie going to the larger list id, a
    transposed operand, an off-by-one over the list range."""
    x, cent = _int_case(21, 3000, 37, 8)
    exact = ((x[:, None, :].astype(np.int64) - cent[None].astype(np.int64)) ** 2).sum(-1)
    want = exact.argmin(1)                  # numpy argmin keeps the first minimum
    got = oracle.assign(x, cent)
    np.testing.assert_array_equal(got, want)
    assert got[0] == 0 and got[1] == 1 and got[3] == 0   # duplicates -> lower id
    assert (exact.min(1) == exact[np.arange(len(x)), got]).all()


def test_assign_ip_integer_bruteforce():
    x, cent = _int_case(22, 2000, 29, 6)
    x -= 8
    cent -= 8
    sc = (x[:, None, :].astype(np.int64) * cent[None].astype(np.int64)).sum(-1)
    want = np.argmax(sc, 1)                 # first maximum = smallest list id
    np.testing.assert_array_equal(oracle.assign(x, cent, oracle.IP), want)


@pytest.mark.parametrize("m", [1, 3, 8, 37, 50])
def test_probe_order_equals_integer_lexsort(m):
    """Probe set = first m lists by (distance, list id)."""
    x, cent = _int_case(23, 500, 37, 8)
    exact = ((x[:, None, :].astype(np.int64) - cent[None].astype(np.int64)) ** 2).sum(-1)
    got = oracle.probe(x, cent, m)
    mm = min(m, 37)
    for i in range(len(x)):
        order = np.lexsort((np.arange(37), exact[i]))
        np.testing.assert_array_equal(got[i, :mm], order[:mm])
        assert (got[i, mm:] == -1).all()


# ------------------------------------------------------------------ mutation

def _membership(ix):
    return {str(k): v.tolist() for k, v in ix.membership().items()}


def test_golden_mutation_sequence():
    """Hand-derived states after every operation (upsert, duplicate ids in a
    batch, idempotent and duplicate removes, pool exhaustion, id range)."""
    g = json.load(open(os.path.join(GOLD, "mutation_small.json")))
    ix = oracle.OracleIndex(g["dim"], len(g["centroids"]), np.array(g["centroids"], np.float32),
                            g["metric"], g["slab_capacity"], g["num_slabs"], g["id_capacity"])
    for n, st in enumerate(g["steps"]):
        if st["op"] == "add":
            status = ix.add(np.array(st["x"], np.float32), np.array(st["ids"], np.int64))
        else:
            status, nrem = ix.remove(np.array(st["ids"], np.int64))
            if "n_removed" in st:
                assert nrem == st["n_removed"], n
        assert status == st["status"], n
        assert _membership(ix) == {k: sorted(v) for k, v in st["lists"].items()}, n
        assert ix.used_slabs() == st["used_slabs"], n
        for idk, row in st.get("rows", {}).items():
            np.testing.assert_array_equal(ix.row_of(int(idk)), np.array(row, np.float32))
    s = g["searches_after_last_step"]
    for case in s["cases"]:
        status, dist, lab = ix.search(np.array([s["query"]], np.float32), case["k"], case["nprobe"])
        assert status == 0
        assert lab[0].tolist() == case["ids"]
        assert dist[0].tolist() == [float(v) for v in case["dist"]]


def test_golden_search_ip():
    g = json.load(open(os.path.join(GOLD, "search_ip_small.json")))
    ix = oracle.OracleIndex(g["dim"], len(g["centroids"]), np.array(g["centroids"], np.float32),
                            g["metric"], g["slab_capacity"], g["num_slabs"], g["id_capacity"])
    assert ix.add(np.array(g["add"]["x"], np.float32), np.array(g["add"]["ids"])) == 0
    assert _membership(ix) == g["lists"]
    for case in g["cases"]:
        st, dist, lab = ix.search(np.array([g["query"]], np.float32), case["k"], case["nprobe"])
        assert st == 0
        assert lab[0].tolist() == case["ids"]
        assert dist[0].tolist() == [float(v) for v in case["dist"]]


def test_random_ops_invariants():
    """Random add/upsert/remove sequence: each live id sits in the list of its
    nearest centroid, exactly once; sum of lengths = live; used slabs =
    sum ceil(len/C); removed ids are absent."""
    rng = np.random.default_rng(31)
    d, nlist, C = 6, 9, 4
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    ix = oracle.OracleIndex(d, nlist, cent, oracle.L2, C, num_slabs=10_000, id_capacity=300)
    live = {}
    for step in range(40):
        nadd = int(rng.integers(0, 30))
        ids = rng.integers(0, 300, nadd)
        x = rng.standard_normal((nadd, d)).astype(np.float32)
        assert ix.add(x, ids) == 0
        for i, u in enumerate(ids):
            live[int(u)] = x[i]
        rem = rng.integers(0, 300, int(rng.integers(0, 25)))
        st, nr = ix.remove(rem)
        assert st == 0
        gone = {int(u) for u in rem if int(u) in live}
        assert nr == len(gone)
        for u in gone:
            del live[u]
        mem = ix.membership()
        allids = np.concatenate([v for v in mem.values()]) if mem else np.zeros(0, np.int64)
        assert sorted(allids.tolist()) == sorted(live)
        assert ix.live() == len(live)
        for l, v in mem.items():
            for u in v:
                assert oracle.assign(live[int(u)][None], cent)[0] == l
                np.testing.assert_array_equal(ix.row_of(int(u)), live[int(u)])
        ln = ix.list_len()
        assert ix.used_slabs() == int(sum((n + C - 1) // C for n in ln))


def test_nospace_leaves_state_unchanged():
    rng = np.random.default_rng(32)
    d, nlist, C = 4, 3, 8
    cent = np.eye(3, 4, dtype=np.float32) * 10
    ix = oracle.OracleIndex(d, nlist, cent, oracle.L2, C, num_slabs=3, id_capacity=100)
    x = np.tile(cent[0], (8, 1)) + rng.standard_normal((8, 4)).astype(np.float32) * 0.1
    assert ix.add(x, np.arange(8)) == 0                     # list 0: 8 entries, 1 slab
    before = _membership(ix)
    x2 = np.tile(cent[0], (17, 1)).astype(np.float32)
    assert ix.add(x2, np.arange(8, 25)) == oracle.ERR_NOSPACE  # would need 4 slabs
    assert _membership(ix) == before
    assert ix.add(x2[:16], np.arange(8, 24)) == 0              # exactly 3 slabs
    assert ix.used_slabs() == 3


# -------------------------------------------------------------------- search

def _int_index(seed, n, nlist, d, C=4, metric=oracle.L2):
    rng = np.random.default_rng(seed)
    cent = rng.integers(0, 32, (nlist, d)).astype(np.float32)
    x = rng.integers(0, 32, (n, d)).astype(np.float32)
    x[n // 2: n // 2 + 20] = x[:20]                 # duplicate rows: equal distances
    ix = oracle.OracleIndex(d, nlist, cent, metric, C, num_slabs=100_000, id_capacity=n)
    assert ix.add(x, np.arange(n)) == 0
    return ix, x, cent


def _brute_int(x, q, ids, k, metric=oracle.L2):
    xi = x.astype(np.int64)
    out_d, out_i = [], []
    for qq in q.astype(np.int64):
        if metric == oracle.L2:
            dd = ((xi - qq) ** 2).sum(1)
            order = np.lexsort((ids, dd))
        else:
            dd = (xi * qq).sum(1)
            order = np.lexsort((ids, -dd))
        order = order[:k]
        out_d.append(dd[order])
        out_i.append(ids[order])
    return np.array(out_d), np.array(out_i)


def test_search_full_probe_equals_bruteforce():
    """nprobe = nlist is exact kNN over the live set (textbook special case);
    integer data makes the reference exact, ties resolve to the smaller id."""
    ix, x, cent = _int_index(41, 2000, 13, 10)
    rng = np.random.default_rng(42)
    q = rng.integers(0, 32, (40, 10)).astype(np.float32)
    q[:5] = x[:5]
    st, dist, lab = ix.search(q, 15, 13)
    assert st == 0
    wd, wi = _brute_int(x, q, np.arange(2000), 15)
    np.testing.assert_array_equal(lab, wi)
    np.testing.assert_array_equal(dist, wd.astype(np.float32))


def test_search_nlist1_is_flat_and_ip():
    rng = np.random.default_rng(43)
    x = rng.integers(-8, 8, (700, 5)).astype(np.float32)
    cent = np.zeros((1, 5), np.float32)
    for metric in (oracle.L2, oracle.IP):
        ix = oracle.OracleIndex(5, 1, cent, metric, 64, 1000, 700)
        assert ix.add(x, np.arange(700)) == 0
        q = rng.integers(-8, 8, (20, 5)).astype(np.float32)
        st, dist, lab = ix.search(q, 12, 1)
        wd, wi = _brute_int(x, q, np.arange(700), 12, metric)
        np.testing.assert_array_equal(lab, wi)
        np.testing.assert_array_equal(dist, wd.astype(np.float32))


def test_search_restricted_probes_bruteforce():
    """With nprobe < nlist the result is exact kNN over the union of the probe
    lists (computed here from integer brute force on the probe set)."""
    ix, x, cent = _int_index(44, 3000, 17, 8)
    rng = np.random.default_rng(45)
    q = rng.integers(0, 32, (30, 8)).astype(np.float32)
    lists = oracle.assign(x, cent)
    st, dist, lab = ix.search(q, 10, 3)
    exact_c = ((q[:, None, :].astype(np.int64) - cent[None].astype(np.int64)) ** 2).sum(-1)
    for i in range(len(q)):
        probes = np.lexsort((np.arange(17), exact_c[i]))[:3]
        sel = np.flatnonzero(np.isin(lists, probes))
        wd, wi = _brute_int(x[sel], q[i:i + 1], sel.astype(np.int64), 10)
        np.testing.assert_array_equal(lab[i], wi[0])
        np.testing.assert_array_equal(dist[i], wd[0].astype(np.float32))


def test_search_padding_per_query_k_and_nprobe():
    ix, x, cent = _int_index(46, 50, 5, 4)
    q = x[:6]
    kpq = np.array([0, 1, 5, 20, 60, 3], np.int32)
    npq = np.array([1, 2, 5, 9, 5, 1], np.int32)
    st, dist, lab = ix.search(q, 60, 0, k_per_query=kpq, nprobe_per_query=npq)
    assert st == 0
    for i in range(6):
        st1, d1, l1 = ix.search(q[i:i + 1], int(kpq[i]) if kpq[i] else 1, int(npq[i]))
        kk = int(kpq[i])
        np.testing.assert_array_equal(lab[i, :kk], l1[0, :kk])
        assert (lab[i, kk:] == -1).all() and np.isinf(dist[i, kk:]).all()
    # query 4 asks for 60 of 50 live entries over all lists
    assert (lab[4, :50] >= 0).all() and (lab[4, 50:] == -1).all()


def test_deleted_never_returned_and_exact_knn():
    ix, x, cent = _int_index(47, 1500, 7, 6)
    rm = np.arange(0, 1500, 3)
    st, nr = ix.remove(rm)
    assert nr == len(rm)
    q = x[:30]
    st, dist, lab = ix.search(q, 10, 7)
    assert not np.isin(lab, rm).any()
    keep = np.setdiff1d(np.arange(1500), rm)
    wd, wi = _brute_int(x[keep], q, keep, 10)
    np.testing.assert_array_equal(lab, wi)
    kd, ki = ix.knn_exact(q, 10)                       # FP64 exact, same ties
    np.testing.assert_array_equal(ki, wi)
    np.testing.assert_array_equal(kd, wd.astype(np.float64))


def test_knn_exact_ip_bruteforce_before_and_after_deletes():
    """The inner-product branch of the FP64 exact kNN (the recall ground truth
    of the inner-product precision form): on integer data every product and
    partial sum is exact, so numpy brute force ranked by descending score,
    ties to the smaller id, is an independent reference.  Duplicated rows
    give exact ties; signed values give negative scores (a sign slip in the
    score, or an ascending order, fails)."""
    rng = np.random.default_rng(48)
    n, d, nlist = 1800, 9, 6
    cent = rng.integers(-16, 17, (nlist, d)).astype(np.float32)
    x = rng.integers(-16, 17, (n, d)).astype(np.float32)
    x[n // 2: n // 2 + 30] = x[:30]
    ix = oracle.OracleIndex(d, nlist, cent, oracle.IP, 8, num_slabs=100_000, id_capacity=n)
    assert ix.add(x, np.arange(n)) == 0
    q = rng.integers(-16, 17, (25, d)).astype(np.float32)
    q[:4] = x[:4]
    q[4] = -x[5]
    for live in (np.arange(n), None):
        if live is None:
            rm = rng.choice(n, n // 3, replace=False)
            st, nr = ix.remove(rm)
            assert st == 0 and nr == len(rm)
            live = np.setdiff1d(np.arange(n), rm)
        kd, ki = ix.knn_exact(q, 12)
        wd, wi = _brute_int(x[live], q, live.astype(np.int64), 12, metric=oracle.IP)
        np.testing.assert_array_equal(ki, wi)
        np.testing.assert_array_equal(kd, wd.astype(np.float64))
        assert (np.diff(kd, axis=1) <= 0).all()          # scores descending
    # more results asked for than live entries: padding with -1 and -inf
    small = oracle.OracleIndex(d, nlist, cent, oracle.IP, 8, num_slabs=100, id_capacity=n)
    assert small.add(x[:3], np.arange(3)) == 0
    kd, ki = small.knn_exact(q[:2], 5)
    wd, wi = _brute_int(x[:3], q[:2], np.arange(3), 3, metric=oracle.IP)
    np.testing.assert_array_equal(ki[:, :3], wi)
    assert (ki[:, 3:] == -1).all() and (kd[:, 3:] == -np.inf).all()


def test_ip_signed_zero_scores_tie_on_id():
    """An inner product of tiny values rounds to -0 or +0 with the sign of the
    exact sum; both are the score 0, so the order among them is by id alone.
    Catches a ranking on the raw sign bit (which would put every +0 first)."""
    rng = np.random.default_rng(47)
    n, d = 300, 3
    x = (rng.choice([-1.0, 1.0], (n, d)) * 1e-30).astype(np.float32)
    ix = oracle.OracleIndex(d, 1, np.zeros((1, d), np.float32), oracle.IP, 64, 100, n)
    assert ix.add(x, rng.permutation(n).astype(np.int64)) == 0
    q = np.full((4, d), 1e-30, np.float32)
    st, dist, lab = ix.search(q, 20, 1)
    assert st == 0
    signs = {bool(np.signbit(v)) for v in dist.ravel()}
    assert (dist == 0).all() and signs == {False, True}, "the sample must mix -0 and +0 scores"
    np.testing.assert_array_equal(lab, np.tile(np.arange(20), (4, 1)))
