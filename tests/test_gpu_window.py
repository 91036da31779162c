"""Full-size parity on the sliding-window workload (1,000,000 x 128 fp32,
1,024 lists, slab 64) in the launch configuration the benchmark times:
bulk load in 65,536-vector batches, then window steps of +10,000 / 10,000
queries (nprobe 32, k 10) / -10,000 oldest.

Membership is compared in full (every id of the window); search is compared
on a seeded sample of queries, which the oracle evaluates one by one.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2601_11808_amd as sivf
import workloads
from tests.gpu_common import compare_results, say
from tests.invariants import check_dump, membership_of, same_membership

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def window():
    w = workloads.window()
    x, ids = w.base()
    return w, x, ids, w.queries()


def test_window_full_size(window):
    w, x, ids, q = window
    dev = torch.device("cuda:0")
    steps = 2
    num_slabs = int(1.15 * (w.n_base + 2 * w.batch) / w.slab) + w.nlist
    ix = sivf.Index(w.dim, w.nlist, w.centroids, metric=w.metric, slab_capacity=w.slab, num_slabs=num_slabs,
                    id_capacity=w.n_base + w.batch * (steps + 2), max_batch=65536, max_queries=w.n_queries,
                    max_k=16, max_nprobe=128)
    xd, idd = torch.from_numpy(x).to(dev), torch.from_numpy(ids).to(dev)
    for s in range(0, x.shape[0], 65536):
        ix.add(xd[s:s + 65536], idd[s:s + 65536])
    assert ix.sync() == 0
    say("  gpu bulk load done")
    ref = oracle.OracleIndex(w.dim, w.nlist, w.centroids, w.metric, w.slab, num_slabs,
                             w.n_base + w.batch * (steps + 2))
    assert ref.add(x, ids) == 0
    say("  oracle bulk load done")
    d = ix.dump()
    check_dump(d, w.slab, num_slabs)
    assert same_membership(membership_of(d), ref.membership())
    rng = np.random.default_rng(2024)
    qs = np.sort(rng.choice(w.n_queries, size=300, replace=False))
    qd = torch.from_numpy(q).to(dev)
    for t in range(1, steps + 1):
        xb, idb = w.stream_batch(t)
        old = w.oldest_ids(t)
        gd, gl, nrem = ix.step(xb, idb, qd, w.k, w.nprobe, old)
        assert ix.sync() == 0
        assert ref.add(xb, idb) == 0
        st, rd, rl = ref.search(q[qs], w.k, w.nprobe)
        st, rn = ref.remove(old)
        assert int(nrem.item()) == rn == w.batch
        nbit = compare_results(gd.cpu().numpy()[qs], gl.cpu().numpy()[qs], rd, rl)
        d = ix.dump()
        check_dump(d, w.slab, num_slabs)
        assert same_membership(membership_of(d), ref.membership())
        say(f"  step {t}: membership exact, {len(qs)} sampled queries identical "
            f"({nbit} distances differ in any bit)")
    # probes at full size match the oracle on a sample
    gp = ix.probe(qd[:2000], w.nprobe).cpu().numpy()
    np.testing.assert_array_equal(gp, oracle.probe(q[:2000], w.centroids, w.nprobe, w.metric))
