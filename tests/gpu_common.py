"""Helpers shared by the GPU parity tests: run the HIP library and the CPU
oracle on the same seeded inputs and compare."""
import sys

import numpy as np

import oracle
import paper_2601_11808_amd as sivf
from tests.invariants import check_dump, membership_of, same_membership

RTOL = 1e-5   # FP32 search distances: relative tolerance against the oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Pair:
    """A GPU index and an oracle index with identical configuration."""

    def __init__(self, dim, nlist, cent, metric=0, C=64, num_slabs=4096, id_capacity=1 << 16,
                 max_batch=8192, max_queries=1024, max_k=64, max_nprobe=64):
        self.C, self.num_slabs, self.dim, self.metric = C, num_slabs, dim, metric
        self.gpu = sivf.Index(dim, nlist, cent, metric=metric, slab_capacity=C, num_slabs=num_slabs,
                              id_capacity=id_capacity, max_batch=max_batch, max_queries=max_queries,
                              max_k=max_k, max_nprobe=max_nprobe)
        self.ref = oracle.OracleIndex(dim, nlist, cent, metric, C, num_slabs, id_capacity)

    def add(self, x, ids):
        self.gpu.add(x, ids)
        gs = self.gpu.sync()
        rs = self.ref.add(x, ids)
        assert gs == rs, (gs, rs)
        return gs

    def remove(self, ids):
        nr = self.gpu.remove(ids)
        gs = self.gpu.sync()
        rs, rn = self.ref.remove(ids)
        assert gs == rs, (gs, rs)
        if rs == 0:
            assert int(nr.item()) == rn, (int(nr.item()), rn)
        return gs

    def check_state(self):
        d = self.gpu.dump()
        check_dump(d, self.C, self.num_slabs)
        gm, om = membership_of(d), self.ref.membership()
        assert same_membership(gm, om), "membership differs from the oracle"
        st = self.gpu.stats()
        assert st["live"] == self.ref.live()
        assert st["used_slabs"] == self.ref.used_slabs()
        assert st["used_slabs"] + st["free_slabs"] == self.num_slabs
        return d

    def check_search(self, q, k, nprobe, kpq=None, npq=None):
        gd, gl = self.gpu.search(q, k, nprobe, k_per_query=kpq, nprobe_per_query=npq)
        assert self.gpu.sync() == 0
        st, rd, rl = self.ref.search(q, k, nprobe, k_per_query=kpq, nprobe_per_query=npq)
        assert st == 0
        return compare_results(gd.cpu().numpy(), gl.cpu().numpy(), rd, rl)


def compare_results(gd, gl, rd, rl):
    """Ids identical; distances within RTOL where finite, same padding.
    Returns the number of distances that differ in any bit."""
    np.testing.assert_array_equal(gl, rl)
    fin = np.isfinite(rd)
    np.testing.assert_array_equal(np.isfinite(gd), fin)
    np.testing.assert_array_equal(gd[~fin], rd[~fin])
    err = np.abs(gd[fin].astype(np.float64) - rd[fin]) / np.maximum(np.abs(rd[fin]).astype(np.float64), 1e-30)
    assert (err <= RTOL).all(), float(err.max())
    return int((gd.view(np.uint32) != rd.view(np.uint32)).sum())
