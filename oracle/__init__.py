"""CPU reference oracle for the streaming IVF index (ctypes binding).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, sequential
contiguous-array IVF written in C (``sivf_oracle.c``).  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import this module;
the GPU library never loads it, and the two share no code.

Every function here only marshals numpy arrays into the C routines; the
arithmetic lives in ``sivf_oracle.c`` where each routine cites the passage of
the paper it follows.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sivf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_NOSPACE, ERR_ID_RANGE = 0, -1, -2, -3
L2, IP = 0, 1

# Flags: no contraction, no fast-math, so every fma in the source is the only
# fused operation and FP32/FP64 rounding follows IEEE-754 step by step.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall"]


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (seconds)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ct.CDLL(_LIB)
        P = ct.c_void_p
        i32, i64 = ct.c_int32, ct.c_int64
        L.orc_coarse_dist.restype = ct.c_double
        L.orc_coarse_dist.argtypes = [P, P, ct.c_int, ct.c_int]
        L.orc_fine_dist.restype = ct.c_float
        L.orc_fine_dist.argtypes = [P, P, ct.c_int, ct.c_int]
        L.orc_assign.restype = None
        L.orc_assign.argtypes = [i64, P, ct.c_int, ct.c_int, P, ct.c_int, P]
        L.orc_probe.restype = None
        L.orc_probe.argtypes = [i64, P, ct.c_int, ct.c_int, P, ct.c_int, ct.c_int, P]
        L.orc_create.restype = P
        L.orc_create.argtypes = [ct.c_int, ct.c_int, P, ct.c_int, ct.c_int, i64, i64]
        L.orc_destroy.restype = None
        L.orc_destroy.argtypes = [P]
        L.orc_add.restype = ct.c_int
        L.orc_add.argtypes = [P, i64, P, P]
        L.orc_remove.restype = ct.c_int
        L.orc_remove.argtypes = [P, i64, P, P]
        L.orc_search.restype = ct.c_int
        L.orc_search.argtypes = [P, i64, P, ct.c_int, P, ct.c_int, P, P, P]
        L.orc_knn_live.restype = ct.c_int
        L.orc_knn_live.argtypes = [P, i64, P, ct.c_int, P, P]
        L.orc_used_slabs.restype = i64
        L.orc_used_slabs.argtypes = [P]
        L.orc_live.restype = i64
        L.orc_live.argtypes = [P]
        L.orc_list_len.restype = None
        L.orc_list_len.argtypes = [P, P]
        L.orc_ids_by_list.restype = None
        L.orc_ids_by_list.argtypes = [P, P]
        L.orc_list_of.restype = i32
        L.orc_list_of.argtypes = [P, i64]
        L.orc_row_of.restype = ct.c_int
        L.orc_row_of.argtypes = [P, i64, P]
        L.orc_num_threads.restype = ct.c_int
        L.orc_num_threads.argtypes = []
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def num_threads() -> int:
    return lib().orc_num_threads()


def coarse_dist(x, c, metric=L2) -> float:
    x, c = _f32(x), _f32(c)
    assert x.shape == c.shape and x.ndim == 1
    return lib().orc_coarse_dist(_ptr(x), _ptr(c), x.shape[0], metric)


def fine_dist(q, x, metric=L2) -> np.float32:
    q, x = _f32(q), _f32(x)
    assert q.shape == x.shape and q.ndim == 1
    return np.float32(lib().orc_fine_dist(_ptr(q), _ptr(x), q.shape[0], metric))


def assign(x, centroids, metric=L2) -> np.ndarray:
    x, c = _f32(x), _f32(centroids)
    out = np.empty(x.shape[0], dtype=np.int32)
    lib().orc_assign(x.shape[0], _ptr(x), x.shape[1], c.shape[0], _ptr(c), metric, _ptr(out))
    return out


def probe(q, centroids, m, metric=L2) -> np.ndarray:
    q, c = _f32(q), _f32(centroids)
    out = np.empty((q.shape[0], m), dtype=np.int32)
    lib().orc_probe(q.shape[0], _ptr(q), q.shape[1], c.shape[0], _ptr(c), metric, m, _ptr(out))
    return out


class OracleIndex:
    """Contiguous-array IVF with the GPU index's semantics (see sivf_oracle.c)."""

    def __init__(self, dim, nlist, centroids, metric=L2, slab_capacity=64,
                 num_slabs=1 << 20, id_capacity=1 << 20):
        c = _f32(centroids)
        assert c.shape == (nlist, dim)
        self.dim, self.nlist, self.metric = dim, nlist, metric
        self.slab_capacity, self.num_slabs, self.id_capacity = slab_capacity, num_slabs, id_capacity
        self._h = lib().orc_create(dim, nlist, _ptr(c), metric, slab_capacity, num_slabs, id_capacity)
        if not self._h:
            raise ValueError("orc_create rejected the configuration")

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def add(self, x, ids) -> int:
        x = _f32(x).reshape(-1, self.dim)
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        assert ids.shape[0] == x.shape[0]
        return lib().orc_add(self._h, ids.shape[0], _ptr(x), _ptr(ids))

    def remove(self, ids):
        """Returns (status, n_removed)."""
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        nr = ct.c_int64(0)
        st = lib().orc_remove(self._h, ids.shape[0], _ptr(ids), ct.byref(nr))
        return st, nr.value

    def search(self, q, k, nprobe, k_per_query=None, nprobe_per_query=None):
        """Returns (status, dist[nq,k] float32, labels[nq,k] int64)."""
        q = _f32(q).reshape(-1, self.dim)
        nq = q.shape[0]
        kpq = None if k_per_query is None else np.ascontiguousarray(k_per_query, dtype=np.int32)
        npq = None if nprobe_per_query is None else np.ascontiguousarray(nprobe_per_query, dtype=np.int32)
        dist = np.empty((nq, k), dtype=np.float32)
        lab = np.empty((nq, k), dtype=np.int64)
        st = lib().orc_search(self._h, nq, _ptr(q), k, _ptr(kpq), nprobe, _ptr(npq), _ptr(dist), _ptr(lab))
        return st, dist, lab

    def knn_exact(self, q, k):
        """Exact FP64 top-k over the live set: (dist[nq,k] float64, labels)."""
        q = _f32(q).reshape(-1, self.dim)
        dist = np.empty((q.shape[0], k), dtype=np.float64)
        lab = np.empty((q.shape[0], k), dtype=np.int64)
        lib().orc_knn_live(self._h, q.shape[0], _ptr(q), k, _ptr(dist), _ptr(lab))
        return dist, lab

    def used_slabs(self) -> int:
        return lib().orc_used_slabs(self._h)

    def live(self) -> int:
        return lib().orc_live(self._h)

    def list_len(self) -> np.ndarray:
        out = np.empty(self.nlist, dtype=np.int64)
        lib().orc_list_len(self._h, _ptr(out))
        return out

    def ids_by_list(self):
        """(list_len[nlist], ids concatenated per list, ascending within a list)."""
        ln = self.list_len()
        out = np.empty(int(ln.sum()), dtype=np.int64)
        lib().orc_ids_by_list(self._h, _ptr(out))
        return ln, out

    def membership(self) -> dict:
        """{list id: sorted id array} for non-empty lists."""
        ln, ids = self.ids_by_list()
        offs = np.concatenate([[0], np.cumsum(ln)])
        return {l: ids[offs[l]:offs[l + 1]] for l in range(self.nlist) if ln[l] > 0}

    def list_of(self, id_) -> int:
        return lib().orc_list_of(self._h, int(id_))

    def row_of(self, id_):
        out = np.empty(self.dim, dtype=np.float32)
        if lib().orc_row_of(self._h, int(id_), _ptr(out)) != 0:
            return None
        return out
