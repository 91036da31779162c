"""Streaming IVF index on AMD Instinct MI355X: Python binding of libsivf.

Thin ctypes layer over the C ABI in ``include/sivf.h``: every call marshals
torch tensors (device memory) and a HIP stream into the library, whose HIP
kernels do all of the work.  PyTorch only provides device memory and
streams.  There is no fallback: if ``libsivf.so`` is not built, or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsivf.so")

OK, ERR_ARG, ERR_NOSPACE, ERR_ID_RANGE, ERR_DEVICE, ERR_STATE, ERR_LIVE_ID, ERR_TOO_LARGE = 0, -1, -2, -3, -4, -5, -6, -7
L2, IP = 0, 1
F32, BF16, F16 = 0, 1, 2
DELETE_COMPACT, DELETE_LAZY = 0, 1


class SivfError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class SivfConfig(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("nlist", ct.c_int32), ("slab_capacity", ct.c_int32),
                ("metric", ct.c_int32), ("storage", ct.c_int32), ("rerank_factor", ct.c_int32),
                ("num_slabs", ct.c_int64), ("id_capacity", ct.c_int64),
                ("max_batch", ct.c_int32), ("max_queries", ct.c_int32),
                ("max_k", ct.c_int32), ("max_nprobe", ct.c_int32),
                ("delete_mode", ct.c_int32), ("reserved", ct.c_int32)]


class SivfStepArgs(ct.Structure):
    _fields_ = [("n_add", ct.c_int64), ("x", ct.c_void_p), ("add_ids", ct.c_void_p),
                ("nq", ct.c_int64), ("q", ct.c_void_p), ("k", ct.c_int32), ("nprobe", ct.c_int32),
                ("dist", ct.c_void_p), ("labels", ct.c_void_p),
                ("k_per_query", ct.c_void_p), ("nprobe_per_query", ct.c_void_p),
                ("n_remove", ct.c_int64), ("remove_ids", ct.c_void_p), ("n_removed", ct.c_void_p)]


class SivfDumpInfo(ct.Structure):
    _fields_ = [("live", ct.c_int64), ("used_slabs", ct.c_int64), ("free_slabs", ct.c_int64),
                ("num_slabs", ct.c_int64), ("id_capacity", ct.c_int64),
                ("nlist", ct.c_int32), ("slab_capacity", ct.c_int32), ("positions", ct.c_int64)]


class SivfMaintainReport(ct.Structure):
    _fields_ = [("compacted", ct.c_int64), ("reclaimed", ct.c_int64), ("offloaded_positions", ct.c_int64),
                ("offloaded_lists", ct.c_int32), ("reserved", ct.c_int32)]


# (name, restype, argtypes) of every exported entry point of include/sivf.h
_P, _I32, _I64 = ct.c_void_p, ct.c_int32, ct.c_int64
SIGNATURES = [
    ("sivf_workspace_bytes", ct.c_size_t, [ct.POINTER(SivfConfig)]),
    ("sivf_create", ct.c_int, [ct.POINTER(SivfConfig), _P, _P, ct.c_size_t, _P, ct.POINTER(_P)]),
    ("sivf_destroy", ct.c_int, [_P]),
    ("sivf_add", ct.c_int, [_P, _I64, _P, _P, _P]),
    ("sivf_remove", ct.c_int, [_P, _I64, _P, _P, _P]),
    ("sivf_search", ct.c_int, [_P, _I64, _P, _I32, _P, _I32, _P, _P, _P, _P]),
    ("sivf_tune_search", ct.c_int, [_P, _I64, _P, _I32, _P, _I32, _P, _P, _P, _P, ct.POINTER(_I32),
                                    ct.POINTER(_I32), ct.POINTER(_I32)]),
    ("sivf_set_search_schedule", ct.c_int, [_P, _I32, _I32, _I32]),
    ("sivf_set_deep_schedule", ct.c_int, [_P, _I32, _I32, _I32]),
    ("sivf_tier_bytes", ct.c_int, [_P, _I64, ct.POINTER(ct.c_size_t), ct.POINTER(ct.c_size_t)]),
    ("sivf_tier_attach", ct.c_int, [_P, _I64, _P, ct.c_size_t, _P, ct.c_size_t, _P]),
    ("sivf_tier_offload", ct.c_int, [_P, _I32, _P, ct.POINTER(_I64), _P]),
    ("sivf_tier_reclaim", ct.c_int, [_P, ct.POINTER(_I64), _P]),
    ("sivf_tier_stats", ct.c_int, [_P, ct.POINTER(_I64), ct.POINTER(_I64), ct.POINTER(_I64), ct.POINTER(_I64)]),
    ("sivf_tier_dump", ct.c_int, [_P, _P, _P]),
    ("sivf_list_heat", ct.c_int, [_P, _P, ct.c_int]),
    ("sivf_maintain", ct.c_int, [_P, ct.c_float, _I64, _I32, ct.POINTER(SivfMaintainReport), _P]),
    ("sivf_get_search_schedule", ct.c_int, [_P, _P]),
    ("sivf_step", ct.c_int, [_P, ct.POINTER(SivfStepArgs), _P]),
    ("sivf_graph_create", ct.c_int, [_P, ct.POINTER(SivfStepArgs), ct.POINTER(_P)]),
    ("sivf_graph_launch", ct.c_int, [_P, _P]),
    ("sivf_graph_destroy", ct.c_int, [_P]),
    ("sivf_assign", ct.c_int, [_P, _I64, _P, _P, _P]),
    ("sivf_compact", ct.c_int, [_P, ct.c_float, _P, _P]),
    ("sivf_probe", ct.c_int, [_P, _I64, _P, _I32, _P, _P]),
    ("sivf_probe_noalloc", ct.c_int, [_P, _I64, _P, _I32, _P, _P]),
    ("sivf_coarse_scores", ct.c_int, [_P, _I64, _P, _P, _P]),
    ("sivf_get_rows", ct.c_int, [_P, _I64, _P, _P, _P]),
    ("sivf_sync", ct.c_int, [_P, ct.POINTER(ct.c_int)]),
    ("sivf_stats", ct.c_int, [_P, ct.POINTER(_I64), ct.POINTER(_I64), ct.POINTER(_I64)]),
    ("sivf_dump_info_get", ct.c_int, [_P, ct.POINTER(SivfDumpInfo)]),
    ("sivf_dump", ct.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    ("sivf_profile_enable", ct.c_int, [_P, ct.c_int]),
    ("sivf_profile_read", ct.c_int, [_P, _P, _P]),
    ("sivf_server_create", ct.c_int, [_P, ct.POINTER(_P)]),
    ("sivf_server_destroy", ct.c_int, [_P]),
    ("sivf_server_add", ct.c_int, [_P, _I64, _P, _P, _P, ct.POINTER(_I64)]),
    ("sivf_server_remove", ct.c_int, [_P, _I64, _P, _P, _P, ct.POINTER(_I64)]),
    ("sivf_server_search", ct.c_int, [_P, _I64, _P, _I32, _I32, _P, _P, _P, ct.POINTER(_I64)]),
    ("sivf_server_poll", ct.c_int, [_P, _I64, ct.POINTER(ct.c_int)]),
    ("sivf_server_wait", ct.c_int, [_P, _I64]),
    ("sivf_server_free_slabs", ct.c_int, [_P, ct.POINTER(_I64), ct.POINTER(_I64)]),
    ("sivf_server_batches", ct.c_int, [_P, ct.POINTER(_I64), ct.POINTER(_I64)]),
    ("sivf_save", ct.c_int, [_P, ct.c_char_p]),
    ("sivf_checkpoint_config", ct.c_int, [ct.c_char_p, ct.POINTER(SivfConfig), ct.POINTER(_I64)]),
    ("sivf_load", ct.c_int, [ct.c_char_p, ct.POINTER(SivfConfig), _P, ct.c_size_t, _P, ct.POINTER(_P)]),
    ("sivf_registry_workspace_bytes", ct.c_size_t, [_P]),
    ("sivf_registry_create", ct.c_int, [_P, _P, ct.c_size_t, _P, ct.POINTER(_P)]),
    ("sivf_registry_destroy", ct.c_int, [_P]),
    ("sivf_registry_add", ct.c_int, [_P, _I64, _P, _P, _P]),
    ("sivf_registry_remove", ct.c_int, [_P, _I64, _P, _P, _P]),
    ("sivf_registry_search", ct.c_int, [_P, _I64, _P, _I32, _I32, _P, _P, _P]),
    ("sivf_registry_lookup", ct.c_int, [_P, _I64, _P, _P, _P]),
    ("sivf_registry_sync", ct.c_int, [_P, ct.POINTER(ct.c_int)]),
    ("sivf_registry_save", ct.c_int, [_P, ct.c_char_p]),
    ("sivf_registry_load", ct.c_int, [_P, ct.c_char_p, _P]),
    ("sivf_status_string", ct.c_char_p, [ct.c_int]),
]

_lib = None


def lib():
    """Load libsivf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                               "python paper_2601_11808_amd/build.py")
        L = ct.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(s: int) -> str:
    try:
        return lib().sivf_status_string(int(s)).decode()
    except Exception:
        return "status %d" % s


def _torch():
    import torch
    return torch


def _dev_tensor(a, dtype, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(np.asarray(a), device=device).to(dtype)
    return t.contiguous()


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _check(st, where):
    if st != OK:
        raise SivfError(st, where)


class Index:
    """A streaming IVF index held in one device workspace.

    Arguments mirror ``sivf_config``; ``centroids`` is (nlist, dim) float32.
    All methods take torch tensors (any device; they are moved to the index's
    device) or numpy arrays and enqueue on ``stream`` (default: torch's
    current stream of the device).
    """

    def __init__(self, dim, nlist, centroids, metric=L2, slab_capacity=64, num_slabs=1 << 16,
                 id_capacity=1 << 20, max_batch=1 << 16, max_queries=1 << 14, max_k=64,
                 max_nprobe=256, storage=F32, rerank_factor=0, device="cuda:0", stream=None,
                 delete_mode=DELETE_COMPACT, _checkpoint=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device is available")
        self.device = torch.device(device)
        self.cfg = SivfConfig(dim=dim, nlist=nlist, slab_capacity=slab_capacity, metric=metric,
                              storage=storage, rerank_factor=rerank_factor, num_slabs=num_slabs,
                              id_capacity=id_capacity,
                              max_batch=max_batch, max_queries=max_queries, max_k=max_k,
                              max_nprobe=max_nprobe, delete_mode=delete_mode, reserved=0)
        self.dim, self.nlist, self.metric, self.C = dim, nlist, metric, slab_capacity
        self.lazy = delete_mode == DELETE_LAZY
        nbytes = lib().sivf_workspace_bytes(ct.byref(self.cfg))
        if nbytes == 0:
            raise SivfError(ERR_ARG, "sivf_workspace_bytes (invalid configuration)")
        self.workspace_bytes = nbytes
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ct.c_void_p()
        if _checkpoint is not None:
            cent = None
            _check(lib().sivf_load(str(_checkpoint).encode(), ct.byref(self.cfg), _ptr(self.workspace), nbytes,
                                   self._stream(stream), ct.byref(h)), "sivf_load")
        else:
            cent = _dev_tensor(centroids, torch.float32, self.device)
            assert tuple(cent.shape) == (nlist, dim)
            _check(lib().sivf_create(ct.byref(self.cfg), _ptr(cent), _ptr(self.workspace), nbytes,
                                     self._stream(stream), ct.byref(h)), "sivf_create")
        self._h = h
        self._keep = [cent]
        self._stream(stream)
        self.sync()          # centroids copied: the caller's tensor may go

    @classmethod
    def load(cls, path, device="cuda:0", stream=None, **overrides):
        """An index from a checkpoint written by save().  Capacity arguments
        (num_slabs, id_capacity, slab_capacity, max_batch, max_queries, max_k,
        max_nprobe) may be overridden; the rest come from the file."""
        cfg, live = checkpoint_config(path)
        kw = {k: getattr(cfg, k) for k in ("metric", "slab_capacity", "num_slabs", "id_capacity", "max_batch",
                                            "max_queries", "max_k", "max_nprobe", "storage", "rerank_factor",
                                            "delete_mode")}
        kw.update(overrides)
        return cls(cfg.dim, cfg.nlist, None, device=device, stream=stream, _checkpoint=path, **kw)

    def save(self, path):
        """Write the index's logical content to a file (waits)."""
        _check(lib().sivf_save(self._h, str(path).encode()), "sivf_save")

    # -- helpers ---------------------------------------------------------
    def _stream(self, stream):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ct.c_void_p(s.cuda_stream)

    def close(self):
        if getattr(self, "_h", None):
            lib().sivf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- operations ------------------------------------------------------
    def add(self, x, ids, stream=None):
        torch = _torch()
        x = _dev_tensor(x, torch.float32, self.device).reshape(-1, self.dim)
        ids = _dev_tensor(ids, torch.int64, self.device).reshape(-1)
        assert ids.shape[0] == x.shape[0]
        _check(lib().sivf_add(self._h, x.shape[0], _ptr(x), _ptr(ids), self._stream(stream)), "sivf_add")
        self._keep = [x, ids]
        return self

    def remove(self, ids, stream=None):
        """Returns a device int64 scalar tensor with the number removed."""
        torch = _torch()
        ids = _dev_tensor(ids, torch.int64, self.device).reshape(-1)
        nrem = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(lib().sivf_remove(self._h, ids.shape[0], _ptr(ids), _ptr(nrem), self._stream(stream)),
               "sivf_remove")
        self._keep = [ids]
        return nrem

    def search(self, q, k, nprobe=1, k_per_query=None, nprobe_per_query=None, stream=None, out=None):
        torch = _torch()
        q = _dev_tensor(q, torch.float32, self.device).reshape(-1, self.dim)
        nq = q.shape[0]
        kpq = None if k_per_query is None else _dev_tensor(k_per_query, torch.int32, self.device)
        npq = None if nprobe_per_query is None else _dev_tensor(nprobe_per_query, torch.int32, self.device)
        if out is None:
            dist = torch.empty((nq, k), dtype=torch.float32, device=self.device)
            lab = torch.empty((nq, k), dtype=torch.int64, device=self.device)
        else:
            dist, lab = out
        _check(lib().sivf_search(self._h, nq, _ptr(q), k, _ptr(kpq), nprobe, _ptr(npq), _ptr(dist), _ptr(lab),
                                 self._stream(stream)), "sivf_search")
        self._keep = [q, kpq, npq]
        return dist, lab

    def tune_search(self, q, k, nprobe=1, k_per_query=None, nprobe_per_query=None, stream=None):
        """Pick the fastest search schedule for batches like this one; returns
        (queries per work item, log2 positions per work item, persistent waves)."""
        torch = _torch()
        q = _dev_tensor(q, torch.float32, self.device).reshape(-1, self.dim)
        kpq = None if k_per_query is None else _dev_tensor(k_per_query, torch.int32, self.device)
        npq = None if nprobe_per_query is None else _dev_tensor(nprobe_per_query, torch.int32, self.device)
        dist = torch.empty((q.shape[0], k), dtype=torch.float32, device=self.device)
        lab = torch.empty((q.shape[0], k), dtype=torch.int64, device=self.device)
        t, sh, pm = ct.c_int32(0), ct.c_int32(0), ct.c_int32(0)
        _check(lib().sivf_tune_search(self._h, q.shape[0], _ptr(q), k, _ptr(kpq), nprobe, _ptr(npq), _ptr(dist),
                                      _ptr(lab), self._stream(stream), ct.byref(t), ct.byref(sh), ct.byref(pm)),
               "sivf_tune_search")
        return t.value, sh.value, pm.value

    def set_search_schedule(self, tile, chunk_shift, persistent):
        _check(lib().sivf_set_search_schedule(self._h, tile, chunk_shift, int(persistent)),
               "sivf_set_search_schedule")

    def set_deep_schedule(self, tile, chunk_shift, persistent):
        """Schedule of the k > 64 pass of a certified-scan search."""
        _check(lib().sivf_set_deep_schedule(self._h, tile, chunk_shift, int(persistent)),
               "sivf_set_deep_schedule")

    def search_schedule(self):
        """((tile, chunk_shift, persistent), the same for the k > 64 pass)."""
        v = (ct.c_int32 * 6)()
        _check(lib().sivf_get_search_schedule(self._h, ct.cast(v, ct.c_void_p)), "sivf_get_search_schedule")
        return (v[0], v[1], v[2]), (v[3], v[4], v[5])

    def step(self, x=None, add_ids=None, q=None, k=10, nprobe=1, remove_ids=None, stream=None, out=None,
             k_per_query=None, nprobe_per_query=None):
        """add -> search -> remove; returns (dist, labels, n_removed)."""
        torch = _torch()
        a = SivfStepArgs()
        keep = []
        if x is not None:
            x = _dev_tensor(x, torch.float32, self.device).reshape(-1, self.dim)
            add_ids = _dev_tensor(add_ids, torch.int64, self.device).reshape(-1)
            a.n_add, a.x, a.add_ids = x.shape[0], x.data_ptr(), add_ids.data_ptr()
            keep += [x, add_ids]
        dist = lab = None
        if q is not None:
            q = _dev_tensor(q, torch.float32, self.device).reshape(-1, self.dim)
            if out is None:
                dist = torch.empty((q.shape[0], k), dtype=torch.float32, device=self.device)
                lab = torch.empty((q.shape[0], k), dtype=torch.int64, device=self.device)
            else:
                dist, lab = out
            a.nq, a.q, a.k, a.nprobe = q.shape[0], q.data_ptr(), k, nprobe
            a.dist, a.labels = dist.data_ptr(), lab.data_ptr()
            keep += [q]
            for name, v in (("k_per_query", k_per_query), ("nprobe_per_query", nprobe_per_query)):
                if v is not None:
                    v = _dev_tensor(v, torch.int32, self.device).reshape(-1)
                    setattr(a, name, v.data_ptr())
                    keep.append(v)
        nrem = torch.zeros(1, dtype=torch.int64, device=self.device)
        if remove_ids is not None:
            remove_ids = _dev_tensor(remove_ids, torch.int64, self.device).reshape(-1)
            a.n_remove, a.remove_ids = remove_ids.shape[0], remove_ids.data_ptr()
            keep += [remove_ids]
        a.n_removed = nrem.data_ptr()
        _check(lib().sivf_step(self._h, ct.byref(a), self._stream(stream)), "sivf_step")
        self._keep = keep
        return dist, lab, nrem

    def step_graph(self, x, add_ids, q, k, nprobe, remove_ids, dist, labels, n_removed, k_per_query=None,
                   nprobe_per_query=None):
        """Capture add -> search -> remove on these device buffers as a graph.
        Refill the buffers in place, then call ``launch()`` on the result."""
        return StepGraph(self, x, add_ids, q, k, nprobe, remove_ids, dist, labels, n_removed, k_per_query,
                         nprobe_per_query)

    def assign(self, x, stream=None):
        torch = _torch()
        x = _dev_tensor(x, torch.float32, self.device).reshape(-1, self.dim)
        out = torch.empty(x.shape[0], dtype=torch.int32, device=self.device)
        _check(lib().sivf_assign(self._h, x.shape[0], _ptr(x), _ptr(out), self._stream(stream)), "sivf_assign")
        self._keep = [x]
        return out

    def probe(self, q, nprobe, stream=None):
        torch = _torch()
        q = _dev_tensor(q, torch.float32, self.device).reshape(-1, self.dim)
        out = torch.empty((q.shape[0], nprobe), dtype=torch.int32, device=self.device)
        _check(lib().sivf_probe(self._h, q.shape[0], _ptr(q), nprobe, _ptr(out), self._stream(stream)),
               "sivf_probe")
        self._keep = [q]
        return out

    def probe_noalloc(self, q, nprobe, out=None, stream=None):
        """probe() whose scratch is the library's fixed device array (nothing is
        allocated by the library; `out` may be passed to allocate nothing here
        either)."""
        torch = _torch()
        q = _dev_tensor(q, torch.float32, self.device).reshape(-1, self.dim)
        if out is None:
            out = torch.empty((q.shape[0], nprobe), dtype=torch.int32, device=self.device)
        _check(lib().sivf_probe_noalloc(self._h, q.shape[0], _ptr(q), nprobe, _ptr(out), self._stream(stream)),
               "sivf_probe_noalloc")
        return out

    def coarse_scores(self, x, stream=None):
        torch = _torch()
        x = _dev_tensor(x, torch.float32, self.device).reshape(-1, self.dim)
        out = torch.empty((x.shape[0], self.nlist), dtype=torch.float32, device=self.device)
        _check(lib().sivf_coarse_scores(self._h, x.shape[0], _ptr(x), _ptr(out), self._stream(stream)),
               "sivf_coarse_scores")
        self._keep = [x]
        return out

    def compact(self, min_dead_fraction=0.0, stream=None):
        """Reclaim lazily deleted slots (see sivf_compact); returns a device
        int64 scalar with the number reclaimed by this call."""
        torch = _torch()
        n = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(lib().sivf_compact(self._h, float(min_dead_fraction), _ptr(n), self._stream(stream)), "sivf_compact")
        return n

    def get_rows(self, ids, stream=None):
        torch = _torch()
        ids = _dev_tensor(ids, torch.int64, self.device).reshape(-1)
        out = torch.empty((ids.shape[0], self.dim), dtype=torch.float32, device=self.device)
        _check(lib().sivf_get_rows(self._h, ids.shape[0], _ptr(ids), _ptr(out), self._stream(stream)),
               "sivf_get_rows")
        self._keep = [ids]
        return out

    def sync(self) -> int:
        """Wait; returns the first device-side status since the last sync."""
        st = ct.c_int(0)
        _check(lib().sivf_sync(self._h, ct.byref(st)), "sivf_sync")
        return st.value

    def check(self):
        """sync() and raise SivfError on a device-side failure."""
        st = self.sync()
        if st != OK:
            raise SivfError(st, "device")

    def stats(self):
        a, b, c = ct.c_int64(), ct.c_int64(), ct.c_int64()
        _check(lib().sivf_stats(self._h, ct.byref(a), ct.byref(b), ct.byref(c)), "sivf_stats")
        return {"live": a.value, "used_slabs": b.value, "free_slabs": c.value}

    PROF_KINDS = ("add", "remove", "search", "coarse", "scan", "merge", "scan_deep", "scan_cold")

    def profile(self, on=True):
        _check(lib().sivf_profile_enable(self._h, 1 if on else 0), "sivf_profile_enable")

    def profile_read(self):
        """{class: (total device ms, intervals)} since the last read (waits)."""
        ms = (ct.c_double * len(self.PROF_KINDS))()
        cnt = (ct.c_int64 * len(self.PROF_KINDS))()
        _check(lib().sivf_profile_read(self._h, ct.cast(ms, ct.c_void_p), ct.cast(cnt, ct.c_void_p)),
               "sivf_profile_read")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.PROF_KINDS)}

    def dump(self):
        """Host copy of the index state (numpy arrays), for validation."""
        info = SivfDumpInfo()
        _check(lib().sivf_dump_info_get(self._h, ct.byref(info)), "sivf_dump_info_get")
        out = {
            "list_len": np.empty(info.nlist, np.int32),
            "list_slabs": np.empty(info.used_slabs, np.int32),
            "ids_by_list": np.empty(info.positions, np.int64),
            "free_slabs": np.empty(info.free_slabs, np.int32),
            "slab_owner": np.empty(info.num_slabs, np.int32),
            "slab_ordinal": np.empty(info.num_slabs, np.int32),
            "att": np.empty(info.id_capacity, np.uint32),
        }
        c = lambda a: a.ctypes.data_as(ct.c_void_p)
        _check(lib().sivf_dump(self._h, c(out["list_len"]), c(out["list_slabs"]), c(out["ids_by_list"]),
                               c(out["free_slabs"]), c(out["slab_owner"]), c(out["slab_ordinal"]),
                               c(out["att"])), "sivf_dump")
        out["info"] = {k: getattr(info, k) for k, _ in SivfDumpInfo._fields_}
        return out

    def membership(self):
        """{list id: sorted id array} for non-empty lists (from a dump; with a
        host tier, device and cold entries together)."""
        d = self.dump()
        offs = np.concatenate([[0], np.cumsum(d["list_len"].astype(np.int64))])
        cold = self.tier_dump() if getattr(self, "_tier", None) is not None else None
        if cold is not None:
            coffs = np.concatenate([[0], np.cumsum(cold["cold_len"].astype(np.int64))])
        out = {}
        for l in range(self.nlist):
            v = d["ids_by_list"][offs[l]:offs[l + 1]]
            if cold is not None:
                v = np.concatenate([v, cold["cold_ids"][coffs[l]:coffs[l + 1]]])
            v = v[v >= 0]                      # lazily deleted slots read -1
            if v.shape[0]:
                out[l] = np.sort(v)
        return out

    # -- host tier -------------------------------------------------------
    def tier_attach(self, host_slabs, stream=None):
        """Attach a host tier of host_slabs cold slabs (pinned host memory for
        rows and ids, a device buffer for the rest; see sivf_tier_attach)."""
        torch = _torch()
        hb, db = ct.c_size_t(), ct.c_size_t()
        _check(lib().sivf_tier_bytes(self._h, int(host_slabs), ct.byref(hb), ct.byref(db)), "sivf_tier_bytes")
        host = torch.empty(hb.value, dtype=torch.uint8, pin_memory=True)
        dev = torch.empty(db.value, dtype=torch.uint8, device=self.device)
        _check(lib().sivf_tier_attach(self._h, int(host_slabs), _ptr(host), hb.value, _ptr(dev), db.value,
                                      self._stream(stream)), "sivf_tier_attach")
        self._tier = (host, dev)

    def tier_offload(self, lists, stream=None):
        """Move whole lists to the host tier; returns the positions moved."""
        arr = np.ascontiguousarray(np.asarray(lists, dtype=np.int32).reshape(-1))
        moved = ct.c_int64()
        _check(lib().sivf_tier_offload(self._h, arr.shape[0], arr.ctypes.data_as(ct.c_void_p), ct.byref(moved),
                                       self._stream(stream)), "sivf_tier_offload")
        return moved.value

    def tier_reclaim(self, stream=None):
        """Release dead cold segments; returns the positions released."""
        n = ct.c_int64()
        _check(lib().sivf_tier_reclaim(self._h, ct.byref(n), self._stream(stream)), "sivf_tier_reclaim")
        return n.value

    def tier_stats(self):
        v = [ct.c_int64() for _ in range(4)]
        _check(lib().sivf_tier_stats(self._h, *[ct.byref(x) for x in v]), "sivf_tier_stats")
        return dict(zip(("cold_live", "cold_positions", "cold_used_slabs", "cold_free_slabs"), (x.value for x in v)))

    def tier_dump(self):
        """{"cold_len": int32[nlist], "cold_ids": int64 ids by list (-1: dead)}."""
        clen = np.empty(self.nlist, np.int32)
        _check(lib().sivf_tier_dump(self._h, clen.ctypes.data_as(ct.c_void_p), None), "sivf_tier_dump")
        ids = np.empty(int(clen.astype(np.int64).sum()), np.int64)
        _check(lib().sivf_tier_dump(self._h, None, ids.ctypes.data_as(ct.c_void_p)), "sivf_tier_dump")
        return {"cold_len": clen, "cold_ids": ids}

    def list_heat(self, halve=False):
        h = np.empty(self.nlist, np.int32)
        _check(lib().sivf_list_heat(self._h, h.ctypes.data_as(ct.c_void_p), 1 if halve else 0), "sivf_list_heat")
        return h

    def maintain(self, min_dead_fraction=0.0, min_free_slabs=0, max_offload=0, stream=None):
        """Compaction, dead cold segments, and offload of the least probed
        lists below a free-slab mark (see sivf_maintain); returns its report."""
        r = SivfMaintainReport()
        _check(lib().sivf_maintain(self._h, float(min_dead_fraction), int(min_free_slabs), int(max_offload),
                                   ct.byref(r), self._stream(stream)), "sivf_maintain")
        return {k: getattr(r, k) for k, _ in SivfMaintainReport._fields_ if k != "reserved"}


def checkpoint_config(path):
    """(SivfConfig, live count) stored in a checkpoint file."""
    cfg, live = SivfConfig(), ct.c_int64()
    _check(lib().sivf_checkpoint_config(str(path).encode(), ct.byref(cfg), ct.byref(live)), "sivf_checkpoint_config")
    return cfg, live.value


class Registry:
    """External 64-bit ids over an index (see sivf_registry_* in
    include/sivf.h).  The index must be used only through the registry."""

    def __init__(self, index, stream=None):
        torch = _torch()
        self.index = index
        nbytes = lib().sivf_registry_workspace_bytes(index._h)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=index.device)
        h = ct.c_void_p()
        _check(lib().sivf_registry_create(index._h, _ptr(self.workspace), nbytes, index._stream(stream),
                                          ct.byref(h)), "sivf_registry_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().sivf_registry_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, x, ext_ids, stream=None):
        torch = _torch()
        ix = self.index
        x = _dev_tensor(x, torch.float32, ix.device).reshape(-1, ix.dim)
        ext_ids = _dev_tensor(ext_ids, torch.int64, ix.device).reshape(-1)
        assert ext_ids.shape[0] == x.shape[0]
        _check(lib().sivf_registry_add(self._h, x.shape[0], _ptr(x), _ptr(ext_ids), ix._stream(stream)),
               "sivf_registry_add")
        self._keep = (x, ext_ids)

    def remove(self, ext_ids, stream=None):
        torch = _torch()
        ix = self.index
        ext_ids = _dev_tensor(ext_ids, torch.int64, ix.device).reshape(-1)
        nrem = torch.zeros(1, dtype=torch.int64, device=ix.device)
        _check(lib().sivf_registry_remove(self._h, ext_ids.shape[0], _ptr(ext_ids), _ptr(nrem), ix._stream(stream)),
               "sivf_registry_remove")
        self._keep = (ext_ids,)
        return nrem

    def search(self, q, k, nprobe=1, stream=None):
        torch = _torch()
        ix = self.index
        q = _dev_tensor(q, torch.float32, ix.device).reshape(-1, ix.dim)
        dist = torch.empty((q.shape[0], k), dtype=torch.float32, device=ix.device)
        lab = torch.empty((q.shape[0], k), dtype=torch.int64, device=ix.device)
        _check(lib().sivf_registry_search(self._h, q.shape[0], _ptr(q), k, nprobe, _ptr(dist), _ptr(lab),
                                          ix._stream(stream)), "sivf_registry_search")
        self._keep = (q,)
        return dist, lab

    def lookup(self, ext_ids, stream=None):
        torch = _torch()
        ix = self.index
        ext_ids = _dev_tensor(ext_ids, torch.int64, ix.device).reshape(-1)
        out = torch.empty(ext_ids.shape[0], dtype=torch.int64, device=ix.device)
        _check(lib().sivf_registry_lookup(self._h, ext_ids.shape[0], _ptr(ext_ids), _ptr(out), ix._stream(stream)),
               "sivf_registry_lookup")
        self._keep = (ext_ids,)
        return out

    def sync(self) -> int:
        st = ct.c_int(0)
        _check(lib().sivf_registry_sync(self._h, ct.byref(st)), "sivf_registry_sync")
        return st.value

    def save(self, path):
        _check(lib().sivf_registry_save(self._h, str(path).encode()), "sivf_registry_save")

    def load(self, path, stream=None):
        _check(lib().sivf_registry_load(self._h, str(path).encode(), self.index._stream(stream)),
               "sivf_registry_load")


class StepGraph:
    """A window step captured as a HIP graph over fixed device buffers."""

    def __init__(self, index, x, add_ids, q, k, nprobe, remove_ids, dist, labels, n_removed, k_per_query=None,
                 nprobe_per_query=None):
        extra = tuple(t for t in (k_per_query, nprobe_per_query) if t is not None)
        for t in (x, add_ids, q, remove_ids, dist, labels, n_removed) + extra:
            assert t.is_cuda and t.is_contiguous()
        a = SivfStepArgs()
        a.n_add, a.x, a.add_ids = add_ids.shape[0], x.data_ptr(), add_ids.data_ptr()
        a.nq, a.q, a.k, a.nprobe = q.shape[0], q.data_ptr(), k, nprobe
        a.dist, a.labels = dist.data_ptr(), labels.data_ptr()
        if k_per_query is not None:
            assert k_per_query.dtype == _torch().int32
            a.k_per_query = k_per_query.data_ptr()
        if nprobe_per_query is not None:
            assert nprobe_per_query.dtype == _torch().int32
            a.nprobe_per_query = nprobe_per_query.data_ptr()
        a.n_remove, a.remove_ids, a.n_removed = remove_ids.shape[0], remove_ids.data_ptr(), n_removed.data_ptr()
        self.index = index
        self._bufs = (x, add_ids, q, remove_ids, dist, labels, n_removed) + extra
        h = ct.c_void_p()
        _check(lib().sivf_graph_create(index._h, ct.byref(a), ct.byref(h)), "sivf_graph_create")
        self._h = h

    def launch(self, stream=None):
        _check(lib().sivf_graph_launch(self._h, self.index._stream(stream)), "sivf_graph_launch")

    def close(self):
        if getattr(self, "_h", None):
            lib().sivf_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Overlapping request loop over one index (see sivf_server_* in
    include/sivf.h).  Submit methods return a ticket, or None when an insert
    is refused for lack of free slabs (nothing was enqueued; retry later).
    Device tensors of a request are kept alive until its ticket completes."""

    def __init__(self, index):
        self.index = index
        h = ct.c_void_p()
        _check(lib().sivf_server_create(index._h, ct.byref(h)), "sivf_server_create")
        self._h = h
        self._keep = {}

    def _in_stream(self):
        # inputs are produced (copied, generated) on torch's current stream
        return ct.c_void_p(_torch().cuda.current_stream(self.index.device).cuda_stream)

    def close(self):
        if getattr(self, "_h", None):
            lib().sivf_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, x, ids):
        torch = _torch()
        x = _dev_tensor(x, torch.float32, self.index.device).reshape(-1, self.index.dim)
        ids = _dev_tensor(ids, torch.int64, self.index.device).reshape(-1)
        t = ct.c_int64(0)
        st = lib().sivf_server_add(self._h, x.shape[0], _ptr(x), _ptr(ids), self._in_stream(), ct.byref(t))
        if st == ERR_NOSPACE:
            return None
        _check(st, "sivf_server_add")
        self._keep[t.value] = (x, ids)
        return t.value

    def remove(self, ids):
        """Returns (ticket, device int64 scalar with the number removed)."""
        torch = _torch()
        ids = _dev_tensor(ids, torch.int64, self.index.device).reshape(-1)
        nrem = torch.zeros(1, dtype=torch.int64, device=self.index.device)
        t = ct.c_int64(0)
        _check(lib().sivf_server_remove(self._h, ids.shape[0], _ptr(ids), _ptr(nrem), self._in_stream(),
                                        ct.byref(t)),
               "sivf_server_remove")
        self._keep[t.value] = (ids, nrem)
        return t.value, nrem

    def search(self, q, k, nprobe, out=None):
        """Returns (ticket, dist, labels); read them after the ticket completes.
        ticket is None when the search slots are full (nothing was enqueued;
        retry after a poll)."""
        torch = _torch()
        q = _dev_tensor(q, torch.float32, self.index.device).reshape(-1, self.index.dim)
        if out is None:
            dist = torch.empty((q.shape[0], k), dtype=torch.float32, device=self.index.device)
            lab = torch.empty((q.shape[0], k), dtype=torch.int64, device=self.index.device)
        else:
            dist, lab = out
        t = ct.c_int64(0)
        st = lib().sivf_server_search(self._h, q.shape[0], _ptr(q), k, nprobe, _ptr(dist), _ptr(lab),
                                      self._in_stream(), ct.byref(t))
        if st == ERR_NOSPACE:
            return None, dist, lab
        _check(st, "sivf_server_search")
        self._keep[t.value] = (q, dist, lab)
        return t.value, dist, lab

    def poll(self, ticket):
        d = ct.c_int(0)
        _check(lib().sivf_server_poll(self._h, ticket, ct.byref(d)), "sivf_server_poll")
        if d.value:
            self._keep.pop(ticket, None)
        return bool(d.value)

    def wait(self, ticket):
        _check(lib().sivf_server_wait(self._h, ticket), "sivf_server_wait")
        self._keep.pop(ticket, None)

    def free_slabs(self):
        f, r = ct.c_int64(), ct.c_int64()
        _check(lib().sivf_server_free_slabs(self._h, ct.byref(f), ct.byref(r)), "sivf_server_free_slabs")
        return f.value, r.value

    def batches(self):
        """(search batches launched, search requests they carried)."""
        b, r = ct.c_int64(), ct.c_int64()
        _check(lib().sivf_server_batches(self._h, ct.byref(b), ct.byref(r)), "sivf_server_batches")
        return b.value, r.value
