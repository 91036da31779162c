"""Host-side checks of the C ABI and of the dump validator (no GPU needed)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import paper_2601_11808_amd as sivf
from tests.invariants import check_dump

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sivf.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sivf_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sivf.LIB_PATH):
        from paper_2601_11808_amd import build
        build.build()
    return sivf.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in sivf.SIGNATURES}
    assert set(names) == bound, set(names) ^ bound


def test_struct_layouts_match_header():
    # sizes follow from the field lists in include/sivf.h (natural alignment)
    assert ct.sizeof(sivf.SivfConfig) == 6 * 4 + 2 * 8 + 6 * 4
    assert ct.sizeof(sivf.SivfStepArgs) == 8 + 8 + 8 + 8 + 8 + 4 + 4 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert ct.sizeof(sivf.SivfDumpInfo) == 5 * 8 + 2 * 4 + 8
    assert ct.sizeof(sivf.SivfMaintainReport) == 3 * 8 + 2 * 4


def _cfg(**kw):
    base = dict(dim=128, nlist=1024, slab_capacity=64, metric=0, storage=0, rerank_factor=0,
                num_slabs=20000, id_capacity=1 << 21, max_batch=65536, max_queries=10000,
                max_k=16, max_nprobe=64)
    base.update(kw)
    return sivf.SivfConfig(**base)


def test_workspace_bytes_and_config_validation(lib):
    c = _cfg()
    nb = lib.sivf_workspace_bytes(ct.byref(c))
    pool = 20000 * 64 * (128 * 4 + 4)
    assert nb > pool and nb < pool + (1 << 30)
    bad = [dict(dim=0), dict(nlist=0), dict(slab_capacity=48), dict(slab_capacity=256), dict(slab_capacity=0), dict(metric=2), dict(storage=3), dict(storage=1), dict(rerank_factor=2),
           dict(storage=1, rerank_factor=8, max_k=16), dict(storage=1, rerank_factor=4, dim=512),
           dict(storage=1, rerank_factor=4, slab_capacity=8),
           dict(num_slabs=0), dict(id_capacity=0), dict(max_k=129), dict(max_k=0), dict(storage=1, rerank_factor=1, max_k=65), dict(max_nprobe=0),
           dict(max_nprobe=2000), dict(num_slabs=1 << 30)]
    for b in bad:
        assert lib.sivf_workspace_bytes(ct.byref(_cfg(**b))) == 0, b
    h = ct.c_void_p()
    st = lib.sivf_create(ct.byref(_cfg(dim=0)), ct.c_void_p(1 << 20), ct.c_void_p(1 << 20), 1 << 30, None,
                         ct.byref(h))
    assert st == sivf.ERR_ARG and not h.value
    assert lib.sivf_status_string(-2).decode() == "slab pool exhausted"


def _good_dump():
    # C=2, pool of 6 slabs; list 0: ids [5, 7, 1] in slabs [4, 0]; list 1: id [2] in slab [3]
    C = 2
    d = {
        "list_len": np.array([3, 1], np.int32),
        "list_slabs": np.array([4, 0, 3], np.int32),
        "ids_by_list": np.array([5, 7, 1, 2], np.int64),
        "free_slabs": np.array([1, 2, 5], np.int32),
        "slab_owner": np.array([0, -1, -1, 1, 0, -1], np.int32),
        "slab_ordinal": np.array([1, 0, 0, 0, 0, 0], np.int32),
        "att": np.full(10, 0xFFFFFFFF, np.uint32),
    }
    d["att"][5], d["att"][7], d["att"][1], d["att"][2] = 8, 9, 0, 6
    return d, C, 6


def test_dump_validator_accepts_good_state():
    d, C, ns = _good_dump()
    assert check_dump(d, C, ns)


@pytest.mark.parametrize("corrupt", ["dup_slab", "leak", "free_and_held", "bad_att", "tomb", "dup_id",
                                     "owner", "extra_att"])
def test_dump_validator_rejects_corruption(corrupt):
    d, C, ns = _good_dump()
    if corrupt == "dup_slab":
        d["list_slabs"][2] = 4
    elif corrupt == "leak":
        d["free_slabs"] = d["free_slabs"][:2]
    elif corrupt == "free_and_held":
        d["free_slabs"][0] = 0
    elif corrupt == "bad_att":
        d["att"][7] = 8
    elif corrupt == "tomb":
        d["ids_by_list"][1] = -1
    elif corrupt == "dup_id":
        d["ids_by_list"][1] = 5
    elif corrupt == "owner":
        d["slab_owner"][3] = 0
    elif corrupt == "extra_att":
        d["att"][9] = 3
    with pytest.raises(AssertionError):
        check_dump(d, C, ns)


def test_dump_validator_lazy_slots():
    """With lazy deletes a dead slot reads -1 inside its list: accepted only in
    lazy mode, and only if the address table no longer points there."""
    d, C, ns = _good_dump()
    d["ids_by_list"][1] = -1           # id 7 deleted lazily: its slot stays in list 0
    d["att"][7] = 0xFFFFFFFF
    assert check_dump(d, C, ns, lazy=True)
    with pytest.raises(AssertionError):
        check_dump(d, C, ns)
    d["att"][7] = 9                    # ... but still reachable through the address table
    with pytest.raises(AssertionError):
        check_dump(d, C, ns, lazy=True)
