"""Structural invariants of a device-state dump (host-side check, numpy).

Checks the properties the paper's correctness argument rests on, restated
for dense slab lists (Sec. 3.1 slab pool and free stack; Theorem 1: each
inserted entry owns a unique slot; Theorem 3: a deleted id is absent; the
address table of Sec. 3.4 maps each live id to its slot):
  - each list of n entries holds ceil(n/C) slabs, each slab is held by at most
    one list, and a held slab records its owner and ordinal;
  - used + free = pool size, and no slab is both free and held;
  - every live position holds a real id (no tombstone), each id once;
  - the address table maps exactly the live ids, each to its own slot;
  - with a host tier, entries flagged cold are exactly the live cold ids.
"""
import numpy as np

INVALID = 0xFFFFFFFF
COLD_BIT = 0x80000000


def check_dump(d, C, num_slabs, lazy=False, cold_ids=None):
    """lazy: slots deleted lazily (not yet compacted) read -1 inside the lists;
    the address table must not point at them.  cold_ids: the host tier's ids
    by list (-1 for dead slots), or None without a tier."""
    ln = d["list_len"].astype(np.int64)
    assert (ln >= 0).all()
    ns = (ln + C - 1) // C
    slabs = d["list_slabs"].astype(np.int64)
    assert slabs.shape[0] == ns.sum()
    assert ((slabs >= 0) & (slabs < num_slabs)).all(), "slab id out of range"
    assert np.unique(slabs).shape[0] == slabs.shape[0], "a slab is held twice"
    free = d["free_slabs"].astype(np.int64)
    assert np.unique(free).shape[0] == free.shape[0], "free stack holds a slab twice"
    assert slabs.shape[0] + free.shape[0] == num_slabs, "used + free != pool"
    assert np.intersect1d(slabs, free).shape[0] == 0, "slab both free and held"
    owner, ordn = d["slab_owner"], d["slab_ordinal"]
    lst = np.repeat(np.arange(ln.shape[0]), ns)
    ordinal = np.arange(slabs.shape[0]) - np.repeat(np.cumsum(ns) - ns, ns)
    assert (owner[slabs] == lst).all(), "slab owner mismatch"
    assert (ordn[slabs] == ordinal).all(), "slab ordinal mismatch"
    assert (owner[free] == -1).all(), "free slab still owned"
    ids_all = d["ids_by_list"]
    assert ids_all.shape[0] == ln.sum()
    live = ids_all >= 0
    if not lazy:
        assert live.all(), "tombstone inside a live range"
    if "info" in d:
        assert d["info"]["live"] == int(live.sum()), "live count != live slots"
    ids = ids_all[live]
    assert np.unique(ids).shape[0] == ids.shape[0], "an id is stored twice"
    att = d["att"]
    cold = (att != INVALID) & ((att & COLD_BIT) != 0)
    if cold_ids is None:
        assert not cold.any(), "a cold address without a tier"
    else:
        cl = cold_ids[cold_ids >= 0]
        assert np.unique(cl).shape[0] == cl.shape[0], "a cold id is stored twice"
        assert np.intersect1d(cl, ids).shape[0] == 0, "an id is both cold and on the device"
        assert np.array_equal(np.flatnonzero(cold), np.sort(cl)), "cold addresses != live cold ids"
    valid = (att != INVALID) & ~cold
    assert valid.sum() == ids.shape[0], "address table size != live"
    assert valid[ids].all(), "live id missing from the address table"
    # expected slot of each live entry
    pos = (np.arange(ids_all.shape[0]) - np.repeat(np.cumsum(ln) - ln, ln))[live]
    list_of_entry = np.repeat(np.arange(ln.shape[0]), ln)[live]
    slab_base = np.cumsum(ns) - ns
    slab_of_entry = slabs[slab_base[list_of_entry] + pos // C]
    want = slab_of_entry * C + pos % C
    assert (att[ids].astype(np.int64) == want).all(), "address table points to the wrong slot"
    return True


def membership_of(d):
    """{list: sorted live ids} of the non-empty lists (lazily deleted slots, -1, dropped)."""
    ln = d["list_len"].astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(ln)])
    out = {}
    for l in range(ln.shape[0]):
        v = d["ids_by_list"][offs[l]:offs[l + 1]]
        v = v[v >= 0]
        if v.shape[0]:
            out[l] = np.sort(v)
    return out


def same_membership(a, b):
    if a.keys() != b.keys():
        return False
    return all(np.array_equal(a[k], b[k]) for k in a)
