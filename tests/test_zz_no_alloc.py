"""The probe entry point that allocates nothing (sivf_probe_noalloc): its
scratch is the library's fixed device array.  Two calls in a row, the second
with a smaller input, must return exactly what sivf_probe returns (the exact
probe sets, which are also checked against the oracle), and a request larger
than the fixed scratch must be refused with SIVF_ERR_TOO_LARGE."""
import numpy as np
import pytest

import oracle
import paper_2601_11808_amd as sivf
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("metric", [0, 1])
def test_probe_noalloc_matches_probe(metric):
    rng = np.random.default_rng([91, metric])
    d, nlist = 48, 1000
    cent = rng.standard_normal((nlist, d)).astype(np.float32)
    cent[7] = cent[3]                              # an exact tie: lower list first
    ix = sivf.Index(d, nlist, cent, metric=metric, slab_capacity=64, num_slabs=64, id_capacity=64,
                    max_batch=4096, max_queries=4096, max_k=16, max_nprobe=64)
    for nq, nprobe in [(4000, 17), (333, 5), (2500, 1), (7, 64)]:
        q = rng.standard_normal((nq, d)).astype(np.float32)
        q[:4] = cent[[3, 7, 0, 999]]
        want = ix.probe(q, nprobe).cpu().numpy()
        got = ix.probe_noalloc(q, nprobe).cpu().numpy()
        assert ix.sync() == 0
        np.testing.assert_array_equal(got, want)
        np.testing.assert_array_equal(got[:200], oracle.probe(q[:200], cent, nprobe, metric))
        say(f"  nq={nq} nprobe={nprobe}: identical to sivf_probe")
    # larger than the 16 MiB scratch: 4,200 rows x 1,000 lists x 4 B > 16 MiB
    big = sivf.Index(d, nlist, cent, metric=metric, slab_capacity=64, num_slabs=64, id_capacity=64,
                     max_batch=8192, max_queries=64, max_k=16, max_nprobe=64)
    with pytest.raises(sivf.SivfError) as e:
        big.probe_noalloc(rng.standard_normal((4200, d)).astype(np.float32), 4)
    assert e.value.status == sivf.ERR_TOO_LARGE
    # the index is still usable and the scratch still serves
    q = rng.standard_normal((100, d)).astype(np.float32)
    np.testing.assert_array_equal(big.probe_noalloc(q, 9).cpu().numpy(), big.probe(q, 9).cpu().numpy())
    assert big.sync() == 0
    # nprobe 1 (the nearest-list path) keeps two words per group of 16 lists at 1,000 lists: 63 groups,
    # so 33,288 rows fill the 16 MiB; 40,000 rows are refused, 30,000 are served
    wide = sivf.Index(d, nlist, cent, metric=metric, slab_capacity=64, num_slabs=64, id_capacity=64,
                      max_batch=40000, max_queries=64, max_k=16, max_nprobe=64)
    with pytest.raises(sivf.SivfError) as e:
        wide.probe_noalloc(rng.standard_normal((40000, d)).astype(np.float32), 1)
    assert e.value.status == sivf.ERR_TOO_LARGE
    q = rng.standard_normal((30000, d)).astype(np.float32)
    got = wide.probe_noalloc(q, 1).cpu().numpy()
    np.testing.assert_array_equal(got, wide.probe(q, 1).cpu().numpy())
    np.testing.assert_array_equal(got[:300], oracle.probe(q[:300], cent, 1, metric))
    assert wide.sync() == 0
