"""The allocation-free insert (ckpp_insert_batch_noalloc) against the
insert it varies (ckpp_insert_batch): two tables receive the same batches,
one through each entry point, and must hold the same dictionary (insert
statuses, the found flag and value of every key), each keeping the image
invariants.  Two calls in a row, the second with a smaller batch, at a load
where cuckoo paths (the scratch's use) are common."""

import numpy as np
import pytest

from gpu_util import check_gpu_image, say, to_dev, u64, u8, vals_dev
from oracle import oracle as O
from paper_1712_09624_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("B", [12, 16])
def test_noalloc_insert_equals_insert(B):
    import torch
    from paper_1712_09624_amd.ckpp import Table
    n1 = W.keys_at_load(B, 0.9)
    n2 = W.keys_at_load(B, 0.95) - n1
    keys = W.distinct_five_tuples(n1 + n2, 150 + B)
    vals = W.insertion_values(n1 + n2, 3)
    # the second call also updates some keys of the first
    upd = W.choose_rows(n1, n2 // 4, 151 + B)
    k2 = np.concatenate([keys[n1:], keys[upd]])
    v2 = np.concatenate([vals[n1:], vals[upd] + np.uint64(10**9)])
    a = Table(B, W.HASH_SEED, W.MAX_KICKS, device=0)
    b = Table(B, W.HASH_SEED, W.MAX_KICKS, device=0)
    dev = torch.device("cuda", 0)
    for step, (kk, vv) in enumerate(((keys[:n1], vals[:n1]), (k2, v2))):
        n = len(kk)
        say(f"noalloc insert B={B} call {step}: {n} keys")
        dk, dv = to_dev(kk), vals_dev(vv)
        st_a, nf_a = a.insert(dk, dv)
        st_b = torch.full((n,), 0xEE, dtype=torch.uint8, device=dev)
        nf_b = torch.zeros(1, dtype=torch.int64, device=dev)
        b.insert_noalloc(dk, dv, st_b, nf_b)
        torch.cuda.synchronize()
        assert np.array_equal(u8(st_b), u8(st_a)), f"call {step}: statuses differ"
        assert int(nf_b.item()) == int(nf_a.item())
        check_gpu_image(b, B)
        probe = np.concatenate([keys, W.five_tuples(4096, 152 + B)])
        fa, va = a.lookup(to_dev(probe))
        fb, vb = b.lookup(to_dev(probe))
        assert np.array_equal(u8(fb), u8(fa)), f"call {step}: found flags differ"
        assert np.array_equal(u64(vb), u64(va)), f"call {step}: values differ"
    # and both equal the oracle's dictionary
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS)
    ref.insert(keys[:n1], vals[:n1])
    ref.insert(k2, v2)
    wf, wv, _, _ = ref.lookup(keys)
    fb, vb = b.lookup(to_dev(keys))
    assert np.array_equal(u8(fb), wf) and np.array_equal(u64(vb), wv)
    s = b.stats()
    assert s["locked"] == 0 and s["retry_exhausted"] == 0
    a.close()
    b.close()


def test_noalloc_refuses_timed_tables():
    import torch
    from paper_1712_09624_amd.ckpp import CkppError, Table
    t = Table(6, W.HASH_SEED, W.MAX_KICKS, device=0, timers=True)
    keys = to_dev(W.distinct_five_tuples(4, 153))
    st = torch.empty(4, dtype=torch.uint8, device="cuda:0")
    nf = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    with pytest.raises(CkppError):
        t.insert_noalloc(keys, vals_dev(W.insertion_values(4)), st, nf)
    t.close()
