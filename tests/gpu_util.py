"""Helpers of the GPU tests: device transfers and oracle-side expectations."""

import sys

import numpy as np

from oracle import oracle as O
from paper_1712_09624_amd import workload as W


def torch_dev():
    import torch
    return torch.device("cuda", 0)


def say(msg: str):
    """Names the GPU step about to run (flushed, so a dying box still shows it)."""
    print(f"[gpu-step] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch_dev())


def vals_dev(v: np.ndarray):
    return to_dev(np.ascontiguousarray(v, dtype=np.uint64).view(np.int64))


def u64(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def u8(t) -> np.ndarray:
    return t.cpu().numpy().astype(np.uint8)


def oracle_table(B, keys, vals, plain=False, max_kicks=W.MAX_KICKS):
    t = O.OracleTable(B, W.HASH_SEED, max_kicks, plain)
    st = t.insert(keys, vals)
    return t, st


def check_gpu_image(table, B, plain=False):
    b, k = table.export()
    rc, msg = O.check_image(b, k, B, W.HASH_SEED, plain)
    assert rc == 0, f"GPU image invariant {rc}: {msg}"
    return b, k
