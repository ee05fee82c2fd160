"""MI355X (gfx950) Cuckoo++ hash tables: batched lookup, insert and delete
of 16-byte keys in HIP, behind the C ABI of include/ckpp.h.

    from paper_1712_09624_amd.ckpp import Table
"""

__all__ = ["ckpp", "workload", "build"]
