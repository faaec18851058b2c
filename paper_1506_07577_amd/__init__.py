"""ebbx: the element-parallel tet-FEM map of Ebb's relational runtime on MI355X.

The GPU work lives in the HIP library ``libebbx.so`` behind the C-ABI of
``include/ebbx.h``; ``paper_1506_07577_amd.ebbx`` is its thin ctypes binding
(loaded on first use; it raises if the library is missing).
"""
__all__ = ["meshgen"]
