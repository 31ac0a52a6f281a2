"""MI355X (gfx950) blocked randomized QR with column pivoting (BQRRP).

The compute path is the HIP library ``libqrcp.so`` (C ABI in include/qrcp.h);
``paper_2507_00976_amd.qrcp`` is its ctypes binding.  Import that module
explicitly: it fails loudly when the library is not built.
"""
__all__ = ["qrcp"]
