"""WENO-ZN (arXiv 2004.07954) hot path for MI355X: HIP kernels behind a C ABI (libwenozn.so)
with a thin PyTorch binding.

    from paper_2004_07954_amd import api
    L = api.rhs_1d(u, dx, api.params("euler"))

``inputs`` holds the seeded synthetic workloads; ``api`` the binding.  Importing ``api``
requires the in-tree libwenozn.so (built by ``__graft_entry__.build()``); there is no
fallback path.  Submodules are imported explicitly so that the CPU-only tests can use
``inputs`` without torch or the GPU library.
"""
__all__ = ["api", "inputs"]
