"""Energy-based DG with a Galerkin-difference basis for u_tt = div(c^2 grad u) on MI355X.

The compute path is the C-ABI library ``libgdw.so`` (hand-written HIP for gfx950)
declared in ``include/gdw.h``; :mod:`paper_2105_01722_amd.gdw` is its ctypes binding.
:mod:`paper_2105_01722_amd.inputs` produces the seeded synthetic inputs.

Nothing is imported eagerly, so that ``inputs`` can be used without loading the
HIP library.
"""
__all__ = ["gdw", "inputs"]
