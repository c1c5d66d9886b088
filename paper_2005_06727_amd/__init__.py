"""Sparse Sinkhorn Word Mover's Distance on MI355X (gfx950).

The compute path lives in the HIP/C++ shared library ``libwmd.so`` built from
``csrc/``; ``wmd`` is its thin ctypes binding.  Importing this package loads
nothing: ``from paper_2005_06727_amd import wmd`` loads the library and fails
loudly if it has not been built.
"""
__all__ = ["wmd", "synth"]
