"""Exact linear-memory DTW alignment (divide and conquer over anti-diagonal
wavefront passes) on AMD Instinct MI355X (gfx950).

The compute path is the C-ABI library ``libdtw_hip.so`` built from
``csrc/``; ``dtw.py`` is a thin ctypes binding over it.  Importing the
package loads nothing; ``paper_2008_02734_amd.dtw`` loads the library and
fails loudly when it is missing.
"""
__all__ = ["dtw", "synth"]
