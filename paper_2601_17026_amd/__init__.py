"""Exact surface max-flow on MI355X (gfx950).

The solver lives in a C-ABI shared library built from `csrc/`; `smf` (the
Python binding) marshals torch device tensors into it.  Importing this package
does not load the library; `paper_2601_17026_amd.smf` does.
"""
