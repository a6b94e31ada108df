"""fm-flow: one-loop temperature-flow right-hand side of the N-patch coupling function of the
2D Hubbard model (Rohe & Honerkamp, arXiv:2005.00827) on MI355X (gfx950).

The compute path is the C-ABI library ``libfmflow.so`` (hand-written HIP kernels); the
Python side (:mod:`paper_2005_00827_amd.fm`) only marshals arguments. Importing this package
loads nothing; :func:`paper_2005_00827_amd.fm.load` loads the library and fails loudly when
it is missing.
"""
__version__ = "0.1.0"
