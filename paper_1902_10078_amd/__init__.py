"""Banded-matrix operators for Gaussian Markov models on MI355X (gfx950).

The operators (Cholesky, triangular solves, subset inverse, banded products and
their reverse-mode derivatives) run as hand-written HIP kernels behind the C-ABI
library ``libbandops.so``; :mod:`paper_1902_10078_amd.bandops` is the thin ctypes
binding and :mod:`paper_1902_10078_amd.autograd` the ``torch.autograd.Function``
wrappers.  Importing this package loads nothing; the binding loads the library on
first use and raises if it is missing.
"""

__version__ = "0.1.0"
