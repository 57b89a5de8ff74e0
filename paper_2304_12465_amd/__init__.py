"""gfx950 (MI355X) kernel ridge regression with RPCholesky- and
KRILL-preconditioned conjugate gradient (arXiv 2304.12465).

All arithmetic of the method runs in the HIP library ``libkrr.so``
(``include/krr.h``); this package only marshals arguments to it.  PyTorch
supplies device memory and streams.  Importing ``binding`` raises if the
library has not been built: there is no CPU fallback.
"""
__all__ = ["binding"]
