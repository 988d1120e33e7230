"""MI355X (gfx950) micro-macro KFVS solver for the Boltzmann-BGK / ES-BGK
equations (Rossmanith & Sar, arXiv:2509.21832).

The solver is the HIP library ``libmm.so`` behind the C ABI of
``include/mm.h``; ``binding`` wraps it with ctypes.  Importing the package
does not load the library; ``from paper_2509_21832_amd import binding`` does,
and raises if it is not built.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmm.so")


def Solver(*args, **kwargs):
    from .binding import Solver as _S
    return _S(*args, **kwargs)
