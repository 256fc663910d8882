"""MI355X-native discrete Frechet distance (arXiv 2404.05708's hot path).

The compute path is the HIP library ``libffd.so`` (C ABI in include/ffd.h);
``paper_2404_05708_amd.ffd`` is its thin Python binding.  Importing the
binding raises if the library has not been built.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libffd.so")


def load():
    """Import and return the binding module (raises if libffd.so is missing)."""
    from . import ffd
    return ffd
