"""psk: randomized sketching of tall-and-skinny matrices on AMD Instinct
MI355X (gfx950).

The compute path is the HIP library libpsk.so (C ABI in include/psk.h);
``paper_2203_02798_amd.api`` binds it to PyTorch device tensors.  Importing
this package loads nothing; the first API call loads the library and fails
loudly if it is missing.
"""
from ._lib import PskError  # noqa: F401

__version__ = "0.1.0"


def __getattr__(name):
    if name in ("cs_hash", "sketch_cs", "sketch_gcs", "gram", "rownorms_sq",
                "sketch_qr", "lsq_solve", "workspace_size", "CsrMatrix", "version"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
