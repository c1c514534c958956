"""Sparse Frequent Directions on MI355X (gfx950): a HIP library behind a C ABI (include/sfd.h)
and its Python binding (``paper_1602_00412_amd.sfd``)."""

from . import sfd  # noqa: F401
from .sfd import Sketch, SfdError, load, start_block  # noqa: F401
