"""libpolar: successive-cancellation decoding of long polar codes on MI355X.

The product is the C-ABI library ``libpolar.so`` (declared in include/polar.h,
built from ``csrc/``); ``polar`` is its thin Python binding.
"""
from . import polar  # noqa: F401
