"""MI355X-native hot path of CompactTag (arXiv 2311.04406).

SPDZ2k-style linear layers (products and convolutions) of two to five parties
over Z_{2^64} with 128-bit shares and tags (or Z_{2^32} with 64-bit ones):
output-share products on the int8 matrix cores, CompactTag's optimistic and
compact tags, and batch MAC verification, behind the C ABI of
``include/compacttag.h``.  ``binding`` is the thin ctypes layer over it.
"""
from .binding import (COMPRESS_AUTO, COMPRESS_M, COMPRESS_N, CT_ABORT, CT_OK, MAX_PARTIES, MODE_COMPACT,  # noqa
                      MODE_SPDZ2K, RESULT_WORDS, CheckResult, Context, CtError, Layer, Plan, REQ_CHECK, REQ_PREP, REQ_TAG,
                      Server, load)
