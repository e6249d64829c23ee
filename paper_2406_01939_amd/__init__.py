"""MI355X-native Picard policy simulation for the fulfillment problem (HIP, gfx950).

The GPU path lives in the C-ABI library `libpicard.so` (built from csrc/); `api` holds
the thin Python binding with the same entry-point names.  Importing this package does
not load the library; `api` does, and fails loudly when it is missing.
"""
__all__ = ["api", "instances"]
