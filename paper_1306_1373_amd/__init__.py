"""MI355X-native blockwise 8x8 Cordic-based Loeffler DCT codec.

The codec runs as hand-written HIP kernels for gfx950 behind a C ABI
(``include/dctcodec.h``, built into ``paper_1306_1373_amd/lib/libdctcodec.so``).
:mod:`paper_1306_1373_amd.codec` is the thin Python binding with the same
entry-point names; it only marshals torch device tensors to pointers.

Importing this package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""

__all__ = ["codec", "synth"]
