"""paper_2007_09625_amd -- error-bounded lossy compression of fp32 fields
on AMD MI355X (gfx950) with the cuSZ dual-quantization + Huffman method.

    from paper_2007_09625_amd import compress, decompress
    c = compress(field_cuda_f32, 1e-4)          # value-range-relative eb
    y = decompress(c)                            # |field - y| <= eb_abs

The work runs in hand-written HIP kernels behind the C ABI of ``libdqz.so``
(``include/dqz.h``); this package only marshals arguments.
"""
from .dqz import (DQZ_EB_ABS, DQZ_EB_VALREL, Compressed, Context, DqzError, compress, decompress,  # noqa: F401
                  default_context, dqz_archive_info, dqz_compress_bound)
