"""paper_1109_2348_amd: batched bzip2 compression stages (BWT, MTF,
RUNA/RUNB, Huffman, bit-packing) as HIP kernels for the MI355X, behind the C
ABI in include/bzgpu.h.

    from paper_1109_2348_amd import compress, bwt, mtf, huffman
"""

from . import native  # noqa: F401
from .native import (BzgError, Compressor, Context, bwt, compress, compress_bound, compress_host, decompress,  # noqa: F401
                     context, field_decode, field_encode, fixed_tables_from_sample, huffman, mtf,
                     uniform_offsets)
