"""CPU oracle for the bzip2 compression stages analysed in
"Lossless data compression on GPGPU architectures" (Eirola).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
executes anything under this directory; only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark do.  The oracle shares no code,
tables or constants with the HIP path.

Two tiers compute the same functions:

* ``ref`` (this package, pure Python) -- literal definitions, for inputs of up
  to a few thousand bytes.
* ``cref`` -- the same algorithms in plain C (``ref.c``), for full-size
  blocks, loaded through ctypes.
"""

from . import ref  # noqa: F401
