"""CPU-side checks of the C ABI: the library builds for gfx950, loads, and
exports every symbol the public header declares.  No compute call here."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bzgpu.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*|uint64_t)\s+\**(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def _lib_path():
    from paper_1109_2348_amd import native
    if not os.path.exists(native.LIB_PATH):
        from paper_1109_2348_amd import build
        build.build()
    return native.LIB_PATH


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ["bwt_forward_batch", "mtf_encode_batch", "huffman_encode_batch", "compress_blocks",
              "bzg_create", "bzg_destroy", "bzg_last_error", "bzg_compress_bound"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    for n in _declared():
        assert hasattr(lib, n), f"missing export {n}"


def test_binding_lists_match_header():
    from paper_1109_2348_amd import native
    assert sorted(native.EXPORTS) == _declared()


def test_compress_bound_is_safe_for_worst_expansion():
    from paper_1109_2348_amd import native
    lib = native.lib()
    # every byte alone in a run of four: RLE1 grows by 1.25; 17 bits per symbol
    n = 1_000_000
    bound = lib.bzg_compress_bound(n, 1)
    assert bound % 4 == 0
    assert bound * 8 >= (n * 5 // 4) * 17


def test_null_context_is_rejected():
    from paper_1109_2348_amd import native
    lib = native.lib()
    assert lib.bzg_last_error(None) == b"null context"
    assert lib.compress_blocks(None, None, None, None, 0, 9, None, 0, None, None, None, 0, None) == native.BZG_EINVAL
    assert lib.bwt_forward_batch(None, None, None, None, 0, None, None, None, None, 0, None) == native.BZG_EINVAL
    assert lib.bzg_check(None, None) == native.BZG_EINVAL
    assert lib.bzg_workspace_size(None, 4, None, 0, 9, 1, None) == native.BZG_EINVAL
    assert lib.compress_host(None, None, 0, 0, 9, 0, None, 0, None, None) == native.BZG_EINVAL
    assert lib.decompress(None, None, 0, None, 0, None, None) == native.BZG_EINVAL


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1109_2348_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".c", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "libbzref" not in txt and "ref.c" not in txt, f
