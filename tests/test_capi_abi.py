"""The C-ABI library loads on a machine without a GPU and exports every
function that include/*.h declares (no compute calls here)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(sd_\w+)\s*\(", text, re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sd_create", "sd_destroy", "sd_self_search", "sd_pairs_free", "sd_strerror",
                 "sd_last_error", "sd_get_stats", "sd_pair_distance", "sd_pairs_copy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2403_09010_amd import load_library
    lib = load_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_error_strings_and_null_arguments_without_gpu():
    from paper_2403_09010_amd import load_library
    lib = load_library()
    assert lib.sd_strerror(0) == b"ok"
    assert lib.sd_strerror(-3).startswith(b"sequence length")
    # null arguments are rejected before any device call
    assert lib.sd_create(None, 0, 0) == -1
    assert lib.sd_self_search(None, None, 1, None, None) == -1
    assert lib.sd_last_error(None) == b""


def test_product_path_has_no_fallback():
    # without a usable device the binding raises instead of computing elsewhere
    import paper_2403_09010_amd as p
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    with pytest.raises(p.SymdelError):
        p.Context()
