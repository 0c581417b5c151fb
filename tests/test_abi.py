"""The C ABI: librbk.so loads and exports every function include/rbk.h
declares, and the binding's signature table covers exactly those.  CPU only
(no call touches the GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(rbk_[a-z0-9_]+)\s*\(", txt))
    return names


def test_header_declares_functions():
    names = _declared()
    for must in ("rbk_ctx_create", "rbk_mult_relin", "rbk_rescale", "rbk_rotate", "rbk_rotate_hoisted",
                 "rbk_rotate_hoisted_batch", "rbk_encode", "rbk_encrypt", "rbk_decrypt", "rbk_keygen_relin"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2506_19693_amd import build, rbk

    if not os.path.exists(rbk.LIB_PATH):
        build.build(force=False)
    lib = ctypes.CDLL(rbk.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(rbk.SIGNATURES) == _declared()
    rbk.load()   # applies every signature


def test_binding_refuses_without_gpu():
    import torch

    from paper_2506_19693_amd import rbk

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        rbk.Context(10, [50, 40], [50], 1)
