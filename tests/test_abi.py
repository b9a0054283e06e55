"""The C-ABI library loads and exports every entry point include/cs.h declares
(no device calls)."""
import os
import re

import numpy as np
import pytest

import paper_2512_08465_amd as cs

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "cs.h")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cs_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib = cs.library()
    names = _declared()
    assert "cs_screen" in names and "cs_detail" in names
    for n in names:
        assert hasattr(lib, n), n
        assert n in cs.EXPORTED, n


def test_abi_version_and_record_layout():
    txt = open(HDR).read()
    v = int(re.search(r"#define CS_ABI_VERSION (\d+)", txt).group(1))
    assert cs.library().cs_abi_version() == v
    assert cs.RESULT_DTYPE.itemsize == 48


def test_default_options():
    o = cs.default_options()
    assert o.prec == 0 and o.max_it == 150 and o.tol == 1e-8 and o.near_eps == 1e-6


def test_no_device_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(cs.CSError):
        cs.Context(0)
