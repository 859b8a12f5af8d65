"""Host-side checks that need no GPU: the C-ABI library loads and exports every
entry point its header declares, the binding refuses host tensors, and the
product package never reaches the oracle."""
import ctypes
import os
import re

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mphf.h")
PKG = os.path.join(ROOT, "paper_1702_03154_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mphf_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1702_03154_amd import mphf
    if not os.path.exists(mphf.LIB_PATH):
        from paper_1702_03154_amd import build_lib
        build_lib.build()
    return mphf.LIB_PATH


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ("mphf_build", "mphf_lookup", "mphf_build_ex", "mphf_lookup_ex", "mphf_destroy",
              "mphf_stats", "mphf_export", "mphf_last_error"):
        assert f in fns


def test_library_exports_every_declared_symbol(libpath):
    L = ctypes.CDLL(libpath)
    for f in declared_functions():
        assert hasattr(L, f), f


def test_binding_loads_and_refuses_host_tensors(libpath):
    from paper_1702_03154_amd import mphf
    mphf.lib()
    with pytest.raises(ValueError):
        mphf.build(torch.arange(10, dtype=torch.int64), 2.0)
    o = mphf.Opts()
    assert mphf.lib().mphf_default_opts(ctypes.byref(o)) == 0
    assert (o.max_levels, o.rank_sample, o.mem_budget) == (25, 512, 0)


def test_product_never_imports_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                bad = re.findall(r"(?:from|import)\s+oracle\b|oracle/|mphf_oracle", src)
                assert not bad, (os.path.join(dirpath, f), bad)
