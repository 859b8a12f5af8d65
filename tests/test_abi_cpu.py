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


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's sizes and field offsets."""
    import shutil
    import subprocess
    from paper_1702_03154_amd import mphf
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    prog = tmp_path / "sizes.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "mphf.h"
int main(void) {
    printf("%zu %zu %zu %zu\\n", sizeof(mphf_opts), sizeof(mphf_stats_t), sizeof(mphf_view_t),
           sizeof(mphf_set_info_t));
    printf("%zu %zu %zu %zu\\n", offsetof(mphf_opts, batch_threads), offsetof(mphf_stats_t, n_fallback),
           offsetof(mphf_set_info_t, total_bits), offsetof(mphf_opts, batch_small_every));
    return 0;
}
""")
    exe = tmp_path / "sizes"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    sizes = [int(v) for v in lines[0].split()]
    offs = [int(v) for v in lines[1].split()]
    assert sizes == [ctypes.sizeof(mphf.Opts), ctypes.sizeof(mphf.Stats), ctypes.sizeof(mphf.View),
                     ctypes.sizeof(mphf.SetInfo)]
    assert offs == [mphf.Opts.batch_threads.offset, mphf.Stats.n_fallback.offset,
                    mphf.SetInfo.total_bits.offset, mphf.Opts.batch_small_every.offset]


def test_autotune_cache_keys(tmp_path, monkeypatch):
    """Batches of the same shape share a tuned launch; the cache file round-trips."""
    from paper_1702_03154_amd import autotune, inputs
    monkeypatch.setenv("MPHF_TUNE_CACHE", str(tmp_path / "t.json"))
    a = inputs.set_offsets(torch.tensor([16, 100, 5000, 70]))
    b = inputs.set_offsets(torch.tensor([20, 120, 6000, 100]))   # same power-of-two classes
    c = inputs.set_offsets(torch.tensor([16, 100, 50000, 70]))
    assert autotune.workload_key(a, 2.0, 25) == autotune.workload_key(b, 2.0, 25)
    assert autotune.workload_key(a, 2.0, 25) != autotune.workload_key(c, 2.0, 25)
    assert autotune.workload_key(a, 2.0, 25) != autotune.workload_key(a, 1.0, 25)
    autotune._store({"dev": {"k": {"launch": [512, 4, 2]}}})
    assert autotune._load()["dev"]["k"]["launch"] == [512, 4, 2]
    assert len(list(autotune.candidates())) == 81
    assert autotune.DEFAULT in set(autotune.candidates())
