"""The C-ABI library loads and exports every entry point include/clair.h
declares, and the ctypes mirrors of its structs have the C layout (no GPU)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clair.h")


@pytest.fixture(scope="module", autouse=True)
def _library_built():
    """Build libclair.so with hipcc if this tree has none yet (a fresh
    checkout: the library is not kept in version control)."""
    from paper_2307_00229_amd import build

    if not os.path.exists(build.LIB):
        build.build()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(clair_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_entry_points():
    names = _declared()
    assert "clair_build_R" in names and "clair_build_R_batched" in names
    assert len(names) >= 16


def test_library_exports_every_declared_symbol():
    from paper_2307_00229_amd import clair

    lib = clair.load_library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(clair.EXPORTED) == _declared()


def test_strerror_without_gpu():
    from paper_2307_00229_amd import clair

    for st in range(7):
        assert clair.strerror(st)
    assert "capacity" in clair.strerror(clair.CLAIR_ERR_CAPACITY)


def test_struct_layout_matches_c():
    from paper_2307_00229_amd import clair

    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "clair.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("clair_csr_t %zu\n", sizeof(clair_csr_t));
  printf("clair_csr_out_t %zu\n", sizeof(clair_csr_out_t));
  printf("clair_info_t %zu\n", sizeof(clair_info_t));
  printf("clair_opts_t %zu\n", sizeof(clair_opts_t));
  P(clair_csr_t, val) P(clair_csr_out_t, nnz_capacity) P(clair_csr_out_t, val)
  P(clair_info_t, n_uncovered) P(clair_info_t, n_fp64_rows) P(clair_info_t, n_bf16_retries) P(clair_opts_t, timing)
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    vals = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    vals = {k: int(v) for k, v in vals.items()}
    assert vals["clair_csr_t"] == ctypes.sizeof(clair.CsrIn)
    assert vals["clair_csr_out_t"] == ctypes.sizeof(clair.CsrOut)
    assert vals["clair_info_t"] == ctypes.sizeof(clair.Info)
    assert vals["clair_opts_t"] == ctypes.sizeof(clair.Opts)
    assert vals["clair_csr_t.val"] == clair.CsrIn.val.offset
    assert vals["clair_csr_out_t.nnz_capacity"] == clair.CsrOut.nnz_capacity.offset
    assert vals["clair_csr_out_t.val"] == clair.CsrOut.val.offset
    assert vals["clair_info_t.n_uncovered"] == clair.Info.n_uncovered.offset
    assert vals["clair_info_t.n_fp64_rows"] == clair.Info.n_fp64_rows.offset
    assert vals["clair_info_t.n_bf16_retries"] == clair.Info.n_bf16_retries.offset
    assert vals["clair_opts_t.timing"] == clair.Opts.timing.offset


def test_product_path_does_not_import_oracle():
    import ast

    pkg = os.path.join(ROOT, "paper_2307_00229_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            tree = ast.parse(open(os.path.join(pkg, fn)).read())
            for node in ast.walk(tree):
                if isinstance(node, ast.Import):
                    assert not any(a.name.split(".")[0] == "oracle" for a in node.names), fn
                if isinstance(node, ast.ImportFrom):
                    assert (node.module or "").split(".")[0] != "oracle", fn
    for fn in os.listdir(os.path.join(pkg, "csrc")):
        text = open(os.path.join(pkg, "csrc", fn)).read()
        assert "oracle" not in text.lower(), fn


def test_missing_library_fails_loudly(tmp_path):
    # no CPU fallback: without the HIP library the binding raises
    from paper_2307_00229_amd import clair

    saved = clair._lib
    clair._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            clair.load_library(str(tmp_path / "libclair.so"))
    finally:
        clair._lib = saved


def test_product_code_does_not_use_the_oracle():
    # only tests, the smoke check and the benchmark's CPU baseline may load
    # oracle/; the package and the kernels never do
    pkg = os.path.join(ROOT, "paper_2307_00229_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(import oracle|from oracle)", text, flags=re.M), fn
                assert "clair_oracle" not in text, fn
