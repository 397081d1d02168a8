"""CPU-side checks of the C-ABI library: it loads, it exports every entry
point that include/gg.h declares, and the binding declares a signature for
each. No compute call is made (there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    hdr = open(os.path.join(ROOT, "include", "gg.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(gg_\w+)\s*\(", hdr, re.M)))


def test_header_declares_boundary():
    names = header_functions()
    for need in ("gg_graph_load_csr", "gg_exact_run", "gg_approx_run", "gg_run_begin", "gg_run_step",
                 "gg_run_values", "gg_run_mask", "gg_run_end", "gg_graph_free", "gg_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_2104_10039_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libgg.so not built")
    out = subprocess.check_output(["nm", "-D", "--defined-only", P.LIB_PATH]).decode()
    exported = set(re.findall(r"\sT\s(gg_\w+)$", out, re.M))
    missing = [n for n in header_functions() if n not in exported]
    assert not missing, missing
    L = P.lib()
    for n in header_functions():
        assert n in P.SIGNATURES, n
        getattr(L, n)
    hdr = open(os.path.join(ROOT, "include", "gg.h")).read()
    assert L.gg_version() == int(re.search(r"#define GG_VERSION (\d+)", hdr).group(1))


def test_binding_has_no_fallback():
    """The binding raises when the library is missing instead of computing on the CPU."""
    import paper_2104_10039_amd as P
    src = open(os.path.join(ROOT, "paper_2104_10039_amd", "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    assert "raise ImportError" in src
    saved = P._lib, P.LIB_PATH
    try:
        P._lib = None
        P.LIB_PATH = "/nonexistent/libgg.so"
        with pytest.raises(ImportError):
            P.lib()
    finally:
        P._lib, P.LIB_PATH = saved


def test_product_does_not_touch_oracle():
    pkg = os.path.join(ROOT, "paper_2104_10039_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower().replace("oracle-", ""), f


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that a C compiler gives the header's struct (gcc on the host)."""
    import paper_2104_10039_amd as P
    pairs = {"gg_csr_desc": P.CsrDesc, "gg_app_params": P.AppParams, "gg_correction_policy": P.Policy,
             "gg_run_stats": P.RunStats, "gg_step_info": P.StepInfo, "gg_kernel_profile": P.KernelProfile,
             "gg_tuning": P.Tuning}
    lines = ['#include <stdio.h>', '#include "gg.h"', "int main(void) {"]
    for cname, cls in pairs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = str(tmp_path / "layout")
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", exe, str(src)])
    got = {}
    for line in subprocess.check_output([exe]).decode().splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for cname, cls in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
