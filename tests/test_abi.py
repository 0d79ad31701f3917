"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and the
ctypes structures match the C layout (compiled with gcc from include/aes.h)."""
import ctypes
import os
import subprocess

import pytest

from paper_2104_14101_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = B.load()
    declared = B.declared_functions()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(B._PROTOS), "ctypes prototypes must cover exactly the header"


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "aes.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  printf("aes_options %zu\naes_info %zu\naes_trace_entry %zu\naes_problem %zu\n", sizeof(aes_options),
         sizeof(aes_info), sizeof(aes_trace_entry), sizeof(aes_problem));
  P(aes_options, rho); P(aes_options, seed); P(aes_options, force_reject_at); P(aes_options, trace);
  P(aes_options, x0); P(aes_info, dtilde_final); P(aes_info, status); P(aes_problem, nu); P(aes_problem, ldx);
  P(aes_trace_entry, log_ratio); P(aes_trace_entry, dtilde); P(aes_trace_entry, time_ms);
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                              check=True).stdout.strip().splitlines())
    assert int(out["aes_options"]) == ctypes.sizeof(B.Options)
    assert int(out["aes_info"]) == ctypes.sizeof(B.Info)
    assert int(out["aes_trace_entry"]) == ctypes.sizeof(B.TraceEntry)
    assert int(out["aes_problem"]) == ctypes.sizeof(B.Problem)
    for key, val in out.items():
        if "." in key:
            T, f = key.split(".")
            cls = {"aes_options": B.Options, "aes_info": B.Info, "aes_problem": B.Problem,
                   "aes_trace_entry": B.TraceEntry}[T]
            fname = {"lam": "lam"}.get(f, f)
            assert getattr(cls, fname).offset == int(val), key


def test_default_options_without_gpu():
    lib = B.load()
    o = B.Options()
    lib.aes_default_options(ctypes.byref(o))
    assert o.rho == 0.125 and o.m_init == 1 and o.max_iter == 200 and o.adaptive == 1 and o.force_reject_at == -1


def test_null_handle_is_rejected():
    lib = B.load()
    assert lib.aes_destroy(None) == B.AES_ERR_INVALID_ARG
    assert lib.aes_last_error(None) == b"null handle"
    assert lib.aes_solve(None, None, 1, 1, 1, None, 1, None, 1, 1.0, None, 1e-10, None, None, 1, None) \
        == B.AES_ERR_INVALID_ARG


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2104_14101_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_binding_enums_match_the_header():
    # the Python names map to the values include/aes.h gives the enumerators
    import re

    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "aes.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    vals = {k: int(v) for k, v in re.findall(r"\b(AES_[A-Z0-9_]+)\s*=\s*(\d+)", hdr)}
    expect = {
        "METHODS": {"pcg": "AES_PCG", "ihs": "AES_IHS", "cg": "AES_CG", "polyak": "AES_POLYAK"},
        "SKETCHES": {"srht": "AES_SRHT", "gauss": "AES_GAUSS", "sjlt": "AES_SJLT", "srht_reuse": "AES_SRHT_REUSE",
                     "srht_nested": "AES_SRHT_NESTED"},
        "PRECISIONS": {"fp64": "AES_FP64", "mixed": "AES_MIXED", "mixed_fp32": "AES_MIXED_FP32"},
        "STOPS": {"xrel": "AES_STOP_XREL", "dtilde_rel": "AES_STOP_DTILDE_REL", "fixed": "AES_STOP_FIXED",
                  "remark": "AES_STOP_REMARK"},
    }
    for table, names in expect.items():
        got = getattr(B, table)
        assert set(got) == set(names), table
        for py, c in names.items():
            assert got[py] == vals[c], (table, py)
    # every enumerator of those four enums is reachable from Python
    prefixes = ("AES_PCG", "AES_IHS", "AES_CG", "AES_POLYAK", "AES_SRHT", "AES_GAUSS", "AES_SJLT", "AES_FP64",
                "AES_MIXED", "AES_STOP_")
    declared = {k for k in vals if k.startswith(prefixes)}
    assert declared == {c for names in expect.values() for c in names.values()}
