"""CPU checks of the C ABI: the library loads and exports every declared entry
point, and the binding's structs have the declared sizes.  No compute call
runs here (there is no GPU in this test's environment)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfe.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sfe_[a-z_]+)\s*\(", src)))


def test_header_declares_the_five_calls():
    names = declared_functions()
    for n in ("sfe_build_index", "sfe_seed_hits", "sfe_ungapped_xdrop", "sfe_gapped_ydrop", "sfe_align"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2606_06811_amd import sfe
    if not os.path.exists(sfe.LIB_PATH):
        pytest.skip("libsfe.so not built")
    lib = ctypes.CDLL(sfe.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_device():
    from paper_2606_06811_amd import sfe
    if not os.path.exists(sfe.LIB_PATH):
        pytest.skip("libsfe.so not built")
    L = sfe.lib()
    assert L.sfe_status_str(0) == b"ok"
    assert L.sfe_status_str(-3) == b"output capacity too small"


def test_struct_layouts():
    from paper_2606_06811_amd import sfe
    assert sfe.HIT_DTYPE.itemsize == 16
    assert sfe.HSP_DTYPE.itemsize == 24
    assert sfe.ALN_DTYPE.itemsize == 56
    assert ctypes.sizeof(sfe._Scoring) == 31 * 4
    assert ctypes.sizeof(sfe._AlignOpts) == 40
    src = open(HEADER).read()
    assert "} sfe_aln;                  /* 56 bytes */" in src


def test_binding_structs_match_the_c_header(tmp_path):
    """Sizes and field offsets of the ctypes mirrors equal what a C compiler
    makes of include/sfe.h."""
    import subprocess
    from paper_2606_06811_amd import sfe
    pairs = [("sfe_align_opts", sfe._AlignOpts), ("sfe_stats", sfe._Stats), ("sfe_scoring", sfe._Scoring),
             ("sfe_tuning", sfe._Tuning), ("sfe_tune_entry", sfe._TuneEntry), ("sfe_tune_report", sfe._TuneReport),
             ("sfe_seq", sfe._Seq), ("sfe_seed_spec", sfe._SeedSpec)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sfe.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    c = tmp_path / "sizes.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = []
    for cname, py in pairs:
        want.append(ctypes.sizeof(py))
        want += [getattr(py, f).offset for f, _ in py._fields_]
    assert got == want


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2606_06811_amd import sfe
    monkeypatch.setattr(sfe, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(sfe, "_lib", None)
    with pytest.raises(RuntimeError):
        sfe.lib()
