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
    assert ctypes.sizeof(sfe._AlignOpts) == 48
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


def _lib_or_skip():
    from paper_2606_06811_amd import sfe
    if not os.path.exists(sfe.LIB_PATH):
        pytest.skip("libsfe.so not built")
    return sfe


def test_align_options_resolve_bounds_the_first_batch():
    """Without the nearness rule nothing keeps a region's later HSPs out of the
    first batch, so the automatic batch size falls back to Alg. 3's cap: the
    first batch of a (query, strand) holds at most 256 extensions."""
    sfe = _lib_or_skip()
    on = sfe.sfe_align_opts_resolve()
    assert on["round_k"] == 1 << 20 and on["near_band"] == 32 and on["strands"] == 3
    assert on["max_cells_per_lane"] == 6
    off = sfe.sfe_align_opts_resolve(near_band=-5)
    assert off["near_band"] == -1 and off["round_k"] == 256
    prefix = sfe.sfe_align_opts_resolve(policy=sfe.SFE_POLICY_PREFIX)
    assert prefix["round_k"] == 256
    # an explicit batch size is the caller's choice
    assert sfe.sfe_align_opts_resolve(near_band=-1, round_k=64)["round_k"] == 64
    assert sfe.sfe_align_opts_resolve(max_cells_per_lane=13)["max_cells_per_lane"] == 8
    for bad in (dict(schedule=7), dict(policy=3), dict(strands=4), dict(round_k=-2), dict(arena_bytes=-1),
                dict(max_cells_per_lane=-1), dict(filter=2)):
        with pytest.raises(sfe.SfeError):
            sfe.sfe_align_opts_resolve(**bad)


def _model_blob(params, m, v, steps):
    """A model file laid out as include/sfe.h states (written here from that text)."""
    import struct
    import numpy as np
    body = b"SFEMLP\0\0" + struct.pack("<IIIIq", 1, 1, params.shape[0], 0, steps)
    body += params.astype("<f4").tobytes() + m.astype("<f4").tobytes() + v.astype("<f4").tobytes()
    h = 1469598103934665603
    for b in body:
        h = ((h ^ b) * 1099511628211) & ((1 << 64) - 1)
    return body + struct.pack("<Q", h)


def test_model_file_check_rejects_corruption(tmp_path):
    import numpy as np
    sfe = _lib_or_skip()
    rng = np.random.default_rng(7)
    n = sfe.MLP_NPARAMS
    blob = _model_blob(rng.standard_normal(n), rng.standard_normal(n), rng.random(n), 123)
    assert len(blob) == 116056
    good = tmp_path / "good.sfem"
    good.write_bytes(blob)
    assert sfe.sfe_model_check_file(str(good)) == sfe.SFE_OK
    assert sfe.sfe_model_check_file(str(tmp_path / "missing.sfem")) == sfe.SFE_EIO

    def variant(name, data):
        p = tmp_path / name
        p.write_bytes(data)
        return sfe.sfe_model_check_file(str(p))

    b = bytearray(blob)
    b[0] ^= 1                                            # magic
    assert variant("magic", bytes(b)) == sfe.SFE_EINVAL
    b = bytearray(blob)
    b[8] = 2                                             # version
    assert variant("version", bytes(b)) == sfe.SFE_EINVAL
    b = bytearray(blob)
    b[12] = 2                                            # layout id
    assert variant("layout", bytes(b)) == sfe.SFE_EINVAL
    b = bytearray(blob)
    b[16] ^= 1                                           # parameter count
    assert variant("count", bytes(b)) == sfe.SFE_EINVAL
    b = bytearray(blob)
    b[32 + 4 * 100] ^= 0x10                              # one parameter bit: hash mismatch
    assert variant("flip", bytes(b)) == sfe.SFE_EINVAL
    assert variant("short", blob[:-1]) == sfe.SFE_EINVAL
    assert variant("long", blob + b"\0") == sfe.SFE_EINVAL
