"""CPU checks of the C ABI: the library loads and exports every declared symbol,
and argument validation rejects bad input before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hsm_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("hsm_build_stencils", "hsm_apply_operator", "hsm_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2303_01760_amd import hsm
    L = hsm.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(hsm.SYMBOLS) == set(_declared())
    assert b"gfx950" in L.hsm_version()


def test_build_rejects_bad_arguments_without_a_gpu():
    from paper_2303_01760_amd import hsm
    L = hsm.lib()
    out = ctypes.c_void_p()
    assert L.hsm_build_stencils(None, 0, None, ctypes.byref(out)) == hsm.E_INVALID
    import numpy as np
    offs = np.array([0, 100], np.int64)
    h = np.array([0.1]); m = np.array([7], np.int32)
    ns = hsm.NodeSetC(2, 1, offs.ctypes.data, 1, 1, 1, h.ctypes.data, m.ctypes.data, None)
    assert L.hsm_build_stencils(ctypes.byref(ns), 0, None, ctypes.byref(out)) == hsm.E_INVALID
    assert b"unsupported" in L.hsm_last_error()
    m[0] = 2
    ns.d = 4
    assert L.hsm_build_stencils(ctypes.byref(ns), 0, None, ctypes.byref(out)) == hsm.E_INVALID
    ns.d = 2
    offs[1] = 5   # domain smaller than the stencil
    assert L.hsm_build_stencils(ctypes.byref(ns), 0, None, ctypes.byref(out)) == hsm.E_INVALID
    assert out.value is None


def test_apply_rejects_bad_arguments():
    from paper_2303_01760_amd import hsm
    L = hsm.lib()
    assert L.hsm_apply_operator(None, 1, 0, None, None, None) == hsm.E_INVALID
    assert L.hsm_permute(None, 0, 0, None, None, None) == hsm.E_INVALID
    assert L.hsm_step(None, 1, None) == hsm.E_INVALID


def test_size_limits_and_empty_selections_are_rejected_on_the_host():
    # the largest node count the 32-bit buffer offsets allow, an empty domain,
    # and an apply that selects no bucket are refused before any device work
    import numpy as np
    from paper_2303_01760_amd import hsm
    L = hsm.lib()
    out = ctypes.c_void_p()
    h = np.array([0.1]); m = np.array([2], np.int32)
    too_many = np.array([0, (1 << 28) - 1], np.int64)            # HSM_MAX_NODES + 1
    ns = hsm.NodeSetC(2, 1, too_many.ctypes.data, 1, 1, 1, h.ctypes.data, m.ctypes.data, None)
    assert L.hsm_build_stencils(ctypes.byref(ns), 0, None, ctypes.byref(out)) == hsm.E_INVALID
    assert b"too many nodes" in L.hsm_last_error()
    empty = np.array([0, 0], np.int64)
    ns = hsm.NodeSetC(2, 1, empty.ctypes.data, 1, 1, 1, h.ctypes.data, m.ctypes.data, None)
    assert L.hsm_build_stencils(ctypes.byref(ns), 0, None, ctypes.byref(out)) == hsm.E_INVALID
    assert out.value is None
    assert L.hsm_apply_operator_buckets(None, 1, 0, 0, None, None, None) == hsm.E_INVALID
    assert b"no bucket" in L.hsm_last_error()
    assert L.hsm_stencils_condition(None, None, None) == hsm.E_INVALID


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    # no CPU fallback: with the HIP library absent every entry point raises
    from paper_2303_01760_amd import hsm
    monkeypatch.setattr(hsm, "_lib", None)
    monkeypatch.setattr(hsm, "LIB_PATH", str(tmp_path / "libhsm.so"))
    with pytest.raises(RuntimeError, match="not built"):
        hsm.lib()


def test_bench_refuses_more_than_one_gpu():
    # the library has no multi-GPU path: bench.py says so and exits non-zero before touching a device
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_binding_structs_match_the_c_header(tmp_path):
    # the ctypes mirrors of the ABI's structs against the header itself:
    # every field's offset and each struct's size, from a C program that
    # includes include/hsm.h (compiled here with the host compiler)
    import ctypes
    import os
    import shutil
    import subprocess
    from paper_2303_01760_amd import hsm as H
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"hsm_nodeset": H.NodeSetC, "hsm_stencils_info": H.StencilsInfoC, "hsm_sim_params": H.SimParamsC,
               "hsm_sim_stats": H.SimStatsC}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "hsm.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run([cc, "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, key, val = ln.split()
        got[(cname, key)] = int(val)
    for cname, cls in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
