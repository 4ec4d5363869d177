"""The C-ABI library loads on the CPU host and exports every symbol the
public header declares (no compute calls: there may be no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "abd.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(abd_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("abd_vertex_map", "abd_candidates", "abd_barrier_grad_hess", "abd_ccd_max_step",
              "abd_orthogonality", "abd_newton_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2201_10022_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libabd.so not built")
    L = ctypes.CDLL(_lib.LIB_PATH)
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) == set(_lib.EXPORTS)


def test_binding_has_no_cpu_fallback():
    # the product package must not import the oracle
    pkg = os.path.join(ROOT, "paper_2201_10022_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f


def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes structures have the size and field offsets the C header gives
    them (compiled here with the host C compiler)."""
    import shutil
    import subprocess
    from paper_2201_10022_amd import _lib
    cc = shutil.which("gcc")
    if cc is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("no host C compiler or HIP headers")
    structs = {"abd_scene": _lib.AbdScene, "abd_params": _lib.AbdParams, "abd_stats": _lib.AbdStats,
               "abd_tune": _lib.AbdTune}
    lines = ['#include <stdio.h>', '#include "abd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True, timeout=120)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True, timeout=60).stdout
    got = {}
    for ln in out.splitlines():
        s, f, v = ln.split()
        got[(s, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_binding_signatures_match_the_header_arity():
    """Every binding signature takes as many arguments as the header's
    prototype, pointer arguments are bound as pointers and scalar arguments
    with the header's width and kind."""
    from paper_2201_10022_amd import _lib
    txt = open(os.path.join(ROOT, "include", "abd.h")).read()
    protos = re.findall(r"^\s*(?:int|const char \*)\s*(abd_\w+)\s*\(([^;]*)\)\s*;", txt, re.M)
    assert protos
    scalar = {"int": ctypes.c_int, "int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double}
    for name, args in protos:
        params = [a.strip() for a in args.replace("\n", " ").split(",") if a.strip()]
        if params == ["void"]:
            params = []
        argtypes = _lib.SIGNATURES[name][0]
        assert len(argtypes) == len(params), (name, params)
        for p, t in zip(params, argtypes):
            is_ptr = issubclass(t, (ctypes._Pointer, ctypes.c_void_p, ctypes.c_char_p))
            assert is_ptr == ("*" in p or "hipStream_t" in p), (name, p, t)
            if not is_ptr:
                ctype = " ".join(p.split()[:-1])
                assert ctypes.sizeof(t) == ctypes.sizeof(scalar[ctype]), (name, p, t)
                assert (t is ctypes.c_double) == (ctype == "double"), (name, p, t)
