"""The C ABI without a GPU: the library loads, exports every function that
include/iugkp.h declares, the Python declarations cover them, the ctypes
structures have the header's layout (sizes and field offsets from a C probe
compiled against the header with gcc), and the host-only calls answer."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iugkp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(iugkp_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2506_09465_amd import _lib, build
    if not shutil.which("hipcc") and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("no hipcc")
    build.build(force=False)      # cross-compiles for gfx950 when a source is newer
    return _lib


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    so = C.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing
    bound = {n for n, _, _ in lib.SIGNATURES}
    assert set(names) <= bound, sorted(set(names) - bound)


def test_struct_layout_matches_header(lib, tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    structs = {"iugkp_problem": lib.Problem, "iugkp_options": lib.Options, "iugkp_stats": lib.Stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["return 0; }"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run([gcc, "-std=c11", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            s, f, v = line.split()
            got[(s, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def test_host_only_calls(lib):
    L = lib.lib()
    assert L.iugkp_strerror(lib.E_FIXED_OVERFLOW).decode() == "fixed-point overflow"
    assert L.iugkp_strerror(lib.OK)
    # D_eff tends to lambda^2 / 3 for a cell much finer than the path, lambda delta / 4
    # for a much coarser one
    assert abs(L.iugkp_d_eff(1.0, 1e-3) / (1.0 / 3.0) - 1.0) < 1e-2
    assert abs(L.iugkp_d_eff(1e-3, 1.0) / (1e-3 / 4.0) - 1.0) < 1e-2
    # argument checks answer before any device call
    assert L.iugkp_create(None, None, None, None) == lib.E_INVALID_ARG
    assert L.iugkp_get_residuals(None, None, 0) == lib.E_INVALID_ARG
