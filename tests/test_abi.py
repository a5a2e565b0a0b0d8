"""The C-ABI library loads and exports every symbol include/hsla.h declares
(no GPU needed: nothing here launches work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hsla_[a-z_0-9]+)\s*\(", text)))


def _lib_path():
    return os.path.join(ROOT, "paper_2601_13994_amd", "libhsla.so")


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (torch first: one HIP runtime per process)

    path = _lib_path()
    if not os.path.exists(path):
        from paper_2601_13994_amd import build

        build.build()
    return ctypes.CDLL(path)


def test_exports_match_header(lib):
    names = _declared("hsla.h")
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2601_13994_amd import _lib

    assert sorted(_lib.EXPORTS) == [n for n in _declared("hsla.h")]


def test_host_only_entry_points(lib):
    lib.hsla_status_string.restype = ctypes.c_char_p
    assert lib.hsla_status_string(-2) == b"invalid CSR pattern"
    assert lib.hsla_status_string(0) == b"ok"
    from paper_2601_13994_amd import _lib

    o = _lib.Opts()
    lib.hsla_opts_default(ctypes.byref(o))
    assert o.rtol == 1e-8 and o.precond == 1 and o.method == 0 and o.use_graph == 1
    assert ctypes.sizeof(_lib.Info) == 80


def test_struct_layout_matches_header(tmp_path):
    """ctypes mirrors of hsla_opts / hsla_info have the layout a C compiler
    gives the header's structs (every field's offset, and the sizes)."""
    import subprocess

    from paper_2601_13994_amd import _lib

    lines = []
    structs = (("hsla_opts", _lib.Opts), ("hsla_info", _lib.Info), ("hsla_tuning", _lib.Tuning),
               ("hsla_tune_state", _lib.TuneState))
    for cname, mirror in structs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in mirror._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"hsla.h\"\nint main(void) {\n"
                   + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in filter(None, out):
        parts = line.split()
        got[tuple(parts[:-1])] = int(parts[-1])
    for cname, mirror in structs:
        assert got[(cname, "size")] == ctypes.sizeof(mirror)
        for f, _ in mirror._fields_:
            assert got[(cname, f)] == getattr(mirror, f).offset, (cname, f)


def test_product_path_has_no_cpu_fallback():
    """The package never imports the oracle, and fails loudly without a GPU."""
    import subprocess
    import sys

    code = ("import sys, paper_2601_13994_amd as p, torch\n"
            "assert 'oracle' not in sys.modules\n"
            "try:\n"
            "    p._lib.handle()\n"
            "except RuntimeError as e:\n"
            "    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       env={**os.environ, "HIP_VISIBLE_DEVICES": os.environ.get("HIP_VISIBLE_DEVICES", "")})
    assert r.returncode == 0, r.stderr
    import torch

    if not torch.cuda.is_available():
        assert "raised" in r.stdout
    for f in os.listdir(os.path.join(ROOT, "paper_2601_13994_amd")):
        if f.endswith(".py"):
            src = open(os.path.join(ROOT, "paper_2601_13994_amd", f)).read()
            assert "import oracle" not in src and "from oracle" not in src
