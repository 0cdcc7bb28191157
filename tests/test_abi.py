"""The C-ABI library loads and exports every entry point of include/wproj.h (CPU only, no compute)."""
import ctypes as C
import os
import re

import pytest

import paper_1307_3424_amd as wp
from paper_1307_3424_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?\**\s*\b(wp_[A-Za-z0-9_]+)\s*\(", src, re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    lib = wp.load()
    names = declared_functions()
    assert len(names) >= 14
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(_lib.SIGNATURES) == names


def test_version_and_error_string():
    lib = wp.load()
    assert lib.wp_version().startswith(b"wproj")
    assert isinstance(lib.wp_last_error(), bytes)


@pytest.mark.parametrize("args,frag", [
    ((100, 0.0349, 4, 0.0, 0, 0), b"power of two"),
    ((16, 0.0349, 4, 0.0, 0, 0), b"power of two"),
    ((64, 1.5, 4, 0.0, 0, 0), b"fov_L"),
    ((64, 0.0349, 5, 0.0, 0, 0), b"kb_W"),
    ((64, 0.0349, 4, 0.0, 7, 0), b"chirp"),
    ((64, 0.0349, 4, 0.0, 0, 9), b"aphys"),
])
def test_plan_validation_happens_before_any_device_call(args, frag):
    lib = wp.load()
    h = C.c_void_p()
    st = lib.wp_plan_create(C.byref(h), *args)
    assert st == -1 and not h.value
    assert frag in lib.wp_last_error()


def test_null_arguments_rejected():
    lib = wp.load()
    assert lib.wp_plan_create(None, 64, 0.03, 4, 0.0, 0, 0) == -1
    assert lib.wp_apply_Phi(None, None, None, None, None, None) == -1
    assert lib.wp_build_G_count(None, 10, None, None, None, 0.9, None, None, None, None) == -1
    assert lib.wp_plan_destroy(None) == 0


def test_wp_G_layout_matches_header(tmp_path):
    """Size and field offsets of the binding's wp_G equal what a C compiler makes of the header."""
    import subprocess
    fields = [f for f, _ in _lib.WpG._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"wproj.h\"\nint main(void) {\n"
                   + 'printf("%zu\\n", sizeof(wp_G));\n'
                   + "".join(f'printf("%zu\\n", offsetof(wp_G, {f}));\n' for f in fields) + "return 0; }\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out[0] == C.sizeof(_lib.WpG)
    assert out[1:] == [getattr(_lib.WpG, f).offset for f in fields]


def test_library_db8_filter_matches_oracle_derivation():
    """The library derives Daubechies-8 on its own (host, no GPU): same taps as the oracle."""
    import numpy as np
    from oracle import wavelet
    h = np.array(wp.db8_filter())
    assert np.abs(h - wavelet.daubechies_lowpass(8)).max() < 1e-12
    assert abs(h.sum() - np.sqrt(2)) < 1e-13 and abs(np.dot(h, h) - 1) < 1e-13


def test_library_shares_the_hip_runtime_of_torch():
    """Loading the library before torch must not bring in a second HIP runtime:
    two runtimes in one process make the library's device calls fail."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_1307_3424_amd._lib as L; L.load()\n"
        "paths = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
        "print(len(paths)); print(*sorted(paths))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split()[0] == "1", out.stdout
