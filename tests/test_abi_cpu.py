"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/pw.h, and rejects invalid arguments before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pw.h")
LIB = os.path.join(ROOT, "paper_2507_08578_amd", "libpwdft.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2507_08578_amd import _lib
    return _lib.load(LIB)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pw_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for n in ("pw_apply_h", "pw_cheb_filter", "pw_orthonormalize", "pw_rayleigh_ritz"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_symbol(lib):
    from paper_2507_08578_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_status_strings(lib):
    assert lib.pw_status_string(0) == b"PW_OK"
    assert lib.pw_status_string(5) == b"PW_ERR_NOT_POSDEF"
    assert lib.pw_version().decode().count(".") == 2


def test_invalid_arguments_without_device(lib):
    out = ctypes.c_void_p()
    assert lib.pw_ctx_create(0, None, None) == 1            # out == NULL
    assert lib.pw_ctx_create(-1, None, ctypes.byref(out)) == 1
    assert b"device" in lib.pw_last_error(None)
    assert lib.pw_apply_h(None, 0, 4, None, 10, None, 10) == 1
    assert lib.pw_cheb_filter(None, 0, 8, 0.0, 1.0, -1.0, 4, None, 10, None, 0) == 1
    assert lib.pw_orthonormalize(None, 0, 4, None, 10, None, 0) == 1
    assert lib.pw_rayleigh_ritz(None, 4, None, 10, None, 10, None, None) == 1
    assert lib.pw_ham_destroy(None) == 1
    assert lib.pw_ctx_destroy(None) == 1
    assert b"NULL" in lib.pw_last_error(None)


def _c_layout(tmp_path, ctype, struct):
    """Offsets and size of a C struct of pw.h as gcc lays it out."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    fields = [f[0] for f in struct._fields_]
    src = tmp_path / f"off_{ctype}.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "pw.h"\nint main(void){\n' +
                   "".join(f'printf("%zu\\n", offsetof({ctype}, {f}));\n' for f in fields) +
                   f'printf("%zu\\n", sizeof({ctype}));\nreturn 0;}}\n')
    exe = tmp_path / f"off_{ctype}"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    return fields, out


def test_desc_layout_matches_header(tmp_path):
    """The ctypes mirror of pw_ham_desc has the C compiler's offsets (checked with gcc)."""
    from paper_2507_08578_amd._lib import PwHamDesc
    fields, out = _c_layout(tmp_path, "pw_ham_desc", PwHamDesc)
    assert out[:-1] == [getattr(PwHamDesc, f).offset for f in fields]
    assert out[-1] == ctypes.sizeof(PwHamDesc)


def test_tuning_layout_matches_header(tmp_path):
    from paper_2507_08578_amd._lib import PwTuning
    fields, out = _c_layout(tmp_path, "pw_tuning", PwTuning)
    assert out[:-1] == [getattr(PwTuning, f).offset for f in fields]
    assert out[-1] == ctypes.sizeof(PwTuning)
