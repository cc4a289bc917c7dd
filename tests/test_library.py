"""Host-side checks of the native library (no GPU calls): it loads, and it
exports every symbol include/emin.h declares; the header and the binding
agree on the struct layouts."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "emin.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(emin_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2208_02995_amd import emin

    lib = emin.load_library()
    names = _declared()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(lib, n), f"{n} not exported"
    assert set(names) == set(emin.EXPORTS)


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof from the C header (compiled with gcc) equal the
    ctypes mirrors."""
    import shutil
    import subprocess

    from paper_2208_02995_amd import emin

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "lay.c"
    fields = {"emin_csr": [f for f, _ in emin.emin_csr._fields_],
              "emin_opts": [f for f, _ in emin.emin_opts._fields_],
              "emin_stats": [f for f, _ in emin.emin_stats._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(l.split() for l in out if l.strip())
    for st, fs in fields.items():
        cls = getattr(emin, st)
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in fs:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, f"{st}.{f}"


def test_opts_default_host_only():
    from paper_2208_02995_amd import emin

    o = emin.emin_opts_default()
    assert (o.precision, o.precond, o.block, o.maxit, o.tau, o.pattern_power) == (0, 0, 1, 10, 0.0, 1)


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(OSError):
        _load_fresh(str(tmp_path / "nope.so"))


def _load_fresh(path):
    from paper_2208_02995_amd import emin

    saved = emin._lib
    emin._lib = None
    try:
        return emin.load_library(path)
    finally:
        emin._lib = saved
