"""The C ABI without a GPU: the library loads, exports exactly what include/qmc.h declares,
its host-side setup calls agree with the oracle, and argument errors need no device."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import digital
from synth import sobol_direction_init

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qmc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qmc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2307_15584_amd import _lib

    return _lib.load()


def test_every_declared_symbol_is_exported_and_bound(lib):
    from paper_2307_15584_amd import _lib

    names = _declared()
    assert names, "no declarations parsed"
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_lib.SIGNATURES) == names


def test_version(lib):
    assert lib.qmc_version().decode().startswith("qmc-gfx950")


def test_primitive_polynomials_match_oracle(lib):
    import paper_2307_15584_amd as q

    got = q.qmc_primitive_polynomials(200)
    assert list(map(int, got)) == digital.primitive_polynomials(200)


@pytest.mark.parametrize("s", [1, 4, 32, 64])
def test_sobol_matrices_match_oracle(s):
    import paper_2307_15584_amd as q

    di = sobol_direction_init(s, 0)
    assert np.array_equal(q.qmc_sobol_matrices(s, di), digital.sobol_matrices(s, di))


def test_sobol_matrices_rejects_bad_direction_numbers():
    import paper_2307_15584_amd as q

    di = sobol_direction_init(4, 0)
    di[2, 1] = 2  # even
    with pytest.raises(q.QMCError) as e:
        q.qmc_sobol_matrices(4, di)
    assert e.value.status == 1
    with pytest.raises(q.QMCError) as e:
        q.qmc_sobol_matrices(65, np.ones((65, 16), np.uint32))
    assert e.value.status == 2


@pytest.mark.parametrize("s,columns", [(1, 64), (8, 1), (8, 20), (8, 32), (16, 52), (64, 64)])
def test_wide_sobol_matrices_match_oracle(s, columns):
    import paper_2307_15584_amd as q
    from oracle import partition

    di = sobol_direction_init(s, 0)
    assert np.array_equal(q.qmc_sobol_matrices_wide(s, di, columns), partition.sobol_matrices_wide(s, di, columns))


def test_wide_sobol_matrices_reject_column_counts():
    import paper_2307_15584_amd as q

    di = sobol_direction_init(4, 0)
    for columns in (0, 65):
        with pytest.raises(q.QMCError) as e:
            q.qmc_sobol_matrices_wide(4, di, columns)
        assert e.value.status == 2


def test_generation_rejects_null_context(lib):
    st = lib.qmc_generate_sobol64(None, None, ctypes.c_void_p(16), 64, 4, 3, 5, 1 << 40, 16, None, None, 0,
                                  ctypes.c_void_p(4096), None, 16)
    assert st == 1 and b"context" in lib.qmc_last_error()
    st = lib.qmc_generate_lattice64(None, None, ctypes.c_void_p(16), 4, 3, 5, 1 << 40, 16, None, 0,
                                    ctypes.c_void_p(4096), None, 16)
    assert st == 1 and b"context" in lib.qmc_last_error()
    st = lib.qmc_generate_sobol(None, None, ctypes.c_void_p(16), 4, 0, 16, None, None, 0,
                                ctypes.c_void_p(4096), None, 16)
    assert st == 1
    assert b"context" in lib.qmc_last_error()
    st = lib.qmc_generate_lattice(None, None, ctypes.c_void_p(16), 4, 0, 16, None, 0, ctypes.c_void_p(4096), None, 16)
    assert st == 1


def test_header_constants_match_the_binding():
    """Every #define QMC_* integer in the header has the same value in the Python binding."""
    from paper_2307_15584_amd import _lib

    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    defines = dict(re.findall(r"#define\s+(QMC_[A-Z0-9_]+)\s+(\d+)u?\b", text))
    assert "QMC_PIXEL_HILBERT_SHIFT" in defines and "QMC_LATTICE_INSTANCES4" in defines
    for name, value in defines.items():
        if hasattr(_lib, name):
            assert getattr(_lib, name) == int(value), name
    for name in ("QMC_PIXEL_NUS", "QMC_PIXEL_SHIFT", "QMC_PIXEL_RANDOM_GENERATOR", "QMC_PIXEL_HILBERT_SHIFT",
                 "QMC_LATTICE_INSTANCES4", "QMC_SHIFT_XOR", "QMC_LATTICE_BACKWARD"):
        assert hasattr(_lib, name), name


def test_struct_mirrors_match_the_header(tmp_path):
    """The binding's ctypes structs have the C structs' size and field offsets (compiled with gcc
    against include/qmc.h)."""
    import shutil
    import subprocess

    from paper_2307_15584_amd import _lib

    if not shutil.which("gcc"):
        pytest.skip("no host C compiler")
    mirrors = {"qmc_sampler": _lib.Sampler, "qmc_integrand": _lib.Integrand}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "qmc.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
