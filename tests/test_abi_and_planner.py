"""CPU tests of the C ABI: the library loads, exports every function that
include/lx.h declares, and its host planner (Leja points, scalar phi_l,
divided differences) agrees with the oracle.  No device calls."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle.leja import leja_points, newton_coeffs, phi_mp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "lx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lx_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2310_08344_amd.binding import Library
    return Library.load()


def test_library_exports_every_declared_function(lib):
    names = _declared_functions()
    assert "lx_phi_leja" in names and "lx_spectrum" in names and "lx_exprb_step" in names
    raw = ctypes.CDLL(lib.path)
    for name in names:
        assert hasattr(raw, name), name


def test_binding_covers_the_header(lib):
    from paper_2310_08344_amd.binding import EXPORTED
    assert sorted(EXPORTED) == _declared_functions()


def test_struct_layouts_match_the_header(lib, tmp_path):
    """Sizes and field offsets of the binding's ctypes structures against a C
    compiler's reading of include/lx.h."""
    import shutil
    import subprocess
    from paper_2310_08344_amd.binding import Instance, InstanceResult, LejaOpts, Operator, Stats
    structs = {"lx_operator": Operator, "lx_leja_opts": LejaOpts, "lx_stats": Stats, "lx_instance": Instance,
               "lx_instance_result": InstanceResult}
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lx.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_leja_points_agree_with_oracle(lib):
    M = 1001
    x = lib.leja_points(M)
    xo = leja_points(M)
    assert x[0] == 2.0 and x[1] == -2.0 and x[2] == 0.0
    assert np.max(np.abs(x - xo)) <= 1e-14


@pytest.mark.parametrize("l", [0, 1, 2, 3, 6])
def test_phi_scalar_agrees_with_oracle(lib, l):
    import mpmath as mp
    for z in [-300.0, -105.0, -26.0, -3.0, -1.5, -1.4999, -0.3, -1e-12, 0.0, 1e-9, 0.9, 1.5, 4.0]:
        with mp.workdps(40):
            ref = float(phi_mp(l, z))
        got = lib.phi_scalar(l, z)
        assert abs(got - ref) <= 4e-16 * max(abs(ref), 1e-300) + 1e-300, (l, z, got, ref)


@pytest.mark.parametrize("l,hgamma,alpha,sigma", [(0, 5.1, 1.0, 1.0), (1, 25.6, 1.0, 1.0),
                                                 (3, 25.6, 1.0, 32.0 / 9.0), (1, 52.5, 0.75, 0.75),
                                                 (2, 150.0, 1.0, 1.0)])
def test_newton_coeffs_are_correctly_rounded(lib, l, hgamma, alpha, sigma):
    """The library's double-double divided differences against 50-digit
    ones taken at the library's own Leja points: each coefficient is
    correctly rounded (0.5 ulp, plus one ulp of slack) down to the
    double-double floor of ~1e-32 of max|f|: such terms cannot reach the
    polynomial, whose Newton basis grows by far less than 1e16."""
    import mpmath as mp
    from oracle.leja import divided_differences_mp
    M = 160
    h = 2.0e-3
    gamma = hgamma / h
    c = -2.0 * gamma
    d = lib.newton_coeffs(l, h, c, gamma, M, alpha=alpha, sigma=sigma)
    xl = lib.leja_points(M)
    with mp.workdps(50):
        a = mp.mpf(alpha) * mp.mpf(h)
        fs = [mp.mpf(sigma) * phi_mp(l, a * (mp.mpf(c) + mp.mpf(gamma) * mp.mpf(float(x)))) for x in xl]
        ref = np.array([float(v) for v in divided_differences_mp(xl, fs)])
    err = np.abs(d - ref)
    floor = 1e-30 * np.max(np.abs(ref))
    assert np.all(err <= 2.3e-16 * np.abs(ref) + floor), int(np.argmax(err / (np.abs(ref) + floor)))


def test_newton_coeffs_close_to_oracle_with_its_own_points(lib):
    # the two Leja tables agree to ~2e-15, which moves the coefficients by a
    # similar relative amount
    h, gamma = 1.0, 25.6
    d = lib.newton_coeffs(1, h, -2 * gamma, gamma, 120)
    do = newton_coeffs(1, h, -2 * gamma, gamma, 120)
    assert np.all(np.abs(d - do) <= 1e-13 * np.abs(do) + 1e-30)


def test_planner_rejects_bad_requests(lib):
    from paper_2310_08344_amd.binding import LX_EINVAL
    out = (ctypes.c_double * 4)()
    assert lib.c.lx_leja_points(0, out) == LX_EINVAL
    assert lib.c.lx_leja_points(5000, out) == LX_EINVAL
    assert lib.c.lx_newton_coeffs(-1, 1.0, 1.0, 1.0, -1.0, 0.5, 4, out) == LX_EINVAL
    assert lib.c.lx_newton_coeffs(1, 1.0, 1.0, 1.0, -1.0, 0.5, 4, None) == LX_EINVAL
    assert lib.c.lx_status_string(3) == b"LX_ENOTCONV"
