"""The three-dimensional oracle's pins catch plausible mistakes: each case
compiles a copy of dugks_oracle3d.c with one planted error (on the CPU, into a
temporary directory) and runs the pins of test_oracle3d_pins.py against it in
a child process; the pins must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dugks_oracle3d.c")

MUTATIONS = {
    "mixed_term_sign": ("2.0 * d[0] * d[2] * hx[1]", "-2.0 * d[0] * d[2] * hx[1]"),
    "transverse_displacement_sign": ("d[a] = -XI(c, a, q) * h;", "d[a] = XI(c, a, q) * h;"),
    "face_tau": ("double tb = 0.5 * (tau[ml] + tau[me]);", "double tb = tau[me];"),
    "negative_side_foot_point": ("d[ax] = -0.5 * w[ax] - e * h;  /* from the own",
                                 "d[ax] = 0.5 * w[ax] - e * h;  /* from the own"),
    "equilibrium_component": ("eu += XI(c, a, q) * u[a];", "eu += XI(c, a == 2 ? 1 : a, q) * u[a];"),
    "z_flux_width": ("s += XI(c, ax, q) * (fhi - flo) / w[ax];", "s += XI(c, ax, q) * (fhi - flo) / w[ax == 2 ? 0 : ax];"),
    "mixed_derivative_width": ("hx[p] = s / (4.0 * h[a] * h[b]);", "hx[p] = s / (4.0 * h[a] * h[a]);"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_a_pin(name, tmp_path):
    a, b = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(a) == 1, "the mutation no longer matches the oracle's text"
    path = tmp_path / "mutant.c"
    lib = tmp_path / "mutant.so"
    path.write_text(src.replace(a, b))
    subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", str(path), "-lm", "-o", str(lib)])
    code = (f"import sys, ctypes; sys.path.insert(0, {ROOT!r}); import oracle.oracle3d as o3; "
            f"o3._lib = ctypes.CDLL({str(lib)!r}); import pytest; "
            f"sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', "
            f"{os.path.join(ROOT, 'tests', 'test_oracle3d_pins.py')!r}]))")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 1, r.stdout[-2000:] + r.stderr[-2000:]
