"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every symbol include/dugks.h and include/dugks3d.h declare, and rejects invalid
descriptors before touching the device."""
import os
import re

import numpy as np
import pytest

from paper_1709_05458_amd import cases as C
from paper_1709_05458_amd import dugks

INC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
HDR = os.path.join(INC, "dugks.h")


def declared_functions(path=HDR):
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dugks3?d?_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    names3 = declared_functions(os.path.join(INC, "dugks3d.h"))
    assert len(names3) >= 9 and all(n.startswith("dugks3d_") for n in names3)
    L = dugks.lib()
    for n in names + names3:
        assert hasattr(L, n), n


def test_3d_descriptor_validation_on_the_host():
    def expect(code, case, **kw):
        with pytest.raises(dugks.DugksError) as e:
            dugks.Solver3D(case, **kw)
        assert e.value.code == code, str(e.value)

    RT = 1.0 / 3.0
    bad = C.abc_case(8, C.d3q19(RT))
    bad.tau = np.full(bad.tau.shape, bad.dt / 12.5)     # beyond dt/tau <= 12
    expect(-2, bad)
    bad = C.abc_case(8, C.d3q19(RT), cfl=1.5)           # CFL above 1
    expect(-1, bad)
    bad = C.abc_case(8, C.d3q27(RT), shape=(8, 2, 8))   # too few cells
    expect(-1, bad)
    c2 = C.abc_case(8, C.d3q19(RT))
    c2.rho0 = 0.0
    expect(-1, c2, precision=dugks.FP32_DELTA)
    vs = C.d3q19(RT)
    vs.w = vs.w * 1.01                                  # weights not moment-exact
    expect(-3, C.abc_case(8, vs))
    vs15 = C.d3q27(RT)                                  # a set of neither 19 nor 27 velocities
    keep = np.count_nonzero(vs15.xi, axis=0) != 2
    vs15 = C.VelocitySet("D3Q15", vs15.xi[:, keep], np.where(np.count_nonzero(vs15.xi[:, keep], axis=0) == 0,
                                                             2.0 / 9.0, np.where(np.count_nonzero(
                                                                 vs15.xi[:, keep], axis=0) == 1, 1.0 / 9.0,
                                                                 1.0 / 72.0)), RT)
    expect(-7, C.abc_case(8, vs15))


def test_strerror_covers_codes():
    L = dugks.lib()
    for code in range(0, -8, -1):
        assert L.dugks_strerror(code) not in (b"", b"unknown error")
    assert L.dugks_strerror(-99) == b"unknown error"


def _expect(code, case, **kw):
    with pytest.raises(dugks.DugksError) as e:
        dugks.Solver(case, **kw)
    assert e.value.code == code, str(e.value)


def test_descriptor_validation_on_the_host():
    case = C.tgv_case(16)
    bad = C.tgv_case(16)
    bad.tau[:] = bad.dt / 12.5           # beyond the dt/tau <= 12 bound of the paper
    _expect(-2, bad)
    bad = C.tgv_case(16)
    bad.tau[3, 4] = bad.dt / 13.0        # one cell of a tau field
    _expect(-2, bad)
    bad = C.tgv_case(16)
    bad.dt = 2.0 * bad.grid.dmin / bad.vs.cmax   # CFL 2
    _expect(-1, bad)
    bad = C.tgv_case(16)
    bad.grid = C.uniform_grid(2, 16)     # too few cells
    _expect(-1, bad)
    bad = C.tgv_case(16)
    bad.bc = (C.BC_PERIODIC, C.BC_BOUNCE_BACK, C.BC_PERIODIC, C.BC_PERIODIC)
    _expect(-1, bad)
    # weights that are not moment-exact are refused unless allowed
    nc = C.cavity_case(16, C.newton_cotes(12, 0.5), wall=C.BC_DIFFUSE, tau=0.1)
    _expect(-3, nc)
    # bounce-back needs mirror velocities of equal weight
    vs = C.d2q9(1 / 3)
    vs.w = vs.w.copy()
    vs.w[0], vs.w[8] = vs.w[0] * 1.1, vs.w[8] * 0.9
    bb = C.cavity_case(16, vs, tau=0.1)
    _expect(-1, bb)
    # an unknown time integrator
    _expect(-1, C.tgv_case(16), scheme=7)
    # FP32-delta storage needs a reference density
    c2 = C.tgv_case(16)
    c2.rho0 = 0.0
    _expect(-1, c2, precision=dugks.FP32_DELTA)
    # the time-discretization family takes 1/3 <= a <= 1/2, and only the third-order scheme
    _expect(-1, C.tgv_case(16), family_a=0.7)
    _expect(-1, C.tgv_case(16), family_a=0.45, scheme=dugks.T2S3)
    # an unknown reconstruction
    _expect(-1, C.tgv_case(16), reconstruction=5)
    # no relaxation time at all: no tau, tau0 = 0 and no Knudsen number
    _expect(-1, C.tgv_case(16), kn=(0.0, 1.0))
    assert case is not None


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(dugks, "_lib", None)
    monkeypatch.setattr(dugks, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        dugks.lib()


def test_bench_finds_the_stored_traffic_summary_of_its_default_workload():
    # the name is built from the velocity set's name ("D2Q37"); the file on
    # disk is lower case, and a case-sensitive file system must still find it
    import bench
    from paper_1709_05458_amd import cases as C
    name = bench.traffic_summary_name(2048, C.d2q37(1.0 / 3.0).name)
    assert os.path.exists(os.path.join(bench.PROFILES, name)), name


def test_bench_refuses_more_than_one_gpu():
    # this build measures one GPU; asking for more must fail with a message,
    # before anything touches a device
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
