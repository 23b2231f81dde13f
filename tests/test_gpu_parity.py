"""GPU parity: the HIP sweep (through the C ABI) against the oracle, element
by element on the same seeded inputs.

FP64: one step compared on every (q, cell) of fhat to 1e-13 of its scale;
several steps compared on density and velocity to 1e-12 relative (the target
stated for FP64).  FP32-delta storage: velocity within 1e-5 of its scale.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1709_05458_amd import cases as C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():   # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1709_05458_amd import dugks  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _perturb(case, seed, amp=0.01):
    """Add a seeded smooth + random perturbation to the initial fields."""
    g = case.grid
    X, Y = np.meshgrid((g.xc - g.xf[0]) / (g.xf[-1] - g.xf[0]), (g.yc - g.yf[0]) / (g.yf[-1] - g.yf[0]))
    z = C.normal(seed, 3 * g.nx * g.ny).reshape(3, g.ny, g.nx)
    case.rho = case.rho + amp * (np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + 0.3 * z[0])
    case.ux = case.ux + amp * (np.cos(2 * np.pi * Y) + 0.3 * z[1])
    case.uy = case.uy + amp * (np.sin(4 * np.pi * X) + 0.3 * z[2])
    return case


def _mk(name):
    d2q9 = C.d2q9(1.0 / 3.0)
    if name == "tgv32_d2q9":
        return C.tgv_case(32, d2q9)
    if name == "tgv_ragged_37x29":
        c = C.tgv_case(37, d2q9)
        c.grid = C.uniform_grid(37, 29, 2 * math.pi, 2 * math.pi * 29 / 37)
        c.rho, c.ux, c.uy = (np.ones((29, 37)), np.zeros((29, 37)), np.zeros((29, 37)))
        c.tau = np.full((29, 37), c.tau[0, 0])
        return _perturb(c, 5)
    if name == "tgv24_d2q37":
        return C.tgv_case(24, C.d2q37(1.0 / 3.0))
    if name == "tgv_tau_field":
        c = C.tgv_case(40, d2q9)
        c.tau = C.perturbed_tau(c.tau[0, 0], c.tau.shape, 0.05, 77)
        return c
    if name == "cavity_bb_33x30":
        c = C.cavity_case(33, d2q9, re=100.0)
        c.grid = C.uniform_grid(33, 30)
        c.rho, c.ux, c.uy = (np.ones((30, 33)), np.zeros((30, 33)), np.zeros((30, 33)))
        c.tau = np.full((30, 33), c.tau[0, 0])
        return _perturb(c, 6)
    if name == "cavity_bb_tanh":
        c = C.cavity_case(24, d2q9, grid=C.tanh_grid(24, 24), re=100.0)
        return _perturb(c, 7)
    if name == "couette_ds_d2q9":
        c = C.couette_case(20, d2q9, tau=0.05, U=0.05, cfl=0.5)
        return _perturb(c, 8)
    if name == "cavity_ds_d2q37_tanh":
        vs = C.d2q37(0.5)
        c = C.cavity_case(20, vs, wall=C.BC_DIFFUSE, grid=C.tanh_grid(20, 20), tau=0.05, lid=0.1)
        return _perturb(c, 9)
    if name == "cavity_bb_d2q37_48":
        c = C.cavity_case(48, C.d2q37(1.0 / 3.0), re=200.0)
        return _perturb(c, 10)
    if name == "nc8_ds_tanh":
        vs = C.newton_cotes(8, 0.5, renormalize=True)
        c = C.cavity_case(18, vs, wall=C.BC_DIFFUSE, grid=C.tanh_grid(18, 18), tau=0.3, lid=0.1)
        return _perturb(c, 11)
    if name == "nc16_ds_couette":
        vs = C.newton_cotes(16, 0.5, renormalize=True)
        c = C.couette_case(20, vs, tau=C.kn_to_tau(1.0, 0.5), U=0.146, cfl=0.25,
                           grid=C.Grid(C.uniform_grid(20, 20).xf, C.tanh_faces(20)))
        return _perturb(c, 12)
    if name == "nc28_cavity_kn1":
        # rarefied lid-driven cavity, reduced size: Newton-Cotes 28 x 28 on
        # [-4, 4] sqrt(RT), tanh cells, Kn = 1, diffuse walls, lid 0.146
        vs = C.newton_cotes(28, 0.5)
        c = C.cavity_case(24, vs, wall=C.BC_DIFFUSE, grid=C.tanh_grid(24, 24),
                          tau=C.kn_to_tau(1.0, 0.5), lid=0.146, cfl=0.25)
        return c
    raise KeyError(name)


FP64_CASES = ["tgv32_d2q9", "tgv_ragged_37x29", "tgv24_d2q37", "tgv_tau_field", "cavity_bb_33x30",
              "cavity_bb_tanh", "couette_ds_d2q9", "cavity_ds_d2q37_tanh", "cavity_bb_d2q37_48"]


def _allow(case):
    return abs(case.vs.moment_defect()["sum_w_minus_1"]) > 1e-10


def _pair(case, kappa, **kw):
    o = oracle.Oracle(case, literal_taylor=(kappa == 1.0))
    s = dugks.Solver(case, dugks.FP64, taylor_quad=kappa, allow_defect=_allow(case), **kw)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    return o, s


@pytest.mark.parametrize("kappa", [1.0, 0.5])
@pytest.mark.parametrize("name", FP64_CASES)
def test_fp64_one_step_every_element(name, kappa):
    case = _mk(name)
    say(f"[gpu] fp64 one step {name} kappa={kappa} {case.grid.nx}x{case.grid.ny} Q={case.vs.nq}")
    o, s = _pair(case, kappa)
    fh0 = o.init_fhat()
    assert np.abs(s.get_fhat() - fh0).max() < 1e-15 * np.abs(fh0).max()
    want = o.step(fh0)
    s.step(1)
    s.sync()
    got = s.get_fhat()
    err = np.abs(got - want).max() / np.abs(want).max()
    say(f"    max rel err {err:.2e}  ({s.describe()})")
    assert err < 1e-13
    s.close()


@pytest.mark.parametrize("name,steps", [("tgv32_d2q9", 200), ("tgv24_d2q37", 60),
                                        ("cavity_bb_33x30", 100), ("couette_ds_d2q9", 100),
                                        ("cavity_ds_d2q37_tanh", 40), ("tgv_tau_field", 60)])
def test_fp64_many_steps_macroscopic(name, steps):
    case = _mk(name)
    say(f"[gpu] fp64 {steps} steps {name}")
    o, s = _pair(case, 1.0)
    fh = o.run(o.init_fhat(), steps)
    ro, uxo, uyo = o.moments(fh)
    s.step(steps)
    s.sync()
    r, ux, uy = s.moments()
    us = max(np.abs(uxo).max(), np.abs(uyo).max())
    e_rho = np.abs(r - ro).max() / np.abs(ro).max()
    e_u = max(np.abs(ux - uxo).max(), np.abs(uy - uyo).max()) / us
    say(f"    rho {e_rho:.2e}  u {e_u:.2e}")
    assert e_rho < 1e-12 and e_u < 1e-12
    s.close()


@pytest.mark.parametrize("tile", [(16, 16), (64, 4), (8, 8), (32, 16)])
def test_fp64_tile_shapes_agree(tile):
    case = _mk("cavity_bb_33x30")
    say(f"[gpu] tile {tile}")
    o, s = _pair(case, 1.0, tile=tile)
    want = o.step(o.init_fhat())
    s.step(1)
    got = s.get_fhat()
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()
    s.close()


@pytest.mark.parametrize("name,steps", [("tgv32_d2q9", 200), ("tgv24_d2q37", 100),
                                        ("cavity_bb_33x30", 200), ("couette_ds_d2q9", 200),
                                        ("cavity_ds_d2q37_tanh", 60)])
def test_fp32_delta_against_fp64_oracle(name, steps):
    case = _mk(name)
    say(f"[gpu] fp32-delta {steps} steps {name}")
    o = oracle.Oracle(case)
    fh = o.run(o.init_fhat(), steps)
    ro, uxo, uyo = o.moments(fh)
    s = dugks.Solver(case, dugks.FP32_DELTA)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    s.step(steps)
    s.sync()
    r, ux, uy = s.moments()
    us = max(np.abs(uxo).max(), np.abs(uyo).max())
    e_u = max(np.abs(ux - uxo).max(), np.abs(uy - uyo).max()) / us
    e_rho = np.abs(r - ro).max()
    say(f"    u {e_u:.2e}  rho {e_rho:.2e}")
    assert e_u < 1e-5 and e_rho < 1e-6
    s.close()


def test_periodic_conservation_fp64_and_fp32():
    case = _mk("tgv_ragged_37x29")
    for prec, tol in ((dugks.FP64, 1e-13), (dugks.FP32_DELTA, 1e-9)):
        say(f"[gpu] conservation precision={prec}")
        s = dugks.Solver(case, prec)
        s.init_equilibrium(case.rho, case.ux, case.uy)
        r0, u0, v0 = s.moments()
        s.step(50)
        r1, u1, v1 = s.moments()
        m = r0.sum()
        assert abs(r1.sum() - m) < tol * m
        assert abs((r1 * u1).sum() - (r0 * u0).sum()) < tol * m
        assert abs((r1 * v1).sum() - (r0 * v0).sum()) < tol * m
        s.close()


def test_set_state_get_state_round_trip():
    case = _mk("tgv_tau_field")
    o = oracle.Oracle(case)
    f = o.fhat_to_f(o.run(o.init_fhat(), 3))   # a non-equilibrium physical state
    s = dugks.Solver(case, dugks.FP64)
    s.set_state(f)
    assert np.abs(s.get_fhat() - o.f_to_fhat(f)).max() < 1e-15 * np.abs(f).max()
    assert np.abs(s.get_state() - f).max() < 1e-15 * np.abs(f).max()
    # device pointers through torch
    ft = torch.from_numpy(f.copy()).cuda()
    s.set_state(ft)
    out = torch.empty_like(ft)
    s.get_state(out)
    torch.cuda.synchronize()
    assert np.abs(out.cpu().numpy() - f).max() < 1e-15 * np.abs(f).max()
    s.close()


@pytest.mark.parametrize("name,prec", [("tgv32_d2q9", "FP64"), ("tgv32_d2q9", "FP32_DELTA"),
                                       ("cavity_bb_33x30", "FP64"), ("nc8_ds_tanh", "FP64")])
def test_nonfinite_state_is_reported(name, prec):
    # the stage kernels raise the handle's flag when they write a non-finite
    # value; dugks_sync reports it and clears it
    case = _mk(name)
    s = dugks.Solver(case, getattr(dugks, prec), allow_defect=True)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    s.step(2)
    s.sync()   # finite: no report
    f = s.get_state()
    f[0, 3, 3] = np.nan
    s.set_state(f)
    s.step(1)
    with pytest.raises(dugks.DugksError) as e:
        s.sync()
    assert e.value.code == -6
    s.sync()   # the report cleared the flag; no stage ran since
    s.close()


def test_deterministic_replay():
    case = _mk("cavity_bb_33x30")
    outs = []
    for _ in range(2):
        s = dugks.Solver(case, dugks.FP64)
        s.init_equilibrium(case.rho, case.ux, case.uy)
        s.step(10)
        outs.append(s.get_fhat())
        s.close()
    assert np.array_equal(outs[0], outs[1])


# ---------------------------------------------------------------------------
# any-size velocity-set kernels (q split into chunks across workgroups)
# ---------------------------------------------------------------------------
GENERIC_CASES = [("tgv32_d2q9", True), ("couette_ds_d2q9", True), ("tgv_tau_field", True),
                 ("cavity_ds_d2q37_tanh", True), ("nc8_ds_tanh", False), ("nc16_ds_couette", False),
                 ("nc28_cavity_kn1", False)]


@pytest.mark.parametrize("name,force", GENERIC_CASES)
def test_anysize_fp64_one_step_every_element(name, force):
    case = _mk(name)
    say(f"[gpu] any-size fp64 one step {name} Q={case.vs.nq}")
    o, s = _pair(case, 1.0, force_generic=force)
    assert "any-size" in s.describe()
    want = o.step(o.init_fhat())
    s.step(1)
    s.sync()
    got = s.get_fhat()
    err = np.abs(got - want).max() / np.abs(want).max()
    say(f"    max rel err {err:.2e}  ({s.describe()})")
    assert err < 1e-13
    s.close()


@pytest.mark.parametrize("tile", [(16, 16), (18, 14), (14, 18), (20, 12), (12, 20), (8, 8)])
def test_anysize_ring_tile_shapes(tile):
    """Every ring-tile shape the library may pick (and a small one) gives the
    oracle's step on a walled, stretched grid whose sides are not multiples of
    the tile interior."""
    case = _mk("nc8_ds_tanh")
    say(f"[gpu] any-size tile {tile}")
    o, s = _pair(case, 1.0, tile=tile)
    assert f"tile {tile[0]}x{tile[1]}" in s.describe()
    want = o.step(o.init_fhat())
    s.step(1)
    s.sync()
    got = s.get_fhat()
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()
    s.close()


@pytest.mark.parametrize("name,force,steps", [("tgv32_d2q9", True, 100), ("nc8_ds_tanh", False, 40),
                                              ("nc28_cavity_kn1", False, 20)])
def test_anysize_fp64_many_steps(name, force, steps):
    case = _mk(name)
    say(f"[gpu] any-size fp64 {steps} steps {name}")
    o, s = _pair(case, 1.0, force_generic=force)
    fh = o.run(o.init_fhat(), steps)
    ro, uxo, uyo = o.moments(fh)
    s.step(steps)
    s.sync()
    r, ux, uy = s.moments()
    us = max(np.abs(uxo).max(), np.abs(uyo).max())
    e_u = max(np.abs(ux - uxo).max(), np.abs(uy - uyo).max()) / us
    e_rho = np.abs(r - ro).max() / np.abs(ro).max()
    say(f"    rho {e_rho:.2e}  u {e_u:.2e}")
    assert e_rho < 1e-12 and e_u < 1e-12
    s.close()


@pytest.mark.parametrize("name,steps", [("nc16_ds_couette", 100), ("nc28_cavity_kn1", 40)])
def test_anysize_fp32_delta(name, steps):
    case = _mk(name)
    say(f"[gpu] any-size fp32-delta {steps} steps {name}")
    o = oracle.Oracle(case)
    fh = o.run(o.init_fhat(), steps)
    ro, uxo, uyo = o.moments(fh)
    s = dugks.Solver(case, dugks.FP32_DELTA, allow_defect=_allow(case))
    s.init_equilibrium(case.rho, case.ux, case.uy)
    s.step(steps)
    s.sync()
    r, ux, uy = s.moments()
    us = max(np.abs(uxo).max(), np.abs(uyo).max())
    e_u = max(np.abs(ux - uxo).max(), np.abs(uy - uyo).max()) / us
    say(f"    u {e_u:.2e}  rho {np.abs(r - ro).max():.2e}")
    assert e_u < 1e-5
    s.close()


def test_anysize_rejects_bounce_back():
    case = C.cavity_case(16, C.newton_cotes(8, 0.5, renormalize=True), tau=0.2)
    with pytest.raises(dugks.DugksError) as e:
        dugks.Solver(case)
    assert e.value.code == -7


def test_any_size_profiling_times_faces_and_update_without_changing_results():
    # while profiling, the any-size stages launch their four kernels with
    # events between them: the same kernels in the same order on one stream
    case = _mk("nc8_ds_tanh")
    say("[gpu] any-size profiling nc8_ds_tanh FP32-delta")
    runs = []
    for prof in (False, True):
        s = dugks.Solver(case, dugks.FP32_DELTA, allow_defect=True)
        s.init_equilibrium(case.rho, case.ux, case.uy)
        if prof:
            s.prof_begin(64)
        s.step(3)
        if prof:
            f_ms, f_n = s.prof_query(dugks.K_LQ_FACES)
            u_ms, u_n = s.prof_query(dugks.K_LQ_UPDATE)
            a_ms, a_n = s.prof_query(dugks.K_STAGE_A)
            s.prof_end()
            assert (f_n, u_n, a_n) == (6, 6, 0) and f_ms > 0 and u_ms > 0
        runs.append(s.get_fhat())
        s.close()
    assert np.array_equal(runs[0], runs[1])
