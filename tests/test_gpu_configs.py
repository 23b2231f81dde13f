"""The largest velocity set and the uneven batch of the measured workloads,
against the oracle:

* Newton-Cotes 101 x 101 velocities (the rarefied cavity's set) on a small
  tanh-stretched cavity with diffuse walls at Kn = 1: FP64 every element
  after one step, FP32-delta u after a few steps;
* a batch whose instances include Newton-Cotes sets of 33^2 and more and
  Kn = 1e-3 (dt/tau near 8), each FP32-delta instance against the FP64
  oracle, not only against its single-instance twin.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1709_05458_amd import cases as C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():   # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1709_05458_amd import dugks, tune  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _nc101_cavity():
    vs = C.newton_cotes(101, 0.5)
    c = C.cavity_case(12, vs, wall=C.BC_DIFFUSE, grid=C.tanh_grid(12, 12), tau=C.kn_to_tau(1.0, 0.5),
                      lid=0.146, cfl=0.25)
    z = C.normal(303, 3 * c.ncell).reshape(3, 12, 12)
    c.rho = c.rho + 0.01 * z[0]
    c.ux = c.ux + 0.01 * z[1]
    c.uy = c.uy + 0.01 * z[2]
    return c


def test_newton_cotes_101_fp64_every_element():
    case = _nc101_cavity()
    assert case.vs.nq == 10201
    o = oracle.Oracle(case)
    f0 = o.equilibrium(case.rho, case.ux, case.uy)
    s = dugks.Solver(case, dugks.FP64, allow_defect=True)
    s.set_state(f0)
    say(f"NC 101^2 FP64: {s.describe()}")
    s.step(1)
    got = s.get_fhat()
    ref = o.step(o.f_to_fhat(f0))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  one step, every element: {err:.2e}")
    assert err <= 1e-13
    s.close()


def test_newton_cotes_101_fp32_delta_velocity():
    case = _nc101_cavity()
    o = oracle.Oracle(case)
    f0 = o.equilibrium(case.rho, case.ux, case.uy)
    s = dugks.Solver(case, dugks.FP32_DELTA, allow_defect=True)
    s.set_state(f0)
    n = 5
    s.step(n)
    s.sync()
    _, ux, uy = s.moments()
    _, uxo, uyo = o.moments(o.run(o.f_to_fhat(f0), n))
    U = case.meta["U"]
    err = max(np.abs(ux - uxo).max(), np.abs(uy - uyo).max()) / U
    say(f"NC 101^2 FP32-delta, {n} steps: max |u - u_oracle| / U = {err:.2e}")
    assert err <= 1e-5
    s.close()


def test_batch_with_large_sets_and_small_knudsen_against_the_oracle():
    # instances drawn like the 64-cavity workload but small: sides 16..22,
    # Newton-Cotes sets 33^2..36^2, Kn in [1e-3, 10^-2.5] (dt = min(CFL dx / C, 8 tau))
    cases = C.batch_cases(6, seed=2, nmin=16, nmax=22, ncmin=33, ncmax=36, kn_lo=-3.0, kn_hi=-2.5)
    assert any(c.vs.nq >= 33 * 33 for c in cases)
    assert max(c.dt / c.tau.min() for c in cases) > 7.0
    for k, c in enumerate(cases):
        z = C.normal(500 + k, 3 * c.ncell).reshape(3, c.grid.ny, c.grid.nx)
        c.rho = c.rho + 0.005 * z[0]
        c.ux = c.ux + 0.002 * z[1]
        c.uy = c.uy + 0.002 * z[2]
    tiles = tune.tiles_for(cases, dugks.FP32_DELTA)
    b = dugks.BatchSolver(cases, dugks.FP32_DELTA, tiles=tiles)
    for inst, c in zip(b.instances, cases):
        inst.init_equilibrium(c.rho, c.ux, c.uy)
    n = 10
    b.step(n)
    b.sync()
    worst = 0.0
    for k, (inst, c) in enumerate(zip(b.instances, cases)):
        _, ux, uy = inst.moments()
        o = oracle.Oracle(c)
        _, uxo, uyo = o.moments(o.run(o.init_fhat(), n))
        U = c.meta["U"]
        err = max(np.abs(ux - uxo).max(), np.abs(uy - uyo).max()) / U
        say(f"  instance {k} {c.name} (dt/tau {c.dt / c.tau.min():.2f}): |u - u_oracle| / U = {err:.2e}")
        worst = max(worst, err)
    assert worst <= 1e-5
    b.close()
