"""Edge cases of the sweep through the C ABI, against the oracle: the
smallest grids the library accepts (3 x 3: every stencil wraps or meets both
walls, and one tile is much larger than the grid), a 3-cell-wide strip, each
kernel family (lattice periodic, lattice walls, any-size), and a zero-step
call, which must leave the state untouched."""
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


def _pert(c, seed, amp=0.01):
    z = C.normal(seed, 3 * c.grid.nx * c.grid.ny).reshape(3, c.grid.ny, c.grid.nx)
    c.rho = c.rho + 0.3 * amp * z[0]
    c.ux = c.ux + amp * z[1]
    c.uy = c.uy + amp * z[2]
    return c


def _mk(name):
    d2q9 = C.d2q9(1.0 / 3.0)
    if name == "tgv3_d2q9":
        c = C.tgv_case(3, d2q9)
        c.tau = np.full_like(c.tau, c.dt / 6.0)   # dt/tau = 6 (the CFL step on 3 cells is long)
        return _pert(c, 1)
    if name == "cavity3_bb_d2q9":
        return _pert(C.cavity_case(3, d2q9, tau=0.05, lid=0.05), 2)
    if name == "cavity3_ds_nc6":
        vs = C.newton_cotes(6, 0.5, renormalize=True)
        return _pert(C.cavity_case(3, vs, wall=C.BC_DIFFUSE, tau=0.3, lid=0.1, cfl=0.25), 3)
    if name == "strip3x40_d2q37":
        c = C.tgv_case(40, C.d2q37(1.0 / 3.0))
        c.grid = C.uniform_grid(3, 40, 2 * np.pi * 3 / 40, 2 * np.pi)
        c.rho, c.ux, c.uy = np.ones((40, 3)), np.zeros((40, 3)), np.zeros((40, 3))
        c.tau = np.full((40, 3), c.tau[0, 0])
        return _pert(c, 21)
    raise KeyError(name)


NAMES = ["tgv3_d2q9", "cavity3_bb_d2q9", "cavity3_ds_nc6", "strip3x40_d2q37"]


@pytest.mark.parametrize("name", NAMES)
def test_smallest_grids_match_the_oracle(name):
    case = _mk(name)
    print(f"[gpu] edge {name} {case.grid.nx}x{case.grid.ny} Q={case.vs.nq}", file=sys.stderr, flush=True)
    o = oracle.Oracle(case, literal_taylor=True)
    fh = o.init_fhat()
    s = dugks.Solver(case, dugks.FP64)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    want = o.step(fh)
    s.step(1)
    s.sync()
    err = np.abs(s.get_fhat() - want).max() / np.abs(want).max()
    print(f"    one step, every element {err:.2e} ({s.describe()})", file=sys.stderr, flush=True)
    assert err < 1e-13
    for _ in range(9):
        want = o.step(want)
    s.step(9)
    ro, uo, vo = o.moments(want)
    r, u, v = s.moments()
    assert np.abs(r - ro).max() < 1e-12 * np.abs(ro).max()
    assert max(np.abs(u - uo).max(), np.abs(v - vo).max()) < 1e-12 * max(np.abs(uo).max(), np.abs(vo).max())
    s.close()
    # FP32-delta on the same grid: velocity within 1e-5 of its scale after 10 steps
    s = dugks.Solver(case, dugks.FP32_DELTA)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    s.step(10)
    _, u32, v32 = s.moments()
    s.close()
    assert max(np.abs(u32 - uo).max(), np.abs(v32 - vo).max()) < 1e-5 * max(np.abs(uo).max(), np.abs(vo).max())


@pytest.mark.parametrize("precision", [dugks.FP64, dugks.FP32_DELTA])
def test_zero_steps_leave_the_state_untouched(precision):
    case = _mk("tgv3_d2q9")
    s = dugks.Solver(case, precision)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    s.step(2)
    before = s.get_fhat()
    s.step(0)
    s.sync()
    assert np.array_equal(before, s.get_fhat())
    s.close()
