"""Walled uniform grids large enough that the fast-kind tiles form a rectangle
and the general kernel is launched over the ring of wall tiles around it
(one block per ring tile).  150 x 150 cells leave ragged tiles on both axes
for every tile shape here; the parity bar is the oracle's, element by element
after one step in FP64, then density and velocity after 10 steps, and the
FP32-delta velocity after 10 steps (the wall conditions of the cavity section:
bounce-back and diffuse walls, a moving lid)."""
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


def _case(lattice, wall, seed):
    vs = C.d2q37(1.0 / 3.0) if lattice == "d2q37" else C.d2q9(1.0 / 3.0)
    c = C.cavity_case(150, vs, wall=wall, tau=0.002, lid=0.05)
    z = C.normal(seed, 3 * 150 * 150).reshape(3, 150, 150)
    c.rho = c.rho + 0.003 * z[0]
    c.ux = c.ux + 0.01 * z[1]
    c.uy = c.uy + 0.01 * z[2]
    return c


CASES = [("d2q9", C.BC_BOUNCE_BACK, (32, 8)), ("d2q9", C.BC_DIFFUSE, (32, 8)),
         ("d2q37", C.BC_BOUNCE_BACK, (16, 16)), ("d2q37", C.BC_BOUNCE_BACK, (32, 8)),
         ("d2q37", C.BC_DIFFUSE, (16, 16))]


@pytest.mark.parametrize("lattice,wall,tile", CASES)
def test_wall_ring_matches_the_oracle(lattice, wall, tile):
    case = _case(lattice, wall, 31 + CASES.index((lattice, wall, tile)))
    print(f"[gpu] ring {lattice} wall {wall} 150x150 tile {tile}", file=sys.stderr, flush=True)
    o = oracle.Oracle(case, literal_taylor=True)
    want = o.step(o.init_fhat())
    s = dugks.Solver(case, dugks.FP64, tile=tile)
    s.init_equilibrium(case.rho, case.ux, case.uy)
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
    s.close()
    scale = max(np.abs(uo).max(), np.abs(vo).max())
    assert np.abs(r - ro).max() < 1e-12 * np.abs(ro).max()
    assert max(np.abs(u - uo).max(), np.abs(v - vo).max()) < 1e-12 * scale
    s = dugks.Solver(case, dugks.FP32_DELTA, tile=tile)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    s.step(10)
    _, u32, v32 = s.moments()
    s.close()
    e32 = max(np.abs(u32 - uo).max(), np.abs(v32 - vo).max()) / scale
    print(f"    10 steps: FP32-delta u {e32:.2e} of the velocity scale", file=sys.stderr, flush=True)
    assert e32 < 1e-5
