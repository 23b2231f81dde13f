"""The paper's doubly periodic shear-layer workload (k = 80, delta = 0.05,
nu = 1e-4, Re = 10^4, 128 x 128 cells, D2Q9), through the C ABI.

* Parity: the oracle's steps from the same seeded fields (FP64 every element
  after one step, density and velocity after 20; FP32-delta velocity).
* The run to t = 1 (the paper shows t = 0.8 and 1.0): finite, mass and
  momentum conserved, and the flow's symmetry kept; FP32-delta on the same
  flow (its gap to FP64 grows with the step count here, see the test).  The initial state is
  invariant under T: (x, y) -> (x + 1/2, 1 - y) with (u_x, u_y) -> (u_x, -u_y),
  and so is the scheme on an even grid with a velocity set closed under
  xi_y -> -xi_y; only rounding (a different order of the q sums) breaks it.
* Refinement: 128^2, 256^2 and 512^2 to t = 1, compared at the 128^2 cell
  centres through exact Fourier interpolation of the finer fields.
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


def _solver(case, precision, scheme=dugks.T3S3):
    s = dugks.Solver(case, precision, scheme=scheme)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    return s


def _sym_err(ux, uy):
    n = ux.shape[1]
    uT = np.roll(ux[::-1, :], -n // 2, axis=1)
    vT = -np.roll(uy[::-1, :], -n // 2, axis=1)
    return max(np.abs(ux - uT).max(), np.abs(uy - vT).max())


def _at_coarse_centres(a, nc):
    """Values of the periodic cell-centred field a (nf x nf) at the centres of
    an nc x nc grid on the same square, by Fourier interpolation."""
    nf = a.shape[0]
    r = nf // nc
    s = (r - 1) / 2.0                       # coarse centre I sits at fine index r I + s
    k = np.fft.fftfreq(nf) * nf
    ph = np.exp(2j * math.pi * k * s / nf)
    A = np.fft.fft2(a) * ph[:, None] * ph[None, :]
    return np.real(np.fft.ifft2(A))[::r, ::r]


def test_shear_fp64_parity_with_oracle():
    case = C.shear_layer_case(128)
    say(f"[gpu] shear 128^2 fp64 parity, dt {case.dt:.3e} dt/tau 10")
    o = oracle.Oracle(case, literal_taylor=True)
    s = _solver(case, dugks.FP64)
    fh = o.init_fhat()
    want = o.step(fh)
    s.step(1)
    s.sync()
    err = np.abs(s.get_fhat() - want).max() / np.abs(want).max()
    say(f"    one step, every element: {err:.2e}")
    assert err < 1e-13
    fh = want
    for _ in range(19):
        fh = o.step(fh)
    s.step(19)
    ro, uo, vo = o.moments(fh)
    r, u, v = s.moments()
    e_rho = np.abs(r - ro).max() / np.abs(ro).max()
    e_u = max(np.abs(u - uo).max(), np.abs(v - vo).max())
    say(f"    20 steps: rho {e_rho:.2e}  u {e_u:.2e} (U = 1)")
    assert e_rho < 1e-12 and e_u < 1e-12
    s.close()


def test_shear_fp32_delta_against_oracle():
    case = C.shear_layer_case(128)
    say("[gpu] shear 128^2 fp32-delta 100 steps vs oracle")
    o = oracle.Oracle(case, literal_taylor=True)
    fh = o.run(o.init_fhat(), 100)
    ro, uo, vo = o.moments(fh)
    s = _solver(case, dugks.FP32_DELTA)
    s.step(100)
    r, u, v = s.moments()
    e_u = max(np.abs(u - uo).max(), np.abs(v - vo).max())
    say(f"    u {e_u:.2e} (U = 1)  rho {np.abs(r - ro).max():.2e}")
    assert e_u < 1e-5
    s.close()


def _run_to_end(n, precision=dugks.FP64, scheme=dugks.T3S3):
    case = C.shear_layer_case(n)
    s = _solver(case, precision, scheme)
    r0, u0, v0 = s.moments()
    s.step(case.steps)
    s.sync()
    r, u, v = s.moments()
    s.close()
    return case, (r0, u0, v0), (r, u, v)


def test_shear_layer_to_t1_conserves_and_keeps_the_symmetry():
    say("[gpu] shear 128^2 to t = 1, FP64 and FP32-delta")
    case, (r0, u0, v0), (r, u, v) = _run_to_end(128)
    say(f"    {case.steps} steps; initial symmetry error {_sym_err(u0, v0):.1e}")
    assert np.isfinite(u).all() and np.isfinite(v).all()
    m = r0.sum()
    e_m = abs(r.sum() - m) / m
    e_px = abs((r * u).sum() - (r0 * u0).sum()) / m
    e_py = abs((r * v).sum() - (r0 * v0).sum()) / m
    sym = _sym_err(u, v)
    ke0 = (r0 * (u0 ** 2 + v0 ** 2)).sum()
    ke = (r * (u ** 2 + v ** 2)).sum()
    say(f"    mass {e_m:.1e}  momentum {e_px:.1e} {e_py:.1e}  symmetry {sym:.1e}  KE ratio {ke / ke0:.5f}")
    assert e_m < 1e-12 and e_px < 1e-12 and e_py < 1e-12
    assert sym < 1e-9
    assert 0.9 < ke / ke0 < 1.0            # viscous decay only
    # FP32-delta: per-step rounding of the stored state puts noise of about
    # 1e-7 U into the conserved moments.  At Re = 10^4 with this small step,
    # viscosity damps grid-scale noise by only nu (pi/dx)^2 dt = 1e-3 per step,
    # so it random-walks, and the shear instability amplifies what survives
    # (the FP64 symmetry error above grows 10^4-fold by t = 1).  Measured
    # gap: 2.4e-7 after 1 step, 6.4e-6 after 100, 2.5e-5 after 1000, 2.2e-3
    # at t = 1.  The bar holds the FP32 run on the same flow to 0.5%.
    _, _, (r32, u32, v32) = _run_to_end(128, dugks.FP32_DELTA)
    d32 = max(np.abs(u32 - u).max(), np.abs(v32 - v).max())
    say(f"    FP32-delta against FP64 at t = 1: max |du| {d32:.2e} (U = 1)")
    assert d32 < 5e-3


def test_shear_layer_refinement():
    say("[gpu] shear refinement 128^2 / 256^2 / 512^2 to t = 1, FP64")
    sol = {}
    for n in (128, 256, 512):
        case, _, (r, u, v) = _run_to_end(n)
        assert np.isfinite(u).all()
        sol[n] = (u, v)
        say(f"    {n}^2: {case.steps} steps, CFL {case.dt * case.vs.cmax / case.grid.dmin:.3f}, "
            f"max|u_y| {np.abs(v).max():.4f}")
    at = {n: tuple(_at_coarse_centres(a, 128) for a in sol[n]) for n in sol}

    def dist(a, b):
        return math.sqrt(sum(((x - y) ** 2).sum() for x, y in zip(a, b)) /
                         sum((y ** 2).sum() for y in b))
    d1 = dist(at[128], at[256])
    d2 = dist(at[256], at[512])
    order = math.log(d1 / d2, 2)
    say(f"    |u128 - u256| {d1:.3e}  |u256 - u512| {d2:.3e}  observed order {order:.2f}")
    assert d2 < d1
    assert order > 1.5
    # the paper's comparison on this flow: the second-order time step on the
    # same meshes, both measured against the 512^2 T3S3 field
    for n in (128, 256):
        _, _, (_, u2, v2) = _run_to_end(n, dugks.FP64, dugks.T2S3)
        e2 = dist(tuple(_at_coarse_centres(a, 128) for a in (u2, v2)), at[512])
        e3 = dist(at[n], at[512])
        say(f"    {n}^2 against 512^2 T3S3: T3S3 {e3:.3e}  T2S3 {e2:.3e}")
