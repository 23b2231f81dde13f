"""T2S3 on the GPU: the paper's second-order comparison scheme (Remark I's
T2 step with the full step on the flux, state ftilde = f - (dt/2) Omega) with
the same third-order interface reconstruction (eq. flux_DS), through the C
ABI, against the oracle's independent T2 step.

Both sides start from the seeded macroscopic fields: the library from
dugks_init_equilibrium, the oracle from its own equilibrium (for moment-exact
weights the T2 state of an equilibrium is the equilibrium itself).

FP64: one step on every element to 1e-13 of the scale; 40 steps on density and
velocity to 1e-12 relative.  FP32-delta: velocity within 1e-5 of its scale.
The paper's convergence table (Taylor vortex, dt/tau = 4) has T2S3 rows: the
GPU run is checked against them (golden fixture).
"""
import math
import os
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
from test_gpu_parity import _allow, _mk  # noqa: E402  (seeded cases shared with the T3S3 parity tests)

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_t3s3.txt")

# lattice fast tiles (D2Q9, D2Q37), a tau field, bounce-back walls, diffuse
# walls on a stretched grid, and the any-size kernels (Newton-Cotes 8 x 8)
CASES = ["tgv32_d2q9", "tgv24_d2q37", "tgv_tau_field", "cavity_bb_33x30", "cavity_ds_d2q37_tanh", "nc8_ds_tanh"]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(case, precision=dugks.FP64):
    o = oracle.Oracle(case, literal_taylor=True)
    s = dugks.Solver(case, precision, allow_defect=_allow(case), scheme=dugks.T2S3)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    return o, s, o.equilibrium(case.rho, case.ux, case.uy)


@pytest.mark.parametrize("name", CASES)
def test_t2s3_fp64_one_step_every_element(name):
    case = _mk(name)
    say(f"[gpu] t2s3 fp64 one step {name} {case.grid.nx}x{case.grid.ny} Q={case.vs.nq}")
    o, s, ft0 = _pair(case)
    scale = np.abs(ft0).max()
    assert np.abs(s.get_fhat() - ft0).max() <= 1e-14 * scale
    want = o.t2_step(ft0, case.dt)
    s.step(1)
    s.sync()
    err = np.abs(s.get_fhat() - want).max() / np.abs(want).max()
    say(f"    max rel err {err:.2e}  ({s.describe()})")
    assert err < 1e-13
    s.close()


@pytest.mark.parametrize("name", CASES)
def test_t2s3_fp64_many_steps_macroscopic(name):
    steps = 40
    case = _mk(name)
    say(f"[gpu] t2s3 fp64 {steps} steps {name}")
    o, s, ft = _pair(case)
    for _ in range(steps):
        ft = o.t2_step(ft, case.dt)
    ro, uxo, uyo = o.moments(ft)
    s.step(steps)
    s.sync()
    r, ux, uy = s.moments()
    us = max(np.abs(uxo).max(), np.abs(uyo).max())
    e_rho = np.abs(r - ro).max() / np.abs(ro).max()
    e_u = max(np.abs(ux - uxo).max(), np.abs(uy - uyo).max()) / us
    say(f"    rho {e_rho:.2e}  u {e_u:.2e}")
    assert e_rho < 1e-12 and e_u < 1e-12
    s.close()


@pytest.mark.parametrize("name", ["tgv32_d2q9", "tgv24_d2q37", "nc8_ds_tanh"])
def test_t2s3_fp32_delta_against_fp64_oracle(name):
    steps = 100
    case = _mk(name)
    say(f"[gpu] t2s3 fp32-delta {steps} steps {name}")
    o, s, ft = _pair(case, dugks.FP32_DELTA)
    for _ in range(steps):
        ft = o.t2_step(ft, case.dt)
    ro, uxo, uyo = o.moments(ft)
    s.step(steps)
    s.sync()
    r, ux, uy = s.moments()
    us = max(np.abs(uxo).max(), np.abs(uyo).max())
    e_u = max(np.abs(ux - uxo).max(), np.abs(uy - uyo).max()) / us
    e_rho = np.abs(r - ro).max()
    say(f"    u {e_u:.2e}  rho {e_rho:.2e}")
    assert e_u < 1e-5 and e_rho < 1e-6
    s.close()


def test_t2s3_takes_the_dt_over_tau_guard_and_conserves():
    # the whole T2S3 step is bounded too (cavity: dt/tau = 9 at CFL 1), so it
    # shares the T3S3 guard of 12
    case = _mk("tgv32_d2q9")
    case.tau = np.full_like(case.tau, case.dt / 12.5)
    with pytest.raises(dugks.DugksError) as e:
        dugks.Solver(case, dugks.FP64, scheme=dugks.T2S3)
    assert e.value.code == -2
    case.tau = np.full_like(case.tau, case.dt / 12.0)
    o, s, ft0 = _pair(case)
    want = o.t2_step(ft0, case.dt)
    r0, u0, v0 = s.moments()
    s.step(1)
    assert np.abs(s.get_fhat() - want).max() < 1e-13 * np.abs(want).max()
    s.step(49)
    r1, u1, v1 = s.moments()
    m = r0.sum()
    assert abs(r1.sum() - m) < 1e-13 * m
    assert abs((r1 * u1).sum() - (r0 * u0).sum()) < 1e-13 * m
    assert abs((r1 * v1).sum() - (r0 * v0).sum()) < 1e-13 * m
    s.close()


def test_t2s3_state_round_trip_and_unsupported_calls():
    case = _mk("tgv_tau_field")
    o = oracle.Oracle(case)
    f = o.fhat_to_f(o.run(o.init_fhat(), 3))   # a non-equilibrium physical state
    s = dugks.Solver(case, dugks.FP64, scheme=dugks.T2S3)
    s.set_state(f)
    # the stored variable is ftilde = f + dt/(2 tau) (f - E(f))
    rho, ux, uy = o.moments(f)
    E = o.equilibrium(rho, ux, uy)
    ft = f + case.dt / (2.0 * case.tau)[None] * (f - E)
    assert np.abs(s.get_fhat() - ft).max() < 1e-15 * np.abs(f).max()
    assert np.abs(s.get_state() - f).max() < 1e-15 * np.abs(f).max()
    with pytest.raises(dugks.DugksError) as e:
        s.backward(f, 2, 1, dL_du=np.zeros((2, case.grid.ny, case.grid.nx)))
    assert e.value.code == -7
    s.close()
    with pytest.raises(dugks.DugksError) as e:
        dugks.BatchSolver([_mk("tgv32_d2q9")], dugks.FP64, scheme=dugks.T2S3)
    assert e.value.code == -1


def _table_case(N, dt=1e-5, nu=0.01):
    tau = dt / 4.0
    RT = nu / tau
    g = C.uniform_grid(N, N, 1.0, 1.0)
    A = B = 2 * math.pi
    rho, ux, uy = C.taylor_green_fields(g.xc, g.yc, 0.0, 1.0, A, B, nu, RT)
    return C.Case(f"tv{N}", g, C.d2q9(RT), dt, np.full((N, N), tau), (C.BC_PERIODIC,) * 4,
                  np.zeros((4, 2)), rho, ux, uy, 1.0, int(round(1.0 / dt)),
                  {"u0": 1.0, "A": A, "B": B, "nu": nu})


def test_t2s3_convergence_table_rows():
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    paper = {int(n): float(e) for m, n, e in rows if m == "T2S3"}
    res = {}
    for N in sorted(paper):
        case = _table_case(N)
        s = dugks.Solver(case, dugks.FP64, scheme=dugks.T2S3)
        s.set_state(oracle.chapman_enskog_tgv(case))
        s.step(case.steps)
        s.sync()
        _, ux, uy = s.moments()
        t = case.steps * case.dt
        _, uxa, uya = C.taylor_green_fields(case.grid.xc, case.grid.yc, t, 1.0, 2 * math.pi, 2 * math.pi,
                                            0.01, case.vs.RT)
        res[N] = math.sqrt(((ux - uxa) ** 2 + (uy - uya) ** 2).sum() / (uxa ** 2 + uya ** 2).sum())
        say(f"T2S3 N {N:3d}: E(u) = {res[N]:.3e} (paper {paper[N]:.3e})")
        s.close()
    Ns = sorted(res)
    orders = [math.log(res[a] / res[b]) / math.log(b / a) for a, b in zip(Ns, Ns[1:])]
    say("T2S3 observed orders " + " ".join(f"{o:.2f}" for o in orders))
    # within the band of the paper's errors and second order in between
    for N in Ns:
        assert 0.3 * paper[N] < res[N] < 1.25 * paper[N]
    assert all(1.7 < o < 3.3 for o in orders)
