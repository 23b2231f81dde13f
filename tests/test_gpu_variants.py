"""Variants of the method on the GPU (variant.hip through the C ABI) against
the oracle's independent implementations, FP64:

* the member a of the time-discretization family (paper section "Time
  discretization"; reading: A = a/2, K from A = (3K-2)/(6K-3));
* the cell-average reading with the two-point Gauss face rule;
* the S2 reconstruction of the original DUGKS and, with the Remark-I step,
  the paper's T2S2 comparison scheme.

Every element after one step within 1e-13 of the field scale; rho and u after
20 steps within 1e-12 relative.  The paper's convergence table is run for the
variants in tests/test_gpu_table1.py.
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


def _tgv(nx, ny, vs, seed):
    c = C.tgv_case(nx, vs)
    c.grid = C.uniform_grid(nx, ny, 2 * math.pi, 2 * math.pi * ny / nx)
    X, Y = np.meshgrid(c.grid.xc, c.grid.yc)
    z = C.normal(seed, 3 * nx * ny).reshape(3, ny, nx)
    u0 = c.meta["u0"]
    c.rho = 1.0 + 0.01 * np.cos(X) * np.sin(Y) + 1e-3 * z[0]
    c.ux = -u0 * np.cos(X) * np.sin(Y) + 1e-3 * u0 * z[1]
    c.uy = u0 * np.sin(X) * np.cos(Y) + 1e-3 * u0 * z[2]
    c.tau = np.full((ny, nx), c.tau[0, 0])
    return c


# (name, velocity set, family_a (0 = T2 step), reconstruction, kappa, tau field)
VARIANTS = [
    ("a045_point_k1", "d2q9", 0.45, dugks.RECON_POINT, 1.0, False),
    ("a05_point_k1_d2q37", "d2q37", 0.5, dugks.RECON_POINT, 1.0, False),
    ("a13_avg_khalf", "d2q9", 1.0 / 3.0, dugks.RECON_CELL_AVERAGE, 0.5, False),
    ("a04_avg_k1_taufield", "d2q9", 0.4, dugks.RECON_CELL_AVERAGE, 1.0, True),
    ("a13_s2", "d2q9", 1.0 / 3.0, dugks.RECON_S2, 1.0, False),
    ("t2s2", "d2q9", 0.0, dugks.RECON_S2, 1.0, False),
    ("t2_avg_khalf", "d2q9", 0.0, dugks.RECON_CELL_AVERAGE, 0.5, False),
    ("a045_avg_nc8", "nc8", 0.45, dugks.RECON_CELL_AVERAGE, 0.5, False),
]


def _vs(name):
    if name == "d2q9":
        return C.d2q9(1.0 / 3.0)
    if name == "d2q37":
        return C.d2q37(1.0 / 3.0)
    return C.newton_cotes(8, 1.0 / 3.0, renormalize=True)


def _pair(name, vsname, a, recon, kappa, tau_field):
    case = _tgv(24, 20, _vs(vsname), 17)
    if tau_field:
        case.tau = C.perturbed_tau(case.tau[0, 0], case.tau.shape, 0.05, 19)
    t2 = a == 0.0
    allow = abs(case.vs.moment_defect()["sum_w_minus_1"]) > 1e-10
    s = dugks.Solver(case, dugks.FP64, taylor_quad=kappa, scheme=dugks.T2S3 if t2 else dugks.T3S3,
                     family_a=0.0 if t2 else a, reconstruction=recon, tau_field=tau_field, allow_defect=allow)
    o = oracle.Oracle(case, literal_taylor=(kappa == 1.0), recon=recon, a_param=a if not t2 else 1.0 / 3.0)
    f0 = o.equilibrium(case.rho, case.ux, case.uy)
    s.set_state(f0)
    if t2:
        x0 = o.f_to_ftilde(f0, case.dt)
        step = lambda x: o.t2_step(x, case.dt)
    else:
        x0 = o.f_to_fhat_a(f0)
        step = o.step_a
    return case, s, o, x0, step


@pytest.mark.parametrize("v", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_variant_matches_the_oracle(v):
    name = v[0]
    say(f"variant {name}")
    case, s, o, x0, step = _pair(*v)
    assert "variant" in s.describe()
    # the stored state of the library equals the oracle's state variable
    got0 = s.get_fhat()
    assert np.abs(got0 - x0).max() <= 1e-14 * np.abs(x0).max()
    # one step, every element
    s.step(1)
    ref1 = step(x0)
    got1 = s.get_fhat()
    e1 = np.abs(got1 - ref1).max() / np.abs(ref1).max()
    # 20 steps: rho and u
    x = ref1
    for _ in range(19):
        x = step(x)
    s.step(19)
    s.sync()
    r, ux, uy = s.moments()
    ro, uxo, uyo = o.moments(x)
    er = np.abs(r - ro).max() / np.abs(ro).max()
    eu = max(np.abs(ux - uxo).max(), np.abs(uy - uyo).max()) / max(np.abs(uxo).max(), np.abs(uyo).max())
    say(f"  one step {e1:.2e}; 20 steps rho {er:.2e} u {eu:.2e}")
    assert e1 <= 1e-13 and er <= 1e-12 and eu <= 1e-12
    s.close()


def test_variants_refuse_what_they_do_not_run():
    case = _tgv(16, 16, C.d2q9(1.0 / 3.0), 3)
    for kw in ({"precision": dugks.FP32_DELTA, "family_a": 0.45},
               {"precision": dugks.FP64, "reconstruction": dugks.RECON_S2, "case": "cavity"}):
        c = C.cavity_case(16, C.d2q9(1.0 / 3.0), re=100.0) if kw.pop("case", None) else case
        with pytest.raises(dugks.DugksError) as e:
            dugks.Solver(c, **kw)
        assert e.value.code == -7
    s = dugks.Solver(case, dugks.FP64, family_a=0.45)
    s.init_equilibrium(case.rho, case.ux, case.uy)
    with pytest.raises(dugks.DugksError) as e:
        s.backward(s.get_state(), 2, 1, None, np.zeros((2, 16, 16)))
    assert e.value.code == -7
    s.close()
