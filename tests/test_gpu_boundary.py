"""Boundary features of the C ABI on the GPU: graph replay of single-handle
steps (bit for bit the direct launches), the relaxation time from Kn and a
reference length (paper, "Numerical tests": lambda = tau sqrt(pi RT / 2)),
and the caller's device allocator (here torch's caching allocator)."""
import math
import sys

import numpy as np
import pytest

from paper_1709_05458_amd import cases as C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():   # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1709_05458_amd import dugks  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = {
    "tgv48_d2q37_fp32": (lambda: C.tgv_case(48, C.d2q37(1.0 / 3.0)), dugks.FP32_DELTA),
    "tgv40_d2q9_fp64": (lambda: C.tgv_case(40, C.d2q9(1.0 / 3.0)), dugks.FP64),
    "cavity50_d2q9_fp32": (lambda: C.cavity_case(50, C.d2q9(1.0 / 3.0), re=100.0), dugks.FP32_DELTA),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_graph_replay_equals_direct_launches(name):
    mk, prec = CASES[name]
    case = mk()
    # direct: kernel timing on keeps every call on direct launches
    a = dugks.Solver(case, prec)
    a.init_equilibrium(case.rho, case.ux, case.uy)
    a.prof_begin(64)
    a.step(1)
    a.step(5)
    a.step(2)
    a.prof_end()
    # graph: the first call launches directly, later calls replay the
    # captured step of each parity
    b = dugks.Solver(case, prec)
    b.init_equilibrium(case.rho, case.ux, case.uy)
    b.step(1)
    b.step(5)
    b.step(2)
    a.sync()
    b.sync()
    fa, fb = a.get_fhat(), b.get_fhat()
    say(f"{name}: graph vs direct bitwise {np.array_equal(fa, fb)}")
    assert np.array_equal(fa, fb)
    a.close()
    b.close()


def test_relaxation_time_from_the_knudsen_number():
    vs = C.newton_cotes(8, 0.5, renormalize=True)
    kn, L = 0.3, 1.0
    tau = kn * L / math.sqrt(math.pi * 0.5 / 2.0)
    case = C.cavity_case(20, vs, wall=C.BC_DIFFUSE, tau=tau, lid=0.1, cfl=0.25)
    a = dugks.Solver(case, dugks.FP64)
    b = dugks.Solver(case, dugks.FP64, kn=(kn, L))
    for s in (a, b):
        s.init_equilibrium(case.rho, case.ux, case.uy)
        s.step(5)
    fa, fb = a.get_fhat(), b.get_fhat()
    assert np.abs(fa - fb).max() <= 1e-15 * np.abs(fa).max()
    a.close()
    b.close()


def test_caller_device_allocator():
    calls = {"alloc": 0, "free": 0}

    def alloc(nbytes, ctx):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes))

    def free(ptr, ctx):
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(ptr)

    cb = (dugks.ALLOC_FN(alloc), dugks.FREE_FN(free))
    case = C.tgv_case(32, C.d2q9(1.0 / 3.0))
    a = dugks.Solver(case, dugks.FP64)
    b = dugks.Solver(case, dugks.FP64, allocator=cb)
    for s in (a, b):
        s.init_equilibrium(case.rho, case.ux, case.uy)
        s.step(4)
    assert np.array_equal(a.get_fhat(), b.get_fhat())
    # the adjoint workspace comes from the same allocator
    f0 = torch.from_numpy(b.get_state()).cuda()
    du = torch.zeros((2, 32, 32), dtype=torch.float64, device="cuda")
    n_before = calls["alloc"]
    b.backward(f0, 3, 2, None, du)
    assert calls["alloc"] == n_before + 1
    a.close()
    b.close()
    say(f"allocator calls: {calls}")
    assert calls["alloc"] > 5 and calls["free"] == calls["alloc"]
