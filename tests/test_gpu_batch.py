"""Batched stepping: many uneven instances per launch, replayed from a
captured graph, must give each instance exactly what it gets alone (same
kernels; the small any-size instances here keep their velocity chunks in the
batch) and match the oracle."""
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


def small_batch():
    d2q9 = C.d2q9(1.0 / 3.0)
    out = [C.cavity_case(20, d2q9, tau=0.02, lid=0.05),
           C.tgv_case(24, d2q9),
           C.cavity_case(18, C.newton_cotes(8, 0.5, renormalize=True), wall=C.BC_DIFFUSE,
                         grid=C.tanh_grid(18, 18), tau=0.3, lid=0.1),
           C.couette_case(16, C.newton_cotes(10, 0.5, renormalize=True), tau=0.5, U=0.1, cfl=0.25),
           C.cavity_case(24, C.d2q37(1.0 / 3.0), tau=0.03, lid=0.05),
           C.cavity_case(37, d2q9, tau=0.01, lid=0.05)]
    for k, c in enumerate(out):
        z = C.normal(100 + k, 3 * c.ncell).reshape(3, c.grid.ny, c.grid.nx)
        c.rho = c.rho + 0.005 * z[0]
        c.ux = c.ux + 0.005 * z[1]
        c.uy = c.uy + 0.005 * z[2]
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_instances_and_oracle(precision):
    cases = small_batch()
    say(f"[gpu] batch of {len(cases)} precision={precision}")
    b = dugks.BatchSolver(cases, precision)
    say("   ", b.describe())
    for inst, c in zip(b.instances, cases):
        inst.init_equilibrium(c.rho, c.ux, c.uy)
    b.step(2)
    b.step(3)       # two-step graph, then two-step + one-step graphs
    b.sync()
    for k, (inst, c) in enumerate(zip(b.instances, cases)):
        got = inst.get_fhat()
        s = dugks.Solver(c, precision, allow_defect=abs(c.vs.moment_defect()["sum_w_minus_1"]) > 1e-10)
        s.init_equilibrium(c.rho, c.ux, c.uy)
        s.step(5)
        alone = s.get_fhat()
        s.close()
        assert np.array_equal(got, alone), (k, np.abs(got - alone).max())
        if precision == 0:
            o = oracle.Oracle(c)
            want = o.run(o.init_fhat(), 5)
            err = np.abs(got - want).max() / np.abs(want).max()
            say(f"    instance {k} ({c.name}) rel err vs oracle {err:.2e}")
            assert err < 1e-13
    b.close()


def test_batch_graph_replays_many_times():
    cases = small_batch()[:3]
    b = dugks.BatchSolver(cases, dugks.FP64)
    singles = []
    for inst, c in zip(b.instances, cases):
        inst.init_equilibrium(c.rho, c.ux, c.uy)
        s = dugks.Solver(c, dugks.FP64, allow_defect=abs(c.vs.moment_defect()["sum_w_minus_1"]) > 1e-10)
        s.init_equilibrium(c.rho, c.ux, c.uy)
        singles.append(s)
    for rep in range(4):
        b.step(2)
        torch.cuda.synchronize()
        for s in singles:
            s.step(2)
        for inst, s in zip(b.instances, singles):
            assert np.array_equal(inst.get_fhat(), s.get_fhat()), rep
    for s in singles:
        s.close()
    b.close()


def test_batch_rejects_separately_stepped_instance():
    cases = small_batch()[:2]
    b = dugks.BatchSolver(cases, dugks.FP64)
    for inst, c in zip(b.instances, cases):
        inst.init_equilibrium(c.rho, c.ux, c.uy)
    b.instances[0].step(1)
    with pytest.raises(dugks.DugksError):
        b.step(1)
    b.close()


def test_autotuner_picks_a_candidate(tmp_path, monkeypatch):
    monkeypatch.setenv("DUGKS_TUNE_CACHE", str(tmp_path / "tune.json"))
    c = C.tgv_case(128)
    t = tune.best_tile(c, dugks.FP32_DELTA)
    assert t in tune.CANDIDATES_256
    assert tune.best_tile(c, dugks.FP32_DELTA) == t      # cached
    assert (tmp_path / "tune.json").exists()
