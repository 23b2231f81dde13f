"""GPU parity of the three-dimensional sweep (include/dugks3d.h, through the C
ABI) against the three-dimensional oracle, on the same seeded inputs.

FP64: every (q, cell) of fhat after one and after three steps within 1e-13 of
its scale, on boxes with ragged tiles (the kernels tile 16 x 8 x 2 cells), a
varying relaxation field, both velocity sets and both coefficients of the
quadratic term.  FP32-delta storage: velocity within 1e-5 of its scale.
Larger boxes, where the oracle would be slow: conservation, and the ABC
flow's viscous decay."""
import math
import sys

import numpy as np
import pytest

from oracle.oracle3d import Oracle3
from paper_1709_05458_amd import cases as C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():   # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1709_05458_amd import dugks  # noqa: E402

RT = 1.0 / 3.0


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _vs(lattice):
    if lattice.endswith("_reversed"):
        vs = getattr(C, lattice[:-9])(RT)
        return C.VelocitySet(vs.name + "r", vs.xi[:, ::-1].copy(), vs.w[::-1].copy(), RT)
    return getattr(C, lattice)(RT)


def _case(shape, lattice, seed=3, tau_field=True, cfl=0.5):
    vs = _vs(lattice)
    c = C.abc_case(0, vs, nu=0.02, ma=0.1, cfl=cfl, noise=0.3, seed=seed, shape=shape)
    tau0 = max(float(c.tau.reshape(-1)[0]), c.dt / 4.0)   # dt / tau <= 4 on coarse boxes
    # a field within +-20% (uniform), so that no cell passes the dt/tau bound
    u = C.uniform01(seed + 100, c.tau.size).reshape(c.tau.shape)
    c.tau = tau0 * (0.8 + 0.4 * u) if tau_field else np.full(c.tau.shape, tau0)
    return c


def _f0(o, case, seed):
    """Equilibrium of the case's fields plus a seeded non-equilibrium part."""
    E = o.equilibrium(case.rho, case.u)
    z = C.normal(seed, E.size).reshape(E.shape)
    return E * (1.0 + 0.02 * z)


PARITY = [((12, 10, 7), "d3q19", 1.0), ((12, 10, 7), "d3q27", 1.0), ((9, 11, 5), "d3q19", 0.5),
          ((8, 8, 4), "d3q27", 0.5), ((3, 4, 3), "d3q19", 1.0), ((16, 9, 9), "d3q27", 1.0),
          # the velocities in another order: the kernels with run-time window tables
          ((12, 10, 7), "d3q19_reversed", 1.0), ((9, 11, 5), "d3q27_reversed", 0.5)]


@pytest.mark.parametrize("shape,lattice,kq", PARITY, ids=[f"{s[0]}x{s[1]}x{s[2]}_{l}_k{k}" for s, l, k in PARITY])
def test_fp64_every_element_vs_oracle(shape, lattice, kq):
    say(f"3d fp64 parity {shape} {lattice} kq={kq}")
    case = _case(shape, lattice)
    o = Oracle3(case, literal_taylor=(kq == 1.0))
    f0 = _f0(o, case, 41)
    s = dugks.Solver3D(case, precision=dugks.FP64, taylor_quad=kq)
    s.set_state(f0)
    fh0 = o.f_to_fhat(f0)
    scale = np.abs(fh0).max()
    assert np.abs(s.get_fhat() - fh0).max() < 1e-14 * scale
    ref = fh0
    for nsteps in (1, 2):
        s.step(nsteps)
        ref = o.run(ref, nsteps)
        err = np.abs(s.get_fhat() - ref).max() / scale
        say(f"  after {nsteps} more: max rel {err:.3e}")
        assert err < 1e-13, err
    rho, u = s.moments()
    r_ref, u_ref = o.moments(ref)
    assert np.abs(rho - r_ref).max() < 1e-13
    assert np.abs(u - u_ref).max() < 1e-12 * np.abs(u_ref).max()
    # the physical distribution (inverse of the fhat map)
    assert np.abs(s.get_state() - o.fhat_to_f(ref)).max() < 1e-13 * scale
    s.close()


@pytest.mark.parametrize("lattice", ["d3q19", "d3q27"])
def test_fp32_delta_velocity_vs_oracle(lattice):
    say(f"3d fp32-delta parity {lattice}")
    case = _case((12, 10, 7), lattice, seed=5)
    o = Oracle3(case)
    f0 = _f0(o, case, 43)
    s = dugks.Solver3D(case, precision=dugks.FP32_DELTA)
    s.set_state(f0)
    s.step(5)
    ref = o.run(o.f_to_fhat(f0), 5)
    rho, u = s.moments()
    r_ref, u_ref = o.moments(ref)
    du = np.abs(u - u_ref).max() / np.abs(u_ref).max()
    say(f"  u max rel {du:.3e}, rho max {np.abs(rho - r_ref).max():.3e}")
    assert du < 1e-5, du
    assert np.abs(rho - r_ref).max() < 1e-6
    s.close()


def test_init_equilibrium_and_moments_round_trip():
    case = _case((10, 9, 8), "d3q19", tau_field=False)
    s = dugks.Solver3D(case, precision=dugks.FP64)
    s.init_equilibrium(case.rho, case.u)
    rho, u = s.moments()
    assert np.abs(rho - case.rho).max() < 1e-14
    assert np.abs(u - case.u).max() < 1e-14
    o = Oracle3(case)
    E = o.equilibrium(case.rho, case.u)
    assert np.abs(s.get_state() - E).max() < 1e-15
    # device pointers
    rt = torch.tensor(case.rho.reshape(-1), dtype=torch.float64, device="cuda")
    ut = torch.tensor(case.u.reshape(-1), dtype=torch.float64, device="cuda")
    s.init_equilibrium(rt, ut)
    ft = torch.empty(case.vs.nq * case.ncell, dtype=torch.float64, device="cuda")
    s.get_state(ft)
    torch.cuda.synchronize()
    assert np.abs(ft.cpu().numpy().reshape(E.shape) - E).max() < 1e-15
    s.close()


@pytest.mark.parametrize("precision", [dugks.FP64, dugks.FP32_DELTA])
def test_conservation_on_a_larger_box(precision):
    say(f"3d conservation 40x36x28 precision={precision}")
    case = _case((40, 36, 28), "d3q27", seed=9)
    s = dugks.Solver3D(case, precision=precision)
    s.init_equilibrium(case.rho, case.u)
    r0, u0 = s.moments()
    m0, p0 = r0.sum(), (r0 * u0).sum(axis=(1, 2, 3))
    s.step(50)
    r1, u1 = s.moments()
    assert np.isfinite(r1).all()
    tol = 1e-13 if precision == dugks.FP64 else 1e-8
    assert abs(r1.sum() - m0) < tol * m0, (r1.sum() - m0) / m0
    assert np.abs((r1 * u1).sum(axis=(1, 2, 3)) - p0).max() < tol * m0
    s.close()


@pytest.mark.parametrize("precision", [dugks.FP64, dugks.FP32_DELTA])
def test_abc_flow_viscous_decay_at_32_cubed(precision):
    """The ABC flow decays as exp(-nu t), nu = tau RT; with the Taylor factor
    1/2 within 1% at 16 cells per period on the oracle, here at 32."""
    say(f"3d ABC decay 32^3 precision={precision}")
    vs = C.d3q19(RT)
    nu = 0.05
    case = C.abc_case(32, vs, nu=nu, ma=0.05, cfl=0.5)
    s = dugks.Solver3D(case, precision=precision, taylor_quad=0.5)
    s.init_equilibrium(case.rho, case.u)
    shape = case.u

    def amp():
        _, u = s.moments()
        return float((u * shape).sum() / (shape * shape).sum())

    s.step(20)
    a1 = amp()
    s.step(60)
    a2 = amp()
    rate = -math.log(a2 / a1) / (60 * case.dt)
    say(f"  rate / nu - 1 = {rate / nu - 1:.3e}")
    assert abs(rate / nu - 1.0) < 0.01
    s.close()


def test_64_cubed_one_step_every_element_vs_oracle():
    """A larger box (1024 tiles) in the bench's kernels: FP64 every element, FP32-delta velocity."""
    say("3d 64^3 D3Q19 one step vs oracle")
    case = C.abc_case(64, C.d3q19(RT), nu=0.01, ma=0.05, cfl=0.5, noise=0.3, seed=21)
    o = Oracle3(case)
    f0 = _f0(o, case, 47)
    ref = o.step(o.f_to_fhat(f0))
    s = dugks.Solver3D(case, precision=dugks.FP64)
    s.set_state(f0)
    s.step(1)
    err = np.abs(s.get_fhat() - ref).max() / np.abs(ref).max()
    say(f"  fp64 max rel {err:.3e}")
    assert err < 1e-13, err
    s.close()
    s = dugks.Solver3D(case, precision=dugks.FP32_DELTA)
    s.set_state(f0)
    s.step(1)
    _, u = s.moments()
    _, u_ref = o.moments(ref)
    du = np.abs(u - u_ref).max() / np.abs(u_ref).max()
    say(f"  fp32-delta u max rel {du:.3e}")
    assert du < 1e-5, du
    s.close()


def test_bench_configuration_128_cubed_properties():
    """The bench's workload and launch configuration (128^3, D3Q19, FP32-delta,
    the lattice kernels), where the oracle would take minutes per step:
    conservation and agreement with an FP64 run from the same start; and the
    ABC flow's viscous decay rate, measured after the initial layer of the
    equilibrium start (t > 10 tau)."""
    say("3d 128^3 D3Q19 bench configuration")
    nu = 0.05
    case = C.abc_case(128, C.d3q19(RT), nu=nu, ma=0.05, cfl=0.5)
    tau = nu / RT
    n1 = int(math.ceil(10 * tau / case.dt))
    runs = {}
    for prec, kq in ((dugks.FP32_DELTA, 1.0), (dugks.FP64, 1.0), (dugks.FP32_DELTA, 0.5)):
        s = dugks.Solver3D(case, precision=prec, taylor_quad=kq)
        s.init_equilibrium(case.rho, case.u)
        r0, u0 = s.moments()
        s.step(n1)
        _, ua = s.moments()
        s.step(100)
        r1, u1 = s.moments()
        runs[(prec, kq)] = (r0, u0, ua, r1, u1)
        s.close()
    r0, u0, ua, r1, u1 = runs[(dugks.FP32_DELTA, 1.0)]
    m0 = r0.sum()
    assert abs(r1.sum() - m0) < 1e-9 * m0
    assert np.abs((r1 * u1).sum(axis=(1, 2, 3)) - (r0 * u0).sum(axis=(1, 2, 3))).max() < 1e-9 * m0
    u64 = runs[(dugks.FP64, 1.0)][4]
    gap = np.abs(u1 - u64).max() / np.abs(u64).max()
    say(f"  fp32 vs fp64 u max rel {gap:.3e}")
    assert gap < 1e-5
    shape = case.u
    amp = lambda u: float((u * shape).sum() / (shape * shape).sum())
    rates = {}
    for kq in (1.0, 0.5):
        _, _, ua, _, u1 = runs[(dugks.FP32_DELTA, kq)]
        rates[kq] = -math.log(amp(u1) / amp(ua)) / (100 * case.dt) / nu - 1.0
        say(f"  kappa {kq}: decay rate / nu - 1 = {rates[kq]:.3e}")
    assert abs(rates[0.5]) < 0.01   # measured -0.77%
    assert abs(rates[1.0]) < 0.02   # measured -0.80%


def test_box_beyond_2_31_elements_matches_a_thin_box():
    """Maximum-size case: 256 x 256 x 1800 cells, D3Q19 FP32-delta, so that
    velocity x cell offsets pass 2^31 (2.24e9 per array).  Every cell's
    arithmetic depends only on its neighbourhood and the run's constants, so
    a state uniform along z evolves, bit for bit, as the same state on a box
    of 4 cells along z: the moments of every z plane of the large box must
    equal those of the thin box exactly."""
    props = torch.cuda.get_device_properties(0)
    if props.total_memory < 96 * 2 ** 30:   # pragma: no cover
        pytest.skip("needs about 70 GB of device memory")
    vs = C.d3q19(RT)
    nx = ny = 256
    # a power-of-two cell width: L / n is exactly h on every axis of both boxes
    h = 1.0 / 32
    x = (np.arange(nx) + 0.5) * h * (2.0 * math.pi / (nx * h))
    X, Y = np.meshgrid(x, x)   # (ny, nx), phases over one period
    ux = 0.05 * np.sin(X) * np.cos(Y) + 0.005 * C.normal(61, nx * ny).reshape(ny, nx)
    uy = -0.05 * np.cos(X) * np.sin(Y) + 0.005 * C.normal(62, nx * ny).reshape(ny, nx)
    uz = 0.02 * np.sin(X + Y)
    rho = 1.0 + 0.01 * C.normal(63, nx * ny).reshape(ny, nx)
    dt = 0.5 * h / vs.cmax
    tau0 = 0.02

    def run(nz):
        shape = (nz, ny, nx)
        r = np.ascontiguousarray(np.broadcast_to(rho, shape))
        u = np.ascontiguousarray(np.broadcast_to(np.stack([ux, uy, uz])[:, None], (3,) + shape))
        case = C.Case3(f"z-uniform {nz}", (nx, ny, nz), (nx * h, ny * h, nz * h), vs, dt,
                       np.array(tau0), r, u)
        say(f"3d z-uniform box {nx}x{ny}x{nz} D3Q19 fp32-delta, {vs.nq * nx * ny * nz} elements per array")
        s = dugks.Solver3D(case, precision=dugks.FP32_DELTA)
        s.init_equilibrium(r, u)
        del r, u
        s.step(3)
        out = s.moments()
        s.close()
        return out

    rs, us = run(4)
    assert np.ptp(rs, axis=0).max() == 0.0 and np.ptp(us, axis=1).max() == 0.0
    assert np.abs(us[0, 0] - ux).max() > 1e-6   # three steps changed the state
    rb, ub = run(1800)
    assert vs.nq * rb.size > 2 ** 31
    assert np.array_equal(rb, np.broadcast_to(rs[:1], rb.shape))
    del rb
    for d in range(3):
        assert np.array_equal(ub[d], np.broadcast_to(us[d, :1], ub[d].shape)), d
