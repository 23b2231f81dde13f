"""Oracle of the T3S3-DUGKS step: a plain, slow FP64 C implementation
(dugks_oracle.c) written from the paper, plus a ctypes wrapper and the few
numpy helpers the pin tests need.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the library and
its Python binding never do.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from ctypes import POINTER, c_double, c_int

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dugks_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_CS = os.path.join(HERE, "liboracle_cs.so")


def build(force: bool = False) -> None:
    """Compile the oracle twice: real (double) and complex-step (double
    complex); and the three-dimensional oracle (oracle3d.py)."""
    base = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp", SRC, "-lm"]
    for out, extra in ((LIB, []), (LIB_CS, ["-DORACLE_COMPLEX"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            tmp = out + ".tmp"
            subprocess.check_call(base[:1] + extra + base[1:] + ["-o", tmp])
            os.replace(tmp, out)
    from . import oracle3d
    oracle3d.build(force)


class _OcCase(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nq", c_int),
                ("xf", POINTER(c_double)), ("yf", POINTER(c_double)),
                ("xi", POINTER(c_double)), ("w", POINTER(c_double)),
                ("opp", POINTER(c_int)),
                ("RT", c_double), ("dt", c_double),
                ("bc", c_int * 4), ("uw", (c_double * 2) * 4),
                ("literal_ftilde", c_int), ("literal_fbp", c_int),
                ("literal_taylor", c_int), ("recon", c_int), ("a_param", c_double)]

# interface reconstructions (dugks_oracle.c, "Variants"): point values with
# the midpoint face rule (the paper's choice), cell averages with the two-point
# Gauss rule, and the original DUGKS linear reconstruction S2
RECON_POINT, RECON_CELL_AVERAGE, RECON_S2 = 0, 1, 2


_libs = {}


def _lib(cs: bool):
    key = bool(cs)
    if key not in _libs:
        build()
        lib = ctypes.CDLL(LIB_CS if cs else LIB)
        _libs[key] = lib
    return _libs[key]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """Wrapper around one `cases.Case` (grid, velocity set, tau, walls).

    Arrays are numpy, layout [q][y][x] for distributions and [y][x] for cell
    fields.  With ``complex_step=True`` every array is complex128 and the C
    code runs in complex arithmetic (for complex-step derivatives)."""

    def __init__(self, case, complex_step: bool = False, literal_ftilde: bool = False,
                 literal_fbp: bool = False, literal_taylor: bool = True,
                 dt: float | None = None, recon: int = RECON_POINT, a_param: float = 1.0 / 3.0):
        self.case = case
        self.cs = complex_step
        self.dtype = np.complex128 if complex_step else np.float64
        self.lib = _lib(complex_step)
        self.prefix = "oc_cs_" if complex_step else "oc_"
        g, vs = case.grid, case.vs
        self._keep = [np.ascontiguousarray(g.xf, dtype=np.float64),
                      np.ascontiguousarray(g.yf, dtype=np.float64),
                      np.ascontiguousarray(vs.xi.reshape(-1), dtype=np.float64),
                      np.ascontiguousarray(vs.w, dtype=np.float64),
                      np.ascontiguousarray(vs.opp, dtype=np.int32)]
        c = _OcCase()
        c.nx, c.ny, c.nq = g.nx, g.ny, vs.nq
        c.xf = self._keep[0].ctypes.data_as(POINTER(c_double))
        c.yf = self._keep[1].ctypes.data_as(POINTER(c_double))
        c.xi = self._keep[2].ctypes.data_as(POINTER(c_double))
        c.w = self._keep[3].ctypes.data_as(POINTER(c_double))
        c.opp = self._keep[4].ctypes.data_as(POINTER(c_int))
        c.RT = vs.RT
        c.dt = case.dt if dt is None else dt
        for k in range(4):
            c.bc[k] = int(case.bc[k])
            c.uw[k][0] = float(case.u_wall[k][0])
            c.uw[k][1] = float(case.u_wall[k][1])
        c.literal_ftilde = int(literal_ftilde)
        c.literal_fbp = int(literal_fbp)
        c.literal_taylor = int(literal_taylor)
        c.recon = int(recon)
        c.a_param = float(a_param)
        self.c = c
        self.shape_q = (vs.nq, g.ny, g.nx)
        self.shape_c = (g.ny, g.nx)
        self.tau = self._arr(case.tau, self.shape_c)

    def _fn(self, name):
        return getattr(self.lib, self.prefix + name)

    def _arr(self, a, shape):
        a = np.ascontiguousarray(np.asarray(a, dtype=self.dtype).reshape(shape))
        return a

    def set_tau(self, tau):
        self.tau = self._arr(tau, self.shape_c)

    # -- pieces ------------------------------------------------------------
    def equilibrium(self, rho, ux, uy):
        rho, ux, uy = (self._arr(a, self.shape_c) for a in (rho, ux, uy))
        f = np.empty(self.shape_q, dtype=self.dtype)
        self._fn("equilibrium")(ctypes.byref(self.c), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(f))
        return f

    def moments(self, f):
        f = self._arr(f, self.shape_q)
        out = [np.empty(self.shape_c, dtype=self.dtype) for _ in range(3)]
        self._fn("cell_moments")(ctypes.byref(self.c), _ptr(f), *map(_ptr, out))
        return tuple(out)

    def f_to_fhat(self, f):
        f = self._arr(f, self.shape_q)
        out = np.empty_like(f)
        self._check(self._fn("f_to_fhat")(ctypes.byref(self.c), _ptr(self.tau), _ptr(f), _ptr(out)))
        return out

    def fhat_to_f(self, fhat):
        fhat = self._arr(fhat, self.shape_q)
        out = np.empty_like(fhat)
        self._check(self._fn("fhat_to_f")(ctypes.byref(self.c), _ptr(self.tau), _ptr(fhat), _ptr(out)))
        return out

    def face_values(self, B, rho_cell, h):
        B = self._arr(B, self.shape_q)
        rho_cell = self._arr(rho_cell, self.shape_c)
        nq, ny, nx = self.shape_q
        fx = np.zeros((nq, ny, nx + 1), dtype=self.dtype)
        fy = np.zeros((nq, ny + 1, nx), dtype=self.dtype)
        self._fn("face_values")(ctypes.byref(self.c), _ptr(B), _ptr(rho_cell), c_double(h),
                                _ptr(fx), _ptr(fy))
        return fx, fy

    def face_point_values(self, B, rho_cell, h):
        """Interface values at the face quadrature points of the variant
        readings: fx [q][point][y][x-face], fy [q][point][y-face][x]."""
        B = self._arr(B, self.shape_q)
        rho_cell = self._arr(rho_cell, self.shape_c)
        nq, ny, nx = self.shape_q
        npt = 2 if self.c.recon == RECON_CELL_AVERAGE else 1
        fx = np.zeros((nq, npt, ny, nx + 1), dtype=self.dtype)
        fy = np.zeros((nq, npt, ny + 1, nx), dtype=self.dtype)
        self._fn("face_point_values")(ctypes.byref(self.c), _ptr(B), _ptr(rho_cell), c_double(h),
                                      _ptr(fx), _ptr(fy))
        return fx, fy

    def flux(self, B, rho_cell, h):
        B = self._arr(B, self.shape_q)
        rho_cell = self._arr(rho_cell, self.shape_c)
        L = np.empty(self.shape_q, dtype=self.dtype)
        self._check(self._fn("flux")(ctypes.byref(self.c), _ptr(self.tau), _ptr(B),
                                     _ptr(rho_cell), c_double(h), _ptr(L)))
        return L

    def step(self, fhat):
        fhat = self._arr(fhat, self.shape_q)
        out = np.empty_like(fhat)
        self._check(self._fn("t3s3_step")(ctypes.byref(self.c), _ptr(self.tau), _ptr(fhat), _ptr(out)))
        return out

    def stage_a(self, fhat):
        fhat = self._arr(fhat, self.shape_q)
        out = np.empty_like(fhat)
        self._check(self._fn("t3s3_stage_a")(ctypes.byref(self.c), _ptr(self.tau), _ptr(fhat), _ptr(out)))
        return out

    def run(self, fhat, nsteps: int):
        fhat = self._arr(fhat, self.shape_q).copy()
        self._check(self._fn("t3s3_run")(ctypes.byref(self.c), _ptr(self.tau), _ptr(fhat), c_int(nsteps)))
        return fhat

    # -- the time-discretization family (member a_param) ----------------------
    def step_a(self, fhat):
        fhat = self._arr(fhat, self.shape_q)
        out = np.empty_like(fhat)
        self._check(self._fn("t3a_step")(ctypes.byref(self.c), _ptr(self.tau), _ptr(fhat), _ptr(out)))
        return out

    def run_a(self, fhat, nsteps: int):
        fhat = self._arr(fhat, self.shape_q).copy()
        self._check(self._fn("t3a_run")(ctypes.byref(self.c), _ptr(self.tau), _ptr(fhat), c_int(nsteps)))
        return fhat

    def f_to_fhat_a(self, f):
        f = self._arr(f, self.shape_q)
        out = np.empty_like(f)
        self._check(self._fn("f_to_fhat_a")(ctypes.byref(self.c), _ptr(self.tau), _ptr(f), _ptr(out)))
        return out

    def fhat_to_f_a(self, fhat):
        fhat = self._arr(fhat, self.shape_q)
        out = np.empty_like(fhat)
        self._check(self._fn("fhat_to_f_a")(ctypes.byref(self.c), _ptr(self.tau), _ptr(fhat), _ptr(out)))
        return out

    def f_to_ftilde(self, f, delta: float):
        f = self._arr(f, self.shape_q)
        out = np.empty_like(f)
        self._check(self._fn("f_to_ftilde")(ctypes.byref(self.c), _ptr(self.tau), c_double(delta),
                                            _ptr(f), _ptr(out)))
        return out

    def t2_run(self, ft, delta: float, nsteps: int):
        for _ in range(nsteps):
            ft = self.t2_step(ft, delta)
        return ft

    def t2_step(self, ft, delta: float):
        ft = self._arr(ft, self.shape_q)
        out = np.empty_like(ft)
        self._check(self._fn("t2_step")(ctypes.byref(self.c), _ptr(self.tau), c_double(delta),
                                        _ptr(ft), _ptr(out)))
        return out

    def num_threads(self) -> int:
        f = self._fn("num_threads")
        f.restype = c_int
        return int(f())

    # -- convenience ---------------------------------------------------------
    def init_fhat(self, rho=None, ux=None, uy=None):
        """fhat at t = 0 from an equilibrium initial state f = E(rho, u)."""
        case = self.case
        rho = case.rho if rho is None else rho
        ux = case.ux if ux is None else ux
        uy = case.uy if uy is None else uy
        return self.f_to_fhat(self.equilibrium(rho, ux, uy))

    @staticmethod
    def _check(rc):
        if rc == -2:
            raise ValueError("the S2 reconstruction of the oracle takes periodic grids only")
        if rc != 0:
            raise MemoryError("oracle allocation failed")


# ---------------------------------------------------------------------------
# numpy helpers used by the pin tests (test infrastructure as well)
# ---------------------------------------------------------------------------
def chapman_enskog_tgv(case, t: float = 0.0, cell_average: bool = False):
    """Initial distribution of the Taylor-Green case by the Navier-Stokes
    Chapman-Enskog form f = f^eq - tau (d_t f^eq + xi . grad f^eq) (paper,
    Taylor vortex flow section), with rho, u and their space/time derivatives
    taken analytically from the Taylor-Green solution.  With cell_average
    (uniform grids) every Fourier mode of the fields is replaced by its
    average over the cell (to second order in the amplitude, the cell
    average of f)."""
    g, vs = case.grid, case.vs
    u0, A, B, nu = (case.meta[k] for k in ("u0", "A", "B", "nu"))
    RT, rho0 = vs.RT, case.rho0
    X, Y = np.meshgrid(g.xc, g.yc)
    al = A * A + B * B
    d = np.exp(-nu * al * t)
    if cell_average:
        hx, hy = 0.5 * (g.xf[1] - g.xf[0]), 0.5 * (g.yf[1] - g.yf[0])
        s1 = np.sinc(A * hx / np.pi) * np.sinc(B * hy / np.pi)   # modes of A x and B y
        sx2, sy2 = np.sinc(2 * A * hx / np.pi), np.sinc(2 * B * hy / np.pi)
    else:
        s1 = sx2 = sy2 = 1.0
    ux = -(u0 / A) * np.cos(A * X) * np.sin(B * Y) * d * s1
    uy = (u0 / B) * np.sin(A * X) * np.cos(B * Y) * d * s1
    p = -(u0 ** 2 / 4) * (np.cos(2 * A * X) / A ** 2 * sx2 + np.cos(2 * B * Y) / B ** 2 * sy2) * d * d
    rho = rho0 + p / RT
    # derivatives
    ux_x = u0 * np.sin(A * X) * np.sin(B * Y) * d * s1
    ux_y = -(u0 * B / A) * np.cos(A * X) * np.cos(B * Y) * d * s1
    uy_x = (u0 * A / B) * np.cos(A * X) * np.cos(B * Y) * d * s1
    uy_y = -u0 * np.sin(A * X) * np.sin(B * Y) * d * s1
    ux_t = -nu * al * ux
    uy_t = -nu * al * uy
    p_x = (u0 ** 2 / 2) * np.sin(2 * A * X) / A * d * d * sx2
    p_y = (u0 ** 2 / 2) * np.sin(2 * B * Y) / B * d * d * sy2
    p_t = -2 * nu * al * p
    r_x, r_y, r_t = p_x / RT, p_y / RT, p_t / RT
    nq = vs.nq
    f = np.empty((nq,) + X.shape)
    for q in range(nq):
        ex, ey, w = vs.xi[0, q], vs.xi[1, q], vs.w[q]
        eu = ex * ux + ey * uy
        uu = ux * ux + uy * uy
        poly = 1 + eu / RT + eu * eu / (2 * RT * RT) - uu / (2 * RT)
        E = w * rho * poly
        dE_drho = w * poly
        dE_dux = w * rho * (ex / RT + eu * ex / RT ** 2 - ux / RT)
        dE_duy = w * rho * (ey / RT + eu * ey / RT ** 2 - uy / RT)

        def D(rd, uxd, uyd):
            return dE_drho * rd + dE_dux * uxd + dE_duy * uyd
        dt_E = D(r_t, ux_t, uy_t)
        dx_E = D(r_x, ux_x, uy_x)
        dy_E = D(r_y, ux_y, uy_y)
        f[q] = E - case.tau * (dt_E + ex * dx_E + ey * dy_E)
    return f
