"""ctypes wrapper of the three-dimensional oracle (dugks_oracle3d.c): one
T3S3 step on a triply periodic box of uniform cells, in plain FP64.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module; the library and
its Python binding never do.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from ctypes import c_double, c_int, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dugks_oracle3d.c")
LIB = os.path.join(HERE, "liboracle3d.so")


def build(force: bool = False) -> None:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", SRC, "-lm", "-o", tmp])
        os.replace(tmp, LIB)


class _O3Case(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int), ("nq", c_int),
                ("dx", c_double), ("dy", c_double), ("dz", c_double),
                ("xi", c_void_p), ("w", c_void_p),
                ("RT", c_double), ("dt", c_double), ("literal_taylor", c_int)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(LIB)
    return _lib


class Oracle3:
    """Oracle of one `cases.Case3`.  Distributions are numpy arrays
    [q][z][y][x], cell fields [z][y][x], velocities u[3][z][y][x]."""

    def __init__(self, case, literal_taylor: bool = True, dt: float | None = None):
        self.case = case
        self.lib = _load()
        nx, ny, nz = case.n
        self.shape = (nz, ny, nx)
        self.nq = case.vs.nq
        self._xi = np.ascontiguousarray(case.vs.xi.reshape(3, -1), dtype=np.float64)
        self._w = np.ascontiguousarray(case.vs.w, dtype=np.float64)
        h = case.h
        self.c = _O3Case(nx, ny, nz, self.nq, h[0], h[1], h[2], self._xi.ctypes.data, self._w.ctypes.data,
                         case.vs.RT, case.dt if dt is None else dt, 1 if literal_taylor else 0)
        self.tau = np.ascontiguousarray(np.broadcast_to(case.tau, self.shape), dtype=np.float64)

    def _f(self, f):
        a = np.ascontiguousarray(f, dtype=np.float64)
        if a.shape != (self.nq,) + self.shape:
            raise ValueError(f"distribution of shape {a.shape}, expected {(self.nq,) + self.shape}")
        return a

    def equilibrium(self, rho, u):
        rho = np.ascontiguousarray(np.broadcast_to(rho, self.shape), dtype=np.float64)
        u = np.ascontiguousarray(np.broadcast_to(u, (3,) + self.shape), dtype=np.float64)
        E = np.empty((self.nq,) + self.shape)
        self.lib.o3_equilibrium(ctypes.byref(self.c), rho.ctypes.data_as(c_void_p), u.ctypes.data_as(c_void_p),
                                E.ctypes.data_as(c_void_p))
        return E

    def moments(self, f):
        f = self._f(f)
        rho = np.empty(self.shape)
        u = np.empty((3,) + self.shape)
        self.lib.o3_cell_moments(ctypes.byref(self.c), f.ctypes.data_as(c_void_p), rho.ctypes.data_as(c_void_p),
                                 u.ctypes.data_as(c_void_p))
        return rho, u

    def f_to_fhat(self, f):
        """fhat = f - dt/4 Omega(f), Omega = (E - f) / tau (the step's state)."""
        rho, u = self.moments(f)
        E = self.equilibrium(rho, u)
        return f - self.c.dt / 4.0 * (E - f) / self.tau

    def fhat_to_f(self, fhat):
        """Inverse of f_to_fhat (the moments of f and fhat agree)."""
        rho, u = self.moments(fhat)
        E = self.equilibrium(rho, u)
        k = self.c.dt / (4.0 * self.tau)
        return (fhat + k * E) / (1.0 + k)

    def init_fhat(self):
        """fhat of the equilibrium at the case's initial rho, u."""
        return self.f_to_fhat(self.equilibrium(self.case.rho, self.case.u))

    def face_values(self, B, h: float):
        """Interface values fbar (eq. interfaceEvof) at the low face of every
        cell along each axis, [3][q][z][y][x]."""
        B = self._f(B)
        out = np.empty((3, self.nq) + self.shape)
        self._check(self.lib.o3_face_values(ctypes.byref(self.c), B.ctypes.data_as(c_void_p), c_double(h),
                                            out.ctypes.data_as(c_void_p)))
        return out

    def flux(self, B, h: float):
        B = self._f(B)
        L = np.empty_like(B)
        self._check(self.lib.o3_flux(ctypes.byref(self.c), self.tau.ctypes.data_as(c_void_p), B.ctypes.data_as(c_void_p),
                                     c_double(h), L.ctypes.data_as(c_void_p)))
        return L

    def step(self, fhat):
        fhat = self._f(fhat)
        out = np.empty_like(fhat)
        self._check(self.lib.o3_t3s3_step(ctypes.byref(self.c), self.tau.ctypes.data_as(c_void_p),
                                          fhat.ctypes.data_as(c_void_p), out.ctypes.data_as(c_void_p)))
        return out

    def run(self, fhat, nsteps: int):
        f = self._f(fhat).copy()
        self._check(self.lib.o3_run(ctypes.byref(self.c), self.tau.ctypes.data_as(c_void_p), f.ctypes.data_as(c_void_p),
                                    c_int(nsteps)))
        return f

    @staticmethod
    def _check(rc):
        if rc != 0:
            raise MemoryError("oracle3d: allocation failed")
