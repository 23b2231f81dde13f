"""Python binding of libdugks.so (argument marshalling only).

Every step of the sweep runs in the HIP kernels of the library; this module
only turns numpy arrays / torch tensors into pointers and checks status codes.
If the library is not built, importing it raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdugks.so")

FP64, FP32_DELTA = 0, 1
T3S3, T2S3 = 0, 1   # time integrators (dugks_scheme)
RECON_POINT, RECON_CELL_AVERAGE, RECON_S2 = 0, 1, 2   # interface reconstructions (dugks_reconstruction)
# device allocator callbacks of dugks_desc: void *(size_t bytes, void *ctx), void (void *ptr, void *ctx)
ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)
MEM_HOST, MEM_DEVICE = 0, 1
ALLOW_MOMENT_DEFECT = 1
FORCE_GENERIC = 2
K_STAGE_A, K_STAGE_C, K_AUX, K_LQ_FACES, K_LQ_UPDATE, K_ADJ_STEP = 0, 1, 2, 3, 4, 5

STATUS = {0: "DUGKS_OK", -1: "DUGKS_EINVAL", -2: "DUGKS_EUNSTABLE", -3: "DUGKS_EMOMENT",
          -4: "DUGKS_ENOMEM", -5: "DUGKS_EDEVICE", -6: "DUGKS_ENONFINITE", -7: "DUGKS_ENOTSUP"}


class DugksError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str):
        super().__init__(f"{what}: {STATUS.get(code, code)} ({detail})")
        self.code = code


class DugksDesc(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int),
                ("xf", POINTER(c_double)), ("yf", POINTER(c_double)),
                ("nq", c_int),
                ("xi", POINTER(c_double)), ("w", POINTER(c_double)),
                ("RT", c_double), ("dt", c_double),
                ("tau", POINTER(c_double)), ("tau0", c_double),
                ("bc", c_int * 4), ("u_wall", (c_double * 2) * 4),
                ("precision", c_int), ("rho0", c_double), ("taylor_quad", c_double),
                ("stream", c_void_p), ("flags", c_int),
                ("tile_x", c_int), ("tile_y", c_int),
                ("scheme", c_int),
                ("kn", c_double), ("l_ref", c_double),
                ("family_a", c_double), ("reconstruction", c_int),
                ("dev_alloc", c_void_p), ("dev_free", c_void_p), ("alloc_ctx", c_void_p)]


class Dugks3dDesc(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int),
                ("lx", c_double), ("ly", c_double), ("lz", c_double),
                ("nq", c_int),
                ("xi", POINTER(c_double)), ("w", POINTER(c_double)),
                ("RT", c_double), ("dt", c_double),
                ("tau", POINTER(c_double)), ("tau0", c_double),
                ("precision", c_int), ("rho0", c_double), ("taylor_quad", c_double),
                ("stream", c_void_p)]


_lib = None


def lib():
    """Load libdugks.so; raise if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, ip, dp = c_void_p, c_int, POINTER(c_double)
        sig = {
            "dugks_create": ([POINTER(DugksDesc), POINTER(c_void_p)], ip),
            "dugks_destroy": ([vp], ip),
            "dugks_set_state": ([vp, vp, ip], ip),
            "dugks_init_equilibrium": ([vp, vp, vp, vp, ip], ip),
            "dugks_step": ([vp, ip], ip),
            "dugks_moments": ([vp, vp, vp, vp, ip], ip),
            "dugks_get_state": ([vp, vp, ip], ip),
            "dugks_get_fhat": ([vp, vp, ip], ip),
            "dugks_set_tau": ([vp, vp, ip], ip),
            "dugks_sync": ([vp], ip),
            "dugks_backward": ([vp, vp, ip, ip, vp, vp, vp, vp, ip], ip),
            "dugks_backward_noalloc": ([vp, vp, ip, ip, vp, vp, vp, vp], ip),
            "dugks_prof_begin": ([vp, ip], ip),
            "dugks_prof_query": ([vp, ip, dp, POINTER(c_int)], ip),
            "dugks_prof_end": ([vp], ip),
            "dugks_describe": ([vp, c_char_p, ip], ip),
            "dugks_create_batch": ([ip, POINTER(DugksDesc), POINTER(c_void_p)], ip),
            "dugks_batch_size": ([vp, POINTER(c_int)], ip),
            "dugks_batch_instance": ([vp, ip, POINTER(c_void_p)], ip),
            "dugks3d_create": ([POINTER(Dugks3dDesc), POINTER(c_void_p)], ip),
            "dugks3d_destroy": ([vp], ip),
            "dugks3d_set_state": ([vp, vp, ip], ip),
            "dugks3d_init_equilibrium": ([vp, vp, vp, ip], ip),
            "dugks3d_step": ([vp, ip], ip),
            "dugks3d_step_timed": ([vp, ip, dp, dp], ip),
            "dugks3d_moments": ([vp, vp, vp, ip], ip),
            "dugks3d_get_fhat": ([vp, vp, ip], ip),
            "dugks3d_get_state": ([vp, vp, ip], ip),
            "dugks_strerror": ([ip], c_char_p),
            "dugks_last_error_message": ([], c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(rc: int, what: str):
    if rc != 0:
        msg = lib().dugks_last_error_message().decode()
        raise DugksError(rc, what, msg)


def _dptr(a):
    return a.ctypes.data_as(POINTER(c_double))


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr_mem(x, dtype=np.float64):
    """(pointer, mem kind, keep-alive) of a numpy array or torch tensor."""
    if _is_torch(x):
        import torch
        if x.dtype != torch.float64 or not x.is_contiguous():
            raise TypeError("torch tensors passed to the library must be contiguous float64")
        return c_void_p(x.data_ptr()), (MEM_DEVICE if x.is_cuda else MEM_HOST), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return c_void_p(a.ctypes.data), MEM_HOST, a


def _default_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def make_desc(case, precision=FP64, taylor_quad=1.0, stream=None, tile=None, allow_defect=False,
              tau=None, force_generic=False, d=None, scheme=T3S3, tau_field=False, family_a=0.0,
              reconstruction=RECON_POINT, kn=None, allocator=None):
    """Fill a DugksDesc from a cases.Case; returns (desc, arrays to keep alive).
    kn = (Kn, L_ref) leaves tau to the library (tau0 = Kn L_ref / sqrt(pi RT / 2));
    allocator = (dev_alloc, dev_free) as ALLOC_FN / FREE_FN callbacks."""
    g, vs = case.grid, case.vs
    keep = [np.ascontiguousarray(g.xf, dtype=np.float64),
            np.ascontiguousarray(g.yf, dtype=np.float64),
            np.ascontiguousarray(vs.xi.reshape(-1), dtype=np.float64),
            np.ascontiguousarray(vs.w, dtype=np.float64)]
    d = DugksDesc() if d is None else d
    d.nx, d.ny, d.nq = g.nx, g.ny, vs.nq
    d.xf, d.yf = _dptr(keep[0]), _dptr(keep[1])
    d.xi, d.w = _dptr(keep[2]), _dptr(keep[3])
    d.RT, d.dt = vs.RT, case.dt
    tau = case.tau if tau is None else tau
    tau = np.asarray(tau, dtype=np.float64)
    if kn is not None:
        d.tau = POINTER(c_double)()
        d.tau0 = 0.0
        d.kn, d.l_ref = float(kn[0]), float(kn[1])
    elif not tau_field and (tau.ndim == 0 or np.ptp(tau) == 0.0):
        d.tau = POINTER(c_double)()
        d.tau0 = float(tau.reshape(-1)[0])
    else:
        t = np.ascontiguousarray(np.broadcast_to(tau, (g.ny, g.nx)).reshape(-1))
        keep.append(t)
        d.tau = _dptr(t)
        d.tau0 = float(t.mean())
    for k in range(4):
        d.bc[k] = int(case.bc[k])
        d.u_wall[k][0] = float(case.u_wall[k][0])
        d.u_wall[k][1] = float(case.u_wall[k][1])
    d.precision = precision
    d.rho0 = float(case.rho0)
    d.taylor_quad = taylor_quad
    stream = _default_stream() if stream is None else stream
    d.stream = c_void_p(stream) if stream else None
    d.flags = (ALLOW_MOMENT_DEFECT if allow_defect else 0) | (FORCE_GENERIC if force_generic else 0)
    if tile:
        d.tile_x, d.tile_y = tile
    d.scheme = scheme
    d.family_a = float(family_a)
    d.reconstruction = int(reconstruction)
    if allocator is not None:
        keep.extend(allocator)
        d.dev_alloc = ctypes.cast(allocator[0], c_void_p)
        d.dev_free = ctypes.cast(allocator[1], c_void_p)
    return d, keep


class Solver:
    """One DUGKS solver instance (a dugks_t handle); scheme T3S3 (default) or T2S3."""

    def __init__(self, case, precision: int = FP64, taylor_quad: float = 1.0, stream=None,
                 tile=None, allow_defect: bool = False, tau=None, force_generic: bool = False,
                 tau_field: bool = False, scheme: int = T3S3, family_a: float = 0.0,
                 reconstruction: int = RECON_POINT, kn=None, allocator=None, _borrowed=None):
        g, vs = case.grid, case.vs
        self.case = case
        self.nx, self.ny, self.nq = g.nx, g.ny, vs.nq
        self.ncell = g.nx * g.ny
        self.precision = precision
        self._owned = _borrowed is None
        if _borrowed is not None:
            self.h = _borrowed
            return
        d, self._keep = make_desc(case, precision, taylor_quad, stream, tile, allow_defect, tau, force_generic,
                                  scheme=scheme, tau_field=tau_field, family_a=family_a,
                                  reconstruction=reconstruction, kn=kn, allocator=allocator)
        self.tau_field = bool(d.tau)
        self.desc = d
        h = c_void_p()
        check(lib().dugks_create(byref(d), byref(h)), "dugks_create")
        self.h = h

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) and getattr(self, "_owned", True):
            lib().dugks_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(256)
        check(lib().dugks_describe(self.h, buf, 256), "dugks_describe")
        return buf.value.decode()

    # -- state ---------------------------------------------------------------
    def set_state(self, f):
        p, mem, keep = _ptr_mem(f)
        check(lib().dugks_set_state(self.h, p, mem), "dugks_set_state")

    def init_equilibrium(self, rho, ux, uy):
        ps = [_ptr_mem(a) for a in (rho, ux, uy)]
        mems = {m for _, m, _ in ps}
        if len(mems) != 1:
            raise ValueError("rho, ux, uy must all live in the same memory")
        check(lib().dugks_init_equilibrium(self.h, ps[0][0], ps[1][0], ps[2][0], mems.pop()),
              "dugks_init_equilibrium")

    def step(self, n: int = 1):
        check(lib().dugks_step(self.h, int(n)), "dugks_step")

    def sync(self):
        check(lib().dugks_sync(self.h), "dugks_sync")

    def run_until_steady(self, tol: float = 1e-6, every: int = 1000, max_steps: int = 1_000_000):
        """Step until the paper's steady-state criterion holds (cavity section):
        sqrt(sum |u^(n+every) - u^(n)|^2) / sqrt(sum |u^(n+every)|^2) <= tol,
        checked every `every` steps.  Returns (steps taken, last residual); the
        residual is None if fewer than two checks ran.  Raises DugksError on a
        non-finite state."""
        _, ux, uy = self.moments()
        done, res = 0, None
        while done < max_steps:
            n = min(every, max_steps - done)
            self.step(n)
            done += n
            self.sync()
            _, vx, vy = self.moments()
            den = float(np.sqrt((vx * vx + vy * vy).sum()))
            res = float(np.sqrt(((vx - ux) ** 2 + (vy - uy) ** 2).sum())) / den if den > 0 else 0.0
            ux, uy = vx, vy
            if n == every and res <= tol:
                break
        return done, res

    def set_tau(self, tau):
        p, mem, keep = _ptr_mem(tau)
        check(lib().dugks_set_tau(self.h, p, mem), "dugks_set_tau")

    def moments(self, out=None):
        """(rho, ux, uy) as numpy (ny, nx) arrays, or into given device tensors."""
        if out is not None:
            ps = [_ptr_mem(a) for a in out]
            check(lib().dugks_moments(self.h, ps[0][0], ps[1][0], ps[2][0], ps[0][1]), "dugks_moments")
            return out
        r = np.empty(self.ncell)
        u = np.empty(self.ncell)
        v = np.empty(self.ncell)
        check(lib().dugks_moments(self.h, c_void_p(r.ctypes.data), c_void_p(u.ctypes.data),
                                  c_void_p(v.ctypes.data), MEM_HOST), "dugks_moments")
        s = (self.ny, self.nx)
        return r.reshape(s), u.reshape(s), v.reshape(s)

    def _dist(self, fn, out):
        if out is not None:
            p, mem, keep = _ptr_mem(out)
            check(fn(self.h, p, mem), fn.__name__)
            return out
        f = np.empty(self.nq * self.ncell)
        check(fn(self.h, c_void_p(f.ctypes.data), MEM_HOST), fn.__name__)
        return f.reshape(self.nq, self.ny, self.nx)

    def get_state(self, out=None):
        return self._dist(lib().dugks_get_state, out)

    def get_fhat(self, out=None):
        return self._dist(lib().dugks_get_fhat, out)

    # -- adjoint -------------------------------------------------------------
    def backward(self, f0, nsteps: int, ckpt_every: int = 25, dL_drho=None, dL_du=None,
                 want_tau: bool = True):
        """Gradients (dL/df0 [q][y][x], dL/dtau [y][x] or None) of
        L = sum dL_drho * rho(T) + dL_du . u(T) after nsteps steps from the
        physical state f0 (dugks_backward).  Torch device tensors in, torch
        device tensors out; otherwise numpy."""
        if dL_du is None:
            raise ValueError("dL_du is required (zeros for a density-only loss)")
        if _is_torch(f0) and f0.is_cuda:
            import torch
            gf = torch.empty(self.nq, self.ny, self.nx, dtype=torch.float64, device=f0.device)
            gt = torch.empty(self.ny, self.nx, dtype=torch.float64, device=f0.device) if want_tau else None
        else:
            gf = np.empty((self.nq, self.ny, self.nx))
            gt = np.empty((self.ny, self.nx)) if want_tau else None
        pf, mem, k0 = _ptr_mem(f0)
        pu, mu, k1 = _ptr_mem(dL_du)
        pr, mr, k2 = _ptr_mem(dL_drho) if dL_drho is not None else (None, mem, None)
        pg, mg, k3 = _ptr_mem(gf)
        pt, mt, k4 = _ptr_mem(gt) if gt is not None else (None, mem, None)
        if len({mem, mu, mr, mg, mt}) != 1:
            raise ValueError("all arrays of backward must live in the same memory")
        check(lib().dugks_backward(self.h, pf, int(nsteps), int(ckpt_every), pr, pu, pg, pt, mem),
              "dugks_backward")
        return gf, gt

    def backward_noalloc(self, f0, nsteps: int, ckpt_every: int, dL_du, dL_df0, dL_drho=None, dL_dtau=None):
        """dugks_backward_noalloc: the same gradients into caller-owned torch
        device tensors (dL_df0 [q][y][x], dL_dtau [y][x] or None), with the
        workspace in the library's fixed device scratch."""
        for a in (f0, dL_du, dL_df0, dL_drho, dL_dtau):
            if a is not None and not (_is_torch(a) and a.is_cuda):
                raise ValueError("backward_noalloc takes torch device tensors only")
        ptr = lambda a: None if a is None else _ptr_mem(a)[0]
        check(lib().dugks_backward_noalloc(self.h, ptr(f0), int(nsteps), int(ckpt_every), ptr(dL_drho),
                                           ptr(dL_du), ptr(dL_df0), ptr(dL_dtau)),
              "dugks_backward_noalloc")

    # -- timing --------------------------------------------------------------
    def prof_begin(self, max_launches: int):
        check(lib().dugks_prof_begin(self.h, int(max_launches)), "dugks_prof_begin")

    def prof_query(self, kernel: int):
        ms = c_double()
        cnt = c_int()
        check(lib().dugks_prof_query(self.h, int(kernel), byref(ms), byref(cnt)), "dugks_prof_query")
        return ms.value, cnt.value

    def prof_end(self):
        check(lib().dugks_prof_end(self.h), "dugks_prof_end")


def _run_function():
    import torch

    class DugksRun(torch.autograd.Function):
        """(rho(T), u(T)) after `nsteps` steps from the physical initial state
        f0 [q][y][x] with the relaxation-time field tau [y][x]; the backward
        pass is the library's discrete adjoint (dugks_backward), with a
        checkpoint every `ckpt_every` steps."""

        @staticmethod
        def forward(ctx, f0, tau, solver, nsteps, ckpt_every):
            f0 = f0.detach().contiguous()
            if tau is not None:
                tau = tau.detach().contiguous()
                solver.set_tau(tau)
            solver.set_state(f0)
            solver.step(nsteps)
            rho = torch.empty(solver.ny, solver.nx, dtype=torch.float64, device=f0.device)
            u = torch.empty(2, solver.ny, solver.nx, dtype=torch.float64, device=f0.device)
            solver.moments(out=(rho, u[0], u[1]))
            ctx.save_for_backward(f0, tau if tau is not None else torch.empty(0))
            ctx.solver, ctx.nsteps, ctx.ckpt, ctx.has_tau = solver, nsteps, ckpt_every, tau is not None
            return rho, u

        @staticmethod
        def backward(ctx, g_rho, g_u):
            f0, tau = ctx.saved_tensors
            s = ctx.solver
            if ctx.has_tau:
                s.set_tau(tau)
            if g_u is None:
                g_u = torch.zeros(2, s.ny, s.nx, dtype=torch.float64, device=f0.device)
            gr = None if g_rho is None else g_rho.contiguous()
            gf, gt = s.backward(f0, ctx.nsteps, ctx.ckpt, gr, g_u.contiguous(),
                                want_tau=ctx.has_tau and ctx.needs_input_grad[1])
            return gf, gt, None, None, None

    return DugksRun


_RUN = None


def run(f0, tau, solver: Solver, nsteps: int, ckpt_every: int = 25):
    """Differentiable (rho(T), u(T)) of a torch float64 f0 [q][y][x] and tau
    [y][x] (or None): see DugksRun."""
    global _RUN
    if _RUN is None:
        _RUN = _run_function()
    return _RUN.apply(f0, tau, solver, int(nsteps), int(ckpt_every))


class BatchSolver:
    """Many independent instances stepped together (dugks_create_batch)."""

    def __init__(self, cases, precision: int = FP32_DELTA, tiles=None, stream=None,
                 allow_defect=None, taylor_quad: float = 1.0, scheme: int = T3S3):
        n = len(cases)
        descs = (DugksDesc * n)()
        self._keep = []
        stream = _default_stream() if stream is None else stream
        for k, c in enumerate(cases):
            allow = (abs(c.vs.moment_defect()["sum_w_minus_1"]) > 1e-10) if allow_defect is None else allow_defect
            _, keep = make_desc(c, precision, taylor_quad, stream, tiles[k] if tiles else None, allow,
                                d=descs[k], scheme=scheme)
            self._keep.append(keep)
        self._descs = descs
        h = c_void_p()
        check(lib().dugks_create_batch(n, descs, byref(h)), "dugks_create_batch")
        self.h = h
        self.cases = list(cases)
        self.instances = []
        for k, c in enumerate(cases):
            ih = c_void_p()
            check(lib().dugks_batch_instance(h, k, byref(ih)), "dugks_batch_instance")
            self.instances.append(Solver(c, precision, _borrowed=ih))

    def step(self, n: int = 1):
        check(lib().dugks_step(self.h, int(n)), "dugks_step")

    def sync(self):
        check(lib().dugks_sync(self.h), "dugks_sync")

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(256)
        check(lib().dugks_describe(self.h, buf, 256), "dugks_describe")
        return buf.value.decode()

    def prof_begin(self, max_launches: int):
        check(lib().dugks_prof_begin(self.h, int(max_launches)), "dugks_prof_begin")

    def prof_query(self, kernel: int):
        ms = c_double()
        cnt = c_int()
        check(lib().dugks_prof_query(self.h, int(kernel), byref(ms), byref(cnt)), "dugks_prof_query")
        return ms.value, cnt.value

    def close(self):
        if getattr(self, "h", None):
            for inst in self.instances:
                inst.h = None
            lib().dugks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver3D:
    """One three-dimensional solver (a dugks3d_t handle) on a triply periodic
    box of uniform cells, from a cases.Case3; arrays [q][z][y][x]."""

    def __init__(self, case, precision: int = FP64, taylor_quad: float = 1.0, stream=None):
        vs = case.vs
        self.case = case
        self.nx, self.ny, self.nz = case.n
        self.nq = vs.nq
        self.ncell = case.ncell
        self.shape = (self.nz, self.ny, self.nx)
        tau = np.asarray(case.tau, dtype=np.float64)
        self._keep = [np.ascontiguousarray(vs.xi.reshape(-1), dtype=np.float64),
                      np.ascontiguousarray(vs.w, dtype=np.float64),
                      np.ascontiguousarray(np.broadcast_to(tau, self.shape).reshape(-1))]
        d = Dugks3dDesc()
        d.nx, d.ny, d.nz = case.n
        d.lx, d.ly, d.lz = case.L
        d.nq = vs.nq
        d.xi, d.w = _dptr(self._keep[0]), _dptr(self._keep[1])
        d.RT, d.dt = vs.RT, case.dt
        d.tau, d.tau0 = _dptr(self._keep[2]), float(self._keep[2].mean())
        d.precision = precision
        d.rho0 = float(case.rho0)
        d.taylor_quad = taylor_quad
        stream = _default_stream() if stream is None else stream
        d.stream = c_void_p(stream) if stream else None
        self.desc = d
        h = c_void_p()
        check(lib().dugks3d_create(byref(d), byref(h)), "dugks3d_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().dugks3d_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, f):
        p, mem, keep = _ptr_mem(f)
        check(lib().dugks3d_set_state(self.h, p, mem), "dugks3d_set_state")

    def init_equilibrium(self, rho, u):
        pr, mr, kr = _ptr_mem(rho)
        pu, mu, ku = _ptr_mem(u)
        if mr != mu:
            raise ValueError("rho and u must live in the same memory")
        check(lib().dugks3d_init_equilibrium(self.h, pr, pu, mr), "dugks3d_init_equilibrium")

    def step(self, n: int = 1):
        check(lib().dugks3d_step(self.h, int(n)), "dugks3d_step")

    def step_timed(self, n: int):
        """Advance n steps with HIP events around each launch; returns the mean
        (stage A ms, stage C ms)."""
        a, c = c_double(), c_double()
        check(lib().dugks3d_step_timed(self.h, int(n), byref(a), byref(c)), "dugks3d_step_timed")
        return a.value, c.value

    def moments(self):
        """(rho (nz, ny, nx), u (3, nz, ny, nx)) as numpy arrays."""
        r = np.empty(self.ncell)
        u = np.empty(3 * self.ncell)
        check(lib().dugks3d_moments(self.h, c_void_p(r.ctypes.data), c_void_p(u.ctypes.data), MEM_HOST),
              "dugks3d_moments")
        return r.reshape(self.shape), u.reshape((3,) + self.shape)

    def _dist(self, fn, out):
        if out is not None:
            p, mem, keep = _ptr_mem(out)
            check(fn(self.h, p, mem), fn.__name__)
            return out
        f = np.empty(self.nq * self.ncell)
        check(fn(self.h, c_void_p(f.ctypes.data), MEM_HOST), fn.__name__)
        return f.reshape((self.nq,) + self.shape)

    def get_state(self, out=None):
        return self._dist(lib().dugks3d_get_state, out)

    def get_fhat(self, out=None):
        return self._dist(lib().dugks3d_get_fhat, out)
