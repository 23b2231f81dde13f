"""Inputs of the DUGKS sweep: discrete velocity sets, quadrature weights, grids,
initial macroscopic fields and seeded noise.

Nothing here evaluates the scheme (no equilibrium, no flux, no time step): the
module only builds the data that the library (``dugks_create``,
``dugks_init_equilibrium``) and the oracle both take as plain arrays.

Paper: Wu, Shu, Shi & Chen, "A third-order discrete unified gas kinetic scheme
for continuum and rarefied flows: low-speed isothermal case" (arXiv 1709.05458).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Seeded noise: SplitMix64 -> uniform (0,1) -> Box-Muller normals.
# ---------------------------------------------------------------------------
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """n successive outputs of Vigna's SplitMix64 generator started at `seed`."""
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """Uniform doubles in (0, 1) from the top 53 bits of SplitMix64."""
    z = splitmix64(seed, n) >> np.uint64(11)
    return (z.astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def normal(seed: int, n: int) -> np.ndarray:
    """Standard normals by the Box-Muller transform of pairs of uniforms."""
    m = (n + 1) // 2
    u = uniform01(seed, 2 * m)
    r = np.sqrt(-2.0 * np.log(u[0::2]))
    t = 2.0 * math.pi * u[1::2]
    return np.concatenate([r * np.cos(t), r * np.sin(t)])[:n]


# ---------------------------------------------------------------------------
# Discrete velocity sets (paper section "Discrete particle velocities").
# ---------------------------------------------------------------------------
@dataclass
class VelocitySet:
    """Discrete velocities xi[2][Q] and equilibrium weights w[Q].

    ``w`` already holds the Gaussian factor of the Maxwellian, so that the
    low-Mach equilibrium is w_q*rho*[1 + xi.u/RT + (xi.u)^2/(2 RT^2) - u^2/(2RT)].
    ``opp[q]`` is the index of -xi_q (needed by bounce-back walls).
    """

    name: str
    xi: np.ndarray          # (2, Q) float64
    w: np.ndarray           # (Q,) float64
    RT: float
    opp: np.ndarray = field(default=None)   # (Q,) int32
    renormalized: bool = False

    def __post_init__(self):
        self.xi = np.ascontiguousarray(self.xi, dtype=np.float64)
        self.w = np.ascontiguousarray(self.w, dtype=np.float64)
        if self.opp is None:
            self.opp = opposite_index(self.xi)

    @property
    def nq(self) -> int:
        return self.w.shape[0]

    @property
    def cmax(self) -> float:
        """Largest velocity component, the C of the CFL condition."""
        return float(np.max(np.abs(self.xi)))

    def moment_defect(self) -> dict:
        """How far the weights are from reproducing the isothermal Gaussian
        moments that exact mass/momentum conservation needs."""
        w, x, y = self.w, self.xi[0], self.xi[1]
        return {
            "sum_w_minus_1": float(w.sum() - 1.0),
            "sum_w_xi": float(max(abs((w * x).sum()), abs((w * y).sum()))),
            "sum_w_xx_minus_RT": float((w * x * x).sum() / self.RT - 1.0),
            "sum_w_yy_minus_RT": float((w * y * y).sum() / self.RT - 1.0),
            "sum_w_xy": float((w * x * y).sum()),
        }


def opposite_index(xi: np.ndarray) -> np.ndarray:
    """opp[q] = index of -xi_q, or -1 where the set has no mirror velocity."""
    q = xi.shape[1]
    opp = np.full(q, -1, dtype=np.int32)
    scale = max(1e-300, float(np.max(np.abs(xi))))
    for a in range(q):
        d = np.abs(xi + xi[:, a:a + 1]).max(axis=0)
        hit = np.nonzero(d <= 1e-12 * scale)[0]
        if hit.size:
            opp[a] = hit[0]
    return opp


def d2q9(RT: float) -> VelocitySet:
    """Tensor product of the 3-point Gauss-Hermite rule, in the paper's order.

    The paper's 1D weights are printed as (1/3, 2/3, 1/3), which do not sum to
    one; the 2D weights it prints (1/36, 1/9, 4/9) are the products of
    (1/6, 2/3, 1/6), the true 3-point Gauss-Hermite weights, so those are used.
    """
    c = math.sqrt(3.0 * RT)
    e1 = np.array([-1.0, 0.0, 1.0])
    w1 = np.array([1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0])
    xi = np.stack([np.repeat(e1, 3), np.tile(e1, 3)]) * c
    w = np.outer(w1, w1).reshape(-1)
    return VelocitySet("D2Q9", xi, w, RT)


def composite_newton_cotes(n: int) -> np.ndarray:
    """Weights of a closed composite Newton-Cotes rule on n equispaced nodes of
    unit spacing, chosen mirror-symmetric (odd moments of a symmetric velocity
    grid must vanish for mass and momentum to be conserved):
    Boole panels when the interval count m = n-1 is a multiple of 4, else 3/8
    panels when a multiple of 3, else Simpson panels when even; for odd m,
    Simpson panels on both sides of one central 3/8 panel (m = 3 mod 4) or of
    one central 6-point panel (m = 1 mod 4)."""
    if n < 2:
        raise ValueError("need at least 2 nodes")
    m = n - 1
    w = np.zeros(n)
    simpson = np.array([1.0, 4.0, 1.0]) / 3.0
    three8 = np.array([1.0, 3.0, 3.0, 1.0]) * (3.0 / 8.0)
    boole = np.array([7.0, 32.0, 12.0, 32.0, 7.0]) * (2.0 / 45.0)
    six = np.array([19.0, 75.0, 50.0, 50.0, 75.0, 19.0]) * (5.0 / 288.0)

    def add(start, panel):
        w[start:start + len(panel)] += panel

    if m == 1:
        add(0, np.array([0.5, 0.5]))
    elif m % 4 == 0:
        for s in range(0, m, 4):
            add(s, boole)
    elif m % 3 == 0:
        for s in range(0, m, 3):
            add(s, three8)
    elif m % 2 == 0:
        for s in range(0, m, 2):
            add(s, simpson)
    else:
        mid = three8 if m % 4 == 3 else six
        side = (m - (len(mid) - 1)) // 2
        for s in range(0, side, 2):
            add(s, simpson)
        add(side, mid)
        for s in range(side + len(mid) - 1, m, 2):
            add(s, simpson)
    return w


def newton_cotes(n: int, RT: float, half_width: float = 4.0,
                 renormalize: bool = False) -> VelocitySet:
    """n x n uniformly spaced velocities on [-h sqrt(RT), h sqrt(RT)]^2 with
    composite Newton-Cotes weights times the Gaussian factor
    exp(-|xi|^2/2RT)/(2 pi RT).

    ``renormalize`` (not in the paper) rescales w_q by (a + b |xi_q|^2) so
    that sum w = 1 and sum w xi xi = RT I hold to round-off, which is what
    exact conservation of mass and momentum needs.
    """
    # exactly mirror-symmetric nodes: v_k = (2k - (n-1)) * dv / 2
    dv = 2.0 * half_width * math.sqrt(RT) / (n - 1)
    v = (2.0 * np.arange(n) - (n - 1)) * (0.5 * dv)
    W1 = composite_newton_cotes(n) * dv
    vx = np.repeat(v, n)
    vy = np.tile(v, n)
    W = np.outer(W1, W1).reshape(-1)
    w = W * np.exp(-(vx * vx + vy * vy) / (2.0 * RT)) / (2.0 * math.pi * RT)
    if renormalize:
        r2 = vx * vx + vy * vy
        A = np.array([[w.sum(), (w * r2).sum()],
                      [(w * vx * vx).sum(), (w * vx * vx * r2).sum()]])
        a, b = np.linalg.solve(A, np.array([1.0, RT]))
        w = w * (a + b * r2)
    vs = VelocitySet(f"NC{n}x{n}", np.stack([vx, vy]), w, RT,
                     renormalized=renormalize)
    return vs


_D2Q37_SHELLS = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1)]


def _shell_vectors(a: int, b: int):
    out = set()
    for (p, q) in ((a, b), (b, a)):
        for sp in (1, -1):
            for sq in (1, -1):
                out.add((sp * p, sq * q))
    return sorted(out)


def d2q37(RT: float) -> VelocitySet:
    """A 37-velocity integer lattice (shells (0,0), (1,0), (1,1), (2,0), (2,1),
    (2,2), (3,0), (3,1)) scaled by r sqrt(RT).  Not in the paper.

    The 8 shell weights and the scale r are found here by requiring that the
    set reproduce every moment of the unit Gaussian up to degree 9 (odd ones
    vanish by symmetry; the even ones give 9 equations: degree 0 (1), 2 (1),
    4 (2), 6 (2), 8 (3)).  For fixed r the equations are linear in the weights,
    so r is the root of the determinant of the augmented 9x9 system."""
    from scipy.optimize import brentq

    shells = [_shell_vectors(a, b) for (a, b) in _D2Q37_SHELLS]
    # (px, py, gaussian moment) for even monomials up to degree 8
    mons = [(0, 0, 1.0), (2, 0, 1.0), (4, 0, 3.0), (2, 2, 1.0), (6, 0, 15.0),
            (4, 2, 3.0), (8, 0, 105.0), (6, 2, 15.0), (4, 4, 9.0)]

    def system(r):
        A = np.zeros((len(mons), len(shells)))
        b = np.zeros(len(mons))
        for i, (px, py, g) in enumerate(mons):
            b[i] = g
            for s, vecs in enumerate(shells):
                A[i, s] = sum((r * ex) ** px * (r * ey) ** py for ex, ey in vecs)
        return A, b

    def det(r):
        A, b = system(r)
        return np.linalg.det(np.concatenate([A, b[:, None]], axis=1))

    grid = np.linspace(1.0, 1.5, 501)
    vals = [det(r) for r in grid]
    root = None
    for k in range(len(grid) - 1):
        if vals[k] == 0.0 or vals[k] * vals[k + 1] < 0:
            rr = brentq(det, grid[k], grid[k + 1], xtol=1e-15, rtol=1e-15, maxiter=200)
            A, b = system(rr)
            ws, *_ = np.linalg.lstsq(A, b, rcond=None)
            if np.all(ws > 0):
                root = (rr, ws)
                break
    if root is None:
        raise RuntimeError("no positive D2Q37 weight set found")
    r, ws = root
    # Newton polish of (r, weights) on the square 9x9 nonlinear system.
    for _ in range(8):
        A, b = system(r)
        dA = np.zeros_like(A)
        for i, (px, py, g) in enumerate(mons):
            k = px + py
            for s, vecs in enumerate(shells):
                if k:
                    dA[i, s] = k * r ** (k - 1) * sum(ex ** px * ey ** py for ex, ey in vecs)
        F = A @ ws - b
        J = np.concatenate([dA @ ws[:, None], A], axis=1)
        step = np.linalg.solve(J, -F)
        r += step[0]
        ws = ws + step[1:]
    xs, ys, wl = [], [], []
    for s, vecs in enumerate(shells):
        for ex, ey in vecs:
            xs.append(ex)
            ys.append(ey)
            wl.append(ws[s])
    xi = np.array([xs, ys], dtype=np.float64) * (r * math.sqrt(RT))
    vs = VelocitySet("D2Q37", xi, np.array(wl), RT)
    vs.lattice_scale = r
    return vs


# ---------------------------------------------------------------------------
# Grids: tensor-product Cartesian control volumes given by face coordinates.
# ---------------------------------------------------------------------------
@dataclass
class Grid:
    xf: np.ndarray   # (nx+1,) face x-coordinates, increasing
    yf: np.ndarray   # (ny+1,)

    @property
    def nx(self) -> int:
        return self.xf.shape[0] - 1

    @property
    def ny(self) -> int:
        return self.yf.shape[0] - 1

    @property
    def xc(self) -> np.ndarray:
        return 0.5 * (self.xf[1:] + self.xf[:-1])

    @property
    def yc(self) -> np.ndarray:
        return 0.5 * (self.yf[1:] + self.yf[:-1])

    @property
    def dmin(self) -> float:
        return float(min(np.diff(self.xf).min(), np.diff(self.yf).min()))

    def is_uniform(self, rtol=1e-12) -> bool:
        dx, dy = np.diff(self.xf), np.diff(self.yf)
        return bool(np.ptp(dx) <= rtol * dx.max() and np.ptp(dy) <= rtol * dy.max())


def uniform_grid(nx: int, ny: int, Lx: float = 1.0, Ly: float = 1.0,
                 x0: float = 0.0, y0: float = 0.0) -> Grid:
    return Grid(x0 + Lx * np.arange(nx + 1) / nx, y0 + Ly * np.arange(ny + 1) / ny)


def tanh_faces(n: int, beta: float = 1.5) -> np.ndarray:
    """Faces x_k = (1 + tanh(beta (2k/n - 1)) / tanh(beta)) / 2 on [0, 1]."""
    k = np.arange(n + 1)
    return 0.5 * (1.0 + np.tanh(beta * (2.0 * k / n - 1.0)) / math.tanh(beta))


def tanh_grid(nx: int, ny: int, beta: float = 1.5) -> Grid:
    return Grid(tanh_faces(nx, beta), tanh_faces(ny, beta))


# ---------------------------------------------------------------------------
# Boundary codes (shared numbering with include/dugks.h).
# ---------------------------------------------------------------------------
BC_PERIODIC, BC_BOUNCE_BACK, BC_DIFFUSE = 0, 1, 2
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3


# ---------------------------------------------------------------------------
# Initial macroscopic fields.
# ---------------------------------------------------------------------------
def taylor_green_fields(xc, yc, t, u0, A, B, nu, RT, rho0=1.0):
    """Analytic incompressible Taylor-Green vortex (paper's Taylor vortex flow
    section), returned on the cell centres as (rho, ux, uy) with shape
    (ny, nx); density follows the isothermal law rho = rho0 + p/RT."""
    X, Y = np.meshgrid(xc, yc)
    alpha = A * A + B * B
    d = math.exp(-nu * alpha * t)
    ux = -(u0 / A) * np.cos(A * X) * np.sin(B * Y) * d
    uy = (u0 / B) * np.sin(A * X) * np.cos(B * Y) * d
    p = -(u0 * u0 / 4.0) * (np.cos(2 * A * X) / (A * A) + np.cos(2 * B * Y) / (B * B)) * d * d
    rho = rho0 + p / RT
    return rho, ux, uy


@dataclass
class Case:
    """Everything dugks_create needs, plus the initial macroscopic state."""

    name: str
    grid: Grid
    vs: VelocitySet
    dt: float
    tau: np.ndarray           # (ny, nx) per-cell relaxation time
    bc: tuple                 # (west, east, south, north)
    u_wall: np.ndarray        # (4, 2)
    rho: np.ndarray           # (ny, nx)
    ux: np.ndarray
    uy: np.ndarray
    rho0: float = 1.0
    steps: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def ncell(self) -> int:
        return self.grid.nx * self.grid.ny


def tgv_case(n: int, vs: VelocitySet | None = None, nu: float = 0.01,
             ma: float = 0.05, cfl: float = 0.5, noise: float = 0.01,
             seed: int = 1709054580, steps: int = 200, RT: float = 1.0 / 3.0) -> Case:
    """Taylor-Green vortex on [0, 2 pi]^2, periodic, A = B = 1.

    u0 = Ma * sqrt(3 RT); tau = nu / RT; dt = cfl * dx / C with C the largest
    velocity component; additive noise noise*u0*N(0,1) per cell and component.
    """
    vs = vs if vs is not None else d2q9(RT)
    L = 2.0 * math.pi
    g = uniform_grid(n, n, L, L)
    u0 = ma * math.sqrt(3.0 * RT)
    tau0 = nu / RT
    dt = cfl * g.dmin / vs.cmax
    rho, ux, uy = taylor_green_fields(g.xc, g.yc, 0.0, u0, 1.0, 1.0, nu, RT)
    if noise:
        z = normal(seed, 2 * n * n).reshape(2, n, n)
        ux = ux + noise * u0 * z[0]
        uy = uy + noise * u0 * z[1]
    return Case(f"tgv{n}_{vs.name}", g, vs, dt, np.full((n, n), tau0),
                (BC_PERIODIC,) * 4, np.zeros((4, 2)), rho, ux, uy, 1.0, steps,
                {"u0": u0, "nu": nu, "A": 1.0, "B": 1.0, "noise": noise, "seed": seed})


def cavity_case(n: int, vs: VelocitySet | None = None, re: float = 400.0,
                ma: float = 0.1, cfl: float = 0.5, wall: int = BC_BOUNCE_BACK,
                steps: int = 1000, RT: float = 1.0 / 3.0, grid: Grid | None = None,
                tau: float | None = None, lid: float | None = None) -> Case:
    """Lid-driven cavity on [0,1]^2 at rest, walls of kind `wall`, north lid
    moving with u = (U, 0); U = Ma sqrt(3 RT) unless `lid` is given;
    nu = U/Re, tau = nu/RT unless `tau` is given."""
    vs = vs if vs is not None else d2q9(RT)
    g = grid if grid is not None else uniform_grid(n, n)
    U = lid if lid is not None else ma * math.sqrt(3.0 * RT)
    t0 = tau if tau is not None else (U / re) / RT
    dt = cfl * g.dmin / vs.cmax
    uw = np.zeros((4, 2))
    uw[NORTH, 0] = U
    shape = (g.ny, g.nx)
    return Case(f"cavity{n}_{vs.name}", g, vs, dt, np.full(shape, t0),
                (wall,) * 4, uw, np.ones(shape), np.zeros(shape), np.zeros(shape),
                1.0, steps, {"U": U, "Re": re})


def shear_layer_fields(xc, yc, k: float = 80.0, delta: float = 0.05, U: float = 1.0):
    """Doubly periodic shear layers on [0,1]^2 (paper's shear-layer section):
    u_x = U tanh(k (y - 1/4)) for y <= 1/2 and U tanh(k (3/4 - y)) above,
    u_y = U delta sin(2 pi (x + 1/4)); rho = 1.  Shape (ny, nx)."""
    X, Y = np.meshgrid(xc, yc)
    ux = U * np.where(Y <= 0.5, np.tanh(k * (Y - 0.25)), np.tanh(k * (0.75 - Y)))
    uy = U * delta * np.sin(2.0 * math.pi * (X + 0.25))
    return np.ones_like(X), ux, uy


def shear_layer_case(n: int = 128, vs: VelocitySet | None = None, k: float = 80.0,
                     delta: float = 0.05, nu: float = 1e-4, U: float = 1.0, ma: float = 0.15,
                     dt_over_tau: float = 10.0, t_end: float = 1.0) -> Case:
    """The paper's shear-layer workload: k = 80, delta = 0.05, nu = 1e-4
    (Re = U L / nu = 10^4), periodic, n x n uniform cells on [0,1]^2.

    The paper gives neither the lattice temperature nor the step.  RT follows
    from Ma = U / sqrt(3 RT) (0.15, the paper's cavity Mach number), tau =
    nu / RT, and dt = dt_over_tau * tau, below the bound of 12; the CFL
    number dt C / dx is then far below 1 at these sizes.  steps reaches
    t_end."""
    RT = (U / ma) ** 2 / 3.0
    vs = vs if vs is not None else d2q9(RT)
    g = uniform_grid(n, n)
    tau0 = nu / vs.RT
    dt = dt_over_tau * tau0
    if dt * vs.cmax > g.dmin:
        raise ValueError("CFL number above 1 for this size; lower dt_over_tau")
    rho, ux, uy = shear_layer_fields(g.xc, g.yc, k, delta, U)
    return Case(f"shear{n}_{vs.name}", g, vs, dt, np.full((n, n), tau0),
                (BC_PERIODIC,) * 4, np.zeros((4, 2)), rho, ux, uy, 1.0,
                int(round(t_end / dt)), {"U": U, "k": k, "delta": delta, "nu": nu, "Ma": ma})


def couette_case(n: int, vs: VelocitySet, tau: float, U: float, cfl: float = 0.25,
                 grid: Grid | None = None, steps: int = 1000) -> Case:
    """Planar Couette flow: periodic in x, diffuse walls at y = 0 and y = 1
    moving with -U/2 and +U/2."""
    g = grid if grid is not None else uniform_grid(n, n)
    dt = cfl * g.dmin / vs.cmax
    uw = np.zeros((4, 2))
    uw[SOUTH, 0] = -0.5 * U
    uw[NORTH, 0] = 0.5 * U
    shape = (g.ny, g.nx)
    return Case(f"couette{n}_{vs.name}", g, vs, dt, np.full(shape, tau),
                (BC_PERIODIC, BC_PERIODIC, BC_DIFFUSE, BC_DIFFUSE), uw,
                np.ones(shape), np.zeros(shape), np.zeros(shape), 1.0, steps, {"U": U})


def kn_to_tau(kn: float, RT: float, L: float = 1.0) -> float:
    """Mean free path lambda = tau sqrt(pi RT / 2) (paper, numerical tests),
    so tau = Kn L / sqrt(pi RT / 2)."""
    return kn * L / math.sqrt(math.pi * RT / 2.0)


def perturbed_tau(tau0: float, shape, rel: float, seed: int) -> np.ndarray:
    """tau0 * (1 + rel * N(0,1)) per cell, seeded."""
    z = normal(seed, int(np.prod(shape))).reshape(shape)
    return tau0 * (1.0 + rel * z)


def batch_cases(n: int = 64, seed: int = 4, nmin: int = 32, nmax: int = 256,
                ncmin: int = 16, ncmax: int = 40, kn_lo: float = -3.0, kn_hi: float = 1.0) -> list:
    """Independent lid-driven cavity instances of uneven size (seeded):
    side N ~ U{nmin..nmax}; velocity set D2Q9 (probability 1/2; bounce-back,
    RT = 1/3, CFL 0.5) or an n x n Newton-Cotes grid, n ~ U{ncmin..ncmax}
    (moment-renormalised; diffuse walls, RT = 0.5, CFL 0.25); Kn log-uniform
    in [10^kn_lo, 10^kn_hi], tau = Kn sqrt(2 / (pi RT)); lid Ma 0.1 against
    sqrt(3 RT); dt = min(CFL dx / C, 8 tau), which keeps dt/tau <= 8."""
    u = uniform01(seed, 4 * n).reshape(n, 4)
    out = []
    for k in range(n):
        N = nmin + min(nmax - nmin, int(u[k, 0] * (nmax - nmin + 1)))
        kn = 10.0 ** (kn_lo + (kn_hi - kn_lo) * u[k, 2])
        if u[k, 1] < 0.5:
            RT, cfl, wall = 1.0 / 3.0, 0.5, BC_BOUNCE_BACK
            vs = d2q9(RT)
        else:
            RT, cfl, wall = 0.5, 0.25, BC_DIFFUSE
            nc = ncmin + min(ncmax - ncmin, int(u[k, 3] * (ncmax - ncmin + 1)))
            vs = newton_cotes(nc, RT, renormalize=True)
        tau = kn_to_tau(kn, RT)
        lid = 0.1 * math.sqrt(3.0 * RT)
        c = cavity_case(N, vs, wall=wall, tau=tau, lid=lid, cfl=cfl, RT=RT)
        c.dt = min(c.dt, 8.0 * tau)
        c.name = f"batch{k}_{N}_{vs.name}_Kn{kn:.3g}"
        c.meta.update({"Kn": kn, "cfl": cfl})
        out.append(c)
    return out


# ---------------------------------------------------------------------------
# Three space dimensions: velocity sets, the periodic box and its flows.
# A VelocitySet here holds xi with shape (3, Q).
# ---------------------------------------------------------------------------
def d3q27(RT: float) -> VelocitySet:
    """Tensor product of the 3-point Gauss-Hermite rule in three dimensions
    (weights (1/6, 2/3, 1/6) per axis, c = sqrt(3 RT)); q = 9 ix + 3 iy + iz
    over the components (-c, 0, c)."""
    c = math.sqrt(3.0 * RT)
    e1 = np.array([-1.0, 0.0, 1.0])
    w1 = np.array([1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0])
    ix, iy, iz = np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij")
    ix, iy, iz = ix.reshape(-1), iy.reshape(-1), iz.reshape(-1)
    xi = np.stack([e1[ix], e1[iy], e1[iz]]) * c
    w = w1[ix] * w1[iy] * w1[iz]
    return VelocitySet("D3Q27", xi, w, RT)


def d3q19(RT: float) -> VelocitySet:
    """The 19 velocities of D3Q27 with at most two nonzero components, weights
    1/3 (rest), 1/18 (one component) and 1/36 (two), c = sqrt(3 RT): they
    reproduce the isothermal Gaussian moments up to fourth order that the
    second-order equilibrium needs.  Order: that of D3Q27 with the eight
    corner velocities left out."""
    full = d3q27(RT)
    nz = np.count_nonzero(np.abs(full.xi) > 0, axis=0)
    keep = nz <= 2
    wt = np.array([1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0])
    return VelocitySet("D3Q19", full.xi[:, keep], wt[nz[keep]], RT)


@dataclass
class Case3:
    """A triply periodic box of uniform cells, velocity set, tau field and
    initial macroscopic state, arrays [z][y][x]."""

    name: str
    n: tuple                 # (nx, ny, nz)
    L: tuple                 # (Lx, Ly, Lz)
    vs: VelocitySet
    dt: float
    tau: np.ndarray          # (nz, ny, nx)
    rho: np.ndarray          # (nz, ny, nx)
    u: np.ndarray            # (3, nz, ny, nx)
    rho0: float = 1.0
    steps: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def ncell(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def h(self) -> tuple:
        return tuple(self.L[a] / self.n[a] for a in range(3))

    def centres(self):
        """Cell-centre coordinates X, Y, Z, each (nz, ny, nx)."""
        ax = [(np.arange(self.n[a]) + 0.5) * self.h[a] for a in range(3)]
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        return X, Y, Z


def abc_fields(X, Y, Z, u0: float, RT: float, rho0: float = 1.0):
    """Arnold-Beltrami-Childress flow with A = B = C = 1 on [0, 2 pi]^3,
    scaled to peak speed component u0: u = (u0/2)(sin z + cos y,
    sin x + cos z, sin y + cos x).  It is a Beltrami field (curl u = u), so
    u.grad u = grad |u|^2/2 and the incompressible flow decays as
    exp(-nu t) with p = -rho0 |u|^2 / 2; the density follows the
    isothermal law rho = rho0 + p / RT."""
    a = 0.5 * u0
    u = np.stack([a * (np.sin(Z) + np.cos(Y)), a * (np.sin(X) + np.cos(Z)), a * (np.sin(Y) + np.cos(X))])
    rho = rho0 - rho0 * (u * u).sum(axis=0) / (2.0 * RT)
    return rho, u


def abc_case(n: int, vs: VelocitySet | None = None, nu: float = 0.01, ma: float = 0.05,
             cfl: float = 0.5, noise: float = 0.0, seed: int = 1709054583, steps: int = 100,
             RT: float = 1.0 / 3.0, shape: tuple | None = None) -> Case3:
    """ABC flow on [0, 2 pi]^3 (n cells per side, or `shape` = (nx, ny, nz)
    cells over the same box), u0 = Ma sqrt(3 RT), tau = nu / RT,
    dt = cfl dx / C; optional additive noise noise*u0*N(0,1) per cell and
    component (seeded)."""
    vs = vs if vs is not None else d3q19(RT)
    shape = tuple(shape) if shape is not None else (n, n, n)
    L = (2.0 * math.pi,) * 3
    c = Case3("", shape, L, vs, 0.0, np.zeros(0), np.zeros(0), np.zeros(0))
    X, Y, Z = c.centres()
    u0 = ma * math.sqrt(3.0 * RT)
    rho, u = abc_fields(X, Y, Z, u0, RT)
    if noise:
        u = u + noise * u0 * normal(seed, u.size).reshape(u.shape)
    c.name = f"abc{shape[0]}x{shape[1]}x{shape[2]}_{vs.name}"
    c.dt = cfl * min(c.h) / vs.cmax
    c.tau = np.full(rho.shape, nu / RT)
    c.rho, c.u, c.steps = rho, u, steps
    c.meta = {"u0": u0, "nu": nu, "noise": noise, "seed": seed}
    return c
