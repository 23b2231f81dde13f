"""Inputs: velocity sets, quadrature rules, grids and the seeded generator."""
import math
import os
from fractions import Fraction

import numpy as np

from paper_1709_05458_amd import cases as C

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_d2q9_matches_paper_table():
    # golden: the 2D velocities and weights printed in the paper's
    # "Discrete particle velocities" section
    rows = [l.split() for l in open(os.path.join(GOLD, "d2q9_weights.txt"))
            if l.strip() and not l.startswith("#")]
    RT = 0.7
    vs = C.d2q9(RT)
    c = math.sqrt(3 * RT)
    for q, (ex, ey, w) in enumerate(rows):
        assert vs.xi[0, q] == float(ex) * c and vs.xi[1, q] == float(ey) * c
        assert abs(vs.w[q] - float(Fraction(w))) < 1e-16
    assert list(vs.opp) == [8, 7, 6, 5, 4, 3, 2, 1, 0]


def test_gauss_hermite_moments_d2q9_and_d2q37():
    # sum w xi^a eta^b equals the moments of the Gaussian of variance RT up
    # to degree 5 (D2Q9) / 9 (D2Q37)
    def gauss(a, b, RT):
        def m(k):
            return 0.0 if k % 2 else float(np.prod(np.arange(k - 1, 0, -2))) * RT ** (k // 2)
        return m(a) * m(b)
    for vs, deg in ((C.d2q9(0.5), 3), (C.d2q37(0.5), 9)):
        x, y, w = vs.xi[0], vs.xi[1], vs.w
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                if vs.nq == 9 and (a > 3 or b > 3 or (a == 3 and b == 0) or (b == 3 and a == 0)):
                    # D2Q9 is exact only for monomials of degree <= 3 in each direction
                    pass
                got = (w * x ** a * y ** b).sum()
                if vs.nq == 9 and (a >= 4 or b >= 4):
                    continue
                if vs.nq == 9 and (a == 2 and b == 2):
                    assert abs(got - gauss(2, 2, 0.5)) < 1e-14
                    continue
                assert abs(got - gauss(a, b, 0.5)) < 1e-12 * max(1.0, gauss(a, b, 0.5)), (vs.name, a, b)


def test_newton_cotes_rule_exactness():
    # each composite rule integrates polynomials of its panel degree exactly
    for n, deg in ((101, 5), (41, 5), (28, 3), (16, 3), (23, 3), (30, 3), (8, 3), (6, 3),
                   (14, 3), (20, 3), (26, 3), (38, 3)):
        W = C.composite_newton_cotes(n)
        assert np.allclose(W, W[::-1], rtol=0, atol=1e-15), n   # mirror symmetric
        x = np.arange(n, dtype=float)
        L = n - 1
        for k in range(deg + 1):
            exact = L ** (k + 1) / (k + 1)
            assert abs((W * x ** k).sum() - exact) < 1e-9 * exact, (n, k)


def test_newton_cotes_velocity_set_and_renormalisation():
    vs = C.newton_cotes(101, 0.5)
    d = vs.moment_defect()
    # Gaussian tail beyond +-4 sigma in each direction
    tail = math.erfc(4 / math.sqrt(2))
    assert abs(d["sum_w_minus_1"] + 2 * tail) < 2e-5
    assert np.all(vs.opp == np.arange(vs.nq)[::-1])
    r = C.newton_cotes(28, 0.5, renormalize=True).moment_defect()
    assert abs(r["sum_w_minus_1"]) < 1e-14 and abs(r["sum_w_xx_minus_RT"]) < 1e-13


def test_splitmix64_reference_vector():
    # published first outputs of SplitMix64 started at 0
    z = C.splitmix64(0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    g = C.normal(42, 200000)
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1) < 0.01
    assert np.array_equal(C.normal(7, 10), C.normal(7, 10))


def test_grids():
    g = C.tanh_grid(64, 64)
    assert abs(g.xf[0]) < 1e-15 and abs(g.xf[-1] - 1) < 1e-15
    assert abs(g.dmin - 4.88e-3) < 1e-4
    assert not g.is_uniform() and C.uniform_grid(8, 8).is_uniform()
    # mean free path relation lambda = tau sqrt(pi RT / 2)
    tau = C.kn_to_tau(1.0, 0.5)
    assert abs(tau * math.sqrt(math.pi * 0.5 / 2) - 1.0) < 1e-15
