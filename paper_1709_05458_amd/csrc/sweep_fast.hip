// Stage kernels of the lattice sweep (D2Q9, D2Q37) for the common case: a
// uniform grid and a tile clear of walls (periodic or interior), with the
// tile shape fixed at compile time.  One launch is one stage of the step
// (paper, "Computational sequence of the third-order DUGKS"):
//   STAGE 0 (steps (1)-(2)): X = fhat(t_n)          -> out = tilde f(t')
//   STAGE 1 (steps (3)-(4)): X = tilde f(t'), F = fhat(t_n) -> out = fhat(t_{n+1})
//
// The arithmetic is the one of the general kernel in sweep.hip; what differs
// is the schedule:
//  * the halo fill loads every velocity of all of a thread's load slots before
//    it forms any moment, so each per-velocity weight is read once and is dead
//    right after (no scalar-register spills), and LDS / global offsets are
//    compile-time immediates;
//  * the own cell's share of the output is one register per velocity, and
//    every equilibrium term of the output (E^n, E' and the equilibrium part of
//    the recovered interface values, eqs. recover2f and microflux) is summed
//    into one cubic polynomial in the lattice vector before the last pass;
//  * the linear part of the micro-flux is kept as one register per velocity,
//    scaled by per-thread multiples of 1/dx, 1/dy chosen at compile time.
// Every fused multiply-add of this file, and of the inline helpers it takes
// from the headers below, is written out; no other contraction, so that the
// single-instance and batched kernels round identically (a contractible
// multiply and add may be fused in one kernel and not in the other).
#pragma clang fp contract(off)

#include "dugks_internal.h"
#include "lattices.h"
#include "launchers.h"
#include "sweep_common.h"

#include <type_traits>
#include <utility>

namespace dk {

// x / y interface values of the four faces of the own cell from the window
// weights of one velocity (uniform spacing; upwind choice, foot point and
// 3-point derivatives folded into the weights), their moments in double,
// and the linear flux part (added to R with its factor aLs).
template <class Lat, class S, bool DELTA, bool TF, int q, int HX, int PL>
__device__ __forceinline__ void fast_faces(const SweepParams &p, const S *lds, const S *__restrict__ C,
                                           double (&mr)[4], double (&mx)[4], double (&my)[4], const S (&kxm)[4],
                                           const S (&kym)[4], const S (&al)[4], S aLs, S &R)
{
    constexpr int EX = Lat::ex(q), EY = Lat::ey(q), SH = Lat::shell(q);
    const S *P = lds + q * PL;
    S vw = 0, ve = 0, vs = 0, vn = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if ((EX > 0 && k == 3) || (EX < 0 && k == 0)) continue;
#pragma unroll
        for (int b = 0; b < 3; b++) {
            const S c = C[k * 3 + b];
            vw = fmaS(c, P[(b - 1) * HX + (k - 2)], vw);
            ve = fmaS(c, P[(b - 1) * HX + (k - 1)], ve);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if ((EY > 0 && k == 3) || (EY < 0 && k == 0)) continue;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const S c = C[12 + k * 3 + a];
            vs = fmaS(c, P[(k - 2) * HX + (a - 1)], vs);
            vn = fmaS(c, P[(k - 1) * HX + (a - 1)], vn);
        }
    }
    const S v4[4] = {vw, ve, vs, vn};
#pragma unroll
    for (int f = 0; f < 4; f++) {
        const double d = (double)v4[f];
        if (DELTA) {
            mr[f] = __builtin_fma(p.wtab[SH][1], d, mr[f]);
            if (EX) mx[f] = __builtin_fma(EX > 0 ? p.wtab[SH][EX] : -p.wtab[SH][-EX], d, mx[f]);
            if (EY) my[f] = __builtin_fma(EY > 0 ? p.wtab[SH][EY] : -p.wtab[SH][-EY], d, my[f]);
        } else {
            mr[f] += d;
            if (EX) mx[f] = __builtin_fma((double)EX, d, mx[f]);
            if (EY) my[f] = __builtin_fma((double)EY, d, my[f]);
        }
    }
    // linear part of L: -(xi_x/dx)(alpha_e ve - alpha_w vw) - (xi_y/dy)(alpha_n vn - alpha_s vs)
    S l = 0;
    if (EX) {
        const S kx = EX > 0 ? kxm[EX] : -kxm[-EX];
        const S dxv = TF ? fmaS(al[1], ve, -al[0] * vw) : ve - vw;
        l = kx * dxv;
    }
    if (EY) {
        const S ky = EY > 0 ? kym[EY] : -kym[-EY];
        const S dyv = TF ? fmaS(al[3], vn, -al[2] * vs) : vn - vs;
        l = fmaS(ky, dyv, l);
    }
    R = fmaS(aLs, l, R);   // the flux part joins the own-cell part at once
    // keep the next velocity's loads below this one (register pressure)
    __builtin_amdgcn_sched_barrier(0);
}

// index of the rest velocity (its own opposite)
template <class Lat>
constexpr int rest_velocity()
{
    for (int q = 0; q < Lat::Q; q++)
        if (Lat::opp(q) == q) return q;
    return 0;
}

// TF: per-cell relaxation times (a tau field) rather than one tau
template <class Lat, class S, bool DELTA, bool TF, int STAGE, int TX, int TY>
__device__ __forceinline__ void fast_body(const SweepParams &p, const double h, const S *__restrict__ X,
                                          const S *__restrict__ F, S *__restrict__ out,
                                          const S *__restrict__ coef, int tx, int ty)
{
    constexpr int Q = Lat::Q, NT = TX * TY, HX = TX + 4, PL = HX * (TY + 4);
    constexpr int NS = (PL + NT - 1) / NT;
    constexpr int PS = PL + 1;   // plane stride: one spare element takes the writes of unused slots
    using Seq = std::make_integer_sequence<int, Q>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    S *lds = reinterpret_cast<S *>(smem_raw);

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int i0 = tx * TX, j0 = ty * TY;
    const int i = i0 + lx, j = j0 + ly;
    const bool valid = (i < p.nx) && (j < p.ny);
    const size_t n = (size_t)p.ncell;
    const double dt = p.dt, cl = p.clat;

    // ---- load slots: slot 0 is the own cell, the others cover the halo ring
    unsigned cell[NS];   // cell index; byte offsets below fit 32 bits (checked at creation)
    int lpos[NS];
    bool has[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int c = tid + s * NT;
        has[s] = c < PL;
        int hx, hy;
        halo_pos(has[s] ? c : 0, TX, TY, hx, hy);
        // fast tiles are periodic or keep their halo inside the grid
        int gi = i0 + hx - 2, gj = j0 + hy - 2;
        if (gi < 0) gi += p.nx;
        while (gi >= p.nx) gi -= p.nx;
        if (gj < 0) gj += p.ny;
        while (gj >= p.ny) gj -= p.ny;
        cell[s] = (unsigned)gj * (unsigned)p.nx + (unsigned)gi;
        lpos[s] = has[s] ? hy * HX + hx : PL;
    }

    // (unused slots load the own cell again and write the spare element)
    S v[NS][Q];
    S fv[STAGE == 1 ? Q : 1];   // stage C: fhat(t_n) of the own cell, loaded with the halo
    {
        const size_t nf = (size_t)p.ncell_f;
        [&]<int... qs>(std::integer_sequence<int, qs...>) {
            (([&] {
#pragma unroll
                 for (int s = 0; s < NS; s++)
                     v[s][qs] = *(const S *)((const char *)(X + (size_t)qs * n) +
                                             (unsigned)(sizeof(S) * (has[s] ? cell[s] : cell[0])));
                 if constexpr (STAGE == 1)
                     fv[qs] = *(const S *)((const char *)(F + (size_t)qs * nf) + (unsigned)(sizeof(S) * cell[0]));
             }()),
             ...);
        }(Seq{});
    }

    double a0[NS], ax[NS], ay[NS];
#pragma unroll
    for (int s = 0; s < NS; s++) a0[s] = ax[s] = ay[s] = 0.0;
    {
        [&]<int... qs>(std::integer_sequence<int, qs...>) {
            (([&] {
                 constexpr int EX = Lat::ex(qs), EY = Lat::ey(qs), SH = Lat::shell(qs);
#pragma unroll
                 for (int s = 0; s < NS; s++) {
                     const double d = (double)v[s][qs];
                     if (DELTA) {
                         a0[s] = __builtin_fma(p.wtab[SH][1], d, a0[s]);
                         if (EX) ax[s] = __builtin_fma(EX > 0 ? p.wtab[SH][EX] : -p.wtab[SH][-EX], d, ax[s]);
                         if (EY) ay[s] = __builtin_fma(EY > 0 ? p.wtab[SH][EY] : -p.wtab[SH][-EY], d, ay[s]);
                     } else {
                         a0[s] += d;
                         if (EX) ax[s] = __builtin_fma((double)EX, d, ax[s]);
                         if (EY) ay[s] = __builtin_fma((double)EY, d, ay[s]);
                     }
                 }
             }()),
             ...);
        }(Seq{});
    }

    // ---- pre-reconstruction variable B of every slot (eqs. f_bar_1_6 / fbp_5_12)
    EPolyS<S> eb[NS];
    S ccs[NS];
    EPoly ep_own{};
    double rho_own = 1.0;
    const long long ocell = (long long)j * p.nx + i;
    const double tau_o = (TF && valid) ? p.tau[ocell] : p.tau0;
#pragma unroll
    for (int s = 0; s < NS; s++) {
        double rho, drho, mxx, myy;
        phys_moments(p, DELTA, a0[s], ax[s], ay[s], rho, drho, mxx, myy);
        if (!has[s]) { rho = 1.0; drho = DELTA ? 0.0 : 1.0; mxx = myy = 0.0; }
        double cc, ce;
        if (!TF) {
            cc = p.uc.cc[STAGE];
            ce = p.uc.ce[STAGE];
        } else {
            const double tau = has[s] ? p.tau[cell[s]] : p.tau0;
            if (STAGE == 0) {
                const Stage0Coef c0 = stage0_coef(p.t2, tau, dt);
                cc = c0.cc;
                ce = c0.ce;
            } else {
                cc = (24.0 * tau - 5.0 * dt) / (24.0 * tau + 4.0 * dt);
                ce = 9.0 * dt / (24.0 * tau + 4.0 * dt);
            }
        }
        const EPoly e = epoly(rho, drho, mxx, myy, p.iRT, cl, DELTA);
        if (s == 0) { ep_own = e; rho_own = rho; }
        eb[s].set(e, ce);
        ccs[s] = (S)cc;
    }
    {
        // velocities q and opp(q) (e and -e) share the even part of E
        [&]<int... qs>(std::integer_sequence<int, qs...>) {
            (([&] {
                 constexpr int EX = Lat::ex(qs), EY = Lat::ey(qs), QO = Lat::opp(qs);
                 const S wqs = DELTA ? (S)1 : (S)p.wtab[Lat::shell(qs)][1];
                 if constexpr (QO == qs) {
#pragma unroll
                     for (int s = 0; s < NS; s++) {
                         const S e = eb[s].template eval<EX, EY>();
                         lds[qs * PS + lpos[s]] = fmaS(ccs[s], v[s][qs], DELTA ? e : wqs * e);
                     }
                 } else if constexpr (QO > qs) {
#pragma unroll
                     for (int s = 0; s < NS; s++) {
                         S ep, em;
                         eb[s].template eval_pair<EX, EY>(ep, em);
                         lds[qs * PS + lpos[s]] = fmaS(ccs[s], v[s][qs], DELTA ? ep : wqs * ep);
                         lds[QO * PS + lpos[s]] = fmaS(ccs[s], v[s][QO], DELTA ? em : wqs * em);
                     }
                 }
             }()),
             ...);
        }(Seq{});
    }
    (void)rho_own;

    // ---- own cell: the part of the output that does not depend on the faces
    const double c1 = TF ? (12.0 * tau_o - dt) / (12.0 * tau_o + 3.0 * dt) : p.uc.c1;
    const double e1 = TF ? 4.0 * dt / (12.0 * tau_o + 3.0 * dt) : p.uc.e1;
    S R0[Q];
    EPoly EO;   // equilibrium terms of the output (storage units), before the flux part is added
    if (STAGE == 0) {
        // T3S3: tilde f^+(t_n) = 5/4 fbar^{+,dt/6} - 1/4 fhat (eq. f_tilde_1_3);
        // T2S3: ftilde^+ = ((2 tau - dt) ftilde + 2 dt E) / (2 tau + dt)
        double kxd = p.uc.kx0, ked = p.uc.ke0;
        if (TF) {
            const Stage0Coef c0 = stage0_coef(p.t2, tau_o, dt);
            kxd = c0.kx;
            ked = c0.ke;
        }
        const S kx = (S)kxd;
#pragma unroll
        for (int q = 0; q < Q; q++) R0[q] = kx * v[0][q];
        const double k = ked - rounding_of<S>(kxd);
        EO = {ep_own.c0 * k, ep_own.c1x * k, ep_own.c1y * k, ep_own.c2xx * k, ep_own.c2xy * k, ep_own.c2yy * k};
    } else {
        // fhat(t_{n+1}) = a_f fhat + a_G tilde f(t') + a_En E^n + a_Ep E' + 4dt/7 L**
        // (eqs. fhp, collisionterm, feqIntD3rdHat2_DS, with 3 dt/7 L* taken
        // from the T2 update of step 2)
        double a_f = p.uc.a_f, a_En = p.uc.a_En, a_G = p.uc.a_G, a_Ep = p.uc.a_Ep;
        if (TF) {
            const double kw = 6.0 * dt / (6.0 * tau_o + dt);
            a_f = (4.0 - 6.0 * c1) / 7.0;
            a_En = -6.0 / 7.0 * e1;
            a_G = 9.0 / 7.0 - 0.75 * kw;
            a_Ep = 0.75 * kw;
        }
        const S sf = (S)a_f, sg = (S)a_G;
        double b0 = 0, bx = 0, by = 0;
        [&]<int... qs>(std::integer_sequence<int, qs...>) {
            (([&] {
                 constexpr int EX = Lat::ex(qs), EY = Lat::ey(qs), SH = Lat::shell(qs);
                 const S fq = fv[STAGE == 1 ? qs : 0];
                 const double d = (double)fq;
                 if (DELTA) {
                     b0 = __builtin_fma(p.wtab[SH][1], d, b0);
                     if (EX) bx = __builtin_fma(EX > 0 ? p.wtab[SH][EX] : -p.wtab[SH][-EX], d, bx);
                     if (EY) by = __builtin_fma(EY > 0 ? p.wtab[SH][EY] : -p.wtab[SH][-EY], d, by);
                 } else {
                     b0 += d;
                     if (EX) bx = __builtin_fma((double)EX, d, bx);
                     if (EY) by = __builtin_fma((double)EY, d, by);
                 }
                 R0[qs] = fmaS(sf, fq, sg * v[0][qs]);
                 // formed here, before the barrier: the loads of fhat then
                 // overlap the halo loads instead of waiting after the fill
                 asm volatile("" : "+v"(R0[qs]));
             }()),
             ...);
        }(Seq{});
        double rn, drn, mxn, myn;
        phys_moments(p, DELTA, b0, bx, by, rn, drn, mxn, myn);
        const EPoly en = epoly(rn, drn, mxn, myn, p.iRT, cl, DELTA);
        a_En -= rounding_of<S>(a_f);
        a_Ep -= rounding_of<S>(a_G);
        EO = {a_En * en.c0 + a_Ep * ep_own.c0, a_En * en.c1x + a_Ep * ep_own.c1x,
              a_En * en.c1y + a_Ep * ep_own.c1y, a_En * en.c2xx + a_Ep * ep_own.c2xx,
              a_En * en.c2xy + a_Ep * ep_own.c2xy, a_En * en.c2yy + a_Ep * ep_own.c2yy};
    }
    __syncthreads();
    if (!valid) return;   // no barrier below

    // ---- interface recovery weights (eq. recover2f) -------------------------
    double alpha[4], beta[4];
    if (TF) {
        const int im = i > 0 ? i - 1 : p.nx - 1, ip = i < p.nx - 1 ? i + 1 : 0;
        const int jm = j > 0 ? j - 1 : p.ny - 1, jp = j < p.ny - 1 ? j + 1 : 0;
        const double tb[4] = {0.5 * (tau_o + p.tau[(long long)j * p.nx + im]),
                              0.5 * (tau_o + p.tau[(long long)j * p.nx + ip]),
                              0.5 * (tau_o + p.tau[(long long)jm * p.nx + i]),
                              0.5 * (tau_o + p.tau[(long long)jp * p.nx + i])};
#pragma unroll
        for (int k = 0; k < 4; k++) {
            alpha[k] = 2.0 * tb[k] / (2.0 * tb[k] + h);
            beta[k] = h / (2.0 * tb[k] + h);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            alpha[k] = p.uc.alpha[STAGE];
            beta[k] = p.uc.beta[STAGE];
        }
    }
    // multiples m * (-clat/dx) (times alpha when it is the same on all faces)
    S kxm[4], kym[4], al[4];
    {
        const double fx = -cl * p.inv_dx * (TF ? 1.0 : alpha[0]);
        const double fy = -cl * p.inv_dy * (TF ? 1.0 : alpha[0]);
#pragma unroll
        for (int m = 0; m < 4; m++) {
            kxm[m] = (S)(m * fx);
            kym[m] = (S)(m * fy);
            al[m] = (S)alpha[m];
        }
    }

    // ---- interface values, moments, linear flux part -------------------------
    double mr[4] = {0, 0, 0, 0}, mx[4] = {0, 0, 0, 0}, my[4] = {0, 0, 0, 0};
    const S aLs = (S)(STAGE == 0 ? p.uc.aL0 : 4.0 * dt / 7.0);
    {
        const S *base = lds + (ly + 2) * HX + (lx + 2);
        [&]<int... qs>(std::integer_sequence<int, qs...>) {
            (fast_faces<Lat, S, DELTA, TF, qs, HX, PS>(p, base, coef + qs * 24, mr, mx, my, kxm, kym, al, aLs, R0[qs]),
             ...);
        }(Seq{});
    }

    // ---- equilibrium part of the recovered interface values: -(xi_x/dx)(beta_e E_e -
    //      beta_w E_w) - (xi_y/dy)(beta_n E_n - beta_s E_s), a cubic in the lattice vector
    EPoly ef[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        double rho, drho, mxx, myy;
        phys_moments(p, DELTA, mr[k], mx[k], my[k], rho, drho, mxx, myy);
        ef[k] = epoly(rho, drho, mxx, myy, p.iRT, cl, DELTA);
    }
    const double aL = STAGE == 0 ? p.uc.aL0 : 4.0 * dt / 7.0;
    const double kx = -p.inv_dx * cl * aL, ky = -p.inv_dy * cl * aL;
    const double A0 = beta[1] * ef[1].c0 - beta[0] * ef[0].c0, A1 = beta[1] * ef[1].c1x - beta[0] * ef[0].c1x,
                 A2 = beta[1] * ef[1].c1y - beta[0] * ef[0].c1y, A3 = beta[1] * ef[1].c2xx - beta[0] * ef[0].c2xx,
                 A4 = beta[1] * ef[1].c2xy - beta[0] * ef[0].c2xy, A5 = beta[1] * ef[1].c2yy - beta[0] * ef[0].c2yy;
    const double B0 = beta[3] * ef[3].c0 - beta[2] * ef[2].c0, B1 = beta[3] * ef[3].c1x - beta[2] * ef[2].c1x,
                 B2 = beta[3] * ef[3].c1y - beta[2] * ef[2].c1y, B3 = beta[3] * ef[3].c2xx - beta[2] * ef[2].c2xx,
                 B4 = beta[3] * ef[3].c2xy - beta[2] * ef[2].c2xy, B5 = beta[3] * ef[3].c2yy - beta[2] * ef[2].c2yy;
    // output = R0 + aL * La + [w_q] * M(e), M = EO + aL * (flux cubic)
    const S m0 = (S)EO.c0;
    const S m_x = (S)(EO.c1x + kx * A0), m_y = (S)(EO.c1y + ky * B0);
    const S m_xx = (S)(EO.c2xx + kx * A1), m_xy = (S)(EO.c2xy + kx * A2 + ky * B1), m_yy = (S)(EO.c2yy + ky * B2);
    const S m_xxx = (S)(kx * A3), m_xxy = (S)(kx * A4 + ky * B3), m_xyy = (S)(kx * A5 + ky * B4),
            m_yyy = (S)(ky * B5);
    const size_t no = (size_t)p.ncell_o;
    const unsigned oc = (unsigned)ocell;
    // M at e and -e (velocities q and opp(q)) from its even (m0 and quadratic)
    // and odd (linear and cubic) parts
    auto store = [&](int q, S M, S wq) {
        const S r = R0[q];
        *(S *)((char *)(out + (size_t)q * no) + (unsigned)(sizeof(S) * oc)) = DELTA ? r + M : fmaS(wq, M, r);
    };
    [&]<int... qs>(std::integer_sequence<int, qs...>) {
        (([&] {
             constexpr int EX = Lat::ex(qs), EY = Lat::ey(qs), QO = Lat::opp(qs);
             const S wq = DELTA ? (S)1 : (S)p.wtab[Lat::shell(qs)][1];
             if constexpr (QO == qs) {
                 store(qs, m0, wq);
             } else if constexpr (QO > qs) {
                 S ev = m0;
                 if (EX) ev = fmaS((S)(EX * EX), m_xx, ev);
                 if (EX && EY) ev = fmaS((S)(EX * EY), m_xy, ev);
                 if (EY) ev = fmaS((S)(EY * EY), m_yy, ev);
                 S od = (S)0;
                 bool first = true;
                 auto term = [&](S k, S m) {
                     od = first ? k * m : fmaS(k, m, od);
                     first = false;
                 };
                 if (EX) term((S)EX, m_x);
                 if (EY) term((S)EY, m_y);
                 if (EX) term((S)(EX * EX * EX), m_xxx);
                 if (EX && EY) term((S)(EX * EX * EY), m_xxy);
                 if (EX && EY) term((S)(EX * EY * EY), m_xyy);
                 if (EY) term((S)(EY * EY * EY), m_yyy);
                 store(qs, ev + od, wq);
                 store(QO, ev - od, wq);
             }
         }()),
         ...);
    }(Seq{});
    // non-finite flag: a non-finite value anywhere in the cell's neighbourhood
    // reaches every velocity through the moments, so the rest velocity's
    // output (the value stored above) is tested
    constexpr int QR = rest_velocity<Lat>();
    const S vr = DELTA ? R0[QR] + m0 : fmaS((S)p.wtab[Lat::shell(QR)][1], m0, R0[QR]);
    if (!__builtin_isfinite(vr)) *p.bad = 1;
}

// Waves per SIMD the register budget is cut for: two where the tile's LDS lets
// two blocks share a CU, else one (FP64 D2Q37: one block per CU, so the
// kernel may use the whole register file instead of spilling)
template <class Lat, class S, int TX, int TY>
constexpr int fast_waves_per_eu()
{
    return 2 * sizeof(S) * Lat::Q * ((TX + 4) * (TY + 4) + 1) <= 160 * 1024 ? 2 : 1;
}

template <class Lat, class S, bool DELTA, bool TF, int STAGE, int TX, int TY>
__global__ void __launch_bounds__(TX * TY)
    __attribute__((amdgpu_waves_per_eu(fast_waves_per_eu<Lat, S, TX, TY>())))
sweep_fast(const SweepParams p, const double h, const S *__restrict__ X, const S *__restrict__ F,
           S *__restrict__ out, const S *__restrict__ coef)
{
    int tx, ty;
    tile_of_block(p, tx, ty);
    if (!tile_is_fast(p, tx * TX, ty * TY, TX, TY)) return;
    fast_body<Lat, S, DELTA, TF, STAGE, TX, TY>(p, h, X, F, out, coef, tx, ty);
}

template <class Lat, class S, bool DELTA, bool TF, int STAGE, int TX, int TY>
__global__ void __launch_bounds__(TX * TY)
    __attribute__((amdgpu_waves_per_eu(fast_waves_per_eu<Lat, S, TX, TY>())))
sweep_fast_batched(const SweepParams *__restrict__ P, const StageIO *__restrict__ io,
                   const int4 *__restrict__ work)
{
    const int4 w = work[blockIdx.x];
    const SweepParams &p = P[w.x];
    const StageIO &a = io[w.x];
    fast_body<Lat, S, DELTA, TF, STAGE, TX, TY>(p, a.h, (const S *)a.X, (const S *)a.F, (S *)a.out,
                                               (const S *)a.coef, w.y, w.z);
}

// ---------------------------------------------------------------------------
// Host side: compiled tile shapes and dispatch.
// ---------------------------------------------------------------------------
template <class Lat, class S, bool DELTA, int TX, int TY>
static hipError_t fast_smem_t(size_t bytes)
{
    const void *fns[8] = {(const void *)sweep_fast<Lat, S, DELTA, false, 0, TX, TY>,
                          (const void *)sweep_fast<Lat, S, DELTA, false, 1, TX, TY>,
                          (const void *)sweep_fast<Lat, S, DELTA, true, 0, TX, TY>,
                          (const void *)sweep_fast<Lat, S, DELTA, true, 1, TX, TY>,
                          (const void *)sweep_fast_batched<Lat, S, DELTA, false, 0, TX, TY>,
                          (const void *)sweep_fast_batched<Lat, S, DELTA, false, 1, TX, TY>,
                          (const void *)sweep_fast_batched<Lat, S, DELTA, true, 0, TX, TY>,
                          (const void *)sweep_fast_batched<Lat, S, DELTA, true, 1, TX, TY>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class Lat, class S, bool DELTA, int TX, int TY>
static hipError_t fast_launch_t(int stage, const SweepParams &p, double h, const void *X, const void *F,
                                void *out, const void *coef, hipStream_t s)
{
    const dim3 grid(((p.nx + TX - 1) / TX) * ((p.ny + TY - 1) / TY));
    const size_t smem = sizeof(S) * Lat::Q * ((size_t)(TX + 4) * (TY + 4) + 1);
    const dim3 block(TX * TY);
    const S *x = (const S *)X, *f = (const S *)F, *c = (const S *)coef;
    S *o = (S *)out;
    if (p.tau_field) {
        if (stage == 0)
            hipLaunchKernelGGL((sweep_fast<Lat, S, DELTA, true, 0, TX, TY>), grid, block, smem, s, p, h, x, f, o, c);
        else
            hipLaunchKernelGGL((sweep_fast<Lat, S, DELTA, true, 1, TX, TY>), grid, block, smem, s, p, h, x, f, o, c);
    } else {
        if (stage == 0)
            hipLaunchKernelGGL((sweep_fast<Lat, S, DELTA, false, 0, TX, TY>), grid, block, smem, s, p, h, x, f, o, c);
        else
            hipLaunchKernelGGL((sweep_fast<Lat, S, DELTA, false, 1, TX, TY>), grid, block, smem, s, p, h, x, f, o, c);
    }
    return hipGetLastError();
}

template <class Lat, class S, bool DELTA, int TX, int TY>
static hipError_t fast_launch_batched_t(int stage, bool tf, const SweepParams *P, const StageIO *io,
                                        const int4 *work, int nwork, size_t smem, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    const dim3 grid(nwork), block(TX * TY);
    if (tf) {
        if (stage == 0)
            hipLaunchKernelGGL((sweep_fast_batched<Lat, S, DELTA, true, 0, TX, TY>), grid, block, smem, s, P, io, work);
        else
            hipLaunchKernelGGL((sweep_fast_batched<Lat, S, DELTA, true, 1, TX, TY>), grid, block, smem, s, P, io, work);
    } else {
        if (stage == 0)
            hipLaunchKernelGGL((sweep_fast_batched<Lat, S, DELTA, false, 0, TX, TY>), grid, block, smem, s, P, io, work);
        else
            hipLaunchKernelGGL((sweep_fast_batched<Lat, S, DELTA, false, 1, TX, TY>), grid, block, smem, s, P, io, work);
    }
    return hipGetLastError();
}

template <class Lat, class S, bool DELTA>
hipError_t fast_smem(int tx, int ty, size_t bytes)
{
#define DUGKS_FS(A, B) if (tx == A && ty == B) return fast_smem_t<Lat, S, DELTA, A, B>(bytes);
    DUGKS_FAST_SHAPES(DUGKS_FS)
#undef DUGKS_FS
    return hipErrorInvalidValue;
}

template <class Lat, class S, bool DELTA>
hipError_t fast_stage(int stage, const SweepParams &p, double h, const void *X, const void *F, void *out,
                      const void *coef, hipStream_t s)
{
#define DUGKS_FS(A, B) \
    if (p.tile_x == A && p.tile_y == B) return fast_launch_t<Lat, S, DELTA, A, B>(stage, p, h, X, F, out, coef, s);
    DUGKS_FAST_SHAPES(DUGKS_FS)
#undef DUGKS_FS
    return hipErrorInvalidValue;
}

template <class Lat, class S, bool DELTA>
hipError_t fast_stage_batched(int stage, int tx, int ty, bool tf, const SweepParams *P, const StageIO *io,
                              const int4 *work, int nwork, size_t smem, hipStream_t s)
{
#define DUGKS_FS(A, B) \
    if (tx == A && ty == B) return fast_launch_batched_t<Lat, S, DELTA, A, B>(stage, tf, P, io, work, nwork, smem, s);
    DUGKS_FAST_SHAPES(DUGKS_FS)
#undef DUGKS_FS
    return hipErrorInvalidValue;
}

// The build compiles this file once per lattice and precision (see sweep.hip).
#if defined(DK_LAT) && defined(DK_DELTA)
using InstLat = std::conditional_t<DK_LAT == 9, LatD2Q9, LatD2Q37>;
using InstS = std::conditional_t<DK_DELTA != 0, float, double>;
template hipError_t fast_smem<InstLat, InstS, DK_DELTA != 0>(int, int, size_t);
template hipError_t fast_stage<InstLat, InstS, DK_DELTA != 0>(int, const SweepParams &, double, const void *,
                                                               const void *, void *, const void *, hipStream_t);
template hipError_t fast_stage_batched<InstLat, InstS, DK_DELTA != 0>(int, int, int, bool, const SweepParams *,
                                                                       const StageIO *, const int4 *, int,
                                                                       size_t, hipStream_t);
#endif

}  // namespace dk
