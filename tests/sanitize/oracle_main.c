/* Test driver: runs the FP64 oracle's entry points (the ten-component step,
 * its observables and inversion, and the reduced state's step and recovery)
 * on a small ragged grid with a tabulated EOS, viscosity, bulk and the
 * regulator on, so that a build with -fsanitize=address,undefined checks the
 * oracle's memory accesses and arithmetic.  Prints "ok" and returns 0 when
 * every call returned normally and the results are finite. */
#include "../../oracle/kt_oracle.c"

#include <stdio.h>

#define NX 7
#define NY 6
#define NE 5
#define NC (NX * NY * NE)
#define NT 64

static int finite_all(const double *a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

int main(void)
{
    static double tp[NT], tc[NT], tt[NT];
    const double ln_e0 = log(1e-8), dln = 0.35, a_sb = 16.0 * M_PI * M_PI / 30.0;
    for (int i = 0; i < NT; ++i) {
        const double e = exp(ln_e0 + dln * i);
        tc[i] = 1.0 / 3.0 - 0.05 * exp(-0.5 * log(e) * log(e) / 4.0);
        tp[i] = tc[i] * e;
        tt[i] = pow(e / a_sb, 0.25);
    }
    const ora_eos eos = {0, a_sb, NT, ln_e0, dln, tp, tc, tt};
    ora_params P;
    memset(&P, 0, sizeof(P));
    P.nx = NX; P.ny = NY; P.neta = NE;
    P.dx = 0.3; P.dy = 0.35; P.deta = 0.2; P.dtau = 0.01;
    P.cartesian = 0; P.periodic[2] = 1;
    P.theta = 1.4; P.eta_s = 0.2; P.zeta_coef = 0.1; P.taupipi = 10.0 / 7.0;
    P.regulate = 1; P.xi0 = 0.1; P.rho_max = 1.0; P.e_floor = 1e-6;
    P.newton_tol = 1e-12; P.newton_max = 50; P.regulate_bulk = 1; P.m2_delta = 1e-3;
    P.floor_resets_q = 1; P.zeta_model = 0; P.zeta_tc = 1.0;

    static double e0[NC], u0[4 * NC], pi0[10 * NC], Pi0[NC], q[NQ * NC];
    const double tau0 = 0.7;
    for (int c = 0; c < NC; ++c) {
        const int i = c % NX, j = (c / NX) % NY, k = c / (NX * NY);
        e0[c] = 5.0 + 3.0 * sin(0.9 * i + 0.3 * k) * cos(0.7 * j);
        if (i == 0 && j == 0) e0[c] = 1e-7;       /* one cell below the floor */
        const double ux = 0.3 * sin(0.5 * j + k), uy = 0.2 * cos(0.4 * i), ue = 0.1 * sin(0.6 * k) / tau0;
        u0[4 * c + 1] = ux; u0[4 * c + 2] = uy; u0[4 * c + 3] = ue;
        u0[4 * c] = sqrt(1.0 + ux * ux + uy * uy + tau0 * tau0 * ue * ue);
        Pi0[c] = -0.01 * e0[c];
    }
    ora_tmunu(&P, &eos, tau0, NC, e0, u0, pi0, Pi0, q);

    static double e[NC], u[4 * NC], up[4 * NC], obs[64], rq[NQ * NC];
    ora_stats st;
    memset(&st, 0, sizeof(st));
    ora_init(&P, &eos, tau0, q, e, u, up);
    double tau = tau0;
    if (ora_step(&P, &eos, &tau, q, e, u, up, 3, &st) != 0) return 2;
    ora_observables(&P, &eos, tau, q, e, u, obs);
    ora_rhs(&P, &eos, tau, q, e, u, up, rq);
    static double e2[NC], u2[4 * NC];
    static int32_t it[NC], fl[NC];
    ora_recover(&P, &eos, tau, NC, q, NULL, e2, u2, it, fl);
    if (!finite_all(q, NQ * NC) || !finite_all(e, NC) || !finite_all(u, 4 * NC) || !finite_all(rq, NQ * NC)
        || !finite_all(e2, NC))
        return 3;

    /* reduced state from the same initial data */
    static double r[NR * NC], er[NC], u3[3 * NC], up3[3 * NC], qf[NQ * NC], uf[4 * NC];
    ora_tmunu(&P, &eos, tau0, NC, e0, u0, pi0, Pi0, q);
    for (int c = 0; c < NC; ++c)
        for (int m = 0; m < NR; ++m) r[NR * c + m] = q[NQ * c + RED_IDX[m]];
    ora_init_reduced(&P, &eos, tau0, r, er, u3, up3);
    double taur = tau0, tau_prev = tau0;
    int64_t fp[2] = {0, 0};
    memset(&st, 0, sizeof(st));
    if (ora_step_reduced(&P, &eos, &taur, &tau_prev, r, er, u3, up3, 3, &st, fp) != 0) return 4;
    ora_expand(&P, taur, NC, r, u3, qf, uf);
    static double er2[NC], ur2[4 * NC];
    static int32_t itr[NC], ps[NC], flr[NC];
    ora_recover_reduced(&P, &eos, taur, NC, r, er2, ur2, itr, ps, flr);
    if (!finite_all(r, NR * NC) || !finite_all(er, NC) || !finite_all(qf, NQ * NC) || !finite_all(er2, NC))
        return 5;
    printf("ok %.6g %.6g %lld\n", tau, taur, (long long)fp[0]);
    return 0;
}
