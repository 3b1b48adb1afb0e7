/*
 * kt_oracle.c -- plain, slow FP64 CPU reference for one Kurganov-Tadmor /
 * Heun step of (3+1)d second-order viscous hydrodynamics in Milne
 * coordinates (tau, x, y, eta_s), following Bazow, Heinz & Strickland,
 * "Massively parallel simulations of relativistic fluid dynamics on graphics
 * processing units with CUDA" (arXiv:1608.06577).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * Style: every quantity is written from its definition in the paper, with
 * explicit loops, 4x4 tensors and generic contractions with the metric
 * g_{mu nu} = diag(1,-1,-1,-tau^2) and the two Milne Christoffel symbols
 * (Sec. 2.4).  Cell data are kept as arrays of structures.  No blocking, no
 * fusion, no reuse of faces between cells: each cell recomputes the two
 * faces it needs in every direction, as Alg. 3 does.
 *
 * Readings of the paper taken where it is silent, garbled or inconsistent
 * (the same readings are used by the HIP path):
 *   - Face primitives for the local speed and the flux come from inverting
 *     the reconstructed q^+ and q^- (Sec. 3.1, last paragraph; Alg. 3).
 *   - Source vector J (Sec. 3.1) = (S_c + G_c, S_pi + G_pi): the conserved
 *     components get no q*div(v) term (their flux form, Sec. 2.4 energy and
 *     momentum equations, has none); S_pi and S_Pi carry it (App. B).
 *   - T^{ij} = v^i T^{tau j} - P g^{ij} - v^i pi^{tau j} + pi^{ij}  (Sec. 2.4:
 *     the last pi^{tau i} of Eq. Tij must read pi^{tau j}).
 *   - App. B, S_c^x: the third derivative is d/deta (as in the momentum
 *     equation of Sec. 2.4), not d/dy.
 *   - G_pi is computed from its definition u^a Gamma^mu_{ab} pi^{b nu} + (mu<->nu)
 *     (Sec. 2.4); App. B's factor 2 in G_pi^{tau x}, G_pi^{tau y} does not follow.
 *   - In App. A the operator written D in the shear components is the
 *     convective derivative d of the contravariant components.
 *   - Vorticity sign: omega^{mu nu} = (nabla^mu u^nu - nabla^nu u^mu)/2 and the
 *     term +2 tau_pi pi^<mu_l omega^nu>l of the main text (Sec. 2.1/2.2).
 *   - minmod uses sgn(0) = 0 (Sec. 3.1).
 *   - Stage 1 is evaluated at tau^n; the recovery of q*, stage 2 and the final
 *     recovery at tau^{n+1} (Sec. 4.3).
 *   - Regulator (Sec. 3.2, Eq. rho): sqrt(e^2 + 3 P^2) with P = P0 + Pi, the
 *     shorthand of Sec. 2.4 that Eq. rho prints; the second and third ratios
 *     use absolute values; the third is the largest |pi^{lambda mu} u_mu|
 *     over lambda in an orthonormal frame (the eta component multiplied by
 *     tau); the factor is 1 when rho = 0.  pi^{mu nu} is rescaled, and Pi too
 *     when regulate_bulk is set.
 *   - Recovery guards (Sec. 3.2 leaves them open), see recover() below.
 *   - Transport coefficients (Sec. 2.2) with eta/s fixed and
 *     zeta/s = zeta_coef (1/3 - c_s^2): 1/tau_pi = T / (5 eta/s),
 *     1/tau_Pi = 15 (1/3 - c_s^2) T / zeta_coef.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 15           /* T^{tau mu} (4), pi^{mu nu} (10), Pi (1): Sec. 3.1 */

/* ------------------------------------------------------------------ */
/* Public parameter structures (mirrored by ctypes in oracle/__init__.py) */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t nx, ny, neta;
    double dx, dy, deta;
    double dtau;
    int32_t cartesian;        /* 0: Milne (tau,x,y,eta_s); 1: Cartesian (t,x,y,z) */
    int32_t periodic[3];      /* per axis: 0 copy (outflow) ghosts, 1 periodic */
    double theta;             /* generalized minmod parameter, 1..2 */
    double eta_s;             /* eta/s; 0 means ideal (pi not evolved) */
    double zeta_coef;         /* zeta/s = zeta_coef (1/3 - c_s^2); 0: Pi not evolved */
    double taupipi;           /* tau_pipi / tau_pi */
    int32_t regulate;
    double xi0, rho_max;
    double e_floor;
    double newton_tol;
    int32_t newton_max;
    int32_t regulate_bulk;    /* 1: the regulator factor also rescales Pi */
    double m2_delta;          /* M^2 clamp margin: M2max = (1 - m2_delta) W min(E - e_floor, W) */
    int32_t floor_resets_q;   /* 1: a floored cell's state q is reset to (e_floor,0,0,0; 0; 0) */
    int32_t zeta_model;       /* 0: zeta/s = zeta_coef (1/3 - c_s^2); 1: zeta_coef times the
                               * parametrization of Sec. 2.2 (Eq. zetas) at x = T / zeta_tc */
    double zeta_tc;           /* T_c of zeta_model 1, in the EOS's temperature unit */
} ora_params;

/* zeta/s of Sec. 2.2 (Eq. zetas, T_c = 200 MeV there), x = T / T_c: a
 * quadratic around T_c joined to exponential tails towards the QGP (above)
 * and hadron-gas (below) values.  The printed range of the quadratic branch
 * is garbled; it is read as 0.995 <= x <= 1.05, between the other two. */
double ora_zeta_over_s_paper(double x)
{
    if (x > 1.05)
        return 0.9 * exp(-(x - 1.0) / 0.025) + 0.25 * exp(-(x - 1.0) / 0.13) + 0.001;
    if (x < 0.995)
        return 0.9 * exp((x - 1.0) / 0.0025) + 0.22 * exp((x - 1.0) / 0.022) + 0.03;
    return -13.45 + 27.55 * x - 13.77 * x * x;
}

typedef struct {
    int32_t conformal;        /* 1: p = e/3, T = (e/a)^{1/4} */
    double a_sb;
    int32_t n;                /* table nodes */
    double ln_e0, dln;
    const double *p, *cs2, *T;
} ora_eos;

typedef struct {   /* cell recoveries only */
    int64_t newton_iters, n_recover, n_floor, n_clamp, n_fallback;
} ora_stats;

/* recovery flags */
#define FL_FLOOR 1
#define FL_CLAMP 2
#define FL_FALLBACK 4

/* ------------------------------------------------------------------ */
/* Geometry (Sec. 2.4)                                                */
/* ------------------------------------------------------------------ */

static void metric(double tau, int cart, double glo[4], double ghi[4])
{
    glo[0] = 1.0; glo[1] = -1.0; glo[2] = -1.0;
    glo[3] = cart ? -1.0 : -tau * tau;
    for (int m = 0; m < 4; ++m) ghi[m] = 1.0 / glo[m];
}

/* Gamma^mu_{a b}: in Milne coordinates the only nonzero symbols are
 * Gamma^eta_{tau eta} = Gamma^eta_{eta tau} = 1/tau and Gamma^tau_{eta eta} = tau. */
static double christoffel(int mu, int a, int b, double tau, int cart)
{
    if (cart) return 0.0;
    if (mu == 3 && ((a == 0 && b == 3) || (a == 3 && b == 0))) return 1.0 / tau;
    if (mu == 0 && a == 3 && b == 3) return tau;
    return 0.0;
}

static const int PI_IDX[4][4] = {{4, 5, 6, 7}, {5, 8, 9, 10}, {6, 9, 11, 12}, {7, 10, 12, 13}};

static void pi_tensor(const double *q, double pi[4][4])
{
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) pi[m][n] = q[PI_IDX[m][n]];
}

/* ------------------------------------------------------------------ */
/* Equation of state                                                   */
/* ------------------------------------------------------------------ */

/* Table on ln-uniform nodes e_i = exp(ln_e0 + i dln): between the two nodes
 * bracketing e, p/e, T/e^{1/4} and c_s^2 are interpolated linearly in ln e
 * (exact for p proportional to e and T to e^{1/4}).  Outside the table the
 * ratios p/e and T/e^{1/4} and c_s^2 of the nearest end node are kept. */
static void eos_eval(const ora_eos *eos, double e, double *p, double *cs2, double *T)
{
    if (eos->conformal) {
        *p = e / 3.0;
        *cs2 = 1.0 / 3.0;
        *T = e > 0.0 ? sqrt(sqrt(e / eos->a_sb)) : 0.0;
        return;
    }
    const int n = eos->n;
    double x = (log(e) - eos->ln_e0) / eos->dln;
    int i;
    double t;
    if (!(x >= 0.0)) { i = 0; t = 0.0; }
    else if (x >= (double)(n - 1)) { i = n - 2; t = 1.0; }
    else { i = (int)floor(x); if (i > n - 2) i = n - 2; t = x - (double)i; }
    double e0 = exp(eos->ln_e0 + eos->dln * (double)i);
    double e1 = exp(eos->ln_e0 + eos->dln * (double)(i + 1));
    double r0 = eos->p[i] / e0, r1 = eos->p[i + 1] / e1;
    double s0 = eos->T[i] / sqrt(sqrt(e0)), s1 = eos->T[i + 1] / sqrt(sqrt(e1));
    *p = (r0 + t * (r1 - r0)) * e;
    *T = (s0 + t * (s1 - s0)) * sqrt(sqrt(e));
    *cs2 = eos->cs2[i] + t * (eos->cs2[i + 1] - eos->cs2[i]);
}

static double eos_p(const ora_eos *eos, double e)
{
    double p, c, T;
    eos_eval(eos, e, &p, &c, &T);
    return p;
}

/* ------------------------------------------------------------------ */
/* Conserved variables from primitives: Sec. 2.4, Eqs. Ttt, Tti        */
/* ------------------------------------------------------------------ */

static void tmunu_from_primitives(const ora_params *P, const ora_eos *eos, double tau,
                                  double e, const double u[4], const double pi10[10],
                                  double Pi, double q[NQ])
{
    double glo[4], ghi[4];
    metric(tau, P->cartesian, glo, ghi);
    double Pcal = eos_p(eos, e) + Pi;                 /* script P = P0 + Pi */
    double pi[4][4];
    double qq[NQ] = {0};
    for (int c = 0; c < 10; ++c) qq[4 + c] = pi10[c];
    qq[14] = Pi;
    pi_tensor(qq, pi);
    for (int nu = 0; nu < 4; ++nu)   /* T^{tau nu} = (e+P) u^tau u^nu - P g^{tau nu} + pi^{tau nu} */
        q[nu] = (e + Pcal) * u[0] * u[nu] - Pcal * (nu == 0 ? ghi[0] : 0.0) + pi[0][nu];
    for (int c = 4; c < NQ; ++c) q[c] = qq[c];
}

/* ------------------------------------------------------------------ */
/* Recovery of (e, u^mu) from T^{tau mu}, pi^{tau mu}, Pi (Sec. 2.4,   */
/* Eqs. eInferred, utInferred, uiInferred; Newton-Raphson, Sec. 3.2)   */
/* ------------------------------------------------------------------ */

/* Guards (the paper leaves them open; the HIP path applies the same):
 *  - E = T^tt - pi^tt not above e_floor (or not a number): e = e_floor, u = (1,0,0,0).
 *  - W = E + p(e_floor) + Pi not positive: the same floor state.
 *  - M^2 above M2max = (1 - m2_delta) W min(E - e_floor, W): M is rescaled to M2max.
 *    This keeps the root of f inside (e_floor, E] and e + P > 0.
 *  - Conformal EOS without bulk: closed form e = sqrt(4E^2 - 3M^2) - E.
 *  - Otherwise Newton on f(e) = e - E + M^2/(E + P(e)), f' = 1 - M^2 c_s^2/(E+P)^2,
 *    iterates clamped to [e_floor, E], started from the conformal closed form;
 *    once |f| <= tol E, one more iteration is taken and the loop stops.
 *  - No convergence within newton_max iterations: bisection on [e_floor, E]. */
static int recover_from(const ora_params *P, const ora_eos *eos, double tau, const double q[NQ],
                        double e_start, double *e_out, double u_out[4], int *iters)
{
    double glo[4], ghi[4];
    metric(tau, P->cartesian, glo, ghi);
    const int bulk = P->zeta_coef > 0.0;
    const double ef = P->e_floor;
    double E = q[0] - q[4];
    double M[4] = {0.0, q[1] - q[5], q[2] - q[6], q[3] - q[7]};
    double Pi = bulk ? q[14] : 0.0;
    int flags = 0;
    *iters = 0;

    double W = E + eos_p(eos, ef) + Pi;
    double M2 = 0.0;
    for (int i = 1; i < 4; ++i) M2 += -glo[i] * M[i] * M[i];   /* M^2 = Mx^2 + My^2 + tau^2 Meta^2 */
    if (!(E > ef) || !(W > 0.0) || !(M2 == M2) || !(M2 < INFINITY)) {
        *e_out = ef;
        u_out[0] = 1.0; u_out[1] = u_out[2] = u_out[3] = 0.0;
        return FL_FLOOR;
    }
    double M2max = (1.0 - P->m2_delta) * W * fmin(E - ef, W);
    if (M2 > M2max) {
        double s = sqrt(M2max / M2);
        for (int i = 1; i < 4; ++i) M[i] *= s;
        M2 = M2max;
        flags |= FL_CLAMP;
    }
    double e;
    double econf = sqrt(4.0 * E * E - 3.0 * M2) - E;
    if (eos->conformal && !bulk) {
        e = fmax(econf, ef);
    } else {
        e = fmin(fmax(e_start > 0.0 ? e_start : econf, ef), E);
        int done = 0, n = 0;
        while (n < P->newton_max) {
            double p, cs2, T;
            eos_eval(eos, e, &p, &cs2, &T);
            double A = E + p + Pi;
            double f = e - E + M2 / A;
            double df = 1.0 - M2 * cs2 / (A * A);
            int conv = fabs(f) <= P->newton_tol * E;
            e = fmin(fmax(e - f / df, ef), E);
            ++n;
            if (conv) { done = 1; break; }
        }
        *iters = n;
        if (!done) {
            double lo = ef, hi = E;
            for (int k = 0; k < 200; ++k) {
                double mid = 0.5 * (lo + hi);
                double f = mid - E + M2 / (E + eos_p(eos, mid) + Pi);
                e = mid;
                if (fabs(f) <= P->newton_tol * E || hi - lo <= 4e-16 * hi) break;
                if (f < 0.0) lo = mid; else hi = mid;
            }
            flags |= FL_FALLBACK;
        }
    }
    double Pcal = eos_p(eos, e) + Pi;
    double ut = sqrt((E + Pcal) / (e + Pcal));
    u_out[0] = ut;
    for (int i = 1; i < 4; ++i) u_out[i] = M[i] / ((e + Pcal) * ut);
    *e_out = e;
    return flags;
}

/* the same, started from the conformal closed form */
static int recover(const ora_params *P, const ora_eos *eos, double tau, const double q[NQ],
                   double *e_out, double u_out[4], int *iters)
{
    return recover_from(P, eos, tau, q, -1.0, e_out, u_out, iters);
}

/* ------------------------------------------------------------------ */
/* Regulator of the shear stress (Sec. 3.2, Eqs. regPimunu, rho)       */
/* ------------------------------------------------------------------ */

static double regulate_cell(const ora_params *P, const ora_eos *eos, double tau, double q[NQ],
                            double e, const double u[4])
{
    if (!P->regulate || !(P->eta_s > 0.0)) return 1.0;
    double glo[4], ghi[4];
    metric(tau, P->cartesian, glo, ghi);
    double pi[4][4];
    pi_tensor(q, pi);
    double Pi = P->zeta_coef > 0.0 ? q[14] : 0.0;
    double Pcal = eos_p(eos, e) + Pi;   /* script P = P0 + Pi (Sec. 2.4) */
    double B[4][4];   /* Pi^{mu nu} = Pi Delta^{mu nu} + pi^{mu nu} */
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n)
            B[m][n] = Pi * ((m == n ? ghi[m] : 0.0) - u[m] * u[n]) + pi[m][n];
    /* |Pi^{mu nu}|: the Frobenius norm of its components in the fluid rest
       frame.  For B transverse to u it is sqrt(B^{mu nu} B_{mu nu}), the paper's
       norm; the evolved pi is transverse only to truncation error, and there
       B:B can vanish or be negative.  The rest-frame components: B in the
       orthonormal frame of the coordinates (the eta row and column times
       sqrt(-g_33)), then the pure boost L with L u = (1, 0, 0, 0):
       L^0_0 = gamma, L^0_i = L^i_0 = -u^i, L^i_j = delta_ij + u^i u^j / (1 + gamma). */
    double sc[4], ut[4];
    for (int m = 0; m < 4; ++m) {
        sc[m] = sqrt(fabs(glo[m]));
        ut[m] = u[m] * sc[m];
    }
    double L[4][4];
    L[0][0] = ut[0];
    for (int i = 1; i < 4; ++i) {
        L[0][i] = L[i][0] = -ut[i];
        for (int j = 1; j < 4; ++j) L[i][j] = (i == j ? 1.0 : 0.0) + ut[i] * ut[j] / (1.0 + ut[0]);
    }
    double BB = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            double s = 0.0;
            for (int m = 0; m < 4; ++m)
                for (int n = 0; n < 4; ++n) s += L[a][m] * L[b][n] * B[m][n] * sc[m] * sc[n];
            BB += s * s;
        }
    double nB = sqrt(fmax(BB, 0.0));
    double rho = nB / (P->rho_max * sqrt(e * e + 3.0 * Pcal * Pcal));
    if (nB > 0.0) {
        double tr = 0.0;
        for (int m = 0; m < 4; ++m) tr += glo[m] * pi[m][m];
        double r2 = fabs(tr) / (P->xi0 * P->rho_max * nB);
        double r3 = 0.0;
        for (int l = 0; l < 4; ++l) {
            double w = 0.0;
            for (int m = 0; m < 4; ++m) w += pi[l][m] * glo[m] * u[m];
            w = fabs(w) * sqrt(fabs(glo[l]));
            if (w > r3) r3 = w;
        }
        r3 /= P->xi0 * P->rho_max * nB;
        if (r2 > rho) rho = r2;
        if (r3 > rho) rho = r3;
    }
    double fac = rho > 0.0 ? tanh(rho) / rho : 1.0;
    for (int c = 4; c < 14; ++c) q[c] *= fac;
    if (P->regulate_bulk) q[14] *= fac;
    return fac;
}

/* ------------------------------------------------------------------ */
/* Kinematic quantities: theta, sigma, omega, Du (Sec. 2.4, App. A)    */
/* ------------------------------------------------------------------ */

typedef struct {
    double theta;
    double sigma[4][4];     /* sigma^{mu nu} */
    double omega[4][4];     /* omega^{mu nu} = (nabla^mu u^nu - nabla^nu u^mu)/2 */
    double Du_lo[4];        /* D u_mu */
    double Delta[4][4];     /* Delta^{mu nu} */
} kin_t;

/* du[a][m] = partial_a u^m.  Covariant derivative u^m_{;a} = partial_a u^m + Gamma^m_{ab} u^b. */
static void kinematics(double tau, int cart, const double u[4], const double du[4][4], kin_t *K)
{
    double glo[4], ghi[4];
    metric(tau, cart, glo, ghi);
    double cov[4][4];
    for (int a = 0; a < 4; ++a)
        for (int m = 0; m < 4; ++m) {
            double s = du[a][m];
            for (int b = 0; b < 4; ++b) s += christoffel(m, a, b, tau, cart) * u[b];
            cov[a][m] = s;
        }
    double th = 0.0;
    for (int m = 0; m < 4; ++m) th += cov[m][m];
    K->theta = th;
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) K->Delta[m][n] = (m == n ? ghi[m] : 0.0) - u[m] * u[n];
    double nab[4][4];   /* nabla^m u^n = Delta^{m a} u^n_{;a} */
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            double s = 0.0;
            for (int a = 0; a < 4; ++a) s += K->Delta[m][a] * cov[a][n];
            nab[m][n] = s;
        }
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            K->sigma[m][n] = 0.5 * (nab[m][n] + nab[n][m]) - th / 3.0 * K->Delta[m][n];
            K->omega[m][n] = 0.5 * (nab[m][n] - nab[n][m]);
        }
    for (int m = 0; m < 4; ++m) {
        double s = 0.0;
        for (int a = 0; a < 4; ++a) s += u[a] * cov[a][m];   /* D u^m */
        K->Du_lo[m] = glo[m] * s;
    }
}

/* Second-order terms I_1..I_4 (Sec. 2.4, Eqs. I1-I4), all 16 components. */
static void second_order_terms(double tau, int cart, const double u[4], const double pi[4][4],
                               const kin_t *K, double I1[4][4], double I2[4][4],
                               double I3[4][4], double I4[4][4], double *pi_sigma)
{
    double glo[4], ghi[4];
    metric(tau, cart, glo, ghi);
    double ps = 0.0;   /* pi^a_b sigma^b_a = pi^{mu nu} sigma_{mu nu} */
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) ps += pi[a][b] * glo[b] * K->sigma[b][a] * glo[a];
    *pi_sigma = ps;
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            double s1 = 0.0, s3 = 0.0, s4 = 0.0;
            for (int l = 0; l < 4; ++l) {
                s1 += (pi[l][m] * u[n] + pi[l][n] * u[m]) * K->Du_lo[l];
                /* omega^n_l = omega^{n k} g_{k l} */
                s3 += pi[m][l] * K->omega[n][l] * glo[l] + pi[n][l] * K->omega[m][l] * glo[l];
                /* (1/2) g_{l k} (pi^{m k} sigma^{n l} + pi^{n k} sigma^{m l}), g diagonal */
                s4 += 0.5 * glo[l] * (pi[m][l] * K->sigma[n][l] + pi[n][l] * K->sigma[m][l]);
            }
            I1[m][n] = s1;
            I2[m][n] = K->theta * pi[m][n];
            I3[m][n] = s3;
            I4[m][n] = s4 - K->Delta[m][n] * ps / 3.0;
        }
}

/* ------------------------------------------------------------------ */
/* Grid access with boundary conditions (Sec. 4.1): copy ghosts are    */
/* equivalent to clamping the index to the physical range.             */
/* ------------------------------------------------------------------ */

typedef struct {
    const ora_params *P;
    const ora_eos *eos;
    double tau;
    const double *q;    /* [cell][15] */
    const double *e;    /* [cell] */
    const double *u;    /* [cell][4] */
    const double *up;   /* [cell][4] previous time level */
    ora_stats *st;
} ctx_t;

static int64_t cell_index(const ora_params *P, int i, int j, int k)
{
    return ((int64_t)k * P->ny + j) * P->nx + i;
}

static int wrap_axis(int v, int n, int periodic)
{
    if (periodic) { v %= n; if (v < 0) v += n; return v; }
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

static int64_t neighbour(const ora_params *P, int i, int j, int k, int d, int off)
{
    int c[3] = {i, j, k};
    int n[3] = {P->nx, P->ny, P->neta};
    c[d] = wrap_axis(c[d] + off, n[d], P->periodic[d]);
    return cell_index(P, c[0], c[1], c[2]);
}

/* ------------------------------------------------------------------ */
/* KT numerical flux (Sec. 3.1, Eqs. Hflux, ax, half-cell extrapolation */
/* and the generalized minmod limiter; Alg. 3)                         */
/* ------------------------------------------------------------------ */

static double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

static double minmod2(double x, double y)
{
    return (sgn(x) + sgn(y)) * fmin(fabs(x), fabs(y)) / 2.0;
}

static double minmod3(double x, double y, double z) { return minmod2(x, minmod2(y, z)); }

/* slope (q_d)_c along axis d at cell c, from the cells c-1, c, c+1 */
static double limited_slope(double qm, double q0, double qp, double theta, double h)
{
    return minmod3(theta * (q0 - qm) / h, (qp - qm) / (2.0 * h), theta * (qp - q0) / h);
}

/* flux through the face of cell (i,j,k) on side s (+1: i+1/2, -1: i-1/2) along axis d */
static void face_flux(ctx_t *C, int i, int j, int k, int d, int s, double H[NQ])
{
    const ora_params *P = C->P;
    const double h = d == 0 ? P->dx : (d == 1 ? P->dy : P->deta);
    const int oL = s > 0 ? 0 : -1;   /* left cell of the face relative to (i,j,k) */
    const double *qLm = C->q + NQ * neighbour(P, i, j, k, d, oL - 1);
    const double *qL  = C->q + NQ * neighbour(P, i, j, k, d, oL);
    const double *qR  = C->q + NQ * neighbour(P, i, j, k, d, oL + 1);
    const double *qRp = C->q + NQ * neighbour(P, i, j, k, d, oL + 2);
    double qminus[NQ], qplus[NQ];
    for (int n = 0; n < NQ; ++n) {
        double sL = limited_slope(qLm[n], qL[n], qR[n], P->theta, h);
        double sR = limited_slope(qL[n], qR[n], qRp[n], P->theta, h);
        qminus[n] = qL[n] + 0.5 * h * sL;    /* q^- : left side of the interface */
        qplus[n]  = qR[n] - 0.5 * h * sR;    /* q^+ : right side of the interface */
    }
    double em, ep, um[4], upl[4];
    int itm, itp;
    recover(P, C->eos, C->tau, qminus, &em, um, &itm);
    recover(P, C->eos, C->tau, qplus, &ep, upl, &itp);
    double vm = um[d + 1] / um[0];
    double vp = upl[d + 1] / upl[0];
    double a = fmax(fabs(vm), fabs(vp));
    for (int n = 0; n < NQ; ++n)
        H[n] = (vp * qplus[n] + vm * qminus[n]) / 2.0 - a * (qplus[n] - qminus[n]) / 2.0;
}

/* ------------------------------------------------------------------ */
/* Source terms J = (S_c + G_c, S_pi + G_pi, S_Pi)  (Sec. 3.1, App. B)  */
/* ------------------------------------------------------------------ */

/* A^{i nu} = T^{i nu} - v^i T^{tau nu} written with Eqs. Ttt-Tij:
 * A^{i nu} = -P (g^{i nu} - v^i g^{tau nu}) + pi^{i nu} - v^i pi^{tau nu}  (i spatial). */
static void nonadvective_flux(const ora_params *P, const ora_eos *eos, double tau,
                              const double *q, double e, const double *u, double A[4][4])
{
    double glo[4], ghi[4];
    metric(tau, P->cartesian, glo, ghi);
    double pi[4][4];
    pi_tensor(q, pi);
    if (!(P->eta_s > 0.0))
        for (int m = 0; m < 4; ++m) for (int n = 0; n < 4; ++n) pi[m][n] = 0.0;
    double Pcal = eos_p(eos, e) + (P->zeta_coef > 0.0 ? q[14] : 0.0);
    double v[4] = {1.0, u[1] / u[0], u[2] / u[0], u[3] / u[0]};
    for (int i = 0; i < 4; ++i)
        for (int n = 0; n < 4; ++n) {
            if (i == 0) { A[i][n] = 0.0; continue; }
            double gin = (i == n) ? ghi[i] : 0.0;
            double gtn = (n == 0) ? ghi[0] : 0.0;
            A[i][n] = -Pcal * (gin - v[i] * gtn) + pi[i][n] - v[i] * pi[0][n];
        }
}

static void cell_sources(ctx_t *C, int i, int j, int k, double J[NQ])
{
    const ora_params *P = C->P;
    const double tau = C->tau;
    const int cart = P->cartesian;
    const int shear = P->eta_s > 0.0, bulk = P->zeta_coef > 0.0;
    double glo[4], ghi[4];
    metric(tau, cart, glo, ghi);
    const int64_t c0 = cell_index(P, i, j, k);
    const double *q = C->q + NQ * c0;
    const double *u = C->u + 4 * c0;
    const double *up = C->up + 4 * c0;
    const double e = C->e[c0];
    const double hs[3] = {P->dx, P->dy, P->deta};
    double p0, cs2, T;
    eos_eval(C->eos, e, &p0, &cs2, &T);
    const double Pi = bulk ? q[14] : 0.0;
    double pi[4][4];
    pi_tensor(q, pi);
    if (!shear)
        for (int m = 0; m < 4; ++m) for (int n = 0; n < 4; ++n) pi[m][n] = 0.0;
    double v[4] = {1.0, u[1] / u[0], u[2] / u[0], u[3] / u[0]};

    /* derivatives: backward difference in tau, central differences in space (Sec. 3.1) */
    double du[4][4];
    double divv = 0.0;
    double Sc[4] = {0, 0, 0, 0};
    for (int m = 0; m < 4; ++m) du[0][m] = (u[m] - up[m]) / P->dtau;
    for (int d = 0; d < 3; ++d) {
        int64_t cp = neighbour(P, i, j, k, d, +1), cm = neighbour(P, i, j, k, d, -1);
        const double *upl = C->u + 4 * cp, *umi = C->u + 4 * cm;
        for (int m = 0; m < 4; ++m) du[d + 1][m] = (upl[m] - umi[m]) / (2.0 * hs[d]);
        divv += (upl[d + 1] / upl[0] - umi[d + 1] / umi[0]) / (2.0 * hs[d]);
        double Ap[4][4], Am[4][4];
        nonadvective_flux(P, C->eos, tau, C->q + NQ * cp, C->e[cp], upl, Ap);
        nonadvective_flux(P, C->eos, tau, C->q + NQ * cm, C->e[cm], umi, Am);
        for (int n = 0; n < 4; ++n) Sc[n] -= (Ap[d + 1][n] - Am[d + 1][n]) / (2.0 * hs[d]);
    }

    /* geometric source of the conservation law: d_mu T^{mu nu} = 0 with sqrt(g) = tau,
     * G_c^nu = -(1/tau) T^{tau nu} - Gamma^nu_{mu l} T^{mu l}; T^{tau nu} is the evolved
     * state, T^{ij} = v^i T^{tau j} + A^{ij}. */
    double Tfull[4][4], Ac[4][4];
    nonadvective_flux(P, C->eos, tau, q, e, u, Ac);
    for (int n = 0; n < 4; ++n) { Tfull[0][n] = q[n]; Tfull[n][0] = q[n]; }
    for (int a = 1; a < 4; ++a)
        for (int b = 1; b < 4; ++b) Tfull[a][b] = v[a] * q[b] + Ac[a][b];
    for (int n = 0; n < 4; ++n) {
        double G = cart ? 0.0 : -q[n] / tau;
        for (int m = 0; m < 4; ++m)
            for (int l = 0; l < 4; ++l) G -= christoffel(n, m, l, tau, cart) * Tfull[m][l];
        J[n] = Sc[n] + G;
    }
    for (int c = 4; c < NQ; ++c) J[c] = 0.0;
    if (!shear && !bulk) return;

    kin_t K;
    kinematics(tau, cart, u, du, &K);
    double I1[4][4], I2[4][4], I3[4][4], I4[4][4], pis;
    second_order_terms(tau, cart, u, pi, &K, I1, I2, I3, I4, &pis);
    const double dPi = 1.0 - 3.0 * cs2;   /* 3 (1/3 - c_s^2) */
    const double d13 = dPi / 3.0;         /* 1/3 - c_s^2 */

    if (shear) {
        /* shear coefficients near the conformal limit (Sec. 2.2) */
        const double inv_tpi = T / (5.0 * P->eta_s);
        const double eta_tpi = (e + p0) / 5.0;
        const double dpipi = 4.0 / 3.0, tpipi = P->taupipi, lpiPi = 6.0 / 5.0;
        for (int m = 0; m < 4; ++m)
            for (int n = m; n < 4; ++n) {
                double Ipi = I1[m][n] + dpipi * I2[m][n] - I3[m][n] + tpipi * I4[m][n]
                           - lpiPi * Pi * K.sigma[m][n];
                double Gdef = 0.0;   /* u^a Gamma^m_{ab} pi^{b n} + u^a Gamma^n_{ab} pi^{b m} */
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b)
                        Gdef += u[a] * (christoffel(m, a, b, tau, cart) * pi[b][n]
                                      + christoffel(n, a, b, tau, cart) * pi[b][m]);
                double rhs = 2.0 * eta_tpi * K.sigma[m][n] - pi[m][n] * inv_tpi - Ipi - Gdef;
                J[PI_IDX[m][n]] = rhs / u[0] + pi[m][n] * divv;
            }
    }
    if (bulk) {
        /* zeta / tau_Pi = 15 (1/3 - c_s^2)^2 (e + P) in both models, so that
         * 1/tau_Pi = 15 (1/3 - c_s^2)^2 T / (zeta/s) */
        const double inv_tPi = P->zeta_model == 1
            ? 15.0 * d13 * d13 * T / (P->zeta_coef * ora_zeta_over_s_paper(T / P->zeta_tc))
            : 15.0 * d13 * T / P->zeta_coef;
        const double zeta_tPi = 15.0 * d13 * d13 * (e + p0);
        const double dPiPi = 2.0 / 3.0, lPipi = 8.0 / 5.0 * d13;
        double IPi = dPiPi * Pi * K.theta - lPipi * pis;
        J[14] = (-zeta_tPi * K.theta - Pi * inv_tPi - IPi) / u[0] + Pi * divv;
    }
}

/* ------------------------------------------------------------------ */
/* Semi-discrete operator C[q] (Sec. 3.1, Eq. semiDiscreteKT)          */
/* ------------------------------------------------------------------ */

static void cell_rhs(ctx_t *C, int i, int j, int k, double out[NQ])
{
    const ora_params *P = C->P;
    const double hs[3] = {P->dx, P->dy, P->deta};
    double J[NQ];
    cell_sources(C, i, j, k, J);
    for (int n = 0; n < NQ; ++n) out[n] = 0.0;
    for (int d = 0; d < 3; ++d) {
        double Hp[NQ], Hm[NQ];
        face_flux(C, i, j, k, d, +1, Hp);
        face_flux(C, i, j, k, d, -1, Hm);
        for (int n = 0; n < NQ; ++n) out[n] -= (Hp[n] - Hm[n]) / hs[d];
    }
    for (int n = 0; n < NQ; ++n) out[n] += J[n];
    if (!(P->eta_s > 0.0)) for (int n = 4; n < 14; ++n) out[n] = 0.0;
    if (!(P->zeta_coef > 0.0)) out[14] = 0.0;
}

static void rhs_all(ctx_t *C, double *rhs)
{
    const ora_params *P = C->P;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < P->neta; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i)
                cell_rhs(C, i, j, k, rhs + NQ * cell_index(P, i, j, k));
}

/* recover (e, u) of every cell of q at tau, then regulate pi (Sec. 4.3 steps 2-3, 8) */
static void recover_all(const ora_params *P, const ora_eos *eos, double tau, double *q,
                        double *e, double *u, ora_stats *st, int do_regulate)
{
    const int64_t n = (int64_t)P->nx * P->ny * P->neta;
    int64_t it_sum = 0, nfl = 0, ncl = 0, nfb = 0;
#pragma omp parallel for schedule(static) reduction(+ : it_sum, nfl, ncl, nfb)
    for (int64_t c = 0; c < n; ++c) {
        int it;
        int f = recover(P, eos, tau, q + NQ * c, e + c, u + 4 * c, &it);
        if ((f & FL_FLOOR) && P->floor_resets_q) {
            double *qc = q + NQ * c;
            for (int m = 0; m < NQ; ++m) qc[m] = 0.0;
            qc[0] = P->e_floor;
        }
        it_sum += it;
        nfl += (f & FL_FLOOR) != 0;
        ncl += (f & FL_CLAMP) != 0;
        nfb += (f & FL_FALLBACK) != 0;
        if (do_regulate) regulate_cell(P, eos, tau, q + NQ * c, e[c], u + 4 * c);
    }
    if (st) {
        st->newton_iters += it_sum;
        st->n_floor += nfl;
        st->n_clamp += ncl;
        st->n_fallback += nfb;
        st->n_recover += n;
    }
}

/* ------------------------------------------------------------------ */
/* Exported entry points                                               */
/* ------------------------------------------------------------------ */

/* q (n x 15) from primitives e (n), u (n x 4), pi (n x 10), Pi (n). */
void ora_tmunu(const ora_params *P, const ora_eos *eos, double tau, int64_t n, const double *e,
               const double *u, const double *pi, const double *Pi, double *q)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c)
        tmunu_from_primitives(P, eos, tau, e[c], u + 4 * c, pi + 10 * c, Pi[c], q + NQ * c);
}

/* standalone recovery of n cells; iters/flags nullable; e_start (nullable):
 * per-cell Newton start, values <= 0 meaning the conformal closed form */
void ora_recover(const ora_params *P, const ora_eos *eos, double tau, int64_t n, const double *q,
                 const double *e_start, double *e, double *u, int32_t *iters, int32_t *flags)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        int it;
        int f = recover_from(P, eos, tau, q + NQ * c, e_start ? e_start[c] : -1.0, e + c, u + 4 * c, &it);
        if (iters) iters[c] = it;
        if (flags) flags[c] = f;
    }
}

void ora_regulate(const ora_params *P, const ora_eos *eos, double tau, int64_t n, double *q,
                  const double *e, const double *u, double *factor)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        double f = regulate_cell(P, eos, tau, q + NQ * c, e[c], u + 4 * c);
        if (factor) factor[c] = f;
    }
}

void ora_eos_eval(const ora_eos *eos, int64_t n, const double *e, double *p, double *cs2, double *T)
{
    for (int64_t c = 0; c < n; ++c) eos_eval(eos, e[c], p + c, cs2 + c, T + c);
}

/* initial recovery at tau0: e, u from q; u_prev = u (Sec. 4.3 footnote) */
void ora_init(const ora_params *P, const ora_eos *eos, double tau0, const double *q,
              double *e, double *u, double *up)
{
    const int64_t n = (int64_t)P->nx * P->ny * P->neta;
    recover_all(P, eos, tau0, (double *)q, e, u, NULL, 0);
    memcpy(up, u, sizeof(double) * 4 * n);
}

/* C[q] for all cells at tau with e, u the primitives of q and up the previous u */
void ora_rhs(const ora_params *P, const ora_eos *eos, double tau, const double *q,
             const double *e, const double *u, const double *up, double *rhs)
{
    ctx_t C = {P, eos, tau, q, e, u, up, NULL};
    rhs_all(&C, rhs);
}

/* n_steps Heun steps in place (Sec. 3.1 Eqs. step1-finalStep with s = 2; Sec. 4.3):
 *   q*    = q^n + dtau C[q^n; e^n, u^n, u^{n-1}]         at tau^n
 *   (e*, u*) <- recover(q*), regulate q*                 at tau^{n+1}
 *   q**   = q* + dtau C[q*; e*, u*, u^n]                 at tau^{n+1}
 *   q^{n+1} = (q^n + q**) / 2;  u^{n-1} <- u^n;  (e, u) <- recover(q^{n+1}), regulate.
 * The work arrays are allocated here. Returns 0 on success. */
int ora_step(const ora_params *P, const ora_eos *eos, double *tau_io, double *q, double *e,
             double *u, double *up, int32_t n_steps, ora_stats *st)
{
    const int64_t n = (int64_t)P->nx * P->ny * P->neta;
    double *qs = malloc(sizeof(double) * NQ * n);
    double *rhs = malloc(sizeof(double) * NQ * n);
    double *us = malloc(sizeof(double) * 4 * n);
    double *es = malloc(sizeof(double) * n);
    if (!qs || !rhs || !us || !es) { free(qs); free(rhs); free(us); free(es); return 1; }
    double tau = *tau_io;
    for (int s = 0; s < n_steps; ++s) {
        const double tau1 = tau + P->dtau;
        ctx_t C1 = {P, eos, tau, q, e, u, up, st};
        rhs_all(&C1, rhs);
        for (int64_t c = 0; c < NQ * n; ++c) qs[c] = q[c] + P->dtau * rhs[c];
        recover_all(P, eos, tau1, qs, es, us, st, 1);
        ctx_t C2 = {P, eos, tau1, qs, es, us, u, st};
        rhs_all(&C2, rhs);
        for (int64_t c = 0; c < NQ * n; ++c) {
            double qss = qs[c] + P->dtau * rhs[c];
            q[c] = (q[c] + qss) / 2.0;
        }
        memcpy(up, u, sizeof(double) * 4 * n);
        recover_all(P, eos, tau1, q, e, u, st, 1);
        tau = tau1;
    }
    *tau_io = tau;
    free(qs); free(rhs); free(us); free(es);
    return 0;
}

/* --- pieces exposed for unit tests of the source algebra --- */

/* out: theta (1), sigma (16), omega (16), Du_lo (4), Delta (16) -> 53 values */
void ora_kinematics(double tau, int32_t cartesian, const double *u, const double *du, double *out)
{
    double d[4][4];
    for (int a = 0; a < 4; ++a) for (int m = 0; m < 4; ++m) d[a][m] = du[4 * a + m];
    kin_t K;
    kinematics(tau, cartesian, u, d, &K);
    out[0] = K.theta;
    for (int m = 0; m < 16; ++m) {
        out[1 + m] = K.sigma[m / 4][m % 4];
        out[17 + m] = K.omega[m / 4][m % 4];
        out[37 + m] = K.Delta[m / 4][m % 4];
    }
    for (int m = 0; m < 4; ++m) out[33 + m] = K.Du_lo[m];
}

/* out: I1, I2, I3, I4 (16 each), pi:sigma (1) -> 65 values; pi16 is the full 4x4 */
void ora_second_order(double tau, int32_t cartesian, const double *u, const double *du,
                      const double *pi16, double *out)
{
    double d[4][4], pi[4][4];
    for (int a = 0; a < 16; ++a) { d[a / 4][a % 4] = du[a]; pi[a / 4][a % 4] = pi16[a]; }
    kin_t K;
    kinematics(tau, cartesian, u, d, &K);
    double I1[4][4], I2[4][4], I3[4][4], I4[4][4], ps;
    second_order_terms(tau, cartesian, u, pi, &K, I1, I2, I3, I4, &ps);
    for (int m = 0; m < 16; ++m) {
        out[m] = I1[m / 4][m % 4];
        out[16 + m] = I2[m / 4][m % 4];
        out[32 + m] = I3[m / 4][m % 4];
        out[48 + m] = I4[m / 4][m % 4];
    }
    out[64] = ps;
}

/* geometric term of the relaxation equation as it enters d/dtau pi (App. B's G_pi):
 * -(u^a Gamma^m_{ab} pi^{b n} + u^a Gamma^n_{ab} pi^{b m}) / u^tau, 16 values */
void ora_gpi(double tau, int32_t cartesian, const double *u, const double *pi16, double *out)
{
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            double G = 0.0;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    G += u[a] * (christoffel(m, a, b, tau, cartesian) * pi16[4 * b + n]
                               + christoffel(n, a, b, tau, cartesian) * pi16[4 * b + m]);
            out[4 * m + n] = -G / u[0];
        }
}

double ora_minmod3(double x, double y, double z) { return minmod3(x, y, z); }

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ==================================================================== */
/* Diagnostics.  Everything above this line defines the step (the       */
/* golden samples of the test suite record its hash); what follows only */
/* reads states.                                                        */
/* ==================================================================== */

/* OpenMP threads of the oracle's loops (the CPU baseline times 1 thread and
 * all of them; results do not depend on the count: cells are independent) */
void ora_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Observables of a state, the definitions of the library's kt_obs written
 * with this file's generic contractions (loops in cell order, one thread):
 *   out[0]      sum of T^{tau tau} times the cell volume dx dy deta (times tau in Milne)
 *   out[1..3]   the same for T^{tau x}, T^{tau y}, T^{tau eta}
 *   out[4], [5] largest e and T(e)
 *   out[6]      largest |v^i| = |u^i/u^tau| over cells and axes, in an orthonormal
 *               frame (the eta component times tau)
 *   out[7]      dtau times the largest |v^i| / d_i (coordinate components)
 *   out[8]      largest |u^mu u_mu - 1|
 *   out[9]      largest max_lambda |pi^{lambda mu} u_mu| / sqrt(|pi^{mu nu} pi_{mu nu}|)
 *               (orthonormal frame), the orthogonality check of Sec. 2.4
 *   out[10]     largest |g_{mu nu} pi^{mu nu}| / sqrt(|pi^{mu nu} pi_{mu nu}|), the
 *               tracelessness check of Sec. 2.4 (both over cells with pi:pi != 0,
 *               0 without shear viscosity)
 *   out[11]     cells with a non-finite value in q, e or u (left out of the rest) */
void ora_observables(const ora_params *P, const ora_eos *eos, double tau, const double *q,
                     const double *e, const double *u, double *out)
{
    const int64_t n = (int64_t)P->nx * P->ny * P->neta;
    double glo[4], ghi[4];
    metric(tau, P->cartesian, glo, ghi);
    const double h[3] = {P->dx, P->dy, P->deta};
    double sum[4] = {0, 0, 0, 0}, emax = 0, Tmax = 0, vmax = 0, cfl = 0, nerr = 0, piu = 0, pitr = 0;
    int64_t nnan = 0;
    for (int64_t c = 0; c < n; ++c) {
        const double *qc = q + NQ * c, *uc = u + 4 * c;
        int finite = isfinite(e[c]);
        for (int k = 0; k < NQ; ++k) finite = finite && isfinite(qc[k]);
        for (int m = 0; m < 4; ++m) finite = finite && isfinite(uc[m]);
        if (!finite) { ++nnan; continue; }
        for (int m = 0; m < 4; ++m) sum[m] += qc[m];
        double p, cs2, T;
        eos_eval(eos, e[c], &p, &cs2, &T);
        if (e[c] > emax) emax = e[c];
        if (T > Tmax) Tmax = T;
        double uu = 0.0;
        for (int m = 0; m < 4; ++m) uu += glo[m] * uc[m] * uc[m];
        if (fabs(uu - 1.0) > nerr) nerr = fabs(uu - 1.0);
        for (int i = 1; i < 4; ++i) {
            double v = fabs(uc[i] / uc[0]);
            if (v * sqrt(fabs(glo[i])) > vmax) vmax = v * sqrt(fabs(glo[i]));
            if (v / h[i - 1] * P->dtau > cfl) cfl = v / h[i - 1] * P->dtau;
        }
        if (P->eta_s > 0.0) {
            double pi[4][4], pp = 0.0, tr = 0.0, w = 0.0;
            pi_tensor(qc, pi);
            for (int m = 0; m < 4; ++m) {
                tr += glo[m] * pi[m][m];
                double s = 0.0;
                for (int k = 0; k < 4; ++k) {
                    pp += glo[m] * glo[k] * pi[m][k] * pi[m][k];
                    s += pi[m][k] * glo[k] * uc[k];
                }
                s = fabs(s) * sqrt(fabs(glo[m]));
                if (s > w) w = s;
            }
            const double np = sqrt(fabs(pp));
            if (np > 0.0) {
                if (w / np > piu) piu = w / np;
                if (fabs(tr) / np > pitr) pitr = fabs(tr) / np;
            }
        }
    }
    const double vol = P->dx * P->dy * P->deta * (P->cartesian ? 1.0 : tau);
    for (int m = 0; m < 4; ++m) out[m] = sum[m] * vol;
    out[4] = emax; out[5] = Tmax; out[6] = vmax; out[7] = cfl; out[8] = nerr;
    out[9] = piu; out[10] = pitr; out[11] = (double)nnan;
}

/* Validity of the second-order truncation (Sec. 7, Eq. inverseReynoldsNumbers2)
 * and the regulation factor (Sec. 3.2, Eqs. regPimunu, rho), per cell of the
 * state (q, e, u) at tau with the previous step's flow up:
 *   J^{mu nu} = 2 tau_pi pi_l^<mu omega^nu>l - delta_pipi pi^{mu nu} theta
 *               - tau_pipi pi^{l<mu} sigma^{nu>}_l + lambda_piPi Pi sigma^{mu nu}
 *   J         = -delta_PiPi Pi theta + lambda_Pipi pi^{mu nu} sigma_{mu nu}
 * (Eq. 14_moment_terms without particle diffusion, coefficients of Sec. 2.2),
 *   rinv2_pi = sqrt(J^{mu nu} J_{mu nu}) / (2 eta sqrt(sigma^{mu nu} sigma_{mu nu})),
 *   rinv2_Pi = |J| / (zeta |theta|),
 * with eta = tau_pi (e + P0)/5 and zeta = tau_Pi 15 (1/3 - c_s^2)^2 (e + P0), so
 * the relaxation times cancel; 0 where the dissipative quantity is not evolved
 * or the numerator vanishes, +inf where only the denominator vanishes.  The
 * gradients are those of the sources: a backward difference in tau and central
 * differences in space of the cell flow.  reg = tanh(rho)/rho of Eq. rho
 * evaluated on the state (1 where it does not regulate).  Outputs nullable. */
void ora_validity2(const ora_params *P, const ora_eos *eos, double tau, const double *q,
                   const double *e, const double *u, const double *up, double *rinv2_pi,
                   double *rinv2_Pi, double *reg)
{
    const int shear = P->eta_s > 0.0, bulk = P->zeta_coef > 0.0;
    const double hs[3] = {P->dx, P->dy, P->deta};
    double glo[4], ghi[4];
    metric(tau, P->cartesian, glo, ghi);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < P->neta; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                const int64_t c = cell_index(P, i, j, k);
                const double *qc = q + NQ * c, *uc = u + 4 * c, *upc = up + 4 * c;
                double du[4][4];
                for (int m = 0; m < 4; ++m) du[0][m] = (uc[m] - upc[m]) / P->dtau;
                for (int d = 0; d < 3; ++d) {
                    const double *ua = u + 4 * neighbour(P, i, j, k, d, +1);
                    const double *ub = u + 4 * neighbour(P, i, j, k, d, -1);
                    for (int m = 0; m < 4; ++m) du[d + 1][m] = (ua[m] - ub[m]) / (2.0 * hs[d]);
                }
                kin_t K;
                kinematics(tau, P->cartesian, uc, du, &K);
                double pi[4][4];
                pi_tensor(qc, pi);
                if (!shear)
                    for (int m = 0; m < 4; ++m) for (int n = 0; n < 4; ++n) pi[m][n] = 0.0;
                double I1[4][4], I2[4][4], I3[4][4], I4[4][4], pis;
                second_order_terms(tau, P->cartesian, uc, pi, &K, I1, I2, I3, I4, &pis);
                double p0, cs2, T;
                eos_eval(eos, e[c], &p0, &cs2, &T);
                const double Pi = bulk ? qc[14] : 0.0;
                const double d13 = 1.0 / 3.0 - cs2;
                if (rinv2_pi) {
                    double v = 0.0;
                    if (shear) {
                        /* J^{mu nu} / tau_pi, with I3 = 2 pi_l^<mu omega^nu>l and
                         * I4 = pi^{l<mu} sigma^{nu>}_l as in the relaxation equation */
                        double XX = 0.0, SS = 0.0;
                        for (int m = 0; m < 4; ++m)
                            for (int n = 0; n < 4; ++n) {
                                double X = I3[m][n] - 4.0 / 3.0 * I2[m][n] - P->taupipi * I4[m][n]
                                         + 6.0 / 5.0 * Pi * K.sigma[m][n];
                                XX += glo[m] * glo[n] * X * X;
                                SS += glo[m] * glo[n] * K.sigma[m][n] * K.sigma[m][n];
                            }
                        const double num = sqrt(fabs(XX));
                        v = num == 0.0 ? 0.0 : num / (2.0 * (e[c] + p0) / 5.0 * sqrt(fabs(SS)));
                    }
                    rinv2_pi[c] = v;
                }
                if (rinv2_Pi) {
                    double v = 0.0;
                    if (bulk) {
                        /* J / tau_Pi over zeta / tau_Pi */
                        const double num = fabs(-2.0 / 3.0 * Pi * K.theta + 8.0 / 5.0 * d13 * pis);
                        v = num == 0.0 ? 0.0 : num / (15.0 * d13 * d13 * (e[c] + p0) * fabs(K.theta));
                    }
                    rinv2_Pi[c] = v;
                }
                if (reg) {
                    double qq[NQ];
                    for (int m = 0; m < NQ; ++m) qq[m] = qc[m];
                    reg[c] = regulate_cell(P, eos, tau, qq, e[c], uc);
                }
            }
}

/* ==================================================================== */
/* Reduced storage (Sec. 2.4, the paragraph with Eqs. pi_tautau ..       */
/* pi_etaeta; Sec. 4.2, last paragraph on memory).  Only the five        */
/* components pi^{xx}, pi^{xy}, pi^{x eta}, pi^{yy}, pi^{y eta} of the    */
/* shear stress and the three u^x, u^y, u^eta of the flow are kept; the   */
/* other five of pi follow from u_mu pi^{mu nu} = 0 and g_{mu nu}         */
/* pi^{mu nu} = 0, and u^tau from u^mu u_mu = 1 (Sec. 2.4).  The step is   */
/* the one above, applied to the state expanded to all components:       */
/*   - the evolved vector is (T^{tau mu}, the five pi, Pi); the other five */
/*     pi components are not evolved but rebuilt from the five and the    */
/*     cell's velocity wherever a cell's full state is needed (sources,   */
/*     and the cells whose reconstruction gives the face states);         */
/*   - the recovery solves for (e, u) and the dependent pi together: with */
/*     pi^{tau mu} of the current velocity iterate, Newton's recovery     */
/*     gives the next velocity, until it stops changing;                  */
/*   - the regulator acts on the full tensor and rescales the five (and   */
/*     Pi as in the full step).                                           */
/* Reading taken: the paper states only that the remaining components are */
/* determined algebraically; the face states use the reconstructed cell    */
/* values of all components, the cells' dependent ones included.          */
/* ==================================================================== */

#define NR 10   /* reduced evolved vector: T^{tau mu} (4), five pi, Pi */
static const int RED_IDX[NR] = {0, 1, 2, 3, 8, 9, 10, 11, 12, 14};   /* positions in q[NQ] */

/* pi^{eta eta}, pi^{tau eta}, pi^{tau y}, pi^{tau x}, pi^{tau tau} of q from its
 * five independent components and the contravariant 3-velocity v^i = u^i / u^tau:
 * Eq. pi_etaeta, then the four orthogonality relations Eq. pi_tautau and the
 * three printed after it, each written as the paper writes it (tau^2 -> 1 in
 * Cartesian coordinates). */
static void pi_dependent(double tau, int cart, const double u[4], double q[NQ])
{
    const double t2 = cart ? 1.0 : tau * tau;
    const double vx = u[1] / u[0], vy = u[2] / u[0], ve = u[3] / u[0];
    const double pxx = q[8], pxy = q[9], pxe = q[10], pyy = q[11], pye = q[12];
    const double pee = (pxx * (vx * vx - 1.0) + pyy * (vy * vy - 1.0) + 2.0 * pxy * vx * vy
                        + 2.0 * t2 * (pxe * vx * ve + pye * vy * ve))
                       / (t2 * (1.0 - t2 * ve * ve));
    const double pte = pxe * vx + pye * vy + t2 * pee * ve;
    const double pty = pxy * vx + pyy * vy + t2 * pye * ve;
    const double ptx = pxx * vx + pxy * vy + t2 * pxe * ve;
    const double ptt = ptx * vx + pty * vy + t2 * pte * ve;
    q[4] = ptt; q[5] = ptx; q[6] = pty; q[7] = pte; q[13] = pee;
}

/* u^tau from u^mu u_mu = 1 at tau (Sec. 2.4) */
static void u_full(double tau, int cart, const double *u3, double u[4])
{
    const double t2 = cart ? 1.0 : tau * tau;
    u[1] = u3[0]; u[2] = u3[1]; u[3] = u3[2];
    u[0] = sqrt(1.0 + u[1] * u[1] + u[2] * u[2] + t2 * u[3] * u[3]);
}

/* full state of a cell from its reduced state r[NR] and flow u3 at tau */
static void expand_cell(const ora_params *P, double tau, const double *r, const double *u3,
                        double q[NQ], double u[4])
{
    for (int c = 0; c < NQ; ++c) q[c] = 0.0;
    for (int k = 0; k < NR; ++k) q[RED_IDX[k]] = r[k];
    u_full(tau, P->cartesian, u3, u);
    if (P->eta_s > 0.0) pi_dependent(tau, P->cartesian, u, q);
}

/* Recovery of (e, u) from the reduced state at tau: fixed point of
 *   u_{k+1} = recover(T^{tau mu}, pi^{tau mu}(five, v(u_k)), Pi)
 * from u_0 = u_start (the cell's flow before the stage, normalised at tau; null:
 * (1, 0, 0, 0), i.e. pi^{tau mu} = 0), stopped when no component of u moves by
 * more than FP_TOL u^tau (the eta component times tau), or after FP_MAX passes
 * (counted as not converged).  The state's dependent components are those of the
 * final u.  Returns the flags of the last recovery. */
static const double FP_TOL = 1e-14;
static const int FP_MAX = 100;

static int recover_reduced(const ora_params *P, const ora_eos *eos, double tau, const double *r,
                           const double *u_start, double *e_out, double u_out[4], int *iters,
                           int *passes, int *conv)
{
    const double t2 = P->cartesian ? 1.0 : tau * tau;
    double q[NQ], u[4] = {1.0, 0.0, 0.0, 0.0};
    if (u_start) u_full(tau, P->cartesian, u_start, u);
    int flags = 0, it_sum = 0, k = 0;
    *conv = 0;
    for (k = 0; k < FP_MAX; ++k) {
        for (int c = 0; c < NQ; ++c) q[c] = 0.0;
        for (int m = 0; m < NR; ++m) q[RED_IDX[m]] = r[m];
        if (P->eta_s > 0.0) pi_dependent(tau, P->cartesian, u, q);
        double un[4], e;
        int it;
        flags = recover(P, eos, tau, q, &e, un, &it);
        it_sum += it;
        *e_out = e;
        double dmax = 0.0;
        for (int m = 0; m < 4; ++m) {
            double d = fabs(un[m] - u[m]) * (m == 3 ? sqrt(t2) : 1.0) / un[0];
            if (d > dmax) dmax = d;
        }
        for (int m = 0; m < 4; ++m) u[m] = un[m];
        if ((flags & FL_FLOOR) || !(P->eta_s > 0.0) || dmax <= FP_TOL) { *conv = 1; ++k; break; }
    }
    for (int m = 0; m < 4; ++m) u_out[m] = u[m];
    *iters = it_sum;
    *passes = k;
    return flags;
}

typedef struct {
    int64_t passes, not_converged;
} ora_fp_stats;

/* recover every cell of the reduced state, reset floor cells, regulate (the
 * full tensor; the five and Pi are rescaled) */
static void recover_all_reduced(const ora_params *P, const ora_eos *eos, double tau, double *r,
                                const double *u_start, double *e, double *u3, ora_stats *st,
                                ora_fp_stats *fs, int do_regulate)
{
    const int64_t n = (int64_t)P->nx * P->ny * P->neta;
    int64_t it_sum = 0, nfl = 0, ncl = 0, nfb = 0, np = 0, nnc = 0;
#pragma omp parallel for schedule(static) reduction(+ : it_sum, nfl, ncl, nfb, np, nnc)
    for (int64_t c = 0; c < n; ++c) {
        double *rc = r + NR * c;
        double u[4];
        int it, passes, conv;
        int f = recover_reduced(P, eos, tau, rc, u_start ? u_start + 3 * c : NULL, e + c, u, &it,
                                &passes, &conv);
        if ((f & FL_FLOOR) && P->floor_resets_q) {
            for (int m = 0; m < NR; ++m) rc[m] = 0.0;
            rc[0] = P->e_floor;
        }
        if (do_regulate) {
            double q[NQ];
            for (int m = 0; m < NQ; ++m) q[m] = 0.0;
            for (int m = 0; m < NR; ++m) q[RED_IDX[m]] = rc[m];
            if (P->eta_s > 0.0) pi_dependent(tau, P->cartesian, u, q);
            regulate_cell(P, eos, tau, q, e[c], u);
            for (int m = 4; m < NR; ++m) rc[m] = q[RED_IDX[m]];
        }
        for (int m = 0; m < 3; ++m) u3[3 * c + m] = u[m + 1];
        it_sum += it;
        nfl += (f & FL_FLOOR) != 0;
        ncl += (f & FL_CLAMP) != 0;
        nfb += (f & FL_FALLBACK) != 0;
        np += passes;
        nnc += !conv;
    }
    if (st) {
        st->newton_iters += it_sum;
        st->n_floor += nfl;
        st->n_clamp += ncl;
        st->n_fallback += nfb;
        st->n_recover += n;
    }
    if (fs) {
        fs->passes += np;
        fs->not_converged += nnc;
    }
}

/* full arrays (q: n x 15, u: n x 4) of a reduced state (r: n x 10, u3: n x 3) at tau */
void ora_expand(const ora_params *P, double tau, int64_t n, const double *r, const double *u3,
                double *q, double *u)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) expand_cell(P, tau, r + NR * c, u3 + 3 * c, q + NQ * c, u + 4 * c);
}

/* the dependent components of n cells (q: n x 15 in and out, u: n x 4) */
void ora_pi_dependent(double tau, int32_t cartesian, int64_t n, const double *u, double *q)
{
    for (int64_t c = 0; c < n; ++c) pi_dependent(tau, cartesian, u + 4 * c, q + NQ * c);
}

/* standalone reduced recovery of n cells (no regulation, no floor reset) */
void ora_recover_reduced(const ora_params *P, const ora_eos *eos, double tau, int64_t n,
                         const double *r, double *e, double *u, int32_t *iters, int32_t *passes,
                         int32_t *flags)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        int it, ps, conv;
        int f = recover_reduced(P, eos, tau, r + NR * c, NULL, e + c, u + 4 * c, &it, &ps, &conv);
        if (iters) iters[c] = it;
        if (passes) passes[c] = conv ? ps : -ps;
        if (flags) flags[c] = f;
    }
}

/* initial recovery of a reduced state at tau0 (no regulation, as ora_init); u_prev = u */
void ora_init_reduced(const ora_params *P, const ora_eos *eos, double tau0, double *r,
                      double *e, double *u3, double *up3)
{
    const int64_t n = (int64_t)P->nx * P->ny * P->neta;
    recover_all_reduced(P, eos, tau0, r, NULL, e, u3, NULL, NULL, 0);
    memcpy(up3, u3, sizeof(double) * 3 * n);
}

/* n_steps Heun steps of the reduced state in place, the step of ora_step on the
 * expanded state.  The previous flow u_prev is normalised at *tau_prev_io, the
 * time of its level: tau - dtau once a step has been taken, tau0 before the
 * first step, whose u_prev is u^0 itself (Sec. 4.3 sets u^{-1} = u^0, the same
 * four-vector).  The recovery of q* starts its
 * fixed point from u^n, that of q^{n+1} from u*.  fp_stats (nullable): passes
 * of the recovery's fixed point and cells where it did not converge. */
int ora_step_reduced(const ora_params *P, const ora_eos *eos, double *tau_io, double *tau_prev_io,
                     double *r, double *e, double *u3, double *up3, int32_t n_steps, ora_stats *st,
                     int64_t *fp_stats)
{
    const int64_t n = (int64_t)P->nx * P->ny * P->neta;
    double *qf = malloc(sizeof(double) * NQ * n);
    double *rhs = malloc(sizeof(double) * NQ * n);
    double *uf = malloc(sizeof(double) * 4 * n);
    double *upf = malloc(sizeof(double) * 4 * n);
    double *rs = malloc(sizeof(double) * NR * n);
    double *us3 = malloc(sizeof(double) * 3 * n);
    double *es = malloc(sizeof(double) * n);
    if (!qf || !rhs || !uf || !upf || !rs || !us3 || !es) {
        free(qf); free(rhs); free(uf); free(upf); free(rs); free(us3); free(es);
        return 1;
    }
    ora_fp_stats fs = {0, 0};
    double tau = *tau_io, tau_prev = *tau_prev_io;
    for (int s = 0; s < n_steps; ++s) {
        const double tau1 = tau + P->dtau;
        /* stage 1 at tau on (q^n, e^n, u^n, u^{n-1}) */
        ora_expand(P, tau, n, r, u3, qf, uf);
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < n; ++c) u_full(tau_prev, P->cartesian, up3 + 3 * c, upf + 4 * c);
        ctx_t C1 = {P, eos, tau, qf, e, uf, upf, st};
        rhs_all(&C1, rhs);
        for (int64_t c = 0; c < n; ++c)
            for (int k = 0; k < NR; ++k) rs[NR * c + k] = r[NR * c + k] + P->dtau * rhs[NQ * c + RED_IDX[k]];
        recover_all_reduced(P, eos, tau1, rs, u3, es, us3, st, &fs, 1);
        /* stage 2 at tau^{n+1} on (q*, e*, u*, u^n) */
        ora_expand(P, tau1, n, rs, us3, qf, uf);
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < n; ++c) u_full(tau1 - P->dtau, P->cartesian, u3 + 3 * c, upf + 4 * c);
        ctx_t C2 = {P, eos, tau1, qf, es, uf, upf, st};
        rhs_all(&C2, rhs);
        for (int64_t c = 0; c < n; ++c)
            for (int k = 0; k < NR; ++k) {
                double rss = rs[NR * c + k] + P->dtau * rhs[NQ * c + RED_IDX[k]];
                r[NR * c + k] = (r[NR * c + k] + rss) / 2.0;
            }
        memcpy(up3, u3, sizeof(double) * 3 * n);
        recover_all_reduced(P, eos, tau1, r, us3, e, u3, st, &fs, 1);
        tau_prev = tau;
        tau = tau1;
    }
    *tau_io = tau;
    *tau_prev_io = tau_prev;
    if (fp_stats) {
        fp_stats[0] += fs.passes;
        fp_stats[1] += fs.not_converged;
    }
    free(qf); free(rhs); free(uf); free(upf); free(rs); free(us3); free(es);
    return 0;
}
