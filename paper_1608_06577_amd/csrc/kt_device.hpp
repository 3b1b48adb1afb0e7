// kt_device.hpp -- device functions of the KT/Heun step for gfx950.
//
// Bazow, Heinz & Strickland, arXiv:1608.06577.  The tensor algebra of
// Sec. 2.4 / App. A / App. B is expanded here for the diagonal Milne metric
// g_{mu nu} = diag(1, -1, -1, -g33), g33 = tau^2 (1 in Cartesian mode), whose
// only Christoffel symbols are Gamma^eta_{tau eta} = 1/tau and
// Gamma^tau_{eta eta} = tau.  Everything is FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ktd {

// evolved components (Sec. 3.1, Eq. qComponents)
enum : int {
    NQ = 15,
    TT = 0, TX = 1, TY = 2, TE = 3,
    PTT = 4, PTX = 5, PTY = 6, PTE = 7, PXX = 8, PXY = 9, PXE = 10, PYY = 11, PYE = 12, PEE = 13,
    BPI = 14
};

// recovery flags
enum : int { F_FLOOR = 1, F_CLAMP = 2, F_FALLBACK = 4 };

// counters, one slot row per wavefront
enum : int {
    C_ITERS_CELLS = 0, C_REC_CELLS, C_ITERS_FACES, C_REC_FACES, C_FLOOR, C_CLAMP, C_FALLBACK,
    C_FALLBACK_FACES,
    C_FP_PASSES, C_FP_NOCONV,   // reduced state: fixed-point passes of the recoveries, cells not converged
    C_COUNT
};

// EOS node layout: p/e, T/e^{1/4}, c_s^2, 1/e_i
constexpr int EOS_W = 4;

struct Eos {
    int conformal;
    double inv_a;          // 1 / a_sb
    int n;
    double ln_e0, inv_dln;
    const double *tab;     // n nodes of EOS_W doubles
};

struct Phys {
    int nx, ny, neta;
    long long ncell, stride;   // cells; distance between component arrays
    double inv_dx, inv_dy, inv_deta;
    double dtau, inv_dtau;
    int periodic[3];
    double theta;
    double eta_s, zeta_coef, taupipi;
    int zeta_model;      // 0: zeta/s = zeta_coef (1/3 - c_s^2); 1: zeta_coef zeta_over_s_paper(T / zeta_tc)
    double zeta_tc;
    int shear, bulk;
    int regulate, regulate_bulk, floor_reset;
    double xi0, rho_max;
    double e_floor, p_floor, m2_delta, newton_tol;
    int newton_max;
    int reduced;         // evolve the five independent pi components only (Sec. 2.4)
};

__host__ __device__ __forceinline__ int pi_index(int m, int n)
{
    // symmetric 4x4 -> position in q
    const int a = m < n ? m : n, b = m < n ? n : m;
    return a == 0 ? PTT + b : (a == 1 ? PXX + (b - 1) : (a == 2 ? PYY + (b - 2) : PEE));
}

// ------------------------------------------------------------------ EOS ---
// Table nodes e_i = exp(ln_e0 + i dln): p/e, T/e^{1/4}, c_s^2 linear in
// ln e between the bracketing nodes, end-node values outside the table.
// The bracket is found from a single-precision log2; the weight
// t = ln(e/e_i)/dln comes from ln(1+z), z = e/e_i - 1, |z| < 2 dln, by its
// series to z^8 (truncation below 1e-18 for dln <= 0.01), so no
// double-precision logarithm is evaluated.  Both nodes of the guessed
// bracket are read together with 1/e_i (one memory round trip); only when
// the weight falls outside [0, 1) is the bracket moved by one node and read
// again.
struct EosBracket {
    double a[EOS_W], b[EOS_W];   // nodes i and i+1
    double t;                    // weight of node i+1
};

__host__ __device__ __forceinline__ void eos_read(const Eos &E, int i, double a[EOS_W], double b[EOS_W])
{
    const double *r = E.tab + EOS_W * i;
#pragma unroll
    for (int k = 0; k < EOS_W; ++k) {
        a[k] = r[k];
        b[k] = r[EOS_W + k];
    }
}

// t = ln(e/e_i)/dln for the bracket B (node i = B.a)
__host__ __device__ __forceinline__ double eos_weight(const Eos &E, const EosBracket &B, double e)
{
    const double z = fma(e, B.a[3], -1.0);
    // ln(1+z) = z - z^2/2 + z^3/3 - ... - z^8/8
    double l = -1.0 / 8.0;
    l = fma(l, z, 1.0 / 7.0);
    l = fma(l, z, -1.0 / 6.0);
    l = fma(l, z, 1.0 / 5.0);
    l = fma(l, z, -1.0 / 4.0);
    l = fma(l, z, 1.0 / 3.0);
    l = fma(l, z, -1.0 / 2.0);
    l = fma(l, z, 1.0);
    return l * z * E.inv_dln;
}

__host__ __device__ __forceinline__ void eos_locate(const Eos &E, double e, EosBracket &B)
{
    const float lf = log2f((float)e);
    const double x = ((double)lf * 0.6931471805599453 - E.ln_e0) * E.inv_dln;
    if (!(x > -0.5)) {                 // below the table (or not a number)
        eos_read(E, 0, B.a, B.b);
        B.t = 0.0;
        return;
    }
    if (x > (double)(E.n - 1) + 0.5) {
        eos_read(E, E.n - 2, B.a, B.b);
        B.t = 1.0;
        return;
    }
    int i = (int)floor(x);
    i = i < 0 ? 0 : (i > E.n - 2 ? E.n - 2 : i);
    eos_read(E, i, B.a, B.b);
    double t = eos_weight(E, B, e);
    if (t < 0.0) {
        if (i > 0) {
            t += 1.0;
            eos_read(E, i - 1, B.a, B.b);
        } else t = 0.0;
    } else if (t >= 1.0) {
        if (i < E.n - 2) {
            t -= 1.0;
            eos_read(E, i + 1, B.a, B.b);
        } else t = 1.0;
    }
    B.t = t;
}

// p and c_s^2
__host__ __device__ __forceinline__ void eos_pc(const Eos &E, double e, double &p, double &cs2)
{
    if (E.conformal) {
        p = e * (1.0 / 3.0);
        cs2 = 1.0 / 3.0;
        return;
    }
    EosBracket B;
    eos_locate(E, e, B);
    p = (B.a[0] + B.t * (B.b[0] - B.a[0])) * e;
    cs2 = B.a[2] + B.t * (B.b[2] - B.a[2]);
}

// p, c_s^2 and T
__host__ __device__ __forceinline__ void eos_full(const Eos &E, double e, double &p, double &cs2,
                                                  double &T)
{
    if (E.conformal) {
        p = e * (1.0 / 3.0);
        cs2 = 1.0 / 3.0;
        T = e > 0.0 ? sqrt(sqrt(e * E.inv_a)) : 0.0;
        return;
    }
    EosBracket B;
    eos_locate(E, e, B);
    p = (B.a[0] + B.t * (B.b[0] - B.a[0])) * e;
    cs2 = B.a[2] + B.t * (B.b[2] - B.a[2]);
    T = (B.a[1] + B.t * (B.b[1] - B.a[1])) * sqrt(sqrt(e));
}

// p and c_s^2 at e, reusing the bracket B of an earlier evaluation when e
// lies inside it (successive Newton iterates mostly do), so that no table
// read is needed; have: B holds a bracket
__host__ __device__ __forceinline__ void eos_pc_near(const Eos &E, double e, EosBracket &B, bool &have,
                                                     double &p, double &cs2)
{
    if (E.conformal) {
        p = e * (1.0 / 3.0);
        cs2 = 1.0 / 3.0;
        return;
    }
    const double t = have ? eos_weight(E, B, e) : -1.0;
    if (t >= 0.0 && t < 1.0) {
        B.t = t;
    } else {
        eos_locate(E, e, B);
        have = true;
    }
    p = (B.a[0] + B.t * (B.b[0] - B.a[0])) * e;
    cs2 = B.a[2] + B.t * (B.b[2] - B.a[2]);
}

__host__ __device__ __forceinline__ double eos_p(const Eos &E, double e)
{
    double p, c;
    eos_pc(E, e, p, c);
    return p;
}

// ------------------------------------------------------------- recovery ---
// Inversion of Sec. 2.4 (e = E - M^2/(E + P(e)), u^tau, u^i) by
// Newton-Raphson (Sec. 3.2).  Guards: E <= e_floor, E + p(e_floor) + Pi <= 0
// or non-finite M^2 give the floor state; M^2 is clamped to
// (1 - m2_delta) W min(E - e_floor, W); conformal EOS without bulk uses the
// closed form sqrt(4E^2 - 3M^2) - E; otherwise Newton from e_start (<= 0:
// the conformal value), iterates clamped to [e_floor, E], one extra step
// after |f| <= tol E, bisection if not converged.
// invert_core returns the flags and gives e, p(e) of the equilibrium EOS,
// E = T^{tau tau} - pi^{tau tau} and the (possibly rescaled) M^i.
template <bool CART>
__device__ __forceinline__ int invert_core(const Phys &P, const Eos &E, double tau, double Ttt,
                                           double Ttx, double Tty, double Tte, double ptt,
                                           double ptx, double pty, double pte, double Pi,
                                           double e_start, double &e, double &p_out, double &EE_out,
                                           double M[3], int &iters)
{
    const double ef = P.e_floor;
    const double g33 = CART ? 1.0 : tau * tau;
    const double EE = Ttt - ptt;
    double Mx = Ttx - ptx, My = Tty - pty, Me = Tte - pte;
    double M2 = Mx * Mx + My * My + g33 * (Me * Me);
    const double W = EE + P.p_floor + Pi;
    iters = 0;
    EE_out = EE;
    if (!(EE > ef) || !(W > 0.0) || !(M2 == M2) || !(M2 < INFINITY)) {
        e = ef;
        p_out = P.p_floor;
        M[0] = M[1] = M[2] = 0.0;
        return F_FLOOR;
    }
    int flags = 0;
    const double M2max = (1.0 - P.m2_delta) * W * fmin(EE - ef, W);
    if (M2 > M2max) {
        const double s = sqrt(M2max / M2);
        Mx *= s;
        My *= s;
        Me *= s;
        M2 = M2max;
        flags |= F_CLAMP;
    }
    double x, p;
    if (E.conformal && !P.bulk) {
        x = fmax(sqrt(4.0 * EE * EE - 3.0 * M2) - EE, ef);
        p = x * (1.0 / 3.0);
    } else {
        x = e_start > 0.0 ? e_start : sqrt(4.0 * EE * EE - 3.0 * M2) - EE;
        x = fmin(fmax(x, ef), EE);
        bool done = false;
        int n = 0;
        double cs2;
        EosBracket B;
        bool have = false;
        while (n < P.newton_max) {
            // f = x - E + M^2/A and f' = 1 - M^2 c_s^2 / A^2 with A = E + p(x) + Pi > 0,
            // scaled by A and A^2 so that the step f/f' takes one division
            eos_pc_near(E, x, B, have, p, cs2);
            const double A = EE + p + Pi;
            const double fA = fma(x - EE, A, M2);
            const double dfA2 = fma(-M2, cs2, A * A);
            const bool conv = fabs(fA) <= P.newton_tol * EE * A;
            x = fmin(fmax(x - fA * A / dfA2, ef), EE);
            ++n;
            if (conv) {
                done = true;
                break;
            }
        }
        iters = n;
        if (!done) {
            double lo = ef, hi = EE;
            for (int k = 0; k < 200; ++k) {
                const double mid = 0.5 * (lo + hi);
                const double f = mid - EE + M2 / (EE + eos_p(E, mid) + Pi);
                x = mid;
                if (fabs(f) <= P.newton_tol * EE || hi - lo <= 4e-16 * hi) break;
                if (f < 0.0) lo = mid; else hi = mid;
            }
            flags |= F_FALLBACK;
        }
        eos_pc_near(E, x, B, have, p, cs2);
    }
    e = x;
    p_out = p;
    M[0] = Mx;
    M[1] = My;
    M[2] = Me;
    return flags;
}

// full recovery: u^tau = sqrt((E + P)/(e + P)), u^i = M^i / ((e + P) u^tau), P = p + Pi
template <bool CART>
__device__ __forceinline__ int recover(const Phys &P, const Eos &E, double tau, double Ttt,
                                       double Ttx, double Tty, double Tte, double ptt,
                                       double ptx, double pty, double pte, double Pi,
                                       double e_start, double &e, double &p_out, double u[4],
                                       int &iters)
{
    double EE, M[3];
    const int flags = invert_core<CART>(P, E, tau, Ttt, Ttx, Tty, Tte, ptt, ptx, pty, pte, Pi,
                                        e_start, e, p_out, EE, M, iters);
    if (flags & F_FLOOR) {
        u[0] = 1.0;
        u[1] = u[2] = u[3] = 0.0;
        return flags;
    }
    const double Pc = p_out + Pi;
    const double ut = sqrt((EE + Pc) / (e + Pc));
    const double inv = 1.0 / ((e + Pc) * ut);
    u[0] = ut;
    u[1] = M[0] * inv;
    u[2] = M[1] * inv;
    u[3] = M[2] * inv;
    return flags;
}

// ------------------------------------------------------------ regulator ---
// Sec. 3.2: rho = max( |Pi^{mu nu}| / (rho_max sqrt(e^2 + 3 P^2)),
//                      |pi^mu_mu| / (xi0 rho_max |Pi^{mu nu}|),
//                      max_l |pi^{l mu} u_mu| / (xi0 rho_max |Pi^{mu nu}|) ),
// Pi^{mu nu} = Pi Delta^{mu nu} + pi^{mu nu} and |X| its norm in the fluid rest
// frame, sqrt(h_{mu a} h_{nu b} X^{mu nu} X^{a b}) with h = 2 u u - g: equal to
// sqrt(X^{mu nu} X_{mu nu}) for a tensor transverse to u, and positive where
// the evolved pi is not (X:X alone can vanish or turn negative there).  With
// w^l = pi^{l m} u_m (the bulk part is transverse), |X|^2 = X:X - 4 w.w +
// 4 (u.w)^2;
// P = P0 + Pi (the shorthand of Sec. 2.4 that Eq. rho uses),
// the eta row of pi.u taken in the tetrad (times sqrt(g33)); pi (and Pi
// when regulate_bulk) are multiplied by tanh(rho)/rho.
template <bool CART>
__device__ __forceinline__ double regulate(const Phys &P, double tau, double q[NQ], double e,
                                           double p0, const double u[4])
{
    const double g33 = CART ? 1.0 : tau * tau;
    const double glo[4] = {1.0, -1.0, -1.0, -g33};
    const double ghi[4] = {1.0, -1.0, -1.0, -1.0 / g33};
    const double Pi = P.bulk ? q[BPI] : 0.0;
    double BB = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int n = m; n < 4; ++n) {
            const double B = Pi * ((m == n ? ghi[m] : 0.0) - u[m] * u[n]) + q[pi_index(m, n)];
            BB += (m == n ? 1.0 : 2.0) * glo[m] * glo[n] * B * B;
        }
    }
    const double ul[4] = {u[0], -u[1], -u[2], -g33 * u[3]};
    double w[4], ww = 0.0, uw = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        w[l] = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) w[l] += q[pi_index(l, m)] * ul[m];
        ww += glo[l] * w[l] * w[l];
        uw += ul[l] * w[l];
    }
    const double nB = sqrt(fmax(BB - 4.0 * ww + 4.0 * uw * uw, 0.0));
    const double Pc = p0 + Pi;
    double rho = nB / (P.rho_max * sqrt(e * e + 3.0 * Pc * Pc));
    if (nB > 0.0) {
        const double tr = q[PTT] - q[PXX] - q[PYY] - g33 * q[PEE];
        const double lim = 1.0 / (P.xi0 * P.rho_max * nB);
        rho = fmax(rho, fabs(tr) * lim);
        double r3 = 0.0;
#pragma unroll
        for (int l = 0; l < 4; ++l) r3 = fmax(r3, fabs(w[l]) * (l == 3 ? sqrt(g33) : 1.0));
        rho = fmax(rho, r3 * lim);
    }
    const double fac = rho > 0.0 ? tanh(rho) / rho : 1.0;
#pragma unroll
    for (int c = PTT; c <= PEE; ++c) q[c] *= fac;
    if (P.regulate_bulk) q[BPI] *= fac;
    return fac;
}

// ------------------------------------------------------ reduced state ---
// Sec. 2.4: u_mu pi^{mu nu} = 0 and g_{mu nu} pi^{mu nu} = 0 leave five
// components of pi independent.  Given pi^{xx}, pi^{xy}, pi^{x eta}, pi^{yy},
// pi^{y eta} and the flow (v^i = u^i / u^tau, g33 = tau^2 or 1):
//   each row of the orthogonality relation, pi^{m tau} = pi^{m x} v^x +
//   pi^{m y} v^y + g33 pi^{m eta} v^eta (m = x, y, eta, then tau), and the
//   trace pi^{tau tau} = pi^{xx} + pi^{yy} + g33 pi^{eta eta} fix pi^{eta eta}
//   first (Eq. pi_etaeta): inserting the rows into the trace gives
//   g33 (1 - g33 v_eta^2) pi^{eta eta} = pi^{xx}(v_x^2 - 1) + pi^{yy}(v_y^2 - 1)
//     + 2 pi^{xy} v_x v_y + 2 g33 v_eta (pi^{x eta} v_x + pi^{y eta} v_y),
//   then pi^{tau eta}, pi^{tau y}, pi^{tau x} and pi^{tau tau} (Eq. pi_tautau
//   and the relations after it).
// q holds the ten pi components at PTT..PEE; the five dependent ones are written.
template <bool CART>
__device__ __forceinline__ void pi_dependent_of(double tau, const double u[4], double q[NQ])
{
    const double g33 = CART ? 1.0 : tau * tau;
    const double iut = 1.0 / u[0];
    const double vx = u[1] * iut, vy = u[2] * iut, ve = u[3] * iut;
    const double a = q[PXX], b = q[PXY], c = q[PXE], d = q[PYY], f = q[PYE];
    const double rhs = a * (vx * vx - 1.0) + d * (vy * vy - 1.0) + 2.0 * b * vx * vy
                       + 2.0 * g33 * ve * (c * vx + f * vy);
    const double pee = rhs / (g33 * (1.0 - g33 * ve * ve));
    const double pte = c * vx + f * vy + g33 * pee * ve;
    const double pty = b * vx + d * vy + g33 * f * ve;
    const double ptx = a * vx + b * vy + g33 * c * ve;
    q[PEE] = pee;
    q[PTE] = pte;
    q[PTY] = pty;
    q[PTX] = ptx;
    q[PTT] = ptx * vx + pty * vy + g33 * pte * ve;
}

// components of q that the reduced state does not evolve
__host__ __device__ __forceinline__ bool pi_is_dependent(int c)
{
    return (c >= PTT && c <= PTE) || c == PEE;
}

// ---------------------------------------------------------------- minmod --
// generalized minmod of Sec. 3.1 on undivided differences; sgn(0) = 0.
// R is the arithmetic type (double, or float for the mixed-precision state).
// The nested form minmod(theta a, minmod((a + b)/2, theta b)), a = q0 - qm,
// b = qp - q0 (with a + b taken as qp - qm), equals
// s min(theta |a|, |qp - qm|/2, theta |b|) with s = (sgn a + sgn b)/2: when a
// and b share a sign so does qp - qm, and otherwise both forms give zero.
// One sign factor and two minima instead of two of each.
template <typename R>
__device__ __forceinline__ R slope(R qm, R q0, R qp, R theta)
{
    const R a = q0 - qm, b = qp - q0;
    const R s = copysign(R(0.5), a) + copysign(R(0.5), b);
    return s * fmin(fmin(fabs(theta * a), fabs(R(0.5) * (qp - qm))), fabs(theta * b));
}

// the limiter of a kernel instantiated for theta = 1 (T1) or any theta.  For
// theta = 1 the middle argument |qp - qm|/2 never decides: when a and b share
// a sign, |qp - qm| >= 2 min(|a|, |b|) exactly, and rounding is monotone, so
// fl(qp - qm)/2 >= min(fl|a|, fl|b|); the result is s min(|a|, |b|), bit for
// bit what slope() returns, with five operations fewer.
template <bool T1, typename R>
__device__ __forceinline__ R limited(R qm, R q0, R qp, R theta)
{
    if (T1) {
        const R a = q0 - qm, b = qp - q0;
        const R s = copysign(R(0.5), a) + copysign(R(0.5), b);
        return s * fmin(fabs(a), fabs(b));
    }
    return slope(qm, q0, qp, theta);
}

// ------------------------------------------------- relaxation sources ----
// zeta/s(x), x = T / T_c, of Sec. 2.2 (Eq. zetas): near T_c a parabola, above
// 1.05 T_c two decaying exponentials over the QGP value 0.001, below 0.995 T_c
// two over the hadron-gas value 0.03 (the printed range of the parabola is
// garbled; it lies between the two tails)
__device__ __forceinline__ double zeta_over_s_paper(double x)
{
    const double y = x - 1.0;
    if (x > 1.05) return 0.9 * exp(-y / 0.025) + 0.25 * exp(-y / 0.13) + 0.001;
    if (x < 0.995) return 0.9 * exp(y / 0.0025) + 0.22 * exp(y / 0.022) + 0.03;
    return (-13.77 * x + 27.55) * x - 13.45;
}

// Right-hand side J of the dissipative components (App. B):
//   S_pi + G_pi = [2 (eta/tau_pi) sigma - pi/tau_pi - I_pi - G^{mu nu}] / u^tau + pi d_i v^i
//   S_Pi        = [-(zeta/tau_Pi) theta - Pi/tau_Pi - I_Pi] / u^tau + Pi d_i v^i
// with I_pi = I1 + (4/3) I2 - I3 + (tau_pipi/tau_pi) I4 - (6/5) Pi sigma,
//      I_Pi = (2/3) Pi theta - (8/5)(1/3 - c_s^2) pi:sigma  (Sec. 2.2, 2.4),
// G^{mu nu} = u^a Gamma^mu_{ab} pi^{b nu} + (mu <-> nu).
// C[a][m] = partial_a u^m on entry (a: tau, x, y, eta); pv holds the ten pi
// components in the order of q (pi^{tau tau} first).  Each result is handed
// to emit(c, q_c, J_c) as soon as it is known (c: index in q).  Arithmetic
// in R.
// Kinematics of the flow (Sec. 2.4, App. A) from C[a][m] = partial_a u^m
// (a: tau, x, y, eta): on return C holds the covariant derivative u^m_{;a},
// th = theta, Du = D u^m, Dl = D u_m, sg the ten components of sigma^{mu nu}
// in the order of q's pi, om the antisymmetric omega^{mu nu} for m < n in the
// order (01, 02, 03, 12, 13, 23).  Arithmetic in R.
template <bool CART, typename R>
__device__ __forceinline__ void flow_kinematics(R tau, const R u[4], R C[4][4], R &th, R Du[4], R Dl[4],
                                                R sg[10], R om[6])
{
    const R g33 = CART ? R(1) : tau * tau;
    const R inv_tau = R(1) / tau;
    const R glo[4] = {R(1), R(-1), R(-1), -g33};
    const R ghi[4] = {R(1), R(-1), R(-1), R(-1) / g33};
    // covariant derivative C[a][m] = u^m_{;a}
    if (!CART) {
        C[3][0] += tau * u[3];          // Gamma^tau_{eta eta} u^eta
        C[0][3] += u[3] * inv_tau;      // Gamma^eta_{tau eta} u^eta
        C[3][3] += u[0] * inv_tau;      // Gamma^eta_{eta tau} u^tau
    }
    th = C[0][0] + C[1][1] + C[2][2] + C[3][3];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        Du[m] = u[0] * C[0][m] + u[1] * C[1][m] + u[2] * C[2][m] + u[3] * C[3][m];
        Dl[m] = glo[m] * Du[m];
    }
    // sigma (10) and omega (6) from nabla^m u^n = g^{mm} C[m][n] - u^m D u^n
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = m; n < 4; ++n) {
            const R a = ghi[m] * C[m][n] - u[m] * Du[n];
            const R b = ghi[n] * C[n][m] - u[n] * Du[m];
            const R Dmn = (m == n ? ghi[m] : R(0)) - u[m] * u[n];
            sg[pi_index(m, n) - PTT] = R(0.5) * (a + b) - th * R(1.0 / 3.0) * Dmn;
        }
    int k = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = m + 1; n < 4; ++n) {
            const R a = ghi[m] * C[m][n] - u[m] * Du[n];
            const R b = ghi[n] * C[n][m] - u[n] * Du[m];
            om[k++] = R(0.5) * (a - b);
        }
}

template <bool CART, typename R, typename Emit>
__device__ __forceinline__ void relaxation_sources(const Phys &P, double tau_d, const R pv[10],
                                                   R Pi, R e, R p0, R cs2, R T, const R u[4],
                                                   R C[4][4], R divv, Emit &&emit)
{
    const R tau = R(tau_d);
    const R g33 = CART ? R(1) : tau * tau;
    const R inv_tau = R(1) / tau;
    const R glo[4] = {R(1), R(-1), R(-1), -g33};
    const R ghi[4] = {R(1), R(-1), R(-1), R(-1) / g33};
    R th, Du[4], Dl[4], sg[10], om[6];
    flow_kinematics<CART, R>(tau, u, C, th, Du, Dl, sg, om);
    auto SG = [&](int m, int n) -> R { return sg[pi_index(m, n) - PTT]; };
    auto OM = [&](int m, int n) -> R {
        if (m == n) return R(0);
        const int a = m < n ? m : n, b = m < n ? n : m;
        const int k = a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
        return m < n ? om[k] : -om[k];
    };
    auto PI = [&](int m, int n) -> R { return pv[pi_index(m, n) - PTT]; };
    R pis = R(0);   // pi^{mu nu} sigma_{mu nu}
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = m; n < 4; ++n)
            pis += (m == n ? R(1) : R(2)) * glo[m] * glo[n] * PI(m, n) * SG(m, n);
    const R inv_ut = R(1) / u[0];

    if (P.shear) {
        R av[4];   // a^m = pi^{m l} D u_l
#pragma unroll
        for (int m = 0; m < 4; ++m)
            av[m] = PI(m, 0) * Dl[0] + PI(m, 1) * Dl[1] + PI(m, 2) * Dl[2] + PI(m, 3) * Dl[3];
        const R inv_tpi = T / (R(5) * R(P.eta_s));
        const R eta_tpi = (e + p0) * R(0.2);
        const R h03 = CART ? R(0) : tau * u[3];     // u^a Gamma^tau_{a eta}
        const R h30 = CART ? R(0) : u[3] * inv_tau; // u^a Gamma^eta_{a tau}
        const R h33 = CART ? R(0) : u[0] * inv_tau; // u^a Gamma^eta_{a eta}
        const R taupipi = R(P.taupipi);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = m; n < 4; ++n) {
                R I3 = R(0), c4 = R(0);
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    // pi^{m l} g_ll omega^{n l} + (m <-> n);  pi^{m l} g_ll sigma^{n l} + (m <-> n)
                    I3 += glo[l] * (PI(m, l) * OM(n, l) + PI(n, l) * OM(m, l));
                    c4 += glo[l] * (PI(m, l) * SG(n, l) + PI(n, l) * SG(m, l));
                }
                const R I1 = u[n] * av[m] + u[m] * av[n];
                const R I4 = R(0.5) * c4 - ((m == n ? ghi[m] : R(0)) - u[m] * u[n]) * pis * R(1.0 / 3.0);
                const R s = SG(m, n), pmn = PI(m, n);
                const R Ipi = I1 + R(4.0 / 3.0) * th * pmn - I3 + taupipi * I4 - R(1.2) * Pi * s;
                R G = R(0);
                if (!CART) {
                    const R hm = (m == 0 ? h03 * PI(3, n) : R(0))
                               + (m == 3 ? h30 * PI(0, n) + h33 * PI(3, n) : R(0));
                    const R hn = (n == 0 ? h03 * PI(3, m) : R(0))
                               + (n == 3 ? h30 * PI(0, m) + h33 * PI(3, m) : R(0));
                    G = hm + hn;
                }
                const R rhs = R(2) * eta_tpi * s - pmn * inv_tpi - Ipi - G;
                emit(pi_index(m, n), pmn, rhs * inv_ut + pmn * divv);
            }
    }
    if (P.bulk) {
        const R d = R(1.0 / 3.0) - cs2;
        // zeta / tau_Pi = 15 d^2 (e + P) in both models: 1/tau_Pi = 15 d^2 T / (zeta/s)
        const R inv_tPi = P.zeta_model == 1
            ? R(15) * d * d * T / R(P.zeta_coef * zeta_over_s_paper((double)T / P.zeta_tc))
            : R(15) * d * T / R(P.zeta_coef);
        const R zeta_tPi = R(15) * d * d * (e + p0);
        const R IPi = R(2.0 / 3.0) * Pi * th - R(1.6) * d * pis;
        emit(BPI, Pi, (-zeta_tPi * th - Pi * inv_tPi - IPi) * inv_ut + Pi * divv);
    }
}

// Second-order inverse Reynolds numbers of Sec. 7 (Eq. inverseReynoldsNumbers2)
// of one cell, with the terms of Eq. 14_moment_terms that the relaxation
// equations keep (no particle diffusion) and the coefficients of Sec. 2.2:
//   J^{mu nu} / tau_pi = I3 - (4/3) theta pi - (tau_pipi/tau_pi) I4 + (6/5) Pi sigma,
//   J / tau_Pi         = -(2/3) Pi theta + (8/5)(1/3 - c_s^2) pi^{mu nu} sigma_{mu nu},
// I3 = 2 pi_l^<mu omega^nu>l, I4 = pi^{l<mu} sigma^{nu>}_l as in relaxation_sources;
// with eta / tau_pi = (e + P0)/5 and zeta / tau_Pi = 15 (1/3 - c_s^2)^2 (e + P0)
// the relaxation times cancel:
//   r2pi = sqrt(J:J) / (2 eta sqrt(sigma:sigma)),  r2Pi = |J| / (zeta |theta|);
// 0 where the quantity is not evolved or the numerator vanishes, +inf where
// only the denominator does.  C as for flow_kinematics.  FP64.
template <bool CART>
__device__ __forceinline__ void second_order_reynolds(const Phys &P, double tau, const double pv[10],
                                                      double Pi, double e, double p0, double cs2,
                                                      const double u[4], double C[4][4], double &r2pi,
                                                      double &r2Pi)
{
    const double g33 = CART ? 1.0 : tau * tau;
    const double glo[4] = {1.0, -1.0, -1.0, -g33};
    const double ghi[4] = {1.0, -1.0, -1.0, -1.0 / g33};
    double th, Du[4], Dl[4], sg[10], om[6];
    flow_kinematics<CART, double>(tau, u, C, th, Du, Dl, sg, om);
    auto SG = [&](int m, int n) -> double { return sg[pi_index(m, n) - PTT]; };
    auto OM = [&](int m, int n) -> double {
        if (m == n) return 0.0;
        const int a = m < n ? m : n, b = m < n ? n : m;
        const int k = a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
        return m < n ? om[k] : -om[k];
    };
    auto PI = [&](int m, int n) -> double { return pv[pi_index(m, n) - PTT]; };
    double pis = 0.0, XX = 0.0, SS = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = m; n < 4; ++n) {
            const double w = (m == n ? 1.0 : 2.0) * glo[m] * glo[n];
            pis += w * PI(m, n) * SG(m, n);
            SS += w * SG(m, n) * SG(m, n);
        }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = m; n < 4; ++n) {
            double I3 = 0.0, c4 = 0.0;
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                I3 += glo[l] * (PI(m, l) * OM(n, l) + PI(n, l) * OM(m, l));
                c4 += glo[l] * (PI(m, l) * SG(n, l) + PI(n, l) * SG(m, l));
            }
            const double I4 = 0.5 * c4 - ((m == n ? ghi[m] : 0.0) - u[m] * u[n]) * pis * (1.0 / 3.0);
            const double X = I3 - (4.0 / 3.0) * th * PI(m, n) - P.taupipi * I4 + 1.2 * Pi * SG(m, n);
            XX += (m == n ? 1.0 : 2.0) * glo[m] * glo[n] * X * X;
        }
    r2pi = 0.0;
    if (P.shear) {
        const double num = sqrt(fabs(XX));
        r2pi = num == 0.0 ? 0.0 : num / (0.4 * (e + p0) * sqrt(fabs(SS)));
    }
    r2Pi = 0.0;
    if (P.bulk) {
        const double d = 1.0 / 3.0 - cs2;
        const double num = fabs(-(2.0 / 3.0) * Pi * th + 1.6 * d * pis);
        r2Pi = num == 0.0 ? 0.0 : num / (15.0 * d * d * (e + p0) * fabs(th));
    }
}

}  // namespace ktd
