// kt_main.hip -- kernels and C ABI of the KT/Heun step library (gfx950, FP64).
//
// Bazow, Heinz & Strickland, arXiv:1608.06577.  One Heun step (Sec. 3.1,
// Eqs. step1-finalStep with s = 2) in the order of Sec. 4.3:
//   stage 1  q*      = q^n + dtau C[q^n; e^n, u^n, u^{n-1}]        (tau^n)
//   recover  (e*, u*) from q*, regulate q*                          (tau^{n+1})
//   stage 2  q^{n+1} = (q^n + q* + dtau C[q*; e*, u*, u^n]) / 2     (tau^{n+1})
//   recover  (e, u)^{n+1} from q^{n+1}, regulate                    (tau^{n+1})
// C[q] (Sec. 3.1, Eq. semiDiscreteKT) = -sum_d (H_{+1/2} - H_{-1/2}) / d_d + J,
// with the KT flux H (Eq. Hflux), local speed a = max|v_d| over the two
// reconstructed states (Eq. ax; the face primitives come from inverting
// q^+ and q^-), and the source J of App. B.
//
// Memory: structure of arrays over the physical cells (x fastest), one
// workspace carved into q (15), q* (15), three rotating u buffers (4 each),
// e (1), the EOS table and small reduction buffers.  q^{n+1} overwrites q^n
// in place (each cell reads only its own q^n in stage 2).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "kt.h"
#include "kt_device.hpp"

using namespace ktd;

namespace {

constexpr int BX = 64, BY = 4;   // one wavefront per row of x

// ------------------------------------------------------------------ grid --

struct Fields {       // base pointers; component c of an array is base + c * stride
    const double *q;
    const double *e;
    const double *u;
    const double *up;
};

__device__ __forceinline__ int wrap(int v, int n, int periodic)
{
    if (v < 0) return periodic ? ((v % n) + n) % n : 0;
    if (v >= n) return periodic ? v % n : n - 1;
    return v;
}

__device__ __forceinline__ long long lin(const Phys &P, int i, int j, int k)
{
    return ((long long)k * P.ny + j) * P.nx + i;
}

// neighbour of (i,j,k) at offset o along axis d
__device__ __forceinline__ long long nb(const Phys &P, int i, int j, int k, int d, int o)
{
    if (d == 0) return lin(P, wrap(i + o, P.nx, P.periodic[0]), j, k);
    if (d == 1) return lin(P, i, wrap(j + o, P.ny, P.periodic[1]), k);
    return lin(P, i, j, wrap(k + o, P.neta, P.periodic[2]));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ void count_add(unsigned long long *ctr, int which, long long v)
{
    const long long s = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && s != 0) atomicAdd(ctr + which, (unsigned long long)s);
}

// ------------------------------------------------------------ KT flux ----

// H along axis d through the face between cells o and o+1 (o = -1: i-1/2,
// o = 0: i+1/2) of cell (i,j,k), accumulated into acc with sign sgn/h.
template <bool CART>
__device__ __forceinline__ void face_flux(const Phys &P, const Eos &E, double tau,
                                          const double *__restrict__ q, int i, int j, int k,
                                          int d, int o, double w, double acc[NQ], int &iters)
{
    const long long s0 = nb(P, i, j, k, d, o - 1), s1 = nb(P, i, j, k, d, o);
    const long long s2 = nb(P, i, j, k, d, o + 1), s3 = nb(P, i, j, k, d, o + 2);
    double qm[NQ], qp[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
        const double *qc = q + c * P.stride;
        const double a0 = qc[s0], a1 = qc[s1], a2 = qc[s2], a3 = qc[s3];
        qm[c] = a1 + 0.5 * slope(a0, a1, a2, P.theta);   // q^- : left side of the face
        qp[c] = a2 - 0.5 * slope(a1, a2, a3, P.theta);   // q^+ : right side of the face
    }
    const double Pim = P.bulk ? qm[BPI] : 0.0, Pip = P.bulk ? qp[BPI] : 0.0;
    double em, ep, um[4], upl[4];
    int im, ip;
    recover<CART>(P, E, tau, qm[TT], qm[TX], qm[TY], qm[TE], qm[PTT], qm[PTX], qm[PTY], qm[PTE],
                  Pim, em, um, im);
    recover<CART>(P, E, tau, qp[TT], qp[TX], qp[TY], qp[TE], qp[PTT], qp[PTX], qp[PTY], qp[PTE],
                  Pip, ep, upl, ip);
    iters += im + ip;
    const double vm = um[d + 1] / um[0], vp = upl[d + 1] / upl[0];
    const double a = fmax(fabs(vm), fabs(vp));
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
        const double H = 0.5 * (vp * qp[c] + vm * qm[c]) - 0.5 * a * (qp[c] - qm[c]);
        acc[c] += w * H;
    }
}

// A^{i nu} = T^{i nu} - v^i T^{tau nu} of one cell for axis i = d+1 (Eqs. Ttt-Tij):
//   A^{i tau} = P v^i + pi^{i tau} - v^i pi^{tau tau}
//   A^{i j}   = -P g^{ij} + pi^{ij} - v^i pi^{tau j}
template <bool CART>
__device__ __forceinline__ void nonadvective_row(const Phys &P, const Eos &E, double tau,
                                                 const Fields &F, long long s, int d,
                                                 double A[4])
{
    const long long S = P.stride;
    const double e = F.e[s];
    const double Pc = eos_p(E, e) + (P.bulk ? F.q[BPI * S + s] : 0.0);
    const double v = F.u[(d + 1) * S + s] / F.u[s];
    const int ii = d + 1;
    double pr[4], p0[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        pr[n] = P.shear ? F.q[pi_index(ii, n) * S + s] : 0.0;
        p0[n] = P.shear ? F.q[pi_index(0, n) * S + s] : 0.0;
    }
    const double gii = ii == 3 ? (CART ? -1.0 : -1.0 / (tau * tau)) : -1.0;
    A[0] = Pc * v + pr[0] - v * p0[0];
#pragma unroll
    for (int n = 1; n < 4; ++n) A[n] = (n == ii ? -Pc * gii : 0.0) + pr[n] - v * p0[n];
}

// C[q] at one cell (Sec. 3.1, Eq. semiDiscreteKT with J of App. B)
template <bool CART>
__device__ __forceinline__ void cell_rhs(const Phys &P, const Eos &E, double tau, const Fields &F,
                                         int i, int j, int k, double out[NQ], int &fiters)
{
    const long long S = P.stride;
    const long long s = lin(P, i, j, k);
    const double invh[3] = {P.inv_dx, P.inv_dy, P.inv_deta};
#pragma unroll
    for (int c = 0; c < NQ; ++c) out[c] = 0.0;
    // flux divergence
    for (int d = 0; d < 3; ++d) {
        face_flux<CART>(P, E, tau, F.q, i, j, k, d, -1, invh[d], out, fiters);
        face_flux<CART>(P, E, tau, F.q, i, j, k, d, 0, -invh[d], out, fiters);
    }
    // cell state
    double q[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) q[c] = F.q[c * S + s];
    if (!P.shear)
        for (int c = PTT; c <= PEE; ++c) q[c] = 0.0;
    const double e = F.e[s];
    double u[4], du[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        u[m] = F.u[m * S + s];
        du[0][m] = (u[m] - F.up[m * S + s]) * P.inv_dtau;
    }
    double p0, cs2, T;
    eos_eval(E, e, p0, cs2, T);
    const double Pi = P.bulk ? q[BPI] : 0.0;
    const double Pc = p0 + Pi;
    // central differences (Sec. 3.1): d_i u^m, d_i v^i, S_c = -d_i A^{i nu}
    double divv = 0.0, Sc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
        const long long sp = nb(P, i, j, k, d, 1), sm = nb(P, i, j, k, d, -1);
        const double hh = 0.5 * invh[d];
#pragma unroll
        for (int m = 0; m < 4; ++m) du[d + 1][m] = (F.u[m * S + sp] - F.u[m * S + sm]) * hh;
        divv += (F.u[(d + 1) * S + sp] / F.u[sp] - F.u[(d + 1) * S + sm] / F.u[sm]) * hh;
        double Ap[4], Am[4];
        nonadvective_row<CART>(P, E, tau, F, sp, d, Ap);
        nonadvective_row<CART>(P, E, tau, F, sm, d, Am);
#pragma unroll
        for (int n = 0; n < 4; ++n) Sc[n] -= (Ap[n] - Am[n]) * hh;
    }
    // geometric source of the conservation law (App. B): G^tau = -(T^tt + tau^2 T^ee)/tau,
    // G^x = -T^tx/tau, G^y = -T^ty/tau, G^eta = -3 T^te/tau, with
    // tau^2 T^ee = tau^2 v^eta (T^te - pi^te) + P + tau^2 pi^ee.
    if (!CART) {
        const double inv_tau = 1.0 / tau, t2 = tau * tau;
        const double ve = u[3] / u[0];
        const double t2Tee = t2 * (ve * (q[TE] - q[PTE]) + q[PEE]) + Pc;
        out[TT] += Sc[0] - (q[TT] + t2Tee) * inv_tau;
        out[TX] += Sc[1] - q[TX] * inv_tau;
        out[TY] += Sc[2] - q[TY] * inv_tau;
        out[TE] += Sc[3] - 3.0 * q[TE] * inv_tau;
    } else {
#pragma unroll
        for (int n = 0; n < 4; ++n) out[n] += Sc[n];
    }
    if (P.shear || P.bulk) {
        double J[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) J[c] = 0.0;
        relaxation_sources<CART>(P, tau, q, e, p0, cs2, T, u, du, divv, J);
        for (int c = PTT; c < NQ; ++c) out[c] += J[c];
    }
    if (!P.shear)
        for (int c = PTT; c <= PEE; ++c) out[c] = 0.0;
    if (!P.bulk) out[BPI] = 0.0;
}

// stage 1: out = q + dtau C[q];  stage 2: out = (qn + q + dtau C[q]) / 2 (out may alias qn)
template <bool CART, bool STAGE2>
__global__ __launch_bounds__(BX *BY) void stage_kernel(Phys P, Eos E, double tau, Fields F,
                                                         const double *qn, double *out,
                                                         unsigned long long *ctr)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    const bool active = i < P.nx && j < P.ny;
    int fiters = 0;
    if (active) {
        double C[NQ];
        cell_rhs<CART>(P, E, tau, F, i, j, k, C, fiters);
        const long long s = lin(P, i, j, k);
        const long long S = P.stride;
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
            const double qs = F.q[c * S + s] + P.dtau * C[c];
            out[c * S + s] = STAGE2 ? 0.5 * (qn[c * S + s] + qs) : qs;
        }
    }
    count_add(ctr, C_ITERS_FACES, fiters);
    count_add(ctr, C_REC_FACES, active ? 6 * 2 : 0);
}

// recovery of every cell at tau, then the regulator and the floor reset
template <bool CART>
__global__ __launch_bounds__(256) void recover_kernel(Phys P, Eos E, double tau, double *q,
                                                      double *e_out, double *u_out,
                                                      int do_regulate,
                                                      unsigned long long *ctr)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long S = P.stride;
    int it = 0, fl = 0;
    if (s < P.ncell) {
        double qc[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) qc[c] = q[c * S + s];
        const double Pi = P.bulk ? qc[BPI] : 0.0;
        double e, u[4];
        fl = recover<CART>(P, E, tau, qc[TT], qc[TX], qc[TY], qc[TE], qc[PTT], qc[PTX], qc[PTY],
                           qc[PTE], Pi, e, u, it);
        e_out[s] = e;
#pragma unroll
        for (int m = 0; m < 4; ++m) u_out[m * S + s] = u[m];
        if ((fl & F_FLOOR) && P.floor_reset) {
#pragma unroll
            for (int c = 0; c < NQ; ++c) q[c * S + s] = c == TT ? P.e_floor : 0.0;
        } else if (do_regulate && P.regulate && P.shear) {
            const double p0 = eos_p(E, e);
            regulate<CART>(P, tau, qc, e, p0, u);
#pragma unroll
            for (int c = PTT; c < NQ; ++c) q[c * S + s] = qc[c];
        }
    }
    count_add(ctr, C_ITERS_CELLS, it);
    count_add(ctr, C_REC_CELLS, s < P.ncell ? 1 : 0);
    count_add(ctr, C_FLOOR, (fl & F_FLOOR) ? 1 : 0);
    count_add(ctr, C_CLAMP, (fl & F_CLAMP) ? 1 : 0);
    count_add(ctr, C_FALLBACK, (fl & F_FALLBACK) ? 1 : 0);
}

// T^{tau mu} from primitives (Sec. 2.4, Eqs. Ttt, Tti): (e+P) u^tau u^mu - P g^{tau mu} + pi^{tau mu}
struct PrimPtrs {
    const double *e;
    const double *u[4];
    const double *pi[10];
    const double *Pi;
};

__global__ __launch_bounds__(256) void tmunu_kernel(Phys P, Eos E, PrimPtrs in, double *q)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P.ncell) return;
    const long long S = P.stride;
    const double e = in.e[s];
    const double Pi = in.Pi[s];
    const double Pc = eos_p(E, e) + Pi;
    const double ut = in.u[0][s];
    const double w = (e + Pc) * ut;
#pragma unroll
    for (int m = 0; m < 4; ++m)   // pi^{tau m} are the first four of the ten
        q[m * S + s] = w * in.u[m][s] - (m == 0 ? Pc : 0.0) + in.pi[m][s];
#pragma unroll
    for (int c = 0; c < 10; ++c) q[(PTT + c) * S + s] = in.pi[c][s];
    q[BPI * S + s] = Pi;
}

struct RecIn {
    const double *in[9];
    double *e;
    double *u[4];
    int *iters;
    int *flags;
};

template <bool CART>
__global__ __launch_bounds__(256) void recover_standalone_kernel(Phys P, Eos E, double tau,
                                                                 long long n, RecIn R)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double Pi = (P.bulk && R.in[8]) ? R.in[8][s] : 0.0;
    double e, u[4];
    int it;
    const int fl = recover<CART>(P, E, tau, R.in[0][s], R.in[1][s], R.in[2][s], R.in[3][s],
                                 R.in[4][s], R.in[5][s], R.in[6][s], R.in[7][s], Pi, e, u, it);
    R.e[s] = e;
#pragma unroll
    for (int m = 0; m < 4; ++m) R.u[m][s] = u[m];
    if (R.iters) R.iters[s] = it;
    if (R.flags) R.flags[s] = fl;
}

// ---------------------------------------------------------- observables --
// per-block partial results, reduced by one block afterwards (deterministic)
enum : int {
    O_E = 0, O_MX, O_MY, O_ME,                  // sums
    O_EMAX, O_TMAX, O_VMAX, O_CFL, O_NORM, O_PIU, O_PITR,  // maxima
    O_NAN,                                      // count (as double)
    O_COUNT
};
constexpr int OBS_THREADS = 256;

template <bool CART>
__global__ __launch_bounds__(OBS_THREADS) void obs_partial_kernel(Phys P, Eos E, double tau,
                                                                  const double *q,
                                                                  const double *e,
                                                                  const double *u,
                                                                  double *partial)
{
    __shared__ double red[OBS_THREADS / 64][O_COUNT];
    const long long S = P.stride;
    double acc[O_COUNT];
#pragma unroll
    for (int o = 0; o < O_COUNT; ++o) acc[o] = 0.0;
    const double g33 = CART ? 1.0 : tau * tau;
    const double glo[4] = {1.0, -1.0, -1.0, -g33};
    const double invh[3] = {P.inv_dx, P.inv_dy, P.inv_deta};
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < P.ncell;
         s += (long long)gridDim.x * blockDim.x) {
        double qc[NQ], uc[4];
        bool finite = true;
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
            qc[c] = q[c * S + s];
            finite = finite && isfinite(qc[c]);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            uc[m] = u[m * S + s];
            finite = finite && isfinite(uc[m]);
        }
        const double ec = e[s];
        finite = finite && isfinite(ec);
        if (!finite) {
            acc[O_NAN] += 1.0;
            continue;
        }
        acc[O_E] += qc[TT];
        acc[O_MX] += qc[TX];
        acc[O_MY] += qc[TY];
        acc[O_ME] += qc[TE];
        double p0, cs2, T;
        eos_eval(E, ec, p0, cs2, T);
        acc[O_EMAX] = fmax(acc[O_EMAX], ec);
        acc[O_TMAX] = fmax(acc[O_TMAX], T);
        double cfl = 0.0, vmax = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = fabs(uc[d + 1] / uc[0]);
            vmax = fmax(vmax, d == 2 ? v * sqrt(g33) : v);
            cfl = fmax(cfl, v * invh[d]);
        }
        acc[O_VMAX] = fmax(acc[O_VMAX], vmax);
        acc[O_CFL] = fmax(acc[O_CFL], cfl * P.dtau);
        const double nrm = uc[0] * uc[0] - uc[1] * uc[1] - uc[2] * uc[2] - g33 * uc[3] * uc[3];
        acc[O_NORM] = fmax(acc[O_NORM], fabs(nrm - 1.0));
        if (P.shear) {
            double pp = 0.0, tr = 0.0, tv = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                double w = 0.0;
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const double x = qc[pi_index(m, n)];
                    pp += glo[m] * glo[n] * x * x;
                    w += x * glo[n] * uc[n];
                }
                tr += glo[m] * qc[pi_index(m, m)];
                tv = fmax(tv, fabs(w) * sqrt(fabs(glo[m])));
            }
            const double np = sqrt(fabs(pp));
            if (np > 0.0) {
                acc[O_PIU] = fmax(acc[O_PIU], tv / np);
                acc[O_PITR] = fmax(acc[O_PITR], fabs(tr) / np);
            }
        }
    }
    // block reduction: wave shuffles, then across the 4 waves in LDS
#pragma unroll
    for (int o = 0; o < O_COUNT; ++o) {
        double v = acc[o];
        const bool is_max = o >= O_EMAX && o <= O_PITR;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double w = __shfl_xor(v, off);
            v = is_max ? fmax(v, w) : v + w;
        }
        acc[o] = v;
    }
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int o = 0; o < O_COUNT; ++o) red[wid][o] = acc[o];
    __syncthreads();
    if (threadIdx.x < O_COUNT) {
        const int o = threadIdx.x;
        const bool is_max = o >= O_EMAX && o <= O_PITR;
        double v = red[0][o];
        for (int w = 1; w < OBS_THREADS / 64; ++w) v = is_max ? fmax(v, red[w][o]) : v + red[w][o];
        partial[(long long)blockIdx.x * O_COUNT + o] = v;
    }
}

__global__ void obs_final_kernel(const double *partial, int nblocks, double *out)
{
    const int o = threadIdx.x;
    if (o >= O_COUNT) return;
    const bool is_max = o >= O_EMAX && o <= O_PITR;
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        const double w = partial[(long long)b * O_COUNT + o];
        v = is_max ? fmax(v, w) : v + w;
    }
    out[o] = v;
}

constexpr int OBS_BLOCKS = 512;

}  // namespace

// ======================================================================
// Host side
// ======================================================================

struct kt_ctx {
    kt_params prm;
    Phys P;
    Eos E;
    hipStream_t stream;
    double *ws;
    double *q, *qs, *e, *u[3];   // u[cur], u[prev], u[star] by index below
    int ucur, uprev, ustar;
    double *tab;
    unsigned long long *ctr;
    double *partial, *obs;
    double tau;
    long long step;
    char err[512];
    // profiling: pooled event pairs recorded around launches
    bool prof;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    size_t ev_used;
};

static hipError_t prof_mark(kt_ctx *c, int kind, bool start)
{
    if (!c->prof) return hipSuccess;
    if (start) {
        if (c->ev_used + 2 > c->ev.size()) {
            for (int k = 0; k < 2; ++k) {
                hipEvent_t e;
                hipError_t r = hipEventCreate(&e);
                if (r != hipSuccess) return r;
                c->ev.push_back(e);
                c->ev_kind.push_back(0);
            }
        }
        c->ev_kind[c->ev_used] = kind;
    }
    hipError_t r = hipEventRecord(c->ev[c->ev_used], c->stream);
    c->ev_used += 1;
    return r;
}

static thread_local char g_err[512];

static kt_status fail(kt_ctx *c, kt_status s, const char *fmt, ...)
{
    char *dst = c ? c->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(ctx, call)                                                                     \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((ctx), KT_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
    } while (0)

static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static long long cell_stride(const kt_params *p)
{
    const long long n = (long long)p->nx * p->ny * p->neta;
    return (long long)round_up((size_t)n, 64);   // 512-byte aligned component arrays
}

struct Layout {
    size_t q, qs, u, e, tab, ctr, partial, obs, total;
};

static Layout layout(const kt_params *p, const kt_eos *eos)
{
    Layout L;
    const size_t S = (size_t)cell_stride(p) * sizeof(double);
    size_t off = 0;
    L.q = off;  off += 15 * S;
    L.qs = off; off += 15 * S;
    L.u = off;  off += 12 * S;
    L.e = off;  off += S;
    L.tab = off; off += round_up((size_t)(eos->conformal ? 1 : eos->n) * 3 * sizeof(double), 256);
    L.ctr = off; off += 256;
    L.partial = off; off += round_up((size_t)OBS_BLOCKS * O_COUNT * sizeof(double), 256);
    L.obs = off; off += 256;
    L.total = off;
    return L;
}

static const char *check_args(const kt_params *p, const kt_eos *eos)
{
    if (!p || !eos) return "null params or eos";
    if (p->nx < 1 || p->ny < 1 || p->neta < 1) return "grid sizes must be >= 1";
    if ((long long)p->nx * p->ny * p->neta > (1LL << 31)) return "grid too large";
    if (!(p->dx > 0) || !(p->dy > 0) || !(p->deta > 0)) return "cell sizes must be > 0";
    if (!(p->dtau > 0)) return "dtau must be > 0";
    if (p->coords != KT_MILNE && p->coords != KT_CARTESIAN) return "coords must be KT_MILNE or KT_CARTESIAN";
    if (p->coords == KT_MILNE && !(p->tau0 > 0)) return "tau0 must be > 0 in Milne coordinates";
    for (int d = 0; d < 3; ++d)
        if (p->bc[d] != KT_BC_OUTFLOW && p->bc[d] != KT_BC_PERIODIC) return "bc must be outflow or periodic";
    if (!(p->theta >= 1.0 && p->theta <= 2.0)) return "theta must lie in [1, 2]";
    if (!(p->eta_over_s >= 0) || !(p->zeta_coef >= 0) || !(p->taupipi >= 0)) return "transport parameters must be >= 0";
    if (p->regulate && (!(p->xi0 > 0) || !(p->rho_max > 0))) return "regulator constants must be > 0";
    if (!(p->e_floor > 0)) return "e_floor must be > 0";
    if (!(p->m2_delta > 0 && p->m2_delta < 1)) return "m2_delta must lie in (0, 1)";
    if (!(p->newton_tol > 0) || p->newton_max < 1) return "Newton tolerance and iteration limit must be positive";
    if (eos->conformal) {
        if (!(eos->a_sb > 0)) return "conformal EOS needs a_sb > 0";
    } else {
        if (eos->n < 2) return "EOS table needs n >= 2";
        if (!eos->p || !eos->cs2 || !eos->T) return "EOS table arrays are null";
        if (!(eos->dln_e > 0)) return "EOS table needs dln_e > 0";
    }
    return nullptr;
}

static void fill_phys(const kt_params *p, Phys &P)
{
    P.nx = p->nx; P.ny = p->ny; P.neta = p->neta;
    P.ncell = (long long)p->nx * p->ny * p->neta;
    P.stride = cell_stride(p);
    P.inv_dx = 1.0 / p->dx; P.inv_dy = 1.0 / p->dy; P.inv_deta = 1.0 / p->deta;
    P.dtau = p->dtau; P.inv_dtau = 1.0 / p->dtau;
    for (int d = 0; d < 3; ++d) P.periodic[d] = p->bc[d] == KT_BC_PERIODIC;
    P.theta = p->theta;
    P.eta_s = p->eta_over_s; P.zeta_coef = p->zeta_coef; P.taupipi = p->taupipi;
    P.shear = p->eta_over_s > 0; P.bulk = p->zeta_coef > 0;
    P.regulate = p->regulate != 0; P.regulate_bulk = p->regulate_bulk != 0;
    P.floor_reset = p->floor_resets_q != 0;
    P.xi0 = p->xi0; P.rho_max = p->rho_max;
    P.e_floor = p->e_floor; P.m2_delta = p->m2_delta; P.newton_tol = p->newton_tol;
    P.newton_max = p->newton_max;
}

template <typename K, typename... A>
static hipError_t launch(K kernel, dim3 g, dim3 b, hipStream_t st, A... args)
{
    hipLaunchKernelGGL(kernel, g, b, 0, st, args...);
    return hipGetLastError();
}

static dim3 cells_grid(const Phys &P)
{
    return dim3((P.nx + BX - 1) / BX, (P.ny + BY - 1) / BY, P.neta);
}

static dim3 linear_grid(long long n) { return dim3((unsigned)((n + 255) / 256)); }

static kt_status run_recover(kt_ctx *c, double tau, double *q, double *u_out, int regulate)
{
    const bool cart = c->prm.coords == KT_CARTESIAN;
    hipError_t e = prof_mark(c, 1, true);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "profiling event: %s", hipGetErrorString(e));
    e = cart ? launch(recover_kernel<true>, linear_grid(c->P.ncell), dim3(256), c->stream,
                                 c->P, c->E, tau, q, c->e, u_out, regulate, c->ctr)
                        : launch(recover_kernel<false>, linear_grid(c->P.ncell), dim3(256), c->stream,
                                 c->P, c->E, tau, q, c->e, u_out, regulate, c->ctr);
    if (e == hipSuccess) e = prof_mark(c, 1, false);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "recover kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

static kt_status run_stage(kt_ctx *c, bool stage2, double tau, const Fields &F, double *out)
{
    const bool cart = c->prm.coords == KT_CARTESIAN;
    const dim3 g = cells_grid(c->P), b(BX, BY);
    hipError_t e = prof_mark(c, 0, true);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "profiling event: %s", hipGetErrorString(e));
    if (cart)
        e = stage2 ? launch(stage_kernel<true, true>, g, b, c->stream, c->P, c->E, tau, F,
                            (const double *)c->q, out, c->ctr)
                   : launch(stage_kernel<true, false>, g, b, c->stream, c->P, c->E, tau, F,
                            (const double *)nullptr, out, c->ctr);
    else
        e = stage2 ? launch(stage_kernel<false, true>, g, b, c->stream, c->P, c->E, tau, F,
                            (const double *)c->q, out, c->ctr)
                   : launch(stage_kernel<false, false>, g, b, c->stream, c->P, c->E, tau, F,
                            (const double *)nullptr, out, c->ctr);
    if (e == hipSuccess) e = prof_mark(c, 0, false);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "stage kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

extern "C" {

const char *kt_status_string(kt_status s)
{
    switch (s) {
    case KT_OK: return "ok";
    case KT_E_ARG: return "invalid argument";
    case KT_E_ALLOC: return "workspace too small";
    case KT_E_HIP: return "HIP error";
    case KT_E_STATE: return "invalid state";
    case KT_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *kt_last_error(const kt_ctx *c) { return c ? c->err : g_err; }

size_t kt_workspace_bytes(const kt_params *p, const kt_eos *eos)
{
    if (check_args(p, eos)) return 0;
    return layout(p, eos).total;
}

kt_status kt_init(const kt_params *p, const kt_eos *eos, const kt_init_state *s0, void *d_ws,
                  size_t ws_bytes, hipStream_t stream, kt_ctx **out)
{
    if (!out) return fail(nullptr, KT_E_ARG, "out is null");
    *out = nullptr;
    if (const char *m = check_args(p, eos)) return fail(nullptr, KT_E_ARG, "%s", m);
    if (p->precision != KT_FP64)
        return fail(nullptr, KT_E_UNSUPPORTED, "only KT_FP64 is implemented in this build");
    if (!s0 || !d_ws) return fail(nullptr, KT_E_ARG, "null initial state or workspace");
    if (((uintptr_t)d_ws) % 256) return fail(nullptr, KT_E_ARG, "workspace must be 256-byte aligned");
    const bool have_q = s0->q[0] != nullptr;
    if (have_q) {
        for (int c = 0; c < 15; ++c)
            if (!s0->q[c]) return fail(nullptr, KT_E_ARG, "initial q[%d] is null", c);
    } else {
        if (!s0->e || !s0->Pi) return fail(nullptr, KT_E_ARG, "give either q or (e, u, pi, Pi)");
        for (int m = 0; m < 4; ++m)
            if (!s0->u[m]) return fail(nullptr, KT_E_ARG, "initial u[%d] is null", m);
        for (int c = 0; c < 10; ++c)
            if (!s0->pi[c]) return fail(nullptr, KT_E_ARG, "initial pi[%d] is null", c);
    }
    const bool have_up = s0->u_prev[0] != nullptr;
    if (have_up)
        for (int m = 1; m < 4; ++m)
            if (!s0->u_prev[m]) return fail(nullptr, KT_E_ARG, "u_prev[%d] is null", m);
    const Layout L = layout(p, eos);
    if (ws_bytes < L.total)
        return fail(nullptr, KT_E_ALLOC, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);

    kt_ctx *c = new (std::nothrow) kt_ctx();
    if (!c) return fail(nullptr, KT_E_ALLOC, "host allocation failed");
    c->prm = *p;
    fill_phys(p, c->P);
    c->stream = stream;
    char *base = (char *)d_ws;
    c->ws = (double *)d_ws;
    c->q = (double *)(base + L.q);
    c->qs = (double *)(base + L.qs);
    const long long S = c->P.stride;
    for (int b = 0; b < 3; ++b) c->u[b] = (double *)(base + L.u) + (size_t)4 * S * b;
    c->ucur = 0; c->uprev = 1; c->ustar = 2;
    c->e = (double *)(base + L.e);
    c->tab = (double *)(base + L.tab);
    c->ctr = (unsigned long long *)(base + L.ctr);
    c->partial = (double *)(base + L.partial);
    c->obs = (double *)(base + L.obs);
    c->tau = p->tau0;
    c->step = 0;

    // EOS table: per node p/e, T/e^{1/4}, c_s^2 (node e_i = exp(ln_e0 + i dln_e))
    c->E.conformal = eos->conformal != 0;
    c->E.inv_a = eos->conformal ? 1.0 / eos->a_sb : 0.0;
    c->E.n = eos->conformal ? 0 : eos->n;
    c->E.ln_e0 = eos->ln_e0;
    c->E.inv_dln = eos->conformal ? 0.0 : 1.0 / eos->dln_e;
    c->E.tab = c->tab;
    if (!eos->conformal) {
        double *h = (double *)malloc(sizeof(double) * 3 * eos->n);
        if (!h) { delete c; return fail(nullptr, KT_E_ALLOC, "host allocation failed"); }
        for (int i = 0; i < eos->n; ++i) {
            const double ei = exp(eos->ln_e0 + eos->dln_e * (double)i);
            h[3 * i] = eos->p[i] / ei;
            h[3 * i + 1] = eos->T[i] / sqrt(sqrt(ei));
            h[3 * i + 2] = eos->cs2[i];
        }
        hipError_t e1 = hipMemcpyAsync(c->tab, h, sizeof(double) * 3 * eos->n, hipMemcpyHostToDevice, stream);
        hipError_t e2 = hipStreamSynchronize(stream);
        free(h);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            kt_status st = fail(nullptr, KT_E_HIP, "EOS upload: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
            delete c;
            return st;
        }
    }
    hipError_t he = hipMemsetAsync(c->ctr, 0, 256, stream);
    if (he != hipSuccess) { delete c; return fail(nullptr, KT_E_HIP, "memset: %s", hipGetErrorString(he)); }

    // q^0
    const size_t bytes = sizeof(double) * (size_t)c->P.ncell;
    if (have_q) {
        for (int k = 0; k < 15; ++k) {
            he = hipMemcpyAsync(c->q + k * S, s0->q[k], bytes, hipMemcpyDeviceToDevice, stream);
            if (he != hipSuccess) break;
        }
    } else {
        PrimPtrs in;
        in.e = s0->e;
        for (int m = 0; m < 4; ++m) in.u[m] = s0->u[m];
        for (int k = 0; k < 10; ++k) in.pi[k] = s0->pi[k];
        in.Pi = s0->Pi;
        he = launch(tmunu_kernel, linear_grid(c->P.ncell), dim3(256), stream, c->P, c->E, in, c->q);
    }
    if (he != hipSuccess) { delete c; return fail(nullptr, KT_E_HIP, "initial state: %s", hipGetErrorString(he)); }
    // (e^0, u^0) and u^{-1}
    kt_status st = run_recover(c, c->tau, c->q, c->u[c->ucur], 0);
    if (st != KT_OK) { kt_status r = fail(nullptr, st, "%s", c->err); delete c; return r; }
    for (int m = 0; m < 4 && he == hipSuccess; ++m)
        he = hipMemcpyAsync(c->u[c->uprev] + m * S, have_up ? s0->u_prev[m] : c->u[c->ucur] + m * S,
                            bytes, hipMemcpyDeviceToDevice, stream);
    if (he == hipSuccess) he = hipStreamSynchronize(stream);
    if (he != hipSuccess) { delete c; return fail(nullptr, KT_E_HIP, "init: %s", hipGetErrorString(he)); }
    *out = c;
    return KT_OK;
}

kt_status kt_step(kt_ctx *c, int32_t n_steps)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (n_steps < 0) return fail(c, KT_E_ARG, "n_steps must be >= 0");
    const long long S = c->P.stride;
    for (int s = 0; s < n_steps; ++s) {
        const double tau0 = c->tau, tau1 = c->tau + c->prm.dtau;
        Fields F1 = {c->q, c->e, c->u[c->ucur], c->u[c->uprev]};
        kt_status st = run_stage(c, false, tau0, F1, c->qs);
        if (st != KT_OK) return st;
        st = run_recover(c, tau1, c->qs, c->u[c->ustar], 1);
        if (st != KT_OK) return st;
        Fields F2 = {c->qs, c->e, c->u[c->ustar], c->u[c->ucur]};
        st = run_stage(c, true, tau1, F2, c->q);
        if (st != KT_OK) return st;
        // u^{n-1} <- u^n; (e, u)^{n+1} into the freed buffer
        const int freed = c->uprev;
        st = run_recover(c, tau1, c->q, c->u[freed], 1);
        if (st != KT_OK) return st;
        c->uprev = c->ucur;
        c->ucur = freed;
        c->tau = tau1;
        c->step += 1;
    }
    (void)S;
    return KT_OK;
}

kt_status kt_recover(kt_ctx *c, int64_t n, double tau, const double *const in[9], double *e_out,
                     double *const u_out[4], int32_t *iters_out, int32_t *flags_out)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (n < 0) return fail(c, KT_E_ARG, "n must be >= 0");
    if (n == 0) return KT_OK;
    if (!in || !e_out || !u_out) return fail(c, KT_E_ARG, "null input or output arrays");
    for (int k = 0; k < 8; ++k)
        if (!in[k]) return fail(c, KT_E_ARG, "input %d is null", k);
    for (int m = 0; m < 4; ++m)
        if (!u_out[m]) return fail(c, KT_E_ARG, "u_out[%d] is null", m);
    if (c->prm.coords == KT_MILNE && !(tau > 0)) return fail(c, KT_E_ARG, "tau must be > 0");
    RecIn R;
    for (int k = 0; k < 9; ++k) R.in[k] = in[k];
    R.e = e_out;
    for (int m = 0; m < 4; ++m) R.u[m] = u_out[m];
    R.iters = iters_out;
    R.flags = flags_out;
    hipError_t e = c->prm.coords == KT_CARTESIAN
        ? launch(recover_standalone_kernel<true>, linear_grid(n), dim3(256), c->stream, c->P, c->E, tau, (long long)n, R)
        : launch(recover_standalone_kernel<false>, linear_grid(n), dim3(256), c->stream, c->P, c->E, tau, (long long)n, R);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "recover kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

kt_status kt_observables(kt_ctx *c, kt_obs *host_out, const kt_fields *dev_out)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    const long long S = c->P.stride;
    const size_t bytes = sizeof(double) * (size_t)c->P.ncell;
    hipError_t e = hipSuccess;
    if (dev_out) {
        if (dev_out->e) e = hipMemcpyAsync(dev_out->e, c->e, bytes, hipMemcpyDeviceToDevice, c->stream);
        for (int m = 0; m < 4 && e == hipSuccess; ++m) {
            if (dev_out->u[m])
                e = hipMemcpyAsync(dev_out->u[m], c->u[c->ucur] + m * S, bytes, hipMemcpyDeviceToDevice, c->stream);
            if (e == hipSuccess && dev_out->u_prev[m])
                e = hipMemcpyAsync(dev_out->u_prev[m], c->u[c->uprev] + m * S, bytes, hipMemcpyDeviceToDevice, c->stream);
        }
        for (int k = 0; k < 15 && e == hipSuccess; ++k)
            if (dev_out->q[k]) e = hipMemcpyAsync(dev_out->q[k], c->q + k * S, bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return fail(c, KT_E_HIP, "field export: %s", hipGetErrorString(e));
    }
    double res[O_COUNT];
    unsigned long long ctr[C_COUNT];
    if (host_out) {
        const bool cart = c->prm.coords == KT_CARTESIAN;
        e = cart ? launch(obs_partial_kernel<true>, dim3(OBS_BLOCKS), dim3(OBS_THREADS), c->stream, c->P, c->E, c->tau,
                          (const double *)c->q, (const double *)c->e, (const double *)c->u[c->ucur], c->partial)
                 : launch(obs_partial_kernel<false>, dim3(OBS_BLOCKS), dim3(OBS_THREADS), c->stream, c->P, c->E, c->tau,
                          (const double *)c->q, (const double *)c->e, (const double *)c->u[c->ucur], c->partial);
        if (e == hipSuccess)
            e = launch(obs_final_kernel, dim3(1), dim3(64), c->stream, (const double *)c->partial, OBS_BLOCKS, c->obs);
        if (e == hipSuccess) e = hipMemcpyAsync(res, c->obs, sizeof(res), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(ctr, c->ctr, sizeof(ctr), hipMemcpyDeviceToHost, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "observables: %s", hipGetErrorString(e));
    if (host_out) {
        memset(host_out, 0, sizeof(*host_out));
        const double vol = c->prm.dx * c->prm.dy * c->prm.deta * (c->prm.coords == KT_MILNE ? c->tau : 1.0);
        host_out->tau = c->tau;
        host_out->step = c->step;
        host_out->energy = res[O_E] * vol;
        host_out->momentum[0] = res[O_MX] * vol;
        host_out->momentum[1] = res[O_MY] * vol;
        host_out->momentum[2] = res[O_ME] * vol;
        host_out->e_max = res[O_EMAX];
        host_out->T_max = res[O_TMAX];
        host_out->v_max = res[O_VMAX];
        host_out->cfl = res[O_CFL];
        host_out->norm_err = res[O_NORM];
        host_out->pi_transverse = res[O_PIU];
        host_out->pi_trace = res[O_PITR];
        host_out->n_nan = (int64_t)res[O_NAN];
        host_out->newton_iters_cells = (int64_t)ctr[C_ITERS_CELLS];
        host_out->n_recover_cells = (int64_t)ctr[C_REC_CELLS];
        host_out->newton_iters_faces = (int64_t)ctr[C_ITERS_FACES];
        host_out->n_recover_faces = (int64_t)ctr[C_REC_FACES];
        host_out->n_floor = (int64_t)ctr[C_FLOOR];
        host_out->n_clamp = (int64_t)ctr[C_CLAMP];
        host_out->n_fallback = (int64_t)ctr[C_FALLBACK];
    }
    return KT_OK;
}

kt_status kt_profile_enable(kt_ctx *c, int32_t on)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    c->prof = on != 0;
    return KT_OK;
}

kt_status kt_profile_read(kt_ctx *c, kt_profile *out)
{
    if (!c || !out) return fail(c, KT_E_ARG, "null context or output");
    memset(out, 0, sizeof(*out));
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "profile sync: %s", hipGetErrorString(e));
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]);
        if (e != hipSuccess) return fail(c, KT_E_HIP, "profile events: %s", hipGetErrorString(e));
        const int k = c->ev_kind[i];
        out->ms[k] += ms;
        out->launches[k] += 1;
    }
    c->ev_used = 0;
    return KT_OK;
}

void kt_destroy(kt_ctx *c)
{
    if (!c) return;
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
