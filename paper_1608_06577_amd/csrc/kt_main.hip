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

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "kt.h"
#include "kt_device.hpp"
#include "kt_mlp.hpp"

using namespace ktd;

namespace {

constexpr int KC = 2;      // eta planes per flux block of a single event (2 or 4, the instantiated ones)

// ------------------------------------------------------------------ grid --

// Field pointers of one stage.  T^{tau mu} and u^mu are always FP64; the
// other components (pi, Pi), e, p and the face speeds have the storage type S
// (double, or float for the mixed-precision state).  u stays FP64 because
// the sources take differences of it (the backward difference in tau and
// central differences in space) that cancel several digits.  Component c of
// an array is at base + c * stride; qP holds q's components 4..14.
template <typename S>
struct Fields {
    const double *qT;
    const S *qP;
    const S *e;
    const S *p;
    const double *u;
    const double *up;
    const S *vf;     // face coefficients c^-, c^+ of the KT flux per face, x, y and eta face arrays (see FaceGeo)
};

// Face arrays: the x faces of row (j,k) are i = 0..nx (face i lies between
// cells i-1 and i), likewise for y and eta; each face holds the two
// coefficients of its KT flux H = c^+ q^+ + c^- q^- (face_coefficients).
// Offsets into Fields::vf, in elements.
struct FaceGeo {
    long long nfx, nfy, nfe;          // faces per axis
    long long ox, oy, oe;             // offsets of the three arrays (v^- block then v^+ block)
};

// Cell and face indices are 32-bit; a load adds the byte offset
// idx*sizeof(T) to a per-component base pointer that is uniform across the
// wavefront (kept in scalar registers), so no 64-bit address is formed per
// lane.
typedef uint32_t idx_t;

// The pointers are global memory: the batched kernels read them from a device
// table, where the compiler cannot see their address space and would emit flat
// accesses, which also count against the LDS wait counter and so hold up the
// kernels' LDS exchanges; the cast keeps every access a global one.
#define KT_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ T ld(const T *base, idx_t i)
{
    return *(const KT_GLOBAL T *)((const KT_GLOBAL char *)base + (size_t)(i * (idx_t)sizeof(T)));
}

template <typename T>
__device__ __forceinline__ void st(T *base, idx_t i, T v)
{
    *(KT_GLOBAL T *)((KT_GLOBAL char *)base + (size_t)(i * (idx_t)sizeof(T))) = v;
}

// component c (0..14) of q given as its FP64 part qT (0..3) and qP (4..14)
template <typename S>
__device__ __forceinline__ double ldq(const double *qT, const S *qP, int c, idx_t SS, idx_t s)
{
    return c < PTT ? ld(qT, (idx_t)c * SS + s) : (double)ld(qP, (idx_t)(c - PTT) * SS + s);
}

__host__ __device__ __forceinline__ idx_t fidx_x(int nx, int ny, int i, int j, int k)
{
    return ((idx_t)k * ny + j) * (idx_t)(nx + 1) + i;
}
__host__ __device__ __forceinline__ idx_t fidx_y(int nx, int ny, int i, int j, int k)
{
    return ((idx_t)k * (ny + 1) + j) * (idx_t)nx + i;
}
__host__ __device__ __forceinline__ idx_t fidx_e(int nx, int ny, int i, int j, int k)
{
    return ((idx_t)k * ny + j) * (idx_t)nx + i;
}

__device__ __forceinline__ int wrap(int v, int n, int periodic)
{
    if (v < 0) return periodic ? ((v % n) + n) % n : 0;
    if (v >= n) return periodic ? v % n : n - 1;
    return v;
}

// Blocks are dispatched to the chip's 8 XCDs round robin (block b to XCD
// b % 8), each XCD with its own L2.  This renumbering gives every XCD one
// contiguous range of logical blocks, so neighbouring tiles, which read each
// other's halo cells, share an L2.  It is a bijection on [0, nb) for any nb.
constexpr unsigned NXCD = 8;
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    const unsigned q = nb / NXCD, r = nb % NXCD;
    const unsigned x = b % NXCD, i = b / NXCD;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// tile (bx, by, bz) of logical block L of a gx x gy x gz tiling of a stencil
// launch: x fastest, or (KT_TILE_ZFAST) eta fastest, so that blocks running
// together share their eta-neighbour planes
__device__ __forceinline__ void tile_of_block(unsigned L, unsigned gx, unsigned gy, unsigned gz, unsigned &bx,
                                              unsigned &by, unsigned &bz)
{
#ifdef KT_TILE_ZFAST
    bz = L % gz;
    bx = (L / gz) % gx;
    by = L / (gz * gx);
#else
    (void)gz;
    bx = L % gx;
    by = (L / gx) % gy;
    bz = L / (gx * gy);
#endif
}

// logical (x, y, z) block of a 3D grid after the XCD renumbering
__device__ __forceinline__ void xcd_block3(unsigned &bx, unsigned &by, unsigned &bz)
{
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned L = xcd_block(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    tile_of_block(L, gx, gy, gridDim.z, bx, by, bz);
}

// floor(t / d) for t < 2^32, 1 <= d < 2^30, through a double product and one
// correction: the product is within 2^-20 of t / d, so q is off by at most
// one, and t - q d (taken modulo 2^32) lies in (-d, 2d), inside int range.
__device__ __forceinline__ idx_t udiv(idx_t t, idx_t d, double inv_d)
{
    const idx_t q = (idx_t)((double)t * inv_d);
    const int r = (int)(t - q * d);
    return r < 0 ? q - 1 : (r >= (int)d ? q + 1 : q);
}

// counters: the wave's total of a small non-negative integer v < 2^nbits,
// summed bit by bit from ballots (no cross-lane shuffles); lane 0 adds it to
// the wave's own slot row
__device__ __forceinline__ void slot_add(unsigned long long *slots, long long wave, int which, int v,
                                         int nbits = 1)
{
    unsigned long long tot = 0;
    for (int b = 0; b < nbits; ++b) tot += (unsigned long long)__popcll(__ballot((v >> b) & 1)) << b;
    if ((threadIdx.x & 63) == 0 && tot != 0) slots[wave * C_COUNT + which] += tot;
}

// bits needed for Newton iteration counts (at most newton_max)
__device__ __forceinline__ int iter_bits(const Phys &P) { return 32 - __clz(P.newton_max); }

// Lane exchanges of the flux kernel, whose wave holds 4 rows of 16 cells
// (lane = 16 row + column).  Every lane of the wave must be active.
//   row_next / row_prev: lane l gets lane l+1 / l-1 of its own row of 16 (DPP
//     row shifts, VALU); the last / first lane of a row keeps its own value;
//   half_swap: lane l gets lane l^32 (v_permlane32_swap, VALU);
//   row_down / row_up: lane l gets lane l-16 / l+16 modulo 64 (ds_bpermute).
template <int CTRL> __device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ int half_swap_i(int v)
{
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    // p[0] holds lanes 0-31 of v in both halves, p[1] lanes 32-63
    return (__lane_id() & 32) ? (int)p[0] : (int)p[1];
}
__device__ __forceinline__ int read_lane_i(int v, int src) { return __builtin_amdgcn_ds_bpermute((src & 63) << 2, v); }

template <typename F> __device__ __forceinline__ double per_word(double v, F f)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)f((int)(unsigned)b);
    const unsigned hi = (unsigned)f((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <typename F> __device__ __forceinline__ float per_word(float v, F f)
{
    return __int_as_float(f(__float_as_int(v)));
}
template <typename T> __device__ __forceinline__ T row_next(T v) { return per_word(v, dpp_i<0x101>); }  // row_shl:1
template <typename T> __device__ __forceinline__ T row_prev(T v) { return per_word(v, dpp_i<0x111>); }  // row_shr:1
template <typename T> __device__ __forceinline__ T half_swap(T v) { return per_word(v, half_swap_i); }
template <typename T> __device__ __forceinline__ T row_down(T v)
{
    const int src = (int)__lane_id() - 16;
    return per_word(v, [src](int w) { return read_lane_i(w, src); });
}
template <typename T> __device__ __forceinline__ T row_up(T v)
{
    const int src = (int)__lane_id() + 16;
    return per_word(v, [src](int w) { return read_lane_i(w, src); });
}

// ------------------------------------------------------------ KT flux ----
// One face between a left cell L and a right cell R (Sec. 3.1): with the
// minmod slopes of both cells, the half-cell extrapolations
// q^- = q_L + slope_L/2 and q^+ = q_R - slope_R/2, the velocities of their
// inversions v^-, v^+ (face_speeds_kernel; Sec. 3.1 last paragraph), the
// local speed a = max(|v^-|, |v^+|) and H = (v^+ q^+ + v^- q^-)/2 - a (q^+ - q^-)/2
// (Eqs. Hflux, ax), written H = c^+ q^+ + c^- q^- with the two coefficients
// c^+ = (v^+ - a)/2, c^- = (v^- + a)/2 of the face, which every component of q
// shares: the face kernel stores them, the flux kernel forms each H with two
// operations.
__device__ __forceinline__ void face_coefficients(double vm, double vp, double &cm, double &cp)
{
    const double a = fmax(fabs(vm), fabs(vp));
    cp = 0.5 * (vp - a);
    cm = 0.5 * (vm + a);
}

template <typename R>
__device__ __forceinline__ R face_H(R qm, R qp, R cm, R cp)
{
    return cp * qp + cm * qm;
}

// Face speeds (Sec. 3.1, last paragraph): every face of the grid has two
// reconstructed states, q^- = q_L + slope_L/2 from the cell on its left and
// q^+ = q_R - slope_R/2 from the cell on its right; each is inverted like a
// cell, its Newton iteration started from the conformal closed-form root of
// the state (fewer iterations than the e of the neighbouring cell, and no
// load), and the velocity component normal to the face is stored.
// One thread per face: it reads the four cells of the face's line that the
// two slopes need and inverts q^- and then q^+.
// The launch is cut into three segments of whole blocks, x, y and eta faces,
// in that order; a thread's index within its segment is the face index of
// fidx_x / fidx_y / fidx_e.
constexpr int FACE_BLOCK = 256;   // threads per block of the face kernels
// The face kernels are latency-bound (dependent EOS table reads inside each
// Newton solve): their register budget is that of 6 waves per SIMD; they
// need 68-70 VGPRs, which gives 7 (at 64 VGPRs for 8 waves the batched
// kernel spilled and ran 1.5% slower).

struct FaceLaunch {
    unsigned first_block[3];    // first block of each segment
    unsigned nblocks;           // total
    double inv_nx1, inv_nx, inv_ny1, inv_plane;   // 1/(nx+1), 1/nx, 1/(ny+1), 1/(nx ny)
};

// b: the block within this event's launch; wave: its counter slot row
template <bool CART, bool T1, typename S>
__device__ __forceinline__ void face_speeds_body(const Phys &P, const Eos &E, const FaceGeo G,
                                                 const FaceLaunch L, double tau, const double *qT,
                                                 const S *qP, S *vf,
                                                 unsigned long long *slots, unsigned b, long long wave,
                                                 double (*qpark)[FACE_BLOCK])
{
    typedef S R;   // reconstruction arithmetic; the inversion itself is FP64
    // (selects, not an index into L: a run-time index would put L in scratch memory)
    const int d = (b >= L.first_block[1] ? 1 : 0) + (b >= L.first_block[2] ? 1 : 0);
    const unsigned fb = d == 0 ? L.first_block[0] : (d == 1 ? L.first_block[1] : L.first_block[2]);
    const idx_t t = (idx_t)(b - fb) * FACE_BLOCK + threadIdx.x;
    const long long nf = d == 0 ? G.nfx : (d == 1 ? G.nfy : G.nfe);
    int it = 0, nfb = 0;
    const bool valid = (long long)t < nf;
    if (valid) {
        // (i, j, k) of the face, the line of cells through it along d
        idx_t base, step;
        int pos, n, per;
        if (d == 0) {
            const idx_t n1 = (idx_t)P.nx + 1, r = udiv(t, n1, L.inv_nx1);
            pos = (int)(t - r * n1);
            base = r * (idx_t)P.nx;                    // row (j, k)
            step = 1;
            n = P.nx;
            per = P.periodic[0];
        } else if (d == 1) {
            const idx_t r = udiv(t, (idx_t)P.nx, L.inv_nx), k = udiv(r, (idx_t)(P.ny + 1), L.inv_ny1);
            pos = (int)(r - k * (idx_t)(P.ny + 1));
            base = k * (idx_t)P.nx * P.ny + (t - r * (idx_t)P.nx);
            step = (idx_t)P.nx;
            n = P.ny;
            per = P.periodic[1];
        } else {
            const idx_t plane = (idx_t)P.nx * P.ny, k = udiv(t, plane, L.inv_plane);
            pos = (int)k;
            base = t - k * plane;
            step = plane;
            n = P.neta;
            per = P.periodic[2];
        }
        // face pos lies between cells pos-1 (L) and pos (R)
        const idx_t c0 = base + (idx_t)wrap(pos - 2, n, per) * step;
        const idx_t cL = base + (idx_t)wrap(pos - 1, n, per) * step;
        const idx_t cR = base + (idx_t)wrap(pos, n, per) * step;
        const idx_t c3 = base + (idx_t)wrap(pos + 1, n, per) * step;
        const R theta = R(P.theta);
        const idx_t SS = (idx_t)P.stride;
        // component r (0..8: T^{tau mu}, pi^{tau mu}, Pi) of q^- and q^+
        auto recon = [&](int r, double &qm, double &qp) {
            R a0, a1, a2, a3;
            if (r < 4) {
                const idx_t co = (idx_t)r * SS;
                a0 = R(ld(qT, co + c0)); a1 = R(ld(qT, co + cL));
                a2 = R(ld(qT, co + cR)); a3 = R(ld(qT, co + c3));
            } else {
                const idx_t co = (idx_t)(r < 8 ? r - PTT : BPI - PTT) * SS;
                a0 = R(ld(qP, co + c0)); a1 = R(ld(qP, co + cL));
                a2 = R(ld(qP, co + cR)); a3 = R(ld(qP, co + c3));
            }
            qm = (double)(a1 + R(0.5) * limited<T1>(a0, a1, a2, theta));
            qp = (double)(a2 - R(0.5) * limited<T1>(a1, a2, a3, theta));
        };
        const long long off = d == 0 ? G.ox : (d == 1 ? G.oy : G.oe);
        // q^+ waits in the block's LDS (qpark, this thread's column) while q^- is inverted
        const int tx = threadIdx.x;
        double mm[9], mp[9];
        recon(0, mm[0], mp[0]);
        recon(PTT, mm[4], mp[4]);
        // A state with E = T^{tau tau} - pi^{tau tau} <= e_floor is the floor state
        // whatever its other components (the inversion's first guard).  Vacuum
        // regions make whole waves of such states; they skip the rest.
        if (__all(!(mm[0] - mm[4] > P.e_floor) && !(mp[0] - mp[4] > P.e_floor))) {
            st(vf + off, t, (S)0.0);          // v^- = v^+ = 0: both coefficients vanish
            st(vf + off + nf, t, (S)0.0);
        } else {
            qpark[0][tx] = mp[0];
            qpark[4][tx] = mp[4];
#pragma unroll
            for (int r = 1; r < 9; ++r)
                if (r != PTT) {
                    double x;
                    recon(r, mm[r], x);
                    qpark[r][tx] = x;
                }
            // v^d = u^d / u^tau = M^d / (E + P) (Sec. 2.4), 0 on the floor
            auto speed = [&](const double *m, double e0, int &its) -> double {
                double ee, pe, EE, M[3];
                const double Pi = P.bulk ? m[8] : 0.0;
                const int fl = invert_core<CART>(P, E, tau, m[0], m[1], m[2], m[3], m[4], m[5], m[6], m[7],
                                                 Pi, e0, ee, pe, EE, M, its);
                nfb += (fl & F_FALLBACK) ? 1 : 0;
                const double Md = d == 0 ? M[0] : (d == 1 ? M[1] : M[2]);
                return (fl & F_FLOOR) ? 0.0 : Md / (EE + pe + Pi);
            };
            // (a compiler barrier: the parked values are not carried in registers)
            asm volatile("" ::: "memory");
            int it2 = 0;
            qpark[9][tx] = speed(mm, 0.0, it);        // v^- waits in LDS too
            asm volatile("" ::: "memory");
#pragma unroll
            for (int r = 0; r < 9; ++r) mp[r] = qpark[r][tx];
            const double vp = speed(mp, 0.0, it2);
            it += it2;
            double cm, cp;
            face_coefficients(qpark[9][tx], vp, cm, cp);
            st(vf + off, t, (S)cm);
            st(vf + off + nf, t, (S)cp);
        }
    }
    slot_add(slots, wave, C_ITERS_FACES, it, iter_bits(P) + 1);
    slot_add(slots, wave, C_REC_FACES, valid ? 2 : 0, 2);
    slot_add(slots, wave, C_FALLBACK_FACES, nfb, 2);
}

template <bool CART, bool T1, typename S>
__global__ __launch_bounds__(FACE_BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void face_speeds_kernel(Phys P, Eos E, FaceGeo G, FaceLaunch L,
                                                          double tau, const double *qT, const S *qP,
                                                          S *vf, unsigned long long *slots)
{
    __shared__ double qpark[10][FACE_BLOCK];
    face_speeds_body<CART, T1, S>(P, E, G, L, tau, qT, qP, vf, slots, xcd_block(blockIdx.x, gridDim.x),
                              (long long)blockIdx.x * (FACE_BLOCK / 64) + (threadIdx.x >> 6), qpark);
}

static FaceLaunch face_launch(const FaceGeo &G, int nx, int ny)
{
    FaceLaunch L;
    L.inv_nx1 = 1.0 / (nx + 1.0);
    L.inv_nx = 1.0 / nx;
    L.inv_ny1 = 1.0 / (ny + 1.0);
    L.inv_plane = 1.0 / ((double)nx * ny);
    const long long nf[3] = {G.nfx, G.nfy, G.nfe};
    unsigned acc = 0;
    for (int s = 0; s < 3; ++s) {
        L.first_block[s] = acc;
        acc += (unsigned)((nf[s] + FACE_BLOCK - 1) / FACE_BLOCK);
    }
    L.nblocks = acc;
    return L;
}

// The values of a neighbour cell that the central differences along axis
// i = d+1 need, loaded together (whether or not the fluid is viscous, so
// that no load waits behind a branch)
template <typename S>
struct NbCell {
    double u[4];      // u^mu
    double p, Pi;     // p(e), Pi
    double pt[4];     // pi^{tau mu}
    double pi[3];     // pi^{i x}, pi^{i y}, pi^{i eta}
    __device__ __forceinline__ void load(const Fields<S> &F, idx_t SS, idx_t s, int d)
    {
#pragma unroll
        for (int m = 0; m < 4; ++m) u[m] = ld(F.u, (idx_t)m * SS + s);
        p = (double)ld(F.p, s);
        Pi = (double)ld(F.qP, (idx_t)(BPI - PTT) * SS + s);
#pragma unroll
        for (int n = 0; n < 4; ++n) pt[n] = (double)ld(F.qP, (idx_t)(pi_index(0, n) - PTT) * SS + s);
#pragma unroll
        for (int n = 1; n < 4; ++n) pi[n - 1] = (double)ld(F.qP, (idx_t)(pi_index(d + 1, n) - PTT) * SS + s);
    }
    template <typename Tile>
    __device__ __forceinline__ void from_tile(const Tile &T, int ty, int tx, int d)
    {
#pragma unroll
        for (int m = 0; m < 4; ++m) u[m] = T.v[m][ty][tx];
        p = T.v[4][ty][tx];
        Pi = T.v[5][ty][tx];
#pragma unroll
        for (int n = 0; n < 4; ++n) pt[n] = T.v[6 + n][ty][tx];
#pragma unroll
        for (int n = 1; n < 4; ++n) pi[n - 1] = T.v[6 + pi_index(d + 1, n) - PTT][ty][tx];
    }
};

// The sources kernel's block (64 x 4 cells of one eta plane) with the cells
// on its four sides, in LDS: tile cell (ty, tx) is the cell at x = x0-1+tx,
// y = y0-1+ty (indices wrapped as the boundary conditions say; the four
// corners are not used).  Per cell: u^mu, p, Pi and pi^{tau tau} .. pi^{y eta},
// i.e. qP components 0..8 (all that the x and y differences need).
constexpr int SRC_TX = 66, SRC_TY = 6, SRC_NV = 15;
struct SrcTile {
    double v[SRC_NV][SRC_TY][SRC_TX];
};

// A^{i nu} = T^{i nu} - v^i T^{tau nu} of one cell for axis i = d+1 (Eqs. Ttt-Tij):
//   A^{i tau} = P v^i + pi^{i tau} - v^i pi^{tau tau}
//   A^{i j}   = -P g^{ij} + pi^{ij} - v^i pi^{tau j}
// (FP64: it feeds the conservation law, whose central differences cancel digits)
template <bool CART, typename S>
__device__ __forceinline__ void nonadvective_row(const Phys &P, double tau, const NbCell<S> &N, int d,
                                                 double A[4])
{
    const double Pc = N.p + (P.bulk ? N.Pi : 0.0);
    const int ii = d + 1;
    const double v = N.u[ii] / N.u[0];
    const double gii = ii == 3 ? (CART ? -1.0 : -1.0 / (tau * tau)) : -1.0;
    A[0] = Pc * v;
#pragma unroll
    for (int n = 1; n < 4; ++n) A[n] = n == ii ? -Pc * gii : 0.0;
    if (P.shear) {
        A[0] += N.pt[ii] - v * N.pt[0];
#pragma unroll
        for (int n = 1; n < 4; ++n) A[n] += N.pi[n - 1] - v * N.pt[n];
    }
}

// Sources part of one Euler stage (Sec. 3.1, Eq. semiDiscreteKT, and
// App. B), one thread per cell:
//   stage 1: out = q + dtau J;   stage 2: out = qn + q + dtau J,
// J = S_c + G_c for T^{tau mu} and the relaxation terms for pi and Pi.
// flux_kernel then adds the flux divergence and completes the stage.  Each
// component is written as soon as its J is known.  J is computed in the
// storage type S; T^{tau mu} is accumulated in FP64.  The x and y neighbours
// come from the block's LDS tile T (every thread of the block must call this).
template <bool CART, bool STAGE2, typename S>
__device__ __forceinline__ void sources_body(const Phys &P, const Eos &E, double tau, const Fields<S> &F,
                                             const double *qnT, const S *qnP, double *outT, S *outP,
                                             unsigned bx, unsigned by, unsigned bz, SrcTile &T)
{
    typedef S R;
    const int x0 = bx * 64, y0 = by * 4;
    const int i = x0 + threadIdx.x;
    const int j = y0 + threadIdx.y;
    const int k = bz;
    const idx_t SS = (idx_t)P.stride;
    const idx_t plane = (idx_t)P.nx * P.ny;
    const idx_t kp = (idx_t)k * plane;
    // the tile: every thread stages its own cell (threads outside the grid the
    // cell their index wraps to), and threads 0..135 of the first three waves
    // the 64 cells below and above the block and the 8 left and right of it
    {
        auto stage = [&](int ty, int tx, int gx, int gy) {
            const idx_t g = kp + (idx_t)wrap(gy, P.ny, P.periodic[1]) * P.nx + wrap(gx, P.nx, P.periodic[0]);
            double w[SRC_NV];
#pragma unroll
            for (int m = 0; m < 4; ++m) w[m] = ld(F.u, (idx_t)m * SS + g);
            w[4] = (double)ld(F.p, g);
            w[5] = (double)ld(F.qP, (idx_t)(BPI - PTT) * SS + g);
#pragma unroll
            for (int c = 0; c < 9; ++c) w[6 + c] = (double)ld(F.qP, (idx_t)c * SS + g);
#pragma unroll
            for (int c = 0; c < SRC_NV; ++c) T.v[c][ty][tx] = w[c];
        };
        stage(threadIdx.y + 1, threadIdx.x + 1, i, j);
        const int h = threadIdx.y * 64 + threadIdx.x;
        if (h < 64) stage(0, h + 1, x0 + h, y0 - 1);
        else if (h < 128) stage(5, h - 63, x0 + h - 64, y0 + 4);
        else if (h < 136) {
            const int q = h - 128, right = q & 1, r = q >> 1;
            stage(r + 1, right ? 65 : 0, right ? x0 + 64 : x0 - 1, y0 + r);
        }
    }
    __syncthreads();
    if (i >= P.nx || j >= P.ny) return;
    const int tx = threadIdx.x + 1, ty = threadIdx.y + 1;
    const idx_t rowc = kp + (idx_t)j * P.nx;
    const idx_t s = rowc + i;
    const idx_t col = (idx_t)j * P.nx + i;
    const idx_t nbe[2] = {col + (idx_t)wrap(k - 1, P.neta, P.periodic[2]) * plane,
                          col + (idx_t)wrap(k + 1, P.neta, P.periodic[2]) * plane};
    const double dt = P.dtau;
    // stage 2: q^n, read before the first store (out is the q^n array itself, so
    // a read placed after a store could not be issued early)
    double qn4[4];
    S qn11[NQ - PTT];
    if (STAGE2) {
#pragma unroll
        for (int c = 0; c < PTT; ++c) qn4[c] = ld(qnT, (idx_t)c * SS + s);
#pragma unroll
        for (int c = 0; c < NQ - PTT; ++c)
            qn11[c] = P.reduced && P.shear && pi_is_dependent(c + PTT) ? S(0) : ld(qnP, (idx_t)c * SS + s);
    }
    // T^{tau mu}: FP64 value, source and accumulation
    auto emitT = [&](int c, double qc, double Jc) {
        const idx_t o = (idx_t)c * SS + s;
        const double t = qc + dt * Jc;
        st(outT, o, STAGE2 ? qn4[c] + t : t);
    };
    // (a viscous reduced state evolves five of the ten pi components; the
    // recovery rebuilds the others.  Without shear all ten stay zero and are
    // written as in the ten-component state.)
    auto emitP = [&](int c, R qc, R Jc) {
        if (P.reduced && P.shear && pi_is_dependent(c)) return;
        const idx_t o = (idx_t)(c - PTT) * SS + s;
        const R t = qc + R(dt) * Jc;
        st(outP, o, STAGE2 ? R(qn11[c - PTT]) + t : t);
    };
    const double invhd[3] = {P.inv_dx, P.inv_dy, P.inv_deta};
    R u[4], C[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const double um = T.v[m][ty][tx];
        u[m] = R(um);
        C[0][m] = R((um - ld(F.up, (idx_t)m * SS + s)) * P.inv_dtau);
    }
    // central differences (Sec. 3.1): d_i u^m, d_i v^i, S_c = -d_i A^{i nu} (S_c in FP64)
    R divv = R(0);
    double Sc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double hh = 0.5 * invhd[d];
        NbCell<S> Np, Nm;
        if (d == 0) {
            Np.from_tile(T, ty, tx + 1, 0);
            Nm.from_tile(T, ty, tx - 1, 0);
        } else if (d == 1) {
            Np.from_tile(T, ty + 1, tx, 1);
            Nm.from_tile(T, ty - 1, tx, 1);
        } else {
            Np.load(F, SS, nbe[1], 2);
            Nm.load(F, SS, nbe[0], 2);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) C[d + 1][m] = R((Np.u[m] - Nm.u[m]) * hh);
        divv += R((Np.u[d + 1] / Np.u[0] - Nm.u[d + 1] / Nm.u[0]) * hh);
        double Ap[4], Am[4];
        nonadvective_row<CART, S>(P, tau, Np, d, Ap);
        nonadvective_row<CART, S>(P, tau, Nm, d, Am);
#pragma unroll
        for (int n = 0; n < 4; ++n) Sc[n] -= (Ap[n] - Am[n]) * hh;
    }
    const R e = R(ld(F.e, s));
    const R p0 = R(T.v[4][ty][tx]);
    const R Pim = R(T.v[5][ty][tx]);
    const R Pi = P.bulk ? Pim : R(0);
    R pv[10];
#pragma unroll
    for (int c = 0; c < 9; ++c) pv[c] = R(T.v[6 + c][ty][tx]);
    pv[9] = R(ld(F.qP, (idx_t)9 * SS + s));
    // conservation law: geometric source (App. B) G^tau = -(T^tt + tau^2 T^ee)/tau,
    // G^x = -T^tx/tau, G^y = -T^ty/tau, G^eta = -3 T^te/tau, with
    // tau^2 T^ee = tau^2 v^eta (T^te - pi^te) + P + tau^2 pi^ee.
    {
        double qt[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) qt[n] = ld(F.qT, (idx_t)n * SS + s);
        if (!CART) {
            const double inv_tau = 1.0 / tau, t2 = tau * tau;
            const double ve = T.v[3][ty][tx] / T.v[0][ty][tx];
            const double pte = P.shear ? (double)pv[PTE - PTT] : 0.0, pee = P.shear ? (double)pv[PEE - PTT] : 0.0;
            const double t2Tee = t2 * (ve * (qt[TE] - pte) + pee) + (T.v[4][ty][tx] + (double)Pi);
            emitT(TT, qt[TT], Sc[0] - (qt[TT] + t2Tee) * inv_tau);
            emitT(TX, qt[TX], Sc[1] - qt[TX] * inv_tau);
            emitT(TY, qt[TY], Sc[2] - qt[TY] * inv_tau);
            emitT(TE, qt[TE], Sc[3] - 3.0 * qt[TE] * inv_tau);
        } else {
#pragma unroll
            for (int n = 0; n < 4; ++n) emitT(n, qt[n], Sc[n]);
        }
    }
    // relaxation equations; components that do not evolve keep their value
    if (!P.shear)
        for (int c = 0; c < 10; ++c) emitP(PTT + c, pv[c], R(0));
    if (!P.bulk) emitP(BPI, Pim, R(0));
    if (P.shear || P.bulk) {
        double pe, cs2, T;
        eos_full(E, (double)e, pe, cs2, T);
        relaxation_sources<CART, R>(P, tau, pv, Pi, e, p0, R(cs2), R(T), u, C, divv, emitP);
    }
}

template <bool CART, bool STAGE2, typename S>
__global__ __launch_bounds__(256) void sources_kernel(Phys P, Eos E, double tau, Fields<S> F,
                                                      const double *qnT, const S *qnP,
                                                      double *outT, S *outP)
{
    __shared__ SrcTile T;
    unsigned bx, by, bz;
    xcd_block3(bx, by, bz);
    sources_body<CART, STAGE2, S>(P, E, tau, F, qnT, qnP, outT, outP, bx, by, bz, T);
}

// Flux part of one Euler stage: for a block of 4 waves of 16 x 4 cells (tw
// waves along x and 4 / tw along y: 64 x 4, 32 x 8 or 16 x 16 cells) and KCC
// eta planes, the KT flux divergence D = -sum_d (H_{+1/2} - H_{-1/2}) / d_d of
// every component (Sec. 3.1), then
//   stage 1: out = out + dtau D;   stage 2: out = (out + dtau D) / 2,
// which with sources_kernel gives q + dtau C[q] and (qn + q + dtau C[q]) / 2.
// The block first stages the KT coefficients of all its faces (from
// face_speeds_kernel) in LDS, then takes one component at a time through its
// planes.  A component's eta stencil (planes k0-2 .. k0+KCC+1 of the lane's
// column) is loaded once into registers and the eta face is carried from
// plane to plane in a register, so the values a plane re-reads from its
// neighbours were read moments before by the same block for the same
// component and are still cached (taking all 15 components of a plane before
// the next plane re-reads a plane only after the whole state of the previous
// one has passed through L2).  Each wave holds 16 x 4 cells (x by y; lane =
// 16 row + column), so that a cell's y neighbours are mostly other lanes'
// cells: every lane loads its own cell and one cell of the four halo rows
// (y0-2, y0-1, y0+4, y0+5), and the stencil is assembled by lane exchanges.
// A lane computes the x face on each side of its cell and the y face on each
// side (the coefficients of the far side from the neighbouring lane's LDS
// slot, or from the block's edge slots).
template <typename S, int KCC>
struct FluxLds {
    S x[KCC][2][256];       // c^-, c^+ of the x face left of each cell
    S xr[KCC][2][16];       // ... of the x face right of the last column of each wave row (4 wave + row)
    S y[KCC][2][256];       // ... of the y face below each cell
    S yt[KCC][2][64];       // ... of the y face above the last row of each wave (16 wave + column)
    S e[KCC + 1][2][256];   // ... of the eta face below each cell of planes k0 .. k0 + KCC
};

template <bool STAGE2, bool T1, typename S, int KCC>
__device__ __forceinline__ void flux_body(const Phys &P, const FaceGeo &G, const double *qT, const S *qP,
                                             const S *vf, double *outT, S *outP, FluxLds<S, KCC> &Lc,
                                             unsigned bx, unsigned by, unsigned bz, int tw)
{
    typedef S R;   // flux arithmetic of pi and Pi; T^{tau mu} is done in FP64
    const int lane = threadIdx.x;
    const int w = threadIdx.y;
    const int tid = w * 64 + lane;
    const int xl = lane & 15, r = lane >> 4;
    const int wx = w % tw, wy = w / tw;
    const int i = bx * (16 * tw) + wx * 16 + xl;
    const int j0 = by * (16 / tw) + wy * 4;
    const int j = j0 + r;
    const int k0 = bz * KCC;
    const int m = min(KCC, P.neta - k0);        // planes of this block (>= 1)
    const idx_t plane = (idx_t)P.nx * P.ny;
    const idx_t SS = (idx_t)P.stride;
    const int ic = wrap(i, P.nx, P.periodic[0]);
    const int jc = wrap(j, P.ny, P.periodic[1]);
    const int jh = wrap(j0 + (r < 2 ? r - 2 : r + 2), P.ny, P.periodic[1]);
    const int ifc = i <= P.nx ? i : P.nx;
    const int jfc = j <= P.ny ? (j < P.ny ? jc : P.ny) : jc;
    const bool out_ok = i < P.nx && j < P.ny;
    const int xm2 = wrap(i - 2, P.nx, P.periodic[0]), xm1 = wrap(i - 1, P.nx, P.periodic[0]);
    const int xp1 = wrap(i + 1, P.nx, P.periodic[0]), xp2 = wrap(i + 2, P.nx, P.periodic[0]);
    const S *vfx = vf + G.ox, *vfy = vf + G.oy, *vfe = vf + G.oe;
    const double f = P.dtau;
    const int c0 = P.shear ? PTT : BPI, c1 = P.bulk ? NQ : BPI;
    // the block's face coefficients
#pragma unroll
    for (int kk = 0; kk < KCC; ++kk) {
        if (kk < m) {
            const int k = k0 + kk;
            const idx_t fx = fidx_x(P.nx, P.ny, ifc, jc, k);
            Lc.x[kk][0][tid] = ld(vfx, fx);
            Lc.x[kk][1][tid] = ld(vfx + G.nfx, fx);
            if (xl == 15) {
                // (lanes outside the grid read a face that exists; their value is not used)
                const idx_t fr = fidx_x(P.nx, P.ny, min(i + 1, P.nx), jc, k);
                Lc.xr[kk][0][w * 4 + r] = ld(vfx, fr);
                Lc.xr[kk][1][w * 4 + r] = ld(vfx + G.nfx, fr);
            }
            // (jfc: the face below the lane's row, the grid's top face for the row above
            // the grid, whose lane is the upper neighbour of the grid's last row)
            const idx_t fy0 = fidx_y(P.nx, P.ny, ic, jfc, k);
            Lc.y[kk][0][tid] = ld(vfy, fy0);
            Lc.y[kk][1][tid] = ld(vfy + G.nfy, fy0);
            if (r == 3) {
                const idx_t fy1 = fidx_y(P.nx, P.ny, ic, jc + 1, k);
                Lc.yt[kk][0][w * 16 + xl] = ld(vfy, fy1);
                Lc.yt[kk][1][w * 16 + xl] = ld(vfy + G.nfy, fy1);
            }
        }
    }
#pragma unroll
    for (int kk = 0; kk <= KCC; ++kk) {
        if (kk <= m) {
            const idx_t fe = fidx_e(P.nx, P.ny, ic, jc, k0 + kk);
            Lc.e[kk][0][tid] = ld(vfe, fe);
            Lc.e[kk][1][tid] = ld(vfe + G.nfe, fe);
        }
    }
    __syncthreads();
    const idx_t col = (idx_t)jc * P.nx + ic;
    idx_t zi[KCC + 4];     // the lane's column at planes k0-2 .. k0+KCC+1
#pragma unroll
    for (int t = 0; t < KCC + 4; ++t) zi[t] = col + (idx_t)wrap(k0 - 2 + t, P.neta, P.periodic[2]) * plane;
    // (a lane's x face of the next lane in its row, or its own right face in the last column)
    const int nb = tid + 1;
    const int yup = r < 3 ? tid + 16 : -1;
    auto component = [&](auto rtag, const auto *q, idx_t co, auto *out) {
        typedef decltype(rtag) RR;
        const RR th = RR(P.theta), h = RR(0.5);
        RR z[KCC + 4], yh[KCC], e1[KCC], e2[KCC];
        decltype(rtag) prev[KCC];
#pragma unroll
        for (int t = 0; t < KCC + 4; ++t) z[t] = RR(ld(q, co + zi[t]));
#pragma unroll
        for (int kk = 0; kk < KCC; ++kk) {
            const idx_t kp = (idx_t)wrap(k0 + kk, P.neta, P.periodic[2]) * plane;
            yh[kk] = RR(ld(q, co + kp + (idx_t)jh * P.nx + ic));
            prev[kk] = RR(ld(out, co + kp + (idx_t)jc * P.nx + ic));
            e1[kk] = RR(0);
            e2[kk] = RR(0);
            if (xl == 0 || xl == 15) {
                const idx_t rx = kp + (idx_t)jc * P.nx;
                e1[kk] = RR(ld(q, co + rx + (xl == 0 ? xm1 : xp1)));
                e2[kk] = RR(ld(q, co + rx + (xl == 0 ? xm2 : xp2)));
            }
        }
        RR Hb0 = face_H<RR>(z[1] + h * limited<T1>(z[0], z[1], z[2], th),
                            z[2] - h * limited<T1>(z[1], z[2], z[3], th), RR(Lc.e[0][0][tid]),
                            RR(Lc.e[0][1][tid]));
#pragma unroll
        for (int kk = 0; kk < KCC; ++kk) {
            if (kk >= m) break;     // uniform over the block
            const RR yc = z[kk + 2], eb = z[kk + 1], ed = z[kk + 3], ee = z[kk + 4];
            const RR yhh = yh[kk], edge1 = e1[kk], edge2 = e2[kk];
            const RR o32 = half_swap(yc), h32 = half_swap(yhh);
            const RR ya = r < 2 ? yhh : o32;
            const RR ye = r < 2 ? o32 : yhh;
            const RR mb = r == 3 ? h32 : yc, md = r == 0 ? h32 : yc;
            const RR yb = row_down(mb), yd = row_up(md);
            const RR sb = row_prev(yc), sd = row_next(yc);
            const RR xb = xl == 0 ? edge1 : sb;
            const RR xd = xl == 15 ? edge1 : sd;
            const RR sa = row_prev(xb), se = row_next(xd);
            const RR xa = xl == 0 ? edge2 : sa;
            const RR xe = xl == 15 ? edge2 : se;
            const RR xc = yc;
            const RR cmx = RR(Lc.x[kk][0][tid]), cpx = RR(Lc.x[kk][1][tid]);
            const RR cmr = RR(xl == 15 ? Lc.xr[kk][0][w * 4 + r] : Lc.x[kk][0][nb & 255]);
            const RR cpr = RR(xl == 15 ? Lc.xr[kk][1][w * 4 + r] : Lc.x[kk][1][nb & 255]);
            const RR cmy0 = RR(Lc.y[kk][0][tid]), cpy0 = RR(Lc.y[kk][1][tid]);
            const RR cmy1 = RR(yup >= 0 ? Lc.y[kk][0][yup] : Lc.yt[kk][0][w * 16 + xl]);
            const RR cpy1 = RR(yup >= 0 ? Lc.y[kk][1][yup] : Lc.yt[kk][1][w * 16 + xl]);
            const RR cme = RR(Lc.e[kk + 1][0][tid]), cpe = RR(Lc.e[kk + 1][1][tid]);
            const RR sxb = limited<T1>(xa, xb, xc, th), sxc = limited<T1>(xb, xc, xd, th),
                     sxd = limited<T1>(xc, xd, xe, th);
            const RR Hx = face_H<RR>(xb + h * sxb, xc - h * sxc, cmx, cpx);
            const RR Hown = face_H<RR>(xc + h * sxc, xd - h * sxd, cmr, cpr);
            RR D = (Hx - Hown) * RR(P.inv_dx);
            const RR syb = limited<T1>(ya, yb, yc, th), syc = limited<T1>(yb, yc, yd, th),
                     syd = limited<T1>(yc, yd, ye, th);
            D += (face_H<RR>(yb + h * syb, yc - h * syc, cmy0, cpy0)
                - face_H<RR>(yc + h * syc, yd - h * syd, cmy1, cpy1)) * RR(P.inv_dy);
            const RR sec = limited<T1>(eb, yc, ed, th), sed = limited<T1>(yc, ed, ee, th);
            const RR Ht = face_H<RR>(yc + h * sec, ed - h * sed, cme, cpe);
            D += (Hb0 - Ht) * RR(P.inv_deta);
            Hb0 = Ht;
            if (out_ok) {
                const RR t = prev[kk] + RR(f) * D;
                const idx_t kp = (idx_t)(k0 + kk) * plane;
                st(out, co + kp + (idx_t)jc * P.nx + ic, STAGE2 ? RR(0.5) * t : t);
            }
        }
    };
#pragma unroll 1
    for (int c = 0; c < PTT; ++c) component(0.0, qT, (idx_t)c * SS, outT);
#pragma unroll 1
    for (int c = c0; c < c1; ++c)
        if (!(P.reduced && pi_is_dependent(c))) component(R(0), qP, (idx_t)(c - PTT) * SS, outP);
}

template <bool STAGE2, bool T1, typename S, int KCC>
__global__ __launch_bounds__(256) void flux_kernel(Phys P, FaceGeo G, const double *qT, const S *qP,
                                                      const S *vf, double *outT, S *outP, int tw)
{
    __shared__ FluxLds<S, KCC> Lc;
    unsigned bx, by, bz;
    xcd_block3(bx, by, bz);
    flux_body<STAGE2, T1, S, KCC>(P, G, qT, qP, vf, outT, outP, Lc, bx, by, bz, tw);
}

// recovery of every cell at tau, then the regulator and the floor reset;
// writes e, p(e) and u.  Newton start: the cell's previous e (warm), the
// conformal closed form, or (LEARNED) y_0 e_c from the network of kt_mlp.hpp
// on the matrix cores (K: the packed weights, xs: the wave's LDS rows; every
// lane of the wave must call this).  The inversion and the regulator run in
// FP64 whatever the storage type S.
template <bool CART, bool LEARNED, typename S>
__device__ __forceinline__ void recover_body(const Phys &P, const Eos &E, double tau, double *qT, S *qP,
                                             S *e_io, S *p_out, double *u_out, int do_regulate, int warm,
                                             const ktm::MlpPacked *__restrict__ K,
                                             _Float16 (*xs)[ktm::XS_K], unsigned long long *slots,
                                             idx_t s)
{
    const long long wave = s >> 6;
    const idx_t SS = (idx_t)P.stride;
    int it = 0, fl = 0;
    const bool valid = (long long)s < P.ncell;
    // E = T^{tau tau} - pi^{tau tau} <= e_floor gives the floor state whatever the
    // other components (the inversion's first guard); with the floor reset on, a
    // wave of such cells (vacuum) writes that state without reading the rest or
    // evaluating the network (measured: no gain without the network, where the
    // extra registers cost the batched kernel a wave per SIMD)
    bool vacuum = false;
    if (LEARNED) {
        const bool lane_vac = !valid || !(ld(qT, s) - ldq(qT, qP, PTT, SS, s) > P.e_floor);
        vacuum = P.floor_reset && __all(lane_vac);    // uniform over the wave
    }
    double es = -1.0;
    if (LEARNED && !vacuum) {
        // the network's start, before the cell's state is held in registers;
        // every lane takes part (lanes without a state pass zero features)
        float x[ktm::NI];
#pragma unroll
        for (int f = 0; f < ktm::NI; ++f) x[f] = 0.0f;
        double ec = -1.0;
        if (valid) {
            const double Ttt = ld(qT, s), ptt = ldq(qT, qP, PTT, SS, s);
            if (Ttt > 0.0 && Ttt - ptt > 0.0) {
                const double Ttx = ld(qT, SS + s), Tty = ld(qT, 2 * SS + s), Tte = ld(qT, 3 * SS + s);
                const double ptx = ldq(qT, qP, PTX, SS, s), pty = ldq(qT, qP, PTY, SS, s);
                const double pte = ldq(qT, qP, PTE, SS, s);
                ktm::features<CART>(E, tau, Ttt, Ttx, Tty, Tte, ptt, ptx, pty, pte,
                                    P.bulk ? ldq(qT, qP, BPI, SS, s) : 0.0, x);
                ec = ktm::conformal_root<CART>(P.e_floor, tau, Ttt, Ttx, Tty, Tte, ptt, ptx, pty, pte);
            }
        }
        const float y0 = ktm::forward_y0_mfma(K, x, xs);
        if (ec > 0.0) es = (double)y0 * ec;
    }
    if (vacuum && valid) {
        fl = F_FLOOR;
        st(e_io, s, (S)P.e_floor);
        st(p_out, s, (S)P.p_floor);
#pragma unroll
        for (int m = 0; m < 4; ++m) st(u_out, (idx_t)(m) * SS + s, m == 0 ? 1.0 : 0.0);
#pragma unroll
        for (int c = 0; c < PTT; ++c) st(qT, (idx_t)c * SS + s, c == TT ? P.e_floor : 0.0);
#pragma unroll
        for (int c = PTT; c < NQ; ++c) st(qP, (idx_t)(c - PTT) * SS + s, (S)0);
    } else if (valid) {
        if (!LEARNED && warm) es = (double)ld(e_io, s);
        double qc[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) qc[c] = ldq(qT, qP, c, SS, s);
        const double Pi = P.bulk ? qc[BPI] : 0.0;
        double e, p0, u[4];
        fl = recover<CART>(P, E, tau, qc[TT], qc[TX], qc[TY], qc[TE], qc[PTT], qc[PTX], qc[PTY],
                           qc[PTE], Pi, es, e, p0, u, it);
        st(e_io, s, (S)e);
        st(p_out, s, (S)p0);
#pragma unroll
        for (int m = 0; m < 4; ++m) st(u_out, (idx_t)(m) * SS + s, u[m]);
        if ((fl & F_FLOOR) && P.floor_reset) {
#pragma unroll
            for (int c = 0; c < PTT; ++c) st(qT, (idx_t)c * SS + s, c == TT ? P.e_floor : 0.0);
#pragma unroll
            for (int c = PTT; c < NQ; ++c) st(qP, (idx_t)(c - PTT) * SS + s, (S)0);
        } else if (do_regulate && P.regulate && P.shear) {
            regulate<CART>(P, tau, qc, e, p0, u);
#pragma unroll
            for (int c = PTT; c < NQ; ++c) st(qP, (idx_t)(c - PTT) * SS + s, (S)qc[c]);
        }
    }
    slot_add(slots, wave, C_ITERS_CELLS, it, iter_bits(P));
    slot_add(slots, wave, C_REC_CELLS, valid ? 1 : 0);
    slot_add(slots, wave, C_FLOOR, (fl & F_FLOOR) ? 1 : 0);
    slot_add(slots, wave, C_CLAMP, (fl & F_CLAMP) ? 1 : 0);
    slot_add(slots, wave, C_FALLBACK, (fl & F_FALLBACK) ? 1 : 0);
}

// Recovery of a reduced state (Sec. 2.4; the state evolves T^{tau mu}, the
// five independent pi components and Pi): pi^{tau mu}, which the inversion
// needs, depends on the velocity being recovered, so (e, u) and the dependent
// components are solved together by the fixed point
//   u_{k+1} = inversion of (T^{tau mu}, pi^{tau mu}(five, u_k), Pi),
// started from us (the cell's flow before the stage, u^tau renormalised at
// tau; null: at rest), the first inversion's Newton iteration from the
// conformal closed form and each later one from the previous pass's e (the
// root moves little between passes; every pass converges to the same
// tolerance whatever its start, so only the iteration counts change), stopped
// when no component of u moves by more than FP_TOL u^tau (the eta component
// times sqrt(g33)), on the floor state, without shear (one pass), or after
// FP_MAX passes (counted as not converged).  The dependent components of the
// final u are stored with the five, then the floor reset and the regulator act
// as in recover_body (the regulator on the whole tensor).
constexpr double FP_TOL = 1e-14;
constexpr int FP_MAX = 100;

// The fixed point itself: qc holds T^{tau mu}, the five pi components and Pi
// (its dependent slots are overwritten pass by pass), u the normalised start;
// u receives the flow, e and p0 the last inversion's e and p(e), it the summed
// Newton iterations, passes the passes taken, conv whether the tolerance (or
// the floor, or the absence of shear) ended them.  Returns the last flags.
template <bool CART>
__device__ __forceinline__ int reduced_fixed_point(const Phys &P, const Eos &E, double tau, double qc[NQ],
                                                   double u[4], double &e, double &p0, int &it, int &passes,
                                                   bool &conv)
{
    const double g33 = CART ? 1.0 : tau * tau;
    const double sg = sqrt(g33);
    const double Pi = P.bulk ? qc[BPI] : 0.0;
    int fl = 0;
    it = 0;
    passes = 0;
    conv = false;
    while (passes < FP_MAX) {
        if (P.shear) pi_dependent_of<CART>(tau, u, qc);
        double un[4];
        int its = 0;
        fl = recover<CART>(P, E, tau, qc[TT], qc[TX], qc[TY], qc[TE], qc[PTT], qc[PTX], qc[PTY],
                           qc[PTE], Pi, passes > 0 ? e : -1.0, e, p0, un, its);
        it += its;
        ++passes;
        double dmax = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            dmax = fmax(dmax, fabs(un[m] - u[m]) * (m == 3 ? sg : 1.0) / un[0]);
#pragma unroll
        for (int m = 0; m < 4; ++m) u[m] = un[m];
        if ((fl & F_FLOOR) || !P.shear || dmax <= FP_TOL) {
            conv = true;
            break;
        }
    }
    return fl;
}

template <bool CART, typename S>
__device__ __forceinline__ void recover_reduced_body(const Phys &P, const Eos &E, double tau, double *qT,
                                                     S *qP, S *e_out, S *p_out, double *u_out,
                                                     const double *us, int do_regulate,
                                                     unsigned long long *slots, idx_t s)
{
    const long long wave = s >> 6;
    const idx_t SS = (idx_t)P.stride;
    const double g33 = CART ? 1.0 : tau * tau;
    int it = 0, fl = 0, passes = 0, noconv = 0;
    const bool valid = (long long)s < P.ncell;
    if (valid) {
        double qc[NQ];
#pragma unroll
        for (int c = 0; c < NQ; ++c) qc[c] = pi_is_dependent(c) ? 0.0 : ldq(qT, qP, c, SS, s);
        double u[4] = {1.0, 0.0, 0.0, 0.0};
        if (us) {
#pragma unroll
            for (int m = 1; m < 4; ++m) u[m] = ld(us, (idx_t)m * SS + s);
            u[0] = sqrt(1.0 + u[1] * u[1] + u[2] * u[2] + g33 * u[3] * u[3]);
        }
        // (the loop of reduced_fixed_point written out: calling it here costs this
        // kernel 12-17 more spilled registers and 5% of the reduced step)
        const double Pi = P.bulk ? qc[BPI] : 0.0;
        double e = 0.0, p0 = 0.0;
        bool conv = false;
        const double sg = sqrt(g33);
        while (passes < FP_MAX) {
            if (P.shear) pi_dependent_of<CART>(tau, u, qc);
            double un[4];
            int its = 0;
            fl = recover<CART>(P, E, tau, qc[TT], qc[TX], qc[TY], qc[TE], qc[PTT], qc[PTX], qc[PTY],
                               qc[PTE], Pi, passes > 0 ? e : -1.0, e, p0, un, its);
            it += its;
            ++passes;
            double dmax = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                dmax = fmax(dmax, fabs(un[m] - u[m]) * (m == 3 ? sg : 1.0) / un[0]);
#pragma unroll
            for (int m = 0; m < 4; ++m) u[m] = un[m];
            if ((fl & F_FLOOR) || !P.shear || dmax <= FP_TOL) {
                conv = true;
                break;
            }
        }
        noconv = conv ? 0 : 1;
        st(e_out, s, (S)e);
        st(p_out, s, (S)p0);
#pragma unroll
        for (int m = 0; m < 4; ++m) st(u_out, (idx_t)(m) * SS + s, u[m]);
        if ((fl & F_FLOOR) && P.floor_reset) {
#pragma unroll
            for (int c = 0; c < PTT; ++c) st(qT, (idx_t)c * SS + s, c == TT ? P.e_floor : 0.0);
#pragma unroll
            for (int c = PTT; c < NQ; ++c) st(qP, (idx_t)(c - PTT) * SS + s, (S)0);
        } else if (P.shear) {
            pi_dependent_of<CART>(tau, u, qc);
            if (do_regulate && P.regulate) regulate<CART>(P, tau, qc, e, p0, u);
#pragma unroll
            for (int c = PTT; c < NQ; ++c) st(qP, (idx_t)(c - PTT) * SS + s, (S)qc[c]);
        }
    }
    slot_add(slots, wave, C_ITERS_CELLS, it, 16);     // summed over at most FP_MAX passes
    slot_add(slots, wave, C_REC_CELLS, valid ? 1 : 0);
    slot_add(slots, wave, C_FLOOR, (fl & F_FLOOR) ? 1 : 0);
    slot_add(slots, wave, C_CLAMP, (fl & F_CLAMP) ? 1 : 0);
    slot_add(slots, wave, C_FALLBACK, (fl & F_FALLBACK) ? 1 : 0);
    slot_add(slots, wave, C_FP_PASSES, passes, 32 - __clz(FP_MAX));
    slot_add(slots, wave, C_FP_NOCONV, noconv);
}

// (4 waves per SIMD: 128 VGPRs and a few spilled values instead of 136-148
// VGPRs and 3 waves; measured 1% faster on the reduced step)
template <bool CART, typename S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void recover_reduced_kernel(Phys P, Eos E, double tau, double *qT, S *qP,
                                                              S *e_out, S *p_out, double *u_out,
                                                              const double *us, int do_regulate,
                                                              unsigned long long *slots)
{
    recover_reduced_body<CART, S>(P, E, tau, qT, qP, e_out, p_out, u_out, us, do_regulate, slots,
                                  (idx_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// (the register budget of 4 waves per SIMD: without it the network's
// instantiation held its matrix-core accumulators in 36 AGPRs beside 112
// VGPRs, 3 waves; within 128 it needs no spill and the learned step is 0.07 ms
// faster; the other instantiations use 118-120 either way)
template <bool CART, bool LEARNED, typename S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void recover_kernel(Phys P, Eos E, double tau, double *qT, S *qP,
                                                      S *e_io, S *p_out, double *u_out,
                                                      int do_regulate, int warm,
                                                      const ktm::MlpPacked *__restrict__ K,
                                                      unsigned long long *slots)
{
    __shared__ _Float16 xs[LEARNED ? 256 : 1][ktm::XS_K];
    recover_body<CART, LEARNED, S>(P, E, tau, qT, qP, e_io, p_out, u_out, do_regulate, warm, K,
                                   LEARNED ? xs + (threadIdx.x & ~63u) : xs, slots,
                                   (idx_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ------------------------------------------------------------- batches ---
// One launch advances every event of a batch.  Block g of the launch (after
// the XCD renumbering) belongs to event e = map[g] and is that event's block
// g - first[e]; the event's arguments sit in a device table read with
// wave-uniform loads.  Events share tau (kept on the device so that a
// captured step can be replayed) and the time step.

template <typename S>
struct BStage {             // one event of a stage (sources + flux launches)
    Phys P;
    Eos E;
    FaceGeo G;
    Fields<S> F;            // input of the stage
    const double *qnT;      // q^n (stage 2 only)
    const S *qnP;
    double *outT;
    S *outP;
    unsigned sgx, sgy;      // sources grid (x, y); z = neta
    unsigned fgx, fgy;      // flux grid (x, y); z = ceil(neta / KCC) (the launch's eta planes per block)
    int tw;                 // waves per flux block along x (4, 2 or 1: 64 x 4, 32 x 8, 16 x 16 cells)
};

template <typename S>
struct BRec {               // one event of a recovery launch
    Phys P;
    Eos E;
    double *qT;
    S *qP, *e, *p;
    double *u;
    const double *us;       // flow before the stage (start of a reduced state's fixed point)
    unsigned long long *slots;
};

template <typename S>
struct BFace {              // one event of a face-speed launch
    Phys P;
    Eos E;
    FaceGeo G;
    FaceLaunch L;
    const double *qT;
    const S *qP;
    S *vf;
    unsigned long long *slots;
};

template <bool CART, bool STAGE2, typename S>
__global__ __launch_bounds__(256) void sources_batch(const BStage<S> *__restrict__ tab,
                                                     const unsigned short *__restrict__ map,
                                                     const unsigned *__restrict__ first,
                                                     const double *__restrict__ tau_dev)
{
    const unsigned g = xcd_block(blockIdx.x, gridDim.x);
    const int ev = map[g];
    const BStage<S> &A = tab[ev];
    const unsigned lb = g - first[ev];
    unsigned bx, by, bz;
    tile_of_block(lb, A.sgx, A.sgy, A.P.neta, bx, by, bz);
    const double tau = STAGE2 ? tau_dev[0] + A.P.dtau : tau_dev[0];
    __shared__ SrcTile T;
    sources_body<CART, STAGE2, S>(A.P, A.E, tau, A.F, A.qnT, A.qnP, A.outT, A.outP, bx, by, bz, T);
}

template <bool STAGE2, bool T1, typename S, int KCC>
__global__ __launch_bounds__(256) void flux_batch(const BStage<S> *__restrict__ tab,
                                                  const unsigned short *__restrict__ map,
                                                  const unsigned *__restrict__ first)
{
    __shared__ FluxLds<S, KCC> Lc;
    const unsigned g = xcd_block(blockIdx.x, gridDim.x);
    const int ev = map[g];
    const BStage<S> &A = tab[ev];
    const unsigned lb = g - first[ev];
    unsigned bx, by, bz;
    tile_of_block(lb, A.fgx, A.fgy, (A.P.neta + KCC - 1) / KCC, bx, by, bz);
    flux_body<STAGE2, T1, S, KCC>(A.P, A.G, A.F.qT, A.F.qP, A.F.vf, A.outT, A.outP, Lc, bx, by, bz, A.tw);
}

template <bool CART, typename S, bool RED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void recover_batch(const BRec<S> *__restrict__ tab,
                                                     const unsigned short *__restrict__ map,
                                                     const unsigned *__restrict__ first,
                                                     const double *__restrict__ tau_dev)
{
    const unsigned g = blockIdx.x;
    const int ev = map[g];
    const BRec<S> &A = tab[ev];
    const double tau = tau_dev[0] + A.P.dtau;
    const idx_t s = (idx_t)(g - first[ev]) * 256 + threadIdx.x;
    // events of a batch keep the library's default Newton start (KT_START_CONFORMAL:
    // warm = 0), as a single context does
    if (RED)
        recover_reduced_body<CART, S>(A.P, A.E, tau, A.qT, A.qP, A.e, A.p, A.u, A.us, 1, A.slots, s);
    else
        recover_body<CART, false, S>(A.P, A.E, tau, A.qT, A.qP, A.e, A.p, A.u, 1, 0, nullptr, nullptr, A.slots, s);
}

template <bool CART, bool T1, typename S>
__global__ __launch_bounds__(FACE_BLOCK) __attribute__((amdgpu_waves_per_eu(6))) void faces_batch(const BFace<S> *__restrict__ tab,
                                                   const unsigned short *__restrict__ map,
                                                   const unsigned *__restrict__ first,
                                                   const double *__restrict__ tau_dev)
{
    const unsigned g = xcd_block(blockIdx.x, gridDim.x);
    const int ev = map[g];
    const BFace<S> &A = tab[ev];
    const unsigned lb = g - first[ev];
    const double tau = tau_dev[0] + A.P.dtau;
    __shared__ double qpark[10][FACE_BLOCK];
    face_speeds_body<CART, T1, S>(A.P, A.E, A.G, A.L, tau, A.qT, A.qP, A.vf, A.slots, lb,
                              (long long)lb * (FACE_BLOCK / 64) + (threadIdx.x >> 6), qpark);
}

// tau^{n+1} = tau^n + dtau, one thread (part of the captured step)
__global__ void tau_advance_kernel(double *tau_dev, double dtau)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) tau_dev[0] = tau_dev[0] + dtau;
}

// T^{tau mu} from primitives (Sec. 2.4, Eqs. Ttt, Tti): (e+P) u^tau u^mu - P g^{tau mu} + pi^{tau mu}
struct PrimPtrs {
    const double *e;
    const double *u[4];
    const double *pi[10];
    const double *Pi;
};

// p = p(e) of the equilibrium EOS for every cell (a resumed state given without p)
template <typename S>
__global__ __launch_bounds__(256) void pressure_kernel(Eos E, long long n, const S *e, S *p)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    double pe, cs2;
    eos_pc(E, (double)e[s], pe, cs2);
    p[s] = (S)pe;
}

template <typename S>
__global__ __launch_bounds__(256) void tmunu_kernel(Phys P, Eos E, PrimPtrs in, double *qT, S *qP)
{
    const idx_t s = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((long long)s >= P.ncell) return;
    const idx_t SS = (idx_t)P.stride;
    const double e = ld(in.e, s);
    const double Pi = ld(in.Pi, s);
    const double Pc = eos_p(E, e) + Pi;
    const double ut = ld(in.u[0], s);
    const double w = (e + Pc) * ut;
#pragma unroll
    for (int m = 0; m < 4; ++m)   // pi^{tau m} are the first four of the ten
        st(qT, (idx_t)(m) * SS + s, w * ld(in.u[m], s) - (m == 0 ? Pc : 0.0) + ld(in.pi[m], s));
#pragma unroll
    for (int c = 0; c < 10; ++c) st(qP, (idx_t)c * SS + s, (S)ld(in.pi[c], s));
    st(qP, (idx_t)(BPI - PTT) * SS + s, (S)Pi);
}

// FP64 inputs to the FP32 storage (n elements)
__global__ __launch_bounds__(256) void from_double_kernel(long long n, const double *in, float *out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

// conversion of stored fields to FP64 for export (n elements)
template <typename S>
__global__ __launch_bounds__(256) void to_double_kernel(long long n, const S *in, double *out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

struct RecIn {
    const double *in[9];
    double *e;
    double *u[4];
    int *iters;
    int *flags;
};

template <bool CART, bool LEARNED>
__global__ __launch_bounds__(256) void recover_standalone_kernel(Phys P, Eos E, double tau,
                                                                 long long n, RecIn R,
                                                                 const ktm::MlpPacked *__restrict__ K)
{
    __shared__ _Float16 xs[LEARNED ? 256 : 1][ktm::XS_K];
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    if (!LEARNED && !valid) return;
    const long long sv = valid ? s : 0;     // lanes past n compute on state 0 and store nothing
    const double Pi = (P.bulk && R.in[8]) ? R.in[8][sv] : 0.0;
    const double Ttt = R.in[0][sv], ptt = R.in[4][sv];
    double es = -1.0;
    if (LEARNED) {
        // every lane of the wave takes part in the network (matrix instructions)
        float x[ktm::NI];
#pragma unroll
        for (int f = 0; f < ktm::NI; ++f) x[f] = 0.0f;
        double ec = -1.0;
        if (Ttt > 0.0 && Ttt - ptt > 0.0) {
            ktm::features<CART>(E, tau, Ttt, R.in[1][sv], R.in[2][sv], R.in[3][sv], ptt, R.in[5][sv],
                                R.in[6][sv], R.in[7][sv], Pi, x);
            ec = ktm::conformal_root<CART>(P.e_floor, tau, Ttt, R.in[1][sv], R.in[2][sv], R.in[3][sv], ptt,
                                           R.in[5][sv], R.in[6][sv], R.in[7][sv]);
        }
        const float y0 = ktm::forward_y0_mfma(K, x, xs + (threadIdx.x & ~63u));
        if (ec > 0.0) es = (double)y0 * ec;
        if (!valid) return;
    }
    double e, p, u[4];
    int it;
    const int fl = recover<CART>(P, E, tau, Ttt, R.in[1][s], R.in[2][s], R.in[3][s], ptt,
                                 R.in[5][s], R.in[6][s], R.in[7][s], Pi, es, e, p, u, it);
    R.e[s] = e;
#pragma unroll
    for (int m = 0; m < 4; ++m) R.u[m][s] = u[m];
    if (R.iters) R.iters[s] = it;
    if (R.flags) R.flags[s] = fl;
}

// kt_recover_reduced: the reduced state's coupled recovery of n separate states
// (T^{tau mu}, the five pi components, Pi), started at rest, without regulator
// or floor reset; the dependent components of the final flow are returned.
struct RecRedIn {
    const double *in[10];
    double *e;
    double *u[4];
    double *pi[5];       // pi^{tau tau}, pi^{tau x}, pi^{tau y}, pi^{tau eta}, pi^{eta eta}; nullable
    int *passes;         // negative when the pass limit ended the fixed point; nullable
    int *flags;          // nullable
};

template <bool CART>
__global__ __launch_bounds__(256) void recover_reduced_standalone_kernel(Phys P, Eos E, double tau, long long n,
                                                                         RecRedIn R)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    double qc[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) qc[c] = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) qc[c] = R.in[c][s];
    qc[PXX] = R.in[4][s];
    qc[PXY] = R.in[5][s];
    qc[PXE] = R.in[6][s];
    qc[PYY] = R.in[7][s];
    qc[PYE] = R.in[8][s];
    qc[BPI] = R.in[9] ? R.in[9][s] : 0.0;
    double u[4] = {1.0, 0.0, 0.0, 0.0}, e = 0.0, p0 = 0.0;
    int it = 0, passes = 0;
    bool conv = false;
    const int fl = reduced_fixed_point<CART>(P, E, tau, qc, u, e, p0, it, passes, conv);
    R.e[s] = e;
#pragma unroll
    for (int m = 0; m < 4; ++m) R.u[m][s] = u[m];
    if (R.pi[0]) {
        if (P.shear) {
            pi_dependent_of<CART>(tau, u, qc);
        } else {
            qc[PTT] = qc[PTX] = qc[PTY] = qc[PTE] = qc[PEE] = 0.0;
        }
        const int dep[5] = {PTT, PTX, PTY, PTE, PEE};
#pragma unroll
        for (int k = 0; k < 5; ++k) R.pi[k][s] = qc[dep[k]];
    }
    if (R.passes) R.passes[s] = conv ? passes : -passes;
    if (R.flags) R.flags[s] = fl;
}

// sum of the counter slots: per-block partial sums, then one block adds them
// (integer sums, so the result does not depend on the order)
constexpr int SLOT_BLOCKS = 256;

// the network's start y_0 of n feature vectors (feature-major x[f n + i]) by the
// matrix-core inference the recoveries use (kt_mlp.hpp); lanes past n take part
// with zero features and store nothing
__global__ __launch_bounds__(256) void mlp_y0_kernel(long long n, const float *__restrict__ x, float *y0,
                                                     const ktm::MlpPacked *__restrict__ K)
{
    __shared__ _Float16 xs[256][ktm::XS_K];
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    float f[ktm::NI];
#pragma unroll
    for (int k = 0; k < ktm::NI; ++k) f[k] = valid ? x[k * n + s] : 0.0f;
    const float y = ktm::forward_y0_mfma(K, f, xs + (threadIdx.x & ~63u));
    if (valid) y0[s] = y;
}

__global__ __launch_bounds__(256) void slots_partial_kernel(const unsigned long long *slots,
                                                            long long nwaves,
                                                            unsigned long long *partial)
{
    __shared__ unsigned long long red[4][C_COUNT];
    unsigned long long v[C_COUNT];
#pragma unroll
    for (int c = 0; c < C_COUNT; ++c) v[c] = 0;
    for (long long w = (long long)blockIdx.x * blockDim.x + threadIdx.x; w < nwaves;
         w += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < C_COUNT; ++c) v[c] += slots[w * C_COUNT + c];
    }
#pragma unroll
    for (int c = 0; c < C_COUNT; ++c) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off);
    }
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < C_COUNT; ++c) red[threadIdx.x >> 6][c] = v[c];
    __syncthreads();
    if (threadIdx.x < C_COUNT)
        partial[(long long)blockIdx.x * C_COUNT + threadIdx.x] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

__global__ void slots_final_kernel(const unsigned long long *partial, int nb, unsigned long long *out)
{
    const int c = threadIdx.x;
    if (c >= C_COUNT) return;
    unsigned long long t = 0;
    for (int b = 0; b < nb; ++b) t += partial[(long long)b * C_COUNT + c];
    out[c] = t;
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

template <bool CART, typename ST>
__global__ __launch_bounds__(OBS_THREADS) void obs_partial_kernel(Phys P, Eos E, double tau,
                                                                  const double *qT, const ST *qP,
                                                                  const ST *e, const double *u,
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
            qc[c] = c < PTT ? qT[c * S + s] : (double)qP[(c - PTT) * S + s];
            finite = finite && isfinite(qc[c]);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            uc[m] = (double)u[m * S + s];
            finite = finite && isfinite(uc[m]);
        }
        const double ec = (double)e[s];
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
        eos_full(E, ec, p0, cs2, T);
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

// Validity of the effective theory (Sec. 7, Eq. inverseReynoldsNumbers), per
// cell: T(e), R^{-1}_pi = sqrt(pi^{mu nu} pi_{mu nu}) / P(e) and
// R^{-1}_Pi = |Pi| / P(e), with the metric diag(1, -1, -1, -tau^2) (Milne) or
// diag(1, -1, -1, -1) (Cartesian) lowering both indices.  Each output is
// nullable.
template <bool CART, typename S>
__global__ __launch_bounds__(256) void validity_kernel(Phys P, Eos E, double tau, const S *qP, const S *e,
                                                       double *T_out, double *rpi, double *rPi)
{
    const idx_t SS = (idx_t)P.stride;
    const double w3 = CART ? -1.0 : -tau * tau;
    const double w[4] = {1.0, -1.0, -1.0, w3};
    for (idx_t i = (idx_t)blockIdx.x * blockDim.x + threadIdx.x; i < (idx_t)P.ncell;
         i += (idx_t)gridDim.x * blockDim.x) {
        double pe, cs2, T;
        eos_full(E, (double)e[i], pe, cs2, T);
        double pp = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = m; n < 4; ++n) {
                const double v = (double)qP[(idx_t)(pi_index(m, n) - PTT) * SS + i];
                pp += (m == n ? 1.0 : 2.0) * w[m] * w[n] * v * v;
            }
        const double Pi = (double)qP[(idx_t)(BPI - PTT) * SS + i];
        if (T_out) T_out[i] = T;
        if (rpi) rpi[i] = sqrt(fmax(pp, 0.0)) / pe;
        if (rPi) rPi[i] = fabs(Pi) / pe;
    }
}

// Knudsen numbers of Sec. 7, per cell: Kn_pi = tau_pi theta and
// Kn_Pi = tau_Pi theta, theta = d_mu u^mu + u^tau / tau (Milne) from the same
// differences as the sources kernel (backward in tau from u_prev, central in
// x, y, eta with the boundary conditions), tau_pi = 5 (eta/s) / T and
// 1/tau_Pi as in relaxation_sources; 0 for a component that is not evolved.
template <bool CART, typename S>
__global__ __launch_bounds__(256) void knudsen_kernel(Phys P, Eos E, double tau, const double *u, const double *up,
                                                      const S *e, double *knpi, double *knPi)
{
    const idx_t SS = (idx_t)P.stride;
    const idx_t plane = (idx_t)P.nx * P.ny;
    for (idx_t c = (idx_t)blockIdx.x * blockDim.x + threadIdx.x; c < (idx_t)P.ncell;
         c += (idx_t)gridDim.x * blockDim.x) {
        const int k = (int)(c / plane);
        const idx_t rem = c - (idx_t)k * plane;
        const int j = (int)(rem / P.nx), i = (int)(rem - (idx_t)j * P.nx);
        const idx_t row = (idx_t)k * plane + (idx_t)j * P.nx, col = (idx_t)j * P.nx + i;
        double th = (u[c] - up[c]) * P.inv_dtau;
        th += (u[SS + row + wrap(i + 1, P.nx, P.periodic[0])] - u[SS + row + wrap(i - 1, P.nx, P.periodic[0])])
              * (0.5 * P.inv_dx);
        th += (u[2 * SS + (idx_t)k * plane + (idx_t)wrap(j + 1, P.ny, P.periodic[1]) * P.nx + i]
               - u[2 * SS + (idx_t)k * plane + (idx_t)wrap(j - 1, P.ny, P.periodic[1]) * P.nx + i]) * (0.5 * P.inv_dy);
        th += (u[3 * SS + (idx_t)wrap(k + 1, P.neta, P.periodic[2]) * plane + col]
               - u[3 * SS + (idx_t)wrap(k - 1, P.neta, P.periodic[2]) * plane + col]) * (0.5 * P.inv_deta);
        if (!CART) th += u[c] / tau;
        double pe, cs2, T;
        eos_full(E, (double)e[c], pe, cs2, T);
        if (knpi) knpi[c] = P.shear ? 5.0 * P.eta_s / T * th : 0.0;
        if (knPi) {
            double v = 0.0;
            if (P.bulk) {
                const double d = 1.0 / 3.0 - cs2;
                const double inv_tPi = P.zeta_model == 1
                    ? 15.0 * d * d * T / (P.zeta_coef * zeta_over_s_paper(T / P.zeta_tc))
                    : 15.0 * d * T / P.zeta_coef;
                v = th / inv_tPi;
            }
            knPi[c] = v;
        }
    }
}

// Second-order inverse Reynolds numbers (Sec. 7, Eq. inverseReynoldsNumbers2;
// second_order_reynolds) and the regulation factor tanh(rho)/rho of Sec. 3.2
// (Eqs. regPimunu, rho) evaluated on the current state, per cell: the full
// velocity gradient from the same differences as the sources kernel (backward
// in tau from u_prev, central in x, y, eta with the boundary conditions).
// Each output is nullable.
template <bool CART, typename S>
__global__ __launch_bounds__(256) void validity2_kernel(Phys P, Eos E, double tau, const double *u,
                                                        const double *up, const S *qP, const S *e,
                                                        double *r2pi_out, double *r2Pi_out, double *reg_out)
{
    const idx_t SS = (idx_t)P.stride;
    const idx_t plane = (idx_t)P.nx * P.ny;
    for (idx_t c = (idx_t)blockIdx.x * blockDim.x + threadIdx.x; c < (idx_t)P.ncell;
         c += (idx_t)gridDim.x * blockDim.x) {
        const int k = (int)(c / plane);
        const idx_t rem = c - (idx_t)k * plane;
        const int j = (int)(rem / P.nx), i = (int)(rem - (idx_t)j * P.nx);
        const idx_t row = (idx_t)k * plane + (idx_t)j * P.nx, col = (idx_t)j * P.nx + i;
        const idx_t nb[3][2] = {
            {row + wrap(i + 1, P.nx, P.periodic[0]), row + wrap(i - 1, P.nx, P.periodic[0])},
            {(idx_t)k * plane + (idx_t)wrap(j + 1, P.ny, P.periodic[1]) * P.nx + i,
             (idx_t)k * plane + (idx_t)wrap(j - 1, P.ny, P.periodic[1]) * P.nx + i},
            {(idx_t)wrap(k + 1, P.neta, P.periodic[2]) * plane + col,
             (idx_t)wrap(k - 1, P.neta, P.periodic[2]) * plane + col}};
        const double invh[3] = {P.inv_dx, P.inv_dy, P.inv_deta};
        double uc[4], C[4][4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            uc[m] = u[m * SS + c];
            C[0][m] = (uc[m] - up[m * SS + c]) * P.inv_dtau;
#pragma unroll
            for (int d = 0; d < 3; ++d)
                C[d + 1][m] = (u[m * SS + nb[d][0]] - u[m * SS + nb[d][1]]) * (0.5 * invh[d]);
        }
        double q[NQ];
#pragma unroll
        for (int cc = PTT; cc < NQ; ++cc) q[cc] = (double)qP[(cc - PTT) * SS + c];
        const double ec = (double)e[c];
        const double Pi = P.bulk ? q[BPI] : 0.0;
        double p0, cs2, T;
        eos_full(E, ec, p0, cs2, T);
        if (r2pi_out || r2Pi_out) {
            double r2pi, r2Pi;
            second_order_reynolds<CART>(P, tau, q + PTT, Pi, ec, p0, cs2, uc, C, r2pi, r2Pi);
            if (r2pi_out) r2pi_out[c] = r2pi;
            if (r2Pi_out) r2Pi_out[c] = r2Pi;
        }
        if (reg_out) reg_out[c] = (P.regulate && P.shear) ? regulate<CART>(P, tau, q, ec, p0, uc) : 1.0;
    }
}

// ======================================================================
// Host side
// ======================================================================

struct kt_ctx {
    kt_params prm;
    Phys P;
    Eos E;
    hipStream_t stream;
    double *ws;
    // storage: T^{tau mu} in FP64; pi, Pi, e, p, u and the face speeds in the
    // storage type (8-byte double, or 4-byte float for KT_MIXED)
    bool mixed;
    size_t es;                        // bytes per element of the storage type
    double *qT[2];                    // T^{tau mu} of q (0) and q* (1)
    char *qP[2];                      // components 4..14 of q and q*
    char *e, *p, *u[3], *vf;          // u[cur], u[prev], u[star] by index below
    int ucur, uprev, ustar;
    double *tab;
    unsigned long long *slots, *ctr;
    long long nwaves;
    FaceGeo G;
    double *partial, *obs;
    float *mlp_w, *mlp_m, *mlp_v, *mlp_part;   // network parameters, Adam moments, gradient partials
    ktm::MlpPacked *mlp_pk;    // the parameters in the operand layout of the matrix-core inference
    bool mlp_pk_dirty;         // mlp_w changed since mlp_pk was packed
    double *loss_part;
    bool mlp_ready;
    int inv_start;
    double tau;
    long long step;
    char err[512];
    // profiling: pooled event pairs recorded around launches
    int prof;                  // classes whose launches are timed (bit k: class k)
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    size_t ev_used;
};

static hipError_t prof_mark(kt_ctx *c, int kind, bool start)
{
    if (!((c->prof >> kind) & 1)) return hipSuccess;
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
    size_t qT, qP, qsT, qsP, u, e, p, vf, tab, slots, ctr, partial, obs, mlp, mlp_part, loss_part, mlp_pk, total;
    long long nwaves;
    FaceGeo G;
};

static FaceGeo face_geo(const kt_params *p)
{
    FaceGeo G;
    G.nfx = (long long)(p->nx + 1) * p->ny * p->neta;
    G.nfy = (long long)p->nx * (p->ny + 1) * p->neta;
    G.nfe = (long long)p->nx * p->ny * (p->neta + 1);
    G.ox = 0;
    G.oy = 2 * G.nfx;
    G.oe = G.oy + 2 * G.nfy;
    return G;
}

static long long face_waves(const kt_params *p)
{
    return (long long)face_launch(face_geo(p), p->nx, p->ny).nblocks * (FACE_BLOCK / 64);
}

static long long stage_waves(const kt_params *p)
{
    return (long long)((p->nx + 63) / 64) * ((p->ny + 3) / 4) * p->neta * 4;
}

static long long recover_waves(const kt_params *p)
{
    const long long n = (long long)p->nx * p->ny * p->neta;
    return (n + 255) / 256 * 4;
}

static Layout layout(const kt_params *p, const kt_eos *eos)
{
    Layout L;
    const size_t es = p->precision == KT_MIXED ? sizeof(float) : sizeof(double);
    const size_t S8 = (size_t)cell_stride(p) * sizeof(double), SE = (size_t)cell_stride(p) * es;
    size_t off = 0;   // every array starts on a 256-byte boundary (the stride is a multiple of 64)
    L.qT = off;  off += 4 * S8;
    L.qP = off;  off += 11 * SE;
    L.qsT = off; off += 4 * S8;
    L.qsP = off; off += 11 * SE;
    L.u = off;  off += 12 * S8;   // u^mu is FP64 in both precisions
    L.e = off;  off += SE;
    L.p = off;  off += SE;
    L.G = face_geo(p);
    L.vf = off; off += round_up((size_t)(L.G.oe + 2 * L.G.nfe) * es, 256);
    L.tab = off; off += round_up((size_t)(eos->conformal ? 1 : eos->n) * EOS_W * sizeof(double), 256);
    const long long sw = stage_waves(p), rw = recover_waves(p), fw = face_waves(p);
    L.nwaves = sw > rw ? sw : rw;
    L.nwaves = L.nwaves > fw ? L.nwaves : fw;
    L.slots = off; off += round_up((size_t)L.nwaves * C_COUNT * sizeof(unsigned long long), 256);
    L.ctr = off; off += 256;
    // observables partials, reused afterwards for the counter partials
    L.partial = off;
    off += round_up(std::max((size_t)OBS_BLOCKS * O_COUNT * sizeof(double),
                             (size_t)SLOT_BLOCKS * C_COUNT * sizeof(unsigned long long)), 256);
    L.obs = off; off += 256;
    L.mlp = off; off += round_up((size_t)3 * ktm::NP * sizeof(float), 256);
    L.mlp_part = off; off += round_up((size_t)ktm::BWD_BLOCKS * ktm::NP * sizeof(float), 256);
    L.loss_part = off; off += round_up((size_t)(ktm::LOSS_BLOCKS + 1) * sizeof(double), 256);
    L.mlp_pk = off; off += round_up(sizeof(ktm::MlpPacked), 256);
    L.total = off;
    return L;
}

static const char *check_args(const kt_params *p, const kt_eos *eos)
{
    if (!p || !eos) return "null params or eos";
    if (p->nx < 1 || p->ny < 1 || p->neta < 1) return "grid sizes must be >= 1";
    if ((long long)(p->nx + 1) * (p->ny + 1) * (p->neta + 1) * 15 * 8 >= (1LL << 32))
        return "grid too large: each field array is addressed with 32-bit byte offsets "
               "(15 components x cells x 8 B must stay below 4 GiB)";
    if (!(p->dx > 0) || !(p->dy > 0) || !(p->deta > 0)) return "cell sizes must be > 0";
    if (!(p->dtau > 0)) return "dtau must be > 0";
    if (p->coords != KT_MILNE && p->coords != KT_CARTESIAN) return "coords must be KT_MILNE or KT_CARTESIAN";
    if (p->coords == KT_MILNE && !(p->tau0 > 0)) return "tau0 must be > 0 in Milne coordinates";
    for (int d = 0; d < 3; ++d)
        if (p->bc[d] != KT_BC_OUTFLOW && p->bc[d] != KT_BC_PERIODIC) return "bc must be outflow or periodic";
    if (!(p->theta >= 1.0 && p->theta <= 2.0)) return "theta must lie in [1, 2]";
    if (!(p->eta_over_s >= 0) || !(p->zeta_coef >= 0) || !(p->taupipi >= 0)) return "transport parameters must be >= 0";
    if (p->zeta_model != KT_ZETA_LINEAR && p->zeta_model != KT_ZETA_PAPER) return "zeta_model must be KT_ZETA_LINEAR or KT_ZETA_PAPER";
    if (p->zeta_model == KT_ZETA_PAPER && !(p->zeta_tc > 0)) return "zeta_tc must be > 0 for KT_ZETA_PAPER";
    if (p->regulate && (!(p->xi0 > 0) || !(p->rho_max > 0))) return "regulator constants must be > 0";
    if (!(p->e_floor > 0)) return "e_floor must be > 0";
    if (!(p->m2_delta > 0 && p->m2_delta < 1)) return "m2_delta must lie in (0, 1)";
    if (!(p->newton_tol > 0) || p->newton_max < 1) return "Newton tolerance and iteration limit must be positive";
    if (p->precision != KT_FP64 && p->precision != KT_MIXED) return "precision must be KT_FP64 or KT_MIXED";
    if (p->reduced != 0 && p->reduced != 1) return "reduced must be 0 or 1";
    if (eos->conformal) {
        if (!(eos->a_sb > 0)) return "conformal EOS needs a_sb > 0";
    } else {
        if (eos->n < 2) return "EOS table needs n >= 2";
        if (!eos->p || !eos->cs2 || !eos->T) return "EOS table arrays are null";
        if (!(eos->dln_e > 0)) return "EOS table needs dln_e > 0";
    }
    return nullptr;
}

// EOS table nodes on the host: per node p/e, T/e^{1/4}, c_s^2, 1/e_i with
// e_i = exp(ln_e0 + i dln_e); h holds EOS_W * eos->n doubles
static void eos_nodes_host(const kt_eos *eos, double *h)
{
    for (int i = 0; i < eos->n; ++i) {
        const double ei = exp(eos->ln_e0 + eos->dln_e * (double)i);
        h[EOS_W * i] = eos->p[i] / ei;
        h[EOS_W * i + 1] = eos->T[i] / sqrt(sqrt(ei));
        h[EOS_W * i + 2] = eos->cs2[i];
        h[EOS_W * i + 3] = 1.0 / ei;
    }
}

// kernels instantiated for theta = 1 take the limiter's exact shortcut (limited<true>)
static bool theta_is_one(double theta)
{
#ifdef KT_NO_THETA1
    (void)theta;
    return false;
#else
    return theta == 1.0;
#endif
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
    P.zeta_model = p->zeta_model == KT_ZETA_PAPER ? 1 : 0; P.zeta_tc = p->zeta_tc;
    P.shear = p->eta_over_s > 0; P.bulk = p->zeta_coef > 0;
    P.regulate = p->regulate != 0; P.regulate_bulk = p->regulate_bulk != 0;
    P.floor_reset = p->floor_resets_q != 0;
    P.xi0 = p->xi0; P.rho_max = p->rho_max;
    P.e_floor = p->e_floor; P.m2_delta = p->m2_delta; P.newton_tol = p->newton_tol;
    P.newton_max = p->newton_max;
    P.reduced = p->reduced;
}

template <typename K, typename... A>
static hipError_t launch(K kernel, dim3 g, dim3 b, hipStream_t st, A... args)
{
    hipLaunchKernelGGL(kernel, g, b, 0, st, args...);
    return hipGetLastError();
}

static dim3 linear_grid(long long n) { return dim3((unsigned)((n + 255) / 256)); }

// repack the network's parameters for the matrix-core inference if they
// changed (kt_mlp_set, kt_mlp_adam); stream-ordered
static hipError_t ensure_packed(kt_ctx *c)
{
    if (!c->mlp_pk_dirty) return hipSuccess;
    hipError_t e = launch(ktm::mlp_pack_kernel, dim3(1), dim3(256), c->stream, (const float *)c->mlp_w, c->mlp_pk);
    if (e == hipSuccess) c->mlp_pk_dirty = false;
    return e;
}

// warm != 0: a step's recovery, whose start follows the context's choice
// (previous e, conformal closed form, or the network); warm == 0: conformal.
// which: 0 = q, 1 = q*; ub: u buffer receiving u; us: u buffer holding the
// flow before the stage, where a reduced state's fixed point starts (-1: at rest).
template <typename S>
static kt_status run_recover_t(kt_ctx *c, double tau, int which, int ub, int regulate, int warm, int us)
{
    const bool cart = c->prm.coords == KT_CARTESIAN;
    if (c->P.reduced) {
        hipError_t e = prof_mark(c, 1, true);
        if (e != hipSuccess) return fail(c, KT_E_HIP, "profiling event: %s", hipGetErrorString(e));
        const double *u0 = us >= 0 ? (const double *)c->u[us] : nullptr;
        double *qT = c->qT[which];
        S *qP = (S *)c->qP[which], *ee = (S *)c->e, *pp = (S *)c->p;
        double *uu = (double *)c->u[ub];
        const dim3 g = linear_grid(c->P.ncell), b(256);
        e = cart ? launch(recover_reduced_kernel<true, S>, g, b, c->stream, c->P, c->E, tau, qT, qP, ee, pp, uu,
                          u0, regulate, c->slots)
                 : launch(recover_reduced_kernel<false, S>, g, b, c->stream, c->P, c->E, tau, qT, qP, ee, pp, uu,
                          u0, regulate, c->slots);
        if (e == hipSuccess) e = prof_mark(c, 1, false);
        if (e != hipSuccess) return fail(c, KT_E_HIP, "recover kernel: %s", hipGetErrorString(e));
        return KT_OK;
    }
    const bool learned = warm && c->inv_start == KT_START_LEARNED;
    if (warm && c->inv_start == KT_START_CONFORMAL) warm = 0;
    if (learned) warm = 0;
    hipError_t e = learned ? ensure_packed(c) : hipSuccess;
    if (e != hipSuccess) return fail(c, KT_E_HIP, "network packing: %s", hipGetErrorString(e));
    e = prof_mark(c, 1, true);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "profiling event: %s", hipGetErrorString(e));
    const dim3 g = linear_grid(c->P.ncell), b(256);
    const ktm::MlpPacked *w = c->mlp_pk;
    double *qT = c->qT[which];
    S *qP = (S *)c->qP[which], *ee = (S *)c->e, *pp = (S *)c->p;
    double *uu = (double *)c->u[ub];
    if (cart)
        e = learned ? launch(recover_kernel<true, true, S>, g, b, c->stream, c->P, c->E, tau, qT, qP, ee, pp,
                             uu, regulate, warm, w, c->slots)
                    : launch(recover_kernel<true, false, S>, g, b, c->stream, c->P, c->E, tau, qT, qP, ee, pp,
                             uu, regulate, warm, w, c->slots);
    else
        e = learned ? launch(recover_kernel<false, true, S>, g, b, c->stream, c->P, c->E, tau, qT, qP, ee, pp,
                             uu, regulate, warm, w, c->slots)
                    : launch(recover_kernel<false, false, S>, g, b, c->stream, c->P, c->E, tau, qT, qP, ee, pp,
                             uu, regulate, warm, w, c->slots);
    if (e == hipSuccess) e = prof_mark(c, 1, false);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "recover kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

static kt_status run_recover(kt_ctx *c, double tau, int which, int ub, int regulate, int warm, int us)
{
    return c->mixed ? run_recover_t<float>(c, tau, which, ub, regulate, warm, us)
                    : run_recover_t<double>(c, tau, which, ub, regulate, warm, us);
}

template <typename S>
static kt_status run_faces_t(kt_ctx *c, double tau, int which)
{
    const bool cart = c->prm.coords == KT_CARTESIAN;
    hipError_t e = prof_mark(c, 2, true);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "profiling event: %s", hipGetErrorString(e));
    const FaceLaunch L = face_launch(c->G, c->P.nx, c->P.ny);
    const dim3 g(L.nblocks), b(FACE_BLOCK);
    const double *qT = c->qT[which];
    const S *qP = (const S *)c->qP[which];
    const bool t1 = theta_is_one(c->P.theta);
    auto K = cart ? (t1 ? face_speeds_kernel<true, true, S> : face_speeds_kernel<true, false, S>)
                  : (t1 ? face_speeds_kernel<false, true, S> : face_speeds_kernel<false, false, S>);
    e = launch(K, g, b, c->stream, c->P, c->E, c->G, L, tau, qT, qP, (S *)c->vf, c->slots);
    if (e == hipSuccess) e = prof_mark(c, 2, false);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "face kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

static kt_status run_faces(kt_ctx *c, double tau, int which)
{
    return c->mixed ? run_faces_t<float>(c, tau, which) : run_faces_t<double>(c, tau, which);
}

// one Euler stage on q (stage 1: q^n, src 0, into q*) or q* (stage 2: src 1,
// into q^{n+1} over q^n), with flow u[ub] and previous flow u[ubp]
template <typename S>
static kt_status run_stage_t(kt_ctx *c, bool stage2, double tau, int src, int ub, int ubp)
{
    const bool cart = c->prm.coords == KT_CARTESIAN;
    const Phys &P = c->P;
    const dim3 b(64, 4);
    const dim3 gs((P.nx + 63) / 64, (P.ny + 3) / 4, P.neta);
    Fields<S> F = {c->qT[src], (const S *)c->qP[src], (const S *)c->e, (const S *)c->p,
                   (const double *)c->u[ub], (const double *)c->u[ubp], (const S *)c->vf};
    const int dst = 1 - src;
    double *outT = c->qT[dst];
    S *outP = (S *)c->qP[dst];
    const double *qnT = stage2 ? c->qT[0] : nullptr;
    const S *qnP = stage2 ? (const S *)c->qP[0] : nullptr;
    hipError_t e = prof_mark(c, 3, true);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "profiling event: %s", hipGetErrorString(e));
    if (cart)
        e = stage2 ? launch(sources_kernel<true, true, S>, gs, b, c->stream, P, c->E, tau, F, qnT, qnP, outT, outP)
                   : launch(sources_kernel<true, false, S>, gs, b, c->stream, P, c->E, tau, F, qnT, qnP, outT, outP);
    else
        e = stage2 ? launch(sources_kernel<false, true, S>, gs, b, c->stream, P, c->E, tau, F, qnT, qnP, outT, outP)
                   : launch(sources_kernel<false, false, S>, gs, b, c->stream, P, c->E, tau, F, qnT, qnP, outT, outP);
    if (e == hipSuccess) e = prof_mark(c, 3, false);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "sources kernel: %s", hipGetErrorString(e));
    const dim3 gf((P.nx + 63) / 64, (P.ny + 3) / 4, (P.neta + KC - 1) / KC);
    e = prof_mark(c, 0, true);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "profiling event: %s", hipGetErrorString(e));
    const bool t1 = theta_is_one(P.theta);
    auto K = stage2 ? (t1 ? flux_kernel<true, true, S, KC> : flux_kernel<true, false, S, KC>)
                    : (t1 ? flux_kernel<false, true, S, KC> : flux_kernel<false, false, S, KC>);
    e = launch(K, gf, b, c->stream, P, c->G, F.qT, F.qP, F.vf, outT, outP, 4);
    if (e == hipSuccess) e = prof_mark(c, 0, false);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "flux kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

static kt_status run_stage(kt_ctx *c, bool stage2, double tau, int src, int ub, int ubp)
{
    return c->mixed ? run_stage_t<float>(c, stage2, tau, src, ub, ubp)
                    : run_stage_t<double>(c, stage2, tau, src, ub, ubp);
}

// FP64 device array -> storage-type array (n elements), or a plain copy
static hipError_t store_from_double(kt_ctx *c, char *dst, const double *src, long long n)
{
    if (!c->mixed)
        return hipMemcpyAsync(dst, src, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, c->stream);
    return launch(from_double_kernel, linear_grid(n), dim3(256), c->stream, n, src, (float *)dst);
}

// storage-type array -> FP64 device array
static hipError_t store_to_double(kt_ctx *c, double *dst, const char *src, long long n)
{
    if (!c->mixed)
        return hipMemcpyAsync(dst, src, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, c->stream);
    return launch(to_double_kernel<float>, linear_grid(n), dim3(256), c->stream, n, (const float *)src, dst);
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

    if (!s0 || !d_ws) return fail(nullptr, KT_E_ARG, "null initial state or workspace");
    if (((uintptr_t)d_ws) % 256) return fail(nullptr, KT_E_ARG, "workspace must be 256-byte aligned");
    const bool have_q = s0->q[0] != nullptr;
    // q with e and u: a state exported by kt_observables, taken as it is (resume)
    const bool resume = have_q && s0->e != nullptr;
    if (have_q) {
        for (int c = 0; c < 15; ++c)
            if (!s0->q[c]) return fail(nullptr, KT_E_ARG, "initial q[%d] is null", c);
        if (resume)
            for (int m = 0; m < 4; ++m)
                if (!s0->u[m]) return fail(nullptr, KT_E_ARG, "resume: initial u[%d] is null", m);
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
    c->mixed = p->precision == KT_MIXED;
    c->es = c->mixed ? sizeof(float) : sizeof(double);
    const long long S = c->P.stride;
    const size_t SE = (size_t)S * c->es;
    c->qT[0] = (double *)(base + L.qT);
    c->qP[0] = base + L.qP;
    c->qT[1] = (double *)(base + L.qsT);
    c->qP[1] = base + L.qsP;
    const size_t S8 = (size_t)S * sizeof(double);
    for (int b = 0; b < 3; ++b) c->u[b] = base + L.u + 4 * S8 * b;
    c->ucur = 0; c->uprev = 1; c->ustar = 2;
    c->e = base + L.e;
    c->p = base + L.p;
    c->tab = (double *)(base + L.tab);
    c->slots = (unsigned long long *)(base + L.slots);
    c->ctr = (unsigned long long *)(base + L.ctr);
    c->nwaves = L.nwaves;
    c->vf = base + L.vf;
    c->G = L.G;
    c->partial = (double *)(base + L.partial);
    c->obs = (double *)(base + L.obs);
    c->mlp_w = (float *)(base + L.mlp);
    c->mlp_m = c->mlp_w + ktm::NP;
    c->mlp_v = c->mlp_m + ktm::NP;
    c->mlp_part = (float *)(base + L.mlp_part);
    c->loss_part = (double *)(base + L.loss_part);
    c->mlp_pk = (ktm::MlpPacked *)(base + L.mlp_pk);
    c->mlp_pk_dirty = true;
    c->mlp_ready = false;
    c->inv_start = KT_START_CONFORMAL;   // the oracle's start, and the fastest measured
    c->tau = p->tau0;
    c->step = 0;

    // EOS table: per node p/e, T/e^{1/4}, c_s^2, 1/e_i (node e_i = exp(ln_e0 + i dln_e))
    c->E.conformal = eos->conformal != 0;
    c->E.inv_a = eos->conformal ? 1.0 / eos->a_sb : 0.0;
    c->E.n = eos->conformal ? 0 : eos->n;
    c->E.ln_e0 = eos->ln_e0;
    c->E.inv_dln = eos->conformal ? 0.0 : 1.0 / eos->dln_e;
    c->E.tab = c->tab;
    c->P.p_floor = p->e_floor / 3.0;
    if (!eos->conformal) {
        double *h = (double *)malloc(sizeof(double) * EOS_W * eos->n);
        if (!h) { delete c; return fail(nullptr, KT_E_ALLOC, "host allocation failed"); }
        eos_nodes_host(eos, h);
        Eos hE = c->E;   // same interpolation on the host for p(e_floor)
        hE.tab = h;
        c->P.p_floor = eos_p(hE, p->e_floor);
        hipError_t e1 = hipMemcpyAsync(c->tab, h, sizeof(double) * EOS_W * eos->n, hipMemcpyHostToDevice, stream);
        hipError_t e2 = hipStreamSynchronize(stream);
        free(h);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            kt_status st = fail(nullptr, KT_E_HIP, "EOS upload: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
            delete c;
            return st;
        }
    }
    hipError_t he = hipMemsetAsync(c->slots, 0, (size_t)L.nwaves * C_COUNT * sizeof(unsigned long long), stream);
    if (he != hipSuccess) { delete c; return fail(nullptr, KT_E_HIP, "memset: %s", hipGetErrorString(he)); }

    // q^0
    const size_t bytes = sizeof(double) * (size_t)c->P.ncell;
    if (have_q) {
        for (int k = 0; k < 15 && he == hipSuccess; ++k)
            he = k < PTT ? hipMemcpyAsync(c->qT[0] + k * S, s0->q[k], bytes, hipMemcpyDeviceToDevice, stream)
                         : store_from_double(c, c->qP[0] + (k - PTT) * SE, s0->q[k], c->P.ncell);
    } else {
        PrimPtrs in;
        in.e = s0->e;
        for (int m = 0; m < 4; ++m) in.u[m] = s0->u[m];
        for (int k = 0; k < 10; ++k) in.pi[k] = s0->pi[k];
        in.Pi = s0->Pi;
        he = c->mixed ? launch(tmunu_kernel<float>, linear_grid(c->P.ncell), dim3(256), stream, c->P, c->E, in,
                               c->qT[0], (float *)c->qP[0])
                      : launch(tmunu_kernel<double>, linear_grid(c->P.ncell), dim3(256), stream, c->P, c->E, in,
                               c->qT[0], (double *)c->qP[0]);
    }
    if (he != hipSuccess) { kt_destroy(c); return fail(nullptr, KT_E_HIP, "initial state: %s", hipGetErrorString(he)); }
    // (e^0, u^0) and u^{-1}: recovered from q, or (resume) taken as given with
    // p = p(e) when p is not given
    kt_status st = KT_OK;
    if (resume) {
        he = store_from_double(c, c->e, s0->e, c->P.ncell);
        for (int m = 0; m < 4 && he == hipSuccess; ++m)
            he = hipMemcpyAsync(c->u[c->ucur] + m * S8, s0->u[m], bytes, hipMemcpyDeviceToDevice, stream);
        if (he == hipSuccess)
            he = s0->p ? store_from_double(c, c->p, s0->p, c->P.ncell)
                       : (c->mixed ? launch(pressure_kernel<float>, linear_grid(c->P.ncell), dim3(256), stream, c->E,
                                            (long long)c->P.ncell, (const float *)c->e, (float *)c->p)
                                   : launch(pressure_kernel<double>, linear_grid(c->P.ncell), dim3(256), stream,
                                            c->E, (long long)c->P.ncell, (const double *)c->e, (double *)c->p));
        if (he != hipSuccess) {
            kt_destroy(c);
            return fail(nullptr, KT_E_HIP, "resumed state: %s", hipGetErrorString(he));
        }
    } else {
        st = run_recover(c, c->tau, 0, c->ucur, 0, 0, -1);
    }
    if (st == KT_OK) st = run_faces(c, c->tau, 0);
    if (st != KT_OK) { kt_status r = fail(nullptr, st, "%s", c->err); kt_destroy(c); return r; }
    for (int m = 0; m < 4 && he == hipSuccess; ++m)
        he = hipMemcpyAsync(c->u[c->uprev] + m * S8, have_up ? (const char *)s0->u_prev[m] : c->u[c->ucur] + m * S8,
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
    for (int s = 0; s < n_steps; ++s) {
        const double tau0 = c->tau, tau1 = c->tau + c->prm.dtau;
        // face speeds of q^n are current (computed after the previous recovery)
        kt_status st = run_stage(c, false, tau0, 0, c->ucur, c->uprev);
        if (st != KT_OK) return st;
        st = run_recover(c, tau1, 1, c->ustar, 1, 1, c->ucur);
        if (st == KT_OK) st = run_faces(c, tau1, 1);
        if (st != KT_OK) return st;
        st = run_stage(c, true, tau1, 1, c->ustar, c->ucur);
        if (st != KT_OK) return st;
        // u^{n-1} <- u^n; (e, u)^{n+1} into the freed buffer
        const int freed = c->uprev;
        st = run_recover(c, tau1, 0, freed, 1, 1, c->ustar);
        if (st == KT_OK) st = run_faces(c, tau1, 0);
        if (st != KT_OK) return st;
        c->uprev = c->ucur;
        c->ucur = freed;
        c->tau = tau1;
        c->step += 1;
    }
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
    const bool learned = c->inv_start == KT_START_LEARNED;
    const ktm::MlpPacked *w = c->mlp_pk;
    hipError_t e = learned ? ensure_packed(c) : hipSuccess;
    if (e != hipSuccess) return fail(c, KT_E_HIP, "network packing: %s", hipGetErrorString(e));
    if (c->prm.coords == KT_CARTESIAN)
        e = learned ? launch(recover_standalone_kernel<true, true>, linear_grid(n), dim3(256), c->stream, c->P, c->E, tau, (long long)n, R, w)
                    : launch(recover_standalone_kernel<true, false>, linear_grid(n), dim3(256), c->stream, c->P, c->E, tau, (long long)n, R, w);
    else
        e = learned ? launch(recover_standalone_kernel<false, true>, linear_grid(n), dim3(256), c->stream, c->P, c->E, tau, (long long)n, R, w)
                    : launch(recover_standalone_kernel<false, false>, linear_grid(n), dim3(256), c->stream, c->P, c->E, tau, (long long)n, R, w);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "recover kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

kt_status kt_recover_reduced(kt_ctx *c, int64_t n, double tau, const double *const in[10], double *e_out,
                             double *const u_out[4], double *const pi_out[5], int32_t *passes_out,
                             int32_t *flags_out)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (n < 0) return fail(c, KT_E_ARG, "n must be >= 0");
    if (n == 0) return KT_OK;
    if (!in || !e_out || !u_out) return fail(c, KT_E_ARG, "null input or output arrays");
    for (int k = 0; k < 9; ++k)
        if (!in[k]) return fail(c, KT_E_ARG, "input %d is null", k);
    for (int m = 0; m < 4; ++m)
        if (!u_out[m]) return fail(c, KT_E_ARG, "u_out[%d] is null", m);
    if (pi_out)
        for (int k = 0; k < 5; ++k)
            if (!pi_out[k]) return fail(c, KT_E_ARG, "pi_out[%d] is null", k);
    if (c->prm.coords == KT_MILNE && !(tau > 0)) return fail(c, KT_E_ARG, "tau must be > 0");
    RecRedIn R;
    for (int k = 0; k < 10; ++k) R.in[k] = in[k];
    R.e = e_out;
    for (int m = 0; m < 4; ++m) R.u[m] = u_out[m];
    for (int k = 0; k < 5; ++k) R.pi[k] = pi_out ? pi_out[k] : nullptr;
    R.passes = passes_out;
    R.flags = flags_out;
    const hipError_t e = c->prm.coords == KT_CARTESIAN
        ? launch(recover_reduced_standalone_kernel<true>, linear_grid(n), dim3(256), c->stream, c->P, c->E, tau,
                 (long long)n, R)
        : launch(recover_reduced_standalone_kernel<false>, linear_grid(n), dim3(256), c->stream, c->P, c->E, tau,
                 (long long)n, R);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "recover kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

kt_status kt_observables(kt_ctx *c, kt_obs *host_out, const kt_fields *dev_out)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    const long long S = c->P.stride, n = c->P.ncell;
    const size_t SE = (size_t)S * c->es;
    const size_t bytes = sizeof(double) * (size_t)n;
    hipError_t e = hipSuccess;
    if (dev_out) {
        if (dev_out->e) e = store_to_double(c, dev_out->e, c->e, n);
        if (e == hipSuccess && dev_out->p) e = store_to_double(c, dev_out->p, c->p, n);
        for (int m = 0; m < 4 && e == hipSuccess; ++m) {
            if (dev_out->u[m])
                e = hipMemcpyAsync(dev_out->u[m], (const double *)c->u[c->ucur] + m * S, bytes, hipMemcpyDeviceToDevice,
                                   c->stream);
            if (e == hipSuccess && dev_out->u_prev[m])
                e = hipMemcpyAsync(dev_out->u_prev[m], (const double *)c->u[c->uprev] + m * S, bytes,
                                   hipMemcpyDeviceToDevice, c->stream);
        }
        for (int k = 0; k < 15 && e == hipSuccess; ++k)
            if (dev_out->q[k])
                e = k < PTT ? hipMemcpyAsync(dev_out->q[k], c->qT[0] + k * S, bytes, hipMemcpyDeviceToDevice, c->stream)
                            : store_to_double(c, dev_out->q[k], c->qP[0] + (k - PTT) * SE, n);
        if (e != hipSuccess) return fail(c, KT_E_HIP, "field export: %s", hipGetErrorString(e));
    }
    double res[O_COUNT];
    unsigned long long ctr[C_COUNT];
    if (host_out) {
        const bool cart = c->prm.coords == KT_CARTESIAN;
        const dim3 g(OBS_BLOCKS), b(OBS_THREADS);
        const double *qT = c->qT[0];
        if (c->mixed)
            e = cart ? launch(obs_partial_kernel<true, float>, g, b, c->stream, c->P, c->E, c->tau, qT,
                              (const float *)c->qP[0], (const float *)c->e, (const double *)c->u[c->ucur], c->partial)
                     : launch(obs_partial_kernel<false, float>, g, b, c->stream, c->P, c->E, c->tau, qT,
                              (const float *)c->qP[0], (const float *)c->e, (const double *)c->u[c->ucur], c->partial);
        else
            e = cart ? launch(obs_partial_kernel<true, double>, g, b, c->stream, c->P, c->E, c->tau, qT,
                              (const double *)c->qP[0], (const double *)c->e, (const double *)c->u[c->ucur], c->partial)
                     : launch(obs_partial_kernel<false, double>, g, b, c->stream, c->P, c->E, c->tau, qT,
                              (const double *)c->qP[0], (const double *)c->e, (const double *)c->u[c->ucur], c->partial);
        if (e == hipSuccess)
            e = launch(obs_final_kernel, dim3(1), dim3(64), c->stream, (const double *)c->partial, OBS_BLOCKS, c->obs);
        if (e == hipSuccess)
            e = launch(slots_partial_kernel, dim3(SLOT_BLOCKS), dim3(256), c->stream,
                       (const unsigned long long *)c->slots, c->nwaves, (unsigned long long *)c->partial);
        if (e == hipSuccess)
            e = launch(slots_final_kernel, dim3(1), dim3(64), c->stream,
                       (const unsigned long long *)c->partial, SLOT_BLOCKS, c->ctr);
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
        host_out->n_fallback_faces = (int64_t)ctr[C_FALLBACK_FACES];
        host_out->fp_passes = (int64_t)ctr[C_FP_PASSES];
        host_out->fp_not_converged = (int64_t)ctr[C_FP_NOCONV];
    }
    return KT_OK;
}

kt_status kt_validity(kt_ctx *c, double *T_out, double *rinv_pi, double *rinv_Pi, double *kn_pi,
                      double *kn_Pi, double *rinv2_pi, double *rinv2_Pi, double *reg_factor)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (rinv2_pi || rinv2_Pi || reg_factor) {
        const dim3 g((unsigned)std::min<long long>((c->P.ncell + 255) / 256, 8192)), b(256);
        const double *u = (const double *)c->u[c->ucur], *up = (const double *)c->u[c->uprev];
        const bool cart = c->prm.coords == KT_CARTESIAN;
        hipError_t e;
        if (c->mixed)
            e = cart ? launch(validity2_kernel<true, float>, g, b, c->stream, c->P, c->E, c->tau, u, up,
                              (const float *)c->qP[0], (const float *)c->e, rinv2_pi, rinv2_Pi, reg_factor)
                     : launch(validity2_kernel<false, float>, g, b, c->stream, c->P, c->E, c->tau, u, up,
                              (const float *)c->qP[0], (const float *)c->e, rinv2_pi, rinv2_Pi, reg_factor);
        else
            e = cart ? launch(validity2_kernel<true, double>, g, b, c->stream, c->P, c->E, c->tau, u, up,
                              (const double *)c->qP[0], (const double *)c->e, rinv2_pi, rinv2_Pi, reg_factor)
                     : launch(validity2_kernel<false, double>, g, b, c->stream, c->P, c->E, c->tau, u, up,
                              (const double *)c->qP[0], (const double *)c->e, rinv2_pi, rinv2_Pi, reg_factor);
        if (e != hipSuccess) return fail(c, KT_E_HIP, "second-order validity: %s", hipGetErrorString(e));
    }
    if (kn_pi || kn_Pi) {
        const dim3 g((unsigned)std::min<long long>((c->P.ncell + 255) / 256, 8192)), b(256);
        const double *u = (const double *)c->u[c->ucur], *up = (const double *)c->u[c->uprev];
        const bool cart = c->prm.coords == KT_CARTESIAN;
        hipError_t e;
        if (c->mixed)
            e = cart ? launch(knudsen_kernel<true, float>, g, b, c->stream, c->P, c->E, c->tau, u, up,
                              (const float *)c->e, kn_pi, kn_Pi)
                     : launch(knudsen_kernel<false, float>, g, b, c->stream, c->P, c->E, c->tau, u, up,
                              (const float *)c->e, kn_pi, kn_Pi);
        else
            e = cart ? launch(knudsen_kernel<true, double>, g, b, c->stream, c->P, c->E, c->tau, u, up,
                              (const double *)c->e, kn_pi, kn_Pi)
                     : launch(knudsen_kernel<false, double>, g, b, c->stream, c->P, c->E, c->tau, u, up,
                              (const double *)c->e, kn_pi, kn_Pi);
        if (e != hipSuccess) return fail(c, KT_E_HIP, "knudsen: %s", hipGetErrorString(e));
    }
    if (!T_out && !rinv_pi && !rinv_Pi) return KT_OK;
    const bool cart = c->prm.coords == KT_CARTESIAN;
    const long long n = c->P.ncell;
    const dim3 g((unsigned)std::min<long long>((n + 255) / 256, 8192)), b(256);
    hipError_t e;
    if (c->mixed)
        e = cart ? launch(validity_kernel<true, float>, g, b, c->stream, c->P, c->E, c->tau, (const float *)c->qP[0],
                          (const float *)c->e, T_out, rinv_pi, rinv_Pi)
                 : launch(validity_kernel<false, float>, g, b, c->stream, c->P, c->E, c->tau, (const float *)c->qP[0],
                          (const float *)c->e, T_out, rinv_pi, rinv_Pi);
    else
        e = cart ? launch(validity_kernel<true, double>, g, b, c->stream, c->P, c->E, c->tau, (const double *)c->qP[0],
                          (const double *)c->e, T_out, rinv_pi, rinv_Pi)
                 : launch(validity_kernel<false, double>, g, b, c->stream, c->P, c->E, c->tau, (const double *)c->qP[0],
                          (const double *)c->e, T_out, rinv_pi, rinv_Pi);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "validity: %s", hipGetErrorString(e));
    return KT_OK;
}

kt_status kt_run_to_freezeout(kt_ctx *c, double T_f, int32_t max_steps, int32_t check_every,
                              int32_t *steps_done)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (!steps_done) return fail(c, KT_E_ARG, "steps_done is null");
    *steps_done = 0;
    if (!(T_f > 0) || max_steps < 0 || check_every < 1)
        return fail(c, KT_E_ARG, "need T_f > 0, max_steps >= 0, check_every >= 1");
    kt_obs o;
    kt_status st = kt_observables(c, &o, nullptr);
    while (st == KT_OK && o.T_max >= T_f && *steps_done < max_steps) {
        const int32_t k = std::min(check_every, max_steps - *steps_done);
        st = kt_step(c, k);
        if (st == KT_OK) {
            *steps_done += k;
            st = kt_observables(c, &o, nullptr);
        }
    }
    return st;
}

kt_status kt_set_inv_start(kt_ctx *c, int32_t start)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (start != KT_START_WARM && start != KT_START_CONFORMAL && start != KT_START_LEARNED)
        return fail(c, KT_E_ARG, "unknown start %d", start);
    if (start == KT_START_LEARNED && !c->mlp_ready)
        return fail(c, KT_E_STATE, "the learned start needs parameters (kt_mlp_set)");
    if (c->P.reduced && start != KT_START_CONFORMAL)
        return fail(c, KT_E_UNSUPPORTED, "a reduced state starts every inversion from the conformal closed form");
    c->inv_start = start;
    return KT_OK;
}

kt_status kt_mlp_set(kt_ctx *c, const float *d_params, int32_t n_params)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (!d_params) return fail(c, KT_E_ARG, "null parameters");
    if (n_params != KT_MLP_NPARAMS) return fail(c, KT_E_ARG, "n_params must be %d", KT_MLP_NPARAMS);
    const size_t b = sizeof(float) * ktm::NP;
    hipError_t e = hipMemcpyAsync(c->mlp_w, d_params, b, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->mlp_m, 0, 2 * b, c->stream);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "kt_mlp_set: %s", hipGetErrorString(e));
    c->mlp_ready = true;
    c->mlp_pk_dirty = true;
    return KT_OK;
}

kt_status kt_mlp_get(kt_ctx *c, float *d_params, int32_t n_params)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (!d_params || n_params != KT_MLP_NPARAMS) return fail(c, KT_E_ARG, "need %d parameters", KT_MLP_NPARAMS);
    if (!c->mlp_ready) return fail(c, KT_E_STATE, "no parameters set");
    hipError_t e = hipMemcpyAsync(d_params, c->mlp_w, sizeof(float) * ktm::NP, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "kt_mlp_get: %s", hipGetErrorString(e));
    return KT_OK;
}

kt_status kt_mlp_features(kt_ctx *c, int64_t n, double tau, const double *const in[9],
                          const double *e_in, const double *const u_in[4], float *x, float *y)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (n < 0) return fail(c, KT_E_ARG, "n must be >= 0");
    if (n == 0) return KT_OK;
    if (!in || !x) return fail(c, KT_E_ARG, "null input or output");
    for (int k = 0; k < 8; ++k)
        if (!in[k]) return fail(c, KT_E_ARG, "input %d is null", k);
    if (y && (!e_in || !u_in || !u_in[0] || !u_in[1] || !u_in[2] || !u_in[3]))
        return fail(c, KT_E_ARG, "targets need e and u");
    if (c->prm.coords == KT_MILNE && !(tau > 0)) return fail(c, KT_E_ARG, "tau must be > 0");
    ktm::StateIn S;
    for (int k = 0; k < 9; ++k) S.in[k] = in[k];
    S.e = e_in;
    for (int m = 0; m < 4; ++m) S.u[m] = u_in ? u_in[m] : nullptr;
    hipError_t e = c->prm.coords == KT_CARTESIAN
        ? launch(ktm::features_kernel<true>, linear_grid(n), dim3(256), c->stream, c->P, c->E, tau, (long long)n, S, x, y)
        : launch(ktm::features_kernel<false>, linear_grid(n), dim3(256), c->stream, c->P, c->E, tau, (long long)n, S, x, y);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "features kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

kt_status kt_mlp_fwd(kt_ctx *c, int64_t n, const float *x, float *y, float *act)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (n < 0) return fail(c, KT_E_ARG, "n must be >= 0");
    if (!c->mlp_ready) return fail(c, KT_E_STATE, "no parameters set");
    if (n == 0) return KT_OK;
    if (!x || !y) return fail(c, KT_E_ARG, "null input or output");
    hipError_t e = launch(ktm::forward_kernel, linear_grid(n), dim3(256), c->stream, (long long)n,
                          (const float *)c->mlp_w, x, y, act);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "forward kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

kt_status kt_mlp_y0(kt_ctx *c, int64_t n, const float *x, float *y0)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (n < 0) return fail(c, KT_E_ARG, "n must be >= 0");
    if (!c->mlp_ready) return fail(c, KT_E_STATE, "no parameters set");
    if (n == 0) return KT_OK;
    if (!x || !y0) return fail(c, KT_E_ARG, "null input or output");
    hipError_t e = ensure_packed(c);
    if (e == hipSuccess)
        e = launch(mlp_y0_kernel, linear_grid(n), dim3(256), c->stream, (long long)n, x, y0,
                   (const ktm::MlpPacked *)c->mlp_pk);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "start inference: %s", hipGetErrorString(e));
    return KT_OK;
}

kt_status kt_mlp_loss(kt_ctx *c, int64_t n, const float *y, const float *t, const float *w,
                      float *dy, double *loss)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (n < 1) return fail(c, KT_E_ARG, "n must be >= 1");
    if (!y || !t) return fail(c, KT_E_ARG, "null outputs or targets");
    ktm::LossW W;
    for (int o = 0; o < ktm::NO; ++o) {
        W.w[o] = w ? (double)w[o] : 1.0;
        if (!(W.w[o] >= 0.0)) return fail(c, KT_E_ARG, "loss weights must be >= 0");
    }
    long long nb = (4 * n + 255) / 256;
    nb = nb < ktm::LOSS_BLOCKS ? nb : ktm::LOSS_BLOCKS;
    hipError_t e = launch(ktm::loss_kernel, dim3((unsigned)nb), dim3(256), c->stream, (long long)n, y, t,
                          W, dy, c->loss_part);
    if (e == hipSuccess && loss)
        e = launch(ktm::loss_final_kernel, dim3(1), dim3(64), c->stream, (const double *)c->loss_part,
                   (int)nb, (long long)n, loss);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "loss kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

kt_status kt_mlp_bwd(kt_ctx *c, int64_t n, const float *x, const float *act, const float *dy,
                     float *grad)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (n < 1) return fail(c, KT_E_ARG, "n must be >= 1");
    if (!c->mlp_ready) return fail(c, KT_E_STATE, "no parameters set");
    if (!x || !act || !dy || !grad) return fail(c, KT_E_ARG, "null argument");
    long long nb = (n + ktm::BCH - 1) / ktm::BCH;
    nb = nb < ktm::BWD_BLOCKS ? nb : ktm::BWD_BLOCKS;
    hipError_t e = launch(ktm::backward_kernel, dim3((unsigned)nb), dim3(256), c->stream, (long long)n,
                          (const float *)c->mlp_w, x, act, dy, c->mlp_part);
    if (e == hipSuccess)
        e = launch(ktm::grad_reduce_kernel, dim3((ktm::NP + 255) / 256), dim3(256), c->stream,
                   (const float *)c->mlp_part, (int)nb, grad);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "backward kernel: %s", hipGetErrorString(e));
    return KT_OK;
}

kt_status kt_mlp_adam(kt_ctx *c, const float *grad, float lr, float b1, float b2, float eps, int32_t t)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (!c->mlp_ready) return fail(c, KT_E_STATE, "no parameters set");
    if (!grad || t < 1 || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return fail(c, KT_E_ARG, "invalid Adam arguments");
    const float c1 = (float)(1.0 - pow((double)b1, (double)t));
    const float c2 = (float)(1.0 - pow((double)b2, (double)t));
    hipError_t e = launch(ktm::adam_kernel, dim3((ktm::NP + 255) / 256), dim3(256), c->stream, c->mlp_w,
                          c->mlp_m, c->mlp_v, grad, lr, b1, b2, eps, c1, c2);
    if (e != hipSuccess) return fail(c, KT_E_HIP, "adam kernel: %s", hipGetErrorString(e));
    c->mlp_pk_dirty = true;
    return KT_OK;
}

kt_status kt_profile_enable(kt_ctx *c, int32_t mask)
{
    if (!c) return fail(nullptr, KT_E_ARG, "null context");
    if (mask < 0 || mask > 15) return fail(c, KT_E_ARG, "profile class mask %d not in 0..15", mask);
    c->prof = mask;
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

// ------------------------------------------------- static workspace ----
// The workspace of kt_init_static: one array per GPU, set up with the code
// object and held until the process ends.  In host code `scratch` names a
// host-side stand-in, never the device memory: its device address is taken
// once per device with hipGetSymbolAddress (with that device current) and
// only that address is handed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[KT_STATIC_WS_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_dev[256];      // device address of scratch per device ordinal

static hipError_t scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

extern "C" kt_status kt_init_static(const kt_params *p, const kt_eos *eos, const kt_init_state *s0,
                                    hipStream_t stream, kt_ctx **out)
{
    if (!out) return fail(nullptr, KT_E_ARG, "out is null");
    *out = nullptr;
    if (const char *m = check_args(p, eos)) return fail(nullptr, KT_E_ARG, "%s", m);
    const size_t need = layout(p, eos).total;
    if (need > (size_t)KT_STATIC_WS_BYTES)
        return fail(nullptr, KT_E_ALLOC, "grid needs a %zu-byte workspace; the static workspace holds %zu",
                    need, (size_t)KT_STATIC_WS_BYTES);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= 256)) e = hipErrorInvalidDevice;
    void *ws = nullptr;
    if (e == hipSuccess) e = scratch_address(dev, &ws);
    if (e != hipSuccess) return fail(nullptr, KT_E_HIP, "static workspace: %s", hipGetErrorString(e));
    return kt_init(p, eos, s0, ws, (size_t)KT_STATIC_WS_BYTES, stream, out);
}

// ======================================================================
// Batches of events
// ======================================================================

struct kt_batch {
    int n;
    std::vector<kt_ctx *> ev;
    hipStream_t user;            // the caller's stream
    hipStream_t cap;             // stream the step graph is captured on and replayed on
    hipEvent_t fork_ev, join_ev;
    bool mixed, cart;
    bool reduced;                // reduced states (kt_params.reduced)
    bool theta1;                 // every event limits with theta = 1
    double dtau;
    double *tau_dev;
    char *tab;                   // device tables (see batch_tables)
    size_t tab_bytes;
    int kcc;                     // eta planes per flux block (2 or 4, every event)
    std::vector<int> tw;         // waves per flux block along x, per event
    unsigned nb_src, nb_flux, nb_rec, nb_face;
    size_t o_s1[2], o_s2[2], o_r1[2], o_r2[2], o_f1, o_f2;  // table offsets ([step parity])
    size_t o_fsrc, o_fflux, o_frec, o_fface;                // first-block arrays
    size_t o_msrc, o_mflux, o_mrec, o_mface;                // block -> event maps
    hipGraph_t graph[3];         // one captured step per step parity; [2]: two steps from an even one
    hipGraphExec_t exec[3];
    bool have_graph;
    double tau;
    long long step;
    char err[512];
};

static kt_status bfail(kt_batch *b, kt_status s, const char *fmt, ...)
{
    char *dst = b ? b->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return s;
}

// bytes of the device tables of n events (the larger, FP64 layout), not
// counting the block -> event maps (2 bytes per block, event_blocks)
static size_t batch_table_bytes(int n)
{
    size_t t = 0;
    t += 4 * round_up(sizeof(BStage<double>) * n, 256);
    t += 4 * round_up(sizeof(BRec<double>) * n, 256);
    t += 2 * round_up(sizeof(BFace<double>) * n, 256);
    t += 4 * round_up(sizeof(unsigned) * (n + 1), 256);
    return t;
}

// blocks of every launch kind of one event (flux at one eta plane per block and
// the block shape with the most tiles, the most)
static size_t event_blocks(const kt_params *p)
{
    const size_t sg = (size_t)((p->nx + 63) / 64) * ((p->ny + 3) / 4);
    size_t fg = 0;
    for (int tw = 1; tw <= 4; tw *= 2)
        fg = std::max(fg, (size_t)((p->nx + 16 * tw - 1) / (16 * tw)) * ((p->ny + 16 / tw - 1) / (16 / tw)));
    const size_t ncell = (size_t)p->nx * p->ny * p->neta;
    return (sg + fg) * p->neta + (ncell + 255) / 256 + (size_t)face_launch(face_geo(p), p->nx, p->ny).nblocks;
}

static size_t event_ws(const kt_params *p, const kt_eos *eos)
{
    return round_up(layout(p, eos).total, 256);
}

// the batch's table region: argument tables plus the block -> event maps of nb blocks
static size_t batch_tab_region(int n, size_t nb)
{
    return round_up(batch_table_bytes(n), 256) + round_up(nb * sizeof(unsigned short), 256) + 4 * 256;
}

// Build the per-event argument tables of a step and upload them (the
// caller's stream, synchronised).  Buffers of every event: q (index 0) and
// q* (1); u[2] = u*; at even steps u[0] = u^n and u[1] = u^{n-1}, at odd
// steps the reverse: u^{n+1} is written over u^{n-1}, so the two buffers swap
// roles every step and a table set (and a captured graph) exists for each
// step parity; no u is copied.
template <typename S>
static kt_status batch_tables(kt_batch *b)
{
    const int n = b->n;
    std::vector<BStage<S>> s1[2], s2[2];
    std::vector<BRec<S>> r1[2], r2[2];
    std::vector<BFace<S>> f1(n), f2(n);
    for (int par = 0; par < 2; ++par) {
        s1[par].resize(n);
        s2[par].resize(n);
        r1[par].resize(n);
        r2[par].resize(n);
    }
    std::vector<unsigned> fs(n + 1), ff(n + 1), fr(n + 1), fc(n + 1);
    fs[0] = ff[0] = fr[0] = fc[0] = 0;
    for (int e = 0; e < n; ++e) {
        kt_ctx *c = b->ev[e];
        const Phys &P = c->P;
        auto uu = [&](int k) { return (double *)c->u[k]; };
        for (int par = 0; par < 2; ++par) {
            // u buffers at this step parity: u^n in cur, u^{n-1} in prev, u* in 2;
            // u^{n+1} goes to prev, which makes the roles swap for the next step
            const int cur = par, prev = 1 - par;
            for (int st = 0; st < 2; ++st) {
                BStage<S> &A = st == 0 ? s1[par][e] : s2[par][e];
                const int src = st;
                A.P = P;
                A.E = c->E;
                A.G = c->G;
                A.F = Fields<S>{c->qT[src], (const S *)c->qP[src], (const S *)c->e, (const S *)c->p,
                                (const double *)uu(st == 0 ? cur : 2), (const double *)uu(st == 0 ? prev : cur),
                                (const S *)c->vf};
                A.qnT = st == 1 ? c->qT[0] : nullptr;
                A.qnP = st == 1 ? (const S *)c->qP[0] : nullptr;
                A.outT = c->qT[1 - src];
                A.outP = (S *)c->qP[1 - src];
                A.sgx = (P.nx + 63) / 64;
                A.sgy = (P.ny + 3) / 4;
                A.tw = b->tw[e];
                A.fgx = (P.nx + 16 * A.tw - 1) / (16 * A.tw);
                A.fgy = (P.ny + 16 / A.tw - 1) / (16 / A.tw);
                BRec<S> &R = st == 0 ? r1[par][e] : r2[par][e];
                const int which = st == 0 ? 1 : 0;   // recover q* after stage 1, q after stage 2
                R.P = P;
                R.E = c->E;
                R.qT = c->qT[which];
                R.qP = (S *)c->qP[which];
                R.e = (S *)c->e;
                R.p = (S *)c->p;
                R.u = uu(st == 0 ? 2 : prev);
                R.us = uu(st == 0 ? cur : 2);
                R.slots = c->slots;
            }
        }
        for (int st = 0; st < 2; ++st) {
            const int which = st == 0 ? 1 : 0;   // faces of q* after stage 1, of q after stage 2
            BFace<S> &F = st == 0 ? f1[e] : f2[e];
            F.P = P;
            F.E = c->E;
            F.G = c->G;
            F.L = face_launch(c->G, P.nx, P.ny);
            F.qT = c->qT[which];
            F.qP = (const S *)c->qP[which];
            F.vf = (S *)c->vf;
            F.slots = c->slots;
        }
        const unsigned sg = s1[0][e].sgx * s1[0][e].sgy;
        fs[e + 1] = fs[e] + sg * (unsigned)P.neta;
        ff[e + 1] = ff[e] + s1[0][e].fgx * s1[0][e].fgy * (unsigned)((P.neta + b->kcc - 1) / b->kcc);
        fr[e + 1] = fr[e] + (unsigned)((P.ncell + 255) / 256);
        fc[e + 1] = fc[e] + f1[e].L.nblocks;
    }
    b->nb_src = fs[n];
    b->nb_flux = ff[n];
    b->nb_rec = fr[n];
    b->nb_face = fc[n];
    auto mk = [&](const std::vector<unsigned> &f) {
        std::vector<unsigned short> m(f[n]);
        for (int e = 0; e < n; ++e)
            for (unsigned g = f[e]; g < f[e + 1]; ++g) m[g] = (unsigned short)e;
        return m;
    };
    const std::vector<unsigned short> ms = mk(fs), mf = mk(ff), mr = mk(fr), mc = mk(fc);
    size_t off = 0;
    auto place = [&](size_t bytes) { const size_t o = off; off += round_up(bytes, 256); return o; };
    for (int par = 0; par < 2; ++par) {
        b->o_s1[par] = place(sizeof(BStage<S>) * n);
        b->o_s2[par] = place(sizeof(BStage<S>) * n);
        b->o_r1[par] = place(sizeof(BRec<S>) * n);
        b->o_r2[par] = place(sizeof(BRec<S>) * n);
    }
    b->o_f1 = place(sizeof(BFace<S>) * n);
    b->o_f2 = place(sizeof(BFace<S>) * n);
    b->o_fsrc = place(sizeof(unsigned) * (n + 1));
    b->o_fflux = place(sizeof(unsigned) * (n + 1));
    b->o_frec = place(sizeof(unsigned) * (n + 1));
    b->o_fface = place(sizeof(unsigned) * (n + 1));
    b->o_msrc = place(sizeof(unsigned short) * ms.size());
    b->o_mflux = place(sizeof(unsigned short) * mf.size());
    b->o_mrec = place(sizeof(unsigned short) * mr.size());
    b->o_mface = place(sizeof(unsigned short) * mc.size());
    if (off > b->tab_bytes) return bfail(b, KT_E_ALLOC, "batch tables need %zu bytes", off);
    std::vector<char> h(off, 0);
    auto put = [&](size_t o, const void *src, size_t bytes) { memcpy(h.data() + o, src, bytes); };
    for (int par = 0; par < 2; ++par) {
        put(b->o_s1[par], s1[par].data(), sizeof(BStage<S>) * n);
        put(b->o_s2[par], s2[par].data(), sizeof(BStage<S>) * n);
        put(b->o_r1[par], r1[par].data(), sizeof(BRec<S>) * n);
        put(b->o_r2[par], r2[par].data(), sizeof(BRec<S>) * n);
    }
    put(b->o_f1, f1.data(), sizeof(BFace<S>) * n);
    put(b->o_f2, f2.data(), sizeof(BFace<S>) * n);
    put(b->o_fsrc, fs.data(), sizeof(unsigned) * (n + 1));
    put(b->o_fflux, ff.data(), sizeof(unsigned) * (n + 1));
    put(b->o_frec, fr.data(), sizeof(unsigned) * (n + 1));
    put(b->o_fface, fc.data(), sizeof(unsigned) * (n + 1));
    put(b->o_msrc, ms.data(), sizeof(unsigned short) * ms.size());
    put(b->o_mflux, mf.data(), sizeof(unsigned short) * mf.size());
    put(b->o_mrec, mr.data(), sizeof(unsigned short) * mr.size());
    put(b->o_mface, mc.data(), sizeof(unsigned short) * mc.size());
    hipError_t e = hipMemcpyAsync(b->tab, h.data(), off, hipMemcpyHostToDevice, b->user);
    if (e == hipSuccess) e = hipStreamSynchronize(b->user);
    if (e != hipSuccess) return bfail(b, KT_E_HIP, "batch tables: %s", hipGetErrorString(e));
    return KT_OK;
}

// enqueue one Heun step of every event on stream st (captured into the graph
// of step parity par)
template <bool CART, bool T1, typename S>
static hipError_t batch_step_launches(kt_batch *b, hipStream_t st, int par)
{
    const int n = b->n;
    auto T = [&](size_t o) { return (const void *)(b->tab + o); };
    auto F = [&](size_t o) { return (const unsigned *)(b->tab + o); };
    const double *tau = b->tau_dev;
    const dim3 blk2(64, 4), blk(256);
    auto M = [&](size_t o) { return (const unsigned short *)(b->tab + o); };
    hipError_t e = launch(sources_batch<CART, false, S>, dim3(b->nb_src), blk2, st,
                          (const BStage<S> *)T(b->o_s1[par]), M(b->o_msrc), F(b->o_fsrc), tau);
    auto flux = [&](auto kern, size_t o) {
        return launch(kern, dim3(b->nb_flux), blk2, st, (const BStage<S> *)T(o), M(b->o_mflux), F(b->o_fflux));
    };
    if (e == hipSuccess)
        e = b->kcc == 4 ? flux(flux_batch<false, T1, S, 4>, b->o_s1[par]) : flux(flux_batch<false, T1, S, 2>, b->o_s1[par]);
    auto recover = [&](size_t o) {
        return b->reduced ? launch(recover_batch<CART, S, true>, dim3(b->nb_rec), blk, st, (const BRec<S> *)T(o),
                                   M(b->o_mrec), F(b->o_frec), tau)
                          : launch(recover_batch<CART, S, false>, dim3(b->nb_rec), blk, st, (const BRec<S> *)T(o),
                                   M(b->o_mrec), F(b->o_frec), tau);
    };
    if (e == hipSuccess) e = recover(b->o_r1[par]);
    if (e == hipSuccess)
        e = launch(faces_batch<CART, T1, S>, dim3(b->nb_face), dim3(FACE_BLOCK), st, (const BFace<S> *)T(b->o_f1),
                   M(b->o_mface), F(b->o_fface), tau);
    if (e == hipSuccess)
        e = launch(sources_batch<CART, true, S>, dim3(b->nb_src), blk2, st,
                   (const BStage<S> *)T(b->o_s2[par]), M(b->o_msrc), F(b->o_fsrc), tau);
    if (e == hipSuccess)
        e = b->kcc == 4 ? flux(flux_batch<true, T1, S, 4>, b->o_s2[par]) : flux(flux_batch<true, T1, S, 2>, b->o_s2[par]);
    if (e == hipSuccess) e = recover(b->o_r2[par]);
    if (e == hipSuccess)
        e = launch(faces_batch<CART, T1, S>, dim3(b->nb_face), dim3(FACE_BLOCK), st, (const BFace<S> *)T(b->o_f2),
                   M(b->o_mface), F(b->o_fface), tau);
    if (e == hipSuccess) e = launch(tau_advance_kernel, dim3(1), dim3(64), st, b->tau_dev, b->dtau);
    return e;
}

// stage 1 of the batch without its recovery: the sources and flux launches
// (timed by kt_batch_tune; they only write q*, which every step rewrites)
template <bool CART, bool T1, typename S>
static hipError_t batch_stage1_t(kt_batch *b, hipStream_t st)
{
    const BStage<S> *tab = (const BStage<S> *)(const void *)(b->tab + b->o_s1[b->step & 1]);
    hipError_t e = launch(sources_batch<CART, false, S>, dim3(b->nb_src), dim3(64, 4), st, tab,
                          (const unsigned short *)(b->tab + b->o_msrc), (const unsigned *)(b->tab + b->o_fsrc),
                          (const double *)b->tau_dev);
    const unsigned short *map = (const unsigned short *)(b->tab + b->o_mflux);
    const unsigned *first = (const unsigned *)(b->tab + b->o_fflux);
    if (e == hipSuccess)
        e = b->kcc == 4 ? launch(flux_batch<false, T1, S, 4>, dim3(b->nb_flux), dim3(64, 4), st, tab, map, first)
                        : launch(flux_batch<false, T1, S, 2>, dim3(b->nb_flux), dim3(64, 4), st, tab, map, first);
    return e;
}

template <bool T1>
static hipError_t batch_stage1_t1(kt_batch *b, hipStream_t st)
{
    if (b->mixed)
        return b->cart ? batch_stage1_t<true, T1, float>(b, st) : batch_stage1_t<false, T1, float>(b, st);
    return b->cart ? batch_stage1_t<true, T1, double>(b, st) : batch_stage1_t<false, T1, double>(b, st);
}

static hipError_t batch_stage1(kt_batch *b, hipStream_t st)
{
    return b->theta1 ? batch_stage1_t1<true>(b, st) : batch_stage1_t1<false>(b, st);
}

template <bool T1>
static hipError_t batch_launches_t1(kt_batch *b, hipStream_t st, int par)
{
    if (b->mixed)
        return b->cart ? batch_step_launches<true, T1, float>(b, st, par)
                       : batch_step_launches<false, T1, float>(b, st, par);
    return b->cart ? batch_step_launches<true, T1, double>(b, st, par)
                   : batch_step_launches<false, T1, double>(b, st, par);
}

// theta1: every event limits with theta = 1 (the kernels' exact shortcut)
static hipError_t batch_launches(kt_batch *b, hipStream_t st, int par)
{
    return b->theta1 ? batch_launches_t1<true>(b, st, par) : batch_launches_t1<false>(b, st, par);
}

static void batch_drop_graph(kt_batch *b)
{
    if (b->have_graph) {
        for (int par = 0; par < 3; ++par) {
            (void)hipGraphExecDestroy(b->exec[par]);
            (void)hipGraphDestroy(b->graph[par]);
        }
        b->have_graph = false;
    }
}

static kt_status batch_build_tables(kt_batch *b)
{
    batch_drop_graph(b);
    return b->mixed ? batch_tables<float>(b) : batch_tables<double>(b);
}

extern "C" {

size_t kt_batch_workspace_bytes(const kt_params *p, int32_t n_events, const kt_eos *eos)
{
    if (!p || n_events < 1 || !eos) return 0;
    if (n_events > 65535) return 0;
    size_t t = 0, nb = 0;
    for (int e = 0; e < n_events; ++e) {
        if (check_args(&p[e], eos)) return 0;
        t += event_ws(&p[e], eos);
        nb += event_blocks(&p[e]);
    }
    return t + 256 + batch_tab_region(n_events, nb);
}

void kt_batch_destroy(kt_batch *b)
{
    if (!b) return;
    batch_drop_graph(b);
    if (b->cap) {
        (void)hipStreamSynchronize(b->cap);
        (void)hipStreamDestroy(b->cap);
    }
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    if (b->join_ev) (void)hipEventDestroy(b->join_ev);
    for (kt_ctx *c : b->ev) kt_destroy(c);
    delete b;
}

kt_status kt_batch_init(const kt_params *p, int32_t n_events, const kt_eos *eos,
                        const kt_init_state *s0, void *d_ws, size_t ws_bytes, hipStream_t stream,
                        kt_batch **out)
{
    if (!out) return bfail(nullptr, KT_E_ARG, "out is null");
    *out = nullptr;
    if (!p || !eos || !s0 || !d_ws) return bfail(nullptr, KT_E_ARG, "null argument");
    if (n_events < 1 || n_events > 65535) return bfail(nullptr, KT_E_ARG, "n_events must lie in [1, 65535]");
    if (((uintptr_t)d_ws) % 256) return bfail(nullptr, KT_E_ARG, "workspace must be 256-byte aligned");
    for (int e = 0; e < n_events; ++e) {
        if (const char *m = check_args(&p[e], eos)) return bfail(nullptr, KT_E_ARG, "event %d: %s", e, m);
        if (p[e].coords != p[0].coords || p[e].precision != p[0].precision || p[e].dtau != p[0].dtau ||
            p[e].tau0 != p[0].tau0 || p[e].reduced != p[0].reduced)
            return bfail(nullptr, KT_E_ARG,
                         "event %d: coords, precision, reduced, tau0 and dtau must match event 0", e);
    }
    const size_t need = kt_batch_workspace_bytes(p, n_events, eos);
    if (ws_bytes < need) return bfail(nullptr, KT_E_ALLOC, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    kt_batch *b = new (std::nothrow) kt_batch();
    if (!b) return bfail(nullptr, KT_E_ALLOC, "host allocation failed");
    b->n = n_events;
    b->user = stream;
    b->mixed = p[0].precision == KT_MIXED;
    b->cart = p[0].coords == KT_CARTESIAN;
    b->reduced = p[0].reduced != 0;
    b->theta1 = true;
    for (int k = 0; k < n_events; ++k) b->theta1 = b->theta1 && theta_is_one(p[k].theta);
    b->dtau = p[0].dtau;
    b->tau = p[0].tau0;
    b->kcc = KC;
    b->tw.assign(n_events, 4);
    char *base = (char *)d_ws;
    size_t off = 0;
    for (int e = 0; e < n_events; ++e) {
        kt_ctx *c = nullptr;
        const size_t w = event_ws(&p[e], eos);
        kt_status st = kt_init(&p[e], eos, &s0[e], base + off, w, stream, &c);
        if (st != KT_OK) {
            kt_status r = bfail(nullptr, st, "event %d: %s", e, kt_last_error(nullptr));
            kt_batch_destroy(b);
            return r;
        }
        b->ev.push_back(c);
        off += w;
    }
    b->tau_dev = (double *)(base + off);
    off += 256;
    b->tab = base + off;
    {
        size_t nb = 0;
        for (int e = 0; e < n_events; ++e) nb += event_blocks(&p[e]);
        b->tab_bytes = batch_tab_region(n_events, nb);
    }
    hipError_t he = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&b->join_ev, hipEventDisableTiming);
    if (he == hipSuccess) he = hipMemcpyAsync(b->tau_dev, &b->tau, sizeof(double), hipMemcpyHostToDevice, stream);
    if (he != hipSuccess) {
        kt_status r = bfail(nullptr, KT_E_HIP, "batch init: %s", hipGetErrorString(he));
        kt_batch_destroy(b);
        return r;
    }
    kt_status st = batch_build_tables(b);
    if (st != KT_OK) {
        kt_status r = bfail(nullptr, st, "%s", b->err);
        kt_batch_destroy(b);
        return r;
    }
    *out = b;
    return KT_OK;
}

kt_status kt_batch_step(kt_batch *b, int32_t n_steps)
{
    if (!b) return bfail(nullptr, KT_E_ARG, "null batch");
    if (n_steps < 0) return bfail(b, KT_E_ARG, "n_steps must be >= 0");
    if (n_steps == 0) return KT_OK;
    hipError_t e = hipSuccess;
    if (!b->have_graph) {
        // the u buffers swap roles every step, so there is one graph per step
        // parity, and a third of two steps (even, then odd) that halves the
        // graph launches of longer runs
        int made = 0;
        for (int par = 0; par < 3 && e == hipSuccess; ++par) {
            e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t le = batch_launches(b, b->cap, par & 1);
                if (par == 2 && le == hipSuccess) le = batch_launches(b, b->cap, 1);
                e = hipStreamEndCapture(b->cap, &b->graph[par]);
                if (le != hipSuccess && e == hipSuccess) {
                    (void)hipGraphDestroy(b->graph[par]);
                    e = le;
                } else if (e == hipSuccess) {
                    e = hipGraphInstantiate(&b->exec[par], b->graph[par], nullptr, nullptr, 0);
                    if (e == hipSuccess) made += 1;
                    else (void)hipGraphDestroy(b->graph[par]);
                }
            }
        }
        if (e != hipSuccess) {
            for (int par = 0; par < made; ++par) {
                (void)hipGraphExecDestroy(b->exec[par]);
                (void)hipGraphDestroy(b->graph[par]);
            }
            return bfail(b, KT_E_HIP, "step graph: %s", hipGetErrorString(e));
        }
        b->have_graph = true;
    }
    e = hipEventRecord(b->fork_ev, b->user);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->fork_ev, 0);
    for (int s = 0; s < n_steps && e == hipSuccess;) {
        const int par = (int)((b->step + s) & 1);
        const bool two = par == 0 && n_steps - s >= 2;
        e = hipGraphLaunch(b->exec[two ? 2 : par], b->cap);
        s += two ? 2 : 1;
    }
    if (e == hipSuccess) e = hipEventRecord(b->join_ev, b->cap);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->user, b->join_ev, 0);
    if (e != hipSuccess) return bfail(b, KT_E_HIP, "batch step: %s", hipGetErrorString(e));
    for (int s = 0; s < n_steps; ++s) {
        b->tau = b->tau + b->dtau;
        b->step += 1;
    }
    for (kt_ctx *c : b->ev) {
        c->tau = b->tau;
        c->step = b->step;
        c->ucur = (int)(b->step & 1);   // u^n, u^{n-1} for kt_observables
        c->uprev = 1 - c->ucur;
    }
    return KT_OK;
}

kt_status kt_batch_set_flux_blocks(kt_batch *b, const int32_t *kc, const int32_t *tile_x)
{
    if (!b) return bfail(nullptr, KT_E_ARG, "null batch");
    if (!kc || !tile_x) return bfail(b, KT_E_ARG, "null kc or tile_x");
    for (int ev = 0; ev < b->n; ++ev) {
        if ((kc[ev] != 2 && kc[ev] != 4) || kc[ev] != kc[0])
            return bfail(b, KT_E_ARG, "kc[%d] = %d: every event takes the same, 2 or 4", ev, kc[ev]);
        if (tile_x[ev] != 64 && tile_x[ev] != 32 && tile_x[ev] != 16)
            return bfail(b, KT_E_ARG, "tile_x[%d] = %d is not 64, 32 or 16", ev, tile_x[ev]);
    }
    b->kcc = kc[0];
    for (int ev = 0; ev < b->n; ++ev) b->tw[ev] = tile_x[ev] / 16;
    return batch_build_tables(b);
}

kt_status kt_batch_tune(kt_batch *b, int32_t *kc_out, int32_t *tile_out)
{
    if (!b) return bfail(nullptr, KT_E_ARG, "null batch");
    static const int cand_tw[3] = {4, 2, 1};
    hipEvent_t t0, t1;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) return bfail(b, KT_E_HIP, "tune events: %s", hipGetErrorString(e));
    // The batched stage 1 (sources, then flux: the flux kernel finds the caches as
    // it does in a step) is timed as a whole: the launch shares the chip among all
    // events, so timing each grid shape alone would choose for a different load.
    // The flux block's width (waves along x) is chosen per distinct grid shape, one
    // shape at a time (largest total cells first) with the others held at their
    // current choice; then the eta planes per block (2 or 4, one value for the
    // launch) with those widths.  Both launches only write q*, which the next
    // step's sources kernel overwrites, so timing them on the live state changes
    // no result.
    kt_status st = KT_OK;
    auto time_stage1 = [&](float &tot) {
        st = batch_build_tables(b);
        tot = 0.0f;
        for (int r = 0; r < 4 && e == hipSuccess && st == KT_OK; ++r) {
            e = hipEventRecord(t0, b->user);
            if (e == hipSuccess) e = batch_stage1(b, b->user);
            if (e == hipSuccess) e = hipEventRecord(t1, b->user);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (r > 0) tot += ms;   // the first launch warms caches
        }
    };
    // distinct shapes, largest total cells first
    std::vector<std::vector<int>> shapes;
    std::vector<long long> shape_cells;
    for (int ev = 0; ev < b->n; ++ev) {
        const Phys &P = b->ev[ev]->P;
        int found = -1;
        for (size_t s2 = 0; s2 < shapes.size(); ++s2) {
            const Phys &Q = b->ev[shapes[s2][0]]->P;
            if (Q.nx == P.nx && Q.ny == P.ny && Q.neta == P.neta) found = (int)s2;
        }
        if (found < 0) {
            shapes.push_back({ev});
            shape_cells.push_back(0);
            found = (int)shapes.size() - 1;
        } else {
            shapes[found].push_back(ev);
        }
        shape_cells[found] += (long long)P.nx * P.ny * P.neta;
    }
    std::vector<size_t> order(shapes.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t c2) { return shape_cells[a] > shape_cells[c2]; });
    b->kcc = KC;
    float best = 1e30f;
    for (size_t oi = 0; oi < order.size() && e == hipSuccess && st == KT_OK; ++oi) {
        const std::vector<int> &evs = shapes[order[oi]];
        float best_s = 1e30f;
        int best_tw = b->tw[evs[0]];
        for (int ti = 0; ti < 3 && e == hipSuccess && st == KT_OK; ++ti) {
            for (int ev : evs) b->tw[ev] = cand_tw[ti];
            float tot = 0.0f;
            time_stage1(tot);
            if (e == hipSuccess && st == KT_OK && tot < best_s) {
                best_s = tot;
                best_tw = cand_tw[ti];
            }
        }
        for (int ev : evs) b->tw[ev] = best_tw;
        best = best_s;
    }
    if (e == hipSuccess && st == KT_OK) {
        b->kcc = 4;
        float tot = 0.0f;
        time_stage1(tot);
        if (e == hipSuccess && st == KT_OK && !(tot < best)) b->kcc = 2;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (st != KT_OK) return st;
    if (e != hipSuccess) return bfail(b, KT_E_HIP, "tune: %s", hipGetErrorString(e));
    for (int ev = 0; ev < b->n; ++ev) {
        if (kc_out) kc_out[ev] = b->kcc;
        if (tile_out) tile_out[ev] = 16 * b->tw[ev];
    }
    return batch_build_tables(b);
}

kt_status kt_batch_observables(kt_batch *b, int32_t event, kt_obs *host_out, const kt_fields *dev_out)
{
    if (!b) return bfail(nullptr, KT_E_ARG, "null batch");
    if (event < 0 || event >= b->n) return bfail(b, KT_E_ARG, "event %d out of range", event);
    kt_status st = kt_observables(b->ev[event], host_out, dev_out);
    if (st != KT_OK) return bfail(b, st, "%s", b->ev[event]->err);
    return KT_OK;
}

const char *kt_batch_last_error(const kt_batch *b) { return b ? b->err : g_err; }

}  // extern "C"
