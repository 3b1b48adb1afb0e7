// kt_mlp.hpp -- learned starting value of the cell inversion (gfx950, FP32).
//
// The inversion of Sec. 2.4 / Sec. 3.2 (Newton on f(e) = e - E + M^2/(E + P))
// needs a starting e.  A small network 11 -> 64 -> 64 -> 4 with GELU
// (a Phi(a), exact, through erff) maps features of (T^{tau mu}, pi^{tau mu},
// Pi) to (e/e_c, v^x, v^y, sqrt(g33) v^eta), where e_c = sqrt(4E^2 - 3M^2) - E
// is the root for the conformal EOS without bulk (E = T^{tau tau} -
// pi^{tau tau}, M^i = T^{tau i} - pi^{tau i}); e_0 = y_0 e_c, then Newton
// polishes to the usual tolerance (bisection remains the fallback).
// Features, per state with T0 = T^{tau tau}:
//   T^{tau x}/T0, T^{tau y}/T0, sqrt(g33) T^{tau eta}/T0, pi^{tau tau}/T0,
//   pi^{tau x}/T0, pi^{tau y}/T0, sqrt(g33) pi^{tau eta}/T0, Pi/T0,
//   0.1 ln T0, c_s^2(T0), p(T0)/T0.
// Parameters: one flat FP32 vector W1 (64x11), b1, W2 (64x64), b2, W3 (4x64),
// b3, weights row major, a layer computing a = W h + b.
// Batched arrays are feature-major: x[f*n + i], y[o*n + i], act[k*n + i]
// (k < 64: first-layer pre-activations, k >= 64: second layer).
// Training: mean over samples and outputs of w_o (y_o - t_o)^2, gradients
// reduced per block then summed in a fixed order (deterministic), Adam
// (Kingma & Ba, arXiv:1412.6980).
#pragma once

#include "kt_device.hpp"

namespace ktm {

using namespace ktd;

constexpr int NI = 11, NH = 64, NO = 4;
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH;
constexpr int OW3 = OB2 + NH, OB3 = OW3 + NO * NH, NP = OB3 + NO;   // NP = 5188
constexpr int BWD_BLOCKS = 256;   // blocks (and gradient partials) of the backward pass
constexpr int BCH = 32;           // samples staged per chunk in the backward pass
constexpr int LOSS_BLOCKS = 256;

__device__ __forceinline__ float gelu(float a)
{
    return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f));
}

// d/da [a Phi(a)] = Phi(a) + a phi(a)
__device__ __forceinline__ float gelu_grad(float a)
{
    return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * 0.39894228040143268f * expf(-0.5f * a * a);
}

template <bool CART>
__device__ __forceinline__ void features(const Eos &E, double tau, double Ttt, double Ttx, double Tty,
                                         double Tte, double ptt, double ptx, double pty, double pte,
                                         double Pi, float x[NI])
{
    const double sg = CART ? 1.0 : tau;
    const double inv = 1.0 / Ttt;
    x[0] = (float)(Ttx * inv);
    x[1] = (float)(Tty * inv);
    x[2] = (float)(sg * Tte * inv);
    x[3] = (float)(ptt * inv);
    x[4] = (float)(ptx * inv);
    x[5] = (float)(pty * inv);
    x[6] = (float)(sg * pte * inv);
    x[7] = (float)(Pi * inv);
    x[8] = (float)(log(Ttt) * 0.1);
    double p, cs2;
    eos_pc(E, Ttt, p, cs2);
    x[9] = (float)cs2;
    x[10] = (float)(p * inv);
}

// e_c = sqrt(4E^2 - 3M^2) - E, at least e_floor
template <bool CART>
__device__ __forceinline__ double conformal_root(double e_floor, double tau, double Ttt, double Ttx,
                                                 double Tty, double Tte, double ptt, double ptx,
                                                 double pty, double pte)
{
    const double g33 = CART ? 1.0 : tau * tau;
    const double EE = Ttt - ptt, Mx = Ttx - ptx, My = Tty - pty, Me = Tte - pte;
    const double M2 = Mx * Mx + My * My + g33 * (Me * Me);
    return fmax(sqrt(fmax(4.0 * EE * EE - 3.0 * M2, 0.0)) - EE, e_floor);
}

// first layer of one sample, h1 = GELU(W1 x + b1); if act is non-null,
// act[o*n + i] receives W1 x + b1
__device__ __forceinline__ void layer1(const float *__restrict__ w, const float x[NI], float h1[NH],
                                       float *act, long long n, long long i)
{
#pragma unroll
    for (int o = 0; o < NH; ++o) {
        float a = w[OB1 + o];
#pragma unroll
        for (int f = 0; f < NI; ++f) a = fmaf(w[OW1 + o * NI + f], x[f], a);
        if (act) act[o * n + i] = a;
        h1[o] = gelu(a);
    }
}

// y_0 only (the start of the inversion); weights are read with uniform addresses
__device__ __forceinline__ float forward_y0(const float *__restrict__ w, const float x[NI])
{
    float h1[NH];
    layer1(w, x, h1, nullptr, 0, 0);
    float y0 = w[OB3];
#pragma unroll 2
    for (int o = 0; o < NH; ++o) {
        float a = w[OB2 + o];
#pragma unroll
        for (int k = 0; k < NH; ++k) a = fmaf(w[OW2 + o * NH + k], h1[k], a);
        y0 = fmaf(w[OW3 + o], gelu(a), y0);
    }
    return y0;
}

// ---------------------------------------------------------------- kernels --

struct StateIn {
    const double *in[9];   // T^{tau mu} (4), pi^{tau mu} (4), Pi (nullable)
    const double *e;       // nullable: recovered e and u for the targets
    const double *u[4];
};

template <bool CART>
__global__ __launch_bounds__(256) void features_kernel(Phys P, Eos E, double tau, long long n,
                                                       StateIn S, float *x, float *y)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double Pi = (P.bulk && S.in[8]) ? S.in[8][i] : 0.0;
    float f[NI];
    features<CART>(E, tau, S.in[0][i], S.in[1][i], S.in[2][i], S.in[3][i], S.in[4][i], S.in[5][i],
                   S.in[6][i], S.in[7][i], Pi, f);
#pragma unroll
    for (int k = 0; k < NI; ++k) x[k * n + i] = f[k];
    if (y) {
        const double sg = CART ? 1.0 : tau;
        const double ut = S.u[0][i];
        const double ec = conformal_root<CART>(P.e_floor, tau, S.in[0][i], S.in[1][i], S.in[2][i],
                                               S.in[3][i], S.in[4][i], S.in[5][i], S.in[6][i],
                                               S.in[7][i]);
        y[i] = (float)(S.e[i] / ec);
        y[n + i] = (float)(S.u[1][i] / ut);
        y[2 * n + i] = (float)(S.u[2][i] / ut);
        y[3 * n + i] = (float)(sg * S.u[3][i] / ut);
    }
}

__global__ __launch_bounds__(256) void forward_kernel(long long n, const float *__restrict__ w,
                                                      const float *__restrict__ x,
                                                      float *__restrict__ y, float *__restrict__ act)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float xi[NI], h1[NH];
#pragma unroll
    for (int f = 0; f < NI; ++f) xi[f] = x[f * n + i];
    layer1(w, xi, h1, act, n, i);
    float yo[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) yo[j] = w[OB3 + j];
#pragma unroll 2
    for (int o = 0; o < NH; ++o) {
        float a = w[OB2 + o];
#pragma unroll
        for (int k = 0; k < NH; ++k) a = fmaf(w[OW2 + o * NH + k], h1[k], a);
        if (act) act[(NH + o) * n + i] = a;
        const float h = gelu(a);
#pragma unroll
        for (int j = 0; j < NO; ++j) yo[j] = fmaf(w[OW3 + j * NH + o], h, yo[j]);
    }
#pragma unroll
    for (int j = 0; j < NO; ++j) y[j * n + i] = yo[j];
}

struct LossW {
    double w[NO];
};

// dy = 2 w_o (y - t) / (4 n); per-block partial sums of w_o (y - t)^2 (double)
__global__ __launch_bounds__(256) void loss_kernel(long long n, const float *y, const float *t, LossW W,
                                                   float *dy, double *partial)
{
    __shared__ double red[4];
    double s = 0.0;
    const double scale = 2.0 / (4.0 * (double)n);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < NO * n;
         i += (long long)gridDim.x * blockDim.x) {
        const double w = W.w[i / n];
        const double d = (double)y[i] - (double)t[i];
        if (dy) dy[i] = (float)(scale * w * d);
        s += w * d * d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void loss_final_kernel(const double *partial, int nb, long long n, double *loss)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    *loss = s / (4.0 * (double)n);
}

// Backward pass of sum_i <dy_i, y_i>: chunks of BCH samples are staged in
// LDS, the per-sample deltas d2 = (W3^T dy) GELU'(a2) and d1 = (W2^T d2)
// GELU'(a1) are formed, and each thread accumulates a fixed set of the 5188
// gradient entries (entry e = threadIdx.x + 256 r) over the chunk's samples.
constexpr int BWD_R = (NP + 255) / 256;   // entries per thread

__global__ __launch_bounds__(256) void backward_kernel(long long n, const float *__restrict__ w,
                                                       const float *__restrict__ x,
                                                       const float *__restrict__ act,
                                                       const float *__restrict__ dy,
                                                       float *__restrict__ partial)
{
    __shared__ float sX[BCH][NI + 1];
    __shared__ float sH1[BCH][NH + 1], sD1[BCH][NH + 1], sH2[BCH][NH + 1], sD2[BCH][NH + 1];
    __shared__ float sDY[BCH][NO];
    __shared__ float sW2[NH * NH], sW3[NO * NH];
    const int tid = threadIdx.x;
    for (int k = tid; k < NH * NH; k += 256) sW2[k] = w[OW2 + k];
    for (int k = tid; k < NO * NH; k += 256) sW3[k] = w[OW3 + k];
    float acc[BWD_R];
#pragma unroll
    for (int r = 0; r < BWD_R; ++r) acc[r] = 0.0f;
    for (long long base = (long long)blockIdx.x * BCH; base < n; base += (long long)gridDim.x * BCH) {
        const int ns = (int)((n - base) < BCH ? (n - base) : BCH);
        __syncthreads();   // previous chunk fully consumed (and weights staged)
#pragma unroll 1
        for (int k = tid; k < BCH * NI; k += 256) {
            const int s = k % BCH, f = k / BCH;
            sX[s][f] = s < ns ? x[f * n + base + s] : 0.0f;
        }
#pragma unroll 1
        for (int k = tid; k < BCH * NH; k += 256) {
            const int s = k % BCH, h = k / BCH;
            sH1[s][h] = s < ns ? act[h * n + base + s] : 0.0f;          // a1 for now
            sH2[s][h] = s < ns ? act[(NH + h) * n + base + s] : 0.0f;   // a2 for now
        }
        if (tid < BCH * NO) {
            const int s = tid % BCH, j = tid / BCH;
            sDY[s][j] = s < ns ? dy[j * n + base + s] : 0.0f;
        }
        __syncthreads();
#pragma unroll 1
        for (int k = tid; k < BCH * NH; k += 256) {
            const int o = k % NH, s = k / NH;
            const float a = sH2[s][o];
            float g = 0.0f;
#pragma unroll
            for (int j = 0; j < NO; ++j) g = fmaf(sW3[j * NH + o], sDY[s][j], g);
            sD2[s][o] = g * gelu_grad(a);
            sH2[s][o] = gelu(a);
        }
        __syncthreads();
#pragma unroll 1
        for (int k = tid; k < BCH * NH; k += 256) {
            const int h = k % NH, s = k / NH;
            const float a = sH1[s][h];
            float g = 0.0f;
#pragma unroll 8
            for (int o = 0; o < NH; ++o) g = fmaf(sW2[o * NH + h], sD2[s][o], g);
            sD1[s][h] = g * gelu_grad(a);
            sH1[s][h] = gelu(a);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < BWD_R; ++r) {
            const int e = tid + 256 * r;
            if (e >= NP) continue;
            float a = 0.0f;
            if (e < OB1) {
                const int h = e / NI, f = e - h * NI;
                #pragma unroll 4
                for (int s = 0; s < BCH; ++s) a = fmaf(sD1[s][h], sX[s][f], a);
            } else if (e < OW2) {
                const int h = e - OB1;
                #pragma unroll 4
                for (int s = 0; s < BCH; ++s) a += sD1[s][h];
            } else if (e < OB2) {
                const int o = (e - OW2) / NH, h = (e - OW2) % NH;
                #pragma unroll 4
                for (int s = 0; s < BCH; ++s) a = fmaf(sD2[s][o], sH1[s][h], a);
            } else if (e < OW3) {
                const int o = e - OB2;
                #pragma unroll 4
                for (int s = 0; s < BCH; ++s) a += sD2[s][o];
            } else if (e < OB3) {
                const int j = (e - OW3) / NH, h = (e - OW3) % NH;
                #pragma unroll 4
                for (int s = 0; s < BCH; ++s) a = fmaf(sDY[s][j], sH2[s][h], a);
            } else {
                const int j = e - OB3;
                #pragma unroll 4
                for (int s = 0; s < BCH; ++s) a += sDY[s][j];
            }
            acc[r] += a;
        }
    }
#pragma unroll
    for (int r = 0; r < BWD_R; ++r) {
        const int e = tid + 256 * r;
        if (e < NP) partial[(long long)blockIdx.x * NP + e] = acc[r];
    }
}

// grad[e] = sum over blocks of partial[b][e], in block order
__global__ __launch_bounds__(256) void grad_reduce_kernel(const float *partial, int nb, float *grad)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NP) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += (double)partial[(long long)b * NP + e];
    grad[e] = (float)s;
}

__global__ __launch_bounds__(256) void adam_kernel(float *theta, float *m, float *v, const float *g,
                                                   float lr, float b1, float b2, float eps, float c1,
                                                   float c2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NP) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    theta[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
}

}  // namespace ktm
