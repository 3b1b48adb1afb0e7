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

// ------------------------------------------------- matrix-core inference --
// The start network inside the recovery kernels runs on the matrix cores: the
// 64 cells of a wave are the batch of three small products with fp16 operands
// and fp32 accumulation (v_mfma_f32_16x16x32_f16: A 16x32, B 32x16, D 16x16;
// lane l holds row l%16 of A and column l%16 of B at k = 8(l/16) + j, j < 8,
// and column l%16 of D at rows 4(l/16) + i, i < 4).  fp16 rather than bf16:
// its 11-bit significand keeps the rounding of weights and activations
// (5e-4) below the network's own start error (~1e-3); bf16's (4e-3) would not.
//   layer 1: for each N-tile of 16 cells, B = their features (K = 11 padded
//     to 32, through the wave's LDS rows), four M-tiles of 16 hidden units;
//   layer 2: B = GELU of layer 1's D registers as they are: hidden unit
//     u(mt, l, i) = 16 mt + 4 (l/16) + i sits in register i of D tile mt of
//     lane l, so the K order of a K-step s is h(s, l, j) = u(2s + j/4, l, j%4)
//     and the columns of W2 are permuted to it when the weights are packed
//     (mlp_pack_kernel); no value moves between lanes;
//   layer 3: y_0 only, a dot product of W3's first row with the 16 units a lane
//     holds, summed over the four lanes of the cell's column (two exchanges).
// Lane l keeps y_0 of cell l of the wave.  GELU through erf by Abramowitz &
// Stegun 7.1.26 (|error| < 1.5e-7), well inside fp16.
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

struct MlpPacked {
    h8_t a1[4][64];       // layer 1 A operand: M-tile, lane
    h8_t a2[4][2][64];    // layer 2 A operand: M-tile, K-step, lane
    float b1[NH], b2[NH], w3[NH], b3;
};

constexpr int XS_K = 16;  // fp16 features staged per cell (11 used)

// hidden unit of layer 1 whose GELU lane l passes in slot j of K-step s of layer 2
__host__ __device__ __forceinline__ int mlp_h2(int s, int l, int j)
{
    return 16 * (2 * s + j / 4) + 4 * (l / 16) + (j % 4);
}

// one block of 256 threads: W (FP32, the layout of kt_mlp_set) into K
__global__ __launch_bounds__(256) void mlp_pack_kernel(const float *__restrict__ w, MlpPacked *K)
{
    for (int e = threadIdx.x; e < 4 * 64 * 8; e += 256) {
        const int mt = e / 512, l = (e / 8) % 64, j = e % 8, k = 8 * (l / 16) + j;
        K->a1[mt][l][j] = (_Float16)(k < NI ? w[OW1 + (16 * mt + l % 16) * NI + k] : 0.0f);
    }
    for (int e = threadIdx.x; e < 4 * 2 * 64 * 8; e += 256) {
        const int mt = e / 1024, s = (e / 512) % 2, l = (e / 8) % 64, j = e % 8;
        K->a2[mt][s][l][j] = (_Float16)w[OW2 + (16 * mt + l % 16) * NH + mlp_h2(s, l, j)];
    }
    for (int e = threadIdx.x; e < NH; e += 256) {
        K->b1[e] = w[OB1 + e];
        K->b2[e] = w[OB2 + e];
        K->w3[e] = w[OW3 + e];
    }
    if (threadIdx.x == 0) K->b3 = w[OB3];
}

// GELU(a) = a Phi(a) = a (1 + erf(a / sqrt 2)) / 2, erf by Abramowitz & Stegun 7.1.26
__device__ __forceinline__ float gelu_as(float a)
{
    const float z = fabsf(a) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, z, 1.0f));
    float p = 1.061405429f;
    p = fmaf(p, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    const float erfz = 1.0f - p * t * __expf(-z * z);
    return 0.5f * a * (1.0f + copysignf(erfz, a));
}

// y_0 of the lane's cell from its features x (any values in lanes whose result
// is not used).  Every lane of the wave must call it (the matrix instructions
// work on the whole wave); xs: this wave's 64 x XS_K staging rows in LDS.
__device__ __forceinline__ float forward_y0_mfma(const MlpPacked *__restrict__ K, const float x[NI],
                                                 _Float16 (*xs)[XS_K])
{
    const int l = (int)__lane_id();
    const int g = l >> 4, c = l & 15;
#pragma unroll
    for (int k = 0; k < XS_K; ++k) xs[l][k] = (_Float16)(k < NI ? x[k] : 0.0f);
    __builtin_amdgcn_wave_barrier();
    float y0 = 0.0f;
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
        h8_t b1;
#pragma unroll
        for (int j = 0; j < 8; ++j) b1[j] = g < 2 ? xs[16 * t + c][8 * g + j] : (_Float16)0.0f;
        f4_t d1[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f4_t acc;
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = K->b1[16 * mt + 4 * g + i];
            d1[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(K->a1[mt][l], b1, acc, 0, 0, 0);
        }
        h8_t b2[2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) b2[s][j] = (_Float16)gelu_as(d1[2 * s + j / 4][j % 4]);
        float part = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f4_t acc;
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = K->b2[16 * mt + 4 * g + i];
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(K->a2[mt][0][l], b2[0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(K->a2[mt][1][l], b2[1], acc, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) part = fmaf(K->w3[16 * mt + 4 * g + i], gelu_as(acc[i]), part);
        }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (t == g) y0 = part + K->b3;
    }
    __builtin_amdgcn_wave_barrier();
    return y0;
}

}  // namespace ktm
