// Step-count proposal network for gfx950: features of the residual spectrum,
// BF16 MFMA convolutions (forward, input gradient, weight gradient), the
// regression head with its loss, ordered gradient reduction and Adam.
//
// The network (not part of the paper) maps the residual's power spectrum
// and the mask length L of an outer step to log2(m)/16, m being the inner
// step count that the stop test SD_m <= delta (equation "SD") selects, and
// to log2(L)/16.  Layout: activations channels-last [sample][position][64]
// in bfloat16; six convolutions of kernel 7, stride 2, zero padding 3 and
// ReLU (1024 -> 512 -> ... -> 16 positions); mean over positions; a 64 -> 2
// linear head in FP32.  Parameters live in one FP32 array in the order
// W_l[7][C_in][64], bias_l[64] for l = 0..5 (C_in = 8 for l = 0, else 64),
// Wh[2][64], bh[2].
//
// Every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16: with
// channels-last activations the 7*C_in inputs of one output position are
// contiguous, so a lane's 8-element operand is one 16-byte load.
#pragma once
#include "fif_net_shape.hpp"

namespace fif {

// --------------------------------------------------------- convolutions --

// z[row, o] = bias[o] + sum_k A[row, k] Wf[o, k], A[row, t*CIN + c] =
// in[b, 2q + t - 3, c] (row = b*lout + q), out = bf16(max(z, 0)).
// Wf: bf16 [64][KP] (k >= 7*CIN zero).  kNetRowsWG rows per workgroup; each
// wave owns 64 rows x 64 channels (4 x 4 tiles of 16 x 16), so every weight
// operand it loads feeds four MFMAs.
constexpr int kNetRowsWG = 256;

template <int CIN>
__global__ __launch_bounds__(kNetThreads) void k_conv_fwd(const bf16* __restrict__ in, int lin,
                                                         const bf16* __restrict__ wf,
                                                         const float* __restrict__ bias,
                                                         bf16* __restrict__ out, int nrows)
{
    constexpr int KF = kNetKw * CIN, KP = (KF + 31) / 32 * 32;
    const int lout = lin / 2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r0 = blockIdx.x * kNetRowsWG + wave * 64;
    const int kq = (lane >> 4) * 8;
    const bf16* base[4];
    int qv[4];
    bool live[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int row = r0 + m * 16 + (lane & 15);
        live[m] = row < nrows;
        const int b = live[m] ? row / lout : 0;
        qv[m] = live[m] ? row - b * lout : 0;
        base[m] = in + (int64_t)b * lin * CIN;
    }
    f32x4 acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < KP; k0 += 32) {
        const int k = k0 + kq;
        const int t = k / CIN, c = k - t * CIN;
        bf16x8 w[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) w[n] = *(const bf16x8*)(wf + (n * 16 + (lane & 15)) * KP + k);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int p = 2 * qv[m] + t - 3;
            bf16x8 a = bf16x8_zero();
            if (live[m] && t < kNetKw && p >= 0 && p < lin) a = *(const bf16x8*)(base[m] + (int64_t)p * CIN + c);
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w[n], acc[m][n], 0, 0, 0);
        }
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int col = n * 16 + (lane & 15);
        const float bv = bias[col];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + m * 16 + 4 * (lane >> 4) + i;
                if (r < nrows) out[(int64_t)r * kNetCh + col] = (bf16)fmaxf(acc[m][n][i] + bv, 0.f);
            }
    }
}

// Gradient with respect to the input of a 64-channel layer, masked by the
// input's own ReLU: dprev[b, p, c] = bf16([act[b, p, c] > 0] * sum_{t, o}
// dz[b, (p + 3 - t)/2, o] W[t, c, o]) over the t with p + 3 - t even and
// inside the output.  Wd: bf16 [64 c][7*64] (k = t*64 + o).  Same tiling as
// k_conv_fwd.
__global__ __launch_bounds__(kNetThreads) void k_conv_bwd_data(const bf16* __restrict__ dz, int lin,
                                                              const bf16* __restrict__ wd,
                                                              const bf16* __restrict__ act,
                                                              bf16* __restrict__ dprev, int nrows)
{
    constexpr int KP = kNetKw * kNetCh;
    const int lout = lin / 2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r0 = blockIdx.x * kNetRowsWG + wave * 64;
    const int kq = (lane >> 4) * 8;
    const bf16* base[4];
    int pv[4];
    bool live[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int row = r0 + m * 16 + (lane & 15);
        live[m] = row < nrows;
        const int b = live[m] ? row / lin : 0;
        pv[m] = live[m] ? row - b * lin : 0;
        base[m] = dz + (int64_t)b * lout * kNetCh;
    }
    f32x4 acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < KP; k0 += 32) {
        const int k = k0 + kq;
        const int t = k >> 6, o = k & 63;
        bf16x8 w[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) w[n] = *(const bf16x8*)(wd + (n * 16 + (lane & 15)) * KP + k);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int num = pv[m] + 3 - t;
            const int x = num >> 1;
            bf16x8 a = bf16x8_zero();
            if (live[m] && num >= 0 && (num & 1) == 0 && x < lout) a = *(const bf16x8*)(base[m] + (int64_t)x * kNetCh + o);
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w[n], acc[m][n], 0, 0, 0);
        }
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int col = n * 16 + (lane & 15);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + m * 16 + 4 * (lane >> 4) + i;
                if (r < nrows) {
                    const int64_t e = (int64_t)r * kNetCh + col;
                    const float g = (float)act[e] > 0.f ? acc[m][n][i] : 0.f;
                    dprev[e] = (bf16)g;
                }
            }
    }
}

// Partial weight and bias gradients of one layer over kNetWRows output rows:
// part[k][o] = sum_rows A[row, k] dz[row, o] (k = t*CIN + c, rows of KP), then
// part[KP*64 + o] = sum_rows dz[row, o].  The rows are staged transposed in
// LDS (32 at a time) so that every MFMA operand is one 16-byte LDS read.
template <int CIN>
__global__ __launch_bounds__(kNetThreads) void k_conv_bwd_w(const bf16* __restrict__ in, int lin,
                                                           const bf16* __restrict__ dz,
                                                           float* __restrict__ part, int nrows)
{
    constexpr int KF = kNetKw * CIN, KP = (KF + 31) / 32 * 32;
    constexpr int MT = KP / 16;                 // m tiles
    constexpr int MPW = (MT + 3) / 4;           // m tiles per wave
    constexpr int LD = 40;                      // LDS row stride (elements): 80 B, 16-B aligned
    __shared__ __attribute__((aligned(16))) bf16 As[KP * LD];
    __shared__ __attribute__((aligned(16))) bf16 Bs[kNetCh * LD];
    const int lout = lin / 2;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int kq = (lane >> 4) * 8;
    const int row0 = blockIdx.x * kNetWRows;
    f32x4 acc[MPW][4];
#pragma unroll
    for (int i = 0; i < MPW; ++i)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[i][n] = (f32x4){0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    if (KP > KF) {
        for (int e = tid; e < (KP - KF) * LD; e += kNetThreads) As[KF * LD + e] = (bf16)0.0f;
    }
    for (int rc = 0; rc < kNetWRows; rc += 32) {
        __syncthreads();
        // stage A: 32 rows x 7 taps x CIN/8 groups of 8 channels
        constexpr int NG = CIN / 8;
        for (int e = tid; e < 32 * kNetKw * NG; e += kNetThreads) {
            const int rr = e / (kNetKw * NG);
            const int rem = e - rr * (kNetKw * NG);
            const int t = rem / NG, g = rem - t * NG;
            const int row = row0 + rc + rr;
            bf16x8 v = bf16x8_zero();
            if (row < nrows) {
                const int b = row / lout, q = row - b * lout;
                const int p = 2 * q + t - 3;
                if (p >= 0 && p < lin) v = *(const bf16x8*)(in + ((int64_t)b * lin + p) * CIN + g * 8);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) As[(t * CIN + g * 8 + i) * LD + rr] = v[i];
        }
        // stage B: 32 rows x 8 groups of 8 output channels
        {
            const int rr = tid >> 3, g = tid & 7;
            const int row = row0 + rc + rr;
            bf16x8 v = bf16x8_zero();
            if (row < nrows) v = *(const bf16x8*)(dz + (int64_t)row * kNetCh + g * 8);
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[(g * 8 + i) * LD + rr] = v[i];
        }
        __syncthreads();
        if (tid < kNetCh) {
            float s = 0.f;
#pragma unroll 8
            for (int rr = 0; rr < 32; ++rr) s += (float)Bs[tid * LD + rr];
            bsum += s;
        }
        bf16x8 bop[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) bop[n] = *(const bf16x8*)(Bs + (n * 16 + (lane & 15)) * LD + kq);
#pragma unroll
        for (int i = 0; i < MPW; ++i) {
            const int mt = wave + 4 * i;
            if (mt < MT) {
                const bf16x8 a = *(const bf16x8*)(As + (mt * 16 + (lane & 15)) * LD + kq);
#pragma unroll
                for (int n = 0; n < 4; ++n) acc[i][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bop[n], acc[i][n], 0, 0, 0);
            }
        }
    }
    float* P = part + (int64_t)blockIdx.x * (KP * kNetCh + kNetCh);
#pragma unroll
    for (int i = 0; i < MPW; ++i) {
        const int mt = wave + 4 * i;
        if (mt < MT) {
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const int col = n * 16 + (lane & 15);
#pragma unroll
                for (int j = 0; j < 4; ++j) P[(mt * 16 + 4 * (lane >> 4) + j) * kNetCh + col] = acc[i][n][j];
            }
        }
    }
    if (tid < kNetCh) P[KP * kNetCh + tid] = bsum;
}

// grad[dst + i] = sum over chunks (in chunk order) of part[c*stride + src(i)],
// src(i) = i for the weights (i < nw), KP*64 + (i - nw) for the biases.
__global__ void k_reduce_parts(const float* __restrict__ part, int nchunks, int stride, int nw, int kp64,
                               int n, float* __restrict__ grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int src = i < nw ? i : kp64 + (i - nw);
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * stride + src];
    grad[i] = s;
}

// ----------------------------------------------------------------- head --

// One wave per sample: h = mean over the 16 positions of the last layer,
// y = bh + Wh h.  With targets: per-sample loss (y - t)^2 / (2B), the
// per-sample head gradient parts [Wh (2x64), bh (2)] and the masked,
// bf16-rounded gradient of the last layer's pre-activation.
__global__ __launch_bounds__(64) void k_head(const bf16* __restrict__ a6, const float* __restrict__ wh,
                                            const float* __restrict__ bh, float* __restrict__ y,
                                            const float* __restrict__ target, float* __restrict__ loss_b,
                                            float* __restrict__ hpart, bf16* __restrict__ dz6, int B)
{
    constexpr int NQ = kNetFeat >> kNetLayers;
    const int b = blockIdx.x, c = threadIdx.x;
    const bf16* a = a6 + (int64_t)b * NQ * kNetCh;
    float h = 0.f;
#pragma unroll
    for (int x = 0; x < NQ; ++x) h += (float)a[x * kNetCh + c];
    h *= 1.0f / NQ;
    float yv[kNetOut];
#pragma unroll
    for (int u = 0; u < kNetOut; ++u) {
        float v = wh[u * kNetCh + c] * h;
        // xor butterfly: every lane ends with the same, order-fixed sum
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        yv[u] = v + bh[u];
    }
    if (c < kNetOut) y[b * kNetOut + c] = c == 0 ? yv[0] : yv[1];
    if (!target) return;
    const float invB = 1.0f / (float)B;
    float dy[kNetOut], l = 0.f;
#pragma unroll
    for (int u = 0; u < kNetOut; ++u) {
        const float e = yv[u] - target[b * kNetOut + u];
        dy[u] = e * invB;
        l += e * e;
    }
    if (c == 0) loss_b[b] = l * 0.5f * invB;
    float* hp = hpart + (int64_t)b * (kNetOut * kNetCh + kNetOut);
    float dh = 0.f;
#pragma unroll
    for (int u = 0; u < kNetOut; ++u) {
        hp[u * kNetCh + c] = dy[u] * h;
        dh += wh[u * kNetCh + c] * dy[u];
    }
    if (c < kNetOut) hp[kNetOut * kNetCh + c] = c == 0 ? dy[0] : dy[1];
    const float g = dh * (1.0f / NQ);
    bf16* dz = dz6 + (int64_t)b * NQ * kNetCh;
#pragma unroll
    for (int x = 0; x < NQ; ++x) dz[x * kNetCh + c] = (bf16)((float)a[x * kNetCh + c] > 0.f ? g : 0.f);
}

// loss = sum of the per-sample losses in sample order (one thread)
__global__ void k_sum_loss(const float* __restrict__ loss_b, int B, float* __restrict__ loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += loss_b[b];
    *loss = s;
}

// ------------------------------------------------------------- optimizer --

// Adam on the FP32 master parameters (bias-corrected), then the bf16 copies.
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m1, float* __restrict__ m2,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// bf16 copies of every conv weight: Wf_l[o][t*C_in + c] (forward, KP columns,
// zero padded) and, for l >= 1, Wd_l[c][t*64 + o] (input gradient).
struct NetWeights {
    bf16* wf[kNetLayers];
    bf16* wd[kNetLayers];
};

__global__ void k_pack_weights(const float* __restrict__ p, NetWeights W)
{
    const int l = blockIdx.y;
    const int cin = net_cin(l), kf = net_kf(l), kp = net_kp(l);
    const float* src = p + net_w_off(l);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kp * kNetCh; e += gridDim.x * blockDim.x) {
        const int o = e / kp, k = e - o * kp;
        W.wf[l][e] = (bf16)(k < kf ? src[k * kNetCh + o] : 0.f);
        if (l > 0 && k < kf) {
            // same element in the input-gradient layout
            const int t = k / cin, c = k - t * cin;
            W.wd[l][c * (kNetKw * kNetCh) + t * kNetCh + o] = (bf16)src[k * kNetCh + o];
        }
    }
}

}  // namespace fif
