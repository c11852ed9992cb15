// Proposal hooks of the decomposition: network input features of every
// active signal's residual spectrum, and the proposed inner step count taken
// from the network output.
#pragma once
#include "fif_kernels.hpp"
#include "fif_net_shape.hpp"

namespace fif {

// ------------------------------------------------------------ features --

// One workgroup per signal: channel 0 = log2(mean group power / total power
// + 2^-60) / 16 over 1024 contiguous groups of bins 1..N/2, channel 1 =
// log2(L)/16, channels 2..7 = 0.  Row `slot` of out (bf16 [.][1024][8]).
struct FeatArgs {
    const SigDesc* sigs;
    const SigState* st;
    const double2* spec0;
    const double2* spec1;
    int t;
    uint16_t* out;             // proposal slots, indexed by signal
    uint16_t* rec;             // recorded rows [B][max_imfs], or null
    int max_imfs;
};

__global__ __launch_bounds__(kNetThreads) void k_features(FeatArgs A)
{
    __shared__ double shd[kNetThreads / 64];
    const int s = blockIdx.x;
    const SigState* S = A.st + s;
    if (!S->active) return;
    const SigDesc d = A.sigs[s];
    const double2* R = ((A.t & 1) ? A.spec1 : A.spec0) + d.spec_off;
    const int64_t H = d.N / 2;
    double tot[1] = {0.0};
    for (int64_t j = 1 + threadIdx.x; j <= H; j += kNetThreads) {
        const double2 z = R[j];
        tot[0] += z.x * z.x + z.y * z.y;
    }
    block_sum<double, kNetThreads, 1>(tot, shd);
    const float lch = (float)(log2((double)S->L) / 16.0);
    bf16* o0 = (bf16*)A.out + (int64_t)s * kNetFeat * kNetCin0;
    bf16* o1 = A.rec ? (bf16*)A.rec + ((int64_t)s * A.max_imfs + A.t) * kNetFeat * kNetCin0 : nullptr;
    for (int q = threadIdx.x; q < kNetFeat; q += kNetThreads) {
        const int64_t j0 = ((int64_t)q * H) / kNetFeat;
        const int64_t j1 = max(((int64_t)(q + 1) * H) / kNetFeat, j0 + 1);
        double sum = 0.0;
        for (int64_t j = j0; j < j1; ++j) {
            const double2 z = R[1 + j];
            sum += z.x * z.x + z.y * z.y;
        }
        const double v = tot[0] > 0.0 ? log2(sum / (double)(j1 - j0) / tot[0] + 0x1p-60) / 16.0 : -60.0 / 16.0;
        bf16x8 row = bf16x8_zero();
        row[0] = (bf16)(float)v;
        row[1] = (bf16)lch;
        *(bf16x8*)(o0 + (int64_t)q * kNetCin0) = row;
        if (o1) *(bf16x8*)(o1 + (int64_t)q * kNetCin0) = row;
    }
}

// Proposed step count of signal s0 + i from network output row i (log2(m)/16).
__global__ void k_propose(const float* __restrict__ y, int s0, int n, int64_t cap,
                          const SigState* __restrict__ st, int64_t* __restrict__ prop)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = s0 + i;
    if (!st[s].active) {
        prop[s] = 0;
        return;
    }
    const double lm = 16.0 * (double)y[i * kNetOut];
    const double m = exp2(fmin(fmax(lm, 0.0), 62.0));
    prop[s] = max((int64_t)1, min(cap, (int64_t)llrint(m)));
}

}  // namespace fif
