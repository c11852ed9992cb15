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
    const LenPlan* lens;
    const int32_t* itab;
    const SigState* st;
    const double2* spec0;
    const double2* spec1;
    int t;
    uint16_t* out;             // proposal slots, indexed by signal
    uint16_t* rec;             // recorded rows [B][max_imfs], or null
    int max_imfs;
    int s0;                    // first signal (workgroup b handles signal s0 + b)
};

// Bins are read once, coalesced, in tiles of kFeatTile staged in LDS; each
// group's sum accumulates (in bin order) in an LDS slot owned by one thread
// per tile, and the total is an ordered block sum of the per-thread tile
// sums.
constexpr int kFeatTile = 2048;

__device__ __forceinline__ int64_t feat_j0(int q, int64_t H) { return ((int64_t)q * H) / kNetFeat; }
__device__ __forceinline__ int64_t feat_j1(int q, int64_t H)
{
    return max(((int64_t)(q + 1) * H) / kNetFeat, feat_j0(q, H) + 1);
}

__global__ __launch_bounds__(kNetThreads) void k_features(FeatArgs A)
{
    __shared__ double pw[kFeatTile];
    __shared__ double gs[kNetFeat];
    __shared__ double shd[kNetThreads / 64];
    const int s = A.s0 + blockIdx.x;
    const SigState* S = A.st + s;
    if (!S->active) return;
    const SigDesc d = A.sigs[s];
    const double2* R = ((A.t & 1) ? A.spec1 : A.spec0) + d.spec_off;
    const LenPlan& lp = A.lens[d.len_id];
    const int64_t H = d.N / 2;
    const int tid = threadIdx.x;
    for (int q = tid; q < kNetFeat; q += kNetThreads) gs[q] = 0.0;
    double tot[1] = {0.0};
    for (int64_t t0 = 0; t0 < H; t0 += kFeatTile) {
        const int n = (int)min((int64_t)kFeatTile, H - t0);
        __syncthreads();
        for (int i = tid; i < n; i += kNetThreads) {
            const double2 z = R[pos_of(lp, A.itab, t0 + i + 1)];   // bin t0 + i + 1
            const double v = z.x * z.x + z.y * z.y;
            pw[i] = v;
            tot[0] += v;
        }
        __syncthreads();
        // groups meeting [t0, t0 + n): each summed by one thread, in bin order
        const int qa = (int)max((int64_t)0, (t0 * kNetFeat) / H - 1);
        const int qb = (int)min((int64_t)kNetFeat - 1, ((t0 + n) * kNetFeat) / H + 1);
        for (int q = qa + tid; q <= qb; q += kNetThreads) {
            const int64_t a = max(feat_j0(q, H), t0), b = min(feat_j1(q, H), t0 + n);
            double acc = 0.0;
            for (int64_t u = a; u < b; ++u) acc += pw[u - t0];
            if (b > a) gs[q] += acc;
        }
    }
    block_sum<double, kNetThreads, 1>(tot, shd);
    const float lch = (float)(log2((double)S->L) / 16.0);
    bf16* o0 = (bf16*)A.out + (int64_t)s * kNetFeat * kNetCin0;
    bf16* o1 = A.rec ? (bf16*)A.rec + ((int64_t)s * A.max_imfs + A.t) * kNetFeat * kNetCin0 : nullptr;
    for (int q = tid; q < kNetFeat; q += kNetThreads) {
        const double cnt = (double)(feat_j1(q, H) - feat_j0(q, H));
        const double v = tot[0] > 0.0 ? log2(gs[q] / cnt / tot[0] + 0x1p-60) / 16.0 : -60.0 / 16.0;
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
