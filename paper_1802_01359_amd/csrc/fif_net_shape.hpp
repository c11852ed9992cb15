// Shape of the step-count proposal network: sizes, parameter offsets and the
// bfloat16 vector types shared by the network kernels and the feature kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fif {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNetFeat = 1024;
constexpr int kNetCin0 = 8;
constexpr int kNetCh = 64;
constexpr int kNetKw = 7;
constexpr int kNetLayers = 6;
constexpr int kNetOut = 2;
constexpr int kNetThreads = 256;       // 4 waves, 64 output rows per workgroup
constexpr int kNetWRows = 256;         // rows per workgroup of the weight gradient

__host__ __device__ constexpr int net_cin(int l) { return l == 0 ? kNetCin0 : kNetCh; }
__host__ __device__ constexpr int net_kf(int l) { return kNetKw * net_cin(l); }
__host__ __device__ constexpr int net_kp(int l) { return (net_kf(l) + 31) / 32 * 32; }
__host__ __device__ constexpr int net_len_in(int l) { return kNetFeat >> l; }
__host__ __device__ constexpr int net_w_off(int l)
{
    int off = 0;
    for (int i = 0; i < l; ++i) off += net_kf(i) * kNetCh + kNetCh;
    return off;
}
constexpr int kNetHeadOff = net_w_off(kNetLayers);
constexpr int kNetParams = kNetHeadOff + kNetOut * kNetCh + kNetOut;
static_assert(kNetParams == 147458, "parameter count");

__device__ __forceinline__ bf16x8 bf16x8_zero()
{
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (bf16)0.0f;
    return z;
}

}  // namespace fif
