// gfx950 kernels of the batched FIF hot path.
//
// Per outer step t (Algorithm 2, one IMF):
//   k_scan     combine the run summaries of the residual (extrema count; the
//              min/max come from order-independent atomics), apply the stop
//              rules, fix L, then pick m: one FP32 pass over geometric
//              candidates, safeguarded regula falsi on the Parseval form of
//              SD in FP32, and an FP64 confirmation SD_m <= delta < SD_{m-1}
//              (exact FP64 search around the estimate if it fails);
//   k_single / k_pass1 + k_pass2
//              the inverse transform of z = (g + i (1 - g)) R_hat with
//              g = (1 - lambda)^m: real part = IMF (Theorem 5 / Section 4
//              one-step formula), imaginary part = the new residual, whose
//              extrema are counted on the fly; R_hat <- (1 - g) R_hat.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>

#include "../../include/fif.h"
#include "fif_fft.hpp"
#include "fif_types.hpp"

namespace fif {

// ------------------------------------------------------------------ runs --

__device__ __forceinline__ int sgn_step(double a, double b) { return (b > a) - (b < a); }

__device__ __forceinline__ RunState run_empty()
{
    RunState r;
    r.first = r.last = 0.0;
    r.cnt = 0;
    r.fs = r.ls = 0;
    r.empty = 1;
    r.nonfinite = 0;
    return r;
}

__device__ __forceinline__ void run_push(RunState& r, double v)
{
    if (!isfinite(v)) r.nonfinite = 1;
    if (r.empty) {
        r.first = r.last = v;
        r.empty = 0;
    } else {
        const int d = sgn_step(r.last, v);
        if (d != 0) {
            if (r.ls != 0 && r.ls != d) ++r.cnt;
            if (r.fs == 0) r.fs = (int8_t)d;
            r.ls = (int8_t)d;
        }
        r.last = v;
    }
}

// Word-wise copies of a RunState to and from memory: aggregate copies of
// this struct (three words, the last holding four bytes) were lowered through
// private scratch memory.
static_assert(sizeof(RunState) == 24 && offsetof(RunState, cnt) == 16 && offsetof(RunState, fs) == 20 &&
                  offsetof(RunState, ls) == 21 && offsetof(RunState, empty) == 22 &&
                  offsetof(RunState, nonfinite) == 23,
              "RunState layout");
__device__ __forceinline__ RunState run_load(const RunState* p)
{
    const long long* q = reinterpret_cast<const long long*>(p);
    const long long w0 = q[0], w1 = q[1], w2 = q[2];
    RunState r;
    r.first = __longlong_as_double(w0);
    r.last = __longlong_as_double(w1);
    r.cnt = (int)(w2 & 0xffffffffLL);
    const int b = (int)(w2 >> 32);
    r.fs = (int8_t)(b & 0xff);
    r.ls = (int8_t)((b >> 8) & 0xff);
    r.empty = (int8_t)((b >> 16) & 0xff);
    r.nonfinite = (int8_t)((b >> 24) & 0xff);
    return r;
}

__device__ __forceinline__ void run_store(RunState* p, const RunState& r)
{
    long long* q = reinterpret_cast<long long*>(p);
    const int b = (int)(uint8_t)r.fs | ((int)(uint8_t)r.ls << 8) | ((int)(uint8_t)r.empty << 16) |
                  ((int)(uint8_t)r.nonfinite << 24);
    q[0] = __double_as_longlong(r.first);
    q[1] = __double_as_longlong(r.last);
    q[2] = (long long)(unsigned int)r.cnt | ((long long)b << 32);
}

// a then b
__device__ __forceinline__ RunState run_combine(const RunState& a, const RunState& b)
{
    if (a.empty) return b;
    if (b.empty) return a;
    RunState r;
    const int d = sgn_step(a.last, b.first);
    int cnt = a.cnt + b.cnt;
    int x = a.ls;
    if (d != 0) {
        if (x != 0 && x != d) ++cnt;
        x = d;
    }
    if (b.fs != 0 && x != 0 && x != b.fs) ++cnt;
    r.fs = (int8_t)(a.fs != 0 ? a.fs : (d != 0 ? d : b.fs));
    r.ls = (int8_t)(b.ls != 0 ? b.ls : (d != 0 ? d : a.ls));
    r.cnt = cnt;
    r.first = a.first;
    r.last = b.last;
    r.empty = 0;
    r.nonfinite = a.nonfinite | b.nonfinite;
    return r;
}

// ---------------------------------------------------- wave-level exchange
// ds_swizzle in bit-mask mode: lane l reads lane (l ^ XM) within its half
// wave (XM < 32).  No address registers are needed, unlike ds_bpermute.
template <int XM>
__device__ __forceinline__ int swz_i(int v)
{
    return __builtin_amdgcn_ds_swizzle(v, 0x1F | (XM << 10));
}
template <int XM>
__device__ __forceinline__ float swz(float v)
{
    return __int_as_float(swz_i<XM>(__float_as_int(v)));
}
template <int XM>
__device__ __forceinline__ double swz(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = swz_i<XM>((int)(b & 0xffffffffLL));
    const int hi = swz_i<XM>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ int rdl_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float rdl(float v, int l) { return __int_as_float(rdl_i(__float_as_int(v), l)); }
__device__ __forceinline__ double rdl(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = rdl_i((int)(b & 0xffffffffLL), l);
    const int hi = rdl_i((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Value of r in lane (l ^ XM) (XM < 32).
template <int XM>
__device__ __forceinline__ RunState run_swz(const RunState& r)
{
    RunState o;
    o.first = swz<XM>(r.first);
    o.last = swz<XM>(r.last);
    o.cnt = swz_i<XM>(r.cnt);
    int packed = (int)(uint8_t)r.fs | ((int)(uint8_t)r.ls << 8) | ((int)r.empty << 16) |
                 ((int)r.nonfinite << 24);
    packed = swz_i<XM>(packed);
    o.fs = (int8_t)(packed & 0xff);
    o.ls = (int8_t)((packed >> 8) & 0xff);
    o.empty = (int8_t)((packed >> 16) & 0xff);
    o.nonfinite = (int8_t)((packed >> 24) & 0xff);
    return o;
}

__device__ __forceinline__ RunState run_readlane(const RunState& r, int l)
{
    RunState o;
    o.first = rdl(r.first, l);
    o.last = rdl(r.last, l);
    o.cnt = rdl_i(r.cnt, l);
    int packed = (int)(uint8_t)r.fs | ((int)(uint8_t)r.ls << 8) | ((int)r.empty << 16) |
                 ((int)r.nonfinite << 24);
    packed = rdl_i(packed, l);
    o.fs = (int8_t)(packed & 0xff);
    o.ls = (int8_t)((packed >> 8) & 0xff);
    o.empty = (int8_t)((packed >> 16) & 0xff);
    o.nonfinite = (int8_t)((packed >> 24) & 0xff);
    return o;
}

template <int XM>
__device__ __forceinline__ void run_step(RunState& r, int lane)
{
    RunState o = run_swz<XM>(r);
    if ((lane & (2 * XM - 1)) == 0) r = run_combine(r, o);
}

// Ordered reduction of one RunState per thread (thread order = sample
// order).  Result valid in thread 0.  `sh` holds one RunState per wave.
template <int NT>
__device__ __forceinline__ RunState block_run_reduce(RunState r, RunState* sh)
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    run_step<1>(r, lane);
    run_step<2>(r, lane);
    run_step<4>(r, lane);
    run_step<8>(r, lane);
    run_step<16>(r, lane);
    const RunState upper = run_readlane(r, 32);
    if (lane == 0) run_store(sh + wave, run_combine(r, upper));
    __syncthreads();
    RunState tot = run_empty();
    if (threadIdx.x == 0) {
        for (int w = 0; w < NW; ++w) tot = run_combine(tot, run_load(sh + w));
    }
    __syncthreads();
    return tot;
}

// order-preserving integer key of a double (for atomic min / max)
__device__ __forceinline__ long long dkey(double v)
{
    const long long b = __double_as_longlong(v);
    return b >= 0 ? b : (b ^ 0x7fffffffffffffffLL);
}
__device__ __forceinline__ double dval(long long k)
{
    return __longlong_as_double(k >= 0 ? k : (k ^ 0x7fffffffffffffffLL));
}



// ------------------------------------------------------------ reductions --

// Butterfly sum within each half wave; equal bits in every lane of a half
// (addition is commutative and every lane uses the same tree).
template <typename T>
__device__ __forceinline__ T half_wave_sum(T v)
{
    v += swz<16>(v);
    v += swz<8>(v);
    v += swz<4>(v);
    v += swz<2>(v);
    v += swz<1>(v);
    return v;
}

// Sum of NV values per thread over the block; every thread gets the totals
// (same order everywhere: deterministic).  sh: NV * NT/64 elements.
template <typename T, int NT, int NV>
__device__ __forceinline__ void block_sum(T* v, T* sh)
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const T h = half_wave_sum(v[i]);
        v[i] = rdl(h, 0) + rdl(h, 32);
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[NV * wave + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        T s = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += sh[NV * w + i];
        v[i] = s;
    }
    __syncthreads();
}

// Work item of workgroup b in a grid of G: workgroups are dispatched to the
// eight XCDs in turn (b mod 8), so consecutive items are given to workgroups
// b, b + 8, ... of one XCD: the items of one signal then share that XCD's L2,
// where their partial-line writes (64-byte IMF runs, 12-byte run summaries)
// merge before they reach HBM.  A bijection of [0, G).
__device__ __forceinline__ int xcd_item(int b, int G)
{
    const int per = G >> 3, rem = G & 7, x = b & 7;
    return x * per + min(x, rem) + (b >> 3);
}

// min and max over the block, result in every thread
template <int NT>
__device__ __forceinline__ void block_minmax(double& mn, double& mx, double* sh)
{
    constexpr int NW = NT / 64;
    mn = fmin(mn, swz<16>(mn));
    mx = fmax(mx, swz<16>(mx));
    mn = fmin(mn, swz<8>(mn));
    mx = fmax(mx, swz<8>(mx));
    mn = fmin(mn, swz<4>(mn));
    mx = fmax(mx, swz<4>(mx));
    mn = fmin(mn, swz<2>(mn));
    mx = fmax(mx, swz<2>(mx));
    mn = fmin(mn, swz<1>(mn));
    mx = fmax(mx, swz<1>(mx));
    mn = fmin(rdl(mn, 0), rdl(mn, 32));
    mx = fmax(rdl(mx, 0), rdl(mx, 32));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sh[2 * wave] = mn;
        sh[2 * wave + 1] = mx;
    }
    __syncthreads();
    for (int w = 0; w < NW; ++w) {
        mn = fmin(mn, sh[2 * w]);
        mx = fmax(mx, sh[2 * w + 1]);
    }
    __syncthreads();
}

// ------------------------------------------------------ window spectrum --

// (a * b) mod n for a*b < 2^53 and n < 2^26: the product and q*n are exact
// in FP64; the quotient from the rounded reciprocal is off by at most one.
__device__ __forceinline__ int64_t mulmod53(int64_t a, int64_t b, int64_t n, double inv_n)
{
    const double p = (double)a * (double)b;
    const double dn = (double)n;
    const double q = floor(p * inv_n);
    int64_t r = (int64_t)(p - q * dn);
    if (r < 0) r += n;
    if (r >= n) r -= n;
    return r;
}

// Window spectrum of one plan length at the current L.
struct Lam {
    int64_t N, Lmod;
    int64_t mask;         // N - 1 when N is a power of two (L j mod N by a mask), else 0
    double invN, invL;
    const double* sinT;   // sin(pi u/N), u <= N/2
    const double* isinT;  // 1/sin(pi u/N), 1 <= u <= N/2
    const double* tab;    // sampled window shape: lambda_j of this step by bin, else null
    int inl;              // LenPlan::lam_inline
};

__device__ __forceinline__ Lam make_lam(const LenPlan& lp, const double* dtab, int64_t L, const double* tab)
{
    Lam w;
    w.tab = tab;
    w.mask = ((lp.N & (lp.N - 1)) == 0) ? lp.N - 1 : 0;
    w.N = lp.N;
    w.Lmod = L % lp.N;
    w.invN = lp.invN;
    w.invL = 1.0 / (double)L;
    w.sinT = dtab + lp.sin_off;
    w.isinT = dtab + lp.isin_off;
    w.inl = lp.lam_inline;
    return w;
}

// sin(pi u / N) and 1 / sin(pi u / N) exactly as the table fills compute
// them, so that a sine evaluated in place equals its table entry bit for bit.
__device__ __forceinline__ double sin_u(int64_t u, int64_t N) { return sinpi((double)u / (double)N); }
__device__ __forceinline__ double isin_u(int64_t u, int64_t N) { return 1.0 / sinpi((double)u / (double)N); }

// t = L j mod N folded into [0, N/2] (N <= 2^26, every plan length): for a
// power of two the low 32 bits of the product decide it, otherwise the FP64
// quotient does (mulmod53).
__device__ __forceinline__ int lam_arg(int64_t j, const Lam& w)
{
    const int t = w.mask ? (int)(((uint32_t)w.Lmod * (uint32_t)j) & (uint32_t)w.mask)
                         : (int)mulmod53(w.Lmod, j, w.N, w.invN);
    const int n = (int)w.N;
    return min(t, n - t);
}

// lambda_j = [sin(pi L j / N) / (L sin(pi j / N))]^4, the DFT of the
// circulant column of the triangle-squared window, with L*j reduced mod N
// exactly; the sines come from the tables or are evaluated in place.
__device__ __forceinline__ double lambda_at(int64_t j, const Lam& w)
{
    if (j == 0) return 1.0;
    if (w.tab) return w.tab[j];
    const int t = lam_arg(j, w);
    const double st = w.inl ? sin_u(t, w.N) : w.sinT[t];
    const double is = w.inl == 2 ? isin_u(j, w.N) : w.isinT[j];
    const double q = st * is * w.invL;
    const double q2 = q * q;
    return q2 * q2;
}

// lambda_j in FP32 for the FP32 search for m (the FP64 lambda_at decides
// everywhere else): the reduced argument t = L j mod N is exact as before,
// sin(pi t / N) comes from sinpif instead of a table gather (a random access
// per bin), 1 / sin(pi j / N) from the table (ISIN = false: read in bin
// order) or from sinpif too (ISIN = true).
template <bool ISIN = false>
__device__ __forceinline__ float lambda_f32(int64_t j, const Lam& w, float invNf, float invLf)
{
    if (j == 0) return 1.f;
    if (w.tab) return (float)w.tab[j];
    const int t = lam_arg(j, w);
    const float is = ISIN ? 1.f / sinpif((float)j * invNf) : (float)w.isinT[j];
    const float q = sinpif((float)t * invNf) * is * invLf;
    const float q2 = q * q;
    return fminf(q2 * q2, 1.f);
}

// x^e by binary powering (e >= 0)
__device__ __forceinline__ double ipow(double x, int64_t e)
{
    double r = 1.0;
    while (e) {
        if (e & 1) r *= x;
        x *= x;
        e >>= 1;
    }
    return r;
}

// Noise floor of the relative stop test: bins with |R_j|^2 below this
// fraction of the strongest non-constant bin's are not counted in SD.
constexpr double kSdNoise = 1e-26;

// Exponent above which (1 - lambda)^e is taken as exp(e log1p(-lambda)):
// binary powering carries a relative error of about e ulps of 1 - lambda.
constexpr int64_t kPowByMul = 1023;

// (1 - lambda)^m
__device__ __forceinline__ double gain_pow(double lam, int64_t m)
{
    if (lam >= 1.0) return 0.0;
    if (m <= kPowByMul) return ipow(1.0 - lam, m);
    return exp((double)m * log1p(-lam));
}

// Thresholded gain: a bin whose factor is >= 1 - gamma is taken whole
// (lambda replaced by 0); gamma = 0 leaves the gain unchanged.
__device__ __forceinline__ double gain_th(double g, double gamma)
{
    return (gamma > 0.0 && g >= 1.0 - gamma) ? 1.0 : g;
}

// --------------------------------------------------------------- tables --

__global__ void k_fill_sin(double* __restrict__ out, int64_t N, int64_t count)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < count) out[u] = sin_u(u, N);
}

__global__ void k_fill_isin(double* __restrict__ out, int64_t N, int64_t count)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < count) out[u] = u == 0 ? 0.0 : isin_u(u, N);
}

// exp(-2 pi i k stride / den) for k < count, written at out[k]
__global__ void k_fill_roots(double2* __restrict__ out, int64_t den, int64_t count, int64_t stride)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) {
        double s, c;
        sincospi(2.0 * (double)(k * stride) / (double)den, &s, &c);
        out[k] = make_double2(c, -s);
    }
}

// four-step twiddle exp(-+2 pi i a / N), a < N, from the split tables
// Scalar fields of a length plan held in registers by the step kernels (the
// plan itself sits in global memory, which their stores might alias, so
// reading it inside a loop would reload it).
struct PlanRegs {
    int64_t N;
    int N1, N2, TC, TR, paired, spec_perm;
    int64_t big_lo_off, big_hi_off;
    int big_split, big_shift;
};
__device__ __forceinline__ PlanRegs plan_regs(const LenPlan& lp)
{
    PlanRegs r;
    r.N = lp.N;
    r.N1 = lp.N1;
    r.N2 = lp.N2;
    r.TC = lp.TC;
    r.TR = lp.TR;
    r.paired = lp.paired;
    r.spec_perm = lp.spec_perm;
    r.big_lo_off = lp.big_lo_off;
    r.big_hi_off = lp.big_hi_off;
    r.big_split = lp.big_split;
    r.big_shift = lp.big_shift;
    return r;
}

template <bool INV>
__device__ __forceinline__ double2 big_twiddle(const PlanRegs& lp, const double2* __restrict__ tabs, int64_t a)
{
    const int ai = (int)a;
    double2 w = cmul(tabs[lp.big_hi_off + (ai >> lp.big_shift)], tabs[lp.big_lo_off + (ai & (lp.big_split - 1))]);
    if (INV) w.y = -w.y;
    return w;
}

// ------------------------------------------------------- init statistics --

// Run summary, sum, min and max of one tile of the input signal (first
// outer step's count and rounding floor, non-finite check).
template <typename InT>
__global__ __launch_bounds__(kFftThreads) void k_init_stats(const SigDesc* __restrict__ sigs,
                                                             const Work* __restrict__ work,
                                                             const InT* __restrict__ x,
                                                             RunState* __restrict__ parts,
                                                             double* __restrict__ psum,
                                                             SigState* __restrict__ st)
{
    __shared__ RunState sh[kFftThreads / 64];
    __shared__ double shd[2 * (kFftThreads / 64)];
    const Work w = work[blockIdx.x];
    const SigDesc d = sigs[w.sig];
    const int64_t t0 = (int64_t)w.tile * kFftCap;
    const int64_t len = min((int64_t)kFftCap, d.N - t0);
    const int chunk = (int)((len + kFftThreads - 1) / kFftThreads);
    const int64_t a = (int64_t)threadIdx.x * chunk, b = min(len, a + chunk);
    RunState r = run_empty();
    double s = 0.0, mn = INFINITY, mx = -INFINITY;
    for (int64_t i = a; i < b; ++i) {
        const double v = (double)x[d.off + t0 + i];
        run_push(r, v);
        s += v;
        mn = fmin(mn, v);
        mx = fmax(mx, v);
    }
    double sv[1] = {s};
    block_sum<double, kFftThreads, 1>(sv, shd);
    block_minmax<kFftThreads>(mn, mx, shd);
    r = block_run_reduce<kFftThreads>(r, sh);
    if (threadIdx.x == 0) {
        parts[d.part_off + w.tile] = r;
        psum[d.part_off + w.tile] = sv[0];
        atomicMin(&st[w.sig].kmin, dkey(mn));
        atomicMax(&st[w.sig].kmax, dkey(mx));
    }
}

// ------------------------------------------------ sampled window shapes --

// Folded taps of a sampled window shape for every active signal of
// [s0, s0 + gridDim.x) at its current L: h_q = shape[i] + (shape[i+1] -
// shape[i]) rr / L with |q| K = i L + rr (linear interpolation of the K + 1
// samples at x = |q|/L), for |q| <= L - 1, summed into slot q mod N.  Also
// writes the sum of the taps (H_0).  The taps are unnormalised; the
// eigenvalue table divides by that sum.  Floors of quotients of integers
// below 2^53 are taken in FP64, where they are exact.
__global__ __launch_bounds__(kFftThreads) void k_window_taps(const SigDesc* __restrict__ sigs,
                                                              const SigState* __restrict__ st,
                                                              const double* __restrict__ shape, int K,
                                                              double* __restrict__ taps, double* __restrict__ wsum,
                                                              int s0)
{
    __shared__ double shd[kFftThreads / 64];
    const int s = s0 + blockIdx.x;
    if (!st[s].active) return;
    const SigDesc d = sigs[s];
    const int64_t N = d.N, L = st[s].L;
    const double dN = (double)N, dL = (double)L;
    double acc[1] = {0.0};
    for (int64_t n = threadIdx.x; n < N; n += kFftThreads) {
        // smallest q = n (mod N) with q >= -(L-1), then every N up to L-1
        int64_t q = n - (int64_t)floor((double)(n + L - 1) / dN) * N;
        double v = 0.0;
        for (; q <= L - 1; q += N) {
            const int64_t u = (q < 0 ? -q : q) * (int64_t)K;
            const int64_t i = (int64_t)floor((double)u / dL);
            const int64_t rr = u - i * L;
            v += shape[i] + (shape[i + 1] - shape[i]) * ((double)rr / dL);
        }
        taps[d.off + n] = v;
        acc[0] += v;
    }
    block_sum<double, kFftThreads, 1>(acc, shd);
    if (threadIdx.x == 0) wsum[s] = acc[0];
}

// ------------------------------------------------------ transform modes --

// WINDOW: the forward transform of a sampled window's folded taps (FP64
// input), written out as the eigenvalue table of this step.
enum Mode { MODE_FORWARD = 0, MODE_STEP = 1, MODE_REMAINDER = 2, MODE_WINDOW = 3 };
__host__ __device__ constexpr bool fwd_mode(int m) { return m == MODE_FORWARD || m == MODE_WINDOW; }

// lambda_n = (H_n / H_0)^2 for bin n <= N/2 of the folded taps' transform H
// (real up to rounding for symmetric taps), lambda_0 = 1.  |H_n / H_0|
// below kWindowZero is an exact zero of the window spectrum: the FP64
// transform resolves it only to ~1e-15, and the size of such rounding noise
// would otherwise decide how the SD of later steps ends.
constexpr double kWindowZero = 1e-13;
__device__ __forceinline__ double window_lambda(int64_t n, double hx, double inv_sum)
{
    if (n == 0) return 1.0;
    const double h = hx * inv_sum;
    return fabs(h) < kWindowZero ? 0.0 : fmin(h * h, 1.0);
}

struct StepArgs {
    const SigDesc* sigs;
    const LenPlan* lens;
    const Work* work;
    SigState* st;
    const double* dtab;    // sine tables
    const double2* ctab;   // twiddle tables
    const int32_t* itab;   // storage position <-> bin maps
    double gamma;          // > 0: thresholded IMF
    double* chk;           // deferred FP64 check: 4 partial sums per pass-1 work item
    double* lam;           // sampled window shape: lambda_j per signal (at spec_off), else null
    double* wsum;          // sampled window shape: sum of each signal's taps
    double2* spec0;
    double2* spec1;
    double2* inter;
    RunState* parts;
    double* resid;         // FP64 residuals of signals counted by k_count_resid
    int t;                 // outer step (MODE_STEP)
    int max_imfs;
};

// Spectrum buffer index read by outer step t.
__device__ __forceinline__ double2* spec_in(const StepArgs& A, int buf) { return buf ? A.spec1 : A.spec0; }

// Read-only view of a stored spectrum (elements of type C) that hands out
// FP64 bins, for the searches.
template <typename C>
struct SpecView {
    const C* p;
    __device__ __forceinline__ double2 operator[](int64_t i) const { return to_d(p[i]); }
};
template <typename C>
__device__ __forceinline__ SpecView<C> spec_view(const double2* base, int64_t off)
{
    return SpecView<C>{reinterpret_cast<const C*>(base) + off};
}

// Element z_k of the inverse-transform input for k in [0, N): bin
// j = min(k, N-k) of the current residual spectrum (conjugated for k > N/2)
// times (g_j + i (1 - g_j)) / N.
__device__ __forceinline__ double2 step_input(double2 v, bool mirror, double g, double invN)
{
    const double h = 1.0 - g;
    if (mirror) v.y = -v.y;
    return make_double2((g * v.x - h * v.y) * invN, (g * v.y + h * v.x) * invN);
}

// -------------------------------------------------- single LDS pass (N <= cap)

// One workgroup per signal.  FORWARD: real input -> half spectrum (buffer 0)
// and nothing else.  STEP: apply, inverse transform, IMF row t, run summary,
// min and max of the residual, next spectrum.  REMAINDER: inverse transform
// of the final spectrum, imaginary part only.
// C: element type of the transform and of the stored spectra (double2;
// float2 in the FP32 lane, whose lambda, powers and sums stay FP64).
template <int MODE, typename InT, typename OutT, typename C = double2>
__global__ __launch_bounds__(kFftThreads) void k_single(StepArgs A, const InT* __restrict__ x,
                                                        OutT* __restrict__ imfs, OutT* __restrict__ rem)
{
    extern __shared__ double2 lds_raw[];
    C* lds = reinterpret_cast<C*>(lds_raw);
    __shared__ RunState sh[kFftThreads / 64];
    __shared__ double shd[2 * (kFftThreads / 64)];
    const Work w = A.work[blockIdx.x];
    const SigDesc d = A.sigs[w.sig];
    const LenPlan& lp = A.lens[d.len_id];
    const int N = (int)d.N;
    const int nh = N / 2;
    SigState* S = A.st + w.sig;

    if (fwd_mode(MODE)) {
        if (MODE == MODE_WINDOW && !S->active) return;
        for (int k = threadIdx.x; k < N; k += kFftThreads) lds[k] = to_c<C>(make_double2((double)x[d.off + k], 0.0));
        __syncthreads();
        lds_fft<false, kFftCap>(lds, lp.f1, 1, A.ctab);
        if (MODE == MODE_WINDOW) {
            double* lt = A.lam + d.spec_off;
            const double inv = 1.0 / A.wsum[w.sig];
            for (int k = threadIdx.x; k <= nh; k += kFftThreads) lt[k] = window_lambda(k, lds[k].x, inv);
            return;
        }
        C* out = reinterpret_cast<C*>(A.spec0) + d.spec_off;
        for (int k = threadIdx.x; k <= nh; k += kFftThreads) out[k] = lds[k];
        return;
    }
    if (MODE == MODE_REMAINDER && S->status != 0) {
        for (int k = threadIdx.x; k < N; k += kFftThreads) rem[d.off + k] = (OutT)x[d.off + k];
        return;
    }
    if (MODE == MODE_STEP && !S->active) {
        OutT* row = imfs + (int64_t)A.max_imfs * d.off + (int64_t)A.t * N;
        for (int k = threadIdx.x; k < N; k += kFftThreads) row[k] = (OutT)0;
        return;
    }
    const int buf = (MODE == MODE_STEP) ? (A.t & 1) : S->final_buf;
    const C* Rin = reinterpret_cast<const C*>(spec_in(A, buf)) + d.spec_off;
    C* Rout = reinterpret_cast<C*>(spec_in(A, buf ^ 1)) + d.spec_off;
    const double invN = 1.0 / (double)N;
    const int64_t L = S->L, m = S->m;
    const Lam lw = make_lam(lp, A.dtab, L > 0 ? L : 1, A.lam ? A.lam + d.spec_off : nullptr);
    for (int j = threadIdx.x; j <= nh; j += kFftThreads) {
        const double2 v = to_d(Rin[j]);
        double g = 0.0;
        if (MODE == MODE_STEP) g = gain_th(gain_pow(lambda_at(j, lw), m), A.gamma);
        lds[j] = to_c<C>(step_input(v, false, g, invN));
        if (j != 0 && 2 * j != N) lds[N - j] = to_c<C>(step_input(v, true, g, invN));
        if (MODE == MODE_STEP) Rout[j] = to_c<C>(cscale(v, 1.0 - g));
    }
    __syncthreads();
    lds_fft<true, kFftCap>(lds, lp.f1, 1, A.ctab);
    if (MODE == MODE_REMAINDER) {
        for (int k = threadIdx.x; k < N; k += kFftThreads) rem[d.off + k] = (OutT)lds[k].y;
        return;
    }
    OutT* row = imfs + (int64_t)A.max_imfs * d.off + (int64_t)A.t * N;
    for (int k = threadIdx.x; k < N; k += kFftThreads) row[k] = (OutT)lds[k].x;
    const int chunk = (N + kFftThreads - 1) / kFftThreads;
    const int a = threadIdx.x * chunk, b = min(N, a + chunk);
    RunState r = run_empty();
    double mn = INFINITY, mx = -INFINITY;
    for (int i = a; i < b; ++i) {
        const double y = lds[i].y;
        run_push(r, y);
        mn = fmin(mn, y);
        mx = fmax(mx, y);
    }
    block_minmax<kFftThreads>(mn, mx, shd);
    r = block_run_reduce<kFftThreads>(r, sh);
    if (threadIdx.x == 0) {
        A.parts[d.part_off] = r;
        S->kmin = dkey(mn);
        S->kmax = dkey(mx);
    }
}

// ----------------------------------------------- four-step pass 1 (columns)

// Work tile = TC columns of the N2 x N1 view (element index c + N1 * r).
// Transforms each column over r (length N2), multiplies by the four-step
// twiddle of (r', c) and writes Y[r'][c] to the intermediate.
//
// Paired tiles (N1, N2, TC even): the tile holds h = TC/2 mirror units;
// unit u >= 1 is the column pair {u, N1-u} (slots s and s+h), unit 0 is
// {0, N1/2}.  Element (c, r) with r < N2/2 owns spectrum bin k = c + N1 r
// (every bin below N/2 exactly once); its mirror N - k lies in the same tile
// at (N1-c, N2-1-r) for c != 0 and at (0, N2-r) for c = 0; bin N/2 sits at
// (0, N2/2).  Each bin is then read once and its gain computed once.
// Otherwise tiles are TC consecutive columns and each element reads its bin.
__device__ __forceinline__ int pass1_col(const PlanRegs& lp, int tile, int s)
{
    if (!lp.paired) return tile * lp.TC + s;
    const int h = lp.TC >> 1;
    const int u = tile * h + (s < h ? s : s - h);
    if (s < h) return u;
    return u == 0 ? (lp.N1 >> 1) : lp.N1 - u;
}
__device__ __forceinline__ int pass1_col(const LenPlan& lp, int tile, int s)
{
    return pass1_col(plan_regs(lp), tile, s);
}

// Storage order of the half spectrum (bins 0..N/2).  Two-pass paired plans
// keep it in pass-1 tile order so that pass 1 reads and writes one
// contiguous run per tile: the bins owned by tile t (c + N1*r for its TC
// columns c, slot s, and r < N2/2) sit at t*TC*N2/2 + r*TC + s; bin N/2 stays
// last.  Other plans use bin order.
__device__ __forceinline__ int64_t spec_pos(const LenPlan& lp, int64_t j)
{
    if (!lp.spec_perm) return j;
    const int nh = (int)(lp.N / 2);
    if (j == nh) return nh;
    const int N1 = lp.N1, h = lp.TC >> 1;
    const int r = (int)j / N1, c = (int)j - r * N1;
    int u, s0;
    if (2 * c < N1) {
        u = c;
        s0 = 0;
    } else {
        u = (2 * c == N1) ? 0 : N1 - c;
        s0 = h;
    }
    const int t = u / h;
    return (int64_t)t * (lp.TC * (lp.N2 >> 1)) + (int64_t)r * lp.TC + s0 + (u - t * h);
}

// Bin stored at position p (inverse of spec_pos).
__device__ __forceinline__ int64_t spec_bin(const LenPlan& lp, int64_t p)
{
    if (!lp.spec_perm) return p;
    const int nh = (int)(lp.N / 2);
    if (p == nh) return nh;
    const int owners = lp.TC * (lp.N2 >> 1);
    const int t = (int)p / owners;
    const int f = (int)p - t * owners;
    const int r = f / lp.TC, s = f - r * lp.TC;
    return pass1_col(lp, t, s) + (int64_t)lp.N1 * r;
}

// spec_pos by reciprocal division, exact for j < 2^22 (fdivmod's one-step
// correction), for the one-workgroup scan (j <= 32768), which walks the bins
// in order: the per-bin sine tables are then read coalesced and the
// spectrum in runs of TC/2 bins.
// Copies of the plan fields it needs (kept in registers inside bin loops).
struct SpecMap {
    FastDiv n1, h;
    int perm, nh, N1, hh, TC, owners;
};
__device__ __forceinline__ SpecMap make_specmap(const LenPlan& lp)
{
    SpecMap m;
    m.perm = lp.spec_perm;
    m.nh = (int)(lp.N / 2);
    m.N1 = lp.N1;
    m.hh = lp.TC >> 1;
    m.TC = lp.TC;
    m.owners = lp.TC * (lp.N2 >> 1);
    m.n1 = fastdiv(m.perm ? m.N1 : 1);
    m.h = fastdiv(m.perm ? m.hh : 1);
    return m;
}
__device__ __forceinline__ int pos_small(const SpecMap& m, int j)
{
    if (!m.perm || j == m.nh) return j;
    int c;
    const int r = fdivmod(j, m.n1, c);
    int u, s0;
    if (2 * c < m.N1) {
        u = c;
        s0 = 0;
    } else {
        u = (2 * c == m.N1) ? 0 : m.N1 - c;
        s0 = m.hh;
    }
    int ur;
    const int t = fdivmod(u, m.h, ur);
    return t * m.owners + r * m.TC + s0 + ur;
}

// Table forms: itab[bin_off + p] = bin at position p, itab[pos_off + j] =
// position of bin j (filled once per plan by k_fill_specmap).
__device__ __forceinline__ int64_t bin_at(const LenPlan& lp, const int32_t* __restrict__ itab, int64_t p)
{
    return lp.spec_perm ? (int64_t)itab[lp.bin_off + p] : p;
}
__device__ __forceinline__ int64_t pos_of(const LenPlan& lp, const int32_t* __restrict__ itab, int64_t j)
{
    return lp.spec_perm ? (int64_t)itab[lp.pos_off + j] : j;
}

__global__ void k_fill_specmap(const LenPlan* __restrict__ lpp, int32_t* __restrict__ itab)
{
    const LenPlan& lp = *lpp;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > lp.N / 2) return;
    const int64_t j = spec_bin(lp, p);
    itab[lp.bin_off + p] = (int32_t)j;
    itab[lp.pos_off + j] = (int32_t)p;
}

// The four-step intermediate is stored tile-major: pass-1 tile t writes its
// TC x N2 block (row r', slot s at t*TC*N2 + r'*TC + s) as one run; pass 2
// gathers, for its TR rows, a TR x TC run from every pass-1 tile.

// REDO: the pass that recomputes only the signals whose deferred check
// failed (its own instantiation, so profiles tell it apart).
// TILE: largest tile of the plan's lengths (kTileCap, or kTileCapBig when a
// length needs the wide tiles); it sizes the register staging and the LDS
// passes.
template <int MODE, typename InT, bool REDO = false, int TILE = kTileCap, bool P2 = false, typename C = double2>
__global__ __launch_bounds__(kFftThreads) void k_pass1(StepArgs A, const InT* __restrict__ x)
{
    extern __shared__ double2 lds_raw[];
    C* lds = reinterpret_cast<C*>(lds_raw);
    // the forward transforms gather the input in runs of TC/2 samples, so
    // neighbouring tiles read parts of the same cache lines: their workgroups
    // share an XCD (and its L2) there; the step passes keep the plain order
    const Work w = A.work[fwd_mode(MODE) ? xcd_item(blockIdx.x, gridDim.x) : blockIdx.x];
    const SigDesc d = A.sigs[w.sig];
    const LenPlan& lp = A.lens[d.len_id];
    const PlanRegs pr = plan_regs(lp);
    const int64_t N = d.N;
    const int N1 = lp.N1, N2 = lp.N2, TC = lp.TC;
    SigState* S = A.st + w.sig;
    if ((MODE == MODE_STEP || MODE == MODE_WINDOW) && !S->active) return;
    if (REDO && !S->redo) return;
    if (MODE == MODE_REMAINDER && S->status != 0) return;
    const int total = TC * N2;
    const FastDiv ftc = fastdiv(TC);
    if (fwd_mode(MODE)) {
        for (int f = threadIdx.x; f < total; f += kFftThreads) {
            int s;
            const int r = fdivmod(f, ftc, s);
            lds[f] = to_c<C>(make_double2((double)x[d.off + pass1_col(pr, w.tile, s) + (int64_t)N1 * r], 0.0));
        }
    } else {
        const int buf = (MODE == MODE_STEP) ? (A.t & 1) : S->final_buf;
        const C* Rin = reinterpret_cast<const C*>(spec_in(A, buf)) + d.spec_off;
        C* Rout = reinterpret_cast<C*>(spec_in(A, buf ^ 1)) + d.spec_off;
        const double invN = 1.0 / (double)N;
        const int64_t L = S->L, m = S->m;
        const Lam lw = make_lam(lp, A.dtab, L > 0 ? L : 1, A.lam ? A.lam + d.spec_off : nullptr);
        if (lp.paired) {
            const int h = TC >> 1;
            const int owners = TC * (N2 >> 1);
            // the tile's bins are one contiguous run (tile order, see
            // spec_pos); all of a thread's loads are issued first
            constexpr int PQ = TILE / 2 / kFftThreads + 1;
            C vv[PQ];
            // deferred FP64 check of m: this tile's part of the stop-test sums,
            // over the bins above the scan's noise floor
            const bool chk = MODE == MODE_STEP && S->chk;
            const double qthr = chk ? S->qthr : 0.0;
            double cs[4] = {0.0, 0.0, 0.0, 0.0};
            const int64_t pbase = (int64_t)w.tile * owners;
#pragma unroll
            for (int q = 0; q < PQ; ++q) {
                const int f = threadIdx.x + q * kFftThreads;
                vv[q] = czero<C>();
                if (f < owners)
                    vv[q] = Rin[pbase + f];
                else if (f == owners && w.tile == 0)
                    vv[q] = Rin[N >> 1];
            }
#pragma unroll
            for (int q = 0; q < PQ; ++q) {
                const int f = threadIdx.x + q * kFftThreads;
                if (f > owners || (f == owners && w.tile != 0)) break;
                int s, r;
                if (f < owners) {
                    r = fdivmod(f, ftc, s);
                } else {
                    s = 0;          // bin N/2 at (0, N2/2)
                    r = N2 >> 1;
                }
                const int c = pass1_col(pr, w.tile, s);
                const int k = c + N1 * r;      // N <= 2^26: bin indices fit in 32 bits
                const int64_t pk = (f < owners) ? pbase + f : (N >> 1);
                const double2 v = to_d(vv[q]);
                double g = 0.0;
                if (MODE == MODE_STEP) {
                    // (1-lambda)^m built from (1-lambda)^(m-2) so that the
                    // deferred check gets mu^(m-1) and mu^(m-2) on the way
                    const double lam = lambda_at(k, lw);
                    double y, z;
                    if (lam >= 1.0) {
                        y = (m == 1) ? 1.0 : 0.0;
                        z = (m == 2) ? 1.0 : 0.0;
                        g = 0.0;
                    } else {
                        const double om = 1.0 - lam;
                        z = (m >= 2) ? ((m == 2) ? 1.0 : gain_pow(lam, m - 2)) : 0.0;
                        y = (m >= 2) ? z * om : 1.0;
                        g = y * om;
                    }
                    if (chk && v.x * v.x + v.y * v.y >= qthr) {
                        const double P = ((k == 0 || 2 * k == N) ? 1.0 : 2.0) * (v.x * v.x + v.y * v.y);
                        const double l2 = lam * lam;
                        cs[0] += P * l2 * y * y;
                        cs[1] += P * y * y;
                        cs[2] += P * l2 * z * z;
                        cs[3] += P * z * z;
                    }
                    g = gain_th(g, A.gamma);
                }
                lds[r * TC + s] = to_c<C>(step_input(v, false, g, invN));
                if (f < owners) {
                    int ms, mr;
                    if (c == 0) {
                        ms = s;
                        mr = (N2 - r) % N2;
                    } else {
                        ms = (s == h && w.tile == 0) ? s : (s < h ? s + h : s - h);
                        mr = N2 - 1 - r;
                    }
                    if (!(c == 0 && r == 0)) lds[mr * TC + ms] = to_c<C>(step_input(v, true, g, invN));
                }
                if (MODE == MODE_STEP) Rout[pk] = to_c<C>(cscale(v, 1.0 - g));
            }
            if (chk) {
                __shared__ double shc[4 * (kFftThreads / 64)];
                block_sum<double, kFftThreads, 4>(cs, shc);
                if (threadIdx.x < 4) {
                    const double cv = threadIdx.x == 0 ? cs[0] : threadIdx.x == 1 ? cs[1] : threadIdx.x == 2 ? cs[2] : cs[3];
                    A.chk[((int64_t)d.p1_off + w.tile) * 4 + threadIdx.x] = cv;
                }
            }
        } else {
            const int64_t nh = N / 2;
            // deferred FP64 check as in the paired tiles, each bin counted at
            // its own element (k <= N/2), not at its mirror
            const bool chk = MODE == MODE_STEP && S->chk;
            const double qthr = chk ? S->qthr : 0.0;
            double cs[4] = {0.0, 0.0, 0.0, 0.0};
            for (int f = threadIdx.x; f < total; f += kFftThreads) {
                int s;
                const int r = fdivmod(f, ftc, s);
                const int k = pass1_col(pr, w.tile, s) + N1 * r;   // N <= 2^26
                const bool mirror = k > nh;
                const int j = mirror ? (int)N - k : k;
                const double2 v = to_d(Rin[j]);
                double g = 0.0;
                if (MODE == MODE_STEP) {
                    const double lam = lambda_at(j, lw);
                    if (chk) {
                        // (1-lambda)^m from (1-lambda)^(m-2), as in the paired tiles
                        double y, z;
                        if (lam >= 1.0) {
                            y = (m == 1) ? 1.0 : 0.0;
                            z = (m == 2) ? 1.0 : 0.0;
                            g = 0.0;
                        } else {
                            const double om = 1.0 - lam;
                            z = (m >= 2) ? ((m == 2) ? 1.0 : gain_pow(lam, m - 2)) : 0.0;
                            y = (m >= 2) ? z * om : 1.0;
                            g = y * om;
                        }
                        if (!mirror && v.x * v.x + v.y * v.y >= qthr) {
                            const double P = ((j == 0 || 2 * j == N) ? 1.0 : 2.0) * (v.x * v.x + v.y * v.y);
                            const double l2 = lam * lam;
                            cs[0] += P * l2 * y * y;
                            cs[1] += P * y * y;
                            cs[2] += P * l2 * z * z;
                            cs[3] += P * z * z;
                        }
                    } else {
                        g = gain_pow(lam, m);
                    }
                    g = gain_th(g, A.gamma);
                }
                lds[f] = to_c<C>(step_input(v, mirror, g, invN));
                if (MODE == MODE_STEP && !mirror) Rout[j] = to_c<C>(cscale(v, 1.0 - g));
            }
            if (chk) {
                __shared__ double shu[4 * (kFftThreads / 64)];
                block_sum<double, kFftThreads, 4>(cs, shu);
                if (threadIdx.x < 4) {
                    const double cv = threadIdx.x == 0 ? cs[0] : threadIdx.x == 1 ? cs[1] : threadIdx.x == 2 ? cs[2] : cs[3];
                    A.chk[((int64_t)d.p1_off + w.tile) * 4 + threadIdx.x] = cv;
                }
            }
        }
    }
    __syncthreads();
    if (fwd_mode(MODE))
        lds_fft<false, TILE, P2>(lds, lp.f1, TC, A.ctab);
    else
        lds_fft<true, TILE, P2>(lds, lp.f1, TC, A.ctab);
    C* Y = reinterpret_cast<C*>(A.inter) + d.inter_off;
    for (int f = threadIdx.x; f < total; f += kFftThreads) {
        int s;
        const int rp = fdivmod(f, ftc, s);
        const int c = pass1_col(pr, w.tile, s);
        const int64_t a = (int64_t)rp * c;
        C v = lds[f];
        if (a != 0) {
            const double2 tw = fwd_mode(MODE) ? big_twiddle<false>(pr, A.ctab, a)
                                              : big_twiddle<true>(pr, A.ctab, a);
            v = cmul(v, to_c<C>(tw));
        }
        Y[(int64_t)w.tile * total + f] = v;
    }
}

// -------------------------------------------------- four-step pass 2 (rows)

// One pass-2 work item: its signal, plan fields and rows.
struct P2Item {
    Work w;
    SigDesc d;
    const LenPlan* lp;
    PlanRegs pr;
    int N1, N2, TR, TC, r0, total;
    SigState* S;
};
__device__ __forceinline__ P2Item p2_item(const StepArgs& A, int item)
{
    P2Item t;
    t.w = A.work[item];
    t.d = A.sigs[t.w.sig];
    t.lp = A.lens + t.d.len_id;
    t.pr = plan_regs(*t.lp);
    t.N1 = t.lp->N1;
    t.N2 = t.lp->N2;
    t.TR = t.lp->TR;
    t.TC = t.lp->TC;
    t.r0 = t.w.tile * t.TR;
    t.total = t.TR * t.N1;
    t.S = A.st + t.w.sig;
    return t;
}

// The item's TR x N1 block of the intermediate into registers.  Element
// e = (t * TC + s) * TR + rl: consecutive lanes take consecutive rows of one
// column, so the LDS stores of p2_stage are conflict free; the global reads
// stay within the TR x TC run of pass-1 tile t.
template <int TILE, typename C>
__device__ __forceinline__ void p2_gather(const StepArgs& A, const P2Item& t, C (&yv)[TILE / kFftThreads])
{
    const C* Y = reinterpret_cast<const C*>(A.inter) + t.d.inter_off;
    const FastDiv ftr = fastdiv(t.TR), ftc = fastdiv(t.TC);
    const int64_t blk = (int64_t)t.TC * t.N2;
#pragma unroll
    for (int q = 0; q < TILE / kFftThreads; ++q) {
        const int e = threadIdx.x + q * kFftThreads;
        yv[q] = czero<C>();
        if (e < t.total) {
            int s, rl;
            const int u = fdivmod(e, ftr, rl);
            const int tt = fdivmod(u, ftc, s);
            yv[q] = Y[(int64_t)tt * blk + (int64_t)(t.r0 + rl) * t.TC + s];
        }
    }
}
template <int TILE, typename C>
__device__ __forceinline__ void p2_stage(const P2Item& t, const C (&yv)[TILE / kFftThreads], C* lds)
{
    const FastDiv ftr = fastdiv(t.TR), ftc = fastdiv(t.TC);
#pragma unroll
    for (int q = 0; q < TILE / kFftThreads; ++q) {
        const int e = threadIdx.x + q * kFftThreads;
        if (e < t.total) {
            int s, rl;
            const int u = fdivmod(e, ftr, rl);
            const int tt = fdivmod(u, ftc, s);
            lds[pass1_col(t.pr, tt, s) * t.TR + rl] = yv[q];
        }
    }
}

// Outer step, inactive signal: its rows of IMF t are zero.
template <typename OutT>
__device__ __forceinline__ void p2_zero(const StepArgs& A, const P2Item& t, OutT* __restrict__ imfs)
{
    OutT* row = imfs + (int64_t)A.max_imfs * t.d.off + (int64_t)A.t * t.d.N;
    const FastDiv ftr = fastdiv(t.TR);
    for (int f = threadIdx.x; f < t.total; f += kFftThreads) {
        int rl;
        const int cp = fdivmod(f, ftr, rl);
        row[(int64_t)t.N2 * cp + t.r0 + rl] = (OutT)0;
    }
}

// Outer step, after the row transforms: the IMF rows out of the real parts,
// the residual (imaginary parts) counted: one run summary per column c' (TR
// consecutive samples) and the tile's min and max; thin row tiles hand the
// residual to k_count_resid instead.
template <int TILE, typename OutT, typename C>
__device__ __forceinline__ void p2_step_out(const StepArgs& A, const P2Item& t, OutT* __restrict__ imfs, C* lds,
                                            double* shd)
{
    const int TR = t.TR, N1 = t.N1, N2 = t.N2, r0 = t.r0, total = t.total;
    const FastDiv ftr = fastdiv(TR);
    OutT* row = imfs + (int64_t)A.max_imfs * t.d.off + (int64_t)A.t * t.d.N;
    constexpr int EQ = TILE / kFftThreads;
    double yv[EQ];
#pragma unroll
    for (int q = 0; q < EQ; ++q) {
        const int f = threadIdx.x + q * kFftThreads;
        yv[q] = 0.0;
        if (f < total) {
            int rl;
            const int cp = fdivmod(f, ftr, rl);
            const C v = lds[f];
            row[(int64_t)N2 * cp + r0 + rl] = (OutT)v.x;
            yv[q] = v.y;
        }
    }
    if (t.d.resid_off >= 0) {
        double* y = A.resid + t.d.resid_off;
#pragma unroll
        for (int q = 0; q < EQ; ++q) {
            const int f = threadIdx.x + q * kFftThreads;
            if (f < total) {
                int rl;
                const int cp = fdivmod(f, ftr, rl);
                y[(int64_t)N2 * cp + r0 + rl] = yv[q];
            }
        }
        return;
    }
    // the residual again in LDS, column cp at stride TR + 1 so that the
    // per-column reads below fall in different banks
    __syncthreads();
    double* yp = reinterpret_cast<double*>(lds);
#pragma unroll
    for (int q = 0; q < EQ; ++q) {
        const int f = threadIdx.x + q * kFftThreads;
        if (f < total) {
            int rl;
            const int cp = fdivmod(f, ftr, rl);
            yp[cp * (TR + 1) + rl] = yv[q];
        }
    }
    __syncthreads();
    const int runs_per_row = N2 / TR;
    double mn = INFINITY, mx = -INFINITY;
    for (int cp = threadIdx.x; cp < N1; cp += kFftThreads) {
        RunState r = run_empty();
        for (int rl = 0; rl < TR; ++rl) {
            const double y = yp[cp * (TR + 1) + rl];
            run_push(r, y);
            mn = fmin(mn, y);
            mx = fmax(mx, y);
        }
        A.parts[t.d.part_off + cp * runs_per_row + t.w.tile] = r;
    }
    block_minmax<kFftThreads>(mn, mx, shd);
    if (threadIdx.x == 0) {
        atomicMin(&t.S->kmin, dkey(mn));
        atomicMax(&t.S->kmax, dkey(mx));
    }
}

// Work tile = TR consecutive rows r' of Y.  Transforms each row over c
// (length N1); output element N2 * c' + r'.  STEP: IMF, one run summary per
// c' (TR consecutive samples) and the tile's min/max; FORWARD: half
// spectrum; REMAINDER: y.
template <int MODE, typename InT, typename OutT, int TILE = kTileCap, bool P2 = false, typename C = double2>
__global__ __launch_bounds__(kFftThreads) void k_pass2(StepArgs A, const InT* __restrict__ x,
                                                       OutT* __restrict__ imfs, OutT* __restrict__ rem)
{
    extern __shared__ double2 lds_raw[];
    C* lds = reinterpret_cast<C*>(lds_raw);
    __shared__ double shd[2 * (kFftThreads / 64)];
    const P2Item t = p2_item(A, xcd_item(blockIdx.x, gridDim.x));
    const SigDesc& d = t.d;
    const LenPlan& lp = *t.lp;
    const int64_t N = d.N;
    const int N2 = t.N2, r0 = t.r0, total = t.total;
    SigState* S = t.S;
    const FastDiv ftr = fastdiv(t.TR);
    if (MODE == MODE_WINDOW && !S->active) return;
    if (MODE == MODE_STEP && t.w.tile == 0 && threadIdx.x == 0) S->redo = 0;   // the step is final now
    if (MODE == MODE_STEP && !S->active) {
        p2_zero(A, t, imfs);
        return;
    }
    if (MODE == MODE_REMAINDER && S->status != 0) {
        for (int f = threadIdx.x; f < total; f += kFftThreads) {
            int rl;
            const int cp = fdivmod(f, ftr, rl);
            const int64_t n = (int64_t)N2 * cp + r0 + rl;
            rem[d.off + n] = (OutT)x[d.off + n];
        }
        return;
    }
    {
        C yv[TILE / kFftThreads];
        p2_gather<TILE>(A, t, yv);
        p2_stage<TILE>(t, yv, lds);
    }
    __syncthreads();
    if (fwd_mode(MODE))
        lds_fft<false, TILE, P2>(lds, lp.f2, t.TR, A.ctab);
    else
        lds_fft<true, TILE, P2>(lds, lp.f2, t.TR, A.ctab);
    if (MODE == MODE_WINDOW) {
        double* lt = A.lam + d.spec_off;
        const double inv = 1.0 / A.wsum[t.w.sig];
        const int64_t nh = N / 2;
        for (int f = threadIdx.x; f < total; f += kFftThreads) {
            int rl;
            const int cp = fdivmod(f, ftr, rl);
            const int64_t n = (int64_t)N2 * cp + r0 + rl;
            if (n <= nh) lt[n] = window_lambda(n, lds[f].x, inv);
        }
        return;
    }
    if (MODE == MODE_FORWARD) {
        C* out = reinterpret_cast<C*>(A.spec0) + d.spec_off;
        const int64_t nh = N / 2;
        for (int f = threadIdx.x; f < total; f += kFftThreads) {
            int rl;
            const int cp = fdivmod(f, ftr, rl);
            const int64_t n = (int64_t)N2 * cp + r0 + rl;
            if (n <= nh) out[spec_pos(lp, n)] = lds[f];
        }
        return;
    }
    if (MODE == MODE_REMAINDER) {
        for (int f = threadIdx.x; f < total; f += kFftThreads) {
            int rl;
            const int cp = fdivmod(f, ftr, rl);
            rem[d.off + (int64_t)N2 * cp + r0 + rl] = (OutT)lds[f].y;
        }
        return;
    }
    p2_step_out<TILE>(A, t, imfs, lds, shd);
}

// ------------------------------------------------------------------- scan --

struct ScanArgs {
    const SigDesc* sigs;
    const LenPlan* lens;
    const int32_t* list;      // signal handled by each workgroup
    SigState* st;
    const RunState* parts;
    const double* psum;       // per-tile sums of the input (first step)
    const double* dtab;
    const int32_t* itab;      // storage position <-> bin maps
    const double2* spec0;
    const double2* spec1;
    float* gscr;              // FP32 scratch of the multi-workgroup scan (SigDesc::gs_off)
    BigScan* bigs;            // multi-workgroup scan states (SigDesc::bs)
    double* bpart;            // per-tile partial sums, 2*kBigCand per tile (SigDesc::bt_off)
    double* bqmax;            // per-tile largest |R_j|^2 of the multi-workgroup scan
    fif_imf_info* info;       // [B][max_imfs] or null
    const int64_t* prop;      // proposed m per signal (0: none), or null
    int t;
    int max_imfs;
    double delta;
    int mask_rule;
    double nu;
    int64_t max_inner;
    double floor_tau;
    int stop_mode;            // 0 SD, 1 absolute step norm, 2 a-priori N0
    double* chk;              // deferred FP64 check partials (StepArgs::chk)
    const double* lam;        // sampled window shape: lambda_j per signal (StepArgs::lam)
    int defer;                // 1: leave the FP64 check of paired four-step signals to pass 1
    int redo_only;            // 1: only signals whose deferred check failed
    int mt_shift;             // test hook: added to the deferred FP32 estimate
};

__device__ __forceinline__ int64_t mask_length(int64_t N, int64_t k, int rule, double nu, int64_t fpeak)
{
    if (rule == 0) return (2 * N + k - 1) / k;
    if (rule == 2) return (N + fpeak - 1) / fpeak;
    const int64_t L = 2 * (int64_t)floor(nu * (double)N / (double)k);
    return L < 1 ? 1 : L;
}

// Start of an outer step for one signal (whole workgroup): combine the run
// summaries of the residual in sample order (extrema count; min/max come from
// the atomics), apply the rounding floor and k < 2 stop rules, fix L and the
// per-step power scale.  Leaves L (or -1 when the signal stops) in sh_i[0]
// and the scale in sh_d[0] for every thread.
template <int T>
__device__ __forceinline__ void scan_prologue(const ScanArgs& A, int s, const SigDesc& d, SigState* S,
                                              RunState* shr, int64_t* sh_i, double* sh_d)
{
    const int tid = threadIdx.x;
    const int64_t N = d.N;
    // ---- combine run summaries of the residual (sample order) ----
    {
        const int n = (A.t == 0) ? d.n_init_parts : d.n_parts;
        const RunState* P = A.parts + d.part_off;
        const int chunk = (n + T - 1) / T;
        const int a = tid * chunk, b = min(n, a + chunk);
        RunState r = run_empty();
        for (int i = a; i < b; ++i) r = run_combine(r, run_load(P + i));
        r = block_run_reduce<T>(r, shr);
        if (tid == 0) {
            const double mn = dval(S->kmin), mx = dval(S->kmax);
            S->kmin = dkey(INFINITY);
            S->kmax = dkey(-INFINITY);
            int stop = -1;
            if (A.t == 0) {
                double sum = 0.0;
                for (int i = 0; i < d.n_init_parts; ++i) sum += A.psum[d.part_off + i];
                if (r.nonfinite || !isfinite(sum)) {
                    S->status = FIF_ERR_NONFINITE;
                    stop = FIF_STOP_FAILED;
                } else {
                    S->mean = sum / (double)N;
                    S->maxabs = fmax(fabs(mn), fabs(mx));
                }
            }
            // power-of-two scale of this residual's power spectrum: |R_j| <=
            // N max|r|, so the scaled FP32 powers stay below 2 and late, small
            // residuals do not underflow
            {
                const double top = (double)N * fmax(fabs(mn), fabs(mx));
                S->pscale = (top > 0.0 && isfinite(top)) ? ldexp(1.0, -2 * (ilogb(top) + 1)) : 1.0;
            }
            if (stop < 0) {
                const double dev = fmax(mx - S->mean, S->mean - mn);
                if (dev <= A.floor_tau * S->maxabs)
                    stop = FIF_STOP_FLOOR;
                else if (r.cnt < 2)
                    stop = FIF_STOP_FEW_EXTREMA;
            }
            if (stop >= 0) {
                S->active = 0;
                S->stop_reason = stop;
                S->n_imfs = A.t;
                S->final_buf = A.t & 1;
                sh_i[0] = -1;
            } else {
                S->k = r.cnt;
                sh_i[0] = mask_length(N, r.cnt, A.mask_rule, A.nu, S->fpeak);
            }
            sh_d[0] = S->pscale;
        }
        __syncthreads();
    }
}

// Spectral-peak bin of every active signal s0 + b (mask rule 2): the highest
// bin f in [1, N/2] with |R_f|^2 >= rho max_{1<=j<=N/2} |R_j|^2, or 1 when
// those bins are all zero.  Storage positions 1..N/2 hold bins 1..N/2.
template <typename C = double2>
__global__ __launch_bounds__(256) void k_peak(ScanArgs A, int s0, double rho)
{
    __shared__ double shd[2 * 4];
    const int s = s0 + blockIdx.x;
    SigState* S = A.st + s;
    if (!S->active) return;
    const SigDesc d = A.sigs[s];
    const LenPlan& lp = A.lens[d.len_id];
    const int32_t* btab = lp.spec_perm ? A.itab + lp.bin_off : nullptr;
    const auto R = spec_view<C>((A.t & 1) ? A.spec1 : A.spec0, d.spec_off);
    const int64_t nh = d.N / 2;
    double mn = INFINITY, mx = 0.0;
    for (int64_t p = 1 + threadIdx.x; p <= nh; p += 256) {
        const double2 z = R[p];
        mx = fmax(mx, z.x * z.x + z.y * z.y);
    }
    block_minmax<256>(mn, mx, shd);
    const double thr = rho * mx;
    double best = 0.0;
    mn = INFINITY;
    for (int64_t p = 1 + threadIdx.x; p <= nh; p += 256) {
        const double2 z = R[p];
        if (z.x * z.x + z.y * z.y >= thr) best = fmax(best, (double)(btab ? (int64_t)btab[p] : p));
    }
    block_minmax<256>(mn, best, shd);
    if (threadIdx.x == 0) S->fpeak = (mx > 0.0 && best >= 1.0) ? (int64_t)best : 1;
}

// The start of an outer step alone, for the proposal path: the network needs
// L before the search for m starts.
template <int T>
__global__ __launch_bounds__(T) void k_scan_prologue(ScanArgs A)
{
    __shared__ RunState shr[T / 64];
    __shared__ int64_t sh_i[2];
    __shared__ double sh_d[1];
    const int s = A.list[blockIdx.x];
    const SigDesc d = A.sigs[s];
    SigState* S = A.st + s;
    if (!S->active) return;
    scan_prologue<T>(A, s, d, S, shr, sh_i, sh_d);
    if (threadIdx.x == 0 && sh_i[0] >= 0) S->L = sh_i[0];
}

// Theorem 5: the smallest N0 >= 1 with N0^N0 / (N0+1)^(N0+1) <
// delta / (||U^T r||_inf sqrt(N - 1 - k)), U the unitary DFT (||U^T r||_inf =
// max_j |R_j| / sqrt(N), mzb = max_j |R_j|^2 over every bin), k = gcd(L, N) - 1
// the number of exact zero eigenvalues; compared in logarithms.  For every
// m >= N0, ||s_{m+1} - s_m|| < delta (inequality "N0_discrete").
__device__ __forceinline__ int64_t apriori_n0(double mzb, int64_t L, int64_t N, double delta)
{
    int64_t ga = L, gb = N;
    while (gb) {
        const int64_t r = ga % gb;
        ga = gb;
        gb = r;
    }
    const int64_t rest = N - 1 - (ga - 1);
    const double st_inf = sqrt(mzb / (double)N);
    if (!(st_inf > 0.0) || rest <= 0) return 1;
    const double rhs = log(delta / (st_inf * sqrt((double)rest)));
    auto lhs = [](int64_t n) { return (double)n * log((double)n) - (double)(n + 1) * log((double)(n + 1)); };
    int64_t hi2 = 1;
    while (lhs(hi2) >= rhs && hi2 < ((int64_t)1 << 50)) hi2 *= 2;
    int64_t lo2 = hi2 / 2;
    if (lo2 == 0) return 1;
    while (hi2 - lo2 > 1) {
        const int64_t mid = (lo2 + hi2) / 2;
        if (lhs(mid) < rhs)
            hi2 = mid;
        else
            lo2 = mid;
    }
    return hi2;
}

// Probes of the bracketing phase: m = 1, 2, 4, 16, ..., 4^10.
constexpr int kGeo = 12;
__device__ __forceinline__ int64_t geo_m(int q) { return q == 0 ? 1 : q == 1 ? 2 : ((int64_t)1 << (2 * (q - 1))); }

// One workgroup per signal with at most kScanBins bins, T = kScanBins / BPT
// threads: thread-owned bins j = 1 + tid + i*T (i < BPT) keep log2(mu) and the
// power in registers, power*lambda^2 in LDS.  PRE: k_scan_prologue already ran
// (L and the power scale are in the signal state).  SMODE: the stop mode (a
// compile-time copy of ScanArgs::stop_mode, so the default kernel carries no
// other mode's work).  DEF: the kernel for lists of four-step signals whose
// FP64 check (stop mode 0) is deferred to pass 1 -- the FP32 search only.
// RDO: the redo of the signals whose deferred estimate pass 1 rejected -- the
// FP64 search only, from that estimate (no FP32 state: no dynamic LDS).
template <int BPT, bool PRE, int SMODE, typename C = double2, bool DEF = false, bool RDO = false>
__global__ __launch_bounds__(kScanBins / BPT) void k_scan(ScanArgs A)
{
    static_assert(!DEF || SMODE == 0, "only stop mode 0 defers its check");
    static_assert(!RDO || (PRE && SMODE == 0 && !DEF), "the redo follows a deferred stop-mode-0 check");
    constexpr int T = kScanBins / BPT;
    constexpr int NR = BPT;
    __shared__ RunState shr[T / 64];
    __shared__ double shd[4 * (T / 64)];
    __shared__ float shf[2 * kGeo * (T / 64)];
    __shared__ int64_t sh_i[2];
    __shared__ double sh_d[1];

    const int s = A.list[blockIdx.x];
    const SigDesc d = A.sigs[s];
    SigState* S = A.st + s;
    if (!S->active) return;
    if (A.redo_only && !S->redo) return;
    const LenPlan& lp = A.lens[d.len_id];
    // the DEF kernel is launched in place of the general one when every
    // signal of the list is a four-step signal and stop mode 0 defers
    const bool deferred = DEF || (SMODE == 0 && A.defer && !A.redo_only && lp.two_pass);
    if (DEF && !lp.two_pass) return;
    const int64_t N = d.N;
    const int tid = threadIdx.x;

    // ---- combine run summaries, stop rules, mask length, power scale ----
    if (!PRE) {
        scan_prologue<T>(A, s, d, S, shr, sh_i, sh_d);
    } else if (tid == 0) {
        sh_i[0] = S->L;
        sh_d[0] = S->pscale;
    }
    if (PRE) __syncthreads();
    const int64_t L = sh_i[0];
    if (L < 0) return;

    const int nh = (int)(N / 2);
    const Lam lw = make_lam(lp, A.dtab, L, A.lam ? A.lam + d.spec_off : nullptr);
    const auto R = spec_view<C>((A.t & 1) ? A.spec1 : A.spec0, d.spec_off);
    const double pscale = sh_d[0];
    const double delta = A.delta;
    const float d2f = (float)(delta * delta);
    const float lnd2 = logf(d2f);
    const int64_t cap = A.max_inner;
    uint32_t n32 = 0, n64 = 0;
    // stop mode 1: ||s_{m+1} - s_m||^2 = sum_j P_j lambda_j^2 mu_j^m / (N pscale)
    constexpr bool absm = SMODE == 1;
    const double inv_np = 1.0 / ((double)N * pscale);
    const float lnthr_abs = (float)log(delta * delta * (double)N * pscale);
    auto ok = [&](double sd) { return SMODE != 0 ? sd < delta : sd <= delta; };
    double mz = 0.0;          // largest |R_j|^2, j >= 1
    const SpecMap smap = make_specmap(lp);
    auto weight = [&](int j) -> double { return (2 * (int64_t)j == N) ? 1.0 : 2.0; };

    const double P0 = (R[0].x * R[0].x + R[0].y * R[0].y) * pscale;
    int64_t mt = 0;
    uint32_t flags = 0;
    if constexpr (RDO) {
        // the redo after a rejected deferred estimate: the FP64 search
        // below starts from that estimate (the FP32 search would only
        // find it again)
        mt = S->m;
    } else {
        // ---- first sweep: FP32 copies of the weighted power b, power*lambda^2
        //      a, and tau = log2 mu, mu = (1 - lambda)^2 (DC kept aside since
        //      lambda_0 = 1 contributes to m = 1 only) ----
        float tau_r[NR], b_r[NR];
        extern __shared__ float lds_a[];
        // v: spectrum of bin jb; lambda in FP32 (this search only brackets m)
        const float invNf = 1.f / (float)N, invLf = 1.f / (float)L;
        auto sweep_bin = [&](double2 v, int64_t jb, float& tau, float& av, float& bv) {
            const double P = weight(jb) * (v.x * v.x + v.y * v.y) * pscale;
            const float lf = lambda_f32(jb, lw, invNf, invLf);
            bv = (float)P;
            av = bv * lf * lf;
            tau = 2.8853900817779268f * log1pf(-lf);  // 2 log2(1 - lambda)
        };
        // bins in groups of SG: the group's loads are issued together (memory
        // parallelism), the FP64 work of different groups is kept apart
        // (register pressure).
        constexpr int SG = DEF ? 4 : 8;
        static_assert(NR % SG == 0, "sweep groups");
#pragma unroll
        for (int i0 = 0; i0 < NR; i0 += SG) {
            double2 v[SG];
            int64_t jb[SG];
#pragma unroll
            for (int g = 0; g < SG; ++g) {
                const int j = 1 + tid + (i0 + g) * T;
                v[g] = make_double2(0.0, 0.0);
                jb[g] = 0;
                if (j <= nh) {
                    v[g] = R[pos_small(smap, j)];
                    jb[g] = j;
                }
            }
#pragma unroll
            for (int g = 0; g < SG; ++g) {
                const int i = i0 + g;
                const int j = 1 + tid + i * T;
                float av = 0.f;
                tau_r[i] = 0.f;
                b_r[i] = 0.f;
                if (j <= nh) {
                    sweep_bin(v[g], jb[g], tau_r[i], av, b_r[i]);
                    // after the group's loads were issued, not between them
                    mz = fmax(mz, v[g].x * v[g].x + v[g].y * v[g].y);
                }
                lds_a[i * T + tid] = av;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();

        // per-bin FP32 accumulation of a*x and b*x, x = mu^e = 2^(e tau)
        auto acc_bin = [&](float tau, float av, float bv, float e, float& sa, float& sb) {
            const float xx = __builtin_amdgcn_exp2f(e * tau);
            sa += av * xx;
            sb += bv * xx;
        };

        // f at an arbitrary m (one FP32 pass); m = 1 needs no power (and must not
        // form 0 * tau with tau = -inf for bins whose FP32 lambda rounds to 1)
        auto f32 = [&](int64_t m) -> float {
            float v[2] = {0.f, 0.f};
            const float e = (float)(absm ? m : m - 1);
            if (m == 1 && !absm) {
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    v[0] += lds_a[i * T + tid];
                    v[1] += b_r[i];
                }
            } else {
#pragma unroll
                for (int i = 0; i < NR; ++i) acc_bin(tau_r[i], lds_a[i * T + tid], b_r[i], e, v[0], v[1]);
            }
            if (m == 1 && !absm && tid == 0) {
                v[0] += (float)P0;
                v[1] += (float)P0;
            }
            block_sum<float, T, 2>(v, shf);
            n32 += 1;
            if (absm) return v[0] > 0.f ? (logf(v[0]) - lnthr_abs) : -INFINITY;
            return v[1] > 0.f ? (logf(v[0] / v[1]) - lnd2) : -INFINITY;
        };

        // ---- bracket by probing m = 1, 2, 4, 16, 64, ... (one FP32 pass each,
        //      stopping at the first that satisfies the test), then safeguarded
        //      regula falsi: smallest m <= cap with f(m) <= 0 (f is
        //      non-increasing in m)
        if (SMODE == 2) {
            double mn_unused = INFINITY, mzb = fmax(mz, P0 / pscale);
            block_minmax<T>(mn_unused, mzb, shd);
            const int64_t n0 = apriori_n0(mzb, L, N, delta);
            mt = n0;
            if (mt > cap) {
                mt = cap;
                flags |= FIF_IMF_CAP;
            }
        } else {
            int64_t lo = 0, hi = -1;
            float flo = INFINITY, fhi = 0.f;
            const int64_t mp = A.prop ? A.prop[s] : 0;
            int64_t top = cap;        // largest count the FP32 search considers
            if (mp > 0) {
                // bracket from the proposal: probe it, then walk away from it
                // in steps growing fourfold from mp/16 until f changes sign
                int64_t c = min(mp, cap);
                int64_t step = max((int64_t)1, c >> 4);
                float fc = f32(c);
                if (fc <= 0.f) {
                    hi = c;
                    fhi = fc;
                    while (hi > 1) {
                        c = max((int64_t)1, hi - step);
                        fc = f32(c);
                        if (fc > 0.f) {
                            lo = c;
                            flo = fc;
                            break;
                        }
                        hi = c;
                        fhi = fc;
                        step *= 4;
                    }
                } else {
                    lo = c;
                    flo = fc;
                    while (lo < cap) {
                        c = min(cap, lo + step);
                        fc = f32(c);
                        if (fc <= 0.f) {
                            hi = c;
                            fhi = fc;
                            break;
                        }
                        lo = c;
                        flo = fc;
                        step *= 4;
                    }
                }
            } else {
                // stop mode 1: Theorem 5's N0 satisfies the absolute test, so
                // the search needs no probe above it (Section 4 scans up to N0)
                if (SMODE == 1) {
                    double mn_unused = INFINITY, mzb = fmax(mz, P0 / pscale);
                    block_minmax<T>(mn_unused, mzb, shd);
                    top = min(cap, apriori_n0(mzb, L, N, delta));
                }
                for (int q = 0; q < kGeo; ++q) {
                    const int64_t mq = geo_m(q);
                    if (mq >= top) break;
                    const float fq = f32(mq);
                    if (fq <= 0.f) {
                        hi = mq;
                        fhi = fq;
                        break;
                    }
                    lo = mq;
                    flo = fq;
                }
                if (hi < 0) {
                    // no probe below the top satisfies the test
                    const float fc = f32(top);
                    if (fc <= 0.f) {
                        hi = top;
                        fhi = fc;
                    } else {
                        lo = top;
                    }
                }
            }
            if (hi < 0) {
                mt = top;
            } else {
                int side = 0;  // Illinois: endpoint kept twice in a row gets its f halved
                int64_t last_width = hi - lo;
                bool bisect = false;
                while (hi - lo > 1) {
                    int64_t c;
                    if (bisect || lo == 0 || !isfinite(flo)) {
                        c = lo + (hi - lo) / 2;
                    } else {
                        const double fr = (double)flo / ((double)flo - (double)fhi);
                        c = lo + (int64_t)llrint(fr * (double)(hi - lo));
                    }
                    c = max(lo + 1, min(hi - 1, c));
                    const float fc = f32(c);
                    if (fc <= 0.f) {
                        hi = c;
                        fhi = fc;
                        if (side == 1) flo *= 0.5f;
                        side = 1;
                    } else {
                        lo = c;
                        flo = fc;
                        if (side == -1) fhi *= 0.5f;
                        side = -1;
                    }
                    // force a bisection step when the bracket shrank less than half
                    const int64_t wdt = hi - lo;
                    bisect = (2 * wdt > last_width);
                    last_width = wdt;
                }
                mt = hi;
            }
        }

        // ---- deferred FP64 check: four-step signals leave it to pass 1,
        //      which reads the spectrum and forms the powers anyway; k_verify
        //      accepts the estimate or sends the signal back here (redo_only)
        if (deferred) {
            if (A.mt_shift) mt = max((int64_t)1, min(cap, mt + (int64_t)A.mt_shift));
            // the check in pass 1 counts the same bins as the FP64 evaluation here
            double mn_unused = INFINITY, qm = mz;
            block_minmax<T>(mn_unused, qm, shd);
            if (tid == 0) {
                S->L = L;
                S->m = mt;
                S->chk = 1;
                S->qthr = kSdNoise * qm;
                if (A.info) {
                    fif_imf_info* I = A.info + (int64_t)s * A.max_imfs + A.t;
                    I->k = S->k;
                    I->L = L;
                    I->m = mt;
                    I->flags = 0;
                    I->evals = (n32 & 0xffffu) | (1u << 16);
                }
            }
            return;
        }
    }

    // ---- FP64 SD at m and m-1 (Parseval, FP64 lambda, powers and sums).
    //      Stop mode 0: SD_m^2 is a P mu^(m-1)-weighted mean of lambda^2, so
    //      for large m it is decided by the bins that decay slowest.  Bins
    //      below the noise floor (|R_j|^2 < kSdNoise max_{j>=1} |R_j|^2:
    //      rounding-level content, of the input or of exact zeros) are left
    //      out (the deferred check in pass 1 does the same), and the weights are
    //      summed relative to the largest one (a running maximum of the
    //      exponent, as in a streaming log-sum-exp), so that the sums never
    //      underflow and SD tends to the smallest counted lambda, as in exact
    //      arithmetic.  The FP32 search above only brackets m; this decides.
    double qthr = RDO ? S->qthr : -1.0;   // the noise floor the deferred check used
    auto sd64 = [&](int64_t m, double& sd_m, double& sd_mm1) {
        if (SMODE == 0 && qthr < 0.0) {
            double mn_unused = INFINITY, qm = mz;
            block_minmax<T>(mn_unused, qm, shd);
            qthr = kSdNoise * qm;
        }
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        double amax = -INFINITY;  // stop mode 0, e >= 1: sums are relative to exp(amax)
        const int64_t e = m - 2;  // exponent of mu at m-1; may be -1
        constexpr int DG = 4;     // bins whose loads are issued together
        for (int j0 = 1 + tid; j0 <= nh; j0 += DG * T) {
          double2 zz[DG];
          int64_t jj[DG];
#pragma unroll
          for (int g = 0; g < DG; ++g) {
            const int j = j0 + g * T;
            zz[g] = make_double2(0.0, 0.0);
            jj[g] = 0;
            if (j <= nh) {
                zz[g] = R[pos_small(smap, j)];
                jj[g] = j;
            }
          }
#pragma unroll
          for (int g = 0; g < DG; ++g) {
            if (j0 + g * T > nh) break;
            const double2 z = zz[g];
            const int64_t jb = jj[g];
            const double q = z.x * z.x + z.y * z.y;
            if (SMODE == 0 && q < qthr) continue;   // below the noise floor
            const double P = weight(jb) * q * pscale;
            const double lam = lambda_at(jb, lw);
            const double l2 = lam * lam;
            const double om = 1.0 - lam;
            double xe, xm;  // mu^e, mu^(m-1) (stop mode 0, e >= 1: times exp(-amax))
            if (SMODE == 0) {
                if (e < 0) {
                    xe = 0.0;
                    xm = 1.0;
                } else if (lam >= 1.0) {
                    xe = (e == 0) ? 1.0 : 0.0;
                    xm = 0.0;
                } else if (e == 0) {
                    xe = 1.0;
                    xm = om * om;
                } else {
                    const double a = (double)e * 2.0 * log1p(-lam);
                    if (a > amax) {
                        const double r = (amax == -INFINITY) ? 0.0 : exp(amax - a);
                        v[0] *= r;
                        v[1] *= r;
                        v[2] *= r;
                        v[3] *= r;
                        amax = a;
                    }
                    xe = exp(a - amax);
                    xm = xe * om * om;
                }
            } else {
                if (e < 0)
                    xe = 0.0;
                else if (lam >= 1.0)
                    xe = (e == 0) ? 1.0 : 0.0;
                else if (e <= kPowByMul)
                    xe = ipow(om * om, e);
                else
                    xe = exp((double)e * 2.0 * log1p(-lam));
                xm = (e < 0) ? 1.0 : xe * om * om;
            }
            v[0] += P * l2 * xe;
            v[1] += P * xe;
            v[2] += P * l2 * xm;
            v[3] += P * xm;
          }
        }
        if (SMODE == 0 && e >= 1) {
            // bring every thread's sums to the block's largest exponent
            double mn_unused = INFINITY, am = amax;
            block_minmax<T>(mn_unused, am, shd);
            const double r = (amax == -INFINITY) ? 0.0 : exp(amax - am);
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] *= r;
        }
        if (tid == 0) {
            if (m == 1) {
                v[2] += P0;
                v[3] += P0;
            }
            if (m == 2) {
                v[0] += P0;
                v[1] += P0;
            }
        }
        block_sum<double, T, 4>(v, shd);
        n64 += 1;
        sd_m = v[3] > 0.0 ? sqrt(v[2] / v[3]) : 0.0;
        sd_mm1 = (m == 1) ? INFINITY : (v[1] > 0.0 ? sqrt(v[0] / v[1]) : 0.0);
        if (SMODE != 0) {
            // called with m + 1: the numerators are sum P lambda^2 mu^m and
            // sum P lambda^2 mu^(m-1), i.e. ||s_{m+1} - s_m||^2 and
            // ||s_m - s_{m-1}||^2 times N pscale
            sd_m = sqrt(v[2] * inv_np);
            sd_mm1 = sqrt(v[0] * inv_np);
        }
    };
    // FP64 stop quantities at m and m - 1 for the active stop mode
    auto stop64 = [&](int64_t m, double& sd_m, double& sd_mm1) { sd64(SMODE != 0 ? m + 1 : m, sd_m, sd_mm1); };

    // ---- FP64 confirmation of mt (SD_mt <= delta < SD_{mt-1}); otherwise an
    //      exact FP64 gallop + bisection from mt, then a final evaluation
    int64_t m = mt;
    double sd_m = 0.0, sd_p = 0.0;
    if (SMODE == 2) {
        stop64(m, sd_m, sd_p);      // reported only; m is the a-priori count
    } else {
        // stage 0 confirm, 1 gallop up, 2 gallop down, 3 bisect, 4 final
        int stage = 0;
        int64_t cand = mt, elo = 0, ehi = -1, gstep = 1;
        while (true) {
            double sm, sp;
            stop64(cand, sm, sp);
            const bool okm = ok(sm);
            if (stage == 4) {
                sd_m = sm;
                sd_p = sp;
                break;
            }
            if (stage == 0) {
                // m = 1 has no predecessor to reject it (stop mode 1 reports
                // ||s_1 - s_0|| as sd_prev, which may be below delta too)
                const bool okp = cand > 1 && ok(sp);
                if (okm && !okp) {
                    m = cand;
                    sd_m = sm;
                    sd_p = sp;
                    break;
                }
                flags |= FIF_IMF_REFINED;
                if (!okm) {
                    if (cand >= cap) {
                        m = cap;
                        sd_m = sm;
                        sd_p = sp;
                        break;
                    }
                    elo = cand;
                    stage = 1;
                } else {
                    ehi = cand - 1;  // SD_{cand-1} <= delta
                    stage = 2;
                }
            } else if (stage == 1) {
                if (okm) {
                    ehi = cand;
                    stage = 3;
                } else {
                    elo = cand;
                    if (cand >= cap) {
                        m = cap;
                        sd_m = sm;
                        sd_p = sp;
                        break;
                    }
                }
            } else if (stage == 2) {
                if (okm) {
                    ehi = cand;
                } else {
                    elo = cand;
                    stage = 3;
                }
            } else {
                if (okm)
                    ehi = cand;
                else
                    elo = cand;
            }
            // next candidate
            if (stage == 1) {
                cand = min(cap, elo + gstep);
                gstep *= 2;
            } else if (stage == 2) {
                if (ehi <= 1) {
                    elo = 0;
                    stage = 3;
                } else {
                    cand = max((int64_t)1, ehi - gstep);
                    gstep *= 2;
                }
            }
            if (stage == 3) {
                if (ehi - elo <= 1) {
                    m = ehi;
                    cand = ehi;
                    stage = 4;
                } else {
                    cand = elo + (ehi - elo) / 2;
                }
            }
        }
    }
    if (SMODE != 2 && !ok(sd_m)) flags |= FIF_IMF_CAP;
    if (A.redo_only) flags |= FIF_IMF_REFINED;   // the deferred check rejected the estimate

    if (tid == 0) {
        S->L = L;
        S->m = m;
        S->sd = sd_m;
        S->sd_prev = sd_p;
        S->flags |= (int32_t)flags;
        if (A.info) {
            fif_imf_info* I = A.info + (int64_t)s * A.max_imfs + A.t;
            I->k = S->k;
            I->L = L;
            I->m = m;
            I->sd = sd_m;
            I->sd_prev = sd_p;
            I->flags = flags;
            I->evals = (n32 & 0xffffu) | (n64 << 16);
        }
    }
}

// Deferred FP64 check of m (one thread per signal of the list): the pass-1
// tiles' partial sums in tile order give SD_m and SD_{m-1}; the estimate is
// kept if SD_m <= delta < SD_{m-1} (or m is the cap and SD_m > delta, as the
// in-scan check decides), else the signal is marked for a redo.
__global__ void k_verify(ScanArgs A, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = A.list[i];
    SigState* S = A.st + s;
    if (!S->active || !S->chk) return;
    const SigDesc d = A.sigs[s];
    const LenPlan& lp = A.lens[d.len_id];
    const int tiles = lp.N1 / lp.TC;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < tiles; ++t) {
        const double* c = A.chk + ((int64_t)d.p1_off + t) * 4;
        v[0] += c[0];
        v[1] += c[1];
        v[2] += c[2];
        v[3] += c[3];
    }
    const int64_t m = S->m;
    const double sd_m = v[1] > 0.0 ? sqrt(v[0] / v[1]) : 0.0;
    const double sd_p = (m == 1) ? INFINITY : (v[3] > 0.0 ? sqrt(v[2] / v[3]) : 0.0);
    const bool okm = sd_m <= A.delta, okp = sd_p <= A.delta;
    S->chk = 0;
    if ((okm && !okp) || (!okm && m >= A.max_inner)) {
        const uint32_t flags = okm ? 0u : (uint32_t)FIF_IMF_CAP;
        S->sd = sd_m;
        S->sd_prev = sd_p;
        S->flags |= (int32_t)flags;
        if (A.info) {
            fif_imf_info* I = A.info + (int64_t)s * A.max_imfs + A.t;
            I->sd = sd_m;
            I->sd_prev = sd_p;
            I->flags = flags;
        }
    } else {
        S->redo = 1;
    }
}

// ------------------------------------------------------------- finalize --

__global__ void k_finalize(SigState* __restrict__ st, int B, int max_imfs, int32_t* __restrict__ n_imfs,
                           int32_t* __restrict__ sig_status, fif_imf_info* __restrict__ info)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    SigState* S = st + s;
    if (S->active) {
        S->active = 0;
        S->n_imfs = max_imfs;
        S->stop_reason = FIF_STOP_MAX_IMFS;
        S->final_buf = max_imfs & 1;
    }
    if (n_imfs) n_imfs[s] = S->n_imfs;
    if (sig_status) sig_status[s] = S->status;
    if (info) {
        for (int j = S->n_imfs; j < max_imfs; ++j) {
            fif_imf_info* I = info + (int64_t)s * max_imfs + j;
            I->k = 0;
            I->L = 0;
            I->m = 0;
            I->sd = 0.0;
            I->sd_prev = 0.0;
            I->flags = 0;
            I->evals = 0;
        }
    }
}

__global__ void k_reset_state(SigState* __restrict__ st, int B)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    SigState z;
    z.k = z.L = z.m = 0;
    z.sd = z.sd_prev = 0.0;
    z.mean = z.maxabs = 0.0;
    z.pscale = 1.0;
    z.kmin = dkey(INFINITY);
    z.kmax = dkey(-INFINITY);
    z.active = 1;
    z.n_imfs = 0;
    z.stop_reason = 0;
    z.status = 0;
    z.final_buf = 0;
    z.flags = 0;
    z.fpeak = 1;
    z.chk = 0;
    z.redo = 0;
    st[s] = z;
}

}  // namespace fif
