// LDS-resident mixed-radix Stockham FFT for gfx950 (complex FP64).
//
// A workgroup of kFftThreads threads transforms `batch` independent
// sequences of length n held in LDS, element e of sequence c at
// buf[e * batch + c] (sequence-interleaved, so a global row of `batch`
// consecutive columns maps to consecutive LDS words).  Each pass of radix R
// reads all of its inputs into registers, synchronises, and writes the
// outputs back in place in Stockham (self-sorting) order, so the result is
// in natural order and only n*batch complex words of LDS are needed.
//
// Pass with radix R after radices of product Ns: butterfly j reads
// x[j + r*n/R] (r < R), multiplies input r by w^r with
// w = exp(-+2 pi i (j mod Ns) / (Ns R)), applies the R-point DFT and writes
// element r to (j / Ns) * Ns * R + (j mod Ns) + r * Ns.  The per-pass table
// holds exp(-2 pi i k / (Ns R)), k < Ns; the inverse direction conjugates.
#pragma once
#include <hip/hip_runtime.h>

#include "fif_types.hpp"

namespace fif {

// Complex arithmetic for the two element types of the transforms: double2
// (FP64 transforms) and float2 (the FP32 lane).  Mixed-precision constants
// (the radix-8 and odd-radix cosines) are rounded to the element type.
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, double s)
{
    const float f = (float)s;
    return make_float2(a.x * f, a.y * f);
}
// multiply by s*i, s = +1 (inverse direction) or -1 (forward direction)
template <bool INV>
__device__ __forceinline__ double2 mul_si(double2 a)
{
    return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}
template <bool INV>
__device__ __forceinline__ float2 mul_si(float2 a)
{
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// conversions between the element types and FP64
template <typename C> __device__ __forceinline__ C to_c(double2 v);
template <> __device__ __forceinline__ double2 to_c<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 to_c<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ double2 to_d(double2 v) { return v; }
__device__ __forceinline__ double2 to_d(float2 v) { return make_double2((double)v.x, (double)v.y); }
template <typename C> __device__ __forceinline__ C czero() { return to_c<C>(make_double2(0.0, 0.0)); }

// cos / sin of 2 pi p / R, p <= (R-1)/2, for the odd radices (correctly
// rounded literals)
template <int R>
__device__ __forceinline__ constexpr double odd_cos(int p)
{
    return R == 3 ? (p == 0 ? 1.0 : -0.5)
         : R == 5 ? (p == 0 ? 1.0 : p == 1 ? 0.30901699437494745 : -0.8090169943749475)
                  : (p == 0 ? 1.0 : p == 1 ? 0.6234898018587335
                                  : p == 2 ? -0.2225209339563144 : -0.9009688679024191);
}
template <int R>
__device__ __forceinline__ constexpr double odd_sin(int p)
{
    return R == 3 ? (p == 0 ? 0.0 : 0.8660254037844386)
         : R == 5 ? (p == 0 ? 0.0 : p == 1 ? 0.9510565162951535 : 0.5877852522924731)
                  : (p == 0 ? 0.0 : p == 1 ? 0.7818314824680298
                                  : p == 2 ? 0.9749279121818236 : 0.4338837391175581);
}

// In-register R-point DFT, X_k = sum_r a_r exp(s 2 pi i r k / R).
template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
    template <typename C>
    __device__ __forceinline__ static void run(C* a)
    {
        C t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};

template <bool INV> struct Dft<4, INV> {
    template <typename C>
    __device__ __forceinline__ static void run(C* a)
    {
        C s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
        C s13 = cadd(a[1], a[3]), d13 = mul_si<INV>(csub(a[1], a[3]));
        a[0] = cadd(s02, s13);
        a[2] = csub(s02, s13);
        a[1] = cadd(d02, d13);
        a[3] = csub(d02, d13);
    }
};

template <bool INV> struct Dft<8, INV> {
    template <typename C>
    __device__ __forceinline__ static void run(C* a)
    {
        constexpr double h = 0.7071067811865476;
        C e[4] = {a[0], a[2], a[4], a[6]};
        C o[4] = {a[1], a[3], a[5], a[7]};
        Dft<4, INV>::run(e);
        Dft<4, INV>::run(o);
        // w8^1 = h (1 + s i), w8^2 = s i, w8^3 = h (-1 + s i)
        C o1 = cscale(cadd(o[1], mul_si<INV>(o[1])), h);
        C o2 = mul_si<INV>(o[2]);
        C o3 = cscale(csub(mul_si<INV>(o[3]), o[3]), h);
        a[0] = cadd(e[0], o[0]);
        a[4] = csub(e[0], o[0]);
        a[1] = cadd(e[1], o1);
        a[5] = csub(e[1], o1);
        a[2] = cadd(e[2], o2);
        a[6] = csub(e[2], o2);
        a[3] = cadd(e[3], o3);
        a[7] = csub(e[3], o3);
    }
};

// odd R: pair inputs q and R-q; X_k and X_{R-k} share the cosine part
template <int R, bool INV> struct DftOdd {
    template <typename C>
    __device__ __forceinline__ static void run(C* a)
    {
        constexpr int H = (R - 1) / 2;
        C t[H], u[H];
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            t[q - 1] = cadd(a[q], a[R - q]);
            u[q - 1] = csub(a[q], a[R - q]);
        }
        C x0 = a[0];
#pragma unroll
        for (int q = 0; q < H; ++q) x0 = cadd(x0, t[q]);
        C out[R];
        out[0] = x0;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            C re = a[0];
            C im = czero<C>();
#pragma unroll
            for (int q = 1; q <= H; ++q) {
                const int p = (q * k) % R;
                const int pp = p <= H ? p : R - p;
                const double cs = odd_cos<R>(pp);
                const double sn = p <= H ? odd_sin<R>(pp) : -odd_sin<R>(pp);
                re = cadd(re, cscale(t[q - 1], cs));
                im = cadd(im, cscale(u[q - 1], sn));
            }
            C sim = mul_si<INV>(im);
            out[k] = cadd(re, sim);
            out[R - k] = csub(re, sim);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = out[r];
    }
};
template <bool INV> struct Dft<3, INV> : DftOdd<3, INV> {};
template <bool INV> struct Dft<5, INV> : DftOdd<5, INV> {};
template <bool INV> struct Dft<7, INV> : DftOdd<7, INV> {};

// x / d and x % d for 0 <= x < 2^24, 1 <= d < 2^16: a shift and a mask when
// d is a power of two (a uniform branch), else the FP32 quotient, off by at
// most one, fixed with one correction.
struct FastDiv {
    float r;
    int d;
    int sh;        // log2 d when d is a power of two, else -1
};
__device__ __forceinline__ FastDiv fastdiv(int d)
{
    const int sh = ((d & (d - 1)) == 0) ? __ffs(d) - 1 : -1;
    return {1.0f / (float)d, d, sh};
}
__device__ __forceinline__ int fdivmod(int x, FastDiv f, int& rem)
{
    if (f.sh >= 0) {
        rem = x & (f.d - 1);
        return x >> f.sh;
    }
    int q = (int)((float)x * f.r);
    int r = x - q * f.d;
    if (r < 0) {
        q -= 1;
        r += f.d;
    } else if (r >= f.d) {
        q += 1;
        r -= f.d;
    }
    rem = r;
    return q;
}

// One Stockham pass over `batch` interleaved sequences, CAP >= n * batch,
// elements of type C (double2 or float2; the twiddle tables are FP64).
template <int R, bool INV, int CAP, typename C>
__device__ __forceinline__ void fft_pass(C* __restrict__ buf, int n, int batch, int ns,
                                         const double2* __restrict__ tw)
{
    constexpr int Q = (CAP / R + kFftThreads - 1) / kFftThreads;
    const int nb = n / R;
    const int items = nb * batch;
    const FastDiv fb = fastdiv(batch), fn = fastdiv(ns);
    C v[Q][R];
    int jq[Q], cq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int it = threadIdx.x + q * kFftThreads;
        int c = 0, j = 0;
        if (it < items) {
            j = fdivmod(it, fb, c);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[(j + r * nb) * batch + c];
        }
        jq[q] = j;
        cq[q] = c;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int it = threadIdx.x + q * kFftThreads;
        if (it < items) {
            const int c = cq[q], j = jq[q];
            int k;
            const int jd = fdivmod(j, fn, k);
            if (ns > 1) {
                C w = to_c<C>(tw[k]);
                if (INV) w.y = -w.y;
                C wr = w;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    v[q][r] = cmul(v[q][r], wr);
                    if (r + 1 < R) wr = cmul(wr, w);
                }
            }
            Dft<R, INV>::run(v[q]);
            const int base = jd * ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[(base + r * ns) * batch + c] = v[q][r];
        }
    }
    __syncthreads();
}

// Transform `batch` interleaved sequences of length f.n in place
// (f.n * batch <= CAP).  Caller must __syncthreads() after filling buf.
// P2: the plan has radices 2, 4 and 8 only (kernels without the odd-radix
// passes need fewer registers).
template <bool INV, int CAP, bool P2 = false, typename C>
__device__ __forceinline__ void lds_fft(C* __restrict__ buf, const SubFft& f, int batch,
                                        const double2* __restrict__ twbase)
{
    const double2* tw = twbase + f.tw_off;
    int ns = 1;
    for (int p = 0; p < f.nrad; ++p) {
        const int R = f.rad[p];
        if (P2) {
            switch (R) {
            case 2: fft_pass<2, INV, CAP, C>(buf, f.n, batch, ns, tw); break;
            case 4: fft_pass<4, INV, CAP, C>(buf, f.n, batch, ns, tw); break;
            default: fft_pass<8, INV, CAP, C>(buf, f.n, batch, ns, tw); break;
            }
        } else {
            switch (R) {
            case 2: fft_pass<2, INV, CAP, C>(buf, f.n, batch, ns, tw); break;
            case 3: fft_pass<3, INV, CAP, C>(buf, f.n, batch, ns, tw); break;
            case 4: fft_pass<4, INV, CAP, C>(buf, f.n, batch, ns, tw); break;
            case 5: fft_pass<5, INV, CAP, C>(buf, f.n, batch, ns, tw); break;
            case 7: fft_pass<7, INV, CAP, C>(buf, f.n, batch, ns, tw); break;
            default: fft_pass<8, INV, CAP, C>(buf, f.n, batch, ns, tw); break;
            }
        }
        tw += ns;
        ns *= R;
    }
}

}  // namespace fif
