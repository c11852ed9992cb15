// Host runtime of libfif: plans (radix factorisation, four-step split,
// tiles, work lists, device twiddle and sine tables), workspace layout, and
// the launch sequence of the batched and single-signal decompositions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/fif.h"
#include "fif_bigscan.hpp"
#include "fif_model_internal.hpp"
#include "fif_propose.hpp"
#include "fif_tune.hpp"

using namespace fif;

namespace {

thread_local std::string g_err;

fif_status fail(fif_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(FIF_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// prime factors <= 7 only
bool smooth7(int64_t n)
{
    if (n < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

bool make_subfft(int64_t n, SubFft& f)
{
    std::memset(&f, 0, sizeof(f));
    f.n = (int32_t)n;
    int64_t r = n;
    int e2 = 0;
    while (r % 2 == 0) { r /= 2; ++e2; }
    std::vector<int> rad;
    while (e2 >= 3) { rad.push_back(8); e2 -= 3; }
    if (e2 == 2) rad.push_back(4);
    if (e2 == 1) rad.push_back(2);
    for (int p : {7, 5, 3})
        while (r % p == 0) { rad.push_back(p); r /= p; }
    if (r != 1 || (int)rad.size() > kMaxRadices) return false;
    f.nrad = (int32_t)rad.size();
    for (size_t i = 0; i < rad.size(); ++i) f.rad[i] = (int8_t)rad[i];
    return true;
}

int64_t largest_divisor_at_most(int64_t n, int64_t cap)
{
    for (int64_t d = std::min(n, cap); d >= 1; --d)
        if (n % d == 0) return d;
    return 1;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

namespace fif {
fif_status fif_internal_fail(fif_status st, const std::string& msg) { return fail(st, "%s", msg.c_str()); }
}  // namespace fif

struct fif_plan {
    int device = 0;
    int32_t B = 0, max_imfs = 0;
    fif_options opt;
    std::vector<int64_t> lengths;
    std::vector<SigDesc> sigs;
    std::vector<LenPlan> lens;
    std::vector<Work> w_init, w_single, w_p1, w_p2;
    std::vector<int32_t> scan_small, scan_big;
    std::vector<Work> w_btile, w_count;
    // Signal groups: contiguous signal ranges whose outer steps are issued
    // on separate streams, so that one group's scan (latency bound, one
    // workgroup per signal) runs beside another group's transforms.  Each
    // group owns a contiguous sub-range of every work list.
    struct Range {
        int32_t begin = 0, count = 0;
    };
    struct Group {
        int32_t s0 = 0, s1 = 0;
        Range single, p1, p2, ssmall, sbig, btile, count;
        // signals of the multi-workgroup search that defer their FP64 check
        // (at most kBigDeferTiles tiles): some of them, all of them
        bool big_defer_any = false, big_defer_all = true;
        // kinds among the one-workgroup scan's signals: four-step, one pass
        bool small_two_pass = false, small_one_pass = false;
    };
    std::vector<Group> groups;      // groups[0] is the whole batch when only one
    Group all;
    std::vector<hipStream_t> gstreams;   // streams of groups 1..
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    // graph of the last captured batched call and the arguments it was
    // captured with
    hipGraphExec_t gexec = nullptr;
    std::vector<uintptr_t> gkey;
    size_t lds_single = 0, lds_p1 = 0, lds_p2 = 0;
    bool wide = false;              // a length uses tiles above kTileCap elements
    bool pow2 = false;              // every four-step length has radices 2, 4, 8 only
    bool fp32 = false;              // the FP32 lane (fif_options.precision)
    // device copies (one allocation)
    DevBuf dmeta, dtabs;
    SigDesc* d_sigs = nullptr;
    LenPlan* d_lens = nullptr;
    Work *d_init = nullptr, *d_single = nullptr, *d_p1 = nullptr, *d_p2 = nullptr;
    int32_t *d_scan_small = nullptr, *d_scan_big = nullptr;
    Work *d_btile = nullptr, *d_count = nullptr;
    double* d_dtab = nullptr;
    double2* d_ctab = nullptr;
    int32_t* d_itab = nullptr;
    // workspace layout (byte offsets)
    size_t ws_state = 0, ws_spec0 = 0, ws_spec1 = 0, ws_inter = 0, ws_parts = 0, ws_psum = 0, ws_gscr = 0,
           ws_bigs = 0, ws_bpart = 0, ws_bqmax = 0, ws_resid = 0, ws_feat = 0, ws_prop = 0, ws_chk = 0, ws_total = 0;
    // sampled window shape: its samples (in the FP64 table at wshape_off),
    // and the workspace of the per-step eigenvalue tables
    std::vector<double> wshape;
    int64_t wshape_off = 0;
    size_t ws_taps = 0, ws_lam = 0, ws_wsum = 0;
    int32_t mt_shift = 0;           // test hook (FIF_DEBUG_MT_SHIFT): perturbs the deferred estimate
    // lengths whose choice was measured (fif_plan_create_tuned): their times
    std::map<int64_t, fif_length_plan> tuned;
    // learned proposal of m, and recording of the network inputs
    fif_model* model = nullptr;
    uint16_t* rec = nullptr;
    // kernel timing (fif_plan_profile)
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    bool prof = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    std::vector<std::string> kinds;
    ~fif_plan()
    {
        for (auto& r : recs) {
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
        for (auto s : gstreams) (void)hipStreamDestroy(s);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        for (auto e : ev_join) (void)hipEventDestroy(e);
        if (gexec) (void)hipGraphExecDestroy(gexec);
    }
};

namespace {

// Sizes of the structures host and kernels share, as the device compilation
// saw them.  The host compares them with its own once before any launch: a
// library whose host and device passes were compiled from different sources
// would otherwise hand the kernels misplaced fields.  (Not const: a const
// device array no kernel reads is left out of the device code, and the
// runtime then cannot resolve the host's reference to it.)
__device__ int64_t kDeviceAbi[5] = {(int64_t)sizeof(StepArgs), (int64_t)sizeof(ScanArgs),
                                    (int64_t)sizeof(SigState), (int64_t)sizeof(LenPlan),
                                    (int64_t)sizeof(SigDesc)};

fif_status check_abi()
{
    static std::once_flag once;
    static fif_status st = FIF_OK;
    static std::string msg;
    std::call_once(once, [] {
        int64_t dev[5] = {0, 0, 0, 0, 0};
        const hipError_t e = hipMemcpyFromSymbol(dev, HIP_SYMBOL(kDeviceAbi), sizeof(dev), 0, hipMemcpyDeviceToHost);
        const int64_t host[5] = {(int64_t)sizeof(StepArgs), (int64_t)sizeof(ScanArgs), (int64_t)sizeof(SigState),
                                 (int64_t)sizeof(LenPlan), (int64_t)sizeof(SigDesc)};
        if (e != hipSuccess) {
            st = FIF_ERR_DEVICE;
            msg = std::string("reading the device structure sizes: ") + hipGetErrorString(e);
        } else if (std::memcmp(dev, host, sizeof(dev)) != 0) {
            st = FIF_ERR_DEVICE;
            char buf[256];
            std::snprintf(buf, sizeof(buf),
                          "host and device structure sizes differ (%lld/%lld %lld/%lld %lld/%lld %lld/%lld "
                          "%lld/%lld): the library was built from inconsistent sources",
                          (long long)host[0], (long long)dev[0], (long long)host[1], (long long)dev[1],
                          (long long)host[2], (long long)dev[2], (long long)host[3], (long long)dev[3],
                          (long long)host[4], (long long)dev[4]);
            msg = buf;
        }
    });
    if (st != FIF_OK) return fail(st, "%s", msg.c_str());
    return FIF_OK;
}

fif_status set_lds_limits()
{
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        const int lim = kFftCap * (int)sizeof(double2);
        auto set = [&](const void* f) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
            if (e != hipSuccess && err == hipSuccess) err = e;
        };
        // every instantiation the launches use, for both element types
        auto all = [&](auto tag) {
            using C = decltype(tag);
            set((const void*)k_single<MODE_FORWARD, float, float, C>);
            set((const void*)k_single<MODE_STEP, float, float, C>);
            set((const void*)k_single<MODE_REMAINDER, float, float, C>);
            set((const void*)k_single<MODE_FORWARD, double, double, C>);
            set((const void*)k_single<MODE_STEP, double, double, C>);
            set((const void*)k_single<MODE_REMAINDER, double, double, C>);
            auto tiles = [&](auto tile) {
                constexpr int TL = decltype(tile)::value;
                set((const void*)k_pass1<MODE_FORWARD, float, false, TL, false, C>);
                set((const void*)k_pass1<MODE_REMAINDER, float, false, TL, false, C>);
                set((const void*)k_pass1<MODE_FORWARD, double, false, TL, false, C>);
                set((const void*)k_pass1<MODE_REMAINDER, double, false, TL, false, C>);
                set((const void*)k_pass2<MODE_FORWARD, float, float, TL, false, C>);
                set((const void*)k_pass2<MODE_REMAINDER, float, float, TL, false, C>);
                set((const void*)k_pass2<MODE_FORWARD, double, double, TL, false, C>);
                set((const void*)k_pass2<MODE_REMAINDER, double, double, TL, false, C>);
                auto p2 = [&](auto pow2) {
                    constexpr bool P2 = decltype(pow2)::value;
                    set((const void*)k_pass1<MODE_STEP, float, false, TL, P2, C>);
                    set((const void*)k_pass1<MODE_STEP, float, true, TL, P2, C>);
                    set((const void*)k_pass1<MODE_STEP, double, false, TL, P2, C>);
                    set((const void*)k_pass1<MODE_STEP, double, true, TL, P2, C>);
                    set((const void*)k_pass2<MODE_STEP, float, float, TL, P2, C>);
                    set((const void*)k_pass2<MODE_STEP, double, double, TL, P2, C>);
                };

                p2(std::false_type{});
                p2(std::true_type{});
            };
            tiles(std::integral_constant<int, kTileCap>{});
            tiles(std::integral_constant<int, kTileCapBig>{});
            set((const void*)k_scan<kScanBinsPerThread, false, 0, C>);
            set((const void*)k_scan<kScanBinsPerThread, true, 0, C>);
            set((const void*)k_scan<kScanBinsDeferred, false, 0, C, true>);
            set((const void*)k_scan<kScanBinsDeferred, true, 0, C, true>);
            set((const void*)k_scan<kScanBinsPerThread, false, 1, C>);
            set((const void*)k_scan<kScanBinsPerThread, true, 1, C>);
            set((const void*)k_scan<kScanBinsPerThread, false, 2, C>);
            set((const void*)k_scan<kScanBinsPerThread, true, 2, C>);
        };
        all(double2{});
        all(float2{});
        // sampled window shapes: FP64 transforms only
        set((const void*)k_single<MODE_WINDOW, double, double>);
        set((const void*)k_pass1<MODE_WINDOW, double>);
        set((const void*)k_pass2<MODE_WINDOW, double, double>);
        set((const void*)k_pass1<MODE_WINDOW, double, false, kTileCapBig>);
        set((const void*)k_pass2<MODE_WINDOW, double, double, kTileCapBig>);
    });
    if (err != hipSuccess) return fail(FIF_ERR_DEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(err));
    return FIF_OK;
}

fif_status validate_opts(const fif_options& o)
{
    if (o.mask_rule < 0 || o.mask_rule > 2) return fail(FIF_ERR_INVALID_ARG, "mask_rule must be 0, 1 or 2");
    if (o.stop_mode < 0 || o.stop_mode > 2) return fail(FIF_ERR_INVALID_ARG, "stop_mode must be 0, 1 or 2");
    if (!(o.gamma >= 0.0 && o.gamma < 1.0)) return fail(FIF_ERR_INVALID_ARG, "gamma must be in [0, 1)");
    if (o.mask_rule == 2 && !(o.peak_rho > 0.0 && o.peak_rho <= 1.0))
        return fail(FIF_ERR_INVALID_ARG, "peak_rho must be in (0, 1]");
    if (o.mask_rule == 1 && !(o.nu > 0.0 && std::isfinite(o.nu)))
        return fail(FIF_ERR_INVALID_ARG, "nu must be positive and finite");
    if (o.max_inner < 1 || o.max_inner > (int64_t)1 << 40)
        return fail(FIF_ERR_INVALID_ARG, "max_inner must be in [1, 2^40]");
    if (!(o.floor_tau >= 0.0 && std::isfinite(o.floor_tau)))
        return fail(FIF_ERR_INVALID_ARG, "floor_tau must be finite and >= 0");
    if (o.window) {
        if (o.window_points < 2 || o.window_points > kMaxWindowPoints)
            return fail(FIF_ERR_INVALID_ARG, "window_points must be in [2, %d]", kMaxWindowPoints);
        for (int i = 0; i < o.window_points; ++i)
            if (!(o.window[i] >= 0.0 && std::isfinite(o.window[i])))
                return fail(FIF_ERR_INVALID_ARG, "window sample %d must be finite and >= 0", i);
        if (!(o.window[0] > 0.0)) return fail(FIF_ERR_INVALID_ARG, "the first window sample must be > 0");
        if (o.stop_mode == 2)
            return fail(FIF_ERR_INVALID_ARG, "stop_mode 2 counts the triangle window's zero eigenvalues: "
                                             "not with a sampled window");
    } else if (o.window_points != 0) {
        return fail(FIF_ERR_INVALID_ARG, "window_points given without window samples");
    }
    if (o.precision != FIF_PREC_MIXED && o.precision != FIF_PREC_FP32)
        return fail(FIF_ERR_INVALID_ARG, "precision must be FIF_PREC_MIXED or FIF_PREC_FP32");
    if (o.precision == FIF_PREC_FP32 && o.window)
        return fail(FIF_ERR_INVALID_ARG, "the FP32 lane does not take a sampled window shape");
    return FIF_OK;
}

// Radix plans, four-step split and tiles of one distinct length.
fif_status plan_length(int64_t N, LenPlan& lp)
{
    std::memset(&lp, 0, sizeof(lp));
    lp.N = N;
    if (N <= kFftCap) {
        lp.two_pass = 0;
        lp.N1 = 1;
        lp.N2 = (int32_t)N;
        if (!make_subfft(N, lp.f1))
            return fail(FIF_ERR_UNSUPPORTED_LENGTH, "length %lld has a prime factor > 7", (long long)N);
        lp.TC = lp.TR = 1;
        return FIF_OK;
    }
    // N = N1 * N2, both <= kTileCap (the four-step kernels stage at most
    // kTileCap elements per workgroup), max(N1, N2) smallest
    int64_t best1 = -1;
    for (int64_t n2 = 1; n2 <= kTileCap; ++n2) {
        if (N % n2) continue;
        const int64_t n1 = N / n2;
        if (n1 > kTileCap) continue;
        if (best1 < 0 || std::max(n1, n2) < std::max(best1, N / best1)) best1 = n1;
    }
    if (best1 < 0)
        return fail(FIF_ERR_UNSUPPORTED_LENGTH, "length %lld does not split into two factors <= %d",
                    (long long)N, kTileCap);
    lp.two_pass = 1;
    lp.N1 = (int32_t)best1;
    lp.N2 = (int32_t)(N / best1);
    if (!make_subfft(lp.N2, lp.f1) || !make_subfft(lp.N1, lp.f2))
        return fail(FIF_ERR_UNSUPPORTED_LENGTH, "length %lld has a prime factor > 7", (long long)N);
    lp.TC = (int32_t)largest_divisor_at_most(lp.N1, kTileCap / lp.N2);
    lp.TR = (int32_t)largest_divisor_at_most(lp.N2, kTileCap / lp.N1);
    // a single column (row) per tile reads the spectrum (writes the output)
    // at a stride of N1 (N2) elements: take two per wide tile instead
    if (lp.TC == 1 && lp.N1 % 2 == 0 && 2 * (int64_t)lp.N2 <= kTileCapBig) lp.TC = 2;
    if (lp.TR == 1 && lp.N2 % 2 == 0 && 2 * (int64_t)lp.N1 <= kTileCapBig) lp.TR = 2;
    // mirror-paired column tiles need N1, N2 and the tile width even
    lp.paired = (lp.N1 % 2 == 0 && lp.N2 % 2 == 0 && lp.TC % 2 == 0) ? 1 : 0;
    lp.spec_perm = lp.paired;
    int64_t split = 1;
    int shift = 0;
    while (split * split < N) {
        split *= 2;
        ++shift;
    }
    lp.big_split = (int32_t)split;
    lp.big_shift = shift;
    return FIF_OK;
}

// Length plan from an explicit choice (validated by choice_valid).
fif_status plan_from_choice(const fif_length_plan& c, LenPlan& lp)
{
    if (!choice_valid(c)) return fail(FIF_ERR_INVALID_ARG, "invalid plan choice for length %lld", (long long)c.N);
    std::memset(&lp, 0, sizeof(lp));
    lp.N = c.N;
    auto sub = [](int n, const int8_t* rad, int nr, SubFft& f) {
        std::memset(&f, 0, sizeof(f));
        f.n = n;
        f.nrad = nr;
        for (int i = 0; i < nr; ++i) f.rad[i] = rad[i];
    };
    if (c.N <= kFftCap) {
        lp.two_pass = 0;
        lp.N1 = 1;
        lp.N2 = (int32_t)c.N;
        lp.TC = lp.TR = 1;
        sub((int)c.N, c.rad1, c.n_rad1, lp.f1);
        return FIF_OK;
    }
    lp.two_pass = 1;
    lp.N1 = c.N1;
    lp.N2 = c.N2;
    lp.TC = c.TC;
    lp.TR = c.TR;
    sub(c.N2, c.rad1, c.n_rad1, lp.f1);
    sub(c.N1, c.rad2, c.n_rad2, lp.f2);
    lp.paired = (lp.N1 % 2 == 0 && lp.N2 % 2 == 0 && lp.TC % 2 == 0) ? 1 : 0;
    lp.spec_perm = lp.paired;
    int64_t split = 1;
    int shift = 0;
    while (split * split < c.N) {
        split *= 2;
        ++shift;
    }
    lp.big_split = (int32_t)split;
    lp.big_shift = shift;
    return FIF_OK;
}

// The choice a length plan embodies.
fif_length_plan choice_of(const LenPlan& lp)
{
    fif_length_plan c;
    std::memset(&c, 0, sizeof(c));
    c.N = lp.N;
    c.N1 = lp.two_pass ? lp.N1 : 1;
    c.N2 = lp.two_pass ? lp.N2 : (int32_t)lp.N;
    c.TC = lp.two_pass ? lp.TC : 1;
    c.TR = lp.two_pass ? lp.TR : 1;
    c.n_rad1 = lp.f1.nrad;
    for (int i = 0; i < lp.f1.nrad; ++i) c.rad1[i] = lp.f1.rad[i];
    c.n_rad2 = lp.two_pass ? lp.f2.nrad : 0;
    for (int i = 0; i < c.n_rad2; ++i) c.rad2[i] = lp.f2.rad[i];
    return c;
}

template <typename T>
T* upload(char* dbase, size_t off, const std::vector<T>& v, std::vector<char>& host)
{
    if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
    return reinterpret_cast<T*>(dbase + off);
}

}  // namespace

extern "C" {

void fif_options_default(fif_options* opt)
{
    if (!opt) return;
    opt->mask_rule = 0;
    opt->stop_mode = 0;
    opt->nu = 1.6;
    opt->max_inner = 1000000;
    opt->floor_tau = 1e-9;
    opt->gamma = 0.0;
    opt->peak_rho = 0.1;
    opt->window = nullptr;
    opt->window_points = 0;
    opt->precision = FIF_PREC_MIXED;
}

const char* fif_last_error(void) { return g_err.c_str(); }

const char* fif_status_string(fif_status s)
{
    switch (s) {
    case FIF_OK: return "ok";
    case FIF_ERR_INVALID_ARG: return "invalid argument";
    case FIF_ERR_UNSUPPORTED_LENGTH: return "unsupported length";
    case FIF_ERR_NOMEM: return "out of memory";
    case FIF_ERR_DEVICE: return "device error";
    case FIF_ERR_NONFINITE: return "non-finite input";
    case FIF_ERR_CAPACITY: return "capacity exceeded";
    case FIF_ERR_NOT_FOUND: return "not found";
    }
    return "unknown status";
}

}  // extern "C"

namespace {

using ChoiceMap = std::map<int64_t, fif_length_plan>;

// fif_plan_create, with the choices in `forced` for the lengths it lists.
fif_status create_plan(fif_plan** out, const int64_t* lengths, int32_t B, int32_t max_imfs, const fif_options* opt_in,
                       const ChoiceMap* forced)
{
    g_err.clear();
    if (!out) return fail(FIF_ERR_INVALID_ARG, "plan pointer is null");
    *out = nullptr;
    if (!lengths || B < 1) return fail(FIF_ERR_INVALID_ARG, "need at least one signal length");
    if (max_imfs < 1 || max_imfs > 4096) return fail(FIF_ERR_INVALID_ARG, "max_imfs must be in [1, 4096]");
    fif_options opt;
    fif_options_default(&opt);
    if (opt_in) opt = *opt_in;
    fif_status st = validate_opts(opt);
    if (st) return st;

    std::unique_ptr<fif_plan> p(new fif_plan());
    p->B = B;
    p->max_imfs = max_imfs;
    p->opt = opt;
    p->lengths.assign(lengths, lengths + B);
    if (opt.window) p->wshape.assign(opt.window, opt.window + opt.window_points);
    p->opt.window = nullptr;    // the caller's array is not kept
    std::map<int64_t, int32_t> len_id;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t N = lengths[b];
        if (N < 2) return fail(FIF_ERR_INVALID_ARG, "signal %d: length %lld < 2", b, (long long)N);
        if (N > ((int64_t)1 << 30)) return fail(FIF_ERR_UNSUPPORTED_LENGTH, "signal %d too long", b);
        if (!smooth7(N))
            return fail(FIF_ERR_UNSUPPORTED_LENGTH, "signal %d: length %lld has a prime factor > 7", b,
                        (long long)N);
        if (!len_id.count(N)) {
            LenPlan lp;
            if (forced && forced->count(N))
                st = plan_from_choice(forced->at(N), lp);
            else
                st = plan_length(N, lp);
            if (st) return st;
            len_id[N] = (int32_t)p->lens.size();
            p->lens.push_back(lp);
        }
    }

    // all host-side validation is done: from here on the device is used
    st = check_abi();
    if (st) return st;
    st = set_lds_limits();
    if (st) return st;
    HIP_TRY(hipGetDevice(&p->device));

    // tables: sines (doubles) and twiddles (complex), laid out per length
    int64_t dcount = 0, ccount = 0, icount = 0;
    struct RootReq { int64_t off, den, count, stride; };
    std::vector<RootReq> roots;
    std::vector<std::pair<int64_t, int64_t>> sins;  // (offset, N)
    auto add_sub = [&](SubFft& f) {
        f.tw_off = (int32_t)ccount;
        int64_t ns = 1;
        for (int i = 0; i < f.nrad; ++i) {
            roots.push_back({ccount, ns * f.rad[i], ns, 1});
            ccount += ns;
            ns *= f.rad[i];
        }
    };
    for (auto& lp : p->lens) {
        lp.invN = 1.0 / (double)lp.N;
        lp.sin_off = dcount;
        sins.push_back({dcount, lp.N});
        dcount += lp.N / 2 + 1;
        lp.isin_off = dcount;
        dcount += lp.N / 2 + 1;
        add_sub(lp.f1);
        if (lp.spec_perm) {
            lp.bin_off = icount;
            icount += lp.N / 2 + 1;
            lp.pos_off = icount;
            icount += lp.N / 2 + 1;
        }
        if (lp.two_pass) {
            add_sub(lp.f2);
            lp.big_lo_off = ccount;
            roots.push_back({ccount, lp.N, lp.big_split, 1});
            ccount += lp.big_split;
            lp.big_hi_off = ccount;
            const int64_t nhi = (lp.N + lp.big_split - 1) / lp.big_split;
            roots.push_back({ccount, lp.N, nhi, lp.big_split});
            ccount += nhi;
        }
    }
    p->wshape_off = dcount;
    dcount += (int64_t)p->wshape.size();
    {
        // lambda_j's sines: tables while all of them fit the cache, else
        // both evaluated in place (FIF_LAMBDA_SINES=table|sin|both overrides)
        int64_t sin_bytes = 0;
        for (const auto& lp : p->lens) sin_bytes += (int64_t)sizeof(double) * (lp.N / 2 + 1);
        int inl = sin_bytes > kSinTableHotBytes ? 2 : 0;
        if (const char* env = getenv("FIF_LAMBDA_SINES")) {
            const std::string v(env);
            inl = v == "table" ? 0 : v == "sin" ? 1 : v == "both" ? 2 : inl;
        }
        for (auto& lp : p->lens) {
            lp.lam_inline = inl;
            lp.lam_pad = 0;
        }
    }

    // signals, work lists, workspace sizes
    int64_t off = 0, spec = 0, inter = 0, inter_max = 0, gscr = 0, resid = 0;
    bool any_odd = false, any_two_pass = false;
    p->fp32 = p->opt.precision == FIF_PREC_FP32;
    const size_t esz = p->fp32 ? sizeof(float2) : sizeof(double2);
    int32_t parts = 0, nbig = 0, btiles = 0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t N = lengths[b];
        const int32_t lid = len_id[N];
        const LenPlan& lp = p->lens[lid];
        SigDesc d;
        d.N = N;
        d.off = off;
        d.spec_off = spec;
        d.inter_off = lp.two_pass ? inter : 0;
        d.len_id = lid;
        d.part_off = parts;
        d.n_init_parts = (int32_t)((N + kFftCap - 1) / kFftCap);
        // run summaries per row tile, unless that would make too many of them:
        // then pass 2 writes the FP64 residual and k_count_resid summarizes it
        const bool use_resid = lp.two_pass && (N / lp.TR) > 65536;
        d.resid_off = use_resid ? resid : -1;
        if (use_resid) resid += N;
        d.n_parts = !lp.two_pass ? 1 : (use_resid ? d.n_init_parts : (int32_t)(N / lp.TR));
        d.bs = -1;
        d.bt_off = 0;
        d.n_btiles = 0;
        d.gs_off = 0;
        d.p1_off = (int32_t)p->w_p1.size();
        if (N / 2 > (int64_t)kScanBins) {
            d.bs = nbig++;
            d.bt_off = btiles;
            d.n_btiles = (int32_t)((N / 2 + kBigTile - 1) / kBigTile);
            btiles += d.n_btiles;
            d.gs_off = gscr;
            gscr += 3 * (N / 2);
        }
        p->sigs.push_back(d);
        off += N;
        spec += N / 2 + 1;
        if (lp.two_pass) {
            inter += N;
            inter_max = std::max(inter_max, inter);
        }
        parts += std::max(d.n_parts, d.n_init_parts);
        for (int32_t t = 0; t < d.n_init_parts; ++t) p->w_init.push_back({b, t});
        if (use_resid)
            for (int32_t t = 0; t < d.n_init_parts; ++t) p->w_count.push_back({b, t});
        for (int32_t t = 0; t < d.n_btiles; ++t) p->w_btile.push_back({b, t});
        if (!lp.two_pass) {
            p->w_single.push_back({b, 0});
            p->lds_single = std::max(p->lds_single, (size_t)N * esz);
        } else {
            for (int32_t t = 0; t < lp.N1 / lp.TC; ++t) p->w_p1.push_back({b, t});
            for (int32_t t = 0; t < lp.N2 / lp.TR; ++t) p->w_p2.push_back({b, t});
            p->lds_p1 = std::max(p->lds_p1, (size_t)lp.TC * lp.N2 * esz);
            // pass 2 also lays the FP64 residual out at a row stride of TR + 1
            p->lds_p2 = std::max(p->lds_p2, std::max((size_t)lp.TR * lp.N1 * esz,
                                                     (size_t)(lp.TR + 1) * lp.N1 * sizeof(double)));
            if ((int64_t)lp.TC * lp.N2 > kTileCap || (int64_t)lp.TR * lp.N1 > kTileCap) p->wide = true;
            bool r248 = true;
            for (int i = 0; i < lp.f1.nrad; ++i) r248 = r248 && (lp.f1.rad[i] == 2 || lp.f1.rad[i] == 4 || lp.f1.rad[i] == 8);
            for (int i = 0; i < lp.f2.nrad; ++i) r248 = r248 && (lp.f2.rad[i] == 2 || lp.f2.rad[i] == 4 || lp.f2.rad[i] == 8);
            if (!r248) any_odd = true;
            any_two_pass = true;
        }
        if (d.bs < 0)
            p->scan_small.push_back(b);
        else
            p->scan_big.push_back(b);
    }

    inter = inter_max;
    p->pow2 = any_two_pass && !any_odd;

    // signal groups of about equal sample counts
    {
        const char* env = getenv("FIF_GROUPS");
        int G = env ? atoi(env) : 4;
        G = std::max(1, std::min(G, std::min(B, 8)));
        int64_t total = 0;
        for (int32_t b = 0; b < B; ++b) total += lengths[b];
        auto sub = [](const std::vector<Work>& v, int32_t s0, int32_t s1) {
            fif_plan::Range r;
            const auto lo = std::lower_bound(v.begin(), v.end(), s0, [](const Work& w, int32_t s) { return w.sig < s; });
            const auto hi = std::lower_bound(v.begin(), v.end(), s1, [](const Work& w, int32_t s) { return w.sig < s; });
            r.begin = (int32_t)(lo - v.begin());
            r.count = (int32_t)(hi - lo);
            return r;
        };
        auto subi = [](const std::vector<int32_t>& v, int32_t s0, int32_t s1) {
            fif_plan::Range r;
            const auto lo = std::lower_bound(v.begin(), v.end(), s0);
            const auto hi = std::lower_bound(v.begin(), v.end(), s1);
            r.begin = (int32_t)(lo - v.begin());
            r.count = (int32_t)(hi - lo);
            return r;
        };
        auto make_group = [&](int32_t s0, int32_t s1) {
            fif_plan::Group g;
            g.s0 = s0;
            g.s1 = s1;
            g.single = sub(p->w_single, s0, s1);
            g.p1 = sub(p->w_p1, s0, s1);
            g.p2 = sub(p->w_p2, s0, s1);
            g.btile = sub(p->w_btile, s0, s1);
            g.count = sub(p->w_count, s0, s1);
            g.ssmall = subi(p->scan_small, s0, s1);
            g.sbig = subi(p->scan_big, s0, s1);
            for (int32_t i = 0; i < g.ssmall.count; ++i) {
                const bool tp = p->lens[p->sigs[p->scan_small[g.ssmall.begin + i]].len_id].two_pass != 0;
                g.small_two_pass = g.small_two_pass || tp;
                g.small_one_pass = g.small_one_pass || !tp;
            }
            for (int32_t i = 0; i < g.sbig.count; ++i) {
                const bool dfr = p->sigs[p->scan_big[g.sbig.begin + i]].n_btiles <= kBigDeferTiles;
                g.big_defer_any = g.big_defer_any || dfr;
                g.big_defer_all = g.big_defer_all && dfr;
            }
            return g;
        };
        p->all = make_group(0, B);
        int32_t s0 = 0;
        int64_t acc = 0;
        for (int g = 0; g < G && s0 < B; ++g) {
            int32_t s1 = s0;
            const int64_t target = total * (g + 1) / G;
            while (s1 < B && (s1 == s0 || acc + lengths[s1] <= target || g == G - 1)) acc += lengths[s1++];
            p->groups.push_back(make_group(s0, s1));
            s0 = s1;
        }
    }

    size_t ws = 0;
    p->ws_state = ws = align_up(ws, 256);
    ws += sizeof(SigState) * (size_t)B;
    p->ws_spec0 = ws = align_up(ws, 256);
    ws += sizeof(double2) * (size_t)spec;
    p->ws_spec1 = ws = align_up(ws, 256);
    ws += sizeof(double2) * (size_t)spec;
    p->ws_inter = ws = align_up(ws, 256);
    ws += sizeof(double2) * (size_t)inter;
    p->ws_parts = ws = align_up(ws, 256);
    ws += sizeof(RunState) * (size_t)parts;
    p->ws_psum = ws = align_up(ws, 256);
    ws += sizeof(double) * (size_t)parts;
    p->ws_gscr = ws = align_up(ws, 256);
    ws += sizeof(float) * (size_t)gscr;
    p->ws_bigs = ws = align_up(ws, 256);
    ws += sizeof(BigScan) * (size_t)nbig;
    p->ws_bpart = ws = align_up(ws, 256);
    ws += sizeof(double) * 2 * kBigCand * (size_t)btiles;
    p->ws_bqmax = ws = align_up(ws, 256);
    ws += sizeof(double) * (size_t)btiles;
    p->ws_resid = ws = align_up(ws, 256);
    ws += sizeof(double) * (size_t)resid;
    p->ws_feat = ws = align_up(ws, 256);
    ws += sizeof(uint16_t) * (size_t)kNetFeat * kNetCin0 * (size_t)B;
    p->ws_prop = ws = align_up(ws, 256);
    ws += sizeof(int64_t) * (size_t)B;
    p->ws_chk = ws = align_up(ws, 256);
    ws += sizeof(double) * 4 * (p->w_p1.size() + 1);
    if (!p->wshape.empty()) {
        p->ws_taps = ws = align_up(ws, 256);
        ws += sizeof(double) * (size_t)off;
        p->ws_lam = ws = align_up(ws, 256);
        ws += sizeof(double) * (size_t)spec;
        p->ws_wsum = ws = align_up(ws, 256);
        ws += sizeof(double) * (size_t)B;
    }
    {
        const char* env = getenv("FIF_DEBUG_MT_SHIFT");
        p->mt_shift = env ? atoi(env) : 0;
    }
    p->ws_total = align_up(ws, 256);

    // metadata upload
    size_t mo = 0;
    size_t o_sigs = (mo = align_up(mo, 256));
    mo += sizeof(SigDesc) * p->sigs.size();
    size_t o_lens = (mo = align_up(mo, 256));
    mo += sizeof(LenPlan) * p->lens.size();
    size_t o_init = (mo = align_up(mo, 256));
    mo += sizeof(Work) * p->w_init.size();
    size_t o_single = (mo = align_up(mo, 256));
    mo += sizeof(Work) * p->w_single.size();
    size_t o_p1 = (mo = align_up(mo, 256));
    mo += sizeof(Work) * p->w_p1.size();
    size_t o_p2 = (mo = align_up(mo, 256));
    mo += sizeof(Work) * p->w_p2.size();
    size_t o_ss = (mo = align_up(mo, 256));
    mo += sizeof(int32_t) * p->scan_small.size();
    size_t o_sb = (mo = align_up(mo, 256));
    mo += sizeof(int32_t) * p->scan_big.size();
    size_t o_bt = (mo = align_up(mo, 256));
    mo += sizeof(Work) * p->w_btile.size();
    size_t o_ct = (mo = align_up(mo, 256));
    mo += sizeof(Work) * p->w_count.size();
    mo = align_up(mo, 256);
    std::vector<char> host(mo, 0);
    if (hipMalloc(&p->dmeta.p, mo) != hipSuccess) return fail(FIF_ERR_NOMEM, "plan metadata allocation failed");
    char* db = (char*)p->dmeta.p;
    p->d_sigs = upload(db, o_sigs, p->sigs, host);
    p->d_lens = upload(db, o_lens, p->lens, host);
    p->d_init = upload(db, o_init, p->w_init, host);
    p->d_single = upload(db, o_single, p->w_single, host);
    p->d_p1 = upload(db, o_p1, p->w_p1, host);
    p->d_p2 = upload(db, o_p2, p->w_p2, host);
    p->d_scan_small = upload(db, o_ss, p->scan_small, host);
    p->d_scan_big = upload(db, o_sb, p->scan_big, host);
    p->d_btile = upload(db, o_bt, p->w_btile, host);
    p->d_count = upload(db, o_ct, p->w_count, host);
    HIP_TRY(hipMemcpy(p->dmeta.p, host.data(), mo, hipMemcpyHostToDevice));

    // tables, computed on the device in FP64
    const size_t c_at = align_up(sizeof(double) * (size_t)dcount, 256);
    const size_t i_at = align_up(c_at + sizeof(double2) * (size_t)ccount, 256);
    const size_t tab_bytes = i_at + sizeof(int32_t) * (size_t)icount + 256;
    if (hipMalloc(&p->dtabs.p, tab_bytes) != hipSuccess) return fail(FIF_ERR_NOMEM, "plan table allocation failed");
    p->d_dtab = (double*)p->dtabs.p;
    p->d_ctab = (double2*)((char*)p->dtabs.p + c_at);
    p->d_itab = (int32_t*)((char*)p->dtabs.p + i_at);
    for (size_t i = 0; i < p->lens.size(); ++i) {
        const LenPlan& lp = p->lens[i];
        if (!lp.spec_perm) continue;
        const int64_t cnt = lp.N / 2 + 1;
        k_fill_specmap<<<(unsigned)((cnt + 255) / 256), 256>>>(p->d_lens + i, p->d_itab);
    }
    for (auto& s : sins) {
        const int64_t cnt = s.second / 2 + 1;
        k_fill_sin<<<(unsigned)((cnt + 255) / 256), 256>>>(p->d_dtab + s.first, s.second, cnt);
        k_fill_isin<<<(unsigned)((cnt + 255) / 256), 256>>>(p->d_dtab + s.first + cnt, s.second, cnt);
    }
    for (auto& r : roots) {
        if (r.count <= 0) continue;
        k_fill_roots<<<(unsigned)((r.count + 255) / 256), 256>>>(p->d_ctab + r.off, r.den, r.count, r.stride);
    }
    if (!p->wshape.empty())
        HIP_TRY(hipMemcpy(p->d_dtab + p->wshape_off, p->wshape.data(), sizeof(double) * p->wshape.size(),
                          hipMemcpyHostToDevice));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipDeviceSynchronize());
    *out = p.release();
    return FIF_OK;
}

}  // namespace

extern "C" {

fif_status fif_plan_create(fif_plan** out, const int64_t* lengths, int32_t B, int32_t max_imfs,
                           const fif_options* opt_in)
{
    return create_plan(out, lengths, B, max_imfs, opt_in, nullptr);
}

fif_status fif_plan_workspace_size(const fif_plan* plan, size_t* bytes)
{
    if (!plan || !bytes) return fail(FIF_ERR_INVALID_ARG, "null argument");
    *bytes = plan->ws_total;
    return FIF_OK;
}

fif_status fif_plan_destroy(fif_plan* plan)
{
    delete plan;
    return FIF_OK;
}

}  // extern "C"

namespace {

hipEvent_t take_event(fif_plan* p)
{
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records events around one launch when profiling is on.
struct Timed {
    fif_plan* p;
    hipStream_t s;
    fif_plan::Rec r;
    bool on;
    Timed(const fif_plan* pc, const char* kind, hipStream_t st) : p(const_cast<fif_plan*>(pc)), s(st), on(pc->prof)
    {
        if (!on) return;
        int id = -1;
        for (size_t i = 0; i < p->kinds.size(); ++i)
            if (p->kinds[i] == kind) id = (int)i;
        if (id < 0) {
            id = (int)p->kinds.size();
            p->kinds.push_back(kind);
        }
        r.kind = id;
        r.a = take_event(p);
        r.b = take_event(p);
        if (!r.a || !r.b) {
            on = false;
            return;
        }
        (void)hipEventRecord(r.a, s);
    }
    ~Timed()
    {
        if (!on) return;
        (void)hipEventRecord(r.b, s);
        p->recs.push_back(r);
    }
};

struct Bound {
    StepArgs sa;
    ScanArgs sc;
    SigState* state;
};

Bound bind(const fif_plan* p, void* ws, double delta, fif_imf_info* info)
{
    char* w = (char*)ws;
    Bound b;
    b.state = (SigState*)(w + p->ws_state);
    StepArgs& A = b.sa;
    A.sigs = p->d_sigs;
    A.lens = p->d_lens;
    A.work = nullptr;
    A.st = b.state;
    A.dtab = p->d_dtab;
    A.ctab = p->d_ctab;
    A.itab = p->d_itab;
    A.gamma = p->opt.gamma;
    A.chk = (double*)(w + p->ws_chk);
    A.lam = p->wshape.empty() ? nullptr : (double*)(w + p->ws_lam);
    A.wsum = p->wshape.empty() ? nullptr : (double*)(w + p->ws_wsum);
    A.spec0 = (double2*)(w + p->ws_spec0);
    A.spec1 = (double2*)(w + p->ws_spec1);
    A.inter = (double2*)(w + p->ws_inter);
    A.parts = (RunState*)(w + p->ws_parts);
    A.resid = (double*)(w + p->ws_resid);
    A.t = 0;
    A.max_imfs = p->max_imfs;
    ScanArgs& S = b.sc;
    S.sigs = p->d_sigs;
    S.lens = p->d_lens;
    S.list = nullptr;
    S.st = b.state;
    S.parts = A.parts;
    S.psum = (const double*)(w + p->ws_psum);
    S.dtab = p->d_dtab;
    S.itab = p->d_itab;
    S.spec0 = A.spec0;
    S.spec1 = A.spec1;
    S.gscr = (float*)(w + p->ws_gscr);
    S.bigs = (BigScan*)(w + p->ws_bigs);
    S.bpart = (double*)(w + p->ws_bpart);
    S.bqmax = (double*)(w + p->ws_bqmax);
    S.info = info;
    S.prop = nullptr;
    S.t = 0;
    S.max_imfs = p->max_imfs;
    S.delta = delta;
    S.mask_rule = p->opt.mask_rule;
    S.nu = p->opt.nu;
    S.max_inner = p->opt.max_inner;
    S.floor_tau = p->opt.floor_tau;
    S.stop_mode = p->opt.stop_mode;
    S.chk = A.chk;
    S.lam = A.lam;
    S.defer = p->opt.stop_mode == 0 ? 1 : 0;
    S.redo_only = 0;
    S.mt_shift = p->mt_shift;
    return b;
}

// Four-step passes with the plan's tile size.
// (The outer steps' passes also have variants without the odd radices, for
// plans whose lengths need none.)
template <int MODE, typename T, bool REDO = false, typename C = double2>
void run_pass1(const fif_plan* p, unsigned grid, hipStream_t s, const StepArgs& A, const T* x)
{
    constexpr bool STEP = MODE == MODE_STEP;
    if (p->wide) {
        if (STEP && p->pow2)
            k_pass1<MODE, T, REDO, kTileCapBig, STEP, C><<<grid, kFftThreads, p->lds_p1, s>>>(A, x);
        else
            k_pass1<MODE, T, REDO, kTileCapBig, false, C><<<grid, kFftThreads, p->lds_p1, s>>>(A, x);
    } else {
        if (STEP && p->pow2)
            k_pass1<MODE, T, REDO, kTileCap, STEP, C><<<grid, kFftThreads, p->lds_p1, s>>>(A, x);
        else
            k_pass1<MODE, T, REDO, kTileCap, false, C><<<grid, kFftThreads, p->lds_p1, s>>>(A, x);
    }
}
template <int MODE, typename InT, typename OutT, typename C = double2>
void run_pass2(const fif_plan* p, unsigned grid, hipStream_t s, const StepArgs& A, const InT* x, OutT* imfs,
               OutT* rem)
{
    constexpr bool STEP = MODE == MODE_STEP;
    if (p->wide) {
        if (STEP && p->pow2)
            k_pass2<MODE, InT, OutT, kTileCapBig, STEP, C><<<grid, kFftThreads, p->lds_p2, s>>>(A, x, imfs, rem);
        else
            k_pass2<MODE, InT, OutT, kTileCapBig, false, C><<<grid, kFftThreads, p->lds_p2, s>>>(A, x, imfs, rem);
    } else {
        if (STEP && p->pow2)
            k_pass2<MODE, InT, OutT, kTileCap, STEP, C><<<grid, kFftThreads, p->lds_p2, s>>>(A, x, imfs, rem);
        else
            k_pass2<MODE, InT, OutT, kTileCap, false, C><<<grid, kFftThreads, p->lds_p2, s>>>(A, x, imfs, rem);
    }
}

template <typename T, typename C>
void launch_init_c(const fif_plan* p, Bound& b, const T* x, hipStream_t s)
{
    {
        Timed tm(p, "reset", s);
        k_reset_state<<<(p->B + 255) / 256, 256, 0, s>>>(b.state, p->B);
    }
    if (!p->w_init.empty()) {
        Timed tm(p, "init_stats", s);
        k_init_stats<T><<<(unsigned)p->w_init.size(), kFftThreads, 0, s>>>(p->d_sigs, p->d_init, x, b.sa.parts,
                                                                           (double*)b.sc.psum, b.state);
    }
    StepArgs A = b.sa;
    if (!p->w_single.empty()) {
        A.work = p->d_single;
        Timed tm(p, "single_fwd", s);
        k_single<MODE_FORWARD, T, T, C><<<(unsigned)p->w_single.size(), kFftThreads, p->lds_single, s>>>(A, x, nullptr,
                                                                                                        nullptr);
    }
    if (!p->w_p1.empty()) {
        A.work = p->d_p1;
        {
            Timed tm(p, "pass1_fwd", s);
            run_pass1<MODE_FORWARD, T, false, C>(p, (unsigned)p->w_p1.size(), s, A, x);
        }
        A.work = p->d_p2;
        Timed tm(p, "pass2_fwd", s);
        run_pass2<MODE_FORWARD, T, T, C>(p, (unsigned)p->w_p2.size(), s, A, x, (T*)nullptr, (T*)nullptr);
    }
}
template <typename T>
void launch_init(const fif_plan* p, Bound& b, const T* x, hipStream_t s)
{
    if (p->fp32)
        launch_init_c<T, float2>(p, b, x, s);
    else
        launch_init_c<T, double2>(p, b, x, s);
}

template <bool PRE, typename C = double2>
void launch_k_scan(int mode, int n, size_t lds, hipStream_t s, const ScanArgs& S, const fif_plan::Group& g)
{
    constexpr unsigned TG = kScanBins / kScanBinsPerThread, TD = kScanBins / kScanBinsDeferred;
    if (mode == 1) {
        k_scan<kScanBinsPerThread, PRE, 1, C><<<(unsigned)n, TG, lds, s>>>(S);
    } else if (mode == 2) {
        k_scan<kScanBinsPerThread, PRE, 2, C><<<(unsigned)n, TG, lds, s>>>(S);
    } else if (S.defer && !S.redo_only && !g.small_one_pass) {
        // four-step signals only: the FP32 search (their FP64 check is in
        // pass 1), in the kernel without the FP64 search
        k_scan<kScanBinsDeferred, PRE, 0, C, true><<<(unsigned)n, TD, lds, s>>>(S);
    } else {
        k_scan<kScanBinsPerThread, PRE, 0, C><<<(unsigned)n, TG, lds, s>>>(S);
    }
}

// Eigenvalue tables of a sampled window shape for the active signals of one
// group, at the L the step start just fixed: folded taps, their forward
// transform, lambda_j = (H_j / H_0)^2.
void launch_window(const fif_plan* p, Bound& b, void* ws, hipStream_t s, const fif_plan::Group& g)
{
    Timed tm(p, "window", s);
    double* taps = (double*)((char*)ws + p->ws_taps);
    k_window_taps<<<(unsigned)(g.s1 - g.s0), kFftThreads, 0, s>>>(p->d_sigs, b.state, p->d_dtab + p->wshape_off,
                                                                  (int)p->wshape.size() - 1, taps, b.sa.wsum, g.s0);
    StepArgs A = b.sa;
    if (g.single.count) {
        A.work = p->d_single + g.single.begin;
        k_single<MODE_WINDOW, double, double><<<(unsigned)g.single.count, kFftThreads, p->lds_single, s>>>(
            A, taps, nullptr, nullptr);
    }
    if (g.p1.count) {
        A.work = p->d_p1 + g.p1.begin;
        run_pass1<MODE_WINDOW, double>(p, (unsigned)g.p1.count, s, A, (const double*)taps);
        A.work = p->d_p2 + g.p2.begin;
        run_pass2<MODE_WINDOW, double, double>(p, (unsigned)g.p2.count, s, A, (const double*)taps, (double*)nullptr,
                                               (double*)nullptr);
    }
}

// Search for m of every active signal.  With a proposal model or feature
// recording the step starts (count combine, stop rules, L) run first, then
// the features, the network and the proposals, then the searches.
template <typename C>
void launch_scan(const fif_plan* p, Bound& b, int t, void* ws, hipStream_t s, const fif_plan::Group& g)
{
    ScanArgs S = b.sc;
    S.t = t;
    const bool split = p->model || p->rec || !p->wshape.empty();
    const unsigned nb = (unsigned)g.sbig.count, nt = (unsigned)g.btile.count;
    const Work* btile = p->d_btile + g.btile.begin;
    const size_t scan_lds = sizeof(float) * kScanBins;
    if (p->opt.mask_rule == 2) {
        Timed tm(p, "peak", s);
        k_peak<C><<<(unsigned)(g.s1 - g.s0), 256, 0, s>>>(S, g.s0, p->opt.peak_rho);
    }
    if (!split) {
        if (g.ssmall.count) {
            S.list = p->d_scan_small + g.ssmall.begin;
            Timed tm(p, "scan", s);
            launch_k_scan<false, C>(p->opt.stop_mode, g.ssmall.count, scan_lds, s, S, g);
        }
        if (nb) {
            Timed tm(p, "scan_big", s);
            S.list = p->d_scan_big + g.sbig.begin;
            k_bscan_prep<kScanThreads><<<nb, kScanThreads, 0, s>>>(S);
        }
    } else {
        {
            Timed tm(p, "scan_prologue", s);
            if (g.ssmall.count) {
                S.list = p->d_scan_small + g.ssmall.begin;
                k_scan_prologue<kScanThreads><<<(unsigned)g.ssmall.count, kScanThreads, 0, s>>>(S);
            }
            if (nb) {
                S.list = p->d_scan_big + g.sbig.begin;
                k_bscan_prep<kScanThreads><<<nb, kScanThreads, 0, s>>>(S);
            }
        }
        if (!p->wshape.empty()) launch_window(p, b, ws, s, g);
        char* w = (char*)ws;
        uint16_t* feat = (uint16_t*)(w + p->ws_feat);
        int64_t* prop = (int64_t*)(w + p->ws_prop);
        if (p->model || p->rec) {
            Timed tm(p, "features", s);
            FeatArgs F;
            F.sigs = p->d_sigs;
            F.lens = p->d_lens;
            F.itab = p->d_itab;
            F.st = S.st;
            F.spec0 = S.spec0;
            F.spec1 = S.spec1;
            F.t = t;
            F.out = feat;
            F.rec = p->rec;
            F.max_imfs = p->max_imfs;
            F.s0 = g.s0;
            k_features<<<(unsigned)(g.s1 - g.s0), kNetThreads, 0, s>>>(F);
        }
        if (p->model) {
            Timed tm(p, "propose", s);
            const int mb = model_max_batch(p->model);
            for (int s0 = g.s0; s0 < g.s1; s0 += mb) {
                const int n = std::min(mb, g.s1 - s0);
                const float* y = model_infer(p->model, feat + (size_t)s0 * kNetFeat * kNetCin0, n, s);
                k_propose<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(y, s0, n, p->opt.max_inner, S.st, prop);
            }
            S.prop = prop;
        }
        if (g.ssmall.count) {
            S.list = p->d_scan_small + g.ssmall.begin;
            Timed tm(p, "scan", s);
            launch_k_scan<true, C>(p->opt.stop_mode, g.ssmall.count, scan_lds, s, S, g);
        }
        if (nb && p->model) {
            S.list = p->d_scan_big + g.sbig.begin;
            k_bscan_seed<<<nb, 64, 0, s>>>(S);
        }
    }
    if (nb) {
        Timed tm(p, "scan_big", s);
        S.list = p->d_scan_big + g.sbig.begin;
        // stop mode 0 hands the FP32 estimates to pass 1's check: when every
        // signal of the group defers, the rounds are FP32 rounds only; else
        // each round is an FP32 and an FP64 kernel, each working on the
        // signals in its own phase (one decide after both)
        const bool fp32_only = p->opt.stop_mode == 0 && S.defer && g.big_defer_all;
        k_bscan_round<kScanThreads, true, C, 1><<<nt, kScanThreads, 0, s>>>(S, btile);
        k_bscan_decide<C><<<nb, 64 * kDecideGroups, 0, s>>>(S);
        for (int r = 0; r < kBigRounds; ++r) {
            k_bscan_round<kScanThreads, false, C, 1><<<nt, kScanThreads, 0, s>>>(S, btile);
            if (!fp32_only) k_bscan_round<kScanThreads, false, C, 2><<<nt, kScanThreads, 0, s>>>(S, btile);
            k_bscan_decide<C><<<nb, 64 * kDecideGroups, 0, s>>>(S);
        }
        k_bscan_final<kScanThreads><<<nb, 64, 0, s>>>(S);
    }
}

template <typename T, typename C>
void launch_step_c(const fif_plan* p, Bound& b, int t, const T* x, T* imfs, void* ws, hipStream_t s,
                   const fif_plan::Group& g)
{
    launch_scan<C>(p, b, t, ws, s, g);
    StepArgs A = b.sa;
    A.t = t;
    if (g.single.count) {
        A.work = p->d_single + g.single.begin;
        Timed tm(p, "single_step", s);
        k_single<MODE_STEP, T, T, C><<<(unsigned)g.single.count, kFftThreads, p->lds_single, s>>>(A, x, imfs, nullptr);
    }
    if (g.p1.count) {
        A.work = p->d_p1 + g.p1.begin;
        {
            Timed tm(p, "pass1_step", s);
            run_pass1<MODE_STEP, T, false, C>(p, (unsigned)g.p1.count, s, A, x);
        }
        const unsigned nb = g.big_defer_any ? (unsigned)g.sbig.count : 0u, nt = (unsigned)g.btile.count;
        if (b.sc.defer && (g.ssmall.count || nb)) {
            // deferred FP64 check of m, then the rare redo: exact search and
            // pass 1 again for the signals whose check failed
            Timed tm(p, "verify", s);
            ScanArgs V = b.sc;
            V.t = t;
            const int32_t* small = p->d_scan_small + g.ssmall.begin;
            const int32_t* big = p->d_scan_big + g.sbig.begin;
            if (g.ssmall.count) {
                V.list = small;
                k_verify<<<(unsigned)((g.ssmall.count + 63) / 64), 64, 0, s>>>(V, g.ssmall.count);
            }
            if (nb) {
                V.list = big;
                k_verify<<<(nb + 63) / 64, 64, 0, s>>>(V, (int)nb);
            }
            V.redo_only = 1;
            if (g.ssmall.count) {
                // the FP64 search from each rejected estimate (no FP32 state:
                // the grid's other workgroups, returning at once, need no LDS)
                V.list = small;
                k_scan<kScanBinsRedo, true, 0, C, false, true>
                    <<<(unsigned)g.ssmall.count, kScanBins / kScanBinsRedo, 0, s>>>(V);
            }
            if (nb) {
                // FP64 rounds of the multi-workgroup search for the signals
                // whose check failed (the others return at once)
                V.list = big;
                const Work* btile = p->d_btile + g.btile.begin;
                k_bscan_redo_prep<<<nb, 64, 0, s>>>(V);
                for (int r = 0; r < kBigRedoRounds; ++r) {
                    k_bscan_round<kScanThreads, false, C, 2><<<nt, kScanThreads, 0, s>>>(V, btile);
                    k_bscan_decide<C><<<nb, 64 * kDecideGroups, 0, s>>>(V);
                }
                k_bscan_final<kScanThreads><<<nb, 64, 0, s>>>(V);
            }
            run_pass1<MODE_STEP, T, true, C>(p, (unsigned)g.p1.count, s, A, x);
        }
        A.work = p->d_p2 + g.p2.begin;
        Timed tm(p, "pass2_step", s);
        run_pass2<MODE_STEP, T, T, C>(p, (unsigned)g.p2.count, s, A, x, imfs, (T*)nullptr);
    }
    if (g.count.count) {
        Timed tm(p, "count_resid", s);
        k_count_resid<<<(unsigned)g.count.count, kFftThreads, 0, s>>>(p->d_sigs, p->d_count + g.count.begin, A.resid,
                                                                       A.parts, A.st);
    }
}
template <typename T>
void launch_step(const fif_plan* p, Bound& b, int t, const T* x, T* imfs, void* ws, hipStream_t s,
                 const fif_plan::Group& g)
{
    if (p->fp32)
        launch_step_c<T, float2>(p, b, t, x, imfs, ws, s, g);
    else
        launch_step_c<T, double2>(p, b, t, x, imfs, ws, s, g);
}

template <typename T, typename C>
void launch_final_c(const fif_plan* p, Bound& b, const T* x, T* rem, int32_t* n_imfs, int32_t* sig_status,
                    fif_imf_info* info, hipStream_t s)
{
    {
        Timed tm(p, "finalize", s);
        k_finalize<<<(p->B + 255) / 256, 256, 0, s>>>(b.state, p->B, p->max_imfs, n_imfs, sig_status, info);
    }
    StepArgs A = b.sa;
    if (!p->w_single.empty()) {
        A.work = p->d_single;
        Timed tm(p, "single_rem", s);
        k_single<MODE_REMAINDER, T, T, C><<<(unsigned)p->w_single.size(), kFftThreads, p->lds_single, s>>>(A, x, nullptr,
                                                                                                          rem);
    }
    if (!p->w_p1.empty()) {
        A.work = p->d_p1;
        {
            Timed tm(p, "pass1_rem", s);
            run_pass1<MODE_REMAINDER, T, false, C>(p, (unsigned)p->w_p1.size(), s, A, x);
        }
        A.work = p->d_p2;
        Timed tm(p, "pass2_rem", s);
        run_pass2<MODE_REMAINDER, T, T, C>(p, (unsigned)p->w_p2.size(), s, A, x, (T*)nullptr, rem);
    }
}
template <typename T>
void launch_final(const fif_plan* p, Bound& b, const T* x, T* rem, int32_t* n_imfs, int32_t* sig_status,
                  fif_imf_info* info, hipStream_t s)
{
    if (p->fp32)
        launch_final_c<T, float2>(p, b, x, rem, n_imfs, sig_status, info, s);
    else
        launch_final_c<T, double2>(p, b, x, rem, n_imfs, sig_status, info, s);
}

// Streams and events of the signal groups (created once per plan).
fif_status group_streams(fif_plan* p)
{
    const int G = (int)p->groups.size();
    while ((int)p->gstreams.size() < G - 1) {
        hipStream_t st = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        p->gstreams.push_back(st);
        hipEvent_t ev = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        p->ev_join.push_back(ev);
    }
    if (!p->ev_fork) HIP_TRY(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    return FIF_OK;
}

// one_stream: every signal group on the caller's stream (no group streams or
// events are created), for the entry point that allocates nothing.
template <typename T>
fif_status batched(fif_plan* p, const T* x, double delta, T* imfs, T* rem, int32_t* n_imfs, fif_imf_info* info,
                   int32_t* sig_status, void* ws, void* stream, bool one_stream = false)
{
    g_err.clear();
    if (!p) return fail(FIF_ERR_INVALID_ARG, "plan is null");
    if (!x || !imfs || !rem || !n_imfs || !ws) return fail(FIF_ERR_INVALID_ARG, "null buffer argument");
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(FIF_ERR_INVALID_ARG, "delta must be > 0 and finite");
    if (((uintptr_t)ws) % 256) return fail(FIF_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != p->device) return fail(FIF_ERR_INVALID_ARG, "plan was created on device %d, current is %d", p->device, dev);
    hipStream_t s = (hipStream_t)stream;
    Bound b = bind(p, ws, delta, info);
    launch_init<T>(p, b, x, s);
    // outer steps: one stream per signal group (forked from and joined back
    // to the caller's stream); a single group when the proposal network or
    // feature recording is on (they share buffers across signals) or while
    // profiling (each kernel then runs alone and its events time it alone)
    const int G = (p->model || p->rec || p->prof || one_stream) ? 1 : (int)p->groups.size();
    if (G <= 1) {
        for (int t = 0; t < p->max_imfs; ++t) launch_step<T>(p, b, t, x, imfs, ws, s, p->all);
    } else {
        fif_status gs = group_streams(p);
        if (gs != FIF_OK) return gs;
        HIP_TRY(hipEventRecord(p->ev_fork, s));
        for (int g = 1; g < G; ++g) HIP_TRY(hipStreamWaitEvent(p->gstreams[g - 1], p->ev_fork, 0));
        for (int t = 0; t < p->max_imfs; ++t)
            for (int g = 0; g < G; ++g)
                launch_step<T>(p, b, t, x, imfs, ws, g == 0 ? s : p->gstreams[g - 1], p->groups[g]);
        for (int g = 1; g < G; ++g) {
            HIP_TRY(hipEventRecord(p->ev_join[g - 1], p->gstreams[g - 1]));
            HIP_TRY(hipStreamWaitEvent(s, p->ev_join[g - 1], 0));
        }
    }
    launch_final<T>(p, b, x, rem, n_imfs, sig_status, info, s);
    HIP_TRY(hipGetLastError());
    return FIF_OK;
}

// ------------------------------------------------------------- autotuner

// Synthetic input of the timing runs: three tones per signal plus a small
// deterministic perturbation (any input with several IMFs will do).
__global__ void k_tune_signal(float* __restrict__ x, int64_t total, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t n = i % N;
    const double u = (double)n / (double)N;
    const uint32_t h = (uint32_t)(i * 2654435761u);
    x[i] = (float)(sinpi(2.0 * 3.0 * u) + 0.5 * sinpi(2.0 * (double)(N / 64) * u) +
                   0.25 * sinpi(2.0 * (double)(N / 7) * u) + 1e-3 * ((double)(h >> 8) / 16777216.0 - 0.5));
}

// Largest divisor of n that is at most cap (>= 1).
int64_t divisor_at_most(int64_t n, int64_t cap) { return largest_divisor_at_most(n, std::max<int64_t>(1, cap)); }

// Candidate choices for a two-pass length: the three most balanced splits
// (and the most balanced even-even one), the widest pass-1 / pass-2 tiles and
// half of each (and the widest even pass-1 tile), the built-in radix order
// and its reverse.  The built-in choice comes first.
std::vector<fif_length_plan> tune_candidates(int64_t N)
{
    std::vector<fif_length_plan> out;
    LenPlan lp0;
    if (plan_length(N, lp0) != FIF_OK || !lp0.two_pass) return out;
    out.push_back(choice_of(lp0));
    std::vector<std::pair<int64_t, int64_t>> splits;   // (N1, N2)
    for (int64_t n2 = 2; n2 <= kTileCap; ++n2) {
        if (N % n2) continue;
        const int64_t n1 = N / n2;
        if (n1 < 2 || n1 > kTileCap) continue;
        splits.push_back({n1, n2});
    }
    std::sort(splits.begin(), splits.end(), [](const std::pair<int64_t, int64_t>& a, const std::pair<int64_t, int64_t>& b) {
        const int64_t ma = std::max(a.first, a.second), mb = std::max(b.first, b.second);
        return ma != mb ? ma < mb : a.second > b.second;
    });
    // the most balanced split whose factors are both even (mirror-paired
    // pass-1 tiles need it) joins the three most balanced ones
    auto even = [](const std::pair<int64_t, int64_t>& sp) { return sp.first % 2 == 0 && sp.second % 2 == 0; };
    const auto ev = std::find_if(splits.begin(), splits.end(), even);
    const bool add_even = ev != splits.end() && std::none_of(splits.begin(), splits.begin() + std::min<size_t>(3, splits.size()), even);
    const std::pair<int64_t, int64_t> even_split = add_even ? *ev : std::pair<int64_t, int64_t>(0, 0);
    if (splits.size() > 3) splits.resize(3);
    if (add_even) splits.push_back(even_split);
    for (const auto& sp : splits) {
        const int64_t N1 = sp.first, N2 = sp.second;
        SubFft f1, f2;
        if (!make_subfft(N2, f1) || !make_subfft(N1, f2)) continue;
        const int64_t tc0 = divisor_at_most(N1, kTileCap / N2), tr0 = divisor_at_most(N2, kTileCap / N1);
        // pass-1 tile widths: the widest, half of it, and the widest even one
        // (paired tiles) when both factors are even
        int64_t tce = 0;
        if (even(sp))
            for (int64_t t = kTileCap / N2; t >= 2; --t)
                if (t % 2 == 0 && N1 % t == 0) {
                    tce = t;
                    break;
                }
        const int64_t tcs[3] = {tc0, divisor_at_most(N1, tc0 / 2), tce};
        const int64_t trs[2] = {tr0, divisor_at_most(N2, tr0 / 2)};
        for (int rev = 0; rev < 2; ++rev)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 2; ++b) {
                    if ((a == 1 && tcs[1] == tcs[0]) || (b == 1 && trs[1] == trs[0])) continue;
                    if (a == 2 && (tcs[2] == 0 || tcs[2] == tcs[0] || tcs[2] == tcs[1])) continue;
                    fif_length_plan c;
                    std::memset(&c, 0, sizeof(c));
                    c.N = N;
                    c.N1 = (int32_t)N1;
                    c.N2 = (int32_t)N2;
                    c.TC = (int32_t)tcs[a];
                    c.TR = (int32_t)trs[b];
                    c.n_rad1 = f1.nrad;
                    c.n_rad2 = f2.nrad;
                    for (int i = 0; i < f1.nrad; ++i) c.rad1[i] = f1.rad[rev ? f1.nrad - 1 - i : i];
                    for (int i = 0; i < f2.nrad; ++i) c.rad2[i] = f2.rad[rev ? f2.nrad - 1 - i : i];
                    if (!choice_valid(c)) continue;
                    bool dup = false;
                    for (const auto& o : out)
                        dup = dup || std::memcmp(&o, &c, sizeof(c)) == 0;
                    if (!dup) out.push_back(c);
                }
    }
    return out;
}

// Microseconds of one decomposition (two IMFs) of a synthetic batch of
// length-N signals with choice c, best of three after one warm-up run;
// negative if the plan cannot be built or run.
double time_choice(const fif_length_plan& c, const fif_options& opt)
{
    const int64_t N = c.N;
    const int32_t Bt = (int32_t)std::max<int64_t>(1, std::min<int64_t>(256, ((int64_t)1 << 23) / N));
    const int32_t J = 2;
    std::vector<int64_t> lengths((size_t)Bt, N);
    ChoiceMap forced{{N, c}};
    fif_plan* tp = nullptr;
    if (create_plan(&tp, lengths.data(), Bt, J, &opt, &forced) != FIF_OK) return -1.0;
    std::unique_ptr<fif_plan> hold(tp);
    const int64_t total = (int64_t)Bt * N;
    const size_t bytes = tp->ws_total + sizeof(float) * (size_t)total * (J + 2) + 1024;
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) return -1.0;
    DevBuf buf;
    buf.p = mem;
    char* b = (char*)mem;
    void* ws = b;
    float* x = (float*)(b + align_up(tp->ws_total, 256));
    float* imfs = x + total;
    float* rem = imfs + total * J;
    int32_t* nimf = (int32_t*)(rem + total);
    k_tune_signal<<<(unsigned)((total + 255) / 256), 256>>>(x, total, N);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    double best = -1.0;
    for (int r = 0; r < 4; ++r) {
        (void)hipEventRecord(e0, nullptr);
        if (batched<float>(tp, x, 1e-3, imfs, rem, nimf, nullptr, nullptr, ws, nullptr) != FIF_OK) break;
        (void)hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r > 0 && (best < 0.0 || 1e3 * ms < best)) best = 1e3 * ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

std::string device_key()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::memset(&prop, 0, sizeof(prop));
    (void)hipGetDeviceProperties(&prop, dev);
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    return key_text(prop.gcnArchName) + "/hip" + std::to_string(rt);
}

// ------------------------------------------- entry point without allocation

// Workspace of fif_decompose_batched_static: a fixed array in the library's
// code object.  Every device the library runs on holds its own copy until
// the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[FIF_STATIC_WORKSPACE_BYTES];

struct ScratchAddrs {
    std::mutex mu;
    std::map<int, void*> ptr;      // device -> address of its copy of scratch
};
ScratchAddrs& scratch_addrs()
{
    static ScratchAddrs* a = new ScratchAddrs();
    return *a;
}

// Address of the current device's copy of scratch, looked up once per device.
fif_status scratch_ptr(int dev, void** out)
{
    auto& A = scratch_addrs();
    std::lock_guard<std::mutex> lock(A.mu);
    auto it = A.ptr.find(dev);
    if (it == A.ptr.end()) {
        void* q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q)
            return fail(FIF_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        it = A.ptr.emplace(dev, q).first;
    }
    *out = it->second;
    return FIF_OK;
}

// ------------------------------------------------ single-signal plain form

struct SingleCache {
    std::mutex mu;
    struct Entry {
        fif_plan* plan = nullptr;
        void* ws = nullptr;
        SigState* host_state = nullptr;
    };
    std::map<std::tuple<int, int64_t, int32_t, int32_t, double, int64_t, double, int32_t, double, double,
                        std::vector<double>, int32_t>,
             Entry>
        map;
    ~SingleCache() { clear(); }
    void clear()
    {
        for (auto& kv : map) {
            delete kv.second.plan;
            if (kv.second.ws) (void)hipFree(kv.second.ws);
            if (kv.second.host_state) (void)hipHostFree(kv.second.host_state);
        }
        map.clear();
    }
};
SingleCache& single_cache()
{
    static SingleCache* c = new SingleCache();
    return *c;
}

template <typename T>
fif_status single(const T* x, int64_t N, fif_window window, double delta, int32_t max_imfs, T* imfs, T* rem,
                  int32_t* n_imfs, fif_imf_info* info, const fif_options* opt_in, void* stream)
{
    g_err.clear();
    if (window != FIF_WINDOW_TRI2 && window != FIF_WINDOW_SAMPLED)
        return fail(FIF_ERR_INVALID_ARG, "unknown window %d", (int)window);
    if (!x || !imfs || !rem || !n_imfs) return fail(FIF_ERR_INVALID_ARG, "null buffer argument");
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(FIF_ERR_INVALID_ARG, "delta must be > 0 and finite");
    fif_options opt;
    fif_options_default(&opt);
    if (opt_in) opt = *opt_in;
    if ((window == FIF_WINDOW_SAMPLED) != (opt.window != nullptr))
        return fail(FIF_ERR_INVALID_ARG, "FIF_WINDOW_SAMPLED goes with window samples in the options, "
                                         "FIF_WINDOW_TRI2 without");
    fif_status vst = validate_opts(opt);
    if (vst) return vst;
    if (max_imfs < 1 || max_imfs > 4096) return fail(FIF_ERR_INVALID_ARG, "max_imfs must be in [1, 4096]");
    if (N < 2) return fail(FIF_ERR_INVALID_ARG, "length %lld < 2", (long long)N);
    if (!smooth7(N)) return fail(FIF_ERR_UNSUPPORTED_LENGTH, "length %lld has a prime factor > 7", (long long)N);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    auto& C = single_cache();
    std::lock_guard<std::mutex> lock(C.mu);
    std::vector<double> wkey;
    if (opt.window) wkey.assign(opt.window, opt.window + opt.window_points);
    auto key = std::make_tuple(dev, N, max_imfs, opt.mask_rule, opt.nu, opt.max_inner, opt.floor_tau, opt.stop_mode,
                               opt.gamma, opt.peak_rho, wkey, opt.precision);
    auto it = C.map.find(key);
    if (it == C.map.end()) {
        SingleCache::Entry e;
        fif_status st = fif_plan_create(&e.plan, &N, 1, max_imfs, &opt);
        if (st) return st;
        if (hipMalloc(&e.ws, e.plan->ws_total) != hipSuccess) {
            delete e.plan;
            return fail(FIF_ERR_NOMEM, "workspace allocation failed");
        }
        if (hipHostMalloc((void**)&e.host_state, sizeof(SigState), hipHostMallocDefault) != hipSuccess) {
            delete e.plan;
            (void)hipFree(e.ws);
            return fail(FIF_ERR_NOMEM, "pinned state allocation failed");
        }
        it = C.map.emplace(key, e).first;
    }
    fif_plan* p = it->second.plan;
    SigState* hs = it->second.host_state;
    hipStream_t s = (hipStream_t)stream;
    Bound b = bind(p, it->second.ws, delta, info);
    launch_init<T>(p, b, x, s);
    for (int t = 0; t < max_imfs; ++t) {
        launch_step<T>(p, b, t, x, imfs, it->second.ws, s, p->all);
        HIP_TRY(hipMemcpyAsync(hs, b.state, sizeof(SigState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!hs->active) {
            // zero the rows the remaining steps would have zeroed
            for (int u = t + 1; u < max_imfs; ++u)
                HIP_TRY(hipMemsetAsync(imfs + (int64_t)u * N, 0, sizeof(T) * (size_t)N, s));
            break;
        }
    }
    launch_final<T>(p, b, x, rem, n_imfs, nullptr, info, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(hs, b.state, sizeof(SigState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hs->status != 0) return fail(FIF_ERR_NONFINITE, "signal holds NaN or Inf");
    return FIF_OK;
}

// Capture-once, replay-many form of batched().
template <typename T>
fif_status batched_graph(fif_plan* plan, const T* signals, double delta, T* imfs, T* remainders, int32_t* n_imfs, fif_imf_info* info, int32_t* sig_status,
                                       void* workspace, void* stream)
{
    g_err.clear();
    if (!plan) return fail(FIF_ERR_INVALID_ARG, "plan is null");
    if (!stream) return fail(FIF_ERR_INVALID_ARG, "graph replay needs a non-null stream");
    if (plan->prof) return fail(FIF_ERR_INVALID_ARG, "graph replay is not available while profiling");
    uint64_t dbits;
    std::memcpy(&dbits, &delta, sizeof(dbits));
    const std::vector<uintptr_t> key = {(uintptr_t)signals, (uintptr_t)dbits,       (uintptr_t)imfs,
                                        (uintptr_t)remainders, (uintptr_t)n_imfs, (uintptr_t)info,
                                        (uintptr_t)sig_status, (uintptr_t)workspace, (uintptr_t)plan->model,
                                        (uintptr_t)plan->rec, (uintptr_t)sizeof(T)};
    hipStream_t s = (hipStream_t)stream;
    if (!plan->gexec || key != plan->gkey) {
        if (plan->gexec) {
            HIP_TRY(hipGraphExecDestroy(plan->gexec));
            plan->gexec = nullptr;
        }
        const fif_status gs = group_streams(plan);   // not inside the capture
        if (gs != FIF_OK) return gs;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const fif_status st = batched<T>(plan, signals, delta, imfs, remainders, n_imfs, info, sig_status,
                                             workspace, stream);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(s, &graph);
        if (st != FIF_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (ec != hipSuccess) return fail(FIF_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
        const hipError_t ei = hipGraphInstantiate(&plan->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            plan->gexec = nullptr;
            return fail(FIF_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
        }
        plan->gkey = key;
    }
    HIP_TRY(hipGraphLaunch(plan->gexec, s));
    return FIF_OK;
}

}  // namespace

extern "C" {

fif_status fif_decompose_batched(fif_plan* plan, const float* signals, double delta, float* imfs, float* remainders,
                                 int32_t* n_imfs, fif_imf_info* info, int32_t* sig_status, void* workspace,
                                 void* stream)
{
    return batched<float>(plan, signals, delta, imfs, remainders, n_imfs, info, sig_status, workspace, stream);
}

fif_status fif_decompose_batched_f64(fif_plan* plan, const double* signals, double delta, double* imfs,
                                     double* remainders, int32_t* n_imfs, fif_imf_info* info, int32_t* sig_status,
                                     void* workspace, void* stream)
{
    return batched<double>(plan, signals, delta, imfs, remainders, n_imfs, info, sig_status, workspace, stream);
}

fif_status fif_decompose_batched_graph(fif_plan* plan, const float* signals, double delta, float* imfs,
                                       float* remainders, int32_t* n_imfs, fif_imf_info* info, int32_t* sig_status,
                                       void* workspace, void* stream)
{
    return batched_graph<float>(plan, signals, delta, imfs, remainders, n_imfs, info, sig_status, workspace, stream);
}

fif_status fif_decompose_batched_graph_f64(fif_plan* plan, const double* signals, double delta, double* imfs,
                                           double* remainders, int32_t* n_imfs, fif_imf_info* info,
                                           int32_t* sig_status, void* workspace, void* stream)
{
    return batched_graph<double>(plan, signals, delta, imfs, remainders, n_imfs, info, sig_status, workspace, stream);
}

fif_status fif_decompose_batched_static(fif_plan* plan, const float* signals, double delta, float* imfs,
                                        float* remainders, int32_t* n_imfs, fif_imf_info* info,
                                        int32_t* sig_status, void* stream)
{
    g_err.clear();
    if (!plan) return fail(FIF_ERR_INVALID_ARG, "plan is null");
    if (plan->ws_total > (size_t)FIF_STATIC_WORKSPACE_BYTES)
        return fail(FIF_ERR_CAPACITY, "plan needs %zu bytes of workspace; the static workspace holds %zu",
                    plan->ws_total, (size_t)FIF_STATIC_WORKSPACE_BYTES);
    if (plan->prof) return fail(FIF_ERR_INVALID_ARG, "profiling creates events: not with the static workspace");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != plan->device)
        return fail(FIF_ERR_INVALID_ARG, "plan was created on device %d, current is %d", plan->device, dev);
    void* ws = nullptr;
    const fif_status st = scratch_ptr(dev, &ws);
    if (st != FIF_OK) return st;
    return batched<float>(plan, signals, delta, imfs, remainders, n_imfs, info, sig_status, ws, stream, true);
}

fif_status fif_decompose(const float* signal, int64_t N, fif_window window, double delta, int32_t max_imfs,
                         float* imfs, float* remainder, int32_t* n_imfs, fif_imf_info* info, const fif_options* opt,
                         void* stream)
{
    return single<float>(signal, N, window, delta, max_imfs, imfs, remainder, n_imfs, info, opt, stream);
}

fif_status fif_decompose_f64(const double* signal, int64_t N, fif_window window, double delta, int32_t max_imfs,
                             double* imfs, double* remainder, int32_t* n_imfs, fif_imf_info* info,
                             const fif_options* opt, void* stream)
{
    return single<double>(signal, N, window, delta, max_imfs, imfs, remainder, n_imfs, info, opt, stream);
}

fif_status fif_plan_create_tuned(fif_plan** out, const int64_t* lengths, int32_t B, int32_t max_imfs,
                                 const fif_options* opt_in, const char* tune_cache)
{
    g_err.clear();
    if (!out) return fail(FIF_ERR_INVALID_ARG, "plan pointer is null");
    *out = nullptr;
    if (!lengths || B < 1) return fail(FIF_ERR_INVALID_ARG, "need at least one signal length");
    fif_options opt;
    fif_options_default(&opt);
    if (opt_in) opt = *opt_in;
    fif_status st = validate_opts(opt);
    if (st) return st;
    const char* path = tune_cache ? tune_cache : getenv("FIF_TUNE_CACHE");
    // the FP32 lane's kernels differ: its choices are cached apart
    const std::string key = device_key() + (opt.precision == FIF_PREC_FP32 ? "/fp32" : "");
    ChoiceMap chosen;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t N = lengths[b];
        if (N <= kFftCap || chosen.count(N) || !smooth7(N)) continue;
        fif_length_plan c;
        if (path && cache_lookup(path, key.c_str(), N, &c) == FIF_OK) {
            chosen[N] = c;
            continue;
        }
        const std::vector<fif_length_plan> cands = tune_candidates(N);
        if (cands.empty()) continue;      // create_plan reports the length
        int best = -1;
        double best_us = 0.0, us0 = 0.0;
        for (size_t i = 0; i < cands.size(); ++i) {
            const double us = time_choice(cands[i], opt);
            if (i == 0) us0 = us;
            if (us > 0.0 && (best < 0 || us < best_us)) {
                best = (int)i;
                best_us = us;
            }
        }
        if (best < 0) continue;           // nothing ran: the built-in choice
        c = cands[(size_t)best];
        // times at the cache file's resolution (ns), so that a plan made from
        // the file reports what a freshly tuned one does
        c.us = std::round(best_us * 1e3) / 1e3;
        c.us_default = us0 > 0.0 ? std::round(us0 * 1e3) / 1e3 : 0.0;
        chosen[N] = c;
        if (path) (void)cache_store(path, key.c_str(), c);
    }
    g_err.clear();
    fif_plan* p = nullptr;
    st = create_plan(&p, lengths, B, max_imfs, &opt, &chosen);
    if (st) return st;
    p->tuned = chosen;
    *out = p;
    return FIF_OK;
}

fif_status fif_plan_length_plan(const fif_plan* plan, int64_t N, fif_length_plan* out)
{
    if (!plan || !out) return fail(FIF_ERR_INVALID_ARG, "null argument");
    for (const auto& lp : plan->lens) {
        if (lp.N != N) continue;
        *out = choice_of(lp);
        auto it = plan->tuned.find(N);
        if (it != plan->tuned.end()) {
            out->us = it->second.us;
            out->us_default = it->second.us_default;
        }
        return FIF_OK;
    }
    return fail(FIF_ERR_NOT_FOUND, "the plan has no signal of length %lld", (long long)N);
}

fif_status fif_tune_cache_lookup(const char* path, const char* device_key_in, int64_t N, fif_length_plan* out)
{
    g_err.clear();
    const fif_status st = cache_lookup(path, device_key_in, N, out);
    if (st == FIF_ERR_INVALID_ARG) return fail(st, "null argument");
    return st;
}

fif_status fif_tune_cache_store(const char* path, const char* device_key_in, const fif_length_plan* c)
{
    g_err.clear();
    if (!c) return fail(FIF_ERR_INVALID_ARG, "null choice");
    const fif_status st = cache_store(path, device_key_in, *c);
    if (st != FIF_OK) return fail(st, "invalid choice or unwritable cache file");
    return FIF_OK;
}

fif_status fif_device_tune_key(char* key, int32_t cap)
{
    if (!key || cap < 1) return fail(FIF_ERR_INVALID_ARG, "null or empty key buffer");
    const std::string k = device_key();
    std::strncpy(key, k.c_str(), (size_t)cap - 1);
    key[cap - 1] = 0;
    return FIF_OK;
}

fif_status fif_plan_set_proposal(fif_plan* plan, fif_model* model)
{
    g_err.clear();
    if (!plan) return fail(FIF_ERR_INVALID_ARG, "plan is null");
    if (model && model_device(model) != plan->device)
        return fail(FIF_ERR_INVALID_ARG, "model and plan live on different devices");
    if (model && plan->fp32) return fail(FIF_ERR_INVALID_ARG, "the FP32 lane takes no proposal network");
    plan->model = model;
    return FIF_OK;
}

fif_status fif_plan_record_features(fif_plan* plan, uint16_t* feats)
{
    g_err.clear();
    if (!plan) return fail(FIF_ERR_INVALID_ARG, "plan is null");
    if (((uintptr_t)feats) % 16) return fail(FIF_ERR_INVALID_ARG, "feats must be 16-byte aligned");
    if (feats && plan->fp32) return fail(FIF_ERR_INVALID_ARG, "the FP32 lane records no features");
    plan->rec = feats;
    return FIF_OK;
}

fif_status fif_plan_profile(fif_plan* plan, int32_t enable)
{
    if (!plan) return fail(FIF_ERR_INVALID_ARG, "plan is null");
    plan->prof = enable != 0;
    return FIF_OK;
}

fif_status fif_plan_profile_read(fif_plan* plan, fif_kernel_time* out, int32_t cap, int32_t* n)
{
    if (!plan || !n || (cap > 0 && !out)) return fail(FIF_ERR_INVALID_ARG, "null argument");
    std::vector<double> ms(plan->kinds.size(), 0.0);
    std::vector<int64_t> cnt(plan->kinds.size(), 0);
    hipError_t err = hipSuccess;
    for (auto& r : plan->recs) {
        float e = 0.f;
        if (err == hipSuccess) err = hipEventSynchronize(r.b);
        if (err == hipSuccess) err = hipEventElapsedTime(&e, r.a, r.b);
        ms[r.kind] += e;
        cnt[r.kind] += 1;
        plan->pool.push_back(r.a);
        plan->pool.push_back(r.b);
    }
    plan->recs.clear();
    if (err != hipSuccess) return fail(FIF_ERR_DEVICE, "event timing failed: %s", hipGetErrorString(err));
    int32_t k = 0;
    for (size_t i = 0; i < plan->kinds.size(); ++i) {
        if (cnt[i] == 0) continue;
        if (k < cap) {
            std::memset(out[k].name, 0, sizeof(out[k].name));
            std::strncpy(out[k].name, plan->kinds[i].c_str(), sizeof(out[k].name) - 1);
            out[k].launches = cnt[i];
            out[k].total_ms = ms[i];
        }
        ++k;
    }
    *n = k;
    return FIF_OK;
}

void fif_release_cache(void)
{
    auto& C = single_cache();
    std::lock_guard<std::mutex> lock(C.mu);
    C.clear();
}

}  // extern "C"
