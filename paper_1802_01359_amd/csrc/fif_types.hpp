// Descriptors shared by the host runtime and the gfx950 kernels of libfif.
#pragma once
#include <stdint.h>

namespace fif {

// Largest complex FP64 FFT held in one workgroup's LDS (128 KiB).
constexpr int kFftCap = 8192;
// Elements of one four-step tile (64 KiB of LDS: two workgroups per CU).
constexpr int kTileCap = 4096;
// Elements of a wide four-step tile (128 KiB of LDS, one workgroup per CU):
// used where the kTileCap tile would hold a single column or row (N1 or N2 =
// 4096), so that pass-1 tiles can pair mirror columns and read the spectrum
// in contiguous runs.
constexpr int kTileCapBig = 8192;
// Threads of the FFT workgroups and of the scan workgroups.
constexpr int kFftThreads = 512;
constexpr int kScanThreads = 512;
// The one-workgroup scan (fast path: N/2 <= kScanBins bins, kept in
// registers and LDS): bins per thread of the general kernel (512 threads) and
// of the kernel for signals whose FP64 check is deferred to pass 1 (1024
// threads: no FP64 search in it, so its registers allow 16 waves per CU).
constexpr int kScanBins = 32768;
constexpr int kScanBinsPerThread = 64;
constexpr int kScanBinsDeferred = 32;
// The redo of a rejected deferred estimate (FP64 search only, no bins kept):
// 256 threads, so that the grid's workgroups, nearly all returning at once,
// fit three to a CU.
constexpr int kScanBinsRedo = 128;
constexpr int kMaxRadices = 24;
// Most samples of a sampled window shape.
constexpr int kMaxWindowPoints = 65537;

// Radix plan of one LDS-resident complex FFT of length n.
struct SubFft {
    int32_t n;
    int32_t nrad;
    int32_t tw_off;                // offset (complex elements) of its pass twiddles
    int8_t rad[kMaxRadices];
};

// Per distinct signal length.
struct LenPlan {
    int64_t N;
    int32_t two_pass;              // 0: single LDS pass; 1: N = N1 * N2 four-step
    int32_t N1, N2;                // N1: pass-2 length (columns), N2: pass-1 length (rows)
    int32_t TC, TR;                // pass-1 column tile, pass-2 row tile
    int32_t paired;                // pass-1 tiles hold mirror column pairs {c, N1-c}
    int32_t spec_perm;             // half spectrum stored in pass-1 tile order (paired plans)
    SubFft f1;                     // length N2 (pass 1) or N (single pass)
    SubFft f2;                     // length N1 (pass 2)
    int64_t sin_off;               // offset (doubles) of sin(pi u/N), u = 0..N/2
    int64_t isin_off;              // offset (doubles) of 1/sin(pi u/N), u = 1..N/2
    int64_t big_lo_off, big_hi_off;// offsets (complex) of the four-step twiddle tables
    int64_t bin_off, pos_off;      // offsets (int32) of the storage position <-> bin maps
    double invN;                   // 1/N rounded
    int32_t big_split;             // exp(-2 pi i a/N) = hi[a >> shift] * lo[a & (split-1)]
    int32_t big_shift;             // log2(big_split)
    // where lambda_j's sines come from: 0 both tables; 1 sin(pi t/N), t = L j
    // mod N, evaluated in place (the table gather at t is a random access per
    // bin); 2 both sines evaluated in place.  Same values in every case.
    int32_t lam_inline;
    int32_t lam_pad;
};

// Sine-table bytes of a plan (all lengths) up to which lambda_j reads its
// sines from the tables: beyond, the gathers at L j mod N (random) and at j
// (runs of a tile's width in pass 1) miss the L2 and both sines are
// evaluated in place instead.
constexpr int64_t kSinTableHotBytes = 2 << 20;

// Per signal of the batch.
struct SigDesc {
    int64_t N;
    int64_t off;                   // element offset in packed signals/remainders
    int64_t spec_off;              // complex offset of its half spectrum (N/2+1 bins)
    int64_t inter_off;             // complex offset of its four-step intermediate
    int64_t resid_off;             // offset of its FP64 residual buffer, -1 if unused
    int64_t gs_off;                // offset (floats) of its multi-workgroup scan scratch
    int32_t len_id;
    int32_t part_off;              // offset of its run partials
    int32_t n_parts;               // run partials written per outer step
    int32_t n_init_parts;          // run partials written by the init statistics
    int32_t bs;                    // multi-workgroup scan state index, -1 if not used
    int32_t bt_off;                // first tile of its multi-workgroup scan partials
    int32_t n_btiles;              // tiles of its multi-workgroup scan
    int32_t p1_off;                // its first pass-1 work item (deferred FP64 check partials)
};

// Multi-workgroup search for m (signals with more than one workgroup's bins).
constexpr int kBigTile = 8192;     // bins per workgroup
constexpr int kBigCand = 32;       // most candidates in one round (geometric probe, gallop)
constexpr int kBigRefine = 31;     // candidates per round inside a bracket
constexpr int kBigRounds = 16;     // candidate rounds launched per outer step
constexpr int kBigInactive = 4;    // phase of a signal that is not searching
constexpr int kBigDeferred = 5;    // FP32 estimate handed to pass 1's FP64 check
// Most tiles of a signal whose FP64 check is deferred to pass 1: for one
// signal of 2^24 samples (1024 tiles) the redo launches that deferring needs
// cost more than the FP64 round they replace (measured 0.24 ms per step more),
// for many shorter signals far less.
constexpr int kBigDeferTiles = 64;
constexpr int kBigRedoRounds = 6;  // FP64 rounds after a failed check (gallop, then refine)
struct BigScan {
    int64_t lo, hi;                // FP32 bracket: f(lo) > 0 (lo may be 0), f(hi) <= 0 (hi < 0: none yet)
    int64_t elo, ehi;              // FP64 bracket, same convention
    int64_t mt;                    // FP32 estimate
    int64_t m, L;
    double sd_lo, sd_hi, sd_m, sd_p, pscale;
    double qthr;                   // noise floor of the FP64 phase (relative stop test)
    int64_t cand[kBigCand];
    int32_t phase;                 // 0 first round, 1 FP32 refine, 2 FP64, 3 done, 4 inactive
    int32_t ncand;
    uint32_t n32, n64, flags;
};

// Ordered summary of a run of consecutive samples: enough to count sign
// changes of nonzero forward differences across runs.
struct RunState {
    double first, last;
    int32_t cnt;
    int8_t fs, ls, empty, nonfinite;
};

// Mutable per-signal state in the workspace.
struct SigState {
    int64_t k, L, m;
    int64_t fpeak;                 // spectral-peak bin of this step (mask rule 2)
    double sd, sd_prev;
    double mean, maxabs, pscale;
    double qthr;                   // noise floor of the relative stop test (deferred check)
    // min / max of the residual of the current outer step as order-preserving
    // integer keys, accumulated with atomics (order independent)
    long long kmin, kmax;
    int32_t active;                // 1 while the outer loop runs
    int32_t n_imfs;
    int32_t stop_reason;
    int32_t status;                // 0 or FIF_ERR_NONFINITE
    int32_t final_buf;             // spectrum buffer holding the final residual
    int32_t flags;
    // deferred FP64 check of m: chk = 1 while pass 1 accumulates the FP64
    // stop-test sums of this step; redo = 1 when the check failed and the
    // step is being recomputed (search, pass 1) before pass 2
    int32_t chk, redo;
};

// Work item of the FFT kernels: signal and tile index.
struct Work {
    int32_t sig;
    int32_t tile;
};

}  // namespace fif
