// Search for m when a signal has more spectrum bins than one workgroup holds
// (N/2 > kScanBins).  Same mathematics as k_scan
// (smallest m with SD_m <= delta, SD by Parseval, FP32 bracketing then FP64
// confirmation), spread over tiles of kBigTile bins:
//
//   k_bscan_prep   one workgroup per signal: run summaries, stop rules, L,
//                  power scale, the geometric candidates m = 1, 2, 4, ...
//   k_bscan_round<SWEEP = true>  per tile: FP32 copies (log2 mu,
//                  power*lambda^2, power) to scratch, then the first round
//   k_bscan_round  per tile, a fixed number of launches: partial sums of the
//                  current candidates (FP32 from scratch, or FP64 from the
//                  spectrum in the confirmation phase)
//   k_bscan_final  writes L, m, SD and the IMF record
//
//   k_bscan_decide one small workgroup per signal after every round: adds the
//                  per-tile partial sums in tile order and picks the next
//                  candidates -- up to kBigRefine evenly spaced inside the
//                  bracket, or a gallop when no candidate satisfies the test
//                  yet.
// Signals already decided skip the remaining launches.  Partial sums cross
// workgroups only through kernel boundaries (no device-scope fences).
//
// Stop mode 1 (absolute criterion) searches the count c = m + 1, whose
// numerator sum P lambda^2 mu^(c-1) is ||s_{m+1} - s_m||^2 times N pscale,
// for the smallest c >= 2 below delta^2 N pscale; Theorem 5's N0 (from the
// tiles' largest |R_j|^2) bounds it from above.  Stop mode 2 takes m = N0
// and spends one FP64 round on the reported step norms.
#pragma once
#include "fif_kernels.hpp"

namespace fif {

// geometric probes 1, 2, 4, 8, ...
__device__ __forceinline__ int64_t geo_next(int64_t m) { return m * 2; }

// Candidates strictly inside (lo, hi) at a common spacing D = (hi - lo) div
// (n + 1), at most kBigRefine of them: lo + D, lo + 2D, ..., lo + nD < hi.
// The common spacing lets the tiles build mu^(m-1) of every candidate from
// the previous one by one multiplication.
__device__ __forceinline__ void fill_inside(BigScan* G, int64_t lo, int64_t hi)
{
    const int64_t gap = hi - lo - 1;
    const int n = (int)min((int64_t)kBigRefine, gap);
    const int64_t D = (hi - lo) / (n + 1);
    for (int i = 0; i < n; ++i) G->cand[i] = lo + (int64_t)(i + 1) * D;
    // strictly increasing, and lo + nD <= lo + n (hi - lo) / (n + 1) < hi
    G->ncand = n;
}

// Gallop from lo (SD_lo > delta known): lo + 1, lo + 2, lo + 4, ... capped.
__device__ __forceinline__ void fill_gallop(BigScan* G, int64_t lo, int64_t cap)
{
    int n = 0;
    int64_t step = 1;
    while (n < kBigCand) {
        const int64_t c = min(cap, lo + step);
        if (n > 0 && c == G->cand[n - 1]) break;
        G->cand[n++] = c;
        if (c == cap) break;
        step *= 2;
    }
    G->ncand = n;
}

template <int T>
__global__ __launch_bounds__(T) void k_bscan_prep(ScanArgs A)
{
    __shared__ RunState shr[T / 64];
    __shared__ int64_t sh_i[2];
    __shared__ double sh_d[1];
    const int s = A.list[blockIdx.x];
    const SigDesc d = A.sigs[s];
    SigState* S = A.st + s;
    BigScan* G = A.bigs + d.bs;
    if (!S->active) {
        if (threadIdx.x == 0) G->phase = kBigInactive;
        return;
    }
    scan_prologue<T>(A, s, d, S, shr, sh_i, sh_d);
    if (threadIdx.x == 0) {
        const int64_t L = sh_i[0];
        if (L < 0) {
            G->phase = kBigInactive;
        } else {
            S->L = L;
            G->phase = 0;
            G->L = L;
            G->pscale = sh_d[0];
            G->qthr = 0.0;
            G->n32 = G->n64 = 0;
            G->flags = 0;
            G->hi = -1;
            G->elo = 0;
            G->ehi = -1;
            G->sd_lo = INFINITY;
            G->sd_hi = 0.0;
            // counts searched: m (stop modes 0, 2) or c = m + 1 (stop mode 1)
            const int64_t first = A.stop_mode == 1 ? 2 : 1;
            const int64_t cap = A.max_inner + first - 1;
            G->lo = first - 1;
            int n = 0;
            for (int64_t m = first; m < cap && n < kBigCand - 1; m = geo_next(m)) G->cand[n++] = m;
            G->cand[n++] = cap;
            G->ncand = n;
        }
    }
}

// First-round candidates around a proposed m (one workgroup of 64 threads
// per signal, thread 0 works): m_p * 2^((i - 10)/8), i = 0..20, rounded,
// clamped to [1, cap] and made strictly increasing.  Signals without a
// proposal keep the geometric probes of k_bscan_prep.
__global__ void k_bscan_seed(ScanArgs A)
{
    if (threadIdx.x != 0) return;
    const int s = A.list[blockIdx.x];
    const SigDesc d = A.sigs[s];
    BigScan* G = A.bigs + d.bs;
    if (G->phase != 0 || !A.prop) return;
    const int64_t mp = A.prop[s];
    if (mp <= 0) return;
    const int64_t cap = A.max_inner;
    int n = 0;
    for (int i = 0; i <= 20 && n < kBigCand; ++i) {
        int64_t c = (int64_t)llrint((double)mp * exp2((double)(i - 10) / 8.0));
        c = max((int64_t)1, min(cap, c));
        if (n > 0 && c <= G->cand[n - 1]) continue;
        G->cand[n++] = c;
    }
    G->ncand = n;
}

// Partial sums of the current candidates over this tile's bins, left in
// out[2i] = sum a x, out[2i+1] = sum b x (shared memory, all threads).
// FP32 phases: x = 2^((m-1) tau) from scratch; FP64 phase: mu^(m-1) from the
// spectrum with FP64 lambda, two candidates at a time.
// One level of a reduce-scatter over the 64 lanes of a wave: a lane holding
// 2S values keeps the lower S (lane bit S clear) or the upper S (set), adds
// the partner's copy of the same S (partner = lane ^ S) and drops the rest.
template <int S>
__device__ __forceinline__ void wave_reduce_scatter(float* v, int lane)
{
    const bool up = (lane & S) != 0;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        const float lo = v[i], hi = v[i + S];
        const float send = up ? lo : hi;
        const float keep = up ? hi : lo;
        v[i] = keep + __shfl_xor(send, S);
    }
}

// PHS: 1 the FP32 rounds (phases 0 and 1), 2 the FP64 rounds (phase 2).  A
// kernel holds one kind's code only: the FP32 kind then fits in 128 VGPRs,
// two workgroups per CU.
template <int T, int BPT, typename C, int PHS>
__device__ __forceinline__ void bscan_tile_sums(const ScanArgs& A, const SigDesc& d, const LenPlan& lp,
                                                const BigScan* G, int tile, double* out, float* shf,
                                                double* shd)
{
    const int tid = threadIdx.x;
    const int nh = (int)(d.N / 2);
    const int j0 = 1 + tile * kBigTile;
    const int ph = G->phase;
    const int nc = G->ncand;
    const auto R = spec_view<C>((A.t & 1) ? A.spec1 : A.spec0, d.spec_off);
    if (PHS == 1) {
        const float* tau = A.gscr + d.gs_off;
        const float* av = tau + nh;
        const float* bv = av + nh;
        // x_i = mu^(e_i), e_i = cand_i - 1.  When the round's counts follow
        // one pattern -- even spacing (refinement) or doubling spacing
        // (geometric probes, gallops), the last count possibly off the
        // pattern (the cap) -- x_i = x_(i-1) r_i with r_1 = mu^(e_1 - e_0) and
        // r_(i+1) = r_i (even) or r_i^2 (doubling): three exp2 per bin instead
        // of one per candidate.  Other rounds (a proposal's seeds) take one
        // exp2 per candidate.  The FP32 values only bracket m; the FP64 phase
        // decides.  (The pattern is read from the uniform candidate list.)
        int pat = 0;               // 0 generic, 1 even, 2 doubling
        bool fresh_last = false;   // the last count is formed directly
        if (nc >= 2) {
            const int64_t d1 = G->cand[1] - G->cand[0];
            for (int drop = 0; drop < 2 && pat == 0; ++drop) {
                const int n = nc - drop;      // counts that must follow the pattern
                bool even = true, dbl = true;
                int64_t dp = d1;
                for (int i = 2; i < n; ++i) {
                    const int64_t di = G->cand[i] - G->cand[i - 1];
                    even = even && di == d1;
                    dbl = dbl && di == 2 * dp;
                    dp = di;
                }
                if (n >= 2 && (even || dbl)) {
                    pat = even ? 1 : 2;
                    fresh_last = drop == 1;
                }
            }
        }
        const float e0 = (float)(G->cand[0] - 1);
        const float d1f = nc >= 2 ? (float)(G->cand[1] - G->cand[0]) : 0.f;
        const float elast = (float)(G->cand[nc - 1] - 1);
        const bool dbl = pat == 2;
        float acc[2 * kBigCand];
#pragma unroll
        for (int i = 0; i < 2 * kBigCand; ++i) acc[i] = 0.f;
        // the thread's bins in chunks of CH, each chunk's loads issued
        // together (one memory round trip per chunk; the chunk loop is kept
        // rolled so that only one chunk's values occupy registers); bins past
        // the end of the signal carry a = b = 0
        constexpr int CH = BPT < 8 ? BPT : 8;
        auto load_chunk = [&](int q0, float* tq, float* aq, float* bq) {
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int j = j0 + tid + (q0 + q) * T;
                tq[q] = 0.f;
                aq[q] = 0.f;
                bq[q] = 0.f;
                if (j <= nh) {
                    tq[q] = tau[j - 1];
                    aq[q] = av[j - 1];
                    bq[q] = bv[j - 1];
                }
            }
        };
        if (pat == 0) {
            // one exp2 per candidate and bin; the exponents come from LDS,
            // read anew in every chunk (the compiler barrier keeps the 32
            // values from being held in registers across the chunks)
            __shared__ float she[kBigCand];
            if (tid < kBigCand) she[tid] = tid < nc ? (float)(G->cand[tid] - 1) : 0.f;
            __syncthreads();
#pragma unroll 1
            for (int q0 = 0; q0 < BPT; q0 += CH) {
                asm volatile("" ::: "memory");
                float tq[CH], aq[CH], bq[CH];
                load_chunk(q0, tq, aq, bq);
#pragma unroll
                for (int i = 0; i < kBigCand; ++i) {
                    if (i < nc) {
                        const float ei = she[i];
#pragma unroll
                        for (int q = 0; q < CH; ++q) {
                            const float x = (ei == 0.f) ? 1.f : __builtin_amdgcn_exp2f(ei * tq[q]);
                            acc[2 * i] += aq[q] * x;
                            acc[2 * i + 1] += bq[q] * x;
                        }
                    }
                }
            }
        } else {
#pragma unroll 1
            for (int q0 = 0; q0 < BPT; q0 += CH) {
                float tq[CH], aq[CH], bq[CH];
                load_chunk(q0, tq, aq, bq);
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    const float tj = tq[q], aj = aq[q], bj = bq[q];
                    float x = (e0 == 0.f) ? 1.f : __builtin_amdgcn_exp2f(e0 * tj);
                    float r = __builtin_amdgcn_exp2f(d1f * tj);
                    const float xl = __builtin_amdgcn_exp2f(elast * tj);
#pragma unroll
                    for (int i = 0; i < kBigCand; ++i) {
                        if (i < nc) {
                            if (i > 0) {
                                x *= r;
                                r = dbl ? r * r : r;
                            }
                            const float xi = (fresh_last && i == nc - 1) ? xl : x;
                            acc[2 * i] += aj * xi;
                            acc[2 * i + 1] += bj * xi;
                        }
                    }
                }
            }
        }
        // the 2*kBigCand sums over the workgroup: a reduce-scatter across the
        // wave (each level halves the values a lane keeps, so lane l ends with
        // the wave's sum of value l), then the waves' sums in wave order
        static_assert(2 * kBigCand == 64, "one value per lane after the reduce-scatter");
        const int lane = tid & 63, wave = tid >> 6;
        wave_reduce_scatter<32>(acc, lane);
        wave_reduce_scatter<16>(acc, lane);
        wave_reduce_scatter<8>(acc, lane);
        wave_reduce_scatter<4>(acc, lane);
        wave_reduce_scatter<2>(acc, lane);
        wave_reduce_scatter<1>(acc, lane);
        shf[wave * 64 + lane] = acc[0];
        __syncthreads();
        if (tid < 64) {
            float s = 0.f;
#pragma unroll
            for (int w = 0; w < T / 64; ++w) s += shf[w * 64 + tid];
            out[tid] = (double)s;
        }
    } else {
        const Lam lw = make_lam(lp, A.dtab, G->L, A.lam ? A.lam + d.spec_off : nullptr);
        // position -> bin table of this length, read once (null: bin order)
        const int32_t* btab = lp.spec_perm ? A.itab + lp.bin_off : nullptr;
        const double pscale = G->pscale;
        // relative stop test, as in k_scan: bins below the noise floor are
        // not counted, and each candidate's sums are kept relative to the
        // largest weight (running maximum of the exponent per thread, then the
        // block's); the tile hands over the logarithms of its two sums
        const double qthr = G->qthr;
        for (int c = 0; c < nc; c += 2) {
            const int64_t e0 = G->cand[c] - 1;
            const int64_t e1 = (c + 1 < nc) ? G->cand[c + 1] - 1 : -1;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            double am[2] = {-INFINITY, -INFINITY};
            auto add = [&](int k, int64_t e, double P, double l2, double lam, double lg) {
                if (e < 0 || (e > 0 && lam >= 1.0)) return;
                const double a = (e == 0) ? 0.0 : (double)e * lg;
                if (a > am[k]) {
                    const double r = (am[k] == -INFINITY) ? 0.0 : exp(am[k] - a);
                    acc[2 * k] *= r;
                    acc[2 * k + 1] *= r;
                    am[k] = a;
                }
                const double x = exp(a - am[k]);
                acc[2 * k] += P * l2 * x;
                acc[2 * k + 1] += P * x;
            };
            constexpr int DG = 4;  // bins whose loads are issued together
            for (int q0 = 0; q0 < BPT; q0 += DG) {
              double2 zz[DG];
              int64_t jj[DG];
#pragma unroll
              for (int g = 0; g < DG; ++g) {
                const int j = j0 + tid + (q0 + g) * T;
                zz[g] = make_double2(0.0, 0.0);
                jj[g] = 1;
                if (j <= nh) {
                    zz[g] = R[j];                      // storage position j
                    jj[g] = btab ? (int64_t)btab[j] : (int64_t)j;   // its bin
                }
              }
#pragma unroll
              for (int g = 0; g < DG; ++g) {
                if (j0 + tid + (q0 + g) * T > nh) break;
                const double2 z = zz[g];
                const int64_t jb = jj[g];
                const double q = z.x * z.x + z.y * z.y;
                if (q < qthr) continue;
                const double P = ((2 * jb == d.N) ? 1.0 : 2.0) * q * pscale;
                const double lam = lambda_at(jb, lw);
                const double l2 = lam * lam;
                const double lg = (lam < 1.0) ? 2.0 * log1p(-lam) : 0.0;
                add(0, e0, P, l2, lam, lg);
                add(1, e1, P, l2, lam, lg);
              }
            }
            double mk[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                double mn_unused = INFINITY, M = am[k];
                block_minmax<T>(mn_unused, M, shd);
                const double r = (am[k] == -INFINITY) ? 0.0 : exp(am[k] - M);
                acc[2 * k] *= r;
                acc[2 * k + 1] *= r;
                mk[k] = M;
            }
            block_sum<double, T, 4>(acc, shd);
            if (tid == 0) {
                // log(0) = -inf: an empty sum
                out[2 * c] = log(acc[0]) + mk[0];
                out[2 * c + 1] = log(acc[1]) + mk[0];
                if (c + 1 < nc) {
                    out[2 * c + 2] = log(acc[2]) + mk[1];
                    out[2 * c + 3] = log(acc[3]) + mk[1];
                }
            }
        }
    }
    // DC bin (lambda_0 = 1): contributes to m = 1 only (FP64 phase: to the
    // logarithms of the sums)
    if (tile == 0 && tid == 0) {
        const double P0 = (R[0].x * R[0].x + R[0].y * R[0].y) * G->pscale;
        for (int i = 0; i < nc; ++i)
            if (G->cand[i] == 1) {
                if (ph < 2) {
                    out[2 * i] += P0;
                    out[2 * i + 1] += P0;
                } else if (P0 > 0.0) {
                    for (int k = 0; k < 2; ++k) {
                        const double u = out[2 * i + k], v = log(P0);
                        const double hi = fmax(u, v), lo = fmin(u, v);
                        out[2 * i + k] = hi + log1p(exp(lo - hi));
                    }
                }
            }
    }
    __syncthreads();
}

// Sums over the tiles of every candidate's two partial sums: tot[2i]
// (numerator) and tot[2i+1] (denominator) of candidate i.  kDecideGroups
// groups of 64 threads each add a contiguous range of tiles in tile order;
// the group results are then added in group order, so the result depends
// only on the number of tiles.  LOGS (FP64 phase): the partial sums are
// logarithms, added as a log-sum-exp (each group relative to its largest,
// then the groups relative to theirs); tot holds logarithms too.
constexpr int kDecideGroups = 16;
static_assert(2 * kBigCand <= 64, "one lane per partial sum");
__device__ __forceinline__ void bscan_tile_totals(const ScanArgs& A, const SigDesc& d, int nc, bool logs,
                                                  double* part, double* partm, double* tot)
{
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int nt = d.n_btiles;
    const int t0 = (int)(((int64_t)nt * g) / kDecideGroups), t1 = (int)(((int64_t)nt * (g + 1)) / kDecideGroups);
    double s = 0.0, mx = -INFINITY;
    if (c < 2 * nc) {
        const double* P = A.bpart + (int64_t)d.bt_off * 2 * kBigCand + c;
        if (!logs) {
#pragma unroll 8
            for (int t = t0; t < t1; ++t) s += P[(int64_t)t * 2 * kBigCand];
        } else {
            for (int t = t0; t < t1; ++t) mx = fmax(mx, P[(int64_t)t * 2 * kBigCand]);
            if (mx > -INFINITY)
                for (int t = t0; t < t1; ++t) s += exp(P[(int64_t)t * 2 * kBigCand] - mx);
        }
    }
    part[threadIdx.x] = s;
    partm[threadIdx.x] = mx;
    __syncthreads();
    if (g == 0) {
        if (!logs) {
            double v = 0.0;
            for (int q = 0; q < kDecideGroups; ++q) v += part[q * 64 + c];
            tot[c] = v;
        } else {
            double M = -INFINITY;
            for (int q = 0; q < kDecideGroups; ++q) M = fmax(M, partm[q * 64 + c]);
            double v = 0.0;
            if (M > -INFINITY)
                for (int q = 0; q < kDecideGroups; ++q)
                    if (partm[q * 64 + c] > -INFINITY) v += part[q * 64 + c] * exp(partm[q * 64 + c] - M);
            tot[c] = (M > -INFINITY) ? M + log(v) : -INFINITY;
        }
    }
}

// Thread 0 of the decide workgroup: update the brackets, choose the next
// candidates.
__device__ __forceinline__ void bscan_decide(const ScanArgs& A, int s, const SigDesc& d, BigScan* G,
                                             const double* tot)
{
    const int nc = G->ncand;
    const double* Asum = tot;          // numerator of candidate i at Asum[2i]
    const double* Bsum = tot + 1;      // denominator at Bsum[2i]
    const double delta = A.delta;
    const int mode = A.stop_mode;
    // stop mode 1 counts c = m + 1 (c = 1, m = 0, is never an answer)
    const int64_t first = mode == 1 ? 2 : 1;
    const int64_t cap = A.max_inner + first - 1;
    // ||s_{m+1} - s_m||^2 N pscale below this passes the absolute test
    const double thr_abs = delta * delta * (double)d.N * G->pscale;
    if (G->phase < 2) {
        G->n32 += 1;
        const double d2 = (double)(float)(delta * delta);
        int q = -1;
        for (int i = 0; i < nc; ++i) {
            const bool ok = mode == 1 ? Asum[2 * i] < thr_abs
                                      : (Bsum[2 * i] <= 0.0 || Asum[2 * i] <= d2 * Bsum[2 * i]);
            if (ok) {
                q = i;
                break;
            }
        }
        int64_t lo = G->lo, hi = G->hi;
        if (q >= 0) {
            hi = G->cand[q];
            if (q > 0) lo = G->cand[q - 1];
        } else {
            lo = G->cand[nc - 1];
        }
        if (mode == 1 && G->mt > 0 && (hi < 0 || hi > G->mt)) {
            // Theorem 5: c = N0 + 1 passes the absolute test (G->mt holds it
            // after the first round); the FP64 phase checks the bracket
            hi = G->mt;
        }
        if (lo >= hi && hi >= 0) lo = hi - 1;
        int64_t mt = -1;
        if (q < 0 && lo >= cap)
            mt = cap;
        else if (hi >= 0 && hi - lo <= 1)
            mt = hi;
        G->lo = lo;
        G->hi = hi;
        if (mt >= 0 && mode == 0 && A.defer && d.n_btiles <= kBigDeferTiles) {
            // the FP64 check of SD_mt <= delta < SD_{mt-1} is left to pass 1,
            // which forms every bin's gain anyway; k_verify accepts the
            // estimate or sends the signal to the FP64 rounds of the redo
            if (A.mt_shift) mt = max((int64_t)1, min(cap, mt + (int64_t)A.mt_shift));
            G->phase = kBigDeferred;
            G->mt = mt;
            SigState* S = A.st + s;
            S->L = G->L;
            S->m = mt;
            S->chk = 1;
            S->qthr = G->qthr;
            if (A.info) {
                fif_imf_info* I = A.info + (int64_t)s * A.max_imfs + A.t;
                I->k = S->k;
                I->L = G->L;
                I->m = mt;
                I->flags = 0;
                I->evals = (G->n32 & 0xffffu) | (1u << 16);
            }
        } else if (mt >= 0) {
            // FP64 confirmation of SD_mt <= delta < SD_{mt-1}
            G->phase = 2;
            G->mt = mt;
            if (mt == first) {
                G->cand[0] = 1;
                G->ncand = 1;
            } else {
                G->cand[0] = mt - 1;
                G->cand[1] = mt;
                G->ncand = 2;
            }
        } else if (hi >= 0) {
            G->phase = 1;
            fill_inside(G, lo, hi);
        } else {
            G->phase = 1;
            fill_gallop(G, lo, cap);
        }
        return;
    }
    // FP64 phase: tot holds the logarithms of the sums (-inf: empty)
    G->n64 += 1;
    if (mode == 2) {
        // the a-priori count needs no search: report the step norms at m
        // (c = m + 1) and m - 1 (c = m), computed by this round
        G->m = G->mt;
        G->sd_m = sqrt(exp(Asum[2]) / ((double)d.N * G->pscale));   // c = m + 1
        G->sd_p = sqrt(exp(Asum[0]) / ((double)d.N * G->pscale));   // c = m
        G->phase = 3;
        return;
    }
    int64_t elo = G->elo, ehi = G->ehi;
    double sd_lo = G->sd_lo, sd_hi = G->sd_hi;
    for (int i = 0; i < nc; ++i) {
        const double sd = mode == 1 ? sqrt(exp(Asum[2 * i]) / ((double)d.N * G->pscale))
                                    : (Bsum[2 * i] > -INFINITY ? exp(0.5 * (Asum[2 * i] - Bsum[2 * i])) : 0.0);
        const int64_t c = G->cand[i];
        const bool ok = (mode == 1 ? sd < delta : sd <= delta) && c >= first;
        if (ok) {
            if (ehi < 0 || c < ehi) {
                ehi = c;
                sd_hi = sd;
            }
        } else if (c > elo) {
            elo = c;
            sd_lo = sd;
        }
    }
    if (G->n64 == 1 && !(ehi == G->mt && elo == G->mt - 1)) G->flags |= FIF_IMF_REFINED;
    G->elo = elo;
    G->ehi = ehi;
    G->sd_lo = sd_lo;
    G->sd_hi = sd_hi;
    if (ehi >= 0 && ehi - elo <= 1) {
        G->m = ehi - (first - 1);
        G->sd_m = sd_hi;
        G->sd_p = (mode == 0 && ehi == 1) ? INFINITY : sd_lo;
        G->phase = 3;
    } else if (ehi < 0 && elo >= cap) {
        G->m = cap - (first - 1);
        G->sd_m = sd_lo;
        G->sd_p = sd_lo;
        G->flags |= FIF_IMF_CAP;
        G->phase = 3;
    } else if (ehi < 0) {
        fill_gallop(G, elo, cap);
    } else {
        fill_inside(G, elo, ehi);
    }
}

// One candidate round over one tile (first round: also fill the scratch).
// PHS as for bscan_tile_sums: a round launches the FP32 kind and, unless every
// signal of the group leaves its FP64 check to pass 1, the FP64 kind after it;
// each skips the signals in the other kind's phase.  Every active signal
// enters the sweep in phase 0.
template <int T, bool SWEEP, typename C, int PHS>
__global__ __launch_bounds__(T) void k_bscan_round(ScanArgs A, const Work* __restrict__ work)
{
    static_assert(PHS == 1 || PHS == 2, "one kind of round per kernel");
    static_assert(!SWEEP || PHS == 1, "the sweep opens the FP32 phase");
    constexpr int BPT = kBigTile / T;
    __shared__ double shd[4 * (T / 64)];
    __shared__ float shf[64 * (T / 64)];
    __shared__ double shv[2 * kBigCand];
    const Work w = work[blockIdx.x];
    const SigDesc d = A.sigs[w.sig];
    const LenPlan& lp = A.lens[d.len_id];
    BigScan* G = A.bigs + d.bs;
    const int ph = G->phase;
    if (ph >= 3 || (PHS == 1) != (ph < 2)) return;
    if (SWEEP) {
        const int nh = (int)(d.N / 2);
        float* tau = A.gscr + d.gs_off;
        float* av = tau + nh;
        float* bv = av + nh;
        const auto R = spec_view<C>((A.t & 1) ? A.spec1 : A.spec0, d.spec_off);
        const Lam lw = make_lam(lp, A.dtab, G->L, A.lam ? A.lam + d.spec_off : nullptr);
        // position -> bin table of this length, read once (null: bin order)
        const int32_t* btab = lp.spec_perm ? A.itab + lp.bin_off : nullptr;
        const double pscale = G->pscale;
        const float invNf = 1.f / (float)d.N, invLf = 1.f / (float)G->L;
        double qmx = 0.0;      // largest |R_j|^2 of the tile (noise floor of the FP64 phase)
        constexpr int SG = 4;  // bins whose loads are issued together
        for (int q0 = 0; q0 < BPT; q0 += SG) {
          double2 zz[SG];
          int64_t jj[SG];
#pragma unroll
          for (int g = 0; g < SG; ++g) {
            const int j = 1 + w.tile * kBigTile + threadIdx.x + (q0 + g) * T;
            zz[g] = make_double2(0.0, 0.0);
            jj[g] = 1;
            if (j <= nh) {
                zz[g] = R[j];
                jj[g] = btab ? (int64_t)btab[j] : (int64_t)j;
            }
          }
#pragma unroll
          for (int g = 0; g < SG; ++g) {
            const int j = 1 + w.tile * kBigTile + threadIdx.x + (q0 + g) * T;
            if (j > nh) break;
            const double2 z = zz[g];                   // storage position j
            const int64_t jb = jj[g];                  // its bin
            qmx = fmax(qmx, z.x * z.x + z.y * z.y);
            const double P = ((2 * jb == d.N) ? 1.0 : 2.0) * (z.x * z.x + z.y * z.y) * pscale;
            // lambda in FP32, as in k_scan: these values only bracket m (both
            // sines from sinpif: the bins come in storage order, and these
            // lengths' tables are large)
            const float lf = lambda_f32<true>(jb, lw, invNf, invLf);
            const float pf = (float)P;
            bv[j - 1] = pf;
            av[j - 1] = pf * lf * lf;
            tau[j - 1] = 2.8853900817779268f * log1pf(-lf);
          }
        }
        double mn_unused = INFINITY;
        block_minmax<T>(mn_unused, qmx, shd);
        if (threadIdx.x == 0) A.bqmax[d.bt_off + w.tile] = qmx;
        // each thread reads back only its own bins below
    }
    bscan_tile_sums<T, BPT, C, PHS>(A, d, lp, G, w.tile, shv, shf, shd);
    double* P = A.bpart + ((int64_t)d.bt_off + w.tile) * 2 * kBigCand;
    const int nc = G->ncand;
    if (threadIdx.x < 2 * nc) P[threadIdx.x] = shv[threadIdx.x];
}

// After a round: tile totals in tile order, then the next candidates.
template <typename C = double2>
__global__ __launch_bounds__(64 * kDecideGroups) void k_bscan_decide(ScanArgs A)
{
    __shared__ double part[64 * kDecideGroups];
    __shared__ double partm[64 * kDecideGroups];
    __shared__ double tot[2 * kBigCand];
    __shared__ double shq[2 * kDecideGroups];
    const int s = A.list[blockIdx.x];
    const SigDesc d = A.sigs[s];
    BigScan* G = A.bigs + d.bs;
    if (G->phase >= 3) return;
    // after the sweep: the tiles' largest |R_j|^2 (all threads)
    const bool first = G->phase < 2 && G->n32 == 0;
    double q = 0.0, mn_unused = INFINITY;
    if (first)
        for (int t = threadIdx.x; t < d.n_btiles; t += 64 * kDecideGroups) q = fmax(q, A.bqmax[d.bt_off + t]);
    block_minmax<64 * kDecideGroups>(mn_unused, q, shq);
    bscan_tile_totals(A, d, G->ncand, G->phase >= 2, part, partm, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        bool skip = false;       // stop mode 2: this round only found N0
        if (first) {
            // the tiles' largest |R_j|^2 give the noise floor of the
            // relative test, or Theorem 5's N0 (with the DC bin)
            G->qthr = A.stop_mode == 0 ? kSdNoise * q : 0.0;
            G->mt = 0;
            if (A.stop_mode != 0) {
                const double2 r0 = spec_view<C>((A.t & 1) ? A.spec1 : A.spec0, d.spec_off)[0];
                const int64_t n0 = apriori_n0(fmax(q, r0.x * r0.x + r0.y * r0.y), G->L, d.N, A.delta);
                if (A.stop_mode == 1) {
                    G->mt = min(n0, A.max_inner) + 1;     // as a count c = m + 1
                } else {
                    // m = N0 (capped): one FP64 round for the norms at m, m - 1
                    const int64_t m = min(n0, A.max_inner);
                    if (n0 > A.max_inner) G->flags |= FIF_IMF_CAP;
                    G->n32 = 0;            // no search: the sweep only found N0
                    G->phase = 2;
                    G->mt = m;
                    G->cand[0] = m;        // c = m: ||s_m - s_{m-1}||
                    G->cand[1] = m + 1;    // c = m + 1: ||s_{m+1} - s_m||
                    G->ncand = 2;
                    skip = true;
                }
            }
        }
        if (!skip) bscan_decide(A, s, d, G, tot);
    }
}

// After k_verify: a deferred signal whose check failed goes back to the FP64
// phase, first with the kBigRedoCand consecutive counts around its estimate
// (gallop and refinement follow if the answer lies outside them); the others
// stay deferred (their estimate stands, k_bscan_final leaves them alone).
constexpr int kBigRedoCand = 8;
__global__ void k_bscan_redo_prep(ScanArgs A)
{
    if (threadIdx.x != 0) return;
    const int s = A.list[blockIdx.x];
    const SigDesc d = A.sigs[s];
    BigScan* G = A.bigs + d.bs;
    SigState* S = A.st + s;
    if (G->phase != kBigDeferred || !S->redo) return;
    const int64_t cap = A.max_inner;
    const int64_t lo = max((int64_t)1, min(cap - kBigRedoCand + 1, G->mt - kBigRedoCand / 2));
    int n = 0;
    for (int64_t c = lo; c <= cap && n < kBigRedoCand; ++c) G->cand[n++] = c;
    G->ncand = n;
    G->phase = 2;
    G->elo = 0;
    G->ehi = -1;
    G->sd_lo = INFINITY;
    G->sd_hi = 0.0;
    G->n64 = 0;
    G->flags |= FIF_IMF_REFINED;
}

template <int T>
__global__ __launch_bounds__(T) void k_bscan_final(ScanArgs A)
{
    if (threadIdx.x != 0) return;
    const int s = A.list[blockIdx.x];
    const SigDesc d = A.sigs[s];
    SigState* S = A.st + s;
    BigScan* G = A.bigs + d.bs;
    if (G->phase == kBigInactive || G->phase == kBigDeferred) return;
    uint32_t flags = G->flags;
    if (G->phase != 3) {
        // out of rounds (not expected): keep the FP64-verified upper end
        flags |= FIF_IMF_UNRESOLVED;
        G->m = G->ehi >= 0 ? G->ehi : A.max_inner;
        G->sd_m = G->sd_hi;
        G->sd_p = G->sd_lo;
    }
    S->L = G->L;
    S->m = G->m;
    S->sd = G->sd_m;
    S->sd_prev = G->sd_p;
    S->flags |= (int32_t)flags;
    if (A.info) {
        fif_imf_info* I = A.info + (int64_t)s * A.max_imfs + A.t;
        I->k = S->k;
        I->L = G->L;
        I->m = G->m;
        I->sd = G->sd_m;
        I->sd_prev = G->sd_p;
        I->flags = flags;
        I->evals = (G->n32 & 0xffffu) | (G->n64 << 16);
    }
}

// Run summaries, min and max of the FP64 residual written by k_pass2 for
// signals whose row tiles are too thin for per-tile summaries.  A workgroup
// takes kFftCap samples in halves staged through LDS (coalesced loads; each
// thread then walks a run of consecutive samples); the halves' summaries
// are combined in sample order.
__global__ __launch_bounds__(kFftThreads) void k_count_resid(const SigDesc* __restrict__ sigs,
                                                              const Work* __restrict__ work,
                                                              const double* __restrict__ resid,
                                                              RunState* __restrict__ parts,
                                                              SigState* __restrict__ st)
{
    constexpr int H = kFftCap / 2;
    __shared__ double stg[H];
    __shared__ RunState sh[kFftThreads / 64];
    __shared__ double shd[2 * (kFftThreads / 64)];
    const Work w = work[blockIdx.x];
    const SigDesc d = sigs[w.sig];
    if (!st[w.sig].active) return;
    const int64_t t0 = (int64_t)w.tile * kFftCap;
    const int64_t len = min((int64_t)kFftCap, d.N - t0);
    const double* src = resid + d.resid_off + t0;
    RunState tot = run_empty();
    double mn = INFINITY, mx = -INFINITY;
    for (int h = 0; h < 2; ++h) {
        const int cnt = (int)max((int64_t)0, min((int64_t)H, len - (int64_t)h * H));
        for (int i = threadIdx.x; i < cnt; i += kFftThreads) stg[i] = src[(int64_t)h * H + i];
        __syncthreads();
        const int chunk = (cnt + kFftThreads - 1) / kFftThreads;
        const int a = threadIdx.x * chunk, b = min(cnt, a + chunk);
        RunState r = run_empty();
        for (int i = a; i < b; ++i) {
            const double v = stg[i];
            run_push(r, v);
            mn = fmin(mn, v);
            mx = fmax(mx, v);
        }
        r = block_run_reduce<kFftThreads>(r, sh);
        if (threadIdx.x == 0) tot = run_combine(tot, r);
        __syncthreads();
    }
    block_minmax<kFftThreads>(mn, mx, shd);
    if (threadIdx.x == 0) {
        parts[d.part_off + w.tile] = tot;
        atomicMin(&st[w.sig].kmin, dkey(mn));
        atomicMax(&st[w.sig].kmax, dkey(mx));
    }
}

}  // namespace fif
