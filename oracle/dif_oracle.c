/*
 * Plain FP64 CPU oracle for Discrete Iterative Filtering (DIF).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * path shares no code, header, table or constant with it.
 *
 * What it computes (Cicone & Zhou, "Numerical Analysis for Iterative
 * Filtering with New Efficient Implementations Based on FFT"):
 *
 *   - the discrete iteration s_{m+1} = (I - W) s_m of Section 3 (equations
 *     "s_m+1" and "MatrixForm"), with W the circulant matrix of the window
 *     under periodic extension (equation "W_m", Section 3.1);
 *   - the inner stop quantity SD = ||s_{m+1} - s_m|| / ||s_m|| (equation "SD")
 *     with the optional cap on the number of inner iterations stated next to it;
 *   - the outer loop of Algorithm 2 (DIF): count extrema, fix the filter
 *     length once per inner loop (Section 2, the remark after the mask-length
 *     discussion, and the text after Algorithm 2), iterate, record the IMF,
 *     subtract it, repeat; the final residual is appended (Algorithm 1/2).
 *
 * This is the time-domain definition written out.  No FFT is used anywhere:
 * W x is a periodic convolution evaluated either literally from the folded
 * taps, or as four periodic box sums (the window is a triangle convolved with
 * itself and a triangle is a box convolved with a reversed box), which is the
 * same linear map.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - window: h is the triangle of equation "triangular" sampled at integer
 *     offsets, h_q = (L - |q|)/L^2 for |q| <= L-1 (sum exactly 1); the window
 *     is w = h * h (the double-convolution construction of Section 2 that
 *     makes the spectrum lie in [0,1]); L is the half-support of h;
 *   - mask length: L = ceil(2N/k) (rule 0) or L = 2*floor(nu*N/k) (rule 1,
 *     equation "Unif_Mask_length");
 *   - extrema: k = number of sign changes between consecutive nonzero forward
 *     differences r_{i+1} - r_i, signs taken by comparison, i = 0..N-2
 *     (linear, endpoints excluded, plateaus count once); the outer loop runs
 *     while k >= 2;
 *   - stop test SD <= delta (Section 4 phrasing), checked after every
 *     application of (I - W); m counts applications, IMF = (I - W)^m r;
 *     SD is evaluated as ||W s_m|| / ||s_m||, which equals the defining
 *     quotient exactly in real arithmetic; SD = 0 when ||s_m|| = 0;
 *   - rounding floor: before counting, stop when
 *     max_i |r_i - mean(r)| <= tau * max_i |s_i|.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DIF_OK 0
#define DIF_ERR_ARG -1
#define DIF_ERR_NOMEM -3

/* per-IMF flags */
#define DIF_FLAG_CAP 1 /* inner loop stopped at max_inner, not by SD <= delta */

/* why the outer loop ended */
#define DIF_STOP_MAX_IMFS 0
#define DIF_STOP_FLOOR 1
#define DIF_STOP_FEW_EXTREMA 2

typedef struct {
    int32_t mask_rule;  /* 0: L = ceil(2N/k); 1: L = 2*floor(nu*N/k) */
    int32_t inner_form; /* 0: literal folded taps; 1: four periodic box sums */
    double nu;
    int64_t max_inner;
    double floor_tau;
} dif_opts;

typedef struct {
    int64_t k;          /* extrema count of the residual entering this IMF */
    int64_t L;          /* half-support of the triangle h */
    int64_t m;          /* number of applications of (I - W) */
    double sd;          /* SD_m */
    double sd_prev;     /* SD_{m-1} (+inf when m == 1) */
    double margin_k;    /* min |r_{i+1}-r_i| / max|r| over the residual counted */
    double floor_ratio; /* max|r-mean r| / (tau*max|s|) of that residual */
    int32_t flags;
    int32_t pad;
} dif_imf_info;

/* ------------------------------------------------------------------ */
/* extrema count                                                        */
/* ------------------------------------------------------------------ */

static int sgn_cmp(double a, double b) { return (b > a) - (b < a); }

int64_t dif_count_extrema(const double *r, int64_t n, double *margin_out)
{
    int64_t k = 0;
    int prev = 0;
    double mind = INFINITY, maxr = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double a = fabs(r[i]);
        if (a > maxr) maxr = a;
    }
    for (int64_t i = 0; i + 1 < n; ++i) {
        double ad = fabs(r[i + 1] - r[i]);
        if (ad < mind) mind = ad;
        int d = sgn_cmp(r[i], r[i + 1]);
        if (d == 0) continue;
        if (prev != 0 && d != prev) ++k;
        prev = d;
    }
    if (margin_out) *margin_out = (maxr > 0.0) ? mind / maxr : 0.0;
    return k;
}

/* ------------------------------------------------------------------ */
/* mask length                                                          */
/* ------------------------------------------------------------------ */

int64_t dif_mask_length(int64_t N, int64_t k, int32_t rule, double nu)
{
    if (k <= 0) return -1;
    if (rule == 0) return (2 * N + k - 1) / k;
    /* rule 1: 2 * floor(nu * N / k), never below 1 */
    double q = floor(nu * (double)N / (double)k);
    int64_t L = 2 * (int64_t)q;
    return L < 1 ? 1 : L;
}

/* ------------------------------------------------------------------ */
/* window taps and the circulant column                                 */
/* ------------------------------------------------------------------ */

/*
 * Integer taps of w~ = T * T where T_q = L - |q| (|q| <= L-1), i.e. the
 * unnormalised triangle convolved with itself: length 4L-3, centre index
 * 2L-2.  T itself is a length-L box convolved with a reversed box, so w~ is
 * four boxes convolved; each box convolution is a running sum.  Values are
 * kept in long double (exact integers below 2^64).
 */
static long double *window_taps(int64_t L, int64_t *len_out)
{
    int64_t len = 4 * L - 3;
    long double *a = (long double *)calloc((size_t)len, sizeof(long double));
    long double *b = (long double *)calloc((size_t)len, sizeof(long double));
    if (!a || !b) { free(a); free(b); return NULL; }
    for (int64_t i = 0; i < L; ++i) a[i] = 1.0L;
    int64_t cur = L;
    for (int pass = 0; pass < 3; ++pass) {
        /* b = a convolved with a box of length L */
        int64_t nl = cur + L - 1;
        long double run = 0.0L;
        for (int64_t i = 0; i < nl; ++i) {
            if (i < cur) run += a[i];
            if (i - L >= 0 && i - L < cur) run -= a[i - L];
            b[i] = run;
        }
        long double *t = a; a = b; b = t;
        cur = nl;
    }
    free(b);
    *len_out = len;
    return a;
}

/*
 * Circulant first column c (length N) of W: the taps w~_q / L^4 folded onto
 * residues q mod N (they may wrap several times when the window is longer
 * than the signal).  sum(c) = 1.
 */
int dif_window_column(int64_t N, int64_t L, double *c)
{
    if (N < 1 || L < 1 || !c) return DIF_ERR_ARG;
    int64_t len;
    long double *t = window_taps(L, &len);
    if (!t) return DIF_ERR_NOMEM;
    long double *acc = (long double *)calloc((size_t)N, sizeof(long double));
    if (!acc) { free(t); return DIF_ERR_NOMEM; }
    long double L4 = (long double)L * L * L * L;
    int64_t centre = 2 * L - 2;
    for (int64_t i = 0; i < len; ++i) {
        int64_t q = i - centre;
        int64_t p = ((q % N) + N) % N;
        acc[p] += t[i];
    }
    for (int64_t p = 0; p < N; ++p) c[p] = (double)(acc[p] / L4);
    free(acc);
    free(t);
    return DIF_OK;
}

/* ------------------------------------------------------------------ */
/* one application of W                                                 */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t N, L;
    int32_t form;
    /* literal form: nonzero folded taps (exact integer numerators / L^4) */
    int64_t nnz;
    int64_t *idx;
    long double *val;
    long double L4;
    /* box form scratch */
    long double *buf0, *buf1, *pref;
} wop;

static void wop_free(wop *w)
{
    free(w->idx); free(w->val); free(w->buf0); free(w->buf1); free(w->pref);
    memset(w, 0, sizeof(*w));
}

static int wop_init(wop *w, int64_t N, int64_t L, int32_t form)
{
    memset(w, 0, sizeof(*w));
    w->N = N; w->L = L; w->form = form;
    w->L4 = (long double)L * L * L * L;
    if (form == 0) {
        int64_t len;
        long double *t = window_taps(L, &len);
        if (!t) return DIF_ERR_NOMEM;
        long double *acc = (long double *)calloc((size_t)N, sizeof(long double));
        if (!acc) { free(t); return DIF_ERR_NOMEM; }
        int64_t centre = 2 * L - 2;
        for (int64_t i = 0; i < len; ++i) {
            int64_t q = i - centre;
            acc[((q % N) + N) % N] += t[i];
        }
        free(t);
        int64_t nnz = 0;
        for (int64_t p = 0; p < N; ++p) nnz += (acc[p] != 0.0L);
        w->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz ? nnz : 1));
        w->val = (long double *)malloc(sizeof(long double) * (size_t)(nnz ? nnz : 1));
        if (!w->idx || !w->val) { free(acc); wop_free(w); return DIF_ERR_NOMEM; }
        nnz = 0;
        for (int64_t p = 0; p < N; ++p)
            if (acc[p] != 0.0L) { w->idx[nnz] = p; w->val[nnz] = acc[p]; ++nnz; }
        w->nnz = nnz;
        free(acc);
    } else {
        w->buf0 = (long double *)malloc(sizeof(long double) * (size_t)N);
        w->buf1 = (long double *)malloc(sizeof(long double) * (size_t)N);
        w->pref = (long double *)malloc(sizeof(long double) * (size_t)(2 * N + 1));
        if (!w->buf0 || !w->buf1 || !w->pref) { wop_free(w); return DIF_ERR_NOMEM; }
    }
    return DIF_OK;
}

/*
 * Periodic box sum of length L.  causal: y_i = sum_{t=0}^{L-1} x_{(i-t) mod N};
 * otherwise y_i = sum_{t=0}^{L-1} x_{(i+t) mod N}.  A window longer than N
 * covers the whole period (L div N) times plus a partial window of
 * (L mod N) samples, read off prefix sums over two periods.
 */
static void box_sum(const long double *x, long double *y, long double *pref,
                    int64_t N, int64_t L, int causal)
{
    pref[0] = 0.0L;
    for (int64_t j = 0; j < 2 * N; ++j) pref[j + 1] = pref[j] + x[j % N];
    long double total = pref[N];
    int64_t q = L / N, rem = L % N;
    for (int64_t i = 0; i < N; ++i) {
        long double part;
        if (causal)
            part = pref[i + N + 1] - pref[i + N + 1 - rem];
        else
            part = pref[i + rem] - pref[i];
        y[i] = (long double)q * total + part;
    }
}

/* a = W x */
static void wop_apply(wop *w, const double *x, double *a)
{
    int64_t N = w->N;
    if (w->form == 0) {
        for (int64_t i = 0; i < N; ++i) {
            long double s = 0.0L;
            for (int64_t z = 0; z < w->nnz; ++z) {
                int64_t j = i - w->idx[z];
                if (j < 0) j += N;
                s += w->val[z] * (long double)x[j];
            }
            a[i] = (double)(s / w->L4);
        }
    } else {
        for (int64_t i = 0; i < N; ++i) w->buf0[i] = (long double)x[i];
        /* W = (1/L^4) C A C A with C causal and A anticausal boxes */
        box_sum(w->buf0, w->buf1, w->pref, N, w->L, 0);
        box_sum(w->buf1, w->buf0, w->pref, N, w->L, 1);
        box_sum(w->buf0, w->buf1, w->pref, N, w->L, 0);
        box_sum(w->buf1, w->buf0, w->pref, N, w->L, 1);
        for (int64_t i = 0; i < N; ++i) a[i] = (double)(w->buf0[i] / w->L4);
    }
}

int dif_apply_window(const double *x, int64_t N, int64_t L, int32_t form, double *a)
{
    if (N < 1 || L < 1 || !x || !a) return DIF_ERR_ARG;
    wop w;
    int st = wop_init(&w, N, L, form);
    if (st) return st;
    wop_apply(&w, x, a);
    wop_free(&w);
    return DIF_OK;
}

static long double sumsq(const double *x, int64_t n)
{
    long double s = 0.0L;
    for (int64_t i = 0; i < n; ++i) s += (long double)x[i] * (long double)x[i];
    return s;
}

/*
 * Run n_steps applications of (I - W) from s (in place) and record, per
 * step m = 1..n_steps, SD_m and the absolute step ||s_m - s_{m-1}||.
 * Used to check monotonicity, the a-priori bound and the one-tone decay.
 */
int dif_inner_trace(double *s, int64_t N, int64_t L, int32_t form, int64_t n_steps,
                    double *sd_out, double *step_norm_out)
{
    if (N < 1 || L < 1 || n_steps < 0 || !s) return DIF_ERR_ARG;
    wop w;
    int st = wop_init(&w, N, L, form);
    if (st) return st;
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    if (!a) { wop_free(&w); return DIF_ERR_NOMEM; }
    for (int64_t m = 0; m < n_steps; ++m) {
        wop_apply(&w, s, a);
        long double na = sumsq(a, N), ns = sumsq(s, N);
        if (sd_out) sd_out[m] = (ns > 0.0L) ? (double)sqrtl(na / ns) : 0.0;
        if (step_norm_out) step_norm_out[m] = (double)sqrtl(na);
        for (int64_t i = 0; i < N; ++i) s[i] = s[i] - a[i];
    }
    free(a);
    wop_free(&w);
    return DIF_OK;
}

/* ------------------------------------------------------------------ */
/* the whole decomposition (Algorithm 2)                                */
/* ------------------------------------------------------------------ */

/*
 * s[N] in; imfs[max_imfs][N] and remainder[N] out; info[max_imfs] out.
 * Rows of imfs past *n_imfs are zero.  Returns DIF_OK or an error code.
 */
int dif_decompose(const double *s, int64_t N, double delta, int32_t max_imfs,
                  const dif_opts *opt, double *imfs, double *remainder,
                  int32_t *n_imfs, dif_imf_info *info, int32_t *stop_reason)
{
    if (!s || N < 1 || !(delta > 0.0) || max_imfs < 0 || !opt || !remainder || !n_imfs)
        return DIF_ERR_ARG;
    if (max_imfs > 0 && !imfs) return DIF_ERR_ARG;
    if (opt->max_inner < 1) return DIF_ERR_ARG;

    double *r = (double *)malloc(sizeof(double) * (size_t)N);
    double *x = (double *)malloc(sizeof(double) * (size_t)N);
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    if (!r || !x || !a) { free(r); free(x); free(a); return DIF_ERR_NOMEM; }

    memcpy(r, s, sizeof(double) * (size_t)N);
    double maxs = 0.0;
    for (int64_t i = 0; i < N; ++i) if (fabs(s[i]) > maxs) maxs = fabs(s[i]);
    if (max_imfs > 0) memset(imfs, 0, sizeof(double) * (size_t)N * (size_t)max_imfs);

    int32_t count = 0;
    int32_t reason = DIF_STOP_MAX_IMFS;
    int status = DIF_OK;
    for (int32_t j = 0; j < max_imfs; ++j) {
        /* rounding floor */
        long double sum = 0.0L;
        for (int64_t i = 0; i < N; ++i) sum += r[i];
        double mean = (double)(sum / (long double)N);
        double dev = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double d = fabs(r[i] - mean);
            if (d > dev) dev = d;
        }
        double thr = opt->floor_tau * maxs;
        double floor_ratio = (thr > 0.0) ? dev / thr : (dev > 0.0 ? INFINITY : 0.0);
        if (dev <= thr) { reason = DIF_STOP_FLOOR; break; }

        double margin_k;
        int64_t k = dif_count_extrema(r, N, &margin_k);
        if (k < 2) { reason = DIF_STOP_FEW_EXTREMA; break; }
        int64_t L = dif_mask_length(N, k, opt->mask_rule, opt->nu);

        wop w;
        status = wop_init(&w, N, L, opt->inner_form);
        if (status) break;
        memcpy(x, r, sizeof(double) * (size_t)N);
        int64_t m = 0;
        double sd = 0.0, sd_prev = INFINITY;
        int32_t flags = 0;
        for (;;) {
            wop_apply(&w, x, a);
            long double na = sumsq(a, N), nx = sumsq(x, N);
            double cur = (nx > 0.0L) ? (double)sqrtl(na / nx) : 0.0;
            for (int64_t i = 0; i < N; ++i) x[i] = x[i] - a[i];
            ++m;
            sd_prev = sd;
            sd = cur;
            if (m == 1) sd_prev = INFINITY;
            if (sd <= delta) break;
            if (m >= opt->max_inner) { flags |= DIF_FLAG_CAP; break; }
        }
        wop_free(&w);

        double *imf = imfs + (size_t)j * (size_t)N;
        memcpy(imf, x, sizeof(double) * (size_t)N);
        for (int64_t i = 0; i < N; ++i) r[i] = r[i] - x[i];
        if (info) {
            info[j].k = k; info[j].L = L; info[j].m = m;
            info[j].sd = sd; info[j].sd_prev = sd_prev;
            info[j].margin_k = margin_k; info[j].floor_ratio = floor_ratio;
            info[j].flags = flags; info[j].pad = 0;
        }
        ++count;
    }
    memcpy(remainder, r, sizeof(double) * (size_t)N);
    *n_imfs = count;
    if (stop_reason) *stop_reason = reason;
    free(r); free(x); free(a);
    return status;
}
