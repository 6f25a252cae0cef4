/*
 * sdc_oracle.c -- plain FP64 CPU reference for the binned space- and
 * time-displaced spin pair correlation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it is used by the tests, by the smoke check and by the
 * benchmark's CPU-baseline leg.  It shares no code, header, table or constant
 * generator with the GPU path.
 *
 * What it computes (paper: "Kernel Fusion in Atomistic Spin Dynamics
 * Simulations on Nvidia GPUs using Tensor Core", arXiv 2308.07487):
 *
 *  - the pair correlation of Eq. (4), in its unsubtracted form
 *    <S_i(t0) . S_j(t0 + t)> and, as its second term, the product of the
 *    per-site averages <S_i(t0)> . <S_j(t0 + t)> that the connected form
 *    subtracts, summed over the three components alpha as in
 *    Eq. (3), averaged over time origins t0 = o*s (o = 0..n_o-1) instead of
 *    Monte Carlo realizations, and binned by the displacement of site j (the
 *    later time) relative to site i (the origin);
 *  - for every pair the origin/component sum is the GEMM element of the
 *    N x 3M by 3M x N product of Sec. 3.2; here it is a plain dot product;
 *  - the bin key plays the role of the per-element weight Q(i,j) of Eq. (6):
 *    a value computed from the two positions only;
 *  - the windowed time transform of Sec. 2.2 (the paper uses an FFT plus a
 *    NumPy window; here a direct DFT with the half-Hann window);
 *  - the Landau-Lifshitz equation Eq. (2) for the exchange term of Eq. (1),
 *    integrated with classical RK4 without renormalisation (Sec. 3.1);
 *  - Philox4x32-10 (Salmon et al., SC'11) for seeded initial states.
 *
 * Everything is FP64 except where the bin rule itself is defined in FP32
 * (the radial squared distance, compared against FP32 shell edges).  Build
 * with -ffp-contract=off so that rule is evaluated exactly as written.
 *
 * Parity pins: every function here is pinned in tests/test_oracle.py against
 * closed forms, invariants, numpy library routines or brute force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_SC 0
#define OR_BCC 1
#define OR_RADIAL 2

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 3

/* ------------------------------------------------------------------------ */
/* Bin keys                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int kind;
    int L[3];
    int64_t n;
    int64_t n_bins;
    int32_t *cell;  /* periodic: integer cell coordinates [n][3], in [0, L) */
    int32_t *beta;  /* bcc: sublattice 0 (corner) or 1 (body centre)        */
    const float *pos; /* radial: positions [n][3]                           */
    float *e2;      /* radial: squared shell edges, e2[k] = fp32((k w)^2)   */
    int n_shells;
} okeys;

static int64_t pmod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

/* Periodic lattices: positions must be lattice points (lattice constant 1).
 * sc sites sit at integer points; bcc sites at n or n + (1/2,1/2,1/2).
 * Every site of the L0 x L1 x L2 cell (x2 for bcc) must appear exactly once.
 * Radial: squared edges of n_shells shells of width r_max / n_shells. */
static int okeys_init(okeys *k, const float *pos, int64_t n, int kind,
                      const int32_t *L, int32_t n_shells, float r_max) {
    memset(k, 0, sizeof(*k));
    k->kind = kind;
    k->n = n;
    if (n <= 0 || !pos) return OR_EINVAL;
    if (kind == OR_RADIAL) {
        if (n_shells <= 0 || !(r_max > 0.0f)) return OR_EINVAL;
        k->pos = pos;
        k->n_shells = n_shells;
        k->n_bins = n_shells;
        k->e2 = (float *)malloc(sizeof(float) * (size_t)n_shells);
        if (!k->e2) return OR_ENOMEM;
        double w = (double)r_max / (double)n_shells;
        for (int s = 0; s < n_shells; ++s) {
            double e = (double)s * w;
            k->e2[s] = (float)(e * e);
        }
        return OR_OK;
    }
    if (kind != OR_SC && kind != OR_BCC) return OR_EINVAL;
    for (int a = 0; a < 3; ++a) {
        if (!L || L[a] <= 0) return OR_EINVAL;
        k->L[a] = L[a];
    }
    int64_t cells = (int64_t)L[0] * L[1] * L[2];
    int64_t expect = kind == OR_SC ? cells : 2 * cells;
    if (n != expect) return OR_EINVAL;
    k->n_bins = expect;
    k->cell = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)n);
    k->beta = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    unsigned char *seen = (unsigned char *)calloc((size_t)expect, 1);
    if (!k->cell || !k->beta || !seen) {
        free(seen);
        return OR_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        int b = 0;
        int32_t c[3];
        if (kind == OR_SC) {
            for (int a = 0; a < 3; ++a) {
                double p = pos[3 * i + a];
                double r = floor(p + 0.5);
                if (fabs(p - r) > 1e-3) { free(seen); return OR_EINVAL; }
                c[a] = (int32_t)pmod((int64_t)r, L[a]);
            }
        } else {
            int64_t d[3];
            for (int a = 0; a < 3; ++a) {
                double p = 2.0 * pos[3 * i + a];
                double r = floor(p + 0.5);
                if (fabs(p - r) > 2e-3) { free(seen); return OR_EINVAL; }
                d[a] = (int64_t)r;
            }
            b = (int)pmod(d[0], 2);
            if (pmod(d[1], 2) != b || pmod(d[2], 2) != b) { free(seen); return OR_EINVAL; }
            for (int a = 0; a < 3; ++a) c[a] = (int32_t)pmod((d[a] - b) / 2, L[a]);
        }
        int64_t idx = ((int64_t)c[0] * L[1] + c[1]) * L[2] + c[2];
        if (kind == OR_BCC) idx = 2 * idx + b;
        if (seen[idx]) { free(seen); return OR_EINVAL; }
        seen[idx] = 1;
        k->cell[3 * i + 0] = c[0];
        k->cell[3 * i + 1] = c[1];
        k->cell[3 * i + 2] = c[2];
        k->beta[i] = b;
    }
    free(seen);
    return OR_OK;
}

static void okeys_free(okeys *k) {
    free(k->cell);
    free(k->beta);
    free(k->e2);
    k->cell = NULL;
    k->beta = NULL;
    k->e2 = NULL;
}

/* Radial shell of one squared distance: the largest s with e2[s] <= d2
 * (e2[0] = 0, so s >= 0; distances beyond the last edge fall in the last
 * shell). */
static int64_t oshell(const okeys *k, float d2) {
    int lo = 0, hi = k->n_shells - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (k->e2[mid] <= d2) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* Bin of the ordered pair (i = origin site, j = later site). */
static int64_t okey(const okeys *k, int64_t i, int64_t j) {
    if (k->kind == OR_RADIAL) {
        const float *pi = k->pos + 3 * i, *pj = k->pos + 3 * j;
        float dx = pj[0] - pi[0];
        float dy = pj[1] - pi[1];
        float dz = pj[2] - pi[2];
        float d2 = (dx * dx + dy * dy) + dz * dz;
        return oshell(k, d2);
    }
    const int32_t *ci = k->cell + 3 * i, *cj = k->cell + 3 * j;
    int64_t shift = 0;
    if (k->kind == OR_BCC && k->beta[j] < k->beta[i]) shift = 1;
    int64_t kx = pmod((int64_t)cj[0] - ci[0] - shift, k->L[0]);
    int64_t ky = pmod((int64_t)cj[1] - ci[1] - shift, k->L[1]);
    int64_t kz = pmod((int64_t)cj[2] - ci[2] - shift, k->L[2]);
    int64_t b = (kx * k->L[1] + ky) * k->L[2] + kz;
    if (k->kind == OR_BCC) b = 2 * b + pmod((int64_t)k->beta[j] - k->beta[i], 2);
    return b;
}

int oracle_n_bins(const float *pos, int64_t n, int kind, const int32_t *L,
                  int32_t n_shells, float r_max, int64_t *n_bins) {
    okeys k;
    int rc = okeys_init(&k, pos, n, kind, L, n_shells, r_max);
    if (rc == OR_OK) *n_bins = k.n_bins;
    okeys_free(&k);
    return rc;
}

/* Keys of a list of ordered pairs (used by the key-spec tests). */
int oracle_pair_keys(const float *pos, int64_t n, int kind, const int32_t *L,
                     int32_t n_shells, float r_max, const int64_t *pi,
                     const int64_t *pj, int64_t n_pairs, int64_t *out) {
    okeys k;
    int rc = okeys_init(&k, pos, n, kind, L, n_shells, r_max);
    if (rc != OR_OK) { okeys_free(&k); return rc; }
    for (int64_t p = 0; p < n_pairs; ++p) {
        if (pi[p] < 0 || pi[p] >= n || pj[p] < 0 || pj[p] >= n) { okeys_free(&k); return OR_EINVAL; }
        out[p] = okey(&k, pi[p], pj[p]);
    }
    okeys_free(&k);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Binned correlation                                                        */
/* ------------------------------------------------------------------------ */

/* G_t[i][j] = sum over origins o and components alpha of
 *             S_i^alpha(o*s) * S_j^alpha(o*s + t)        (FP64)
 * This is one element of the per-lag GEMM of Sec. 3.2. */
static double opair(const float *frames, int64_t n, int64_t i, int64_t j,
                    int32_t n_origins, int32_t stride, int32_t lag) {
    double g = 0.0;
    for (int32_t o = 0; o < n_origins; ++o) {
        const float *si = frames + ((int64_t)o * stride * n + i) * 3;
        const float *sj = frames + (((int64_t)o * stride + lag) * n + j) * 3;
        g += (double)si[0] * (double)sj[0];
        g += (double)si[1] * (double)sj[1];
        g += (double)si[2] * (double)sj[2];
    }
    return g;
}

static int check_frames(int64_t n_frames, int32_t n_origins, int32_t stride,
                        const int32_t *lags, int32_t n_lags) {
    if (n_origins <= 0 || stride <= 0 || n_lags < 0) return OR_EINVAL;
    for (int32_t l = 0; l < n_lags; ++l) {
        if (lags[l] < 0) return OR_EINVAL;
        if ((int64_t)(n_origins - 1) * stride + lags[l] >= n_frames) return OR_EINVAL;
    }
    return OR_OK;
}

/*
 * H[l][b] += sum over i in [i_begin, i_end), all j, of G_{lags[l]}[i][j] for
 * key(i,j) = b; counts[b] += number of those ordered pairs (i, j), i = j
 * included.  frames: [n_frames][n][3] fp32.  H: [n_lags][n_bins] fp64.
 * counts may be NULL.  n_threads <= 0 means the OpenMP default.
 * Per-thread private histograms, merged in thread order.
 */
int oracle_binned_corr(const float *pos, int64_t n, int kind, const int32_t *L,
                       int32_t n_shells, float r_max, const float *frames,
                       int64_t n_frames, int32_t n_origins, int32_t stride,
                       const int32_t *lags, int32_t n_lags, int64_t i_begin,
                       int64_t i_end, double *H, uint64_t *counts,
                       int n_threads) {
    okeys k;
    int rc = okeys_init(&k, pos, n, kind, L, n_shells, r_max);
    if (rc != OR_OK) { okeys_free(&k); return rc; }
    rc = check_frames(n_frames, n_origins, stride, lags, n_lags);
    if (rc != OR_OK || i_begin < 0 || i_end > n || i_begin > i_end) {
        okeys_free(&k);
        return OR_EINVAL;
    }
    const int64_t nb = k.n_bins;
    int nt = 1;
#ifdef _OPENMP
    nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nt * (size_t)n_lags * (size_t)nb, sizeof(double));
    uint64_t *pcnt = counts ? (uint64_t *)calloc((size_t)nt * (size_t)nb, sizeof(uint64_t)) : NULL;
    if (!priv || (counts && !pcnt)) {
        free(priv); free(pcnt); okeys_free(&k);
        return OR_ENOMEM;
    }
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *h = priv + (size_t)tid * n_lags * nb;
        uint64_t *c = pcnt ? pcnt + (size_t)tid * nb : NULL;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
        for (int64_t i = i_begin; i < i_end; ++i) {
            for (int64_t j = 0; j < n; ++j) {
                int64_t b = okey(&k, i, j);
                if (c) c[b] += 1;
                for (int32_t l = 0; l < n_lags; ++l)
                    h[(size_t)l * nb + b] += opair(frames, n, i, j, n_origins, stride, lags[l]);
            }
        }
    }
    for (int t = 0; t < nt; ++t) {
        const double *h = priv + (size_t)t * n_lags * nb;
        for (int64_t x = 0; x < (int64_t)n_lags * nb; ++x) H[x] += h[x];
        if (counts)
            for (int64_t b = 0; b < nb; ++b) counts[b] += pcnt[(size_t)t * nb + b];
    }
    free(priv);
    free(pcnt);
    okeys_free(&k);
    return OR_OK;
}

/*
 * Selected bins only: H_sel[l][s] += H[lags[l]][bins[s]] over all ordered
 * pairs.  Scans every pair's key and evaluates the dot product only for
 * pairs falling in a selected bin, so full-size samples stay cheap.
 */
int oracle_binned_corr_select(const float *pos, int64_t n, int kind,
                              const int32_t *L, int32_t n_shells, float r_max,
                              const float *frames, int64_t n_frames,
                              int32_t n_origins, int32_t stride,
                              const int32_t *lags, int32_t n_lags,
                              const int64_t *bins, int32_t n_sel, double *H_sel,
                              uint64_t *counts_sel, int n_threads) {
    okeys k;
    int rc = okeys_init(&k, pos, n, kind, L, n_shells, r_max);
    if (rc != OR_OK) { okeys_free(&k); return rc; }
    rc = check_frames(n_frames, n_origins, stride, lags, n_lags);
    if (rc != OR_OK || n_sel < 0) { okeys_free(&k); return OR_EINVAL; }
    int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)k.n_bins);
    if (!slot) { okeys_free(&k); return OR_ENOMEM; }
    for (int64_t b = 0; b < k.n_bins; ++b) slot[b] = -1;
    for (int32_t s = 0; s < n_sel; ++s) {
        if (bins[s] < 0 || bins[s] >= k.n_bins || slot[bins[s]] >= 0) {
            free(slot); okeys_free(&k);
            return OR_EINVAL;
        }
        slot[bins[s]] = s;
    }
    int nt = 1;
#ifdef _OPENMP
    nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nt * n_lags * (size_t)(n_sel > 0 ? n_sel : 1), sizeof(double));
    uint64_t *pc = (uint64_t *)calloc((size_t)nt * (size_t)(n_sel > 0 ? n_sel : 1), sizeof(uint64_t));
    if (!priv || !pc) { free(priv); free(pc); free(slot); okeys_free(&k); return OR_ENOMEM; }
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *h = priv + (size_t)tid * n_lags * n_sel;
        uint64_t *c = pc + (size_t)tid * n_sel;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t j = 0; j < n; ++j) {
                int32_t s = slot[okey(&k, i, j)];
                if (s < 0) continue;
                c[s] += 1;
                for (int32_t l = 0; l < n_lags; ++l)
                    h[(size_t)l * n_sel + s] += opair(frames, n, i, j, n_origins, stride, lags[l]);
            }
        }
    }
    for (int t = 0; t < nt; ++t) {
        for (int64_t x = 0; x < (int64_t)n_lags * n_sel; ++x) H_sel[x] += priv[(size_t)t * n_lags * n_sel + x];
        if (counts_sel)
            for (int32_t s = 0; s < n_sel; ++s) counts_sel[s] += pc[(size_t)t * n_sel + s];
    }
    free(priv); free(pc); free(slot); okeys_free(&k);
    return OR_OK;
}

/* Per-site averages over the origins, Eq. (4): out[i] = (1/n_o) sum_o
 * S_i(o*s + shift), FP64, [n][3]. */
static void omean(const float *frames, int64_t n, int32_t n_origins, int32_t stride,
                  int32_t shift, double *out) {
    for (int64_t i = 0; i < n; ++i) {
        double a[3] = {0.0, 0.0, 0.0};
        for (int32_t o = 0; o < n_origins; ++o) {
            const float *x = frames + (((int64_t)o * stride + shift) * n + i) * 3;
            a[0] += (double)x[0];
            a[1] += (double)x[1];
            a[2] += (double)x[2];
        }
        for (int c = 0; c < 3; ++c) out[3 * i + c] = a[c] / (double)n_origins;
    }
}

/*
 * Second term of Eq. (4), binned like H: P[l][b] += n_o * sum over ordered
 * pairs (i, j), i in [i_begin, i_end), key(i, j) = b, of
 *     <S_i(t0)> . <S_j(t0 + lags[l])>,
 * where <.> averages over the origins t0 = o*s, o < n_o.  With bins != NULL
 * only the n_sel listed bins are accumulated (P: [n_lags][n_sel]); otherwise
 * P is [n_lags][n_bins].  The connected correlation is H - P.
 */
int oracle_mean_product(const float *pos, int64_t n, int kind, const int32_t *L,
                        int32_t n_shells, float r_max, const float *frames,
                        int64_t n_frames, int32_t n_origins, int32_t stride,
                        const int32_t *lags, int32_t n_lags, int64_t i_begin,
                        int64_t i_end, const int64_t *bins, int32_t n_sel,
                        double *P, int n_threads) {
    okeys k;
    int rc = okeys_init(&k, pos, n, kind, L, n_shells, r_max);
    if (rc != OR_OK) { okeys_free(&k); return rc; }
    rc = check_frames(n_frames, n_origins, stride, lags, n_lags);
    if (rc != OR_OK || i_begin < 0 || i_end > n || i_begin > i_end || (bins && n_sel < 0)) {
        okeys_free(&k);
        return OR_EINVAL;
    }
    const int64_t width = bins ? n_sel : k.n_bins;
    int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)k.n_bins);
    double *m0 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *mt = (double *)malloc(sizeof(double) * 3 * (size_t)n * (size_t)(n_lags > 0 ? n_lags : 1));
    if (!slot || !m0 || !mt) { free(slot); free(m0); free(mt); okeys_free(&k); return OR_ENOMEM; }
    for (int64_t b = 0; b < k.n_bins; ++b) slot[b] = bins ? -1 : (int32_t)b;
    if (bins) {
        for (int32_t q = 0; q < n_sel; ++q) {
            if (bins[q] < 0 || bins[q] >= k.n_bins || slot[bins[q]] >= 0) {
                free(slot); free(m0); free(mt); okeys_free(&k);
                return OR_EINVAL;
            }
            slot[bins[q]] = q;
        }
    }
    omean(frames, n, n_origins, stride, 0, m0);
    for (int32_t l = 0; l < n_lags; ++l) omean(frames, n, n_origins, stride, lags[l], mt + (size_t)l * 3 * n);
    int nt = 1;
#ifdef _OPENMP
    nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nt * n_lags * (size_t)(width > 0 ? width : 1), sizeof(double));
    if (!priv) { free(slot); free(m0); free(mt); okeys_free(&k); return OR_ENOMEM; }
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *h = priv + (size_t)tid * n_lags * width;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t i = i_begin; i < i_end; ++i) {
            for (int64_t j = 0; j < n; ++j) {
                const int32_t q = slot[okey(&k, i, j)];
                if (q < 0) continue;
                for (int32_t l = 0; l < n_lags; ++l) {
                    const double *a = m0 + 3 * i;
                    const double *b = mt + ((size_t)l * n + j) * 3;
                    h[(size_t)l * width + q] += (double)n_origins * (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
                }
            }
        }
    }
    for (int t = 0; t < nt; ++t)
        for (int64_t x = 0; x < (int64_t)n_lags * width; ++x) P[x] += priv[(size_t)t * n_lags * width + x];
    free(priv); free(slot); free(m0); free(mt); okeys_free(&k);
    return OR_OK;
}

/* Self part of the second term of Eq. (4):
 * out[l] += n_o * sum_i <S_i(t0)> . <S_i(t0 + lags[l])>. */
int oracle_self_mean_product(const float *frames, int64_t n, int64_t n_frames,
                             int32_t n_origins, int32_t stride, const int32_t *lags,
                             int32_t n_lags, double *out) {
    int rc = check_frames(n_frames, n_origins, stride, lags, n_lags);
    if (rc != OR_OK || n <= 0) return OR_EINVAL;
    double *m0 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *mt = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!m0 || !mt) { free(m0); free(mt); return OR_ENOMEM; }
    omean(frames, n, n_origins, stride, 0, m0);
    for (int32_t l = 0; l < n_lags; ++l) {
        omean(frames, n, n_origins, stride, lags[l], mt);
        double s = 0.0;
        for (int64_t i = 0; i < 3 * n; ++i) s += m0[i] * mt[i];
        out[l] += (double)n_origins * s;
    }
    free(m0); free(mt);
    return OR_OK;
}

/* Self term: out[l] += sum_o sum_i S_i(o*s) . S_i(o*s + lags[l]). */
int oracle_self_corr(const float *frames, int64_t n, int64_t n_frames,
                     int32_t n_origins, int32_t stride, const int32_t *lags,
                     int32_t n_lags, double *out) {
    int rc = check_frames(n_frames, n_origins, stride, lags, n_lags);
    if (rc != OR_OK || n <= 0) return OR_EINVAL;
    for (int32_t l = 0; l < n_lags; ++l) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += opair(frames, n, i, i, n_origins, stride, lags[l]);
        out[l] += s;
    }
    return OR_OK;
}

/* Windowed DFT of the time series x[0..m): the half-Hann window
 * w_t = (1 + cos(pi t / m)) / 2 (one-sided, w_0 = 1), then
 * X_k = sum_t w_t x_t exp(-2 pi i k t / m), k = 0..m-1.  out: [m][2]. */
int oracle_dft(const double *x, int32_t m, double *out) {
    if (m <= 0) return OR_EINVAL;
    const double pi = 3.14159265358979323846;
    for (int32_t kk = 0; kk < m; ++kk) {
        double re = 0.0, im = 0.0;
        for (int32_t t = 0; t < m; ++t) {
            double w = 0.5 * (1.0 + cos(pi * (double)t / (double)m));
            /* reduce k*t mod m first so the angle stays small and exact */
            int64_t kt = ((int64_t)kk * t) % m;
            double ang = -2.0 * pi * (double)kt / (double)m;
            re += w * x[t] * cos(ang);
            im += w * x[t] * sin(ang);
        }
        out[2 * kk] = re;
        out[2 * kk + 1] = im;
    }
    return OR_OK;
}

/*
 * Normalisation and spectra.
 *   C[l][b]  = H[l][b] / (n_org[l] * count[b])   (0 where count or n_org is 0)
 *   Csum[l]  = sum_b H[l][b] / (N * n_org[l])
 *   Cself[l] = self[l] / (N * n_org[l])
 *   Ssum = DFT(Csum), Sself = DFT(Cself)   (only when the lags are 0..m-1)
 */
int oracle_finalize(const double *H, const uint64_t *counts, int64_t n_bins,
                    int32_t n_lags, int64_t n_sites, const double *n_org,
                    const double *self, double *C, double *Csum, double *Cself,
                    double *Ssum, double *Sself) {
    if (n_bins <= 0 || n_lags <= 0 || n_sites <= 0) return OR_EINVAL;
    for (int32_t l = 0; l < n_lags; ++l) {
        double tot = 0.0;
        for (int64_t b = 0; b < n_bins; ++b) {
            double h = H[(size_t)l * n_bins + b];
            tot += h;
            double den = n_org[l] * (double)counts[b];
            C[(size_t)l * n_bins + b] = den > 0.0 ? h / den : 0.0;
        }
        double d = (double)n_sites * n_org[l];
        Csum[l] = d > 0.0 ? tot / d : 0.0;
        Cself[l] = d > 0.0 ? self[l] / d : 0.0;
    }
    int rc = oracle_dft(Csum, n_lags, Ssum);
    if (rc == OR_OK) rc = oracle_dft(Cself, n_lags, Sself);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Landau-Lifshitz RK4 (Eq. 2 with the Hamiltonian of Eq. 1)                 */
/* ------------------------------------------------------------------------ */

/*
 * Couplings as a CSR list: for site i, neighbours col[row[i]..row[i+1]) with
 * exchange J[...] and DMI vectors Dv[3 (...)] of the ordered pair (i, j),
 * D_ji = -D_ij.  H = sum over bonds (each once) of J_ij S_i.S_j
 * - D_ij.(S_i x S_j), minus A sum_i (S_i^z)^2 and H_z sum_i S_i^z (Eq. (1)),
 * so dH/dS_i = sum_j (J_ij S_j + D_ij x S_j) - 2 A S_i^z z - H_z z, and
 * Eq. (2) gives dS_i/dt = (dH/dS_i) x S_i.
 */
static void oderiv(int64_t n, const int64_t *row, const int32_t *col,
                   const double *J, const double *Dv, double A, double Hz,
                   const double *S, double *D) {
    for (int64_t i = 0; i < n; ++i) {
        const double *si = S + 3 * i;
        /* h = dH/dS_i of Eq. (1): exchange, DMI, anisotropy, field */
        double h0 = 0.0, h1 = 0.0, h2 = 0.0;
        for (int64_t e = row[i]; e < row[i + 1]; ++e) {
            const double *sj = S + 3 * (int64_t)col[e];
            h0 += J[e] * sj[0];
            h1 += J[e] * sj[1];
            h2 += J[e] * sj[2];
            if (Dv) {
                /* -D_ij.(S_i x S_j) = S_i.(D_ij x S_j): gradient D_ij x S_j */
                const double *d = Dv + 3 * e;
                h0 += d[1] * sj[2] - d[2] * sj[1];
                h1 += d[2] * sj[0] - d[0] * sj[2];
                h2 += d[0] * sj[1] - d[1] * sj[0];
            }
        }
        h2 += -2.0 * A * si[2] - Hz;
        D[3 * i + 0] = h1 * si[2] - h2 * si[1];
        D[3 * i + 1] = h2 * si[0] - h0 * si[2];
        D[3 * i + 2] = h0 * si[1] - h1 * si[0];
    }
}

/*
 * Classical RK4 with step dt, no renormalisation, for Eq. (2) with the
 * Hamiltonian of Eq. (1): dS_i/dt = h_i x S_i,
 *   h_i = sum_j J_ij S_j + sum_j D_ij x S_j - 2 A S_i^z z - H_z z,
 * CSR bonds (row, col, J; Dv: [nnz][3] DMI vectors of the ordered pairs, or
 * NULL for none).  init: [n][3] (fp32 input state, promoted).  frames_out:
 * [n_frames][n][3] fp64; frame 0 is the initial state and frame f the state
 * after f steps.
 */
int oracle_ll_rk4_full(int64_t n, const int64_t *row, const int32_t *col,
                       const double *J, const double *Dv, double A, double Hz,
                       const float *init, double dt, int64_t n_frames,
                       double *frames_out) {
    if (n <= 0 || n_frames <= 0) return OR_EINVAL;
    size_t m = 3 * (size_t)n;
    double *S = (double *)malloc(sizeof(double) * m);
    double *T = (double *)malloc(sizeof(double) * m);
    double *k1 = (double *)malloc(sizeof(double) * m);
    double *k2 = (double *)malloc(sizeof(double) * m);
    double *k3 = (double *)malloc(sizeof(double) * m);
    double *k4 = (double *)malloc(sizeof(double) * m);
    if (!S || !T || !k1 || !k2 || !k3 || !k4) {
        free(S); free(T); free(k1); free(k2); free(k3); free(k4);
        return OR_ENOMEM;
    }
    for (size_t x = 0; x < m; ++x) S[x] = (double)init[x];
    memcpy(frames_out, S, sizeof(double) * m);
    for (int64_t f = 1; f < n_frames; ++f) {
        oderiv(n, row, col, J, Dv, A, Hz, S, k1);
        for (size_t x = 0; x < m; ++x) T[x] = S[x] + 0.5 * dt * k1[x];
        oderiv(n, row, col, J, Dv, A, Hz, T, k2);
        for (size_t x = 0; x < m; ++x) T[x] = S[x] + 0.5 * dt * k2[x];
        oderiv(n, row, col, J, Dv, A, Hz, T, k3);
        for (size_t x = 0; x < m; ++x) T[x] = S[x] + dt * k3[x];
        oderiv(n, row, col, J, Dv, A, Hz, T, k4);
        for (size_t x = 0; x < m; ++x)
            S[x] += dt / 6.0 * (k1[x] + 2.0 * k2[x] + 2.0 * k3[x] + k4[x]);
        memcpy(frames_out + (size_t)f * m, S, sizeof(double) * m);
    }
    free(S); free(T); free(k1); free(k2); free(k3); free(k4);
    return OR_OK;
}

/* The exchange-only form (no DMI, anisotropy or field). */
int oracle_ll_rk4(int64_t n, const int64_t *row, const int32_t *col,
                  const double *J, const float *init, double dt,
                  int64_t n_frames, double *frames_out) {
    return oracle_ll_rk4_full(n, row, col, J, NULL, 0.0, 0.0, init, dt, n_frames, frames_out);
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                         */
/* ------------------------------------------------------------------------ */

static void ophilox(uint32_t ctr[4], uint32_t key0, uint32_t key1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key0, k1 = key1;
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    ctr[0] = c0; ctr[1] = c1; ctr[2] = c2; ctr[3] = c3;
}

/* One raw Philox4x32-10 block: out = philox(ctr, key). */
int oracle_philox_block(const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    ophilox(c, key[0], key[1]);
    memcpy(out, c, sizeof(c));
    return OR_OK;
}

/* Raw Philox blocks for counters (c0, c1, c2, c3) = (idx, draw, 0, 0) and key
 * (seed low, seed high): out[4*x .. 4*x+3] for x = 0..n_blocks-1 with
 * idx = idx0 + x. */
int oracle_philox(uint64_t seed, uint32_t draw, int64_t idx0, int64_t n_blocks,
                  uint32_t *out) {
    for (int64_t x = 0; x < n_blocks; ++x) {
        uint32_t c[4] = {(uint32_t)(idx0 + x), draw, (uint32_t)((uint64_t)(idx0 + x) >> 32), 0u};
        ophilox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        memcpy(out + 4 * x, c, sizeof(c));
    }
    return OR_OK;
}

/* 24-bit uniform in [0, 1) from one 32-bit word. */
static double ounif(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

/*
 * Seeded initial states from Philox blocks (counter idx = site, draw 0):
 *   mode 0: uniform unit vectors, z = 2u0 - 1, phi = 2 pi u1;
 *   mode 1: perturbed z-aligned start: tangent v = sigma * (g0, g1) with
 *           Box-Muller normals from (u0, u1), S = (sin|v| v/|v|, cos|v|).
 * out: [n][3] fp64.
 */
int oracle_init_state(uint64_t seed, int64_t n, int mode, double sigma, double *out) {
    const double pi = 3.14159265358979323846;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t c[4] = {(uint32_t)i, 0u, (uint32_t)((uint64_t)i >> 32), 0u};
        ophilox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        double u0 = ounif(c[0]), u1 = ounif(c[1]);
        if (mode == 0) {
            double z = 2.0 * u0 - 1.0;
            double r = sqrt(fmax(0.0, 1.0 - z * z));
            double ph = 2.0 * pi * u1;
            out[3 * i + 0] = r * cos(ph);
            out[3 * i + 1] = r * sin(ph);
            out[3 * i + 2] = z;
        } else if (mode == 1) {
            double rr = sqrt(-2.0 * log(1.0 - u0));
            double g0 = rr * cos(2.0 * pi * u1), g1 = rr * sin(2.0 * pi * u1);
            double v0 = sigma * g0, v1 = sigma * g1;
            double a = sqrt(v0 * v0 + v1 * v1);
            double s = a > 0.0 ? sin(a) / a : 1.0;
            out[3 * i + 0] = s * v0;
            out[3 * i + 1] = s * v1;
            out[3 * i + 2] = cos(a);
        } else {
            return OR_EINVAL;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Metropolis Monte Carlo with an adaptive cone and simulated annealing     */
/* (Sec. 2.1: trial moves in a cone around the spin, Metropolis acceptance, */
/* cone adapted to keep the acceptance rate near a target; Sec. 4.3:        */
/* annealing T_{k+1} = cool T_k down to the target temperature)             */
/* ------------------------------------------------------------------------ */

/* Sweeps of the schedule: temperatures T_k = T_start cool^k (k = 0, 1, ...)
 * while T_k > T_end, sweeps_per_T sweeps each, then sweeps_final at T_end. */
static int64_t omc_schedule(double T_start, double T_end, double cool, int64_t sweeps_per_T,
                            int64_t sweeps_final, double *T_of, int64_t cap) {
    int64_t s = 0;
    for (double T = T_start; T > T_end; T *= cool)
        for (int64_t k = 0; k < sweeps_per_T; ++k) {
            if (T_of && s < cap) T_of[s] = T;
            ++s;
        }
    for (int64_t k = 0; k < sweeps_final; ++k) {
        if (T_of && s < cap) T_of[s] = T_end;
        ++s;
    }
    return s;
}

int oracle_mc_n_sweeps(double T_start, double T_end, double cool, int64_t sweeps_per_T,
                       int64_t sweeps_final, int64_t *n_sweeps) {
    if (!(cool > 0.0 && cool < 1.0) || !(T_end > 0.0) || sweeps_per_T < 1 || sweeps_final < 0)
        return OR_EINVAL;
    *n_sweeps = omc_schedule(T_start, T_end, cool, sweeps_per_T, sweeps_final, NULL, 0);
    return OR_OK;
}

/* Greedy colouring in site order: each site takes the smallest colour that no
 * lower-indexed neighbour has.  Sites of one colour share no bond. */
static int32_t ocolour(int64_t n, const int64_t *row, const int32_t *col, int32_t *colour) {
    int32_t n_col = 0;
    for (int64_t i = 0; i < n; ++i) colour[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = 0;
        for (;;) {
            int used = 0;
            for (int64_t e = row[i]; e < row[i + 1]; ++e)
                if (col[e] < i && colour[col[e]] == c) used = 1;
            if (!used) break;
            ++c;
        }
        colour[i] = c;
        if (c + 1 > n_col) n_col = c + 1;
    }
    return n_col;
}

/* Local energy of site i in state x (Eq. (1)): x.w - A x_z^2 - Hz x_z, with
 * w = sum_j (J_ij S_j + D_ij x S_j) the field of the neighbours. */
static void ofield(int64_t i, const int64_t *row, const int32_t *col, const double *J, const double *Dv,
                   const double *S, double w[3]) {
    w[0] = w[1] = w[2] = 0.0;
    for (int64_t e = row[i]; e < row[i + 1]; ++e) {
        const double *sj = S + 3 * (int64_t)col[e];
        w[0] += J[e] * sj[0];
        w[1] += J[e] * sj[1];
        w[2] += J[e] * sj[2];
        if (Dv) {
            const double *d = Dv + 3 * e;
            w[0] += d[1] * sj[2] - d[2] * sj[1];
            w[1] += d[2] * sj[0] - d[0] * sj[2];
            w[2] += d[0] * sj[1] - d[1] * sj[0];
        }
    }
}

/*
 * Annealed Metropolis sweeps on the bonds (row, col, J, Dv) with anisotropy
 * A and field Hz.  Sweep s updates the colour classes in order; site i draws
 * one Philox4x32-10 block, key = seed, counter = (i low, s low, i high,
 * 2^31 | s high): u_k = (word_k + 1/2) 2^-32.  Trial spin: cos a = 1 - u_0
 * (1 - cos cone), azimuth 2 pi u_1 about the current spin, in the frame
 * e1 = normalised (a - (a.S) S) with a = z (or x when |S_z| >= 0.9),
 * e2 = S x e1; the trial is renormalised.  Accepted when dE <= 0 or
 * u_2 < exp(-dE / T).  After each sweep, rate = accepted / n: cone *= 0.9
 * (not below 1e-3) when rate < acc_target, cone = min(pi, 1.1 cone) when
 * rate > 2 acc_target.
 * site_order != 0 visits the sites in plain index order instead (the
 * textbook sequential sweep; the same draws per site and sweep): the colour
 * classes are a visiting order chosen so that a parallel sweep can reproduce
 * it move for move, and both orders leave the Boltzmann distribution
 * invariant.
 * init: [n][3] fp32; state_out: [n][3] fp64; accepted_out: [n_sweeps] or
 * NULL; info_out[4]: energy per site (Eq. (1)), final cone, last T, colour
 * classes visited (1 in site order).
 */
int oracle_mc_anneal(int64_t n, const int64_t *row, const int32_t *col, const double *J,
                     const double *Dv, double A, double Hz, uint64_t seed, double T_start,
                     double T_end, double cool, int64_t sweeps_per_T, int64_t sweeps_final,
                     double cone0, double acc_target, const float *init, double *state_out,
                     int64_t *accepted_out, double *info_out, int site_order) {
    const double pi = 3.14159265358979323846;
    if (n <= 0 || !(cone0 > 0.0 && cone0 <= pi)) return OR_EINVAL;
    int64_t n_sweeps = 0;
    int rc = oracle_mc_n_sweeps(T_start, T_end, cool, sweeps_per_T, sweeps_final, &n_sweeps);
    if (rc != OR_OK) return rc;
    double *T_of = (double *)malloc(sizeof(double) * (size_t)(n_sweeps > 0 ? n_sweeps : 1));
    int32_t *colour = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!T_of || !colour) {
        free(T_of); free(colour);
        return OR_ENOMEM;
    }
    omc_schedule(T_start, T_end, cool, sweeps_per_T, sweeps_final, T_of, n_sweeps);
    int32_t n_col = ocolour(n, row, col, colour);
    if (site_order) {
        for (int64_t i = 0; i < n; ++i) colour[i] = 0;
        n_col = 1;
    }
    double *S = state_out;
    for (int64_t x = 0; x < 3 * n; ++x) S[x] = (double)init[x];
    double cone = cone0;
    double T = T_start;
    for (int64_t s = 0; s < n_sweeps; ++s) {
        T = T_of[s];
        const double cosc = cos(cone);
        int64_t acc = 0;
        for (int32_t c = 0; c < n_col; ++c)
            for (int64_t i = 0; i < n; ++i) {
                if (colour[i] != c) continue;
                uint32_t ctr[4] = {(uint32_t)i, (uint32_t)s, (uint32_t)((uint64_t)i >> 32),
                                   0x80000000u | (uint32_t)((uint64_t)s >> 32)};
                ophilox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
                const double u0 = ((double)ctr[0] + 0.5) * (1.0 / 4294967296.0);
                const double u1 = ((double)ctr[1] + 0.5) * (1.0 / 4294967296.0);
                const double u2 = ((double)ctr[2] + 0.5) * (1.0 / 4294967296.0);
                double *si = S + 3 * i;
                const double cosa = 1.0 - u0 * (1.0 - cosc);
                const double sina = sqrt(fmax(0.0, 1.0 - cosa * cosa));
                const double cb = cos(2.0 * pi * u1), sb = sin(2.0 * pi * u1);
                double a[3] = {0.0, 0.0, 1.0};
                if (fabs(si[2]) >= 0.9) { a[0] = 1.0; a[2] = 0.0; }
                const double as = a[0] * si[0] + a[1] * si[1] + a[2] * si[2];
                double e1[3] = {a[0] - as * si[0], a[1] - as * si[1], a[2] - as * si[2]};
                const double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
                e1[0] /= l1; e1[1] /= l1; e1[2] /= l1;
                const double e2[3] = {si[1] * e1[2] - si[2] * e1[1], si[2] * e1[0] - si[0] * e1[2],
                                      si[0] * e1[1] - si[1] * e1[0]};
                double t[3];
                for (int k = 0; k < 3; ++k) t[k] = cosa * si[k] + sina * (cb * e1[k] + sb * e2[k]);
                const double lt = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
                t[0] /= lt; t[1] /= lt; t[2] /= lt;
                double w[3];
                ofield(i, row, col, J, Dv, S, w);
                const double dE = ((t[0] - si[0]) * w[0] + (t[1] - si[1]) * w[1] + (t[2] - si[2]) * w[2])
                                  - A * (t[2] * t[2] - si[2] * si[2]) - Hz * (t[2] - si[2]);
                if (dE <= 0.0 || u2 < exp(-dE / T)) {
                    si[0] = t[0]; si[1] = t[1]; si[2] = t[2];
                    ++acc;
                }
            }
        if (accepted_out) accepted_out[s] = acc;
        const double rate = (double)acc / (double)n;
        if (rate < acc_target) cone = fmax(1e-3, 0.9 * cone);
        else if (rate > 2.0 * acc_target) cone = fmin(pi, 1.1 * cone);
    }
    /* energy per site: half of each site's bond energies (every bond seen
     * from both ends) plus its single-site terms */
    double E = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *si = S + 3 * i;
        double eb = 0.0;
        for (int64_t e = row[i]; e < row[i + 1]; ++e) {
            const double *sj = S + 3 * (int64_t)col[e];
            eb += J[e] * (si[0] * sj[0] + si[1] * sj[1] + si[2] * sj[2]);
            if (Dv) {
                const double *d = Dv + 3 * e;
                const double cx = si[1] * sj[2] - si[2] * sj[1];
                const double cy = si[2] * sj[0] - si[0] * sj[2];
                const double cz = si[0] * sj[1] - si[1] * sj[0];
                eb -= d[0] * cx + d[1] * cy + d[2] * cz;
            }
        }
        E += 0.5 * eb - A * si[2] * si[2] - Hz * si[2];
    }
    if (info_out) {
        info_out[0] = E / (double)n;
        info_out[1] = cone;
        info_out[2] = T;
        info_out[3] = (double)n_col;
    }
    free(T_of);
    free(colour);
    return OR_OK;
}
