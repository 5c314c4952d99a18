/*
 * CPU FP64 self-join matrix profile by diagonals: a second, independently
 * formulated reference for full-size profiles, where the brute force
 * (mp_bruteforce.c, m multiply-adds per pair) is too slow.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests; the product library never
 * links it and it shares no code with the HIP path.
 *
 * Definitions followed (paper Section II-B, Def. 2, Def. 3, Def. 6 with
 * T_test = T_train): for every subsequence i the distance to its nearest
 * subsequence j with |i - j| >= excl, the distance being the Euclidean
 * distance of the z-normalised subsequences.  The same readings as the brute
 * force: population sigma; a subsequence is flat when sigma <= 1e-10 max|r|
 * (sigma by two passes over the window, as there), dist(flat, flat) = 0 and
 * dist(flat, non-flat) = sqrt(m); ties go to the smallest j; no admissible j
 * gives P = +inf, I = -1.
 *
 * Formulation (not the one the GPU kernels use): on each diagonal k = j - i
 * the raw dot product QT(i, i+k) = sum_t r[i+t] r[i+k+t] is carried from row
 * to row, QT(i+1, j+1) = QT(i, j) - r[i] r[j] + r[i+m] r[j+m], in
 * double-double arithmetic (error-free products by fma, error-free sums), and
 * recomputed from its definition every 64 rows.  With S_i = sum_t r[i+t] (also
 * double-double), the centred covariance is C = QT - S_i (S_j / m), and
 * d^2 = 2 m - 2 C w with w = 1 / sigma_i * 1 / sigma_j, evaluated in
 * double-double (2 m - 2 hi(C w) is exact where d^2 is small, by Sterbenz's
 * lemma) and rounded once.  Near d = 0 any such evaluation carries the
 * rounding of sigma (about 2 m 1e-16 in d^2); the tests compare squared
 * distances there.
 *
 * Parallelism: OpenMP over groups of NL consecutive diagonals (their cells
 * are computed lane by lane, which the compiler vectorises); each thread
 * keeps its own best partner per row and the partials are reduced in index
 * order at the end.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FLAT_REL 1e-10
#define REFRESH 64
#define NL 8 /* diagonals per vector step */

typedef struct {
    double hi, lo;
} dd;

static inline dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    dd r = {s, (a - (s - bb)) + (b - bb)};
    return r;
}

static inline dd quick_two_sum(double a, double b) {
    double s = a + b;
    dd r = {s, b - (s - a)};
    return r;
}

static inline dd two_prod(double a, double b) {
    double p = a * b;
    dd r = {p, fma(a, b, -p)};
    return r;
}

static inline dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}

static inline dd dd_neg(dd a) {
    dd r = {-a.hi, -a.lo};
    return r;
}

static inline dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}

static inline dd dd_mul_d(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}

static inline dd dd_div_d(dd a, double b) {
    double q1 = a.hi / b;
    dd p = two_prod(q1, b);
    dd r = dd_add(a, dd_neg(p));
    double q2 = r.hi / b;
    return quick_two_sum(q1, q2);
}

static inline int better(double d, int64_t j, double best, int64_t arg) {
    return d < best || (d == best && arg >= 0 && j < arg) || (d == best && arg < 0);
}

int oracle_mp_diag(const double* r, int64_t n, int m, int excl, double* P, int64_t* I) {
    if (m < 2 || n < m || excl < 1) return -1;
    const int64_t n_sub = n - m + 1;
    double scale = 0.0;
    for (int64_t t = 0; t < n; ++t)
        if (fabs(r[t]) > scale) scale = fabs(r[t]);
    /* padded by NL entries (samples, window statistics): the vector lanes past
     * the matrix read finite padding and their results are discarded */
    double* rp = (double*)calloc((size_t)(n + NL), sizeof(double));
    double* sd = (double*)malloc(sizeof(double) * (size_t)n_sub);
    double* isd = (double*)calloc((size_t)(n_sub + NL), sizeof(double));
    dd* S = (dd*)malloc(sizeof(dd) * (size_t)n_sub);
    double* Smh = (double*)calloc((size_t)(n_sub + NL), sizeof(double));  /* S / m, hi and lo parts */
    double* Sml = (double*)calloc((size_t)(n_sub + NL), sizeof(double));
    unsigned char* flat = (unsigned char*)malloc((size_t)n_sub);
#ifdef _OPENMP
    const int nt = omp_get_max_threads();
#else
    const int nt = 1;
#endif
    double* Pt = (double*)malloc(sizeof(double) * (size_t)n_sub * (size_t)nt);
    int64_t* It = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_sub * (size_t)nt);
    if (!rp || !sd || !isd || !S || !Smh || !Sml || !flat || !Pt || !It) {
        free(rp);
        free(sd);
        free(isd);
        free(S);
        free(Smh);
        free(Sml);
        free(flat);
        free(Pt);
        free(It);
        return -2;
    }
    memcpy(rp, r, sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_sub; ++i) {
        dd s = {0.0, 0.0};
        for (int t = 0; t < m; ++t) s = dd_add(s, (dd){r[i + t], 0.0});
        S[i] = s;
        const dd sm = dd_div_d(s, (double)m);
        Smh[i] = sm.hi;
        Sml[i] = sm.lo;
        double sum = 0.0;
        for (int t = 0; t < m; ++t) sum += r[i + t];
        const double mu = sum / m;
        double v = 0.0;
        for (int t = 0; t < m; ++t) {
            const double e = r[i + t] - mu;
            v += e * e;
        }
        sd[i] = sqrt(v / m);
        flat[i] = sd[i] <= FLAT_REL * scale;
        isd[i] = flat[i] ? 0.0 : 1.0 / sd[i];
    }
    for (int64_t q = 0; q < n_sub * (int64_t)nt; ++q) {
        Pt[q] = INFINITY;
        It[q] = -1;
    }
    const double sqrt_m = sqrt((double)m);
#pragma omp parallel
    {
#ifdef _OPENMP
        const int tid = omp_get_thread_num();
#else
        const int tid = 0;
#endif
        double* Pm = Pt + (int64_t)tid * n_sub;
        int64_t* Im = It + (int64_t)tid * n_sub;
        /* NL consecutive diagonals k0 .. k0 + NL - 1 at a time: at row i their
         * cells share the row's samples and statistics, and their columns
         * i + k0 + l are contiguous, so the lanes vectorise */
#pragma omp for schedule(dynamic, 2)
        for (int64_t k0 = excl; k0 < n_sub; k0 += NL) {
            const int nl = (int)(n_sub - k0 < NL ? n_sub - k0 : NL);
            const int64_t len = n_sub - k0;  /* rows of diagonal k0; lane l has len - l */
            double qh[NL], ql[NL];
            for (int64_t i = 0; i < len; ++i) {
                const int64_t j0 = i + k0;
                if (i % REFRESH == 0) {
                    for (int l = 0; l < NL; ++l) {
                        dd q = {0.0, 0.0};
                        if (l < nl && i + l < len)
                            for (int t = 0; t < m; ++t) q = dd_add(q, two_prod(rp[i + t], rp[j0 + l + t]));
                        qh[l] = q.hi;
                        ql[l] = q.lo;
                    }
                } else {
                    const double a0 = rp[i - 1], a1 = rp[i + m - 1];
                    const double* c0 = rp + j0 - 1;
                    const double* c1 = rp + j0 + m - 1;
                    for (int l = 0; l < NL; ++l) {
                        dd q = {qh[l], ql[l]};
                        q = dd_add(q, dd_neg(two_prod(a0, c0[l])));
                        q = dd_add(q, two_prod(a1, c1[l]));
                        qh[l] = q.hi;
                        ql[l] = q.lo;
                    }
                }
                double dl[NL];
                const double sih = S[i].hi, sil = S[i].lo;
                const double wi = isd[i];
                const double* smh = Smh + j0;
                const double* sml = Sml + j0;
                const double* isj = isd + j0;
                for (int l = 0; l < NL; ++l) {
                    const dd c = dd_add((dd){qh[l], ql[l]}, dd_neg(dd_mul((dd){sih, sil}, (dd){smh[l], sml[l]})));
                    const dd x = dd_mul_d(c, wi * isj[l]);
                    const double v = (2.0 * m - 2.0 * x.hi) - 2.0 * x.lo;
                    dl[l] = sqrt(fmax(v, 0.0));
                }
                for (int l = 0; l < nl; ++l) {
                    const int64_t j = j0 + l;
                    if (j >= n_sub) break;
                    double d = dl[l];
                    if (flat[i] && flat[j]) d = 0.0;
                    else if (flat[i] || flat[j]) d = sqrt_m;
                    if (better(d, j, Pm[i], Im[i])) {
                        Pm[i] = d;
                        Im[i] = j;
                    }
                    if (better(d, i, Pm[j], Im[j])) {
                        Pm[j] = d;
                        Im[j] = i;
                    }
                }
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_sub; ++i) {
        double best = INFINITY;
        int64_t arg = -1;
        for (int t = 0; t < nt; ++t) {
            const double d = Pt[(int64_t)t * n_sub + i];
            const int64_t a = It[(int64_t)t * n_sub + i];
            if (a >= 0 && better(d, a, best, arg)) {
                best = d;
                arg = a;
            }
        }
        P[i] = best;
        I[i] = arg;
    }
    free(rp);
    free(sd);
    free(isd);
    free(S);
    free(Smh);
    free(Sml);
    free(flat);
    free(Pt);
    free(It);
    return 0;
}
