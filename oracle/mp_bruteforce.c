/*
 * CPU FP64 brute-force self-join matrix profile.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, by smoke() and by the
 * cpu_baseline leg of bench.py.  The product library never links it and it
 * shares no code with the HIP path.
 *
 * Definitions followed (paper Section II-B): a subsequence is a length-m
 * contiguous slice (Def. 2); the distance between two subsequences is the
 * Euclidean distance of their z-normalised versions (Def. 3); the self-join
 * matrix profile stores, for every subsequence, the distance to its nearest
 * neighbour in the same series (Def. 6 with T_test = T_train, the self-join
 * variant of Section III-B).  Readings the paper leaves open, identical to
 * the numpy oracle in sketchmp_oracle.py:
 *   - population sigma; a subsequence is flat when sigma <= 1e-10 * max|r|,
 *     and a flat subsequence normalises to the zero vector, so
 *     dist(flat, flat) = 0 and dist(flat, non-flat) = sqrt(m);
 *   - (i, j) is a trivial match iff |i - j| < excl;
 *   - nearest-neighbour ties go to the smallest j; no admissible j gives
 *     P = +inf, I = -1.
 * The AB-join (oracle_ab_rows) is Def. 6 with two different series, as in
 * the train/test procedure of Section III-B (Alg. 2's AB-join): for every
 * subsequence of a, the nearest subsequence of b.  There is no trivial-match
 * zone between different series; flatness is judged in each series against
 * its own max|r|.
 * Distances are evaluated from explicit differences of the normalised
 * vectors, never through a correlation, so there is no cancellation.
 * Parallelism: OpenMP over rows (each row is independent).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FLAT_REL 1e-10

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Normalised windows Z (n_sub x m, row-major) and flat flags. */
static int normalise_windows(const double* r, int64_t n, int m, double* Z, unsigned char* flat) {
    int64_t n_sub = n - m + 1;
    double scale = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        double a = fabs(r[t]);
        if (a > scale) scale = a;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_sub; ++i) {
        double s = 0.0;
        for (int t = 0; t < m; ++t) s += r[i + t];
        double mu = s / m;
        double v = 0.0;
        for (int t = 0; t < m; ++t) {
            double e = r[i + t] - mu;
            v += e * e;
        }
        double sd = sqrt(v / m);
        double* z = Z + i * (int64_t)m;
        if (sd <= FLAT_REL * scale) {
            flat[i] = 1;
            for (int t = 0; t < m; ++t) z[t] = 0.0;
        } else {
            flat[i] = 0;
            for (int t = 0; t < m; ++t) z[t] = (r[i + t] - mu) / sd;
        }
    }
    return 0;
}

static void one_row(const double* Z, const unsigned char* flat, int64_t n_sub, int m, int excl, int64_t i,
                    double* P, int64_t* I) {
    double best = INFINITY;
    int64_t arg = -1;
    const double* zi = Z + i * (int64_t)m;
    double sqrt_m = sqrt((double)m);
    for (int64_t j = 0; j < n_sub; ++j) {
        int64_t gap = j > i ? j - i : i - j;
        if (gap < excl) continue;
        double d;
        if (flat[i] && flat[j]) {
            d = 0.0;
        } else if (flat[i] || flat[j]) {
            d = sqrt_m;
        } else {
            const double* zj = Z + j * (int64_t)m;
            double acc = 0.0;
            for (int t = 0; t < m; ++t) {
                double e = zi[t] - zj[t];
                acc += e * e;
            }
            d = sqrt(acc);
        }
        if (d < best) {  /* strict: the smallest j keeps a tie */
            best = d;
            arg = j;
        }
    }
    *P = best;
    *I = arg;
}

/* Profile for the listed rows only (all rows when rows == NULL). Returns 0, or -1 on bad arguments. */
int oracle_mp_rows(const double* r, int64_t n, int m, int excl, const int64_t* rows, int64_t nrows,
                   double* P, int64_t* I) {
    if (m < 2 || n < m || excl < 0) return -1;
    int64_t n_sub = n - m + 1;
    double* Z = (double*)malloc(sizeof(double) * (size_t)n_sub * (size_t)m);
    unsigned char* flat = (unsigned char*)malloc((size_t)n_sub);
    if (!Z || !flat) {
        free(Z);
        free(flat);
        return -2;
    }
    normalise_windows(r, n, m, Z, flat);
    int64_t count = rows ? nrows : n_sub;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < count; ++q) {
        int64_t i = rows ? rows[q] : q;
        if (i < 0 || i >= n_sub) {
            P[q] = NAN;
            I[q] = -2;
            continue;
        }
        one_row(Z, flat, n_sub, m, excl, i, &P[q], &I[q]);
    }
    free(Z);
    free(flat);
    return 0;
}

int oracle_mp_selfjoin(const double* r, int64_t n, int m, int excl, double* P, int64_t* I) {
    return oracle_mp_rows(r, n, m, excl, NULL, 0, P, I);
}

/* Exact distance of explicit pairs (i[q], j[q]) -- used to check reported neighbours. */
int oracle_pair_dist(const double* r, int64_t n, int m, const int64_t* pi, const int64_t* pj, int64_t npairs,
                     double* out) {
    if (m < 2 || n < m) return -1;
    int64_t n_sub = n - m + 1;
    double scale = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        double a = fabs(r[t]);
        if (a > scale) scale = a;
    }
    double sqrt_m = sqrt((double)m);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < npairs; ++q) {
        int64_t a = pi[q], b = pj[q];
        if (a < 0 || b < 0 || a >= n_sub || b >= n_sub) {
            out[q] = NAN;
            continue;
        }
        double mu[2], sd[2];
        int64_t w[2] = {a, b};
        for (int s = 0; s < 2; ++s) {
            double acc = 0.0;
            for (int t = 0; t < m; ++t) acc += r[w[s] + t];
            mu[s] = acc / m;
            double v = 0.0;
            for (int t = 0; t < m; ++t) {
                double e = r[w[s] + t] - mu[s];
                v += e * e;
            }
            sd[s] = sqrt(v / m);
        }
        int fa = sd[0] <= FLAT_REL * scale, fb = sd[1] <= FLAT_REL * scale;
        if (fa && fb) {
            out[q] = 0.0;
        } else if (fa || fb) {
            out[q] = sqrt_m;
        } else {
            double acc = 0.0;
            for (int t = 0; t < m; ++t) {
                double e = (r[a + t] - mu[0]) / sd[0] - (r[b + t] - mu[1]) / sd[1];
                acc += e * e;
            }
            out[q] = sqrt(acc);
        }
    }
    return 0;
}

/* AB-join rows: for each listed subsequence i of a (all when rows == NULL),
 * the nearest subsequence of b.  Returns 0, or -1 / -2 on bad arguments / no memory. */
int oracle_ab_rows(const double* a, int64_t na, const double* b, int64_t nb, int m, const int64_t* rows,
                   int64_t nrows, double* P, int64_t* I) {
    if (m < 2 || na < m || nb < m) return -1;
    int64_t na_sub = na - m + 1, nb_sub = nb - m + 1;
    double* Za = (double*)malloc(sizeof(double) * (size_t)na_sub * (size_t)m);
    double* Zb = (double*)malloc(sizeof(double) * (size_t)nb_sub * (size_t)m);
    unsigned char* fa = (unsigned char*)malloc((size_t)na_sub);
    unsigned char* fb = (unsigned char*)malloc((size_t)nb_sub);
    if (!Za || !Zb || !fa || !fb) {
        free(Za);
        free(Zb);
        free(fa);
        free(fb);
        return -2;
    }
    normalise_windows(a, na, m, Za, fa);
    normalise_windows(b, nb, m, Zb, fb);
    double sqrt_m = sqrt((double)m);
    int64_t count = rows ? nrows : na_sub;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < count; ++q) {
        int64_t i = rows ? rows[q] : q;
        if (i < 0 || i >= na_sub) {
            P[q] = NAN;
            I[q] = -2;
            continue;
        }
        const double* zi = Za + i * (int64_t)m;
        double best = INFINITY;
        int64_t arg = -1;
        for (int64_t j = 0; j < nb_sub; ++j) {
            double d;
            if (fa[i] && fb[j]) {
                d = 0.0;
            } else if (fa[i] || fb[j]) {
                d = sqrt_m;
            } else {
                const double* zj = Zb + j * (int64_t)m;
                double acc = 0.0;
                for (int t = 0; t < m; ++t) {
                    double e = zi[t] - zj[t];
                    acc += e * e;
                }
                d = sqrt(acc);
            }
            if (d < best) {  /* strict: the smallest j keeps a tie */
                best = d;
                arg = j;
            }
        }
        P[q] = best;
        I[q] = arg;
    }
    free(Za);
    free(Zb);
    free(fa);
    free(fb);
    return 0;
}

static void window_moments(const double* r, int64_t w, int m, double* mu, double* sd) {
    double acc = 0.0;
    for (int t = 0; t < m; ++t) acc += r[w + t];
    *mu = acc / m;
    double v = 0.0;
    for (int t = 0; t < m; ++t) {
        double e = r[w + t] - *mu;
        v += e * e;
    }
    *sd = sqrt(v / m);
}

static double max_abs(const double* r, int64_t n) {
    double s = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        double x = fabs(r[t]);
        if (x > s) s = x;
    }
    return s;
}

/* Exact distance of explicit pairs (subsequence pi[q] of a, subsequence pj[q] of b). */
int oracle_ab_pair_dist(const double* a, int64_t na, const double* b, int64_t nb, int m, const int64_t* pi,
                        const int64_t* pj, int64_t npairs, double* out) {
    if (m < 2 || na < m || nb < m) return -1;
    int64_t na_sub = na - m + 1, nb_sub = nb - m + 1;
    double sa = max_abs(a, na), sb = max_abs(b, nb);
    double sqrt_m = sqrt((double)m);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < npairs; ++q) {
        int64_t i = pi[q], j = pj[q];
        if (i < 0 || j < 0 || i >= na_sub || j >= nb_sub) {
            out[q] = NAN;
            continue;
        }
        double mu_a, sd_a, mu_b, sd_b;
        window_moments(a, i, m, &mu_a, &sd_a);
        window_moments(b, j, m, &mu_b, &sd_b);
        int f1 = sd_a <= FLAT_REL * sa, f2 = sd_b <= FLAT_REL * sb;
        if (f1 && f2) {
            out[q] = 0.0;
        } else if (f1 || f2) {
            out[q] = sqrt_m;
        } else {
            double acc = 0.0;
            for (int t = 0; t < m; ++t) {
                double e = (a[i + t] - mu_a) / sd_a - (b[j + t] - mu_b) / sd_b;
                acc += e * e;
            }
            out[q] = sqrt(acc);
        }
    }
    return 0;
}
