/*
 * Double-precision direct-sum reference for the discrete aperiodic ambiguity
 * function and its conjugate-Wirtinger adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls
 * this file: only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header or table with the HIP path.
 *
 * What it computes (paper Sec. 4.1, Eqs. 7-11, with the lag product taken
 * aperiodically, i.e. s[n] = 0 outside [0, N), instead of the circular index
 * of Eq. 8, and the "FFT" of Eq. 11 written out as its defining sum with the
 * library sign e^{-j}):
 *
 *   chi[tau, k] = sum_{n} s[n] * conj(s[n - tau]) * exp(-j 2 pi k n / M)
 *
 * for every lag tau in [-T, T] and every Doppler bin k in [0, M).  The sum
 * runs over the n for which both s[n] and s[n - tau] lie inside [0, N).
 *
 * The adjoint follows the chain rule of Sec. 4.2 (Eq. 15): given the upstream
 * G[tau, k] = dL/d conj(chi[tau, k]) it returns
 *
 *   g[p] = sum_tau ( Q_tau[p] * s[p - tau] + conj(Q_tau[p + tau]) * s[p + tau] )
 *   Q_tau[n] = sum_k G[tau, k] * exp(+j 2 pi k n / M)
 *
 * i.e. dL/d conj(s[p]) through chi, without the energy term (the Python side
 * adds dL/dE * s).  Out-of-range samples contribute nothing.
 *
 * Arrays are interleaved (re, im) doubles.  chi and G are row-major
 * [2T+1][M] with row i <-> tau = i - T.  Twiddles come from libm cos/sin of
 * the integer-reduced angle (k*n mod M), so each carries one rounding.
 * Returns 0 on success, -1 on a bad argument.
 *
 * The periodic (circular) AF of the paper's own Eqs. 2 and 7 and Algorithm 1
 * takes the lag index modulo N and N Doppler bins:
 *
 *   chi_c[tau, k] = sum_{n=0}^{N-1} s[n] * conj(s[(n - tau) mod N]) * exp(-j 2 pi k n / N)
 *
 * for tau, k in [0, N), row-major [N][N] with row tau; its adjoint is the
 * formula above with every sample index taken modulo N and Q_tau over N
 * bins (oracle_chi_circ, oracle_adjoint_circ).
 */
#define _USE_MATH_DEFINES
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* threads the OpenMP loops below use (1 without OpenMP) */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int bad_args(int n, int m, int max_lag)
{
    if (n < 1 || m < 1 || max_lag < 0 || max_lag > n - 1) return 1;
    if ((m & (m - 1)) != 0) return 1; /* M is a power of two */
    return 0;
}

/* w[i] = exp(-j 2 pi i / M), i in [0, M) */
static double *twiddle_table(int m)
{
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)m);
    if (!w) return NULL;
    for (int i = 0; i < m; ++i) {
        double a = -2.0 * M_PI * (double)i / (double)m;
        w[2 * i] = cos(a);
        w[2 * i + 1] = sin(a);
    }
    return w;
}

int oracle_chi(int n, int m, int max_lag, const double *s, double *chi)
{
    if (bad_args(n, m, max_lag) || !s || !chi) return -1;
    double *w = twiddle_table(m);
    if (!w) return -1;
    const int T = max_lag;
    const int rows = 2 * T + 1;
    const int64_t mask = m - 1;

#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < rows; ++i) {
        const int tau = i - T;
        const int lo = tau > 0 ? tau : 0;
        const int hi = tau < 0 ? n + tau : n;
        /* lag product r[t] = s[t] * conj(s[t - tau]) on its support */
        double *r = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        for (int t = lo; t < hi; ++t) {
            double ar = s[2 * t], ai = s[2 * t + 1];
            double br = s[2 * (t - tau)], bi = -s[2 * (t - tau) + 1];
            r[2 * t] = ar * br - ai * bi;
            r[2 * t + 1] = ar * bi + ai * br;
        }
        double *row = chi + (size_t)i * (size_t)m * 2;
        for (int k = 0; k < m; ++k) {
            double re = 0.0, im = 0.0;
            for (int t = lo; t < hi; ++t) {
                /* (k * t) mod M, exact in 64-bit integers */
                int64_t idx = ((int64_t)k * (int64_t)t) & mask;
                double wr = w[2 * idx], wi = w[2 * idx + 1];
                re += r[2 * t] * wr - r[2 * t + 1] * wi;
                im += r[2 * t] * wi + r[2 * t + 1] * wr;
            }
            row[2 * k] = re;
            row[2 * k + 1] = im;
        }
        free(r);
    }
    free(w);
    return 0;
}

/* chi rows for the lags taus[0..count) only (same sums as oracle_chi),
 * parallel over Doppler bins; out is [count][M] interleaved. */
int oracle_chi_rows(int n, int m, int count, const int *taus, const double *s, double *out)
{
    if (n < 1 || m < 1 || (m & (m - 1)) != 0 || count < 0 || !taus || !s || !out) return -1;
    for (int i = 0; i < count; ++i)
        if (taus[i] <= -n || taus[i] >= n) return -1;
    double *w = twiddle_table(m);
    if (!w) return -1;
    const int64_t mask = m - 1;
    double *r = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    if (!r) { free(w); return -1; }
    for (int i = 0; i < count; ++i) {
        const int tau = taus[i];
        const int lo = tau > 0 ? tau : 0;
        const int hi = tau < 0 ? n + tau : n;
        for (int t = lo; t < hi; ++t) {
            double ar = s[2 * t], ai = s[2 * t + 1];
            double br = s[2 * (t - tau)], bi = -s[2 * (t - tau) + 1];
            r[2 * t] = ar * br - ai * bi;
            r[2 * t + 1] = ar * bi + ai * br;
        }
        double *row = out + (size_t)i * (size_t)m * 2;
#pragma omp parallel for schedule(static)
        for (int k = 0; k < m; ++k) {
            double re = 0.0, im = 0.0;
            for (int t = lo; t < hi; ++t) {
                int64_t idx = ((int64_t)k * (int64_t)t) & mask;
                double wr = w[2 * idx], wi = w[2 * idx + 1];
                re += r[2 * t] * wr - r[2 * t + 1] * wi;
                im += r[2 * t] * wi + r[2 * t + 1] * wr;
            }
            row[2 * k] = re;
            row[2 * k + 1] = im;
        }
    }
    free(r);
    free(w);
    return 0;
}

int oracle_adjoint(int n, int m, int max_lag, const double *s, const double *G, double *g)
{
    if (bad_args(n, m, max_lag) || !s || !G || !g) return -1;
    double *w = twiddle_table(m);
    if (!w) return -1;
    const int T = max_lag;
    const int rows = 2 * T + 1;
    const int64_t mask = m - 1;
    /* Q[i][t] = sum_k G[i][k] * conj(w[k t mod M]) for t in [0, N) */
    double *Q = (double *)malloc(sizeof(double) * 2 * (size_t)rows * (size_t)n);
    if (!Q) { free(w); return -1; }

#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < rows; ++i) {
        const double *row = G + (size_t)i * (size_t)m * 2;
        double *q = Q + (size_t)i * (size_t)n * 2;
        for (int t = 0; t < n; ++t) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < m; ++k) {
                int64_t idx = ((int64_t)k * (int64_t)t) & mask;
                double wr = w[2 * idx], wi = -w[2 * idx + 1]; /* e^{+j...} */
                re += row[2 * k] * wr - row[2 * k + 1] * wi;
                im += row[2 * k] * wi + row[2 * k + 1] * wr;
            }
            q[2 * t] = re;
            q[2 * t + 1] = im;
        }
    }

#pragma omp parallel for schedule(static)
    for (int p = 0; p < n; ++p) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < rows; ++i) {
            const int tau = i - T;
            const double *q = Q + (size_t)i * (size_t)n * 2;
            /* Q_tau[p] * s[p - tau], needs p - tau in [0, N) and p >= tau */
            int a = p - tau;
            if (a >= 0 && a < n && p >= (tau > 0 ? tau : 0) && p < (tau < 0 ? n + tau : n)) {
                double qr = q[2 * p], qi = q[2 * p + 1];
                double sr = s[2 * a], si = s[2 * a + 1];
                re += qr * sr - qi * si;
                im += qr * si + qi * sr;
            }
            /* conj(Q_tau[p + tau]) * s[p + tau], needs p + tau in the support of lag tau */
            int b = p + tau;
            if (b >= 0 && b < n && b >= (tau > 0 ? tau : 0) && b < (tau < 0 ? n + tau : n)) {
                double qr = q[2 * b], qi = -q[2 * b + 1];
                double sr = s[2 * b], si = s[2 * b + 1];
                re += qr * sr - qi * si;
                im += qr * si + qi * sr;
            }
        }
        g[2 * p] = re;
        g[2 * p + 1] = im;
    }
    free(Q);
    free(w);
    return 0;
}

/* w[i] = exp(-j 2 pi i / N), i in [0, N), any N >= 1 */
static double *twiddle_table_any(int n)
{
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    if (!w) return NULL;
    for (int i = 0; i < n; ++i) {
        double a = -2.0 * M_PI * (double)i / (double)n;
        w[2 * i] = cos(a);
        w[2 * i + 1] = sin(a);
    }
    return w;
}

int oracle_chi_circ(int n, const double *s, double *chi)
{
    if (n < 1 || !s || !chi) return -1;
    double *w = twiddle_table_any(n);
    if (!w) return -1;

#pragma omp parallel for schedule(dynamic, 1)
    for (int tau = 0; tau < n; ++tau) {
        /* r[t] = s[t] * conj(s[(t - tau) mod N]) for every t */
        double *r = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        for (int t = 0; t < n; ++t) {
            const int u = (t - tau + n) % n;
            double ar = s[2 * t], ai = s[2 * t + 1];
            double br = s[2 * u], bi = -s[2 * u + 1];
            r[2 * t] = ar * br - ai * bi;
            r[2 * t + 1] = ar * bi + ai * br;
        }
        double *row = chi + (size_t)tau * (size_t)n * 2;
        for (int k = 0; k < n; ++k) {
            double re = 0.0, im = 0.0;
            for (int t = 0; t < n; ++t) {
                int64_t idx = ((int64_t)k * (int64_t)t) % n;
                double wr = w[2 * idx], wi = w[2 * idx + 1];
                re += r[2 * t] * wr - r[2 * t + 1] * wi;
                im += r[2 * t] * wi + r[2 * t + 1] * wr;
            }
            row[2 * k] = re;
            row[2 * k + 1] = im;
        }
        free(r);
    }
    free(w);
    return 0;
}

int oracle_adjoint_circ(int n, const double *s, const double *G, double *g)
{
    if (n < 1 || !s || !G || !g) return -1;
    double *w = twiddle_table_any(n);
    if (!w) return -1;
    /* Q[tau][t] = sum_k G[tau][k] * exp(+j 2 pi k t / N) */
    double *Q = (double *)malloc(sizeof(double) * 2 * (size_t)n * (size_t)n);
    if (!Q) { free(w); return -1; }

#pragma omp parallel for schedule(dynamic, 1)
    for (int tau = 0; tau < n; ++tau) {
        const double *row = G + (size_t)tau * (size_t)n * 2;
        double *q = Q + (size_t)tau * (size_t)n * 2;
        for (int t = 0; t < n; ++t) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < n; ++k) {
                int64_t idx = ((int64_t)k * (int64_t)t) % n;
                double wr = w[2 * idx], wi = -w[2 * idx + 1];
                re += row[2 * k] * wr - row[2 * k + 1] * wi;
                im += row[2 * k] * wi + row[2 * k + 1] * wr;
            }
            q[2 * t] = re;
            q[2 * t + 1] = im;
        }
    }

#pragma omp parallel for schedule(static)
    for (int p = 0; p < n; ++p) {
        double re = 0.0, im = 0.0;
        for (int tau = 0; tau < n; ++tau) {
            const double *q = Q + (size_t)tau * (size_t)n * 2;
            /* s[p] appears conjugated in r_tau[t] at t = (p + tau) mod N and
             * plain at t = p: Q_tau[p] * s[(p - tau) mod N] from the plain
             * factor, conj(Q_tau[(p + tau) mod N]) * s[(p + tau) mod N] from
             * the conjugated one */
            const int a = (p - tau + n) % n;
            double qr = q[2 * p], qi = q[2 * p + 1];
            double sr = s[2 * a], si = s[2 * a + 1];
            re += qr * sr - qi * si;
            im += qr * si + qi * sr;
            const int b = (p + tau) % n;
            qr = q[2 * b];
            qi = -q[2 * b + 1];
            sr = s[2 * b];
            si = s[2 * b + 1];
            re += qr * sr - qi * si;
            im += qr * si + qi * sr;
        }
        g[2 * p] = re;
        g[2 * p + 1] = im;
    }
    free(Q);
    free(w);
    return 0;
}
