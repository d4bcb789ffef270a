/*
 * Dense-grid Fourier sum for one separable term of a multi-asset price.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle. Shares no code with the GPU
 * library. Built by oracle/build.py with gcc -O2 -fopenmp.
 *
 * For one term with mean m[d], covariance C[d*d] (row-major), per-coordinate
 * contour shifts alpha[d], half-widths L[d] and payoff factor kinds kind[d], it
 * forms the plain nested sum over the full grid (the nested form of Eq. discr
 * discussed at the end of Sec. III.D, with the multi-asset characteristic
 * function of Sec. III.C):
 *
 *   S = sum_{i in [N]^d}  exp(-i z.m - 1/2 z^T C z) * prod_k h_k(z_k),
 *   z_k = u_k(i_k) + i alpha_k,   u_k(i) = -L_k + (i + 1/2) * 2 L_k / N.
 *
 * exp(-i z.m - 1/2 z^T C z) is the characteristic function of the Gaussian
 * log-price vector evaluated at -z; h_k is the Fourier transform of the k-th
 * payoff factor (kind 0: (e^w - 1)^+ or (1 - e^w)^+, both 1/(iz(1+iz)) on their
 * own strips; kind 1: 1{w<0}, 1/(iz); kind 2: 1{w>0}, -1/(iz)).
 *
 * Kind 3 (every coordinate, asset coordinates w = x) is the call on the minimum with the
 * single-strip transform of Sec. III.C written in the form that direct integration gives:
 * the product of factors is replaced by the joint transform
 *   (-1)^(d+1) / ((1 + i sum_k z_k) prod_k (i z_k)),   Im z_k > 0, sum_k Im z_k > 1.
 *
 * Jumps (Merton's model, the extension named in Sec. VI): with lamT = lambda T > 0 the
 * characteristic function carries the compound-Poisson factor of normally distributed log-jump
 * sizes with mean mJ[d] and covariance CJ[d*d] (in the term's coordinates), evaluated at -z like
 * the Gaussian part:
 *   exp(lamT (exp(-i z.mJ - 1/2 z^T CJ z) - 1)),
 * and m carries the martingale compensator (see fourier.log_moments).
 *
 * Every point evaluates the full quadratic form from scratch: O(d^2) per point,
 * deliberately without any reuse between points. The sum over the last index is
 * accumulated into a row sum, and row sums are accumulated with Kahan
 * compensation per thread, then added.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

static double complex payoff_factor(int kind, double complex z)
{
    double complex iz = I * z;
    if (kind == 0) return 1.0 / (iz * (1.0 + iz));
    if (kind == 1) return 1.0 / iz;
    return -1.0 / iz;
}

static double complex node(int k, int i, int N, const double *L, const double *alpha)
{
    double eta = 2.0 * L[k] / (double)N;
    return (-L[k] + ((double)i + 0.5) * eta) + I * alpha[k];
}

static double complex quad_exponent(int d, const double complex *z, const double *m, const double *C)
{
    double complex e = 0.0;
    for (int k = 0; k < d; ++k) e += -I * z[k] * m[k];
    double complex q = 0.0;
    for (int k = 0; k < d; ++k)
        for (int l = 0; l < d; ++l) q += z[k] * C[k * d + l] * z[l];
    return e - 0.5 * q;
}

static double complex integrand(int d, const double complex *z, const double *m, const double *C,
                                const int *kind, double lamT, const double *mJ, const double *CJ)
{
    double complex e = quad_exponent(d, z, m, C);
    if (lamT > 0.0) e += lamT * (cexp(quad_exponent(d, z, mJ, CJ)) - 1.0);
    double complex h = 1.0;
    if (kind[0] == 3) {
        double complex sz = 0.0;
        for (int k = 0; k < d; ++k) {
            sz += z[k];
            h *= I * z[k];
        }
        h = ((d % 2) ? 1.0 : -1.0) / ((1.0 + I * sz) * h);
        return cexp(e) * h;
    }
    for (int k = 0; k < d; ++k) h *= payoff_factor(kind[k], z[k]);
    return cexp(e) * h;
}

/* Partial sum over the rows [row_begin, row_end) of the grid (a row fixes every index but
 * the last). out[0] + i out[1] = S ; out[2] = sum |F| (for the cancellation diagnostic). */
void dense_term_sum_rows(int d, int N, const double *m, const double *C, const double *L,
                         const double *alpha, const int *kind, double lamT, const double *mJ,
                         const double *CJ, int nthreads, int64_t row_begin, int64_t row_end,
                         double *out)
{
    double sre = 0.0, sim = 0.0, sabs = 0.0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        double complex z[64];
        double are = 0.0, aim = 0.0, cre = 0.0, cim = 0.0, aabs = 0.0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t row = row_begin; row < row_end; ++row) {
            int64_t t = row;
            for (int k = d - 2; k >= 0; --k) {
                z[k] = node(k, (int)(t % N), N, L, alpha);
                t /= N;
            }
            double complex rs = 0.0;
            double ra = 0.0;
            for (int i = 0; i < N; ++i) {
                z[d - 1] = node(d - 1, i, N, L, alpha);
                double complex f = integrand(d, z, m, C, kind, lamT, mJ, CJ);
                rs += f;
                ra += cabs(f);
            }
            /* Kahan accumulation of the row sums */
            double y = creal(rs) - cre;
            double tt = are + y;
            cre = (tt - are) - y;
            are = tt;
            y = cimag(rs) - cim;
            tt = aim + y;
            cim = (tt - aim) - y;
            aim = tt;
            aabs += ra;
        }
#pragma omp critical
        {
            sre += are;
            sim += aim;
            sabs += aabs;
        }
    }
    out[0] = sre;
    out[1] = sim;
    out[2] = sabs;
}

/* The full sum over all N^d points. */
void dense_term_sum(int d, int N, const double *m, const double *C, const double *L,
                    const double *alpha, const int *kind, double lamT, const double *mJ,
                    const double *CJ, int nthreads, double *out)
{
    int64_t rows = 1;
    for (int k = 0; k < d - 1; ++k) rows *= N;
    dense_term_sum_rows(d, N, m, C, L, alpha, kind, lamT, mJ, CJ, nthreads, 0, rows, out);
}

/* Integrand values at npts multi-indices idx[p*d + k] (0-based grid indices). */
void integrand_points(int d, int N, const double *m, const double *C, const double *L,
                      const double *alpha, const int *kind, double lamT, const double *mJ,
                      const double *CJ, int64_t npts, const int32_t *idx, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < npts; ++p) {
        double complex z[64];
        for (int k = 0; k < d; ++k) z[k] = node(k, idx[p * d + k], N, L, alpha);
        double complex f = integrand(d, z, m, C, kind, lamT, mJ, CJ);
        out[2 * p] = creal(f);
        out[2 * p + 1] = cimag(f);
    }
}
