/*
 * Oracle (test infrastructure only): plain FP64 sums for the backprojection
 * algorithm.  Nothing in the product path links or loads this file; only the
 * tests, the smoke check and the benchmark's CPU-baseline leg do.
 *
 * or_bp_eq4          frequency-domain BPA, Sec. II-A eq. (4):
 *                        f(p) = sum_i sum_f s(p'_i, k_f) exp(+j 2 k_f |p - p'_i|)
 *                    with unit weights for the integral measures dp' dk.
 * or_bp_eq4_adjoint  its transpose (the Born forward model of eq. (1)):
 *                        g(p'_i, k_f) = sum_q w(q) exp(-j 2 k_f |q - p'_i|)
 * or_bp_eq4_dpos     d f(q) / d p'_i contracted with a cotangent image:
 *                        G_i = sum_q sum_f Re{ conj(w(q)) s_if j2k_f e^{j2k_f R} } dR/dp'_i
 *                    with dR/dp'_i = -(q - p'_i)/R; the real-valued gradient of
 *                    L = sum_q Re{conj(w) f} with respect to the antenna positions.
 *
 * or_bp_rclin        eq. (4) through range compression (eq. 2) sampled on the
 *                    range grid R_b = b dR and read back by linear interpolation:
 *                        h_i(b) = sum_f s_if c_f exp(+j w_f b dR),  w_f = 2 (k_f - k_c)
 *                        f(q)   = sum_i exp(+j 2 k_c R) [(1 - x) h_i(b) + x h_i(b + 1)]
 *                    with R = |q - p'_i|, b = floor(R / dR), x = R / dR - b and c_f
 *                    the caller's per-frequency pre-correction.
 *
 * Complex arrays are interleaved (re, im) float64.  Points and positions are
 * (n, 3) float64 row-major.  Every loop is written out; no blocking, no
 * recurrences, one libm sin/cos per term.
 */
#include <math.h>
#include <stddef.h>

static double dist3(const double *a, const double *b)
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

void or_bp_eq4(long n_pos, const double *pos, long n_f, const double *k,
               const double *s, long n_pts, const double *pts, double *out,
               int nthreads)
{
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
    for (long q = 0; q < n_pts; ++q) {
        double acc_re = 0.0, acc_im = 0.0;
        for (long i = 0; i < n_pos; ++i) {
            double R = dist3(pts + 3 * q, pos + 3 * i);
            const double *si = s + 2 * n_f * i;
            for (long f = 0; f < n_f; ++f) {
                double ph = 2.0 * k[f] * R;
                double c = cos(ph), sn = sin(ph);
                acc_re += si[2 * f] * c - si[2 * f + 1] * sn;
                acc_im += si[2 * f] * sn + si[2 * f + 1] * c;
            }
        }
        out[2 * q] = acc_re;
        out[2 * q + 1] = acc_im;
    }
}

void or_bp_eq4_adjoint(long n_pos, const double *pos, long n_f, const double *k,
                       long n_pts, const double *pts, const double *w, double *g,
                       int nthreads)
{
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
    for (long i = 0; i < n_pos; ++i) {
        double *gi = g + 2 * n_f * i;
        for (long f = 0; f < n_f; ++f) {
            gi[2 * f] = 0.0;
            gi[2 * f + 1] = 0.0;
        }
        for (long q = 0; q < n_pts; ++q) {
            double R = dist3(pts + 3 * q, pos + 3 * i);
            double wr = w[2 * q], wi = w[2 * q + 1];
            for (long f = 0; f < n_f; ++f) {
                double ph = -2.0 * k[f] * R;
                double c = cos(ph), sn = sin(ph);
                gi[2 * f] += wr * c - wi * sn;
                gi[2 * f + 1] += wr * sn + wi * c;
            }
        }
    }
}

void or_bp_eq4_dpos(long n_pos, const double *pos, long n_f, const double *k,
                    const double *s, long n_pts, const double *pts, const double *w,
                    double *grad, int nthreads)
{
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
    for (long i = 0; i < n_pos; ++i) {
        const double *pi = pos + 3 * i;
        const double *si = s + 2 * n_f * i;
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (long q = 0; q < n_pts; ++q) {
            const double *pq = pts + 3 * q;
            double R = dist3(pq, pi);
            /* d f(q)/dR = sum_f s_f (j 2 k_f) e^{j 2 k_f R} */
            double d_re = 0.0, d_im = 0.0;
            for (long f = 0; f < n_f; ++f) {
                double ph = 2.0 * k[f] * R;
                double c = cos(ph), sn = sin(ph);
                double e_re = si[2 * f] * c - si[2 * f + 1] * sn;
                double e_im = si[2 * f] * sn + si[2 * f + 1] * c;
                d_re += -2.0 * k[f] * e_im;
                d_im += 2.0 * k[f] * e_re;
            }
            /* Re{ conj(w) * df/dR } */
            double dl = w[2 * q] * d_re + w[2 * q + 1] * d_im;
            /* dR/dp'_i = -(q - p'_i)/R */
            gx += dl * (-(pq[0] - pi[0]) / R);
            gy += dl * (-(pq[1] - pi[1]) / R);
            gz += dl * (-(pq[2] - pi[2]) / R);
        }
        grad[3 * i] = gx;
        grad[3 * i + 1] = gy;
        grad[3 * i + 2] = gz;
    }
}

static void profile_at(long n_f, const double *si, const double *w, const double *c,
                       double r, double *hre, double *him)
{
    double are = 0.0, aim = 0.0;
    for (long f = 0; f < n_f; ++f) {
        double ph = w[f] * r;
        double cs = cos(ph), sn = sin(ph);
        are += c[f] * (si[2 * f] * cs - si[2 * f + 1] * sn);
        aim += c[f] * (si[2 * f] * sn + si[2 * f + 1] * cs);
    }
    *hre = are;
    *him = aim;
}

void or_bp_rclin(long n_pos, const double *pos, long n_f, const double *w, const double *c,
                 double kc, double dR, const double *s, long n_pts, const double *pts,
                 double *out, int nthreads)
{
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
    for (long q = 0; q < n_pts; ++q) {
        double acc_re = 0.0, acc_im = 0.0;
        for (long i = 0; i < n_pos; ++i) {
            double R = dist3(pts + 3 * q, pos + 3 * i);
            double t = R / dR;
            double b = floor(t);
            double x = t - b;
            double h0r, h0i, h1r, h1i;
            profile_at(n_f, s + 2 * n_f * i, w, c, b * dR, &h0r, &h0i);
            profile_at(n_f, s + 2 * n_f * i, w, c, (b + 1.0) * dR, &h1r, &h1i);
            double hr = (1.0 - x) * h0r + x * h1r, hi = (1.0 - x) * h0i + x * h1i;
            double ph = 2.0 * kc * R;
            double cs = cos(ph), sn = sin(ph);
            acc_re += hr * cs - hi * sn;
            acc_im += hr * sn + hi * cs;
        }
        out[2 * q] = acc_re;
        out[2 * q + 1] = acc_im;
    }
}
