/*
 * ORACLE - TEST INFRASTRUCTURE ONLY.  Plain FP64 brute-force evaluation of
 * the truncated skeletal density function at arbitrary query points.  Only
 * the tests, the smoke check and the bench's CPU-baseline leg may load it;
 * the product path never does.
 *
 * Definition followed (Formulation section):
 *   eta(p, q)   = |p - q|                                     (eq. 10A)
 *   xi(p, S)    = pmc(p, S) * min_q eta(p, q)                 (eq. 10A)
 *   pmc         = sign((p - q*) . n(q*)), q* the nearest sample (lowest index
 *                 among exact ties); the outward normal supplies the
 *                 orientation that decides inside / outside
 *   cos theta   = (p - q) . n(q) / |p - q|                    (eq. 12a)
 *   zeta        = xi + i eta   (the "+" branch of eq. 11)
 *   lambda      = +lambda1 if Re zeta > 0, -lambda2 if Re zeta < 0  (eq. 16c)
 *   phi(zeta)   = lambda / sqrt(2 pi) * zeta^-2 * g_sigma(|tan arg zeta| - 1),
 *                 g_sigma(x) = exp(-x^2 / (2 sigma^2)) / (sqrt(2 pi) sigma) (eq. 15)
 *   rho(p, S)   = sum_j phi(zeta(p, q_j)) cos theta_j w_j     (eq. 13)
 *   truncation: only samples in the eps-approximate contact region
 *               |p - q_j| <= (1 + eps) |xi| take part        (eq. 10b, 17t)
 *   rho := 0 where pmc = 0 or |xi| < xi_floor: the kernel is singular on the
 *   boundary itself and the affinity is left undefined there.
 *
 * Diagnostics (optional, may be NULL) report how close each query point is
 * to a decision that a lower-precision evaluation could take differently.
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

void oracle_sdf_points(const double *q, const double *nrm, const double *w, long ns,
                       const double *pts, long npts,
                       double lambda1, double lambda2, double sigma, double eps, double xi_floor,
                       double *out_re, double *out_im,
                       double *out_xi,          /* signed xi, or NULL */
                       long *out_nearest,       /* index of q*, or NULL */
                       double *out_trunc_margin,/* min_j |eta_j - (1+eps)|xi|| / |xi|, or NULL */
                       double *out_band_mag,    /* sum of |term_j| over samples with relative margin <= band_rel */
                       double *out_pmc_gap,     /* nearest opposite-side sample distance minus |xi|, or NULL */
                       double band_rel)
{
    const double s2pi = sqrt(2.0 * M_PI);
#pragma omp parallel for schedule(dynamic, 16)
    for (long a = 0; a < npts; ++a) {
        const double px = pts[3 * a], py = pts[3 * a + 1], pz = pts[3 * a + 2];
        /* pass 1: nearest sample (squared distances share the minimiser) */
        double best2 = INFINITY;
        long jbest = -1;
        for (long j = 0; j < ns; ++j) {
            double dx = px - q[3 * j], dy = py - q[3 * j + 1], dz = pz - q[3 * j + 2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < best2) { best2 = d2; jbest = j; }
        }
        double best = sqrt(best2);
        double dot = (px - q[3 * jbest]) * nrm[3 * jbest] + (py - q[3 * jbest + 1]) * nrm[3 * jbest + 1] +
                     (pz - q[3 * jbest + 2]) * nrm[3 * jbest + 2];
        int pmc = dot > 0.0 ? 1 : (dot < 0.0 ? -1 : 0);
        double xi_abs = best;
        double xi = pmc * xi_abs;
        if (out_xi) out_xi[a] = xi;
        if (out_nearest) out_nearest[a] = jbest;
        if (out_pmc_gap) {
            double opp = INFINITY;
            for (long j = 0; j < ns; ++j) {
                double dx = px - q[3 * j], dy = py - q[3 * j + 1], dz = pz - q[3 * j + 2];
                double dj = dx * nrm[3 * j] + dy * nrm[3 * j + 1] + dz * nrm[3 * j + 2];
                int sj = dj > 0.0 ? 1 : (dj < 0.0 ? -1 : 0);
                if (sj != pmc) {
                    double d = sqrt(dx * dx + dy * dy + dz * dz);
                    if (d < opp) opp = d;
                }
            }
            out_pmc_gap[a] = opp - xi_abs;
        }
        double complex acc = 0.0;
        double margin = INFINITY, band = 0.0;
        if (pmc != 0 && xi_abs >= xi_floor) {
            double lam = pmc > 0 ? lambda1 : -lambda2;
            double radius = (1.0 + eps) * xi_abs;
            /* samples farther than the band around the contact sphere can
               neither contribute nor matter to the diagnostics */
            double reach = radius * (1.0 + band_rel) + 1e-300;
            double reach2 = reach * reach;
            for (long j = 0; j < ns; ++j) {
                double dx = px - q[3 * j], dy = py - q[3 * j + 1], dz = pz - q[3 * j + 2];
                double d2 = dx * dx + dy * dy + dz * dz;
                if (d2 > reach2 && !out_trunc_margin) continue;
                double eta = sqrt(d2);
                double m = fabs(eta - radius) / xi_abs;
                if (m < margin) margin = m;
                if (eta > radius && m > band_rel) continue;
                double complex zeta = xi + I * eta;
                double tan_abs = eta / xi_abs; /* |tan arg zeta| = |Im / Re| */
                double x = tan_abs - 1.0;
                double g = exp(-0.5 * x * x / (sigma * sigma)) / (s2pi * sigma);
                double complex phi = lam / s2pi / (zeta * zeta) * g;
                double cos_t = (dx * nrm[3 * j] + dy * nrm[3 * j + 1] + dz * nrm[3 * j + 2]) / eta;
                double complex term = phi * cos_t * w[j];
                if (m <= band_rel) band += cabs(term);
                if (eta <= radius) acc += term;
            }
        }
        out_re[a] = creal(acc);
        out_im[a] = cimag(acc);
        if (out_trunc_margin) out_trunc_margin[a] = margin;
        if (out_band_mag) out_band_mag[a] = band;
    }
}
