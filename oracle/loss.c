/*
 * Eyebox loss and its gradient with respect to the binned irradiance.
 * Test infrastructure (oracle); see oracle.h.
 *
 * Eq. 1: L = L_bright + w_f L_FoV + w_e L_eyebox with L_bright = -(mean
 * throughput).  Throughput of one (wavelength, FoV) point is the fraction of
 * injected power landing in the eyebox, eta = sum_b I_b.  The eyebox profile
 * E_b is the mean of I_b over wavelengths and FoV points; the FoV profile
 * phi_f is the mean of eta over wavelengths.  kind 1 uses coefficients of
 * variation (std / mean, population std) as in the paper; kind 0 uses the
 * population variances (the differentiation workload's loss).  kind 2 is
 * Eq. 1 on pupil images (Results: the images of a grid of pupil positions
 * are the objective; the mean throughput is averaged over pupil positions,
 * FoV samples and colour channels): I_b is then the power fraction through
 * pupil b, the brightness term is the mean of I over (wavelength, FoV,
 * pupil), i.e. mean eta / B, and the CV terms are those of kind 1 with the
 * pupils as the eyebox samples.  With three wavelengths per colour channel
 * the mean over channels equals the mean over wavelengths.  Summed over
 * designs.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

double orc_loss(const double* irr, int32_t D, int32_t n_l, int32_t F, int32_t B,
                int32_t kind, double w_f, double w_e, double* dL_dI)
{
    double total = 0.0;
    double* eyeb = (double*)malloc(sizeof(double) * (size_t)B);
    double* phi = (double*)malloc(sizeof(double) * (size_t)F);
    for (int d = 0; d < D; ++d) {
        const double* Id = irr + (size_t)d * n_l * F * B;
        double npts = (double)n_l * (double)F;
        /* throughput per point and its mean */
        double ibar = 0.0;
        for (int f = 0; f < F; ++f) phi[f] = 0.0;
        for (int b = 0; b < B; ++b) eyeb[b] = 0.0;
        for (int l = 0; l < n_l; ++l)
            for (int f = 0; f < F; ++f) {
                double eta = 0.0;
                for (int b = 0; b < B; ++b) {
                    double v = Id[((size_t)l * F + f) * B + b];
                    eta += v;
                    eyeb[b] += v / npts;
                }
                phi[f] += eta / (double)n_l;
                ibar += eta / npts;
            }
        double ebar = 0.0;
        for (int b = 0; b < B; ++b) ebar += eyeb[b] / (double)B;
        double var_e = 0.0, var_f = 0.0;
        for (int b = 0; b < B; ++b) var_e += (eyeb[b] - ebar) * (eyeb[b] - ebar) / (double)B;
        for (int f = 0; f < F; ++f) var_f += (phi[f] - ibar) * (phi[f] - ibar) / (double)F;
        double L, ce_b, cf_f, c_mean_e, c_mean_f;
        /* weight of the throughput's mean in the brightness term */
        double bright = kind == 2 ? 1.0 / (double)B : 1.0;
        /* dL = -dIbar + a_e dVar_e + a_f dVar_f + m_e dEbar + m_f dIbar */
        double a_e, a_f, m_e, m_f;
        if (kind == 0) {
            L = -ibar + w_e * var_e + w_f * var_f;
            a_e = w_e; a_f = w_f; m_e = 0.0; m_f = 0.0;
        } else {
            double sd_e = sqrt(var_e), sd_f = sqrt(var_f);
            double cv_e = sd_e / ebar, cv_f = sd_f / ibar;
            L = -ibar * bright + w_f * cv_f + w_e * cv_e;
            a_e = sd_e > 0.0 ? w_e / (2.0 * sd_e * ebar) : 0.0;
            a_f = sd_f > 0.0 ? w_f / (2.0 * sd_f * ibar) : 0.0;
            m_e = -w_e * sd_e / (ebar * ebar);
            m_f = -w_f * sd_f / (ibar * ibar);
        }
        total += L;
        if (dL_dI) {
            double* G = dL_dI + (size_t)d * n_l * F * B;
            for (int l = 0; l < n_l; ++l)
                for (int f = 0; f < F; ++f)
                    for (int b = 0; b < B; ++b) {
                        /* dIbar/dI = 1/npts; dEbar/dI = 1/(B npts);
                         * dVar_e/dI = 2 (E_b - Ebar)/(B npts); dVar_f/dI = 2 (phi_f - Ibar)/(F n_l) */
                        ce_b = 2.0 * (eyeb[b] - ebar) / ((double)B * npts);
                        cf_f = 2.0 * (phi[f] - ibar) / ((double)F * (double)n_l);
                        c_mean_e = 1.0 / ((double)B * npts);
                        c_mean_f = 1.0 / npts;
                        G[((size_t)l * F + f) * B + b] = -bright / npts + a_e * ce_b + a_f * cf_f
                                                         + m_e * c_mean_e + m_f * c_mean_f;
                    }
        }
    }
    free(eyeb);
    free(phi);
    return total;
}
