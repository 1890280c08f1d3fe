/*
 * gmo_internal.h -- oracle internals.  TEST INFRASTRUCTURE (see gmo.h).
 */
#ifndef GMO_INTERNAL_H
#define GMO_INTERNAL_H

#include "gmo.h"

/* CGS constants: CODATA 2018 and IAU nominal values. */
#define GMO_CL    2.99792458e10          /* speed of light, cm/s           */
#define GMO_HPL   6.62607015e-27         /* Planck constant, erg s          */
#define GMO_KB    1.380649e-16           /* Boltzmann constant, erg/K       */
#define GMO_EE    4.80320471e-10         /* electron charge, esu            */
#define GMO_ME    9.1093837015e-28       /* electron mass, g                */
#define GMO_MP    1.67262192369e-24      /* proton mass, g                  */
#define GMO_SIGT  6.6524587321e-25       /* Thomson cross section, cm^2     */

/* Hot cross-section table (reading: the paper tabulates sigma_h a priori
 * without stating the ranges). */
#define GMO_SH_NT 64
#define GMO_SH_NE 256
#define GMO_SH_TH_MIN 1e-2
#define GMO_SH_TH_MAX 1e3
#define GMO_SH_E_MIN 1e-12
#define GMO_SH_E_MAX 1e6

/* Every rejection loop stops after this many trials (never reached in the
 * configurations used; counted when it would be). */
#define GMO_MAX_TRIALS 100000

/* Margin on the per-zone frequency rejection bound. */
#define GMO_FMAX_MARGIN 1.02

typedef struct {
    uint64_t seed;
    uint32_t s[3];
    uint32_t block;
} gmo_rng;

double gmo_rng_next(gmo_rng *r);
void   gmo_sample_electron_rng(gmo_rng *r, double theta, double eps, double *gamma,
                               double *beta, double *mu, int64_t *trials);
void   gmo_scatter_in_frame(gmo_rng *r, double theta, double eps, double *gamma_out,
                            double *mu_out, double kout[4], int64_t *e_trials,
                            int64_t *ang_trials);
void   gmo_scatter_in_frame_dist(gmo_rng *r, const gmo_dist *d, double theta, double eps,
                                 double *gamma_out, double *mu_out, double kout[4],
                                 int64_t *e_trials, int64_t *ang_trials);
/* power law in the j = A s g(X) form, X = nu / (nu_c s) */
double gmo_pl_A(const gmo_dist *d, double n_e, double B);
double gmo_pl_nu_c(double B);
double gmo_pl_g(double X, double p);
double gmo_pl_ang(double p);            /* int_0^1 (1 - mu^2)^{(p+1)/4} dmu */
void   gmo_set_error(const char *msg);

#endif
