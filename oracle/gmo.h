/*
 * gmo.h -- plain CPU oracle for grmonty-style superphoton Monte Carlo
 * radiative transfer (Naethe Motta, Nemmen & Joshi, "GPUmonty", arXiv 2602.13198).
 *
 * TEST INFRASTRUCTURE.  This library exists only to check the HIP path.
 * Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
 * may load or call it.  It shares no code, header, table or constant with
 * paper_2602_13198_amd/ and never calls into it.
 *
 * Everything is IEEE double precision, written for readability rather than
 * speed.  Each function cites the passage of the paper it follows
 * (section / equation label).  Where the paper is silent or garbled the
 * reading taken is stated at the point of use.
 *
 * Parity pins: every physics function here is checked in tests/ against
 * closed forms, scipy/mpmath, brute force or invariants (see the test files
 * test_oracle_*.py).  Functions without such a pin say "parity unpinned".
 */
#ifndef GMO_H
#define GMO_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define GMO_OK          0
#define GMO_EINVAL     -1
#define GMO_ENOMEM     -2
#define GMO_ESTATE     -4
#define GMO_EUNSUP     -5

/* ---- metric / grid --------------------------------------------------- */
#define GMO_METRIC_MINKOWSKI_CART 0   /* x^i Cartesian, Gamma == 0          */
#define GMO_METRIC_KS_MKS         1   /* Kerr-Schild in modified coordinates */
#define GMO_METRIC_FLAT_SPH       2   /* flat spacetime, x = (t, ln r, x2, phi),
                                         theta(x2) as in the modified coordinates;
                                         a_spin must be 0, no horizon           */

typedef struct {
    int    metric;
    int    n[3];            /* zones per coordinate                        */
    double x_start[3];      /* lower coordinate edge of the grid           */
    double dx[3];           /* coordinate zone width                       */
    double a_spin;          /* KS only: dimensionless spin                 */
    double h_slope;         /* KS, SPH: polar slope parameter              */
    double L_unit_cm;       /* length unit ell in cm                       */
    double r_record;        /* KS, SPH: record radius in ell               */
} gmo_grid;

/* Electron distribution of a loaded plasma: thermal (Maxwell-Juttner at
 * the zone's Theta_e) or an isotropic power law n(gamma) = n_e C gamma^-p
 * on [g1, g2], the same in every zone (the non-thermal distributions the
 * paper names as future work, Conclusions). */
#define GMO_DIST_THERMAL  0
#define GMO_DIST_POWERLAW 1
typedef struct {
    int    kind;            /* GMO_DIST_*                                   */
    double p, g1, g2;       /* power law: index p > 1, 1 <= g1 < g2         */
} gmo_dist;

/* Zone plasma, row-major zone index z = (i1*n2 + i2)*n3 + i3. */
typedef struct {
    const double *n_e;      /* [nz] electron density cm^-3                 */
    const double *theta_e;  /* [nz] kT_e/(m_e c^2)                         */
    const double *B;        /* [nz] field strength, Gauss                   */
    const double *ucon;     /* [4][nz] fluid 4-velocity, code components    */
    const double *bcon;     /* [4][nz] field direction 4-vector (any norm)  */
    gmo_dist dist;          /* electrons of every zone                     */
} gmo_zones;

typedef struct {
    double   n_target;      /* N_s: expected number of root superphotons    */
    double   nu_min, nu_max;/* emission band, Hz                            */
    int      n_wnodes;      /* weight-table nodes (odd, >= 3)               */
    double   w_floor_rel;   /* weight-table floor relative to its maximum   */
    uint64_t seed;
    int      instance;      /* enters every stream key                      */
} gmo_emit_params;

#define GMO_BIAS_CONST  0
#define GMO_BIAS_THETA2 1
#define GMO_BIAS_GEN2   2
#define GMO_BIAS_TABLE  3   /* b = exp(T_zone(ln eps)), T from gmo_set_bias_table     */
#define GMO_BIAS_WINDOW 4   /* b = w exp(T_zone(ln eps)), w the weight at the start
                               of the step (weight-window splitting)                */

typedef struct {
    int    scattering;      /* 0: no Compton opacity at all                 */
    int    bias_mode;
    double bias_value;      /* CONST: b; THETA2: coefficient; GEN2: R (ell) */
    double bias_max;
    int    n_sc_max;        /* scattering generations allowed               */
    double step_h;          /* step-size factor                             */
    double verlet_tol;      /* corrector tolerance                          */
    int    verlet_max_it;
    double roulette_frac;   /* roulette when w < roulette_frac * w_birth    */
    double roulette_p;      /* survival probability                         */
    double horizon_eps;     /* capture when r < r_h (1 + horizon_eps)       */
    int64_t max_steps;
    int    n_nu;  double nu_lo, nu_hi;  /* tally frequency bins, Hz         */
    int    n_theta;                      /* tally inclination bins          */
    double step_far, r_far; /* outgoing photons beyond r_far: step_h * step_far
                               (spherical grids; 0 or 1: off)              */
} gmo_track_params;

/* Termination kinds written into trace records. */
#define GMO_END_ESCAPE    1
#define GMO_END_OOB       2   /* escaped outside the tally band            */
#define GMO_END_CAPTURE   3
#define GMO_END_ROULETTE  4
#define GMO_END_STUCK     5
#define GMO_END_SPLIT     6   /* b == 1: all weight handed to the child    */

/* One record per finished superphoton (root or child).  112 bytes. */
typedef struct {
    uint32_t s0, s1, s2;    /* stream id                                    */
    int32_t  n_sc;          /* scattering generation                        */
    int32_t  kind;
    int32_t  i_nu, i_theta; /* tally bin, -1 when not tallied               */
    uint32_t n_steps;
    double   w_birth, w_end;
    double   x[4], k[4];    /* state at termination                         */
} gmo_trace_rec;

/* Ledger slots (weights in photons/s, energies in erg/s at infinity). */
enum {
    GMO_L_W_EMIT = 0, GMO_L_E_EMIT,
    GMO_L_W_ESC, GMO_L_E_ESC,
    GMO_L_W_OOB, GMO_L_E_OOB,
    GMO_L_W_ABS, GMO_L_E_ABS,
    GMO_L_W_CAPT, GMO_L_E_CAPT,
    GMO_L_W_CAPLOSS, GMO_L_E_CAPLOSS,
    GMO_L_W_ROUL, GMO_L_E_ROUL,        /* net weight/energy added by roulette */
    GMO_L_W_STUCK, GMO_L_E_STUCK,
    GMO_L_E_COMPTON,                   /* sum over children w(e_child-e_parent) */
    GMO_L_E_DRIFT,                     /* sum w * change of -k_t along steps    */
    GMO_L_N
};

/* Event counters. */
enum {
    GMO_S_ROOTS = 0, GMO_S_CHILDREN, GMO_S_STEPS, GMO_S_VERLET_IT,
    GMO_S_SCATTER, GMO_S_ROUL_KILL, GMO_S_ROUL_SURVIVE, GMO_S_CAPTURED,
    GMO_S_ESCAPED, GMO_S_OOB, GMO_S_STUCK, GMO_S_OVERSHOOT,
    GMO_S_NU_TRIALS, GMO_S_DIR_TRIALS, GMO_S_E_TRIALS, GMO_S_ANG_TRIALS,
    GMO_S_GEN0                          /* GMO_S_GEN0 + g: photons of gen g */
};
#define GMO_MAX_GEN 16
#define GMO_S_N (GMO_S_GEN0 + GMO_MAX_GEN)

/* ---- special functions and sampling primitives (exported for pins) ---- */
void   gmo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double gmo_uniform_at(uint64_t seed, const uint32_t stream[3], uint32_t block);
void   gmo_child_stream(uint64_t seed, const uint32_t parent[3], uint32_t block,
                        uint32_t child[3]);

double gmo_quad(double (*f)(double, void *), void *ctx, double a, double b,
                double rel_tol);
double gmo_k2(double x);                 /* modified Bessel K_2            */
double gmo_k2_of_theta(double theta_e);  /* K_2(1/Theta) with the large-Theta form */
double gmo_g_of_X(double X);             /* Leung et al. fit shape          */
double gmo_G_of_Xc(double Xc);           /* angle integral of the shape     */
double gmo_nu_c(double theta_e, double B);
double gmo_A_coef(double n_e, double theta_e, double B);
double gmo_jnu(double n_e, double theta_e, double B, double nu, double cos_th);
double gmo_Jnu(double n_e, double theta_e, double B, double nu);  /* int j dOmega */
double gmo_planck(double nu, double theta_e);
double gmo_sigma_kn(double eps);        /* sigma_KN / sigma_T              */
double gmo_sigma_hot_direct(double theta_e, double eps); /* sigma_h / sigma_T by quadrature */
void   gmo_sigma_hot_table(double *ln_table);   /* [64][256] ln(sigma_h/sigma_T) */
double gmo_sigma_hot_lookup(const double *ln_table, double theta_e, double eps);

/* Draw one electron (gamma, mu) and the scattered photon in the fluid frame
 * for a photon of fluid-frame energy eps moving along +x of an orthonormal
 * frame, electron direction completed with the frame's y/z axes.  Returns the
 * scattered photon (eps', n') in that frame; the stream counter advances in
 * the same order the transport uses. */
void   gmo_sample_scatter_frame(uint64_t seed, const uint32_t stream[3], uint32_t *block,
                                double theta_e, double eps,
                                double *gamma_out, double *mu_out,
                                double kout[4], int64_t *e_trials, int64_t *ang_trials);
void   gmo_sample_electron(uint64_t seed, const uint32_t stream[3], uint32_t *block,
                           double theta_e, double eps, double *gamma, double *mu,
                           int64_t *trials);

/* Power-law electrons: emissivity (per steradian) and invariant absorption
 * nu alpha at angle arccos(cos_th) to the field, their angle integral, the
 * hot cross section by quadrature, and the scattering of one photon with an
 * electron of the distribution (thermal at theta_e when d is thermal). */
double gmo_pl_jnu(const gmo_dist *d, double n_e, double B, double nu, double cos_th);
double gmo_pl_Jnu(const gmo_dist *d, double n_e, double B, double nu);
double gmo_pl_nualpha(const gmo_dist *d, double n_e, double B, double nu, double cos_th);
double gmo_sigma_pl_direct(const gmo_dist *d, double eps);
void   gmo_sample_scatter_frame_dist(uint64_t seed, const uint32_t stream[3], uint32_t *block,
                                     const gmo_dist *d, double theta_e, double eps,
                                     double *gamma_out, double *mu_out, double kout[4],
                                     int64_t *e_trials, int64_t *ang_trials);

/* Metric at a code-coordinate point: g_{mu nu} (gcov) and, when gcon is not
 * NULL, its inverse.  Christoffel symbols of the second kind, Gam[mu][a][b]. */
void   gmo_gcov(const gmo_grid *grid, const double x[4], double gcov[4][4]);
void   gmo_gcon(const gmo_grid *grid, const double x[4], double gcon[4][4]);
void   gmo_christoffel(const gmo_grid *grid, const double x[4], double Gam[4][4][4]);
double gmo_sqrt_neg_g(const gmo_grid *grid, const double x[4]);
double gmo_r_of_x1(const gmo_grid *grid, double x1);
double gmo_th_of_x2(const gmo_grid *grid, double x2);

/* Integrate a bare null geodesic with the transport's step rule (factor h)
 * and Verlet integrator; out receives n rows (x[4], k[4]).  Stops early when
 * r leaves [r_min, r_max] (KS).  Returns the rows written. */
int    gmo_integrate_geodesic(const gmo_grid *grid, const double x0[4], const double k0[4],
                              double h, double tol, int max_it, int n, double r_min,
                              double r_max, double *out);

/* ---- the method, as a context --------------------------------------- */
typedef struct gmo_ctx gmo_ctx;

gmo_ctx *gmo_create(void);
void     gmo_destroy(gmo_ctx *c);
int      gmo_load_zones(gmo_ctx *c, const gmo_grid *grid, const gmo_zones *z);
int      gmo_make_superphotons(gmo_ctx *c, const gmo_emit_params *p, uint64_t *n_made);
/* Per-zone emission results of the last make: counts [nz], expected counts
 * [nz], per-zone rejection bound [nz], ln w at the weight nodes [n_wnodes]. */
int      gmo_read_emission(const gmo_ctx *c, uint32_t *counts, double *nbar,
                           double *fmax, double *ln_w);
/* Track roots [root_begin, root_end) of the last make and all their
 * descendants.  Trace records are written while trace_n < trace_cap. */
int      gmo_track_scatter(gmo_ctx *c, const gmo_track_params *p,
                           uint64_t root_begin, uint64_t root_end, int n_threads,
                           gmo_trace_rec *trace, uint64_t trace_cap, uint64_t *trace_n);
/* Spectrum [n_theta][n_nu][3] = {sum wE, sum (wE)^2, count}, ledger
 * [GMO_L_N], stats [GMO_S_N]; reset clears all three afterwards. */
int      gmo_read_spectrum(gmo_ctx *c, double *spec, double *ledger, int64_t *stats,
                           int reset);
const char *gmo_last_error(void);

/* ---- tables and records of the learned / adaptive forms --------------
 * Not passages of the paper, which names bias tuning only as future work
 * (Conclusions).  A per-zone table holds n_nodes values per zone on nodes
 * uniform in a log variable over [lo, hi]; between nodes a value is linear
 * in that variable, outside [lo, hi] it is the end node's value.
 *
 * Bias table (variable ln eps, eps the fluid-frame photon energy in
 * m_e c^2): used by GMO_BIAS_TABLE and GMO_BIAS_WINDOW.  Any b >= 1 keeps
 * the estimator unbiased (Scattering section: child w/b, parent w(1-1/b)).
 *
 * Emission table (variable ln nu): m_i(nu) lowers the weight of zone i's
 * superphotons, ln w_i(nu) = ln w(nu) - m_i(nu), which raises its expected
 * count by the same factor inside the integral of the Sampling procedure;
 * the expected emitted luminosity does not change (eq:weight_calc).
 * NULL removes the table.  Both are copied. */
int gmo_set_bias_table(gmo_ctx *c, const double *tab, int n_nodes, double lo, double hi);
int gmo_set_emission_table(gmo_ctx *c, const double *tab, int n_nodes, double lo, double hi);
/* A table's value for zone z at log variable v (which: 0 bias, 1 emission). */
double gmo_table_value(const gmo_ctx *c, int which, int zone, double v);

/* Event records: one per scattering (the child it creates) and one per
 * root whose id is a multiple of root_stride (its emission).  score sums,
 * over the created photon and all its descendants that escape into a
 * tally bin, w E s_bin with E the energy at infinity in erg and s_bin the
 * score weight of the bin (1 when no weights are set). */
typedef struct {
    uint32_t s0, s1, s2;    /* stream of the photon the event created        */
    uint32_t p0, p1, p2;    /* stream of the photon that scattered (0: emission) */
    int32_t  zone;          /* zone whose plasma scattered or emitted        */
    int32_t  gen;           /* generation of the created photon               */
    double   eps;           /* fluid-frame energy of the incoming photon (scattering)
                               or of the emitted photon, m_e c^2              */
    double   w;             /* weight of the created photon                   */
    double   score;
    double   x[3];          /* event position, code coordinates               */
} gmo_event_rec;

/* buf = NULL disables the log.  Records beyond cap are counted, not kept. */
int gmo_set_event_log(gmo_ctx *c, gmo_event_rec *buf, uint64_t cap, uint64_t root_stride);
int gmo_event_count(const gmo_ctx *c, uint64_t *n);
/* Score weights [n_theta][n_nu] of the next track calls (n must match
 * their tally), NULL = 1. */
int gmo_set_score_weights(gmo_ctx *c, const double *sw, int n);

#ifdef __cplusplus
}
#endif
#endif
