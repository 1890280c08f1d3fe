/*
 * gm.h -- C ABI of the MI355X (gfx950) superphoton Monte Carlo library.
 *
 * The library computes the spectrum emerging from hot, magnetised plasma by
 * grmonty-style Monte Carlo radiative transfer (Naethe Motta, Nemmen & Joshi,
 * "GPUmonty", arXiv 2602.13198): superphotons are emitted from each zone in
 * proportion to the thermal synchrotron emissivity, pushed along null
 * geodesics, attenuated by absorption, split by biased thermal Compton
 * scattering into child superphotons, and tallied by (frequency,
 * inclination) when they escape.
 *
 * Conventions
 *  - Every function returns gm_status; on error the message is available
 *    from gm_last_error() (per host thread) and, for GM_EINVAL, the context
 *    is unchanged.  No C++ exception crosses this boundary.
 *  - All work is queued on the HIP stream given to gm_create (NULL = the
 *    null stream).  Functions return once the work is queued, except where
 *    a host output is requested (documented per function), which
 *    synchronises that stream.
 *  - Caller buffers are borrowed for the duration of the call only.  The
 *    context owns every device buffer it allocates; gm_destroy frees them.
 *  - One context per host thread; a context is not thread safe.
 *  - Results depend only on (seed, instance, inputs, parameters): launch
 *    geometry and scheduling change them only through the summation order
 *    of the floating-point tallies.
 */
#ifndef GM_H
#define GM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gm_ctx gm_ctx;

typedef enum {
    GM_OK = 0,
    GM_EINVAL = -1,        /* bad argument; nothing changed                   */
    GM_ENOMEM = -2,        /* device allocation failed, or one root's
                              scattering cascade alone overflows a queue
                              (gm_track_scatter: see there)                */
    GM_EDEVICE = -3,       /* a HIP call failed                               */
    GM_ESTATE = -4,        /* call out of order (e.g. track before make)      */
    GM_EUNSUPPORTED = -5   /* option not built into this library              */
} gm_status;

#define GM_MAX_INSTANCES 64

/* Metric of the zone grid. */
#define GM_METRIC_MINKOWSKI_CART 0   /* flat, x^i Cartesian in units of ell         */
#define GM_METRIC_KS_MKS         1   /* Kerr, Kerr-Schild in modified coordinates:
                                        r = exp(x1), theta = pi x2 + (1-h)/2 sin(2 pi x2),
                                        phi = x3, lengths in r_g = ell              */
#define GM_METRIC_FLAT_SPH       2   /* flat spacetime in the same (ln r, x2, phi)
                                        coordinates, lengths in ell (the sphere
                                        tests of the paper's Tests section: a grid
                                        in t, log r, theta, phi); a_spin must be 0,
                                        no horizon, photons recorded at r_record    */

typedef struct {
    int    metric;          /* GM_METRIC_*                                        */
    int    n[3];            /* zones per coordinate, each >= 1                    */
    double x_start[3];      /* lower coordinate edge                              */
    double dx[3];           /* coordinate zone width, > 0                         */
    double a_spin;          /* Kerr spin |a| < 1 (KS); 0 (flat spherical)         */
    double h_slope;         /* polar slope h in (0, 1] (KS, flat spherical)       */
    double L_unit_cm;       /* length unit ell in cm, > 0                         */
    double r_record;        /* record radius in ell (KS, flat spherical)          */
} gm_grid;

/* Zone plasma in double precision, zone index z = (i1*n2 + i2)*n3 + i3.
 * ucon and bcon are [4][nzones] (component-major).  on_device = 1 means the
 * pointers are device pointers, else host pointers.  Every zone needs finite
 * n_e >= 0, B >= 0 and theta_e; zones with n_e > 0 need theta_e > 0 and
 * u^t > 0, and on (ln r, x2, phi) grids a timelike u at the zone centre.  These checks run on
 * the host for host inputs and in a kernel for device inputs; a failure is
 * GM_EINVAL with the first bad zone named.  bcon gives only the field
 * direction; its normalisation is ignored. */
/* Electrons of every zone of an instance.  Thermal: Maxwell-Juttner at the
 * zone's theta_e (Emissivity and Scattering sections).  Power law (the
 * non-thermal distributions the paper's Conclusions name as future work):
 * isotropic n(gamma) = n_e C gamma^-p on [gamma_min, gamma_max], with the
 * power law's asymptotic synchrotron emissivity and absorption (valid for
 * nu_c(gamma_min) << nu << nu_c(gamma_max)) and Compton scattering off the
 * distribution itself; FP64 only (GM_PRECISION_F32_EMISSIVITY with a power
 * law is GM_EUNSUPPORTED).  Instances share launches only with identical
 * electrons. */
#define GM_DIST_THERMAL  0
#define GM_DIST_POWERLAW 1
typedef struct {
    int    kind;            /* GM_DIST_*                                          */
    double p;               /* power law: index > 1                               */
    double gamma_min, gamma_max;   /* power law: 1 <= gamma_min < gamma_max, finite */
} gm_electrons;

typedef struct {
    int           on_device;
    const double *n_e;      /* electron density, cm^-3                            */
    const double *theta_e;  /* electron temperature kT/(m_e c^2)                  */
    const double *B;        /* field strength, Gauss                              */
    const double *ucon;     /* fluid 4-velocity, contravariant code components    */
    const double *bcon;     /* field direction 4-vector                            */
    gm_electrons  electrons;/* zeroed: thermal                                     */
} gm_zones;

typedef struct {
    double   n_target;      /* N_s, expected number of root superphotons (> 0)    */
    double   nu_min, nu_max;/* emission band in Hz, 0 < nu_min < nu_max          */
    int      n_wnodes;      /* weight-table nodes, odd, 3..4097                    */
    double   w_floor_rel;   /* weight floor relative to the table maximum, >= 0   */
    uint64_t seed;          /* key of every random stream                         */
} gm_emit_params;

/* Scattering bias b >= 1 (Scattering section of the paper). */
#define GM_BIAS_CONST  0    /* b = bias_value                                    */
#define GM_BIAS_THETA2 1    /* b = bias_value * Theta_e^2                        */
#define GM_BIAS_GEN2   2    /* b = (n_sc+1)^2 / (n_e sigma_T bias_value ell)     */
#define GM_BIAS_TABLE  3    /* b = exp T[zone](ln eps), the instance's table
                               (gm_set_bias_table) interpolated in ln eps of
                               the fluid-frame photon energy; bias_value is
                               ignored                                          */
#define GM_BIAS_LEARNED GM_BIAS_TABLE
#define GM_BIAS_WINDOW 4    /* weight window: b = w exp T[zone](ln eps), w the
                               photon's weight at the start of the step, so
                               that heavy photons split more and the children's
                               weights approach 1/importance.  Every mode is
                               clamped to [1, bias_max]; any b >= 1 keeps the
                               estimator unbiased (child w/b, parent w(1-1/b)). */

#define GM_PRECISION_F64 0  /* all transport arithmetic in double                 */
#define GM_PRECISION_F32_EMISSIVITY 1
                            /* emissivity, Kirchhoff absorption and the hot cross
                               section in single precision (log space, FP32 zone
                               records and table); geodesics, step control,
                               optical-depth sums, weights, sampling and tallies
                               in double                                          */

typedef struct {
    int     scattering;     /* 0: no Compton opacity; 1: biased thermal Compton   */
    int     bias_mode;      /* GM_BIAS_*                                          */
    double  bias_value;
    double  bias_max;       /* b is clamped to [1, bias_max]; bias_max >= 1       */
    int     n_sc_max;       /* highest generation that may still scatter, 0..15   */
    double  step_h;         /* step-size factor (Cartesian: fraction of a zone)   */
    double  verlet_tol;     /* corrector tolerance (the paper uses 1e-3)          */
    int     verlet_max_it;  /* corrector iteration cap, >= 1                      */
    double  roulette_frac;  /* Russian roulette when w < roulette_frac * w_birth  */
    double  roulette_p;     /* survival probability, (0, 1]                       */
    double  horizon_eps;    /* capture when r < r_h (1 + horizon_eps)             */
    int64_t max_steps;      /* a photon still alive after this many steps stops   */
    int     n_nu;           /* tally frequency bins, log-uniform on [nu_lo, nu_hi) */
    double  nu_lo, nu_hi;   /* Hz                                                 */
    int     n_theta;        /* tally inclination bins, uniform on [0, pi]         */
    int     precision;      /* GM_PRECISION_*                                     */
    /* Far-field steps (spherical grids; the paper leaves the step rule open):
     * an outgoing photon (k^1 > 0) at r > r_far takes its zone-crossing
     * quotient with step_h * step_far.  0 (or 1): off.  Otherwise step_far
     * must be >= 1, and r_far at least the outer radius of the outermost
     * zone holding plasma and 4 M (outside the photon orbits, where an
     * outgoing photon never turns back), else GM_EINVAL; ignored on the
     * Cartesian grid. */
    double  step_far;
    double  r_far;
} gm_track_params;

/* Ledger slots read by gm_read_spectrum (photons/s and erg/s at infinity). */
enum {
    GM_L_W_EMIT = 0, GM_L_E_EMIT, GM_L_W_ESC, GM_L_E_ESC, GM_L_W_OOB, GM_L_E_OOB,
    GM_L_W_ABS, GM_L_E_ABS, GM_L_W_CAPT, GM_L_E_CAPT, GM_L_W_CAPLOSS, GM_L_E_CAPLOSS,
    GM_L_W_ROUL, GM_L_E_ROUL, GM_L_W_STUCK, GM_L_E_STUCK, GM_L_E_COMPTON, GM_L_E_DRIFT,
    GM_L_N
};

/* Event counters returned by gm_track_scatter. */
enum {
    GM_S_ROOTS = 0, GM_S_CHILDREN, GM_S_STEPS, GM_S_VERLET_IT, GM_S_SCATTER,
    GM_S_ROUL_KILL, GM_S_ROUL_SURVIVE, GM_S_CAPTURED, GM_S_ESCAPED, GM_S_OOB, GM_S_STUCK,
    GM_S_OVERSHOOT, GM_S_NU_TRIALS, GM_S_DIR_TRIALS, GM_S_E_TRIALS, GM_S_ANG_TRIALS,
    GM_S_GEN0  /* GM_S_GEN0 + g: photons of generation g, g < 16 */
};
/* opacity evaluations of the tracking kernels (flat spacetime evaluates
 * once per zone entered: the opacities depend on the zone and on k only) */
#define GM_S_COEF_EVALS (GM_S_GEN0 + 16)
#define GM_S_N (GM_S_GEN0 + 17)

/* Termination kinds in trace records. */
#define GM_END_ESCAPE   1
#define GM_END_OOB      2
#define GM_END_CAPTURE  3
#define GM_END_ROULETTE 4
#define GM_END_STUCK    5
#define GM_END_SPLIT    6

/* One trace record per finished superphoton, 112 bytes. */
typedef struct {
    uint32_t s0, s1, s2;    /* random stream id (identifies the photon)           */
    int32_t  n_sc;          /* scattering generation                              */
    int32_t  kind;          /* GM_END_*                                           */
    int32_t  i_nu, i_theta; /* tally bin or -1                                    */
    uint32_t n_steps;
    double   w_birth, w_end;
    double   x[4], k[4];    /* position and wavevector at the end                 */
} gm_trace_rec;

/* Create a context on HIP device `device` queuing work on `hip_stream`
 * (a hipStream_t, or NULL).  Builds the device tables used by every run. */
gm_status gm_create(gm_ctx **out, int device, void *hip_stream);

/* Free every buffer the context owns (synchronises its stream). */
gm_status gm_destroy(gm_ctx *ctx);

/* Message of the last error on this host thread (never NULL). */
const char *gm_last_error(void);

/* Load the plasma of one instance (0 <= instance < GM_MAX_INSTANCES):
 * validates and copies the zones into packed device records and prepares
 * the per-zone emission constants (Emissivity section).  Replaces what the
 * instance held; its tallies are kept. */
gm_status gm_load_zones(gm_ctx *ctx, int instance, const gm_grid *grid, const gm_zones *zones);

/* Free everything an instance holds (zones, emission tables, tallies,
 * bias and emission tables, score weights); the instance can be loaded
 * again.  Synchronises. */
gm_status gm_unload_zones(gm_ctx *ctx, int instance);

/* The expected number of roots gm_make_superphotons would draw for these
 * parameters (the sum of the zones' expected counts under the instance's
 * emission table), without drawing or allocating any; the instance has to
 * be made again before tracking.  Synchronises. */
gm_status gm_expected_roots(gm_ctx *ctx, int instance, const gm_emit_params *params, double *expected);

/* Superphoton generation (Creation of superphotons and Sampling procedure
 * sections): builds the weight table w(nu) (eq:weight_calc), draws each
 * zone's superphoton count by stochastic rounding of its expectation, and
 * assigns photon ids.  instance = -1 makes every loaded instance with the
 * same parameters.  n_made (may be NULL) receives the number of roots of the
 * last instance made and synchronises the stream. */
gm_status gm_make_superphotons(gm_ctx *ctx, int instance, const gm_emit_params *params,
                               uint64_t *n_made);

/* Track every root made and not yet tracked, and all its descendants, to
 * escape, capture or loss (geodesic, Absorption and Scattering sections),
 * adding to the tallies.  stats (may be NULL) receives GM_S_N counters of
 * this call and synchronises the stream.  Instances of one metric share
 * launches (gm_set_batch); their tallies are kept per block in LDS when
 * they fit the 56 KiB budget, else added to in HBM (gm_set_tally_mode).
 * GM_ENOMEM if the scattering cascade of a single root overflows the photon
 * queue: the instances of the launch group that failed are left as before
 * the call (tallies, ledgers, trace and event-log counts restored, roots
 * still pending); groups tracked before it keep their results. */
gm_status gm_track_scatter(gm_ctx *ctx, const gm_track_params *params, int64_t *stats);

/* The recorded spectrum (Recording of superphotons, the last of the paper's
 * five kernels: each escaping superphoton adds its energy to its frequency
 * bin; inclination bins as in the Tests section's spectra).  Copies the
 * tally of one instance into `out` = [n_theta][n_nu][3] doubles
 * {sum of w E, sum of (w E)^2, number of superphotons}, E the energy at
 * infinity in erg (so sums are erg/s; nu L_nu of a bin is
 * (4 pi / dOmega) sum(w E) / dln(nu)), out_on_device selecting a device or
 * host buffer (caller-owned, n_theta*n_nu*3 doubles); ledger_out (host, may
 * be NULL) receives GM_L_N doubles.  reset = 1 clears the tally and ledger
 * afterwards.  GM_ESTATE if the instance has never been tracked.
 * Synchronises. */
gm_status gm_read_spectrum(gm_ctx *ctx, int instance, double *out, int out_on_device,
                           double *ledger_out, int reset);

/* ---- inspection (tests, diagnostics) --------------------------------- */

/* Per-zone results of the last make of an instance, host buffers, any may
 * be NULL: counts [nz] u32, expected counts [nz], frequency rejection bound
 * [nz], ln w at the weight nodes [n_wnodes].  Synchronises. */
gm_status gm_read_emission(gm_ctx *ctx, int instance, uint32_t *counts, double *nbar,
                           double *fmax, double *ln_w);

/* Record one gm_trace_rec per finished photon into a device buffer of
 * `capacity` records (NULL disables).  Records past the capacity are
 * counted but not written.  gm_trace_count returns the count (synchronises). */
gm_status gm_set_trace(gm_ctx *ctx, void *device_buffer, uint64_t capacity);
gm_status gm_trace_count(gm_ctx *ctx, uint64_t *n);

/* The hot cross-section table ln(sigma_h/sigma_T) [64 ln Theta][256 ln eps]
 * over Theta in [1e-2, 1e3], eps in [1e-12, 1e6], into a host buffer. */
gm_status gm_sigma_hot_table(gm_ctx *ctx, double *host_out);

/* Angle-integrated emissivity shape G(Xc) = int_0^1 s g(Xc/s) dmu,
 * s = sqrt(1-mu^2), evaluated on the device for n host values. */
gm_status gm_eval_G(gm_ctx *ctx, const double *host_x, double *host_out, int n);

/* Scheduling of the tracking kernel (results do not depend on it):
 * track_waves selects the compiled variant targeting 2, 3 or 4 waves per
 * SIMD (fewer registers per lane at higher targets); refill_min (1..64) is
 * the number of idle lanes at which a wave claims new photons. */
gm_status gm_set_tuning(gm_ctx *ctx, int track_waves, int refill_min);

/* Instances per launch (1..GM_MAX_INSTANCES, default all): gm_track_scatter
 * tracks the pending instances of one metric together -- one birth launch
 * and per generation one tracking and one scattering launch over all their
 * photons -- in groups of at most this many (GPU implementation section:
 * batches).  Results do not depend on it. */
gm_status gm_set_batch(gm_ctx *ctx, int max_instances);

/* HIP graphs (scheduling; results do not depend on it): with enable = 1,
 * gm_track_scatter records each root chunk's launch sequence -- counter
 * reset, birth, and per generation the tracking, event-count and
 * scattering kernels -- as a HIP graph by stream capture on a private
 * stream and launches that graph on the context's stream, updating the
 * executable graph in place when only kernel arguments changed (a new
 * instantiation otherwise).  Per-launch event timing (gm_set_timing) is not
 * recorded in this mode.  enable = 0 launches directly (default), -1 only
 * reads the counters: graph launches and instantiations since creation. */
gm_status gm_set_graph(gm_ctx *ctx, int enable, uint64_t *launches, uint64_t *instantiations);

/* Photon queues (scheduling; results do not depend on it beyond the order
 * of FP64 tally sums).  gm_track_scatter runs the roots in chunks of half the
 * queue capacity through all scattering generations.  A chunk whose
 * children overflow a queue is undone -- tallies, ledgers, counters and the
 * trace and event-log counts restored -- and redone in quarters; histories
 * are keyed by their roots, so the redone chunk gives the same photons.
 * GM_ENOMEM only if the cascade of a single root overflows.
 * gm_set_queue_capacity fixes the capacity in entries (0 = automatic:
 * max(2^22, 2 x the roots of all pending instances), at most 2^26;
 * otherwise 64 .. 2^27), 128
 * bytes per entry per queue, two queues.  gm_queue_stats returns the
 * capacity of the last gm_track_scatter and the number of chunks redone
 * since the context was created. */
gm_status gm_set_queue_capacity(gm_ctx *ctx, uint64_t entries);
gm_status gm_queue_stats(gm_ctx *ctx, uint64_t *capacity, uint64_t *chunk_retries);

/* Scattering bias of one instance (GM_BIAS_*, value, maximum), overriding
 * the bias of the track parameters for it, so that instances with
 * different biases share launches; bias_mode < 0 removes the override.
 * Scattering section of the paper (bias b >= 1). */
gm_status gm_set_instance_bias(gm_ctx *ctx, int instance, int bias_mode, double bias_value,
                               double bias_max);

/* Event timing of the tracking kernel: with timing enabled, every launch of
 * the tracking kernel is bracketed by HIP events on the context's stream.
 * gm_read_timing returns the summed event durations (ms) and the number of
 * launches since timing was last enabled (synchronises on the events). */
gm_status gm_set_timing(gm_ctx *ctx, int enable);
gm_status gm_read_timing(gm_ctx *ctx, double *track_ms, uint64_t *track_launches);

/* Register-limited FP64 bound (measurement, not a passage of the paper):
 * runs `chains` (1, 2, 4 or 8) independent chains of `iters` dependent FP64
 * fused multiply-adds x <- fma(x, 0.9999999, 1e-7) per lane, started at
 * x_c = (1 + 1e-9 t) + 1e-3 c (each operation rounded) for global lane t
 * and chain c, on exactly
 * `waves` waves per SIMD on every CU (grid = CUs x waves blocks of 256; each
 * block reserves LDS so that no more blocks fit), and times one launch with
 * HIP events after a short warm-up.  Returns the time (ms) and the attained
 * rate (TFLOP/s, FMA = 2).  host_out (n_out doubles, may be NULL with
 * n_out = 0) receives the sums over chains of the first n_out lanes.
 * GM_EUNSUPPORTED if the LDS cannot pin that occupancy. */
gm_status gm_fma_chain_bound(gm_ctx *ctx, int waves, int chains, int64_t iters, double *ms, double *tflops,
                             double *host_out, int n_out);

/* ---- learned form ----------------------------------------------------
 * Not a passage of the paper: the paper names bias tuning as future work
 * (Conclusions).  A network 6 -> 64 -> 64 -> 2 (tanh hidden layers) is
 * evaluated and trained with matrix-core kernels (BF16 operands, FP32
 * accumulation, FP32 master weights and Adam state on the device).
 * Parameter vector (float32, GM_MLP_PARAMS entries), in order:
 * W1[6][64], b1[64], W2[64][64], b2[64], W3[64][2], b3[2]; a layer maps
 * h -> tanh(h W + b) (the last without tanh).  Feature rows are 8 floats
 * (6 features, 2 ignored), outputs and targets 2 floats per row. */
#define GM_MLP_PARAMS 4738

/* Set the parameters from a host vector; resets the Adam state. */
gm_status gm_mlp_set_params(gm_ctx *ctx, const float *host_params);
/* Copy the FP32 parameters to a host vector (synchronises). */
gm_status gm_mlp_get_params(gm_ctx *ctx, float *host_params);
/* Outputs for n rows: X [n][8] and Y [n][2] are device buffers; stream-
 * ordered, no synchronisation. */
gm_status gm_mlp_forward(gm_ctx *ctx, const float *X, int64_t n, float *Y);
/* Loss of gm_mlp_grad and gm_mlp_train_step: GM_MLP_SQUARED (default)
 * L = sum_rows sum_o C[r][o] (y[r][o] - T[r][o])^2, or GM_MLP_POISSON, the
 * log-link Poisson deviance L = sum C[r][o] (e^{y[r][o]} - T[r][o] y[r][o]),
 * whose minimiser is y = ln E[T] (targets >= 0, mostly zero allowed). */
#define GM_MLP_SQUARED 0
#define GM_MLP_POISSON 1
gm_status gm_mlp_set_loss(gm_ctx *ctx, int kind);
/* Gradient of the loss with respect to the parameters, into host vectors
 * grad [GM_MLP_PARAMS] and loss [1] (either may be NULL).  X [n][8],
 * T [n][2], C [n][2] are device buffers; the caller normalises C.  The
 * result does not depend on scheduling (bitwise).  Synchronises. */
gm_status gm_mlp_grad(gm_ctx *ctx, const float *X, const float *T, const float *C, int64_t n,
                      float *grad, float *loss);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid
 * allocation): gm_mlp_grad without any allocation and without
 * synchronisation.  X [n][8], T [n][2], C [n][2] are device buffers as for
 * gm_mlp_grad; grad_loss is a caller-owned device buffer of
 * GM_MLP_PARAMS + 1 floats that receives the gradient followed by the loss.
 * The per-block partial gradients live in a fixed scratch array of 32 MiB
 * that each GPU holds until the process ends, which limits n to
 * GM_MLP_NOALLOC_MAX_ROWS (GM_EINVAL above it).  Every call on one GPU
 * shares that array: calls that overlap in time on the same GPU (other
 * streams, other contexts) race and give wrong results.  The work is queued
 * on the context's stream; the result is ready when that stream reaches it. */
#define GM_MLP_NOALLOC_MAX_ROWS 56640
gm_status gm_mlp_grad_noalloc(gm_ctx *ctx, const float *X, const float *T, const float *C, int64_t n,
                              float *grad_loss);

/* One Adam step (beta 0.9, 0.999, eps 1e-8) on the same loss with learning
 * rate lr; loss (host, may be NULL: no synchronisation) receives the loss
 * before the step. */
gm_status gm_mlp_train_step(gm_ctx *ctx, const float *X, const float *T, const float *C, int64_t n,
                            float lr, float *loss);

/* `steps` Adam steps of gm_mlp_train_step queued in one call, step s on the
 * rows [k b, (k + 1) b) with k = s mod floor(n / b) (consecutive batches of
 * the rows as given: shuffle them first), learning rate
 * lr0 * decay^(s / steps); loss_first_last (host, may be NULL) receives the
 * loss before the first and before the last step.  The same kernels in the
 * same order as the single steps, so the parameters equal those of the
 * equivalent sequence of gm_mlp_train_step calls bit for bit.  GM_EINVAL
 * for b < 1, b > n or steps < 1.  Synchronises only for loss_first_last. */
gm_status gm_mlp_train_steps(gm_ctx *ctx, const float *X, const float *T, const float *C, int64_t n,
                             int64_t b, int steps, float lr0, float decay, float *loss_first_last);

/* ---- tables and records of the learned and adaptive forms -------------
 * Not passages of the paper, which names tuning the bias "on the fly" as
 * future work (Conclusions); they only change where superphotons are
 * spent, never the expected spectrum.
 *
 * A per-zone table holds n values per zone on nodes uniform in a log
 * variable over [lo, hi]; between nodes a value is linear in that
 * variable, outside [lo, hi] it is the end node's value.  Tables are host
 * arrays [nzones][n], copied (synchronises); GM_ESTATE before gm_load_zones.
 *
 * Bias table T (variable ln eps, eps the fluid-frame photon energy in
 * m_e c^2), used by GM_BIAS_TABLE and GM_BIAS_WINDOW. */
gm_status gm_set_bias_table(gm_ctx *ctx, int instance, const double *table, int n_eps,
                            double ln_eps_lo, double ln_eps_hi);

/* Emission table m (variable ln nu, Hz): zone i's superphotons get the
 * weight w_i(nu) = w(nu) e^{-m_i(ln nu)} (eq:weight_calc), so its expected
 * count at nu rises by e^{m_i} (Sampling procedure) while the expected
 * emitted luminosity is unchanged.  table = NULL removes it.  Takes effect
 * at the next gm_make_superphotons, which then recomputes the expected
 * counts and rejection bounds. */
gm_status gm_set_emission_table(gm_ctx *ctx, int instance, const double *table, int n_nu_nodes,
                                double ln_nu_lo, double ln_nu_hi);

/* Event log: one record per scattering (the child it creates, when the
 * scattering point holds plasma) and one per root whose photon id is a
 * multiple of root_stride (its emission; root_stride = 0: none), written by
 * gm_track_scatter into a caller-owned device buffer of `capacity` records
 * (NULL disables; capacity <= 2^32 - 2).  Records past the capacity are
 * counted, not kept, and start no ancestry.  At the end of gm_track_scatter
 * every record's score holds the sum of w E s_bin over the photon it
 * created and all its descendants that escape into a tally bin (E the
 * energy at infinity in erg, s_bin the instance's score weight of the bin,
 * 1 by default); summation order varies (FP64 atomics).  gm_event_count
 * returns the count (synchronises). */
typedef struct {
    uint32_t s0, s1, s2;    /* stream of the photon the event created (its trace key) */
    uint32_t p0, p1, p2;    /* stream of the photon that scattered (0: emission)   */
    int32_t  zone;          /* zone whose plasma scattered or emitted              */
    int32_t  gen;           /* generation of the created photon                    */
    uint32_t parent;        /* record of the photon that scattered (0xffffffff: none) */
    uint32_t pad;
    double   eps;           /* fluid-frame energy of the incoming or emitted photon,
                               m_e c^2                                              */
    double   w;             /* weight of the created photon                        */
    double   score;
    double   x[3];          /* event position (code coordinates)                   */
} gm_event_rec;
gm_status gm_set_event_log(gm_ctx *ctx, void *device_buffer, uint64_t capacity, uint64_t root_stride);
gm_status gm_event_count(gm_ctx *ctx, uint64_t *n);

/* Least and greatest fluid-frame energy eps (m_e c^2) of the event log's
 * emission records (generation 0, positive weight), found on the device:
 * the band the plain roots were born in, over which the importance forms
 * lay the emission proposal's nodes (the proposal density of the Sampling
 * procedure section, made adaptive).  GM_ESTATE without an event log or
 * without such a record.  Synchronises. */
gm_status gm_event_band(gm_ctx *ctx, double *eps_min, double *eps_max);

/* Tables of an instance built on the device from importance estimates.  A
 * map says which table (bias: nodes in ln eps of the incoming fluid-frame
 * photon energy; emission: nodes in ln nu, Hz, of the emitted photon), its
 * n_nodes nodes over [lo, hi], and how an estimate ln I of the importance of
 * a unit-weight photon created at (zone, node) becomes a table value:
 *   GM_IMP_LINEAR   T = a ln I + b + shift
 *   GM_IMP_MIXTURE  T = ln((1 - alpha) + alpha exp(a ln I + b)) + shift, 0 <= alpha < 1
 * (for the emission table a defensive proposal: no zone emits fewer than
 * 1 - alpha of its plain roots).  Zones without plasma get 0.  The table
 * replaces the instance's table of that kind; an emission table takes
 * effect at the next gm_make_superphotons.  Synchronises. */
#define GM_TABLE_BIAS 0
#define GM_TABLE_EMISSION 1
#define GM_IMP_LINEAR 0
#define GM_IMP_MIXTURE 1
typedef struct {
    int    table;           /* GM_TABLE_*                                          */
    int    n_nodes;         /* 2..4096                                             */
    double lo, hi;          /* node range of the table variable                   */
    int    kind;            /* GM_IMP_*                                            */
    double a, b, alpha;
    double shift;           /* added to every value after the mapping             */
    int    per_photon;      /* cells: 0 = I per unit weight (score / weight),
                               1 = I per photon (score / records)                  */
} gm_importance_map;

/* ln I from the network's output `output` (0 or 1) for every (zone, node):
 * features ln Theta_e, ln n_e, ln(B + 1e-10 G), ln eps, radius (Kerr: ln r
 * of the zone centre; flat: |x| over the grid half-size), cos theta of the
 * centre, standardised as (f - mu) / sd, evaluated on the matrix cores. */
gm_status gm_mlp_fill_table(gm_ctx *ctx, int instance, const gm_importance_map *map, int output,
                            const float mu[6], const float sd[6]);

/* ln I from the event log's records (scattering records for the bias
 * table, emission records for the emission table): summed scores and
 * weights per cell of blocks[0] x blocks[1] x blocks[2] zones and node
 * (nearest node of the record's ln eps, resp. ln nu); gm_cells_accumulate
 * forms the sums (kept in the context) and returns their totals [3]
 * {sum score, sum weight, records}; gm_cells_fill_table then writes the
 * ratio score / weight (per_photon = 0) or score / records (per_photon =
 * 1) of each zone's cell, shrunk towards the overall ratio with `prior`
 * records (cells without records take the overall ratio).  The map of
 * both calls must name the same table and nodes. */
gm_status gm_cells_accumulate(gm_ctx *ctx, int instance, const gm_importance_map *map, const int blocks[3],
                              double totals[3]);
/* Map an instance's table (map->table, with the map's node layout) in
 * place, its values taken as ln I: T <- map(T) for every zone holding
 * plasma (the others keep their neutral value) -- the mixture and the
 * shift of the emission proposal without a second inference. */
gm_status gm_remap_table(gm_ctx *ctx, int instance, const gm_importance_map *map);

/* Copy an instance's bias or emission table (GM_TABLE_*) into a host
 * buffer of n = nzones x nodes doubles; n_nodes (may be NULL) receives the
 * node count; host_out = NULL only reports it.  Synchronises. */
gm_status gm_read_table(gm_ctx *ctx, int instance, int table, double *host_out, int64_t n, int *n_nodes);
gm_status gm_cells_fill_table(gm_ctx *ctx, int instance, const gm_importance_map *map, double prior);

/* Score weights of an instance's event records: host array [n_theta][n_nu]
 * (n must match the tally of the next gm_track_scatter), copied; NULL
 * restores the weight 1. */
gm_status gm_set_score_weights(gm_ctx *ctx, int instance, const double *sw, int n);

/* Where the tallies of a shared launch accumulate (scheduling; results
 * change only through the order of FP64 sums): 0 automatic (per-block LDS
 * tallies when those of the launch group fit 56 KiB, else direct FP64
 * atomics on the instances' tallies in HBM), 1 LDS (GM_EUNSUPPORTED at
 * track time if one instance's tally does not fit), 2 HBM. */
gm_status gm_set_tally_mode(gm_ctx *ctx, int mode);

#ifdef __cplusplus
}
#endif
#endif
