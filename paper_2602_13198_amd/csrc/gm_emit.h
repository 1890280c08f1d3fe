// gm_emit.h -- zone preparation and superphoton generation (device side).
#pragma once

#include "gm_emis32.h"
#include "gm_frame.h"
#include "gm_kerr.h"

namespace gm {

// Packs the caller's zone arrays into 128-byte records and computes the
// per-zone emission constants (Emissivity section): A, nu_c, and the
// zone's emitting volume sqrt(-g) dx1 dx2 dx3 ell^3 at its centre.
struct PrepArgs {
    const double *n_e, *theta, *B, *ucon, *bcon;
    double *zrec, *vol;
    float *zrec32;
    int *emits;
    int n[3];
    double xs[3], dx[3];
    double L3;
    int nz;
    int metric;                  // 0 flat Cartesian; else (ln r, x2, phi) grids: Kerr, flat spherical
    double a_spin, h_slope, r_h;
    int *max_i1;                 // largest first-axis index of a zone holding plasma (-1: none)
    // electrons: 0 thermal; 1 power law, A = pl_aj n_e B, nu alpha = pl_aa n_e X^{-(p+2)/2}
    int dist;
    double pl_aj, pl_aa;
};

__global__ __launch_bounds__(256) void zone_prep_kernel(PrepArgs P)
{
    int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= P.nz) return;
    double ne = P.n_e[z], th = P.theta[z], B = P.B[z];
    double *r = P.zrec + (size_t)z * Z_STRIDE;
    double raw[16];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        raw[Z_U0 + m] = P.ucon[(size_t)m * P.nz + z];
        raw[Z_B0 + m] = P.bcon[(size_t)m * P.nz + z];
    }
    raw[Z_HASB] = (B > 0.0) ? 1.0 : 0.0;
    double sqrt_g = 1.0;
    bool inside = false;
    if (P.metric == 0) {
        // flat metric: normalise u and project/normalise the field direction once
        double g[4][4], u[4], bh[4];
        Minkowski::gcov(nullptr, g);
        bool has_b = fluid_frame(raw, g, u, bh);
#pragma unroll
        for (int m = 0; m < 4; ++m) { r[Z_U0 + m] = u[m]; r[Z_B0 + m] = bh[m]; }
        r[Z_HASB] = has_b ? 1.0 : 0.0;
    } else {
        // Kerr: u and the field direction are normalised with the metric at
        // each point of use; the volume uses sqrt(-g) at the zone centre and
        // zones centred inside the horizon do not emit
#pragma unroll
        for (int m = 0; m < 8; ++m) r[m] = raw[m];
        r[Z_HASB] = raw[Z_HASB];
        int i3 = z % P.n[2], i2 = (z / P.n[2]) % P.n[1], i1 = z / (P.n[2] * P.n[1]);
        double xc1 = P.xs[0] + (i1 + 0.5) * P.dx[0];
        double xc2 = P.xs[1] + (i2 + 0.5) * P.dx[1];
        (void)i3;
        sqrt_g = kerr_sqrt_neg_g(P.a_spin, P.h_slope, xc1, xc2);
        inside = exp(xc1) < P.r_h;
    }
    // power law: nu_c = 3 e B / (2 pi m c), and the absorption coefficient
    // A_a in the slot of 1/Theta (no Kirchhoff law for it)
    const bool pl = P.dist == 1;
    double A = pl ? ((ne > 0.0 && B > 0.0) ? P.pl_aj * ne * B : 0.0) : emis_coef(ne, th, B);
    double nuc = pl ? 3.0 * kE * B / (2.0 * kPi * kMe * kC) : nu_crit(th, B);
    r[Z_A] = A;
    r[Z_NUC] = nuc;
    r[Z_TH] = th;
    r[Z_NE] = ne;
    r[Z_LNTH] = th > 0.0 ? log(th) : 0.0;
    r[Z_INVTH] = pl ? P.pl_aa * ne : (th > 0.0 ? 1.0 / th : 0.0);
    r[Z_INVNUC] = nuc > 0.0 ? 1.0 / nuc : 0.0;
    P.vol[z] = sqrt_g * P.dx[0] * P.dx[1] * P.dx[2] * P.L3;
    P.emits[z] = (A > 0.0 && !inside) ? 1 : 0;
    if (ne > 0.0) atomicMax(P.max_i1, z / (P.n[2] * P.n[1]));
    // the FP32 record of the precision form
    float *f = P.zrec32 + (size_t)z * F_STRIDE;
#pragma unroll
    for (int m = 0; m < 8; ++m) f[m] = (float)r[m];
    f[F_LNA] = A > 0.0 ? (float)log(A) : -INFINITY;
    f[F_LNINVNUC] = nuc > 0.0 ? (float)(-log(nuc)) : 0.0f;
    f[F_TH] = (float)th;
    f[F_INVTH] = th > 0.0 ? (float)(1.0 / th) : 0.0f;
    f[F_LNTH] = th > 0.0 ? (float)log(th) : 0.0f;
    f[F_LNNESIG] = ne > 0.0 ? (float)log(ne * kSigT) : -INFINITY;
    f[F_HASB] = (float)r[Z_HASB];
    f[F_NE] = (float)ne;
}

// Validation of zone inputs that live in device memory (the host path runs
// the same tests on the host): finite n_e >= 0, B >= 0 and Theta_e; where
// n_e > 0, Theta_e > 0 and u^t > 0, and in Kerr a timelike u at the zone
// centre.  The smallest bad zone index is left in *first_bad.
struct CheckArgs {
    const double *n_e, *theta, *B, *ucon;
    int nz;
    int n[3];
    double xs[3], dx[3];
    int kerr;                    // (ln r, x2, phi) grid: Kerr or flat spherical
    double a_spin, mass, h_slope;
    int *first_bad;
};

__global__ __launch_bounds__(256) void zone_check_kernel(CheckArgs C)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.nz) return;
    double ne = C.n_e[i], th = C.theta[i], B = C.B[i];
    bool bad = !(ne >= 0.0) || !isfinite(ne) || !(B >= 0.0) || !isfinite(B) || !isfinite(th);
    if (!bad && ne > 0.0) {
        bad = !(th > 0.0) || !(C.ucon[i] > 0.0);
        if (!bad && C.kerr) {
            int i2 = (i / C.n[2]) % C.n[1], i1 = i / (C.n[2] * C.n[1]);
            KMetric K;
            kerr_metric<false>(C.a_spin, C.mass, C.h_slope, C.xs[0] + (i1 + 0.5) * C.dx[0],
                               C.xs[1] + (i2 + 0.5) * C.dx[1], K);
            double g[4][4], u[4];
            kerr_full(K, g);
#pragma unroll
            for (int m = 0; m < 4; ++m) u[m] = C.ucon[(size_t)m * C.nz + i];
            double uu = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) uu += g[m][n] * u[m] * u[n];
            bad = !(uu < 0.0);
        }
    }
    if (bad) atomicMin(C.first_bad, i);
}

// ---------------------------------------------------------------------------
// Weight table (Creation of superphotons section, eq:weight_calc):
//   w(nu_k) = Delta t Delta(ln nu) / (h N_s) sum_i V_i J_i(nu_k) + floor,
// Delta t = 1 s, Delta(ln nu) = ln(nu_max/nu_min).  Pass 1: per-block
// partial sums over 256 zones for every node; pass 2: each node sums its
// partials in block order (deterministic), then the floor and ln w.
// ---------------------------------------------------------------------------
struct EmitArgs {
    const double *zrec, *vol;
    const int *emits;
    const double *nu_nodes;      // [nw] node frequencies
    int nz, nw;
    GCheb G;
    Elec el;
    double *partial;             // [n_blocks][nw]
    int n_blocks;
    double *w_node, *ln_w;       // [nw]
    double span, n_target, w_floor_rel;
    double *nbar, *fmax;
    uint32_t *count;
    uint32_t key0, key1;
    int inst;
    int *status;
    // emission table (NULL: none): zone i emits with w_i(nu) = w(nu) e^{-m_i(ln nu)},
    // nodes uniform over [mt_lo, mt_hi]; ln nu of weight node k = lnnu_min + span k/(nw-1)
    const double *mtab;
    int mt_n;
    double mt_lo, mt_hi, lnnu_min;
};

GM_D double zone_J(const double *zr, double nu, const GCheb &G, const Elec &El)
{
    return 4.0 * kPi * zr[Z_A] * shape_G(El, G, nu / zr[Z_NUC]);
}

__global__ __launch_bounds__(256) void phi_partial_kernel(EmitArgs E)
{
    __shared__ double red[4];
    int z = blockIdx.x * 256 + threadIdx.x;
    bool on = (z < E.nz) && E.emits[z];
    const double *zr = E.zrec + (size_t)(on ? z : 0) * Z_STRIDE;
    double v = on ? E.vol[z] : 0.0;
    for (int k = 0; k < E.nw; ++k) {
        double val = on ? v * zone_J(zr, E.nu_nodes[k], E.G, E.el) : 0.0;
        for (int off = 32; off >= 1; off >>= 1) val += __shfl_down(val, off);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = val;
        __syncthreads();
        if (threadIdx.x == 0)
            E.partial[(size_t)blockIdx.x * E.nw + k] = ((red[0] + red[1]) + red[2]) + red[3];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void weight_table_kernel(EmitArgs E)
{
    __shared__ double red[256];
    double mx = 0.0;
    for (int k = threadIdx.x; k < E.nw; k += 256) {
        double phi = 0.0;
        for (int b = 0; b < E.n_blocks; ++b) phi += E.partial[(size_t)b * E.nw + k];
        double w = phi * E.span / (kH * E.n_target);
        E.w_node[k] = w;
        mx = fmax(mx, w);
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    double wmax = red[0];
    if (threadIdx.x == 0) *E.status = (wmax > 0.0) ? 0 : 1;
    if (!(wmax > 0.0)) return;
    for (int k = threadIdx.x; k < E.nw; k += 256) {
        double w = E.w_node[k] + E.w_floor_rel * wmax;
        E.w_node[k] = w;
        E.ln_w[k] = log(w);
    }
}

// Per zone (Sampling procedure section): dN/d ln nu = V J / (h w) at the
// nodes, its composite-Simpson integral n-bar, the rejection bound
// F_max = 1.02 max_k J/w, and the count floor(n-bar) + [u < frac(n-bar)]
// with u the first draw of the zone's stream (z, 0, instance<<8 | 2).
// Under an emission table the zone's weights are w e^{-m_i}: more, lighter
// superphotons where m_i > 0, with the same expected luminosity.
__global__ __launch_bounds__(256) void count_kernel(EmitArgs E)
{
    int z = blockIdx.x * 256 + threadIdx.x;
    if (z >= E.nz) return;
    double s = 0.0, fm = 0.0;
    if (E.emits[z]) {
        const double *zr = E.zrec + (size_t)z * Z_STRIDE;
        for (int k = 0; k < E.nw; ++k) {
            double wk_ = E.w_node[k];
            if (E.mtab)
                wk_ *= exp(-zone_table(E.mtab, E.mt_n, E.mt_lo, E.mt_hi, z,
                                       E.lnnu_min + E.span * k / (E.nw - 1)));
            double F = zone_J(zr, E.nu_nodes[k], E.G, E.el) / wk_;
            double wk = (k == 0 || k == E.nw - 1) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
            s += wk * F;
            fm = fmax(fm, F);
        }
    }
    double d = E.span / (E.nw - 1);
    double nb = E.vol[z] / kH * s * d / 3.0;
    E.nbar[z] = nb;
    E.fmax[z] = kFmaxMargin * fm;
    double fl = floor(nb);
    Rng r{(uint32_t)z, 0u, ((uint32_t)E.inst << 8) | 2u, 0u};
    double u = rng_uniform(r, E.key0, E.key1);
    E.count[z] = (uint32_t)fl + ((u < nb - fl) ? 1u : 0u);
}

// Stochastic rounding of the stored expected counts under a new seed (the
// weight table, expected counts and rejection bounds do not depend on it).
__global__ __launch_bounds__(256) void recount_kernel(EmitArgs E)
{
    int z = blockIdx.x * 256 + threadIdx.x;
    if (z >= E.nz) return;
    double nb = E.nbar[z];
    double fl = floor(nb);
    Rng r{(uint32_t)z, 0u, ((uint32_t)E.inst << 8) | 2u, 0u};
    double u = rng_uniform(r, E.key0, E.key1);
    E.count[z] = (uint32_t)fl + ((u < nb - fl) ? 1u : 0u);
}

// ---------------------------------------------------------------------------
// Exclusive scan of the zone counts into 64-bit photon offsets.
// ---------------------------------------------------------------------------
constexpr int kScanItems = 16;
constexpr int kScanTile = 256 * kScanItems;

__global__ __launch_bounds__(256) void scan_tiles_kernel(const uint32_t *cnt, int n,
                                                         unsigned long long *tile_sum)
{
    __shared__ unsigned long long red[256];
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    unsigned long long s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += cnt[base + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void scan_sums_kernel(unsigned long long *tile_sum, int ntiles,
                                                        unsigned long long *total)
{
    // one block: chunked serial scan over the tiles
    __shared__ unsigned long long part[256];
    int per = (ntiles + 255) / 256;
    int lo = threadIdx.x * per, hi = min(ntiles, lo + per);
    unsigned long long s = 0;
    for (int i = lo; i < hi; ++i) s += tile_sum[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long run = 0;
        for (int i = 0; i < 256; ++i) { unsigned long long t = part[i]; part[i] = run; run += t; }
        *total = run;
    }
    __syncthreads();
    unsigned long long run = part[threadIdx.x];
    for (int i = lo; i < hi; ++i) { unsigned long long t = tile_sum[i]; tile_sum[i] = run; run += t; }
}

__global__ __launch_bounds__(256) void scan_write_kernel(const uint32_t *cnt, int n,
                                                         const unsigned long long *tile_off,
                                                         unsigned long long *off)
{
    __shared__ unsigned long long part[256];
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    unsigned long long s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += cnt[base + i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long run = tile_off[blockIdx.x];
        for (int i = 0; i < 256; ++i) { unsigned long long t = part[i]; part[i] = run; run += t; }
    }
    __syncthreads();
    unsigned long long run = part[threadIdx.x];
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) { off[base + i] = run; run += cnt[base + i]; }
}

// Root photon p belongs to the last zone whose offset is <= p.
__global__ __launch_bounds__(256) void fill_zone_of_root_kernel(const unsigned long long *off, int nz,
                                                                unsigned long long n_roots,
                                                                uint32_t *zone_of_root)
{
    unsigned long long p = (unsigned long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= n_roots) return;
    int lo = 0, hi = nz;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= p) lo = mid; else hi = mid;
    }
    zone_of_root[p] = (uint32_t)lo;
}

// ---------------------------------------------------------------------------
// Hot cross-section table (Scattering section):
//   sigma_h = <(1 - beta mu) sigma_KN(gamma eps (1 - beta mu))>
// over isotropic thermal electrons.  One block per (Theta, eps) node.
// Outer: gamma = 1 + v^2 on v in [0, sqrt(740 Theta)] by composite 16-point
// Gauss-Legendre (64 panels); inner: in u = ln(1 - beta mu),
//   (1/(2 beta)) int_{ln(1-beta)}^{ln(1+beta)} e^{2u} sigma_KN(gamma eps e^u) du,
// by composite Gauss-Legendre (8 panels); normalisation by the same outer
// rule.  Entries are ln(sigma_h / sigma_T).
// ---------------------------------------------------------------------------
struct ShBuildArgs {
    const double *gl_x, *gl_w;   // 16-point Gauss-Legendre on [-1, 1]
    double *table;
    double lt0, dt, le0, de;
};

__global__ __launch_bounds__(256) void sigma_hot_build_kernel(ShBuildArgs S)
{
    __shared__ double rn[256], rd[256];
    int node = blockIdx.x;
    int it = node / kShNE, ie = node % kShNE;
    double theta = exp(S.lt0 + S.dt * it);
    double eps = exp(S.le0 + S.de * ie);
    const int NP_OUT = 64, NP_IN = 8, NG = 16;
    double V = sqrt(740.0 * theta);
    double hpan = V / NP_OUT;
    double num = 0.0, den = 0.0;
    for (int q = threadIdx.x; q < NP_OUT * NG; q += blockDim.x) {
        int pan = q / NG, gi = q % NG;
        double v = hpan * (pan + 0.5 + 0.5 * S.gl_x[gi]);
        double wv = 0.5 * hpan * S.gl_w[gi];
        double x = v * v;
        double gam = 1.0 + x;
        double mj = 2.0 * v * v * gam * sqrt(v * v + 2.0) * exp(-x / theta);
        if (mj == 0.0) continue;
        double beta = sqrt(x * (x + 2.0)) / gam;
        double ulo = log1p(-beta), uhi = log1p(beta);
        double hin = (uhi - ulo) / NP_IN;
        double inner = 0.0;
        for (int pi = 0; pi < NP_IN; ++pi)
            for (int gj = 0; gj < NG; ++gj) {
                double u = ulo + hin * (pi + 0.5 + 0.5 * S.gl_x[gj]);
                double eu = exp(u);
                inner += 0.5 * hin * S.gl_w[gj] * eu * eu * sigma_kn(gam * eps * eu);
            }
        inner /= (2.0 * beta);
        num += wv * mj * inner;
        den += wv * mj;
    }
    rn[threadIdx.x] = num;
    rd[threadIdx.x] = den;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) { rn[threadIdx.x] += rn[threadIdx.x + s]; rd[threadIdx.x] += rd[threadIdx.x + s]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) S.table[node] = log(rn[0] / rd[0]);
}

// ---------------------------------------------------------------------------
// Hot cross section of power-law electrons, gamma^-p on [g1, g2] (the
// Scattering section's average with the power law in place of the thermal
// distribution), one block per eps node of the thermal table: outer in
// ln gamma by composite 16-point Gauss-Legendre (64 panels), weight
// gamma^{1-p}; inner in u = ln(1 - beta mu) as for the thermal table;
// normalisation by the same outer rule.  Entries are ln(sigma / sigma_T).
// ---------------------------------------------------------------------------
struct PlBuildArgs {
    const double *gl_x, *gl_w;
    double *table;
    double le0, de;
    double p, lg1, lg2;
};

__global__ __launch_bounds__(256) void sigma_pl_build_kernel(PlBuildArgs S)
{
    __shared__ double rn[256], rd[256];
    const int ie = blockIdx.x;
    const double eps = exp(S.le0 + S.de * ie);
    const int NP_OUT = 64, NP_IN = 8, NG = 16;
    const double h = (S.lg2 - S.lg1) / NP_OUT;
    double num = 0.0, den = 0.0;
    for (int q = threadIdx.x; q < NP_OUT * NG; q += blockDim.x) {
        int pan = q / NG, gi = q % NG;
        double u = S.lg1 + h * (pan + 0.5 + 0.5 * S.gl_x[gi]);
        double wv = 0.5 * h * S.gl_w[gi];
        double gam = exp(u);
        double wt = exp((1.0 - S.p) * u);
        double beta = sqrt((gam - 1.0) * (gam + 1.0)) / gam;
        double ulo = log1p(-beta), uhi = log1p(beta);
        double hin = (uhi - ulo) / NP_IN;
        double inner = 0.0;
        for (int pi = 0; pi < NP_IN; ++pi)
            for (int gj = 0; gj < NG; ++gj) {
                double v = ulo + hin * (pi + 0.5 + 0.5 * S.gl_x[gj]);
                double ev = exp(v);
                inner += 0.5 * hin * S.gl_w[gj] * ev * ev * sigma_kn(gam * eps * ev);
            }
        inner /= (2.0 * beta);
        num += wv * wt * inner;
        den += wv * wt;
    }
    rn[threadIdx.x] = num;
    rd[threadIdx.x] = den;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) { rn[threadIdx.x] += rn[threadIdx.x + s]; rd[threadIdx.x] += rd[threadIdx.x + s]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) S.table[ie] = log(rn[0] / rd[0]);
}

__global__ void eval_G_kernel(GCheb G, const double *x, double *y, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = G_of_Xc(G, x[i]);
}

// FP32 copy of the hot cross-section table (ln sigma_h / sigma_T).
__global__ __launch_bounds__(256) void to_float_kernel(const double *src, float *dst, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

}  // namespace gm
