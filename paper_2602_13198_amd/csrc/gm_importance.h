// gm_importance.h -- per-zone tables of the importance-driven forms, built
// on the device (device side).
//
// A table holds, for every zone, n values on nodes uniform in a log
// variable v (bias table: ln eps of the incoming fluid-frame photon energy;
// emission table: ln nu of the emitted photon), v = ln eps + v_shift.  Its
// values come from an estimate ln I of the importance of a unit-weight
// photon created at (zone, eps), mapped by
//   kind 0:  T = a ln I + b + shift
//   kind 1:  T = ln((1 - alpha) + alpha exp(a ln I + b)) + shift   (defensive mixture)
// The estimate is either the network's output for the zone's features
// (matrix-core inference, features computed from the packed zone records)
// or a ratio of summed scores to summed weights of the event records that
// fall in a coarse spatial cell and a node.  Zones without plasma take a
// neutral value (they never scatter or emit).
#pragma once

#include "gm_kerr.h"
#include "gm_mlp.h"
#include "gm_track.h"

namespace gm {

struct ImpMap {
    int kind;
    double a, b, alpha, shift;
};

GM_D double imp_value(const ImpMap &m, double lnI)
{
    double t = m.a * lnI + m.b;
    if (m.kind == 1) t = log((1.0 - m.alpha) + m.alpha * exp(fmin(t, 700.0)));
    return t + m.shift;
}

// Geometry of a zone grid for the features and the cells.
struct ZoneGeo {
    int n[3];
    double xs[3], dx[3];
    int metric;
    double h_slope, half;
};

GM_D void zone_index3(const ZoneGeo &G, int z, int &i1, int &i2, int &i3)
{
    i3 = z % G.n[2];
    i2 = (z / G.n[2]) % G.n[1];
    i1 = z / (G.n[2] * G.n[1]);
}

// Features of a zone except the photon energy: ln Theta_e, ln n_e,
// ln(B + 1e-10 G) with B recovered from nu_c and Theta_e, the radius
// feature (Kerr: ln r of the centre; flat: |x| over the grid half-size) and
// cos theta of the centre.
GM_D void zone_feats(const double *zr, const ZoneGeo &G, int z, double f[6])
{
    const double th = zr[Z_TH], ne = zr[Z_NE], nuc = zr[Z_NUC];
    f[0] = log(fmax(th, 1e-3));
    f[1] = log(fmax(ne, 1e-300));
    // nu_c = (2/9) (e B / 2 pi m_e c) Theta^2
    const double B = th > 0.0 ? nuc * (9.0 * kPi * kMe * kC / kE) / (th * th) : 0.0;
    f[2] = log(B + 1e-10);
    int i1, i2, i3;
    zone_index3(G, z, i1, i2, i3);
    const double x1 = G.xs[0] + (i1 + 0.5) * G.dx[0];
    const double x2 = G.xs[1] + (i2 + 0.5) * G.dx[1];
    const double x3 = G.xs[2] + (i3 + 0.5) * G.dx[2];
    if (G.metric == 0) {
        const double rr = sqrt(x1 * x1 + x2 * x2 + x3 * x3);
        f[4] = rr / G.half;
        f[5] = rr > 0.0 ? x3 / rr : 0.0;
    } else {
        f[4] = x1;
        f[5] = cos(theta_of_x2(G.h_slope, x2));
    }
    f[3] = 0.0;
}

struct TableFill {
    const double *zrec;
    ZoneGeo G;
    int nz, n_nodes;
    double lo, hi, v_shift;        // nodes over [lo, hi] of v = ln eps + v_shift
    float mu[6], inv_sd[6];        // feature standardisation of the network
    int out_col;                   // network output used
    ImpMap map;
    double neutral;
    double *table;                 // [nz][n_nodes]
};

// One row per (zone, node): features standardised as in training, the
// network's forward pass on the matrix cores, the mapped value written to
// the table.  MlpArgs carries the parameters and the row count.
__global__ __launch_bounds__(64 * kMlpWaves) void mlp_table_kernel(MlpArgs M, TableFill T)
{
    __shared__ float lds[kMlpWaves][2][16 * kTileLd];
    const int w = threadIdx.x >> 6, l = lane_id();
    const long long r0 = ((long long)blockIdx.x * kMlpWaves + w) * 16;
    if (r0 >= M.n) return;                       // whole wave idle: no barrier below is block-wide
    // this lane's input row (layer 1 reads row r0 + l % 16)
    float f[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    {
        const long long r = r0 + (l & 15);
        if (r < M.n) {
            const int z = (int)(r / T.n_nodes), k = (int)(r % T.n_nodes);
            double fd[6];
            zone_feats(T.zrec + (size_t)z * Z_STRIDE, T.G, z, fd);
            fd[3] = T.lo + (T.hi - T.lo) * k / (T.n_nodes - 1) - T.v_shift;
#pragma unroll
            for (int m = 0; m < 6; ++m) f[m] = (float)((fd[m] - (double)T.mu[m]) * (double)T.inv_sd[m]);
        }
    }
    f32x4 y = mlp_tile_forward_f(M, r0, lds[w][0], lds[w][1], [&](long long, int k) {
        float v = 0.0f;
#pragma unroll
        for (int m = 0; m < 6; ++m) v = (k == m) ? f[m] : v;
        return v;
    });
    if ((l & 15) == T.out_col) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long r = r0 + 4 * (l >> 4) + j;
            if (r < M.n) {
                const int z = (int)(r / T.n_nodes);
                const bool on = T.zrec[(size_t)z * Z_STRIDE + Z_NE] > 0.0;
                T.table[r] = on ? imp_value(T.map, (double)y[j]) : T.neutral;
            }
        }
    }
}

// Cells of blocks b[0] x b[1] x b[2] zones.
struct CellArgs {
    ZoneGeo G;
    int b[3], nc[3];
    int n_nodes;
    double lo, hi, v_shift;
    int records;                   // 0: emission records (generation 0), 1: scattering records
    const EventRec *ev;
    unsigned long long n_ev;
    double *acc;                   // [n_cells][n_nodes][3]: summed score, summed weight, count
    // fill
    int nz;
    const double *zrec;
    double prior_w, ratio_all;     // shrinkage: prior weight (or records) and the overall ratio
    int per_photon;                // ratio over records instead of summed weight
    ImpMap map;
    double neutral;
    double *table;
};

GM_D int cell_of_zone(const CellArgs &C, int z)
{
    int i1, i2, i3;
    zone_index3(C.G, z, i1, i2, i3);
    return ((i1 / C.b[0]) * C.nc[1] + i2 / C.b[1]) * C.nc[2] + i3 / C.b[2];
}

GM_D int node_of(const CellArgs &C, double v)
{
    double p = (v - C.lo) / (C.hi - C.lo) * (C.n_nodes - 1);
    return (int)fmin(fmax(rint(p), 0.0), (double)(C.n_nodes - 1));
}

// Least and greatest eps of the event log's emission records (generation
// 0, positive weight): the bit patterns of positive doubles order like
// their values, so each wave reduces them as integers and its first lane
// merges them with one atomic min and one atomic max.
__global__ __launch_bounds__(256) void event_band_kernel(const EventRec *ev, unsigned long long n,
                                                         unsigned long long *mm)
{
    unsigned long long lo = ~0ull, hi = 0ull;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        const EventRec &r = ev[i];
        if (r.gen == 0 && r.w > 0.0 && r.eps > 0.0 && r.eps <= 1.7976931348623157e308) {
            const unsigned long long u = (unsigned long long)__double_as_longlong(r.eps);
            lo = min(lo, u);
            hi = max(hi, u);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, (unsigned long long)__shfl_xor(lo, o));
        hi = max(hi, (unsigned long long)__shfl_xor(hi, o));
    }
    if (lane_id() == 0) {
        atomicMin(&mm[0], lo);
        atomicMax(&mm[1], hi);
    }
}

__global__ __launch_bounds__(256) void cells_accumulate_kernel(CellArgs C)
{
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < C.n_ev;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        const EventRec &e = C.ev[i];
        const bool take = (C.records == 0) ? (e.gen == 0) : (e.gen > 0);
        if (!take || !(e.w > 0.0) || !(e.eps > 0.0) || e.zone < 0) continue;
        const int c = cell_of_zone(C, e.zone);
        const int k = node_of(C, log(e.eps) + C.v_shift);
        double *a = C.acc + ((size_t)c * C.n_nodes + k) * 3;
        atomicAdd(&a[0], e.score);
        atomicAdd(&a[1], e.w);
        atomicAdd(&a[2], 1.0);
    }
}

__global__ __launch_bounds__(256) void cells_fill_kernel(CellArgs C)
{
    const long long n = (long long)C.nz * C.n_nodes;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(r / C.n_nodes), k = (int)(r % C.n_nodes);
        if (!(C.zrec[(size_t)z * Z_STRIDE + Z_NE] > 0.0)) {
            C.table[r] = C.neutral;
            continue;
        }
        // the node's centre in v, and the cell node holding it
        const double v = C.lo + (C.hi - C.lo) * k / (C.n_nodes - 1);
        const double *a = C.acc + ((size_t)cell_of_zone(C, z) * C.n_nodes + node_of(C, v)) * 3;
        const double den = C.per_photon ? a[2] : a[1];
        const double ratio = a[2] > 0.0 ? (a[0] + C.prior_w * C.ratio_all) / (den + C.prior_w) : C.ratio_all;
        C.table[r] = imp_value(C.map, log(fmax(ratio, 1e-300)));
    }
}

// In-place mapping of a table's values, taken as ln I: t <- map(t) for every
// (zone, node) of a zone with plasma (the others keep their neutral value).
struct RemapArgs {
    const double *zrec;
    int nz, n_nodes;
    ImpMap map;
    double *table;
};

__global__ __launch_bounds__(256) void remap_table_kernel(RemapArgs R)
{
    const long long n = (long long)R.nz * R.n_nodes;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(r / R.n_nodes);
        if (R.zrec[(size_t)z * Z_STRIDE + Z_NE] > 0.0) R.table[r] = imp_value(R.map, R.table[r]);
    }
}

}  // namespace gm
