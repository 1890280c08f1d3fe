// gm_api.hip -- the C ABI of include/gm.h: context, device buffers, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gm.h"
#include "gm_bound.h"
#include "gm_emit.h"
#include "gm_host_tables.h"
#include "gm_importance.h"
#include "gm_mlp.h"
#include "gm_track.h"
#include "gm_track_ks.h"

using namespace gm;

static_assert(sizeof(TraceRec) == sizeof(gm_trace_rec), "trace record layout");
static_assert(sizeof(TraceRec) == 112, "trace record layout");
static_assert(sizeof(EventRec) == sizeof(gm_event_rec), "event record layout");
static_assert(kMlpParams == GM_MLP_PARAMS, "network parameter count");

// Scratch of the allocation-free gradient entry point (gm_mlp_grad_noalloc):
// the per-block partial gradients, kMlpParams + 1 floats for every block of
// kMlpGradRows rows.  Each GPU the library runs on holds one copy until the
// process ends; host code reaches it only through the address returned by
// hipGetSymbolAddress for that device.
constexpr size_t kScratchFloats = (size_t)8 << 20;                    // 32 MiB
constexpr long long kNoAllocMaxRows =
    (long long)(kScratchFloats / (gm::kMlpParams + 1)) * gm::kMlpGradRows;
static __device__ __align__(256) float scratch[kScratchFloats];
static_assert(kNoAllocMaxRows == GM_MLP_NOALLOC_MAX_ROWS, "row limit of the public header");

namespace {

thread_local std::string g_err = "";

gm_status fail(gm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(GM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));       \
    } while (0)

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t count)
    {
        if (count <= n && p) return hipSuccess;
        if (p) { (void)hipFree(p); p = nullptr; n = 0; }
        hipError_t e = hipMalloc((void **)&p, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) n = count;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

struct Instance {
    bool loaded = false, made = false;
    gm_grid grid{};
    int nz = 0;
    int max_i1 = -1;                           // last first-axis zone index holding plasma
    DevBuf<double> zrec, vol;
    DevBuf<float> zrec32;
    DevBuf<int> emits;
    // last make
    gm_emit_params ep{};
    int nw = 0;
    double lnnu_min = 0, lnnu_span = 0;
    DevBuf<double> nu_nodes, w_node, ln_w, nbar, fmax, partial;
    DevBuf<uint32_t> count, zone_of_root;
    DevBuf<unsigned long long> offset, tile;
    DevBuf<unsigned long long> roots;          // [0] n_roots, [1] root cursor
    unsigned long long n_roots = 0;
    bool pending = false;                      // roots made, not yet tracked
    bool dirty = false;                        // tally holds data since the last reset
    // tallies
    int n_nu = 0, n_theta = 0;
    DevBuf<double> spec, ledger;
    DevBuf<unsigned long long> stats;
    // per-instance bias overriding the track call's (bias_mode < 0: none)
    int bias_mode = -1;
    double bias_value = 0.0, bias_max = 0.0;
    // bias table [nz][lnb_n] (ln b, or ln of the weight-window factor)
    DevBuf<double> lnb;
    int lnb_n = 0;
    double lnb_lo = 0.0, lnb_hi = 0.0;
    // emission table [nz][mt_n] (NULL: none); a new table invalidates the
    // stored expected counts
    DevBuf<double> mtab;
    int mt_n = 0;
    double mt_lo = 0.0, mt_hi = 0.0;
    bool mt_on = false;
    // score weights [n_theta][n_nu] of the event records (none: 1)
    DevBuf<double> sw;
    int sw_n = 0;
    // electrons; the power law's hot cross-section table, built on first use
    gm_electrons el{};
    DevBuf<double> sigpl;
    bool sigpl_built = false;
};

}  // namespace

struct gm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 0;
    Instance inst[GM_MAX_INSTANCES];
    // tables
    DevBuf<double> gcheb, sh_table, gl_x, gl_w;
    DevBuf<float> sh_table32;
    GCheb G{};
    ShTable sh{};
    ShTable32 sh32{};
    bool sh_built = false;
    // photon queues (ping-pong between generations) and per-generation counters
    unsigned long long child_cap = 0;           // allocated entries per queue
    unsigned long long queue_cap = 0;           // entries in use (<= child_cap)
    unsigned long long queue_cap_set = 0;       // fixed by gm_set_queue_capacity, 0 = automatic
    // accumulators of the instances of a root chunk, kept to redo the chunk
    DevBuf<double> bak_d, call_bak_d;
    DevBuf<unsigned long long> bak_u, call_bak_u;
    unsigned long long chunk_retries = 0;
    DevBuf<double> qd[2][13];
    DevBuf<uint32_t> qu[2][5];
    DevBuf<int32_t> qi[2][3];
    DevBuf<unsigned long long> ctr;             // [gen][2]: count, cursor
    DevBuf<int> flags;                          // [0] overflow, [1] status
    // tuning of the tracking launch (waves per SIMD of the compiled variant,
    // idle lanes before a wave claims new photons, instances per launch)
    int track_waves = 2;
    int refill_min = 8;
    int max_batch = GM_MAX_INSTANCES;
    DevBuf<TArgs> inst_args;
    DevBuf<unsigned long long> root_off, inst_ctr;
    // HIP graph of a chunk's launch sequence (captured on a private stream,
    // launched on the context's stream; the executable graph is updated in
    // place while only kernel arguments change)
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    unsigned long long graph_launches = 0, graph_instantiations = 0;
    // optional event timing of the tracking launches
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    double track_ms = 0.0;
    unsigned long long track_launches = 0;
    // trace and scattering-event log
    TraceRec *trace = nullptr;
    unsigned long long trace_cap = 0;
    DevBuf<unsigned long long> trace_n;
    EventRec *evlog = nullptr;
    unsigned long long evlog_cap = 0, root_stride = 0;
    DevBuf<unsigned long long> evlog_n;
    // tallies of a shared launch: 0 automatic (LDS when they fit), 1 LDS, 2 HBM
    int tally_mode = 0;
    // learned form: network parameters (FP32 master, BF16 copies), Adam state
    DevBuf<float> mlp_p, mlp_m, mlp_v, mlp_g, mlp_gpart;
    DevBuf<short> mlp_pb;
    bool mlp_ready = false;
    long long mlp_t = 0;
    int mlp_loss = 0;
    float *scratch = nullptr;                   // this device's copy of the scratch array
    // cell sums of the event records (adaptive form) and their layout
    DevBuf<double> cell_acc;
    DevBuf<unsigned long long> band_mm;
    gm_importance_map cell_map{};
    int cell_blocks[3] = {0, 0, 0}, cell_nc[3] = {0, 0, 0};
    int cell_inst = -1;
    double cell_tot[3] = {0.0, 0.0, 0.0};
};

static gm_status set_device(gm_ctx *c)
{
    HIPCHK(hipSetDevice(c->device));
    return GM_OK;
}

// Device address of the scratch array on the current device `device`,
// looked up once per device.
static gm_status scratch_address(int device, float **out)
{
    static std::mutex mu;
    static float *addr[256] = {};
    if (device < 0 || device >= 256) return fail(GM_EINVAL, "device %d", device);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GM_EDEVICE, "scratch address on device %d: %s", device, hipGetErrorString(e));
        addr[device] = (float *)p;
    }
    *out = addr[device];
    return GM_OK;
}

static gm_status build_tables(gm_ctx *c)
{
    host::GChebHost T = host::build_G_cheb();
    HIPCHK(c->gcheb.ensure(T.coef.size()));
    HIPCHK(hipMemcpy(c->gcheb.p, T.coef.data(), T.coef.size() * sizeof(double), hipMemcpyHostToDevice));
    c->G.coef = c->gcheb.p;
    c->G.t_lo = T.t_lo;
    c->G.t_hi = T.t_hi;
    c->G.inv_h = 1.0 / T.h;
    c->G.ln_c0 = T.ln_c0;
    c->G.n_pieces = T.n_pieces;
    c->G.deg = T.deg;
    std::vector<double> x, w;
    host::gauss_legendre(16, x, w);
    HIPCHK(c->gl_x.ensure(16));
    HIPCHK(c->gl_w.ensure(16));
    HIPCHK(hipMemcpy(c->gl_x.p, x.data(), 16 * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->gl_w.p, w.data(), 16 * sizeof(double), hipMemcpyHostToDevice));
    return GM_OK;
}

// Electron descriptor of an instance for the kernels.
static Elec elec_of(const Instance &I)
{
    Elec E{};
    E.kind = I.el.kind;
    if (E.kind == GM_DIST_POWERLAW) {
        const double p = I.el.p;
        E.p = p;
        E.ga = std::pow(I.el.gamma_min, 1.0 - p);
        E.gb = std::pow(I.el.gamma_max, 1.0 - p);
        E.inv1mp = 1.0 / (1.0 - p);
        E.eg = -0.5 * (p - 1.0);
        E.ea = -0.5 * (p + 2.0);
        E.ang = 0.5 * std::sqrt(kPi) * std::tgamma(0.25 * (p + 5.0)) / std::tgamma(0.25 * (p + 7.0));
        E.sig = I.sigpl.p;
        E.le0 = std::log(kShEMin);
        E.inv_de = (kShNE - 1) / (std::log(kShEMax) - std::log(kShEMin));
    }
    return E;
}

static bool same_electrons(const gm_electrons &a, const gm_electrons &b)
{
    return a.kind == b.kind && (a.kind == GM_DIST_THERMAL ||
                                (a.p == b.p && a.gamma_min == b.gamma_min && a.gamma_max == b.gamma_max));
}

// The power law's hot cross section of an instance (its eps nodes those of
// the thermal table).
static gm_status ensure_sigma_pl(gm_ctx *c, Instance &I)
{
    if (I.sigpl_built) return GM_OK;
    HIPCHK(I.sigpl.ensure(kShNE));
    PlBuildArgs S;
    S.gl_x = c->gl_x.p;
    S.gl_w = c->gl_w.p;
    S.table = I.sigpl.p;
    S.le0 = std::log(kShEMin);
    S.de = (std::log(kShEMax) - std::log(kShEMin)) / (kShNE - 1);
    S.p = I.el.p;
    S.lg1 = std::log(I.el.gamma_min);
    S.lg2 = std::log(I.el.gamma_max);
    sigma_pl_build_kernel<<<kShNE, 256, 0, c->stream>>>(S);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    I.sigpl_built = true;
    return GM_OK;
}

static gm_status ensure_sigma_hot(gm_ctx *c)
{
    if (c->sh_built) return GM_OK;
    HIPCHK(c->sh_table.ensure(kShNT * kShNE));
    ShBuildArgs S;
    S.gl_x = c->gl_x.p;
    S.gl_w = c->gl_w.p;
    S.table = c->sh_table.p;
    S.lt0 = std::log(kShThMin);
    S.dt = (std::log(kShThMax) - std::log(kShThMin)) / (kShNT - 1);
    S.le0 = std::log(kShEMin);
    S.de = (std::log(kShEMax) - std::log(kShEMin)) / (kShNE - 1);
    sigma_hot_build_kernel<<<kShNT * kShNE, 256, 0, c->stream>>>(S);
    HIPCHK(hipGetLastError());
    HIPCHK(c->sh_table32.ensure(kShNT * kShNE));
    to_float_kernel<<<(kShNT * kShNE + 255) / 256, 256, 0, c->stream>>>(c->sh_table.p, c->sh_table32.p, kShNT * kShNE);
    HIPCHK(hipGetLastError());
    c->sh32.t = c->sh_table32.p;
    c->sh32.lt0 = (float)S.lt0;
    c->sh32.inv_dt = (float)(1.0 / S.dt);
    c->sh32.le0 = (float)S.le0;
    c->sh32.inv_de = (float)(1.0 / S.de);
    c->sh.t = c->sh_table.p;
    c->sh.lt0 = S.lt0;
    c->sh.inv_dt = 1.0 / S.dt;
    c->sh.le0 = S.le0;
    c->sh.inv_de = 1.0 / S.de;
    c->sh_built = true;
    return GM_OK;
}

extern "C" {

const char *gm_last_error(void) { return g_err.c_str(); }

gm_status gm_create(gm_ctx **out, int device, void *hip_stream)
{
    if (!out) return fail(GM_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(GM_EINVAL, "device %d of %d", device, ndev);
    gm_ctx *c = new gm_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    gm_status s = set_device(c);
    if (s != GM_OK) { delete c; return s; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete c; return fail(GM_EDEVICE, "device properties"); }
    c->n_cu = prop.multiProcessorCount;
    s = scratch_address(device, &c->scratch);
    if (s != GM_OK) { delete c; return s; }
    s = build_tables(c);
    if (s == GM_OK && (c->ctr.ensure(2 * 32) != hipSuccess || c->flags.ensure(4) != hipSuccess ||
                       c->trace_n.ensure(1) != hipSuccess || c->evlog_n.ensure(1) != hipSuccess))
        s = fail(GM_ENOMEM, "counters");
    if (s != GM_OK) { gm_destroy(c); return s; }
    *out = c;
    return GM_OK;
}

gm_status gm_destroy(gm_ctx *c)
{
    if (!c) return GM_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
    for (auto &I : c->inst) {
        I.zrec.release(); I.zrec32.release(); I.vol.release(); I.emits.release(); I.nu_nodes.release();
        I.w_node.release(); I.ln_w.release(); I.nbar.release(); I.fmax.release();
        I.partial.release(); I.count.release(); I.zone_of_root.release(); I.offset.release();
        I.tile.release(); I.roots.release(); I.spec.release(); I.ledger.release(); I.stats.release();
        I.lnb.release(); I.mtab.release(); I.sw.release();
    }
    c->inst_args.release(); c->root_off.release(); c->inst_ctr.release();
    c->bak_d.release(); c->bak_u.release(); c->call_bak_d.release(); c->call_bak_u.release();
    c->cell_acc.release();
    c->band_mm.release();
    c->mlp_p.release(); c->mlp_m.release(); c->mlp_v.release(); c->mlp_g.release();
    c->mlp_gpart.release(); c->mlp_pb.release(); c->evlog_n.release();
    c->gcheb.release(); c->sh_table.release(); c->sh_table32.release(); c->gl_x.release(); c->gl_w.release();
    for (int b = 0; b < 2; ++b) {
        for (auto &d : c->qd[b]) d.release();
        for (auto &d : c->qu[b]) d.release();
        for (auto &d : c->qi[b]) d.release();
    }
    c->ctr.release(); c->flags.release(); c->trace_n.release();
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto &pr : c->ev_pending) { c->ev_pool.push_back(pr.first); c->ev_pool.push_back(pr.second); }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
    return GM_OK;
}

// Mass of the Kerr-Schild form a grid uses: 1 for Kerr, 0 for flat spherical.
static double metric_mass(int metric) { return metric == GM_METRIC_KS_MKS ? 1.0 : 0.0; }

gm_status gm_load_zones(gm_ctx *c, int instance, const gm_grid *g, const gm_zones *z)
{
    if (!c || !g || !z) return fail(GM_EINVAL, "NULL argument");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    if (g->metric != GM_METRIC_MINKOWSKI_CART && g->metric != GM_METRIC_KS_MKS && g->metric != GM_METRIC_FLAT_SPH)
        return fail(GM_EINVAL, "unknown metric %d", g->metric);
    if (g->metric == GM_METRIC_FLAT_SPH && g->a_spin != 0.0)
        return fail(GM_EINVAL, "the flat spherical grid takes a_spin = 0");
    for (int j = 0; j < 3; ++j)
        if (g->n[j] < 1 || !(g->dx[j] > 0.0) || !std::isfinite(g->x_start[j]))
            return fail(GM_EINVAL, "grid axis %d", j);
    if (!(g->L_unit_cm > 0.0)) return fail(GM_EINVAL, "L_unit_cm must be > 0");
    const bool kerr = g->metric != GM_METRIC_MINKOWSKI_CART;     // (ln r, x2, phi) grid
    const double mass = metric_mass(g->metric);
    if (kerr) {
        if (!(std::fabs(g->a_spin) < 1.0)) return fail(GM_EINVAL, "spin |a| must be < 1");
        if (!(g->h_slope > 0.0 && g->h_slope <= 1.0)) return fail(GM_EINVAL, "h_slope must be in (0, 1]");
        if (g->x_start[1] < 0.0 || g->x_start[1] + g->n[1] * g->dx[1] > 1.0 + 1e-12)
            return fail(GM_EINVAL, "x2 range must lie in [0, 1]");
        if (!(g->r_record > std::exp(g->x_start[0])))
            return fail(GM_EINVAL, "r_record must exceed the inner radius");
    }
    long long nzl = (long long)g->n[0] * g->n[1] * g->n[2];
    if (nzl > (1ll << 31) - 1) return fail(GM_EINVAL, "too many zones");
    int nz = (int)nzl;
    if (!z->n_e || !z->theta_e || !z->B || !z->ucon || !z->bcon) return fail(GM_EINVAL, "zone array NULL");
    const gm_electrons &el = z->electrons;
    if (el.kind != GM_DIST_THERMAL &&
        !(el.kind == GM_DIST_POWERLAW && el.p > 1.0 && el.gamma_min >= 1.0 && el.gamma_max > el.gamma_min &&
          std::isfinite(el.gamma_max)))
        return fail(GM_EINVAL, "bad electron distribution");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    // stage inputs on the device
    const double *src[5] = {z->n_e, z->theta_e, z->B, z->ucon, z->bcon};
    size_t cnt[5] = {(size_t)nz, (size_t)nz, (size_t)nz, 4 * (size_t)nz, 4 * (size_t)nz};
    if (!z->on_device) {
        // validate on the host before anything changes
        for (int i = 0; i < nz; ++i) {
            double ne = z->n_e[i], th = z->theta_e[i], B = z->B[i];
            if (!(ne >= 0.0) || !std::isfinite(ne) || !(B >= 0.0) || !std::isfinite(B) || !std::isfinite(th))
                return fail(GM_EINVAL, "zone %d: bad n_e/B/theta", i);
            if (ne > 0.0 && !(th > 0.0)) return fail(GM_EINVAL, "zone %d: n_e > 0 needs theta_e > 0", i);
            if (ne > 0.0 && !(z->ucon[i] > 0.0)) return fail(GM_EINVAL, "zone %d: u^t must be > 0", i);
            if (ne > 0.0 && kerr) {
                // the fluid velocity must be timelike at the zone centre
                int i2 = (i / g->n[2]) % g->n[1], i1 = i / (g->n[2] * g->n[1]);
                KMetric K;
                kerr_metric<false>(g->a_spin, mass, g->h_slope, g->x_start[0] + (i1 + 0.5) * g->dx[0],
                                   g->x_start[1] + (i2 + 0.5) * g->dx[1], K);
                double gm4[4][4], u[4];
                kerr_full(K, gm4);
                for (int m = 0; m < 4; ++m) u[m] = z->ucon[(size_t)m * nz + i];
                double uu = 0.0;
                for (int m = 0; m < 4; ++m)
                    for (int n = 0; n < 4; ++n) uu += gm4[m][n] * u[m] * u[n];
                if (!(uu < 0.0)) return fail(GM_EINVAL, "zone %d: u is not timelike", i);
            }
        }
    }
    if (z->on_device) {
        // validate on the device before anything changes
        CheckArgs V;
        V.n_e = z->n_e; V.theta = z->theta_e; V.B = z->B; V.ucon = z->ucon; V.nz = nz;
        for (int j = 0; j < 3; ++j) { V.n[j] = g->n[j]; V.xs[j] = g->x_start[j]; V.dx[j] = g->dx[j]; }
        V.kerr = kerr ? 1 : 0;
        V.a_spin = g->a_spin;
        V.mass = mass;
        V.h_slope = g->h_slope;
        V.first_bad = c->flags.p + 2;
        int first = INT_MAX;
        HIPCHK(hipMemcpyAsync(V.first_bad, &first, sizeof(int), hipMemcpyHostToDevice, c->stream));
        zone_check_kernel<<<(nz + 255) / 256, 256, 0, c->stream>>>(V);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&first, V.first_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (first != INT_MAX) return fail(GM_EINVAL, "zone %d: bad n_e/B/theta/u (device input)", first);
    }
    Instance &I = c->inst[instance];
    DevBuf<double> stage[5];
    const double *dsrc[5];
    for (int k = 0; k < 5; ++k) {
        if (z->on_device) { dsrc[k] = src[k]; continue; }
        if (stage[k].ensure(cnt[k]) != hipSuccess) {
            for (auto &b : stage) b.release();
            return fail(GM_ENOMEM, "zone staging");
        }
        if (hipMemcpyAsync(stage[k].p, src[k], cnt[k] * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess) {
            for (auto &b : stage) b.release();
            return fail(GM_EDEVICE, "zone upload");
        }
        dsrc[k] = stage[k].p;
    }
    if (I.zrec.ensure((size_t)nz * Z_STRIDE) != hipSuccess || I.zrec32.ensure((size_t)nz * F_STRIDE) != hipSuccess ||
        I.vol.ensure(nz) != hipSuccess || I.emits.ensure(nz) != hipSuccess) {
        for (auto &b : stage) b.release();
        return fail(GM_ENOMEM, "zone records");
    }
    PrepArgs P;
    P.n_e = dsrc[0]; P.theta = dsrc[1]; P.B = dsrc[2]; P.ucon = dsrc[3]; P.bcon = dsrc[4];
    P.zrec = I.zrec.p; P.zrec32 = I.zrec32.p; P.vol = I.vol.p; P.emits = I.emits.p;
    for (int j = 0; j < 3; ++j) { P.n[j] = g->n[j]; P.xs[j] = g->x_start[j]; P.dx[j] = g->dx[j]; }
    P.L3 = g->L_unit_cm * g->L_unit_cm * g->L_unit_cm;
    P.nz = nz;
    P.metric = g->metric;
    P.a_spin = g->a_spin;
    P.h_slope = g->h_slope;
    P.r_h = kerr_horizon(g->a_spin, mass);
    P.dist = el.kind;
    P.pl_aj = P.pl_aa = 0.0;
    if (el.kind == GM_DIST_POWERLAW) {
        const double p = el.p;
        const double C = (p - 1.0) / (std::pow(el.gamma_min, 1.0 - p) - std::pow(el.gamma_max, 1.0 - p));
        P.pl_aj = std::sqrt(3.0) * kE * kE * kE * C * std::tgamma((3.0 * p + 19.0) / 12.0) *
                  std::tgamma((3.0 * p - 1.0) / 12.0) / (4.0 * kPi * kMe * kC * kC * (p + 1.0));
        P.pl_aa = std::sqrt(3.0) * kE * kE * C * std::tgamma((3.0 * p + 2.0) / 12.0) *
                  std::tgamma((3.0 * p + 22.0) / 12.0) / (12.0 * kMe * kC);
    }
    P.max_i1 = c->flags.p + 3;
    int max_i1 = -1;
    HIPCHK(hipMemcpyAsync(P.max_i1, &max_i1, sizeof(int), hipMemcpyHostToDevice, c->stream));
    zone_prep_kernel<<<(nz + 255) / 256, 256, 0, c->stream>>>(P);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&max_i1, P.max_i1, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    hipError_t e2 = hipStreamSynchronize(c->stream);     // staging buffers are freed next
    for (auto &b : stage) b.release();
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(GM_EDEVICE, "zone prep: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    I.grid = *g;
    I.nz = nz;
    I.max_i1 = max_i1;
    if (!same_electrons(I.el, el)) I.sigpl_built = false;
    I.el = el;
    I.loaded = true;
    I.made = false;
    I.pending = false;
    return GM_OK;
}

gm_status gm_unload_zones(gm_ctx *c, int instance)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    HIPCHK(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    Instance &I = c->inst[instance];
    I.zrec.release(); I.zrec32.release(); I.vol.release(); I.emits.release(); I.nu_nodes.release();
    I.w_node.release(); I.ln_w.release(); I.nbar.release(); I.fmax.release();
    I.partial.release(); I.count.release(); I.zone_of_root.release(); I.offset.release();
    I.tile.release(); I.roots.release(); I.spec.release(); I.ledger.release(); I.stats.release();
    I.lnb.release(); I.mtab.release(); I.sw.release();
    I = Instance();
    return GM_OK;
}

static gm_status make_one(gm_ctx *c, int instance, const gm_emit_params *p, uint64_t *n_made,
                          double *expected = nullptr)
{
    Instance &I = c->inst[instance];
    if (!I.loaded) return fail(GM_ESTATE, "instance %d has no zones", instance);
    const int nz = I.nz, nw = p->n_wnodes;
    const int nblk = (nz + 255) / 256;
    if (I.nu_nodes.ensure(nw) != hipSuccess || I.w_node.ensure(nw) != hipSuccess ||
        I.ln_w.ensure(nw) != hipSuccess || I.nbar.ensure(nz) != hipSuccess ||
        I.fmax.ensure(nz) != hipSuccess || I.count.ensure(nz) != hipSuccess ||
        I.offset.ensure((size_t)nz + 1) != hipSuccess || I.partial.ensure((size_t)nblk * nw) != hipSuccess ||
        I.tile.ensure((size_t)nz / kScanTile + 2) != hipSuccess || I.roots.ensure(2) != hipSuccess)
        return fail(GM_ENOMEM, "emission buffers");
    const double lnmin = std::log(p->nu_min), span = std::log(p->nu_max / p->nu_min);
    // the weight table, expected counts and rejection bounds depend on the
    // zones and on everything in the parameters but the seed: reuse them
    const bool reuse = I.made && I.ep.n_target == p->n_target && I.ep.nu_min == p->nu_min &&
                       I.ep.nu_max == p->nu_max && I.ep.n_wnodes == p->n_wnodes &&
                       I.ep.w_floor_rel == p->w_floor_rel;   // (a new emission table clears made)
    if (!reuse) {
        std::vector<double> nus(nw);
        for (int k = 0; k < nw; ++k) nus[k] = std::exp(lnmin + span * k / (nw - 1));
        HIPCHK(hipMemcpyAsync(I.nu_nodes.p, nus.data(), nw * sizeof(double), hipMemcpyHostToDevice, c->stream));
    }
    EmitArgs E;
    E.zrec = I.zrec.p; E.vol = I.vol.p; E.emits = I.emits.p; E.nu_nodes = I.nu_nodes.p;
    E.nz = nz; E.nw = nw; E.G = c->G; E.el = elec_of(I); E.partial = I.partial.p; E.n_blocks = nblk;
    E.w_node = I.w_node.p; E.ln_w = I.ln_w.p; E.span = span; E.n_target = p->n_target;
    E.w_floor_rel = p->w_floor_rel; E.nbar = I.nbar.p; E.fmax = I.fmax.p; E.count = I.count.p;
    E.key0 = (uint32_t)p->seed; E.key1 = (uint32_t)(p->seed >> 32); E.inst = instance;
    E.status = c->flags.p + 1;
    E.mtab = I.mt_on ? I.mtab.p : nullptr;
    E.mt_n = I.mt_n;
    E.mt_lo = I.mt_lo;
    E.mt_hi = I.mt_hi;
    E.lnnu_min = lnmin;
    if (reuse) {
        recount_kernel<<<nblk, 256, 0, c->stream>>>(E);
    } else {
        I.made = false;          // until this make succeeds, nothing is reusable
        phi_partial_kernel<<<nblk, 256, 0, c->stream>>>(E);
        weight_table_kernel<<<1, 256, 0, c->stream>>>(E);
        count_kernel<<<nblk, 256, 0, c->stream>>>(E);
    }
    if (expected) {
        // expected roots only: no draw, no root table
        std::vector<double> nb(nz);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(nb.data(), I.nbar.p, (size_t)nz * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        int status = 0;
        HIPCHK(hipMemcpyAsync(&status, c->flags.p + 1, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        I.made = false;
        if (status != 0) return fail(GM_EINVAL, "no zone emits in the band [%g, %g] Hz", p->nu_min, p->nu_max);
        double t = 0.0;
        for (double v : nb) t += v;
        *expected = t;
        return GM_OK;
    }
    const int ntile = (nz + kScanTile - 1) / kScanTile;
    scan_tiles_kernel<<<ntile, 256, 0, c->stream>>>(I.count.p, nz, I.tile.p);
    scan_sums_kernel<<<1, 256, 0, c->stream>>>(I.tile.p, ntile, I.offset.p + nz);
    scan_write_kernel<<<ntile, 256, 0, c->stream>>>(I.count.p, nz, I.tile.p, I.offset.p);
    HIPCHK(hipGetLastError());
    int status = 0;
    unsigned long long total = 0;
    HIPCHK(hipMemcpyAsync(&status, c->flags.p + 1, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&total, I.offset.p + nz, sizeof(total), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (status != 0) return fail(GM_EINVAL, "no zone emits in the band [%g, %g] Hz", p->nu_min, p->nu_max);
    if (total > 0) {
        if (I.zone_of_root.ensure(total) != hipSuccess) return fail(GM_ENOMEM, "root table (%llu)", total);
        unsigned long long nb = (total + 255) / 256;
        fill_zone_of_root_kernel<<<(unsigned)nb, 256, 0, c->stream>>>(I.offset.p, nz, total, I.zone_of_root.p);
        HIPCHK(hipGetLastError());
    }
    unsigned long long rc[2] = {total, 0ull};
    HIPCHK(hipMemcpyAsync(I.roots.p, rc, sizeof(rc), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    I.ep = *p;
    I.nw = nw;
    I.lnnu_min = lnmin;
    I.lnnu_span = span;
    I.n_roots = total;
    I.made = true;
    I.pending = true;
    if (n_made) *n_made = total;
    return GM_OK;
}

gm_status gm_expected_roots(gm_ctx *c, int instance, const gm_emit_params *p, double *expected)
{
    if (!c || !p || !expected) return fail(GM_EINVAL, "NULL argument");
    if (!(p->nu_min > 0.0) || !(p->nu_max > p->nu_min) || p->n_wnodes < 3 || p->n_wnodes > 4097 ||
        !(p->n_wnodes & 1) || !(p->n_target > 0.0) || !(p->w_floor_rel >= 0.0))
        return fail(GM_EINVAL, "bad emission parameters");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    return make_one(c, instance, p, nullptr, expected);
}

gm_status gm_make_superphotons(gm_ctx *c, int instance, const gm_emit_params *p, uint64_t *n_made)
{
    if (!c || !p) return fail(GM_EINVAL, "NULL argument");
    if (!(p->nu_min > 0.0) || !(p->nu_max > p->nu_min) || p->n_wnodes < 3 || p->n_wnodes > 4097 ||
        !(p->n_wnodes & 1) || !(p->n_target > 0.0) || !(p->w_floor_rel >= 0.0))
        return fail(GM_EINVAL, "bad emission parameters");
    if (instance < -1 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    if (instance >= 0) return make_one(c, instance, p, n_made);
    bool any = false;
    for (int i = 0; i < GM_MAX_INSTANCES; ++i)
        if (c->inst[i].loaded) {
            any = true;
            s = make_one(c, i, p, n_made);
            if (s != GM_OK) return s;
        }
    return any ? GM_OK : fail(GM_ESTATE, "no instance loaded");
}

static gm_status ensure_children(gm_ctx *c, unsigned long long cap)
{
    c->queue_cap = cap;
    if (c->child_cap >= cap) return GM_OK;
    for (int b = 0; b < 2; ++b) {
        for (auto &d : c->qd[b])
            if (d.ensure(cap) != hipSuccess) return fail(GM_ENOMEM, "photon queue of %llu", cap);
        for (auto &d : c->qu[b])
            if (d.ensure(cap) != hipSuccess) return fail(GM_ENOMEM, "photon queue of %llu", cap);
        for (auto &d : c->qi[b])
            if (d.ensure(cap) != hipSuccess) return fail(GM_ENOMEM, "photon queue of %llu", cap);
    }
    c->child_cap = cap;
    return GM_OK;
}

static PhotonQ queue(gm_ctx *c, int b)
{
    PhotonQ q;
    for (int m = 0; m < 3; ++m) q.x[m] = c->qd[b][m].p;
    for (int m = 0; m < 4; ++m) q.k[m] = c->qd[b][3 + m].p;
    q.w = c->qd[b][7].p; q.wb = c->qd[b][8].p; q.x1 = c->qd[b][9].p;
    q.nua = c->qd[b][10].p; q.nus = c->qd[b][11].p; q.b = c->qd[b][12].p;
    q.s0 = c->qu[b][0].p; q.s1 = c->qu[b][1].p; q.s2 = c->qu[b][2].p; q.blk = c->qu[b][3].p;
    q.ev = c->qu[b][4].p;
    q.n_sc = c->qi[b][0].p; q.zone = c->qi[b][1].p; q.inst = c->qi[b][2].p;
    return q;
}

static gm_status take_event_pair(gm_ctx *c, hipEvent_t &a, hipEvent_t &b)
{
    for (int i = 0; i < 2; ++i) {
        hipEvent_t e;
        if (!c->ev_pool.empty()) {
            e = c->ev_pool.back();
            c->ev_pool.pop_back();
        } else {
            HIPCHK(hipEventCreate(&e));
        }
        (i == 0 ? a : b) = e;
    }
    c->ev_pending.emplace_back(a, b);
    return GM_OK;
}

// Fold finished event pairs into the running totals (synchronises on them).
static gm_status drain_events(gm_ctx *c)
{
    for (auto &pr : c->ev_pending) {
        HIPCHK(hipEventSynchronize(pr.second));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
        c->track_ms += ms;
        c->track_launches += 1;
        c->ev_pool.push_back(pr.first);
        c->ev_pool.push_back(pr.second);
    }
    c->ev_pending.clear();
    return GM_OK;
}

__global__ void reset_counters_kernel(unsigned long long *ctr, int n, int *overflow)
{
    int i = threadIdx.x;
    if (i < n) ctr[i] = 0ull;
    if (i == 0 && overflow) *overflow = 0;
}

// Tally buffers of an instance for a track call (allocated or reshaped when
// needed; stats cleared).
static gm_status prepare_instance(gm_ctx *c, Instance &I, const gm_track_params *tp)
{
    const size_t nspec = (size_t)tp->n_theta * tp->n_nu * 3;
    const bool reshape = I.spec.p && (I.n_nu != tp->n_nu || I.n_theta != tp->n_theta);
    if (reshape && I.dirty) return fail(GM_EINVAL, "tally shape changed without a reset read");
    if (!I.spec.p || reshape) {
        if (I.spec.ensure(nspec) != hipSuccess || I.ledger.ensure(L_N) != hipSuccess ||
            I.stats.ensure(S_N) != hipSuccess)
            return fail(GM_ENOMEM, "tallies");
        HIPCHK(hipMemsetAsync(I.spec.p, 0, nspec * sizeof(double), c->stream));
        HIPCHK(hipMemsetAsync(I.ledger.p, 0, L_N * sizeof(double), c->stream));
    }
    I.n_nu = tp->n_nu;
    I.n_theta = tp->n_theta;
    I.dirty = true;
    HIPCHK(hipMemsetAsync(I.stats.p, 0, S_N * sizeof(unsigned long long), c->stream));
    return GM_OK;
}

// The argument block of one instance (its geometry, plasma, emission and
// tally pointers, plus the transport parameters shared by the launch).
static TArgs fill_args(gm_ctx *c, int ii, const gm_track_params *tp)
{
    Instance &I = c->inst[ii];
    TArgs A{};
    A.zrec = I.zrec.p;
    A.zrec32 = I.zrec32.p;
    A.sh32 = c->sh32;
    A.ln_c2_2h = (float)std::log(kC * kC / (2.0 * kH));
    for (int j = 0; j < 3; ++j) {
        A.n[j] = I.grid.n[j];
        A.xs[j] = I.grid.x_start[j];
        A.dx[j] = I.grid.dx[j];
        A.inv_dx[j] = 1.0 / I.grid.dx[j];
        A.xe[j] = I.grid.x_start[j] + I.grid.n[j] * I.grid.dx[j];
    }
    A.inv_n3 = 1.0 / I.grid.n[2];
    A.C = kH * I.grid.L_unit_cm / kMeC2;
    A.inst = ii;
    A.key0 = (uint32_t)I.ep.seed;
    A.key1 = (uint32_t)(I.ep.seed >> 32);
    A.zone_of_root = I.zone_of_root.p;
    A.lnnu_min = I.lnnu_min;
    A.lnnu_span = I.lnnu_span;
    A.n_wnodes = I.nw;
    A.ln_w = I.ln_w.p;
    A.fmax = I.fmax.p;
    A.G = c->G;
    A.el = elec_of(I);
    A.spec = I.spec.p;
    A.ledger = I.ledger.p;
    A.stats = I.stats.p;
    A.n_nu = tp->n_nu;
    A.n_theta = tp->n_theta;
    A.ln_nu_lo = std::log(tp->nu_lo);
    A.inv_dln_nu = 1.0 / (std::log(tp->nu_hi / tp->nu_lo) / tp->n_nu);
    A.scattering = tp->scattering;
    A.bias_mode = I.bias_mode >= 0 ? I.bias_mode : tp->bias_mode;
    A.n_sc_max = tp->n_sc_max;
    A.bias_value = I.bias_mode >= 0 ? I.bias_value : tp->bias_value;
    A.bias_max = I.bias_mode >= 0 ? I.bias_max : tp->bias_max;
    A.step_h = tp->step_h;
    A.step_far = tp->step_far > 1.0 ? tp->step_far : 1.0;
    A.r_far = tp->step_far > 1.0 ? tp->r_far : HUGE_VAL;
    A.roulette_frac = tp->roulette_frac;
    A.roulette_p = tp->roulette_p;
    A.max_steps = tp->max_steps;
    A.L_unit_cm = I.grid.L_unit_cm;
    A.sh = c->sh;
    A.trace = c->trace;
    A.trace_n = c->trace_n.p;
    A.trace_cap = c->trace_cap;
    A.evlog = c->evlog;
    A.evlog_n = c->evlog_n.p;
    A.evlog_cap = c->evlog_cap;
    A.root_stride = c->root_stride;
    A.sw = I.sw_n == tp->n_nu * tp->n_theta ? I.sw.p : nullptr;
    A.lnb = I.lnb.p;
    A.lnb_n = I.lnb_n;
    A.lnb_lo = I.lnb_lo;
    A.lnb_hi = I.lnb_hi;
    A.mtab = I.mt_on ? I.mtab.p : nullptr;
    A.mt_n = I.mt_n;
    A.mt_lo = I.mt_lo;
    A.mt_hi = I.mt_hi;
    A.overflow = c->flags.p;
    A.cap = c->queue_cap;
    A.refill_min = c->refill_min;
    A.a_spin = I.grid.a_spin;
    A.mass = metric_mass(I.grid.metric);
    A.h_slope = I.grid.h_slope;
    A.r_h = kerr_horizon(I.grid.a_spin, A.mass);
    A.r_capture = A.r_h * (1.0 + tp->horizon_eps);
    A.r_record = I.grid.r_record;
    A.i1_plasma_max = (double)I.max_i1;
    A.verlet_tol = tp->verlet_tol;
    A.verlet_max_it = tp->verlet_max_it;
    A.inv_sc[0] = 1.0 / I.grid.dx[0];
    A.inv_sc[1] = 1.0 / I.grid.dx[1];
    A.inv_sc[2] = 1.0 / std::min(I.grid.dx[2], kPi * I.grid.dx[1]);
    return A;
}

// Track the pending roots of a set of instances of one metric in shared
// launches: one birth, and per generation one tracking and one scattering
// launch over the photons of all of them (each photon carries its
// instance), root ranges chunked by queue capacity.
static gm_status track_batch(gm_ctx *c, const std::vector<int> &ids, const gm_track_params *tp,
                             bool hbm_tally, std::vector<long long> &acc)
{
    const int n_inst = (int)ids.size();
    const size_t nspec = (size_t)tp->n_theta * tp->n_nu * 3;
    // per instance in LDS: ledger and counters, and the tally unless it is
    // added to in HBM directly
    const size_t lds_stride = L_N + S_N + (hbm_tally ? 0 : nspec);
    const size_t lds_track = (size_t)n_inst * lds_stride * 8 + kEvBytesPerBlock;
    const size_t lds_small = (size_t)n_inst * (L_N + S_N) * 8;
    const bool kerr = c->inst[ids[0]].grid.metric != GM_METRIC_MINKOWSKI_CART;
    const bool f32 = tp->precision == GM_PRECISION_F32_EMISSIVITY;
    using KernelFn = void (*)(TArgs);
#define GM_TRACK_VARIANTS(K, F, B) {K<2, F, B>, K<3, F, B>, K<4, F, B>}
#define GM_TRACK_VARIANTS_KS(F, B, CB) {track_kernel_ks<2, F, B, CB>, track_kernel_ks<3, F, B, CB>, track_kernel_ks<4, F, B, CB>}
    // [kerr][constant bias][f32][batched][waves - 2]; the flat tracker has no
    // constant-bias form
    static const KernelFn track_fns[2][2][2][2][3] = {
        {{{GM_TRACK_VARIANTS(track_kernel_flat, false, false), GM_TRACK_VARIANTS(track_kernel_flat, false, true)},
          {GM_TRACK_VARIANTS(track_kernel_flat, true, false), GM_TRACK_VARIANTS(track_kernel_flat, true, true)}},
         {{GM_TRACK_VARIANTS(track_kernel_flat, false, false), GM_TRACK_VARIANTS(track_kernel_flat, false, true)},
          {GM_TRACK_VARIANTS(track_kernel_flat, true, false), GM_TRACK_VARIANTS(track_kernel_flat, true, true)}}},
        {{{GM_TRACK_VARIANTS_KS(false, false, false), GM_TRACK_VARIANTS_KS(false, true, false)},
          {GM_TRACK_VARIANTS_KS(true, false, false), GM_TRACK_VARIANTS_KS(true, true, false)}},
         {{GM_TRACK_VARIANTS_KS(false, false, true), GM_TRACK_VARIANTS_KS(false, true, true)},
          {GM_TRACK_VARIANTS_KS(true, false, true), GM_TRACK_VARIANTS_KS(true, true, true)}}}};
#undef GM_TRACK_VARIANTS
#undef GM_TRACK_VARIANTS_KS
    bool const_bias = true;
    for (int k = 0; k < n_inst; ++k) {
        const Instance &I = c->inst[ids[k]];
        const_bias = const_bias && (I.bias_mode >= 0 ? I.bias_mode : tp->bias_mode) == GM_BIAS_CONST;
    }
    // one instance: the arguments travel as kernel arguments; several: per
    // instance from device memory, one instance per pass of a wave
    const KernelFn track_fn = track_fns[kerr][const_bias][f32][n_inst > 1][c->track_waves - 2];
    const KernelFn birth_fn = kerr ? (KernelFn)birth_kernel<KerrMKS, false>
                                   : f32 ? (KernelFn)birth_kernel<Minkowski, true> : (KernelFn)birth_kernel<Minkowski, false>;
    const bool batched = n_inst > 1;
    static const KernelFn scatter_fns[2][2][2] = {
        {{scatter_kernel_flat<false, false>, scatter_kernel_flat<false, true>},
         {scatter_kernel_flat<true, false>, scatter_kernel_flat<true, true>}},
        {{scatter_kernel_ks<false>, scatter_kernel_ks<true>}, {scatter_kernel_ks<false>, scatter_kernel_ks<true>}}};
    const KernelFn scatter_fn = scatter_fns[kerr][f32][batched];
    int occ = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, track_fn, 256, lds_track));
    occ = std::max(occ, 1);
    const int grid = c->n_cu * occ;
    // the rejection trials: one resident wave set, each lane running through
    // its share of the chunk's roots
    int occ_s = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_s, birth_sample_kernel, 256, lds_small));
    const unsigned long long grid_s_max = (unsigned long long)c->n_cu * std::max(occ_s, 1);

    std::vector<TArgs> args(n_inst);
    std::vector<unsigned long long> off(n_inst + 1, 0);
    for (int k = 0; k < n_inst; ++k) {
        gm_status s = prepare_instance(c, c->inst[ids[k]], tp);
        if (s != GM_OK) return s;
        args[k] = fill_args(c, ids[k], tp);
        const gm_grid &G = c->inst[ids[k]].grid;
        if (tp->step_far > 1.0 && G.metric != GM_METRIC_MINKOWSKI_CART) {
            // outside the plasma and the photon orbits: no turning back
            const double r_pl = std::exp(G.x_start[0] + (c->inst[ids[k]].max_i1 + 1) * G.dx[0]);
            if (!(tp->r_far >= r_pl && tp->r_far >= 4.0 * metric_mass(G.metric)))
                return fail(GM_EINVAL, "r_far %g must be >= the plasma's outer radius %g and 4 M", tp->r_far, r_pl);
        }
        off[k + 1] = off[k] + c->inst[ids[k]].n_roots;
    }
    if (c->inst_args.ensure(n_inst) != hipSuccess || c->root_off.ensure(n_inst + 1) != hipSuccess ||
        c->inst_ctr.ensure(2 * GM_MAX_INSTANCES) != hipSuccess)
        return fail(GM_ENOMEM, "launch arguments");
    HIPCHK(hipMemcpyAsync(c->inst_args.p, args.data(), n_inst * sizeof(TArgs), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->root_off.p, off.data(), (n_inst + 1) * sizeof(unsigned long long),
                          hipMemcpyHostToDevice, c->stream));
    TArgs L = args[0];
    L.insts = c->inst_args.p;
    L.n_inst = n_inst;
    L.root_off = c->root_off.p;
    L.lds_stride = (int)lds_stride;
    L.inst_count = c->inst_ctr.p;
    L.inst_cursor = c->inst_ctr.p + GM_MAX_INSTANCES;

    // generations 0 .. n_sc_max: only photons below the cap can scatter
    const int ngen = tp->scattering ? tp->n_sc_max + 1 : 1;
    const unsigned long long total = off[n_inst];
    // roots in chunks of half the queue; a chunk whose scattering cascade
    // overflows the queue is undone (tallies, ledgers, counters, trace and
    // event-log counts restored) and redone in quarters -- every history is
    // keyed by its root, so the redone chunk gives the same photons
    unsigned long long chunk = std::max<unsigned long long>(1, c->queue_cap / 2);
    const size_t nacc_d = nspec + L_N, nacc_u = S_N;
    if (c->bak_d.ensure((size_t)n_inst * nacc_d) != hipSuccess ||
        c->bak_u.ensure((size_t)n_inst * nacc_u + 2) != hipSuccess ||
        c->call_bak_d.ensure((size_t)n_inst * nacc_d) != hipSuccess ||
        c->call_bak_u.ensure((size_t)n_inst * nacc_u + 2) != hipSuccess)
        return fail(GM_ENOMEM, "chunk backup");
    // accumulators before the chunk (b = bak) or the call (b = call_bak)
    auto save = [&](DevBuf<double> &bd, DevBuf<unsigned long long> &bu) -> gm_status {
        for (int k = 0; k < n_inst; ++k) {
            Instance &I = c->inst[ids[k]];
            HIPCHK(hipMemcpyAsync(bd.p + k * nacc_d, I.spec.p, nspec * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(bd.p + k * nacc_d + nspec, I.ledger.p, L_N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(bu.p + k * nacc_u, I.stats.p, S_N * sizeof(unsigned long long), hipMemcpyDeviceToDevice, c->stream));
        }
        unsigned long long *bn = bu.p + (size_t)n_inst * nacc_u;
        HIPCHK(hipMemcpyAsync(bn, c->trace_n.p, sizeof(unsigned long long), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(bn + 1, c->evlog_n.p, sizeof(unsigned long long), hipMemcpyDeviceToDevice, c->stream));
        return GM_OK;
    };
    auto restore = [&](DevBuf<double> &bd, DevBuf<unsigned long long> &bu) -> gm_status {
        for (int k = 0; k < n_inst; ++k) {
            Instance &I = c->inst[ids[k]];
            HIPCHK(hipMemcpyAsync(I.spec.p, bd.p + k * nacc_d, nspec * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(I.ledger.p, bd.p + k * nacc_d + nspec, L_N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(I.stats.p, bu.p + k * nacc_u, S_N * sizeof(unsigned long long), hipMemcpyDeviceToDevice, c->stream));
        }
        unsigned long long *bn = bu.p + (size_t)n_inst * nacc_u;
        HIPCHK(hipMemcpyAsync(c->trace_n.p, bn, sizeof(unsigned long long), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->evlog_n.p, bn + 1, sizeof(unsigned long long), hipMemcpyDeviceToDevice, c->stream));
        return GM_OK;
    };
    gm_status bs = save(c->call_bak_d, c->call_bak_u);
    if (bs != GM_OK) return bs;
    // event records of this call: their scores are passed up the ancestry
    // once every chunk is done
    unsigned long long ev_lo = 0;
    if (c->evlog) {
        HIPCHK(hipMemcpyAsync(&ev_lo, c->evlog_n.p, sizeof(ev_lo), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    const hipStream_t run_stream = c->stream;
    if (c->use_graph && !c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    // the launches of one chunk: issued on c->stream, which is the capture
    // stream while a graph is being recorded (nothing runs then)
    auto issue_chunk = [&](unsigned long long start, unsigned long long cnt) -> gm_status {
        gm_status st = save(c->bak_d, c->bak_u);
        if (st != GM_OK) return st;
        reset_counters_kernel<<<1, 64, 0, c->stream>>>(c->ctr.p, 64, c->flags.p);
        L.root_begin = start;
        L.root_count = cnt;
        L.dst = queue(c, 0);
        L.src_count = c->ctr.p;                       // generation-0 count
        birth_sample_kernel<<<(unsigned)std::min<unsigned long long>((cnt + 255) / 256, grid_s_max), 256, lds_small,
                              c->stream>>>(L);
        HIPCHK(hipGetLastError());
        birth_fn<<<(unsigned)((cnt + 255) / 256), 256, lds_small, c->stream>>>(L);
        HIPCHK(hipGetLastError());
        for (int g = 0; g < ngen; ++g) {
            L.gen = g;
            // one instance: the queues alternate and children replace their
            // events in place; batched: photons always come from queue 0 and
            // events go to queue 1, from where the scattering kernel writes
            // the children back to queue 0 grouped by instance
            L.src = queue(c, batched ? 0 : (g & 1));
            L.dst = queue(c, batched ? 1 : ((g + 1) & 1));
            L.out = queue(c, 0);
            L.src_count = c->ctr.p + 2 * g;
            L.src_cursor = c->ctr.p + 2 * g + 1;
            L.dst_count = c->ctr.p + 2 * (g + 1);
            // per-launch event timing only when launched directly
            const bool timed = c->timing && !c->use_graph;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timed) {
                gm_status ts = take_event_pair(c, e0, e1);
                if (ts != GM_OK) return ts;
                HIPCHK(hipEventRecord(e0, c->stream));
            }
            track_fn<<<grid, 256, lds_track, c->stream>>>(L);
            HIPCHK(hipGetLastError());
            if (timed) HIPCHK(hipEventRecord(e1, c->stream));
            if (g + 1 < ngen) {
                if (batched) {
                    reset_counters_kernel<<<1, 2 * GM_MAX_INSTANCES, 0, c->stream>>>(c->inst_ctr.p, 2 * GM_MAX_INSTANCES, nullptr);
                    count_events_kernel<<<c->n_cu * 4, 256, 0, c->stream>>>(L);
                }
                scatter_fn<<<c->n_cu * 8, 256, lds_small, c->stream>>>(L);
                HIPCHK(hipGetLastError());
            }
        }
        return GM_OK;
    };
    for (unsigned long long start = 0; start < total;) {
        const unsigned long long cnt = std::min(chunk, total - start);
        if (!c->use_graph) {
            bs = issue_chunk(start, cnt);
            if (bs != GM_OK) return bs;
        } else {
            HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            c->stream = c->cap_stream;
            bs = issue_chunk(start, cnt);
            hipGraph_t gr = nullptr;
            const hipError_t ec = hipStreamEndCapture(c->cap_stream, &gr);
            c->stream = run_stream;
            if (bs != GM_OK || ec != hipSuccess) {
                if (gr) (void)hipGraphDestroy(gr);
                return bs != GM_OK ? bs : fail(GM_EDEVICE, "graph capture: %s", hipGetErrorString(ec));
            }
            // reuse the executable graph when only kernel arguments changed
            if (c->graph_exec) {
                hipGraphNode_t bad = nullptr;
                hipGraphExecUpdateResult res;
                if (hipGraphExecUpdate(c->graph_exec, gr, &bad, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
                    (void)hipGetLastError();
                    (void)hipGraphExecDestroy(c->graph_exec);
                    c->graph_exec = nullptr;
                }
            }
            hipError_t ei = hipSuccess;
            if (!c->graph_exec) {
                ei = hipGraphInstantiate(&c->graph_exec, gr, nullptr, nullptr, 0);
                c->graph_instantiations += 1;
            }
            (void)hipGraphDestroy(gr);
            if (ei != hipSuccess) {
                c->graph_exec = nullptr;
                return fail(GM_EDEVICE, "graph instantiation: %s", hipGetErrorString(ei));
            }
            HIPCHK(hipGraphLaunch(c->graph_exec, c->stream));
            c->graph_launches += 1;
        }
        int ovf = 0;
        HIPCHK(hipMemcpyAsync(&ovf, c->flags.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (!ovf) {
            start += cnt;
            continue;
        }
        // a single root's cascade overflows: the call is undone for these
        // instances (accumulators and counts as before it; roots still pending)
        if (cnt == 1) {
            bs = restore(c->call_bak_d, c->call_bak_u);
            if (bs != GM_OK) return bs;
            HIPCHK(hipStreamSynchronize(c->stream));
            return fail(GM_ENOMEM, "the scattering cascade of root %llu alone overflows the photon queue of %llu",
                        start, c->queue_cap);
        }
        // undo the chunk: tallies, ledgers, counters, trace and event-log counts
        bs = restore(c->bak_d, c->bak_u);
        if (bs != GM_OK) return bs;
        c->chunk_retries += 1;
        chunk = std::max<unsigned long long>(1, cnt / 4);
    }
    if (c->evlog) {
        unsigned long long ev_hi = 0;
        HIPCHK(hipMemcpyAsync(&ev_hi, c->evlog_n.p, sizeof(ev_hi), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        ev_hi = std::min(ev_hi, c->evlog_cap);
        if (ev_hi > ev_lo) {
            const unsigned nb = (unsigned)std::min<unsigned long long>((ev_hi - ev_lo + 255) / 256, 4096);
            for (int g = tp->n_sc_max; g >= 1; --g)
                score_propagate_kernel<<<nb, 256, 0, c->stream>>>(c->evlog, ev_lo, ev_hi, g);
            HIPCHK(hipGetLastError());
        }
    }
    // counters of every instance, one synchronisation
    std::vector<unsigned long long> st((size_t)n_inst * S_N);
    for (int k = 0; k < n_inst; ++k)
        HIPCHK(hipMemcpyAsync(st.data() + (size_t)k * S_N, c->inst[ids[k]].stats.p, S_N * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int k = 0; k < n_inst; ++k) {
        for (int i = 0; i < S_N; ++i) acc[i] += (long long)st[(size_t)k * S_N + i];
        c->inst[ids[k]].pending = false;
    }
    return GM_OK;
}

gm_status gm_track_scatter(gm_ctx *c, const gm_track_params *tp, int64_t *stats)
{
    if (!c || !tp) return fail(GM_EINVAL, "NULL argument");
    if (tp->n_nu < 1 || tp->n_theta < 1 || !(tp->nu_lo > 0.0) || !(tp->nu_hi > tp->nu_lo) ||
        !(tp->bias_max >= 1.0) || !(tp->step_h > 0.0) || tp->verlet_max_it < 1 || tp->n_sc_max < 0 ||
        tp->n_sc_max > 15 || !(tp->roulette_p > 0.0 && tp->roulette_p <= 1.0) || tp->max_steps < 1 ||
        tp->bias_mode < 0 || tp->bias_mode > 4 || (tp->bias_mode < 3 && !(tp->bias_value > 0.0)) ||
        !(tp->step_far == 0.0 || (tp->step_far >= 1.0 && std::isfinite(tp->step_far))))
        return fail(GM_EINVAL, "bad track parameters");
    if (tp->precision != GM_PRECISION_F64 && tp->precision != GM_PRECISION_F32_EMISSIVITY)
        return fail(GM_EINVAL, "precision %d", tp->precision);
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    bool any = false;
    for (auto &I : c->inst) any |= I.pending;
    if (!any) return fail(GM_ESTATE, "no superphotons made since the last track");
    for (int i = 0; i < GM_MAX_INSTANCES; ++i) {
        const Instance &I = c->inst[i];
        const int mode = I.bias_mode >= 0 ? I.bias_mode : tp->bias_mode;
        if (I.pending && (mode == GM_BIAS_TABLE || mode == GM_BIAS_WINDOW) && (!I.lnb.p || I.lnb_n < 2))
            return fail(GM_ESTATE, "instance %d has no bias table", i);
        if (I.pending && I.sw_n && I.sw_n != tp->n_nu * tp->n_theta)
            return fail(GM_EINVAL, "instance %d: score weights of %d bins, tally of %d", i, I.sw_n,
                        tp->n_nu * tp->n_theta);
    }
    for (int i = 0; i < GM_MAX_INSTANCES; ++i) {
        Instance &I = c->inst[i];
        if (!I.pending || I.el.kind == GM_DIST_THERMAL) continue;
        if (tp->precision != GM_PRECISION_F64)
            return fail(GM_EUNSUPPORTED, "instance %d: power-law electrons run in FP64 only", i);
        if (tp->scattering) {
            s = ensure_sigma_pl(c, I);
            if (s != GM_OK) return s;
        }
    }
    if (tp->scattering) {
        s = ensure_sigma_hot(c);
        if (s != GM_OK) return s;
    }
    // room for the roots of every pending instance (shared launches run
    // them as one chunk) and as many children per generation
    unsigned long long pending = 0;
    for (auto &I : c->inst)
        if (I.pending) pending += I.n_roots;
    unsigned long long need = std::max(1ull << 22, 2 * pending);
    need = std::min(need, 1ull << 26);
    if (c->queue_cap_set) need = c->queue_cap_set;
    s = ensure_children(c, need);
    if (s != GM_OK) return s;
    // instances of one metric share launches (at most max_batch).  56 KiB
    // of per-block accumulators and the event staging keep two blocks on a
    // CU: the tallies stay in LDS when those of the group fit, else every
    // escape adds to the instance's tally in HBM directly
    const size_t per_small = (size_t)(L_N + S_N) * 8;
    const size_t per_inst = per_small + (size_t)tp->n_theta * tp->n_nu * 3 * 8;
    const size_t acc_budget = 56 * 1024;
    std::vector<long long> acc(S_N, 0);
    std::vector<bool> taken(GM_MAX_INSTANCES, false);
    for (int lead = 0; lead < GM_MAX_INSTANCES; ++lead) {
        // the pending instances of lead's metric and electrons, in order
        if (!c->inst[lead].pending || taken[lead]) continue;
        std::vector<int> pend;
        for (int i = lead; i < GM_MAX_INSTANCES; ++i)
            if (c->inst[i].pending && !taken[i] && c->inst[i].grid.metric == c->inst[lead].grid.metric &&
                same_electrons(c->inst[i].el, c->inst[lead].el)) {
                pend.push_back(i);
                taken[i] = true;
            }
        const int want = std::min((int)pend.size(), c->max_batch);
        const int lds_fit = (int)(acc_budget / per_inst);
        bool hbm = c->tally_mode == 2 || (c->tally_mode == 0 && lds_fit < want);
        if (c->tally_mode == 1 && lds_fit < 1)
            return fail(GM_EUNSUPPORTED, "tally of %d bins exceeds the LDS budget", tp->n_theta * tp->n_nu);
        const int group = hbm ? std::min(want, (int)(acc_budget / per_small)) : std::min(want, lds_fit);
        for (size_t g0 = 0; g0 < pend.size(); g0 += group) {
            std::vector<int> ids(pend.begin() + g0, pend.begin() + std::min(pend.size(), g0 + group));
            s = track_batch(c, ids, tp, hbm, acc);
            if (s != GM_OK) return s;
        }
    }
    if (stats)
        for (int i = 0; i < S_N; ++i) stats[i] = acc[i];
    return GM_OK;
}

gm_status gm_read_spectrum(gm_ctx *c, int instance, double *out, int out_on_device, double *ledger_out,
                           int reset)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    Instance &I = c->inst[instance];
    if (!I.spec.p) return fail(GM_ESTATE, "instance %d has no tally", instance);
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    const size_t nspec = (size_t)I.n_theta * I.n_nu * 3;
    if (out)
        HIPCHK(hipMemcpyAsync(out, I.spec.p, nspec * sizeof(double),
                              out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    if (ledger_out)
        HIPCHK(hipMemcpyAsync(ledger_out, I.ledger.p, L_N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (reset) {
        HIPCHK(hipMemsetAsync(I.spec.p, 0, nspec * sizeof(double), c->stream));
        HIPCHK(hipMemsetAsync(I.ledger.p, 0, L_N * sizeof(double), c->stream));
        I.dirty = false;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return GM_OK;
}

gm_status gm_read_emission(gm_ctx *c, int instance, uint32_t *counts, double *nbar, double *fmax, double *ln_w)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    Instance &I = c->inst[instance];
    if (!I.made) return fail(GM_ESTATE, "instance %d: nothing made", instance);
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    HIPCHK(hipStreamSynchronize(c->stream));
    if (counts) HIPCHK(hipMemcpy(counts, I.count.p, (size_t)I.nz * 4, hipMemcpyDeviceToHost));
    if (nbar) HIPCHK(hipMemcpy(nbar, I.nbar.p, (size_t)I.nz * 8, hipMemcpyDeviceToHost));
    if (fmax) HIPCHK(hipMemcpy(fmax, I.fmax.p, (size_t)I.nz * 8, hipMemcpyDeviceToHost));
    if (ln_w) HIPCHK(hipMemcpy(ln_w, I.ln_w.p, (size_t)I.nw * 8, hipMemcpyDeviceToHost));
    return GM_OK;
}

gm_status gm_set_trace(gm_ctx *c, void *buf, uint64_t capacity)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (buf && capacity == 0) return fail(GM_EINVAL, "zero capacity");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    c->trace = (TraceRec *)buf;
    c->trace_cap = buf ? capacity : 0;
    HIPCHK(hipMemsetAsync(c->trace_n.p, 0, sizeof(unsigned long long), c->stream));
    return GM_OK;
}

gm_status gm_trace_count(gm_ctx *c, uint64_t *n)
{
    if (!c || !n) return fail(GM_EINVAL, "NULL argument");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    unsigned long long v = 0;
    HIPCHK(hipMemcpyAsync(&v, c->trace_n.p, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *n = v;
    return GM_OK;
}

gm_status gm_sigma_hot_table(gm_ctx *c, double *host_out)
{
    if (!c || !host_out) return fail(GM_EINVAL, "NULL argument");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    s = ensure_sigma_hot(c);
    if (s != GM_OK) return s;
    HIPCHK(hipMemcpyAsync(host_out, c->sh_table.p, kShNT * kShNE * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return GM_OK;
}

gm_status gm_set_tuning(gm_ctx *c, int track_waves, int refill_min)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (track_waves < 2 || track_waves > 4) return fail(GM_EINVAL, "track_waves %d not in 2..4", track_waves);
    if (refill_min < 1 || refill_min > 64) return fail(GM_EINVAL, "refill_min %d not in 1..64", refill_min);
    c->track_waves = track_waves;
    c->refill_min = refill_min;
    return GM_OK;
}

gm_status gm_set_instance_bias(gm_ctx *c, int instance, int bias_mode, double bias_value, double bias_max)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    if (bias_mode > 4 || (bias_mode >= 0 && !(bias_max >= 1.0)) ||
        (bias_mode >= 0 && bias_mode < 3 && !(bias_value > 0.0)))
        return fail(GM_EINVAL, "bad bias");
    Instance &I = c->inst[instance];
    I.bias_mode = bias_mode < 0 ? -1 : bias_mode;
    I.bias_value = bias_value;
    I.bias_max = bias_max;
    return GM_OK;
}

gm_status gm_set_queue_capacity(gm_ctx *c, uint64_t entries)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (entries != 0 && (entries < 64 || entries > (1ull << 27)))
        return fail(GM_EINVAL, "queue capacity %llu not 0 or in [64, 2^27]", (unsigned long long)entries);
    c->queue_cap_set = entries;
    return GM_OK;
}

gm_status gm_queue_stats(gm_ctx *c, uint64_t *capacity, uint64_t *chunk_retries)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (capacity) *capacity = c->queue_cap;
    if (chunk_retries) *chunk_retries = c->chunk_retries;
    return GM_OK;
}

gm_status gm_set_graph(gm_ctx *c, int enable, uint64_t *launches, uint64_t *instantiations)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (launches) *launches = c->graph_launches;
    if (instantiations) *instantiations = c->graph_instantiations;
    if (enable >= 0) c->use_graph = enable != 0;
    return GM_OK;
}

gm_status gm_set_batch(gm_ctx *c, int max_instances)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (max_instances < 1 || max_instances > GM_MAX_INSTANCES)
        return fail(GM_EINVAL, "max_instances %d not in 1..%d", max_instances, GM_MAX_INSTANCES);
    c->max_batch = max_instances;
    return GM_OK;
}

gm_status gm_set_timing(gm_ctx *c, int enable)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    s = drain_events(c);
    if (s != GM_OK) return s;
    c->timing = enable != 0;
    c->track_ms = 0.0;
    c->track_launches = 0;
    return GM_OK;
}

gm_status gm_read_timing(gm_ctx *c, double *track_ms, uint64_t *track_launches)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    s = drain_events(c);
    if (s != GM_OK) return s;
    if (track_ms) *track_ms = c->track_ms;
    if (track_launches) *track_launches = c->track_launches;
    return GM_OK;
}

gm_status gm_fma_chain_bound(gm_ctx *c, int waves, int chains, int64_t iters, double *ms, double *tflops,
                             double *host_out, int n_out)
{
    if (!c || waves < 1 || waves > 8 || iters < 1 || n_out < 0 || (n_out > 0 && !host_out))
        return fail(GM_EINVAL, "bad argument");
    using Fn = void (*)(double, double, long long, double *);
    Fn fn = chains == 1 ? (Fn)fma_chain_kernel<1> : chains == 2 ? (Fn)fma_chain_kernel<2>
          : chains == 4 ? (Fn)fma_chain_kernel<4> : chains == 8 ? (Fn)fma_chain_kernel<8> : nullptr;
    if (!fn) return fail(GM_EINVAL, "chains must be 1, 2, 4 or 8");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    int lds_cu = 0;
    HIPCHK(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->device));
    // at most `waves` blocks per CU: each reserves more than 1/(waves+1) of the LDS
    size_t lds = std::min<size_t>((size_t)lds_cu / (size_t)waves, 64 * 1024) & ~(size_t)1023;
    int occ = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 256, lds));
    if (occ != waves)
        return fail(GM_EUNSUPPORTED, "%d waves per SIMD cannot be pinned (%zu bytes of LDS per block give %d blocks per CU)",
                    waves, lds, occ);
    const int grid = c->n_cu * waves;
    const size_t n = (size_t)grid * 256;
    if (n_out > (int64_t)n) return fail(GM_EINVAL, "n_out above %zu", n);
    DevBuf<double> out;
    if (out.ensure(n) != hipSuccess) return fail(GM_ENOMEM, "bound buffer");
    const double m = 0.9999999, a = 1e-7;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        fn<<<grid, 256, lds, c->stream>>>(m, a, (long long)std::min<int64_t>(iters, 1024), out.p);   // warm-up
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    if (e == hipSuccess) {
        fn<<<grid, 256, lds, c->stream>>>(m, a, (long long)iters, out.p);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess && n_out > 0)
        e = hipMemcpyAsync(host_out, out.p, (size_t)n_out * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    out.release();
    if (e != hipSuccess) return fail(GM_EDEVICE, "fma chain bound: %s", hipGetErrorString(e));
    if (ms) *ms = t;
    if (tflops) *tflops = 2.0 * (double)chains * (double)iters * (double)n / ((double)t * 1e-3) * 1e-12;
    return GM_OK;
}

gm_status gm_eval_G(gm_ctx *c, const double *hx, double *hy, int n)
{
    if (!c || !hx || !hy || n < 0) return fail(GM_EINVAL, "bad argument");
    if (n == 0) return GM_OK;
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    DevBuf<double> dx, dy;
    if (dx.ensure(n) != hipSuccess || dy.ensure(n) != hipSuccess) { dx.release(); dy.release(); return fail(GM_ENOMEM, "eval buffers"); }
    hipError_t e = hipMemcpyAsync(dx.p, hx, n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        eval_G_kernel<<<(n + 255) / 256, 256, 0, c->stream>>>(c->G, dx.p, dy.p, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hy, dy.p, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dx.release();
    dy.release();
    if (e != hipSuccess) return fail(GM_EDEVICE, "eval_G: %s", hipGetErrorString(e));
    return GM_OK;
}

gm_status gm_set_event_log(gm_ctx *c, void *buf, uint64_t capacity, uint64_t root_stride)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (buf && (capacity == 0 || capacity > 0xfffffffeull)) return fail(GM_EINVAL, "capacity not in [1, 2^32 - 2]");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    c->evlog = (EventRec *)buf;
    c->evlog_cap = buf ? capacity : 0;
    c->root_stride = buf ? root_stride : 0;
    HIPCHK(hipMemsetAsync(c->evlog_n.p, 0, sizeof(unsigned long long), c->stream));
    return GM_OK;
}

gm_status gm_event_count(gm_ctx *c, uint64_t *n)
{
    if (!c || !n) return fail(GM_EINVAL, "NULL argument");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    unsigned long long v = 0;
    HIPCHK(hipMemcpyAsync(&v, c->evlog_n.p, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *n = v;
    return GM_OK;
}

gm_status gm_event_band(gm_ctx *c, double *eps_min, double *eps_max)
{
    if (!c || !eps_min || !eps_max) return fail(GM_EINVAL, "NULL argument");
    if (!c->evlog) return fail(GM_ESTATE, "no event log set");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    if (c->band_mm.ensure(2) != hipSuccess) return fail(GM_ENOMEM, "band");
    unsigned long long n_ev = 0, mm[2] = {~0ull, 0ull};
    HIPCHK(hipMemcpyAsync(c->band_mm.p, mm, sizeof(mm), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(&n_ev, c->evlog_n.p, sizeof(n_ev), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    n_ev = std::min(n_ev, c->evlog_cap);
    if (n_ev > 0) {
        const unsigned nb = (unsigned)std::min<unsigned long long>((n_ev + 255) / 256, 2048);
        event_band_kernel<<<nb, 256, 0, c->stream>>>(c->evlog, n_ev, c->band_mm.p);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(mm, c->band_mm.p, sizeof(mm), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (mm[0] > mm[1]) return fail(GM_ESTATE, "no emission records in the event log");
    std::memcpy(eps_min, &mm[0], sizeof(double));
    std::memcpy(eps_max, &mm[1], sizeof(double));
    return GM_OK;
}

gm_status gm_set_bias_table(gm_ctx *c, int instance, const double *ln_b, int n_eps, double ln_eps_lo,
                            double ln_eps_hi)
{
    if (!c || !ln_b) return fail(GM_EINVAL, "NULL argument");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    Instance &I = c->inst[instance];
    if (!I.loaded) return fail(GM_ESTATE, "instance %d has no zones", instance);
    if (n_eps < 2 || n_eps > 4096 || !(ln_eps_hi > ln_eps_lo)) return fail(GM_EINVAL, "bad bias table shape");
    const size_t n = (size_t)I.nz * n_eps;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(ln_b[i])) return fail(GM_EINVAL, "bias table entry %zu not finite", i);
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    if (I.lnb.ensure(n) != hipSuccess) return fail(GM_ENOMEM, "bias table");
    HIPCHK(hipMemcpyAsync(I.lnb.p, ln_b, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    I.lnb_n = n_eps;
    I.lnb_lo = ln_eps_lo;
    I.lnb_hi = ln_eps_hi;
    return GM_OK;
}

gm_status gm_set_emission_table(gm_ctx *c, int instance, const double *m, int n_nodes, double ln_nu_lo,
                                double ln_nu_hi)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    Instance &I = c->inst[instance];
    if (!I.loaded) return fail(GM_ESTATE, "instance %d has no zones", instance);
    if (!m) {
        I.mt_on = false;
        I.made = false;          // the expected counts change with the table
        return GM_OK;
    }
    if (n_nodes < 2 || n_nodes > 4096 || !(ln_nu_hi > ln_nu_lo)) return fail(GM_EINVAL, "bad emission table shape");
    const size_t n = (size_t)I.nz * n_nodes;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(m[i])) return fail(GM_EINVAL, "emission table entry %zu not finite", i);
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    if (I.mtab.ensure(n) != hipSuccess) return fail(GM_ENOMEM, "emission table");
    HIPCHK(hipMemcpyAsync(I.mtab.p, m, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    I.mt_n = n_nodes;
    I.mt_lo = ln_nu_lo;
    I.mt_hi = ln_nu_hi;
    I.mt_on = true;
    I.made = false;
    return GM_OK;
}

gm_status gm_set_score_weights(gm_ctx *c, int instance, const double *sw, int n)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    Instance &I = c->inst[instance];
    if (!sw) { I.sw_n = 0; return GM_OK; }
    if (n < 1) return fail(GM_EINVAL, "bad score weights");
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(sw[i])) return fail(GM_EINVAL, "score weight %d not finite", i);
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    if (I.sw.ensure(n) != hipSuccess) return fail(GM_ENOMEM, "score weights");
    HIPCHK(hipMemcpyAsync(I.sw.p, sw, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    I.sw_n = n;
    return GM_OK;
}

gm_status gm_set_tally_mode(gm_ctx *c, int mode)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (mode < 0 || mode > 2) return fail(GM_EINVAL, "tally mode %d not in 0..2", mode);
    c->tally_mode = mode;
    return GM_OK;
}

// ---- tables of the importance-driven forms --------------------------------
static gm_status check_map(const gm_ctx *c, int instance, const gm_importance_map *m)
{
    if (!c || !m) return fail(GM_EINVAL, "NULL argument");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    if (!c->inst[instance].loaded) return fail(GM_ESTATE, "instance %d has no zones", instance);
    if ((m->table != GM_TABLE_BIAS && m->table != GM_TABLE_EMISSION) || m->n_nodes < 2 || m->n_nodes > 4096 ||
        !(m->hi > m->lo) || (m->kind != GM_IMP_LINEAR && m->kind != GM_IMP_MIXTURE) || !std::isfinite(m->a) ||
        !std::isfinite(m->b) || !std::isfinite(m->shift) ||
        (m->kind == GM_IMP_MIXTURE && !(m->alpha >= 0.0 && m->alpha < 1.0)))
        return fail(GM_EINVAL, "bad importance map");
    return GM_OK;
}

static ZoneGeo zone_geo_of(const gm_grid &g)
{
    ZoneGeo G{};
    for (int j = 0; j < 3; ++j) { G.n[j] = g.n[j]; G.xs[j] = g.x_start[j]; G.dx[j] = g.dx[j]; }
    G.metric = g.metric;
    G.h_slope = g.h_slope;
    G.half = 0.0;
    for (int j = 0; j < 3; ++j) G.half = std::max(G.half, 0.5 * g.n[j] * g.dx[j]);
    return G;
}

// The instance's table a map writes (allocated as needed), with its node
// layout recorded; the emission table invalidates the stored counts.
static gm_status map_target(gm_ctx *c, int instance, const gm_importance_map *m, double **out)
{
    Instance &I = c->inst[instance];
    const size_t n = (size_t)I.nz * m->n_nodes;
    if (m->table == GM_TABLE_BIAS) {
        if (I.lnb.ensure(n) != hipSuccess) return fail(GM_ENOMEM, "bias table");
        I.lnb_n = m->n_nodes; I.lnb_lo = m->lo; I.lnb_hi = m->hi;
        *out = I.lnb.p;
    } else {
        if (I.mtab.ensure(n) != hipSuccess) return fail(GM_ENOMEM, "emission table");
        I.mt_n = m->n_nodes; I.mt_lo = m->lo; I.mt_hi = m->hi; I.mt_on = true;
        I.made = false;
        *out = I.mtab.p;
    }
    return GM_OK;
}

static double map_v_shift(const gm_importance_map *m)
{
    return m->table == GM_TABLE_EMISSION ? std::log(kMeC2 / kH) : 0.0;
}

gm_status gm_remap_table(gm_ctx *c, int instance, const gm_importance_map *m)
{
    gm_status s = check_map(c, instance, m);
    if (s != GM_OK) return s;
    Instance &I = c->inst[instance];
    const bool bias = m->table == GM_TABLE_BIAS;
    double *tab = bias ? I.lnb.p : I.mtab.p;
    const int n = bias ? I.lnb_n : I.mt_n;
    const double lo = bias ? I.lnb_lo : I.mt_lo, hi = bias ? I.lnb_hi : I.mt_hi;
    if (!tab || n != m->n_nodes || lo != m->lo || hi != m->hi || (!bias && !I.mt_on))
        return fail(GM_ESTATE, "no table of this instance with the map's node layout");
    s = set_device(c);
    if (s != GM_OK) return s;
    RemapArgs R;
    R.zrec = I.zrec.p;
    R.nz = I.nz;
    R.n_nodes = n;
    R.map = ImpMap{m->kind, m->a, m->b, m->alpha, m->shift};
    R.table = tab;
    const long long cnt = (long long)I.nz * n;
    remap_table_kernel<<<(unsigned)std::min<long long>((cnt + 255) / 256, 65536), 256, 0, c->stream>>>(R);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    if (!bias) I.made = false;
    return GM_OK;
}

gm_status gm_mlp_fill_table(gm_ctx *c, int instance, const gm_importance_map *m, int output, const float *mu,
                            const float *sd)
{
    gm_status s = check_map(c, instance, m);
    if (s != GM_OK) return s;
    if (output < 0 || output >= kMlpOut || !mu || !sd) return fail(GM_EINVAL, "bad network output or scaling");
    for (int i = 0; i < kMlpIn; ++i)
        if (!std::isfinite(mu[i]) || !(sd[i] > 0.0f)) return fail(GM_EINVAL, "feature scaling %d", i);
    if (!c->mlp_ready) return fail(GM_ESTATE, "network parameters not set");
    s = set_device(c);
    if (s != GM_OK) return s;
    Instance &I = c->inst[instance];
    double *tab = nullptr;
    s = map_target(c, instance, m, &tab);
    if (s != GM_OK) return s;
    TableFill T{};
    T.zrec = I.zrec.p;
    T.G = zone_geo_of(I.grid);
    T.nz = I.nz;
    T.n_nodes = m->n_nodes;
    T.lo = m->lo; T.hi = m->hi; T.v_shift = map_v_shift(m);
    for (int i = 0; i < kMlpIn; ++i) { T.mu[i] = mu[i]; T.inv_sd[i] = 1.0f / sd[i]; }
    T.out_col = output;
    T.map = ImpMap{m->kind, m->a, m->b, m->alpha, m->shift};
    T.neutral = 0.0;
    T.table = tab;
    MlpArgs M{};
    M.n = (long long)I.nz * m->n_nodes;
    M.P = c->mlp_p.p;
    M.Pb = c->mlp_pb.p;
    const long long rows_per_block = 16LL * kMlpWaves;
    mlp_table_kernel<<<(unsigned)((M.n + rows_per_block - 1) / rows_per_block), 64 * kMlpWaves, 0, c->stream>>>(M, T);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return GM_OK;
}

gm_status gm_read_table(gm_ctx *c, int instance, int table, double *host_out, int64_t n, int *n_nodes)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (instance < 0 || instance >= GM_MAX_INSTANCES) return fail(GM_EINVAL, "instance %d", instance);
    const Instance &I = c->inst[instance];
    const bool bias = table == GM_TABLE_BIAS;
    if (!bias && table != GM_TABLE_EMISSION) return fail(GM_EINVAL, "table %d", table);
    const double *src = bias ? I.lnb.p : (I.mt_on ? I.mtab.p : nullptr);
    const int nn = bias ? I.lnb_n : I.mt_n;
    if (!src || nn < 2) return fail(GM_ESTATE, "instance %d has no such table", instance);
    if (n_nodes) *n_nodes = nn;
    if (!host_out) return GM_OK;
    if (n != (int64_t)I.nz * nn) return fail(GM_EINVAL, "table holds %lld values", (long long)I.nz * nn);
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    HIPCHK(hipMemcpyAsync(host_out, src, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return GM_OK;
}

gm_status gm_cells_accumulate(gm_ctx *c, int instance, const gm_importance_map *m, const int *blocks,
                              double *totals)
{
    gm_status s = check_map(c, instance, m);
    if (s != GM_OK) return s;
    if (!blocks || blocks[0] < 1 || blocks[1] < 1 || blocks[2] < 1) return fail(GM_EINVAL, "bad cell blocks");
    if (!c->evlog) return fail(GM_ESTATE, "no event log set");
    s = set_device(c);
    if (s != GM_OK) return s;
    const Instance &I = c->inst[instance];
    CellArgs C{};
    C.G = zone_geo_of(I.grid);
    for (int j = 0; j < 3; ++j) { C.b[j] = blocks[j]; C.nc[j] = (I.grid.n[j] + blocks[j] - 1) / blocks[j]; }
    C.n_nodes = m->n_nodes;
    C.lo = m->lo; C.hi = m->hi; C.v_shift = map_v_shift(m);
    C.records = m->table == GM_TABLE_BIAS ? 1 : 0;
    const size_t n_acc = (size_t)C.nc[0] * C.nc[1] * C.nc[2] * m->n_nodes * 3;
    if (c->cell_acc.ensure(n_acc) != hipSuccess) return fail(GM_ENOMEM, "cell sums");
    HIPCHK(hipMemsetAsync(c->cell_acc.p, 0, n_acc * sizeof(double), c->stream));
    unsigned long long n_ev = 0;
    HIPCHK(hipMemcpyAsync(&n_ev, c->evlog_n.p, sizeof(n_ev), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    C.ev = c->evlog;
    C.n_ev = std::min(n_ev, c->evlog_cap);
    C.acc = c->cell_acc.p;
    if (C.n_ev > 0) {
        const unsigned nb = (unsigned)std::min<unsigned long long>((C.n_ev + 255) / 256, 8192);
        cells_accumulate_kernel<<<nb, 256, 0, c->stream>>>(C);
        HIPCHK(hipGetLastError());
    }
    std::vector<double> acc(n_acc);
    HIPCHK(hipMemcpyAsync(acc.data(), c->cell_acc.p, n_acc * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    double t[3] = {0.0, 0.0, 0.0};
    for (size_t i = 0; i < n_acc; i += 3) { t[0] += acc[i]; t[1] += acc[i + 1]; t[2] += acc[i + 2]; }
    for (int j = 0; j < 3; ++j) { c->cell_tot[j] = t[j]; c->cell_blocks[j] = C.b[j]; c->cell_nc[j] = C.nc[j]; }
    c->cell_map = *m;
    c->cell_inst = instance;
    if (totals) for (int j = 0; j < 3; ++j) totals[j] = t[j];
    return GM_OK;
}

gm_status gm_cells_fill_table(gm_ctx *c, int instance, const gm_importance_map *m, double prior)
{
    gm_status s = check_map(c, instance, m);
    if (s != GM_OK) return s;
    if (c->cell_inst != instance || c->cell_map.table != m->table || c->cell_map.n_nodes != m->n_nodes ||
        c->cell_map.lo != m->lo || c->cell_map.hi != m->hi)
        return fail(GM_ESTATE, "no cell sums of this instance, table and node layout (gm_cells_accumulate first)");
    if (!(prior >= 0.0) || !(c->cell_tot[1] > 0.0)) return fail(GM_EINVAL, "bad prior or no record weight");
    s = set_device(c);
    if (s != GM_OK) return s;
    const Instance &I = c->inst[instance];
    double *tab = nullptr;
    s = map_target(c, instance, m, &tab);
    if (s != GM_OK) return s;
    CellArgs C{};
    C.G = zone_geo_of(I.grid);
    for (int j = 0; j < 3; ++j) { C.b[j] = c->cell_blocks[j]; C.nc[j] = c->cell_nc[j]; }
    C.n_nodes = m->n_nodes;
    C.lo = m->lo; C.hi = m->hi; C.v_shift = map_v_shift(m);
    C.acc = c->cell_acc.p;
    C.nz = I.nz;
    C.zrec = I.zrec.p;
    C.per_photon = m->per_photon ? 1 : 0;
    if (C.per_photon) {
        C.ratio_all = c->cell_tot[0] / std::max(c->cell_tot[2], 1.0);
        C.prior_w = prior;                                                    // `prior` records
    } else {
        C.ratio_all = c->cell_tot[0] / c->cell_tot[1];
        C.prior_w = prior * c->cell_tot[1] / std::max(c->cell_tot[2], 1.0);  // `prior` records' mean weight
    }
    C.map = ImpMap{m->kind, m->a, m->b, m->alpha, m->shift};
    C.neutral = 0.0;
    C.table = tab;
    const long long n = (long long)I.nz * m->n_nodes;
    cells_fill_kernel<<<(unsigned)std::min<long long>((n + 255) / 256, 65536), 256, 0, c->stream>>>(C);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return GM_OK;
}

static gm_status mlp_buffers(gm_ctx *c)
{
    if (c->mlp_p.ensure(kMlpParams) != hipSuccess || c->mlp_m.ensure(kMlpParams) != hipSuccess ||
        c->mlp_v.ensure(kMlpParams) != hipSuccess || c->mlp_g.ensure(kMlpParams + 1) != hipSuccess ||
        c->mlp_pb.ensure(kMlpBf16) != hipSuccess)
        return fail(GM_ENOMEM, "network buffers");
    return GM_OK;
}

gm_status gm_mlp_set_params(gm_ctx *c, const float *params)
{
    if (!c || !params) return fail(GM_EINVAL, "NULL argument");
    for (int i = 0; i < kMlpParams; ++i)
        if (!std::isfinite(params[i])) return fail(GM_EINVAL, "parameter %d not finite", i);
    gm_status s = set_device(c);
    if (s == GM_OK) s = mlp_buffers(c);
    if (s != GM_OK) return s;
    HIPCHK(hipMemcpyAsync(c->mlp_p.p, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemsetAsync(c->mlp_m.p, 0, kMlpParams * sizeof(float), c->stream));
    HIPCHK(hipMemsetAsync(c->mlp_v.p, 0, kMlpParams * sizeof(float), c->stream));
    mlp_sync_bf16_kernel<<<(kMlpBf16 + 255) / 256, 256, 0, c->stream>>>(c->mlp_p.p, c->mlp_pb.p);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->mlp_t = 0;
    c->mlp_ready = true;
    return GM_OK;
}

gm_status gm_mlp_set_loss(gm_ctx *c, int kind)
{
    if (!c) return fail(GM_EINVAL, "NULL context");
    if (kind != GM_MLP_SQUARED && kind != GM_MLP_POISSON) return fail(GM_EINVAL, "loss kind %d", kind);
    c->mlp_loss = kind;
    return GM_OK;
}

gm_status gm_mlp_get_params(gm_ctx *c, float *params)
{
    if (!c || !params) return fail(GM_EINVAL, "NULL argument");
    if (!c->mlp_ready) return fail(GM_ESTATE, "network parameters not set");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    HIPCHK(hipMemcpyAsync(params, c->mlp_p.p, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return GM_OK;
}

gm_status gm_mlp_forward(gm_ctx *c, const float *X, int64_t n, float *Y)
{
    if (!c || (n > 0 && (!X || !Y)) || n < 0) return fail(GM_EINVAL, "bad argument");
    if (!c->mlp_ready) return fail(GM_ESTATE, "network parameters not set");
    if (n == 0) return GM_OK;
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    MlpArgs M{};
    M.X = X; M.Y = Y; M.n = n; M.P = c->mlp_p.p; M.Pb = c->mlp_pb.p;
    const long long rows_per_block = 16LL * kMlpWaves;
    mlp_forward_kernel<<<(unsigned)((n + rows_per_block - 1) / rows_per_block), 64 * kMlpWaves, 0, c->stream>>>(M);
    HIPCHK(hipGetLastError());
    return GM_OK;
}

// Gradient (and loss) of the weighted squared loss over n rows into mlp_g.
// The gradient of the loss over n rows into c->mlp_g (loss in its last
// entry); with adam, the same launches end in that Adam step of the FP32
// master and the BF16 copy.
static gm_status mlp_gradient(gm_ctx *c, const float *X, const float *T, const float *C, int64_t n,
                              const AdamArgs *adam = nullptr)
{
    const long long nb = (n + kMlpGradRows - 1) / kMlpGradRows;
    if (c->mlp_gpart.ensure((size_t)nb * (kMlpParams + 1)) != hipSuccess) return fail(GM_ENOMEM, "gradient partials");
    MlpArgs M{};
    M.X = X; M.T = T; M.C = C; M.n = n; M.P = c->mlp_p.p; M.Pb = c->mlp_pb.p;
    M.gpart = c->mlp_gpart.p; M.loss_scale = 1.0f; M.loss_kind = c->mlp_loss;
    mlp_grad_kernel<<<(unsigned)nb, 64 * kMlpGradWaves, 0, c->stream>>>(M);
    HIPCHK(hipGetLastError());
    if (adam)
        mlp_reduce_adam_kernel<<<kMlpReduceBlocks, 256, 0, c->stream>>>(c->mlp_gpart.p, (int)nb, c->mlp_g.p, *adam);
    else
        mlp_reduce_kernel<<<kMlpReduceBlocks, 256, 0, c->stream>>>(c->mlp_gpart.p, (int)nb, c->mlp_g.p);
    HIPCHK(hipGetLastError());
    return GM_OK;
}

gm_status gm_mlp_grad(gm_ctx *c, const float *X, const float *T, const float *C, int64_t n, float *grad,
                      float *loss)
{
    if (!c || !X || !T || !C || n <= 0 || n > (1LL << 31)) return fail(GM_EINVAL, "bad argument");
    if (!c->mlp_ready) return fail(GM_ESTATE, "network parameters not set");
    gm_status s = set_device(c);
    if (s == GM_OK) s = mlp_gradient(c, X, T, C, n);
    if (s != GM_OK) return s;
    if (grad) HIPCHK(hipMemcpyAsync(grad, c->mlp_g.p, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    if (loss) HIPCHK(hipMemcpyAsync(loss, c->mlp_g.p + kMlpParams, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return GM_OK;
}

gm_status gm_mlp_grad_noalloc(gm_ctx *c, const float *X, const float *T, const float *C, int64_t n,
                              float *grad_loss)
{
    if (!c || !X || !T || !C || !grad_loss || n <= 0) return fail(GM_EINVAL, "bad argument");
    if (n > kNoAllocMaxRows)
        return fail(GM_EINVAL, "%lld rows exceed the %lld rows of the fixed scratch (%zu MiB)", (long long)n,
                    kNoAllocMaxRows, kScratchFloats * sizeof(float) >> 20);
    if (!c->mlp_ready) return fail(GM_ESTATE, "network parameters not set");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    const long long nb = (n + kMlpGradRows - 1) / kMlpGradRows;
    MlpArgs M{};
    M.X = X; M.T = T; M.C = C; M.n = n; M.P = c->mlp_p.p; M.Pb = c->mlp_pb.p;
    M.gpart = c->scratch; M.loss_scale = 1.0f; M.loss_kind = c->mlp_loss;
    // every block writes all of its partial (no clearing needed)
    mlp_grad_kernel<<<(unsigned)nb, 64 * kMlpGradWaves, 0, c->stream>>>(M);
    HIPCHK(hipGetLastError());
    mlp_reduce_kernel<<<kMlpReduceBlocks, 256, 0, c->stream>>>(c->scratch, (int)nb, grad_loss);
    HIPCHK(hipGetLastError());
    return GM_OK;
}

gm_status gm_mlp_train_step(gm_ctx *c, const float *X, const float *T, const float *C, int64_t n, float lr,
                            float *loss)
{
    if (!c || !X || !T || !C || n <= 0 || n > (1LL << 31) || !(lr > 0.0f)) return fail(GM_EINVAL, "bad argument");
    if (!c->mlp_ready) return fail(GM_ESTATE, "network parameters not set");
    gm_status s = set_device(c);
    if (s != GM_OK) return s;
    AdamArgs A{};
    A.P = c->mlp_p.p; A.m = c->mlp_m.p; A.v = c->mlp_v.p; A.g = c->mlp_g.p; A.Pb = c->mlp_pb.p;
    A.lr = lr; A.beta1 = 0.9f; A.beta2 = 0.999f; A.eps = 1e-8f;
    A.bc1 = (float)(1.0 - std::pow(0.9, (double)(c->mlp_t + 1)));
    A.bc2 = (float)(1.0 - std::pow(0.999, (double)(c->mlp_t + 1)));
    s = mlp_gradient(c, X, T, C, n, &A);
    if (s != GM_OK) return s;
    c->mlp_t += 1;
    if (loss) {
        HIPCHK(hipMemcpyAsync(loss, c->mlp_g.p + kMlpParams, sizeof(float), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return GM_OK;
}

gm_status gm_mlp_train_steps(gm_ctx *c, const float *X, const float *T, const float *C, int64_t n, int64_t b,
                             int steps, float lr0, float decay, float *loss_first_last)
{
    if (!c || !X || !T || !C || n <= 0 || n > (1LL << 31) || b < 1 || b > n || steps < 1 || !(lr0 > 0.0f) ||
        !(decay > 0.0f))
        return fail(GM_EINVAL, "bad argument");
    const int64_t per_pass = n / b;
    for (int st = 0; st < steps; ++st) {
        const int64_t k = st % per_pass;
        // the learning rate of step st, as the single steps' caller forms it
        const float lr = (float)((double)lr0 * std::pow((double)decay, (double)st / (double)steps));
        float *loss = nullptr;
        if (loss_first_last && (st == 0 || st == steps - 1)) loss = loss_first_last + (st == 0 ? 0 : 1);
        gm_status s = gm_mlp_train_step(c, X + k * b * kMlpXStride, T + k * b * kMlpOut, C + k * b * kMlpOut, b, lr,
                                        loss);
        if (s != GM_OK) return s;
    }
    return GM_OK;
}

}  // extern "C"
