// lb2d_api.cpp -- host runtime behind the C ABI of include/lb2d.h.
//
// Holds the command state of one lattice (the paper's command API, Sec.
// "Commands"), checks the ordering rules the paper states, lays the
// caller-owned workspace out, and drives the gfx950 kernels on the bound
// stream (HIP graphs for the time loop).
#include "lb2d.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lb2d_common.hpp"
#include "lb2d_kernels.hpp"

using namespace lb2d;

namespace {

constexpr int kGraphSteps = 60;  // steps per captured graph
static_assert(kGraphSteps % 2 == 0 && kGraphSteps % kMultiSteps == 0,
              "graphs start and end at the same parity and hold whole multi-step launches");
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Circle {
    int xc, yc;
    double r;
};
struct Rect {
    int x0, x1, y0, y1;
};
// One obstacle command in order (0 circle, 1 rectangle, 2 host mask) with
// the reflected share R of its solids per component.
struct ObstacleOp {
    int kind, index;
    double R[2];
};

}  // namespace

struct lb2d_ctx {
    int device = 0;
    std::string err;
    // command state
    bool have_lattice = false, have_fluids = false, have_solute = false;
    bool have_style = false, have_force = false, bound = false;
    int nx = 0, ny = 0, ncomp = 1;
    double tau[2] = {1.0, 1.0}, alpha[2] = {4.0 / 9.0, 4.0 / 9.0};
    double force[2][2] = {{0, 0}, {0, 0}}, accel[2][2] = {{0, 0}, {0, 0}};
    bool inter = false;
    double G = 0.0;
    double psi0 = 0.0, psi_rho0 = 1.0;  // one-component interforce psi
    double psi0a = 0.0, rho0a = 1.0;  // one-component adhesiveforce psi
    bool ads[2] = {false, false};
    double Gads[2] = {0.0, 0.0};
    int q = 0;
    double tau_s = 1.0;
    bool isol = false;               // intersolute command
    double is_G = 0.0, is_psi0 = 0.0, is_C0 = 1.0;
    std::vector<SoluteOpen> sopens;  // solute openings
    bool reaction = false;
    double kr = 0, Cs = 0, b0 = 0, bmax = 0;
    uint64_t seed = 0;
    std::vector<Circle> circles;
    std::vector<Rect> rects;
    std::vector<std::vector<uint8_t>> host_masks;
    std::vector<double> rho0[2], ux0[2], uy0[2];
    std::vector<double> C0, Cux, Cuy;
    int storage = kF32;
    bool storage_chosen = false;
    bool sr = false;          // stochastic rounding of 16-bit storage
    unsigned sr_seed = 0;
    // device
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    void *f[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    void *g[2] = {nullptr, nullptr};
    uint8_t *mask = nullptr, *trig = nullptr;
    uint16_t *links = nullptr;
    double *b = nullptr, *staging = nullptr, *partial = nullptr, *gpartial = nullptr;
    double *totals = nullptr;
    long long *dstep = nullptr;
    unsigned *gflag = nullptr;
    uint8_t *gseg = nullptr;  // two flag rows of growth_segments(nx, ny) bytes
    size_t staging_doubles = 0;
    double rho_ref[2] = {1.0, 1.0};
    int64_t t = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // kGraphSteps steps, by the parity they start at
    std::map<int, hipGraphExec_t> tail_graphs;      // fewer steps, by 2 x count + start parity
    // population plane geometry: brick layout, padded to whole bricks
    unsigned pnx = 0;
    size_t pplane = 0;
    // timing
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double kernel_ms = 0.0;
    int64_t kernel_launches = 0;

    int fail(int code, const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    size_t n() const { return (size_t)nx * ny; }
    std::vector<OpenSpec> opens;  // momentum openings
    int bstyle = 0;               // boundary_style: 0 noslip, 1 slip, 2 mixed, 3 hybrid
    double style_R[2] = {0.0, 0.0};  // R given to the next obstacles
    double grow_R = 0.0;             // R of solids made by growth
    std::vector<ObstacleOp> oops;
    double *refl_dev = nullptr;
    bool slip_any() const {
        if (grow_R > 0.0) return true;
        for (const auto &o : oops)
            if (o.R[0] > 0.0 || o.R[1] > 0.0) return true;
        return false;
    }
    bool plain() const {
        return ncomp == 1 && q == 0 && !inter && !ads[0] && !ads[1] && opens.empty() && !slip_any();
    }
    bool has_gradient() const {
        for (const auto &o : opens)
            if (o.style == 4) return true;
        return false;
    }
    bool sc() const { return inter; }  // cohesion: two components, or psi form
};

struct lb2d_batch {
    int device = 0;
    std::string err;
    std::vector<lb2d_ctx *> lat;
    bool final_ = false;
    int storage = kF32;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    PlainLattice *d_lat = nullptr;
    Tile *d_tiles = nullptr;
    size_t max_tiles = 0;
    int ntiles = 0;
    int tile_w = 64, tile_h = 4, schedule = 0, bpc = 0, grid = 0;
    bool multi = false;    // the chosen tiles are the multi-step kernel's
    // one-step tiles of the storage's default shape, lattice by lattice, for
    // the leftover steps when the multi-step kernel was chosen
    Tile *d_tiles1 = nullptr;
    int ntiles1 = 0, tile_w1 = 64, tile_h1 = 4;
    size_t max_plane = 0;  // largest population plane of the lattices
    bool nt = false;       // streaming stores: the lattices' populations exceed the last-level cache
    bool sr = false;       // stochastic rounding (every lattice of the batch asked for it)
    unsigned long long *d_step = nullptr;  // device step count shared by the lattices (stochastic rounding)
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // kGraphSteps steps, by start parity
    int64_t t = 0;
    // the autotuner's trials: tile width, height, schedule, blocks per CU
    // and milliseconds per step (empty when the choice came from a cache)
    std::vector<std::array<double, 5>> trials;
    int fail(int code, const char *fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
};

namespace {

#define HIPCHK(ctx, call)                                                                 \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) return (ctx)->fail(LB2D_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool is_nan(double v) { return std::isnan(v); }

// Workspace layout of one lattice.
struct Layout {
    size_t f[2][2], g[2], mask, trig, links, b, staging, partial, gpartial, totals, dstep, gflag, gseg, refl, total;
    size_t staging_doubles;
};

// Padded plane geometry of the populations for the given storage.
void plane_geometry(const lb2d_ctx *c, int storage, unsigned *pnx, size_t *pplane) {
    const unsigned bh = (unsigned)brick_h_for((int)storage_bytes(storage));
    const unsigned bw = (unsigned)brick_w_for((int)storage_bytes(storage));
    const unsigned px = (unsigned)((c->nx + bw - 1) / bw * bw);
    const unsigned py = (unsigned)((c->ny + bh - 1) / bh * bh);
    *pnx = px;
    *pplane = (size_t)px * py;
}

Layout make_layout(const lb2d_ctx *c, int storage) {
    Layout L{};
    const size_t n = c->n();
    unsigned pnx;
    size_t pplane;
    plane_geometry(c, storage, &pnx, &pplane);
    const size_t pop = align_up(9 * pplane * storage_bytes(storage));
    size_t off = 0;
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < 2; ++k) {
            L.f[p][k] = (k < c->ncomp) ? off : (size_t)-1;
            if (k < c->ncomp) off += pop;
        }
    for (int p = 0; p < 2; ++p) {
        // solute: q brick-layout planes
        L.g[p] = c->q ? off : (size_t)-1;
        if (c->q) off += align_up((size_t)c->q * pplane * storage_bytes(storage));
    }
    L.mask = off;
    off += align_up(n);
    L.trig = off;
    off += align_up(n);
    // 16-bit link words; the region is padded to whole 32-bit words (the
    // growth kernel updates them with 32-bit atomic ORs)
    L.links = off;
    off += align_up(2 * n + 2);
    L.b = off;
    if (c->reaction) off += align_up(n * 8);
    // staging: 3 doubles per node (host transfers, read-outs, budgets,
    // shape tables)
    size_t sd = 3 * n;
    const size_t shapes = 2 * c->circles.size() + c->circles.size() + 2 * c->rects.size() + 16;
    sd = std::max(sd, shapes + (size_t)c->ny * 8 + 64);
    L.staging_doubles = sd;
    L.staging = off;
    off += align_up(sd * 8);
    L.partial = off;
    off += align_up((size_t)full_slots(c->nx, c->ny) * 4 * 8);
    L.gpartial = off;
    off += align_up((size_t)growth_blocks(c->nx, c->ny) * 4 * 8);
    L.totals = off;
    off += align_up(16 * 8);
    L.dstep = off;
    off += align_up(8);
    L.gflag = off;
    off += align_up(8);
    L.gseg = off;
    off += align_up(2 * (size_t)growth_segments(c->nx, c->ny));
    // reflected shares of slip/mixed solids, per component
    L.refl = off;
    if (c->slip_any()) off += align_up((size_t)c->ncomp * n * 8);
    L.total = off;
    return L;
}

// Bytes of all population buffers of a bound lattice (both parities, every
// fluid component and the solute).
static size_t population_bytes(const lb2d_ctx *c) {
    return 2ull * (size_t)(c->ncomp + (c->q ? 1 : 0)) * 9ull * c->pplane * storage_bytes(c->storage);
}
// Streaming stores once the populations no longer fit in the last-level
// cache (measured: plain stores win while the next step can find the
// populations there).
static bool stream_stores(const lb2d_ctx *c) { return population_bytes(c) > kLastLevelCache; }

FullParams full_params(const lb2d_ctx *c) {
    FullParams p{};
    for (int pp = 0; pp < 2; ++pp) {
        for (int k = 0; k < 2; ++k) p.f[pp][k] = c->f[pp][k];
        p.g[pp] = c->g[pp];
    }
    p.mask = c->mask;
    p.links = c->links;
    p.trig = c->trig;
    p.b = c->b;
    p.partial = c->partial;
    p.gpartial = c->gpartial;
    p.totals = c->totals;
    p.dstep = c->dstep;
    p.gflag = c->gflag;
    p.gseg[0] = c->gseg;
    p.gseg[1] = c->gseg + growth_segments(c->nx, c->ny);
    p.nx = c->nx;
    p.ny = c->ny;
    p.ncomp = c->ncomp;
    StepCoef<double> &k8 = p.cd;
    for (int k = 0; k < 2; ++k) {
        k8.tau[k] = c->tau[k];
        k8.omega[k] = 1.0 / c->tau[k];
        k8.A0[k] = 2.25 * c->alpha[k];
        k8.A1[k] = 1.8 * (1.0 - c->alpha[k]);
        k8.rho_ref[k] = c->rho_ref[k];
        for (int d = 0; d < 2; ++d) {
            k8.force[k][d] = c->force[k][d];
            k8.accel[k][d] = c->accel[k][d];
        }
        k8.Gads[k] = c->ads[k] ? c->Gads[k] : 0.0;
    }
    k8.G = c->inter ? c->G : 0.0;
    k8.psi0 = c->psi0;
    k8.rho0 = c->psi_rho0;
    k8.psi0a = c->psi0a;
    k8.rho0a = c->rho0a;
    p.has_ads = (c->ads[0] || c->ads[1]) ? 1 : 0;
    p.ads_psi = (c->ncomp == 1 && c->ads[0]) ? 1 : 0;
    p.psi = (c->ncomp == 1 && c->inter) ? 1 : 0;
    k8.omega_s = c->q ? 1.0 / c->tau_s : 0.0;
    p.sxper = p.syper = 1;
    p.nsopen = (int)c->sopens.size();
    for (int k = 0; k < p.nsopen; ++k) {
        p.sopen[k] = c->sopens[k];
        if (c->sopens[k].wall < 2) p.sxper = 0;
        else p.syper = 0;
    }
    k8.Dsol = c->q ? (c->q == 4 ? 0.5 : 1.0 / 3.0) * (c->tau_s - 0.5) : 0.0;
    k8.Cs = c->Cs;
    p.slip = c->refl_dev ? 1 : 0;
    for (int k = 0; k < 2; ++k) {
        p.refl[k] = (c->refl_dev && k < c->ncomp) ? c->refl_dev + (size_t)k * c->n() : nullptr;
        p.grow_R[k] = c->grow_R;
    }
    p.isol = c->isol ? 1 : 0;
    p.is_G = c->is_G;
    p.is_psi0 = c->is_psi0;
    p.is_C0 = c->is_C0;
    p.tau_s = c->tau_s;
    p.sr = c->sr ? 1 : 0;
    p.sr_seed = c->sr_seed;
    p.nopen = (int)c->opens.size();
    for (int k = 0; k < p.nopen; ++k) p.open[k] = c->opens[k];
    // per-link rate k_i = kr w_i / W (W = 1/6 for D2Q9, 1/4 for D2Q4: the
    // links of a flat wall add up to kr); a link's deposit is
    // 2 k_i / (2 w_i + k_i) (g_out - w_i Cs).  D2Q4 has no diagonal links.
    p.sq = c->q;
    const double wa = c->q == 4 ? 0.25 : 1.0 / 9.0, wd = 1.0 / 36.0;
    const double iW = c->q == 4 ? 4.0 : 6.0;
    const double ka = c->kr * wa * iW, kd = c->kr * wd * iW;
    k8.rlink[0] = 2.0 * ka / (2.0 * wa + ka);
    k8.rlink[1] = 2.0 * kd / (2.0 * wd + kd);
    k8.rlink_cs[0] = k8.rlink[0] * wa * c->Cs;
    k8.rlink_cs[1] = k8.rlink[1] * wd * c->Cs;
    // FP32 copy (each value rounded once)
    StepCoef<float> &k4 = p.cf;
    for (int k = 0; k < 2; ++k) {
        k4.tau[k] = (float)k8.tau[k];
        k4.omega[k] = (float)k8.omega[k];
        k4.A0[k] = (float)k8.A0[k];
        k4.A1[k] = (float)k8.A1[k];
        k4.rho_ref[k] = (float)k8.rho_ref[k];
        for (int d = 0; d < 2; ++d) {
            k4.force[k][d] = (float)k8.force[k][d];
            k4.accel[k][d] = (float)k8.accel[k][d];
        }
        k4.Gads[k] = (float)k8.Gads[k];
        k4.rlink[k] = (float)k8.rlink[k];
        k4.rlink_cs[k] = (float)k8.rlink_cs[k];
    }
    k4.G = (float)k8.G;
    k4.Dsol = (float)k8.Dsol;
    k4.psi0 = (float)k8.psi0;
    k4.rho0 = (float)k8.rho0;
    k4.psi0a = (float)k8.psi0a;
    k4.rho0a = (float)k8.rho0a;
    k4.omega_s = (float)k8.omega_s;
    k4.Cs = (float)k8.Cs;
    p.b0 = c->b0;
    p.bmax = c->bmax;
    p.seed = c->seed;
    p.nblk_main = full_slots(c->nx, c->ny);
    p.nblk_grow = growth_blocks(c->nx, c->ny);
    p.pnx = c->pnx;
    p.pplane = c->pplane;
    return p;
}

PlainLattice plain_lattice(const lb2d_ctx *c) {
    PlainLattice L{};
    L.f[0] = c->f[0][0];
    L.f[1] = c->f[1][0];
    L.links = c->links;
    L.nx = c->nx;
    L.ny = c->ny;
    L.pnx = c->pnx;
    L.plane = c->pplane;
    L.tau = c->tau[0];
    L.omega = 1.0 / c->tau[0];
    L.Fx = c->force[0][0];
    L.Fy = c->force[0][1];
    L.ax = c->accel[0][0];
    L.ay = c->accel[0][1];
    L.rho_ref = c->rho_ref[0];
    L.omega_f = (float)L.omega;
    L.tau_f = (float)L.tau;
    L.Fx_f = (float)L.Fx;
    L.Fy_f = (float)L.Fy;
    L.ax_f = (float)L.ax;
    L.ay_f = (float)L.ay;
    L.rho_ref_f = (float)L.rho_ref;
    L.step = (const unsigned long long *)c->dstep;
    L.seed = c->sr_seed;
    return L;
}

int check_ctx(lb2d_ctx *c) { return c ? LB2D_OK : LB2D_E_INVAL; }

int pre_command(lb2d_ctx *c, bool need_lattice = true) {
    if (!c) return LB2D_E_INVAL;
    if (c->bound) return c->fail(LB2D_E_STATE, "commands must come before lb2d_bind");
    if (need_lattice && !c->have_lattice) return c->fail(LB2D_E_ORDER, "the lattice command must come first");
    return LB2D_OK;
}

// One step on the stream `s` at the given parity; k: its offset in the launch group, tick: steps to add to the
// device step counter after it (stochastic rounding keys its stream on it).
hipError_t enqueue_step(lb2d_ctx *c, int parity, int k, int tick, hipStream_t s) {
    if (c->plain()) {
        hipError_t e = launch_plain(c->storage, plain_lattice(c), parity, c->sr, stream_stores(c), k, s);
        if (e == hipSuccess && c->sr && tick) e = launch_tick((unsigned long long *)c->dstep, tick, s);
        return e;
    }
    const FullParams p = full_params(c);
    hipError_t e = launch_full(c->storage, p, parity, c->sc(), c->reaction, s);
    if (e == hipSuccess && c->has_gradient()) e = launch_open_gradient(c->storage, p, parity ^ 1, s);
    if (e != hipSuccess) return e;
    if (c->q) e = launch_growth(c->storage, p, parity ^ 1, c->reaction, s);
    else if (c->sr) e = launch_tick((unsigned long long *)c->dstep, 1, s);
    return e;
}

// The launches of `len` steps from a step of parity p0 (the state is in
// buffer p0).  The one-fluid step on a lattice that satisfies multi_fits
// runs as multi-step launches (each p -> p^1, multi_steps() steps ahead),
// then single steps; the device step counter (read only by stochastic
// rounding) advances once, after the last of them.
hipError_t enqueue_group(lb2d_ctx *c, int len, int p0, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (!c->plain()) {
        for (int k = 0; k < len && e == hipSuccess; ++k) e = enqueue_step(c, (p0 + k) & 1, k, 0, s);
        return e;
    }
    const PlainLattice L = plain_lattice(c);
    const bool nt = stream_stores(c);
    int k = 0;
    const int ms = multi_steps();
    if (multi_fits(c->storage, c->nx, c->ny))
        for (; k + ms <= len && e == hipSuccess; k += ms)
            e = launch_plain_ms(c->storage, L, (p0 + k) & 1, c->sr, nt, k, s);
    for (; k < len && e == hipSuccess; ++k) e = launch_plain(c->storage, L, (p0 + k) & 1, c->sr, nt, k, s);
    if (e == hipSuccess && c->sr && len > 0) e = launch_tick((unsigned long long *)c->dstep, len, s);
    return e;
}

// The launch graph of `len` steps starting at a step of parity p0 (len <=
// kGraphSteps; captured once per length and parity and kept until
// lb2d_destroy).
int build_graph(lb2d_ctx *c, int len, int p0, hipGraphExec_t *out) {
    hipGraphExec_t &g = len == kGraphSteps ? c->graph[p0] : c->tail_graphs[2 * len + p0];
    if (g) {
        *out = g;
        return LB2D_OK;
    }
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t gr = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipError_t e = enqueue_group(c, len, p0, c->cap_stream);
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &gr);
    if (e != hipSuccess) return c->fail(LB2D_E_HIP, "graph capture: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return c->fail(LB2D_E_HIP, "graph capture end: %s", hipGetErrorString(e2));
    HIPCHK(c, hipGraphInstantiate(&g, gr, nullptr, nullptr, 0));
    HIPCHK(c, hipGraphDestroy(gr));
    // upload the executable graph now, so that its first launch costs what
    // every later one does
    HIPCHK(c, hipGraphUpload(g, c->stream));
    *out = g;
    return LB2D_OK;
}

// How lb2d_iteration splits nsteps from step t: whole graphs of
// kGraphSteps, then one graph of the remaining steps (a single launch for
// one step); every graph of the call starts at the parity of t, since
// kGraphSteps is even.
struct StepPlan {
    int64_t graphs, tail;
    int p0;
};
StepPlan step_plan(int64_t t, int64_t nsteps) {
    StepPlan q{};
    q.graphs = nsteps / kGraphSteps;
    q.tail = nsteps % kGraphSteps;
    q.p0 = (int)(t & 1);
    return q;
}

int upload(lb2d_ctx *c, double *dst, const std::vector<double> &src, double fill) {
    const size_t n = c->n();
    if (src.empty()) {
        HIPCHK(c, launch_fill_f64(dst, fill, n, c->stream));
    } else {
        HIPCHK(c, hipMemcpyAsync(dst, src.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    }
    return LB2D_OK;
}

double mean_of(const std::vector<double> &v) {
    double s = 0.0;
    for (double x : v) s += x;
    return v.empty() ? 1.0 : s / (double)v.size();
}

}  // namespace

namespace {

struct TuneCand {
    int w, h, sched, bpc;
};

// schedule 0: lattice by lattice; 1: largest lattices first; 2: tiles of
// all lattices interleaved round-robin.
std::vector<Tile> make_tiles(const lb2d_batch *b, int w, int h, int sched) {
    std::vector<int> order(b->lat.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    if (sched == 1)
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int c) { return b->lat[a]->n() > b->lat[c]->n(); });
    std::vector<std::vector<Tile>> per(b->lat.size());
    for (int k : order) {
        const lb2d_ctx *c = b->lat[k];
        for (int y0 = 0; y0 < c->ny; y0 += h)
            for (int x0 = 0; x0 < c->nx; x0 += w) per[k].push_back({k, x0, y0, 0});
    }
    std::vector<Tile> out;
    if (sched == 2) {
        size_t mx = 0;
        for (auto &v : per) mx = std::max(mx, v.size());
        for (size_t i = 0; i < mx; ++i)
            for (int k : order)
                if (i < per[k].size()) out.push_back(per[k][i]);
    } else {
        for (int k : order) out.insert(out.end(), per[k].begin(), per[k].end());
    }
    return out;
}

int batch_grid(int ntiles, int bpc, int cus) {
    if (bpc <= 0) return ntiles;
    return std::min(ntiles, bpc * cus);
}

std::string batch_key(const lb2d_batch *b) {
    unsigned long long h = 1469598103934665603ull;
    auto mix = [&](unsigned long long v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    mix(b->lat.size());
    mix(b->storage);
    for (auto *c : b->lat) {
        mix(c->nx);
        mix(c->ny);
    }
    char buf[32];
    snprintf(buf, sizeof(buf), "%016llx", h);
    return buf;
}

}  // namespace

// Scratch of lb2d_budgets_noalloc (for callers that cannot allocate device
// memory): the per-row partials, the eight sums and the tally totals of one
// budget reduction, in a file-scope device array of 4 MiB that every GPU the
// library runs on holds until the process ends (lattices of up to 65533
// rows).  Host code uses the array only through the device address that
// hipGetSymbolAddress returns, once per device, with that device current.
namespace {
constexpr size_t kBudgetScratchDoubles = (size_t)1 << 19;
static __device__ __align__(256) double scratch[kBudgetScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the context's (current) device.
int budget_scratch(lb2d_ctx *c, double **out) {
    if (c->device >= kMaxDevices) return c->fail(LB2D_E_INVAL, "device %d beyond %d", c->device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[c->device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return c->fail(LB2D_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch[c->device] = (double *)ptr;
    }
    *out = g_scratch[c->device];
    return LB2D_OK;
}
}  // namespace

// ======================================================================
extern "C" {

int lb2d_create(lb2d_ctx **out, int hip_device) {
    if (!out) return LB2D_E_INVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    if (hip_device < 0 || (ndev > 0 && hip_device >= ndev)) return LB2D_E_INVAL;
    lb2d_ctx *c = new lb2d_ctx();
    c->device = hip_device;
    *out = c;
    return LB2D_OK;
}

int lb2d_destroy(lb2d_ctx *c) {
    if (!c) return LB2D_E_INVAL;
    // work still queued on the bound stream reads the caller's workspace:
    // finish it before the caller may free that memory
    if (c->bound) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
    }
    if (c->graph[0] || c->graph[1] || c->cap_stream || c->ev0 || !c->tail_graphs.empty()) {
        (void)hipSetDevice(c->device);
        for (hipGraphExec_t g : c->graph)
            if (g) (void)hipGraphExecDestroy(g);
        for (auto &kv : c->tail_graphs)
            if (kv.second) (void)hipGraphExecDestroy(kv.second);
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
        if (c->ev0) (void)hipEventDestroy(c->ev0);
        if (c->ev1) (void)hipEventDestroy(c->ev1);
    }
    delete c;
    return LB2D_OK;
}

const char *lb2d_last_error(const lb2d_ctx *c) {
    if (!c) return "null context";
    return c->err.c_str();
}

int lb2d_lattice(lb2d_ctx *c, const char *style, int nx, int ny, double tau) {
    int rc = pre_command(c, false);
    if (rc) return rc;
    if (c->have_lattice) return c->fail(LB2D_E_ORDER, "lattice given twice");
    if (!style || std::strcmp(style, "d2q9") != 0)
        return c->fail(LB2D_E_UNSUPPORTED, "lattice style must be \"d2q9\"");
    if (nx < 3 || ny < 3) return c->fail(LB2D_E_INVAL, "lattice needs at least 3x3 nodes");
    if ((double)nx * (double)ny > 4.0e9) return c->fail(LB2D_E_SIZE, "lattice too large");
    if (!(tau > 0.5)) return c->fail(LB2D_E_INVAL, "tau must exceed 1/2");
    c->nx = nx;
    c->ny = ny;
    c->tau[0] = c->tau[1] = tau;
    c->have_lattice = true;
    return LB2D_OK;
}

int lb2d_fluids(lb2d_ctx *c, double tau1, double tau2, double alpha1, double alpha2) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (c->have_fluids) return c->fail(LB2D_E_ORDER, "fluids given twice");
    if (!c->opens.empty()) return c->fail(LB2D_E_ORDER, "fluids must precede the momentum openings");
    if (c->have_force || !c->rho0[0].empty())
        return c->fail(LB2D_E_ORDER, "fluids must precede forces and initial fields");
    if (!(tau1 > 0.5) || !(tau2 > 0.5)) return c->fail(LB2D_E_INVAL, "tau1, tau2 must exceed 1/2");
    if (is_nan(alpha1)) alpha1 = 4.0 / 9.0;
    if (is_nan(alpha2)) alpha2 = 4.0 / 9.0;
    if (!(alpha1 >= 0.0 && alpha1 < 1.0) || !(alpha2 >= 0.0 && alpha2 < 1.0))
        return c->fail(LB2D_E_INVAL, "alpha must lie in [0, 1)");
    c->ncomp = 2;
    c->tau[0] = tau1;
    c->tau[1] = tau2;
    c->alpha[0] = alpha1;
    c->alpha[1] = alpha2;
    c->have_fluids = true;
    return LB2D_OK;
}

int lb2d_solute(lb2d_ctx *c, double tau_s, int q) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (c->have_solute) return c->fail(LB2D_E_ORDER, "solute given twice");
    if (q != 9 && q != 4) return c->fail(LB2D_E_INVAL, "solute lattice must be 9 (D2Q9) or 4 (D2Q4)");
    if (!(tau_s > 0.5)) return c->fail(LB2D_E_INVAL, "tau_s must exceed 1/2");
    c->q = q;
    c->tau_s = tau_s;
    c->have_solute = true;
    return LB2D_OK;
}

int lb2d_intersolute(lb2d_ctx *c, double G, double psi0, double C0) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (!c->have_solute) return c->fail(LB2D_E_ORDER, "intersolute needs the solute command first");
    if (!std::isfinite(G) || !std::isfinite(psi0)) return c->fail(LB2D_E_INVAL, "G and psi0 must be finite");
    if (!(C0 > 0.0) || !std::isfinite(C0)) return c->fail(LB2D_E_INVAL, "C0 must be positive");
    c->isol = true;
    c->is_G = G;
    c->is_psi0 = psi0;
    c->is_C0 = C0;
    return LB2D_OK;
}

// Node range overlap of two openings on the box edge: same wall and
// overlapping ranges, or perpendicular walls that both hold their corner.
static bool openings_share_node(const lb2d_ctx *c, int w1, int lo1, int hi1, int w2, int lo2, int hi2) {
    if (w1 == w2) return lo1 <= hi2 && lo2 <= hi1;
    if ((w1 < 2) == (w2 < 2)) return false;  // opposite walls
    auto corner_in = [&](int w, int a, int b, int other) {
        const int k = (w < 2) ? (other == 2 ? 0 : c->ny - 1) : (other == 0 ? 0 : c->nx - 1);
        return a <= k && k <= b;
    };
    return corner_in(w1, lo1, hi1, w2) && corner_in(w2, lo2, hi2, w1);
}

int lb2d_solute_opening_range(lb2d_ctx *c, const char *wall, int lo, int hi, const char *kind, const char *style,
                              double value, double v) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (!c->have_solute) return c->fail(LB2D_E_ORDER, "solute openings need the solute command first");
    if (!wall || !style || !kind) return c->fail(LB2D_E_INVAL, "null wall, kind or style");
    SoluteOpen o{};
    if (!std::strcmp(wall, "xlo")) o.wall = 0;
    else if (!std::strcmp(wall, "xhi")) o.wall = 1;
    else if (!std::strcmp(wall, "ylo")) o.wall = 2;
    else if (!std::strcmp(wall, "yhi")) o.wall = 3;
    else return c->fail(LB2D_E_INVAL, "wall must be xlo, xhi, ylo or yhi");
    if (!std::strcmp(kind, "inlet")) o.outlet = 0;
    else if (!std::strcmp(kind, "outlet")) o.outlet = 1;
    else return c->fail(LB2D_E_INVAL, "kind must be inlet or outlet");
    if (!std::strcmp(style, "dirichlet")) o.style = 1;
    else if (!std::strcmp(style, "adiabatic")) o.style = 2;
    else if (!std::strcmp(style, "flux")) o.style = 3;
    else return c->fail(LB2D_E_INVAL, "style must be dirichlet, adiabatic or flux");
    const int len = o.wall < 2 ? c->ny : c->nx;
    if (lo < 0 || hi < lo || hi >= len) return c->fail(LB2D_E_INVAL, "opening range %d..%d outside 0..%d", lo, hi, len - 1);
    if (!std::isfinite(value) || !std::isfinite(v)) return c->fail(LB2D_E_INVAL, "opening values must be finite");
    if (o.style == 3 && !(v > 0.0)) return c->fail(LB2D_E_INVAL, "flux openings need v > 0");
    if (o.style == 3 && o.outlet) {
        // the outlet rule C = (v C0 - D C1)/(v - D) is singular at v = D
        const double D = (c->q == 4 ? 0.5 : 1.0 / 3.0) * (c->tau_s - 0.5);
        if (std::fabs(v - D) <= 1e-9 * std::max(v, D))
            return c->fail(LB2D_E_INVAL, "flux outlet with v equal to the diffusivity D = %g", D);
    }
    if ((int)c->sopens.size() >= kMaxOpen) return c->fail(LB2D_E_SIZE, "at most %d solute openings", kMaxOpen);
    for (const auto &q : c->sopens)
        if (openings_share_node(c, q.wall, q.lo, q.hi, o.wall, lo, hi))
            return c->fail(LB2D_E_INVAL, "two solute openings share a node");
    o.lo = lo;
    o.hi = hi;
    o.value = value;
    o.v = v;
    c->sopens.push_back(o);
    return LB2D_OK;
}

int lb2d_solute_opening(lb2d_ctx *c, const char *wall, const char *style, double value) {
    if (!c) return LB2D_E_INVAL;
    if (!wall || !style) return c->fail(LB2D_E_INVAL, "null wall or style");
    if (std::strcmp(wall, "xlo") && std::strcmp(wall, "xhi")) return c->fail(LB2D_E_INVAL, "wall must be xlo or xhi");
    if (!std::strcmp(style, "flux"))
        return c->fail(LB2D_E_INVAL, "flux openings need a velocity: use lb2d_solute_opening_range");
    return lb2d_solute_opening_range(c, wall, 0, c->have_lattice ? c->ny - 1 : 0,
                                     std::strcmp(wall, "xlo") ? "outlet" : "inlet", style, value, 0.0);
}

int lb2d_boundary_style(lb2d_ctx *c, const char *style, double R) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (!style) return c->fail(LB2D_E_INVAL, "null style");
    double v;
    if (!std::strcmp(style, "noslip")) {
        c->bstyle = 0;
        v = 0.0;
    } else if (!std::strcmp(style, "slip")) {
        c->bstyle = 1;
        v = 1.0;
    } else if (!std::strcmp(style, "mixed")) {
        if (!(R >= 0.0 && R <= 1.0)) return c->fail(LB2D_E_INVAL, "the mixed style needs 0 <= R <= 1");
        c->bstyle = 2;
        v = R;
    } else if (!std::strcmp(style, "hybrid")) {
        c->bstyle = 3;
        v = 0.0;
    } else {
        return c->fail(LB2D_E_INVAL, "unknown boundary style %s", style);
    }
    c->style_R[0] = c->style_R[1] = v;
    c->grow_R = c->bstyle == 3 ? 0.0 : v;
    c->have_style = true;
    return LB2D_OK;
}

int lb2d_obstacle_style(lb2d_ctx *c, int comp, const char *style, double R) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (c->bstyle != 3) return c->fail(LB2D_E_ORDER, "per-obstacle styles need boundary_style hybrid");
    if (comp < 0 || comp >= c->ncomp) return c->fail(LB2D_E_INVAL, "component %d does not exist", comp);
    if (!style) return c->fail(LB2D_E_INVAL, "null style");
    if (!std::strcmp(style, "noslip")) c->style_R[comp] = 0.0;
    else if (!std::strcmp(style, "slip")) c->style_R[comp] = 1.0;
    else if (!std::strcmp(style, "mixed")) {
        if (!(R >= 0.0 && R <= 1.0)) return c->fail(LB2D_E_INVAL, "the mixed style needs 0 <= R <= 1");
        c->style_R[comp] = R;
    } else {
        return c->fail(LB2D_E_INVAL, "style must be noslip, slip or mixed");
    }
    return LB2D_OK;
}

int lb2d_momentum_opening(lb2d_ctx *c, const char *wall, int lo, int hi, int comp, const char *kind,
                          const char *style, double v, double rho) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (!wall || !kind || !style) return c->fail(LB2D_E_INVAL, "null wall, kind or style");
    OpenSpec o{};
    if (!std::strcmp(wall, "xlo")) o.wall = 0;
    else if (!std::strcmp(wall, "xhi")) o.wall = 1;
    else if (!std::strcmp(wall, "ylo")) o.wall = 2;
    else if (!std::strcmp(wall, "yhi")) o.wall = 3;
    else return c->fail(LB2D_E_INVAL, "wall must be xlo, xhi, ylo or yhi");
    if (!std::strcmp(kind, "inlet")) o.outlet = 0;
    else if (!std::strcmp(kind, "outlet")) o.outlet = 1;
    else return c->fail(LB2D_E_INVAL, "kind must be inlet or outlet");
    if (!std::strcmp(style, "poiseuille")) o.style = 1;
    else if (!std::strcmp(style, "uniform")) o.style = 2;
    else if (!std::strcmp(style, "dirichlet")) o.style = 3;
    else if (!std::strcmp(style, "gradient")) o.style = 4;
    else return c->fail(LB2D_E_INVAL, "style must be poiseuille, uniform, dirichlet or gradient");
    if (comp < 0 || comp >= c->ncomp) return c->fail(LB2D_E_INVAL, "component %d does not exist", comp);
    const int len = o.wall < 2 ? c->ny : c->nx;
    if (lo < 0 || hi < lo || hi >= len) return c->fail(LB2D_E_INVAL, "opening range %d..%d outside 0..%d", lo, hi, len - 1);
    if (!(rho > 0.0) || !std::isfinite(rho)) return c->fail(LB2D_E_INVAL, "rho must be positive");
    if (!std::isfinite(v) || std::fabs(v) >= 1.0) return c->fail(LB2D_E_INVAL, "|v| must be below 1");
    if ((int)c->opens.size() >= kMaxOpen) return c->fail(LB2D_E_SIZE, "at most %d openings", kMaxOpen);
    // no node may belong to two openings of one component
    for (const auto &q : c->opens)
        if (q.comp == comp && openings_share_node(c, q.wall, q.lo, q.hi, o.wall, lo, hi))
            return c->fail(LB2D_E_INVAL, "two momentum openings of one component share a node");
    o.lo = lo;
    o.hi = hi;
    o.comp = comp;
    o.v = v;
    o.rho = rho;
    c->opens.push_back(o);
    return LB2D_OK;
}

int lb2d_rounding(lb2d_ctx *c, const char *mode, uint64_t seed) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (!mode) return c->fail(LB2D_E_INVAL, "null mode");
    if (!std::strcmp(mode, "nearest")) c->sr = false;
    else if (!std::strcmp(mode, "stochastic")) c->sr = true;
    else return c->fail(LB2D_E_INVAL, "rounding mode must be nearest or stochastic");
    c->sr_seed = (unsigned)(seed ^ (seed >> 32));
    return LB2D_OK;
}

int lb2d_obstacle_rect(lb2d_ctx *c, int x0, int x1, int y0, int y1) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (!c->have_style) return c->fail(LB2D_E_ORDER, "obstacle must follow boundary_style");
    if (x0 < 0 || y0 < 0 || x1 >= c->nx || y1 >= c->ny || x0 > x1 || y0 > y1)
        return c->fail(LB2D_E_INVAL, "rectangle outside the lattice or empty");
    c->rects.push_back({x0, x1, y0, y1});
    c->oops.push_back({1, (int)c->rects.size() - 1, {c->style_R[0], c->style_R[1]}});
    return LB2D_OK;
}

int lb2d_obstacle_circle(lb2d_ctx *c, int xc, int yc, double r) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (!c->have_style) return c->fail(LB2D_E_ORDER, "obstacle must follow boundary_style");
    if (xc < 0 || yc < 0 || xc >= c->nx || yc >= c->ny || !(r >= 0.0) || !std::isfinite(r))
        return c->fail(LB2D_E_INVAL, "circle centre outside the lattice or bad radius");
    c->circles.push_back({xc, yc, r});
    c->oops.push_back({0, (int)c->circles.size() - 1, {c->style_R[0], c->style_R[1]}});
    return LB2D_OK;
}

int lb2d_obstacle_mask(lb2d_ctx *c, const uint8_t *host_mask) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (!c->have_style) return c->fail(LB2D_E_ORDER, "obstacle must follow boundary_style");
    if (!host_mask) return c->fail(LB2D_E_INVAL, "null mask");
    c->host_masks.emplace_back(host_mask, host_mask + c->n());
    c->oops.push_back({2, (int)c->host_masks.size() - 1, {c->style_R[0], c->style_R[1]}});
    return LB2D_OK;
}

int lb2d_surface_reaction(lb2d_ctx *c, double kr, double Cs, const char *style, double b0, double bmax,
                          uint64_t seed) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (!c->have_solute) return c->fail(LB2D_E_ORDER, "surface_reaction needs the solute command first");
    if (!style || std::strcmp(style, "growth") != 0) return c->fail(LB2D_E_INVAL, "style must be \"growth\"");
    if (!(kr >= 0.0) || !std::isfinite(Cs) || !std::isfinite(b0) || std::isnan(bmax))
        return c->fail(LB2D_E_INVAL, "bad reaction parameters");
    c->reaction = true;
    c->kr = kr;
    c->Cs = Cs;
    c->b0 = b0;
    c->bmax = bmax;
    c->seed = seed;
    return LB2D_OK;
}

int lb2d_set_fields(lb2d_ctx *c, int comp, const double *rho, const double *ux, const double *uy) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (comp < 0 || comp >= c->ncomp) return c->fail(LB2D_E_INVAL, "component %d does not exist", comp);
    if (!rho) return c->fail(LB2D_E_INVAL, "null density");
    const size_t n = c->n();
    for (size_t k = 0; k < n; ++k) {
        if (!(rho[k] > 0.0) || !std::isfinite(rho[k])) return c->fail(LB2D_E_INVAL, "density must be positive");
        if ((ux && !std::isfinite(ux[k])) || (uy && !std::isfinite(uy[k])))
            return c->fail(LB2D_E_INVAL, "velocity must be finite");
    }
    c->rho0[comp].assign(rho, rho + n);
    if (ux) c->ux0[comp].assign(ux, ux + n); else c->ux0[comp].clear();
    if (uy) c->uy0[comp].assign(uy, uy + n); else c->uy0[comp].clear();
    return LB2D_OK;
}

int lb2d_set_concentration(lb2d_ctx *c, const double *C, const double *ux, const double *uy) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (!c->have_solute) return c->fail(LB2D_E_ORDER, "concentration0 needs the solute command first");
    if (!C) return c->fail(LB2D_E_INVAL, "null concentration");
    const size_t n = c->n();
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(C[k]) || (ux && !std::isfinite(ux[k])) || (uy && !std::isfinite(uy[k])))
            return c->fail(LB2D_E_INVAL, "concentration and velocity must be finite");
    c->C0.assign(C, C + n);
    if (ux) c->Cux.assign(ux, ux + n); else c->Cux.clear();
    if (uy) c->Cuy.assign(uy, uy + n); else c->Cuy.clear();
    return LB2D_OK;
}

static int add_force(lb2d_ctx *c, int mode, double value, int comp, bool accel) {
    int rc = pre_command(c);
    if (rc) return rc;
    if (mode < 0 || mode > 8) return c->fail(LB2D_E_INVAL, "mode must be 0..8");
    if (comp < 0 || comp >= c->ncomp) return c->fail(LB2D_E_INVAL, "component %d does not exist", comp);
    if (!std::isfinite(value)) return c->fail(LB2D_E_INVAL, "value must be finite");
    static const int EXh[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int EYh[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    double(*dst)[2] = accel ? c->accel : c->force;
    dst[comp][0] += value * EXh[mode];
    dst[comp][1] += value * EYh[mode];
    c->have_force = true;
    return LB2D_OK;
}

int lb2d_aveforce(lb2d_ctx *c, int mode, double value, int comp) { return add_force(c, mode, value, comp, false); }
int lb2d_aveacceleration(lb2d_ctx *c, int mode, double value, int comp) {
    return add_force(c, mode, value, comp, true);
}

// psi0, rho0 of the one-component forms: both given, psi0 finite, rho0 > 0;
// the two-component forms take neither (NaN).
static int psi_args(lb2d_ctx *c, double psi0, double rho0, const char *cmd) {
    if (c->ncomp == 2) {
        if (!is_nan(psi0) || !is_nan(rho0))
            return c->fail(LB2D_E_INVAL, "%s: the two-component form takes no psi0, rho0 (pass NaN)", cmd);
        return LB2D_OK;
    }
    if (!std::isfinite(psi0) || !(rho0 > 0.0) || !std::isfinite(rho0))
        return c->fail(LB2D_E_INVAL, "%s: the one-component form needs finite psi0 and rho0 > 0", cmd);
    return LB2D_OK;
}

int lb2d_interforce(lb2d_ctx *c, double G, double psi0, double rho0) {
    int rc = pre_command(c);
    if (rc) return rc;
    if ((rc = psi_args(c, psi0, rho0, "interforce"))) return rc;
    if (!std::isfinite(G)) return c->fail(LB2D_E_INVAL, "G must be finite");
    c->inter = true;
    c->G = G;
    c->psi0 = psi0;
    c->psi_rho0 = rho0;
    c->have_force = true;
    return LB2D_OK;
}

int lb2d_adhesiveforce(lb2d_ctx *c, double G, double psi0, double rho0, int comp) {
    int rc = pre_command(c);
    if (rc) return rc;
    if ((rc = psi_args(c, psi0, rho0, "adhesiveforce"))) return rc;
    if (comp < 0 || comp >= c->ncomp) return c->fail(LB2D_E_INVAL, "component %d does not exist", comp);
    if (!std::isfinite(G)) return c->fail(LB2D_E_INVAL, "G must be finite");
    c->ads[comp] = true;
    c->Gads[comp] = G;
    if (c->ncomp == 1) {
        c->psi0a = psi0;
        c->rho0a = rho0;
    }
    c->have_force = true;
    return LB2D_OK;
}

int lb2d_workspace_bytes(lb2d_ctx *c, int storage, size_t *bytes) {
    if (!c || !bytes) return LB2D_E_INVAL;
    if (!c->have_lattice) return c->fail(LB2D_E_ORDER, "the lattice command must come first");
    if (storage < kF64 || storage > kBF16) return c->fail(LB2D_E_INVAL, "unknown storage format");
    if (c->sr && storage != kF16 && storage != kBF16)
        return c->fail(LB2D_E_UNSUPPORTED, "stochastic rounding applies to 16-bit storage only");
    if (c->bound && storage != c->storage) return c->fail(LB2D_E_STATE, "already bound");
    *bytes = make_layout(c, storage).total;
    if (!c->bound) {
        c->storage = storage;
        c->storage_chosen = true;
    }
    return LB2D_OK;
}

int lb2d_bind(lb2d_ctx *c, void *dev_ptr, size_t bytes, void *hip_stream) {
    if (!c) return LB2D_E_INVAL;
    if (c->bound) return c->fail(LB2D_E_STATE, "already bound");
    if (!c->have_lattice) return c->fail(LB2D_E_ORDER, "the lattice command must come first");
    if (!c->storage_chosen) return c->fail(LB2D_E_ORDER, "call lb2d_workspace_bytes before lb2d_bind");
    if (!dev_ptr || ((uintptr_t)dev_ptr % kAlign) != 0)
        return c->fail(LB2D_E_INVAL, "workspace must be a 256-byte aligned device pointer");
    const Layout L = make_layout(c, c->storage);
    if (bytes < L.total) return c->fail(LB2D_E_SIZE, "workspace of %zu bytes, %zu needed", bytes, L.total);
    if (c->sr && c->storage != kF16 && c->storage != kBF16)
        return c->fail(LB2D_E_UNSUPPORTED, "stochastic rounding applies to 16-bit storage only");
    if (c->sr) {
        unsigned pnx;
        size_t pplane;
        plane_geometry(c, c->storage, &pnx, &pplane);
        if ((unsigned long long)pplane * 9ull * 2ull >= (1ull << 32))
            return c->fail(LB2D_E_SIZE, "stochastic rounding needs population arrays below 4 GiB");
    }
    HIPCHK(c, hipSetDevice(c->device));
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, dev_ptr) != hipSuccess || attr.type != hipMemoryTypeDevice ||
        attr.device != c->device) {
        (void)hipGetLastError();
        return c->fail(LB2D_E_INVAL, "workspace is not device memory of device %d", c->device);
    }
    c->ws = (char *)dev_ptr;
    c->ws_bytes = bytes;
    c->stream = (hipStream_t)hip_stream;
    plane_geometry(c, c->storage, &c->pnx, &c->pplane);
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < c->ncomp; ++k) c->f[p][k] = c->ws + L.f[p][k];
    for (int p = 0; p < 2; ++p) c->g[p] = c->q ? (void *)(c->ws + L.g[p]) : nullptr;
    c->mask = (uint8_t *)(c->ws + L.mask);
    c->trig = (uint8_t *)(c->ws + L.trig);
    c->links = (uint16_t *)(c->ws + L.links);
    c->b = c->reaction ? (double *)(c->ws + L.b) : nullptr;
    c->staging = (double *)(c->ws + L.staging);
    c->staging_doubles = L.staging_doubles;
    c->partial = (double *)(c->ws + L.partial);
    c->gpartial = (double *)(c->ws + L.gpartial);
    c->totals = (double *)(c->ws + L.totals);
    c->dstep = (long long *)(c->ws + L.dstep);
    c->gflag = (unsigned *)(c->ws + L.gflag);
    c->gseg = (uint8_t *)(c->ws + L.gseg);
    c->refl_dev = c->slip_any() ? (double *)(c->ws + L.refl) : nullptr;
    const size_t n = c->n();
    hipStream_t s = c->stream;

    // a1: obstacles -> mask
    HIPCHK(c, launch_fill_u8(c->mask, 0, n, s));
    HIPCHK(c, launch_fill_u8(c->trig, 0, n, s));
    for (const auto &hm : c->host_masks) {
        HIPCHK(c, hipMemcpyAsync(c->staging, hm.data(), n, hipMemcpyHostToDevice, s));
        HIPCHK(c, launch_or_mask(c->mask, (const uint8_t *)c->staging, n, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    if (!c->circles.empty()) {
        std::vector<int> cxy(2 * c->circles.size());
        std::vector<double> cr(c->circles.size());
        for (size_t k = 0; k < c->circles.size(); ++k) {
            cxy[2 * k] = c->circles[k].xc;
            cxy[2 * k + 1] = c->circles[k].yc;
            cr[k] = c->circles[k].r;
        }
        double *dr = c->staging;
        int *dxy = (int *)(c->staging + cr.size());
        HIPCHK(c, hipMemcpyAsync(dr, cr.data(), cr.size() * 8, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(dxy, cxy.data(), cxy.size() * 4, hipMemcpyHostToDevice, s));
        HIPCHK(c, launch_raster_circles(c->mask, c->nx, c->ny, dxy, dr, (int)c->circles.size(), s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    if (!c->rects.empty()) {
        std::vector<int> rr(4 * c->rects.size());
        for (size_t k = 0; k < c->rects.size(); ++k) {
            rr[4 * k] = c->rects[k].x0;
            rr[4 * k + 1] = c->rects[k].x1;
            rr[4 * k + 2] = c->rects[k].y0;
            rr[4 * k + 3] = c->rects[k].y1;
        }
        HIPCHK(c, hipMemcpyAsync(c->staging, rr.data(), rr.size() * 4, hipMemcpyHostToDevice, s));
        HIPCHK(c, launch_raster_rects(c->mask, c->nx, (const int *)c->staging, (int)c->rects.size(), s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    // a2: populations at equilibrium of the initial fields
    for (int k = 0; k < c->ncomp; ++k) {
        // momentum openings override the initial fields on their nodes:
        // their density and (velocity styles) their velocity
        std::vector<double> r0 = c->rho0[k], ux0 = c->ux0[k], uy0 = c->uy0[k];
        bool any = false;
        for (const auto &o : c->opens) any |= o.comp == k;
        if (any) {
            if (r0.empty()) r0.assign(n, 1.0);
            if (ux0.empty()) ux0.assign(n, 0.0);
            if (uy0.empty()) uy0.assign(n, 0.0);
            for (const auto &o : c->opens) {
                if (o.comp != k) continue;
                const int nxw = o.wall == 0 ? 1 : o.wall == 1 ? -1 : 0, nyw = o.wall == 2 ? 1 : o.wall == 3 ? -1 : 0;
                for (int j = o.lo; j <= o.hi; ++j) {
                    const int x = o.wall == 0 ? 0 : o.wall == 1 ? c->nx - 1 : j;
                    const int y = o.wall == 2 ? 0 : o.wall == 3 ? c->ny - 1 : j;
                    const size_t sidx = (size_t)y * c->nx + x;
                    const double un = o.style <= 2 ? opening_normal_velocity(o, j) : 0.0;
                    r0[sidx] = o.rho;
                    ux0[sidx] = un * nxw;
                    uy0[sidx] = un * nyw;
                }
            }
        }
        const double rr = r0.empty() ? 1.0 : mean_of(r0);
        c->rho_ref[k] = (double)(float)rr;
        int e;
        if ((e = upload(c, c->staging, r0, 1.0))) return e;
        if ((e = upload(c, c->staging + n, ux0, 0.0))) return e;
        if ((e = upload(c, c->staging + 2 * n, uy0, 0.0))) return e;
        HIPCHK(c, launch_init_fluid(c->storage, c->f[0][k], c->staging, c->staging + n, c->staging + 2 * n, n,
                                    2.25 * c->alpha[k], 1.8 * (1.0 - c->alpha[k]), c->rho_ref[k],
                                    (unsigned)c->nx, c->pnx, c->pplane, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    if (c->q) {
        int e;
        if ((e = upload(c, c->staging, c->C0, 0.0))) return e;
        if ((e = upload(c, c->staging + n, c->Cux, 0.0))) return e;
        if ((e = upload(c, c->staging + 2 * n, c->Cuy, 0.0))) return e;
        HIPCHK(c, launch_init_solute(c->storage, c->g[0], c->staging, c->staging + n, c->staging + 2 * n, n, c->q,
                                     (unsigned)c->nx, c->pnx, c->pplane, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    if (c->refl_dev) {
        // reflected shares, obstacle commands in order (a later obstacle
        // overrides an earlier one on shared nodes); circles use the same
        // minimum-image rule as the rasteriser
        std::vector<double> rf((size_t)c->ncomp * n, 0.0);
        auto put = [&](size_t node, const double *R) {
            for (int k = 0; k < c->ncomp; ++k) rf[(size_t)k * n + node] = R[k];
        };
        for (const auto &op : c->oops) {
            if (op.kind == 0) {
                const Circle &ci = c->circles[op.index];
                const int h = (ci.r < (double)(c->nx + c->ny)) ? (int)ci.r + 1 : c->nx + c->ny;
                const bool all = 2 * h + 1 >= c->nx || 2 * h + 1 >= c->ny;
                const int ylo = all ? 0 : ci.yc - h, yhi = all ? c->ny - 1 : ci.yc + h;
                const int xlo = all ? 0 : ci.xc - h, xhi = all ? c->nx - 1 : ci.xc + h;
                for (int yy = ylo; yy <= yhi; ++yy)
                    for (int xx = xlo; xx <= xhi; ++xx) {
                        const int gx = ((xx % c->nx) + c->nx) % c->nx, gy = ((yy % c->ny) + c->ny) % c->ny;
                        long dx = ((gx - ci.xc) % c->nx + c->nx) % c->nx, dy = ((gy - ci.yc) % c->ny + c->ny) % c->ny;
                        if (c->nx - dx < dx) dx = c->nx - dx;
                        if (c->ny - dy < dy) dy = c->ny - dy;
                        if ((double)(dx * dx + dy * dy) <= ci.r * ci.r) put((size_t)gy * c->nx + gx, op.R);
                    }
            } else if (op.kind == 1) {
                const Rect &re = c->rects[op.index];
                for (int yy = re.y0; yy <= re.y1; ++yy)
                    for (int xx = re.x0; xx <= re.x1; ++xx) put((size_t)yy * c->nx + xx, op.R);
            } else {
                const auto &hm = c->host_masks[op.index];
                for (size_t k = 0; k < n; ++k)
                    if (hm[k]) put(k, op.R);
            }
        }
        HIPCHK(c, hipMemcpyAsync(c->refl_dev, rf.data(), rf.size() * 8, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    if (c->reaction) HIPCHK(c, launch_init_b(c->b, c->mask, c->b0, n, s));
    HIPCHK(c, launch_links(c->mask, c->links, c->nx, c->ny, s));
    HIPCHK(c, launch_fill_f64(c->totals, 0.0, 16, s));
    HIPCHK(c, launch_fill_f64(c->partial, 0.0, (size_t)full_slots(c->nx, c->ny) * 4, s));
    HIPCHK(c, launch_fill_f64(c->gpartial, 0.0, (size_t)growth_blocks(c->nx, c->ny) * 4, s));
    HIPCHK(c, launch_fill_u8((uint8_t *)c->dstep, 0, 8, s));
    HIPCHK(c, launch_fill_u8((uint8_t *)c->gflag, 0, 8, s));
    HIPCHK(c, launch_fill_u8(c->gseg, 0, 2 * (size_t)growth_segments(c->nx, c->ny), s));
    HIPCHK(c, hipStreamSynchronize(s));
    c->t = 0;
    c->bound = true;
    return LB2D_OK;
}

int lb2d_iteration(lb2d_ctx *c, int64_t nsteps) {
    if (!c) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "bind the lattice before iteration");
    if (nsteps < 0) return c->fail(LB2D_E_INVAL, "nsteps must be >= 0");
    HIPCHK(c, hipSetDevice(c->device));
    int64_t left = nsteps;
    if (c->timing) {
        // one launch at a time, the dominant (step) kernel bracketed by events
        for (; left > 0; --left) {
            const int parity = (int)(c->t & 1);
            HIPCHK(c, hipEventRecord(c->ev0, c->stream));
            if (c->plain()) {
                HIPCHK(c, launch_plain(c->storage, plain_lattice(c), parity, c->sr, stream_stores(c), 0, c->stream));
                HIPCHK(c, hipEventRecord(c->ev1, c->stream));
                if (c->sr) HIPCHK(c, launch_tick((unsigned long long *)c->dstep, 1, c->stream));
            } else {
                const FullParams p = full_params(c);
                HIPCHK(c, launch_full(c->storage, p, parity, c->sc(), c->reaction, c->stream));
                if (c->has_gradient()) HIPCHK(c, launch_open_gradient(c->storage, p, parity ^ 1, c->stream));
                HIPCHK(c, hipEventRecord(c->ev1, c->stream));
                if (c->q) HIPCHK(c, launch_growth(c->storage, p, parity ^ 1, c->reaction, c->stream));
                else if (c->sr) HIPCHK(c, launch_tick((unsigned long long *)c->dstep, 1, c->stream));
            }
            HIPCHK(c, hipEventSynchronize(c->ev1));
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
            c->kernel_ms += ms;
            c->kernel_launches += 1;
            c->t += 1;
        }
        return LB2D_OK;
    }
    const StepPlan q = step_plan(c->t, left);
    hipGraphExec_t g = nullptr;
    if (q.graphs) {
        int rc = build_graph(c, kGraphSteps, q.p0, &g);
        if (rc) return rc;
        for (int64_t k = 0; k < q.graphs; ++k) {
            HIPCHK(c, hipGraphLaunch(g, c->stream));
            c->t += kGraphSteps;
        }
    }
    if (q.tail == 1) {
        HIPCHK(c, enqueue_step(c, q.p0, 0, 1, c->stream));
        c->t += 1;
    } else if (q.tail > 1) {
        int rc = build_graph(c, (int)q.tail, q.p0, &g);
        if (rc) return rc;
        HIPCHK(c, hipGraphLaunch(g, c->stream));
        c->t += q.tail;
    }
    return LB2D_OK;
}

int lb2d_steps_per_launch(lb2d_ctx *c, int *steps) {
    if (!c || !steps) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    *steps = c->plain() && multi_fits(c->storage, c->nx, c->ny) ? multi_steps() : 1;
    return LB2D_OK;
}

int lb2d_prepare(lb2d_ctx *c, int64_t nsteps) {
    if (!c) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "bind the lattice before preparing its steps");
    if (nsteps < 0) return c->fail(LB2D_E_INVAL, "nsteps must be >= 0");
    HIPCHK(c, hipSetDevice(c->device));
    const StepPlan q = step_plan(c->t, nsteps);
    hipGraphExec_t g = nullptr;
    int rc = LB2D_OK;
    if (q.graphs) rc = build_graph(c, kGraphSteps, q.p0, &g);
    if (!rc && q.tail > 1) rc = build_graph(c, (int)q.tail, q.p0, &g);
    return rc;
}

int lb2d_moments(lb2d_ctx *c, int comp, double *rho, double *ux, double *uy) {
    if (!c || !rho || !ux || !uy) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    if (comp < -1 || comp >= c->ncomp) return c->fail(LB2D_E_INVAL, "component %d does not exist", comp);
    HIPCHK(c, hipSetDevice(c->device));
    const size_t n = c->n();
    const FullParams p = full_params(c);
    HIPCHK(c, launch_moments(c->storage, p, (int)(c->t & 1), comp, c->staging, c->staging + n,
                             c->staging + 2 * n, c->stream));
    HIPCHK(c, hipMemcpyAsync(rho, c->staging, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ux, c->staging + n, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(uy, c->staging + 2 * n, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LB2D_OK;
}

int lb2d_solute_state(lb2d_ctx *c, double *C, double *b) {
    if (!c) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    if (!c->q) return c->fail(LB2D_E_ORDER, "no solute in this lattice");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t n = c->n();
    const FullParams p = full_params(c);
    HIPCHK(c, launch_solute_state(c->storage, p, (int)(c->t & 1), c->reaction ? 1 : 0, c->staging,
                                  c->staging + n, c->stream));
    if (C) HIPCHK(c, hipMemcpyAsync(C, c->staging, n * 8, hipMemcpyDeviceToHost, c->stream));
    if (b) HIPCHK(c, hipMemcpyAsync(b, c->staging + n, n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LB2D_OK;
}

int lb2d_mask(lb2d_ctx *c, uint8_t *m) {
    if (!c || !m) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(m, c->mask, c->n(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LB2D_OK;
}

// Budgets of a bound lattice with the reduction's scratch (per-row
// partials, the eight sums, the fixed-order tally totals) at part / out8 /
// totals: the workspace's staging area for lb2d_budgets, the library's
// static array for lb2d_budgets_noalloc.
static int budgets_with(lb2d_ctx *c, double *out, double *part, double *out8, double *totals) {
    FullParams p = full_params(c);
    p.totals = totals;
    HIPCHK(c, launch_budgets(c->storage, p, (int)(c->t & 1), c->q ? 1 : 0, c->reaction ? 1 : 0, part, out8,
                             c->stream));
    if (c->q) HIPCHK(c, launch_tally_final(p, c->stream));
    double v8[8], tot[16];
    for (int k = 0; k < 16; ++k) tot[k] = 0.0;
    HIPCHK(c, hipMemcpyAsync(v8, out8, sizeof(v8), hipMemcpyDeviceToHost, c->stream));
    // without a solute nothing is tallied: the totals stay zero
    if (c->q) HIPCHK(c, hipMemcpyAsync(tot, totals, sizeof(tot), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < LB2D_NBUDGET; ++k) out[k] = 0.0;
    out[LB2D_B_MASS0] = v8[0];
    out[LB2D_B_MASS1] = v8[1];
    out[LB2D_B_MOMX] = v8[2];
    out[LB2D_B_MOMY] = v8[3];
    out[LB2D_B_SOLUTE] = v8[4];
    out[LB2D_B_DEPOSIT] = v8[5];
    out[LB2D_B_FLUID] = v8[6];
    out[LB2D_B_REMOVED0] = tot[6];
    out[LB2D_B_REMOVED1] = tot[7];
    out[LB2D_B_REMOVED_C] = tot[8];
    out[LB2D_B_INFLOW] = tot[9];
    out[LB2D_B_OUTFLOW] = tot[10];
    out[LB2D_B_GROWN] = tot[12];
    out[LB2D_B_CONSUMED] = tot[14];
    out[LB2D_B_STEPS] = (double)c->t;
    return LB2D_OK;
}

int lb2d_budgets(lb2d_ctx *c, double *out) {
    if (!c || !out) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    HIPCHK(c, hipSetDevice(c->device));
    return budgets_with(c, out, c->staging, c->staging + (size_t)c->ny * 8, c->totals);
}

int lb2d_budgets_noalloc(lb2d_ctx *c, double *out) {
    if (!c || !out) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    const size_t need = (size_t)c->ny * 8 + 8 + 16;
    if (need > kBudgetScratchDoubles)
        return c->fail(LB2D_E_SIZE, "lb2d_budgets_noalloc: %d rows exceed its limit of %d rows", c->ny,
                       (int)((kBudgetScratchDoubles - 24) / 8));
    HIPCHK(c, hipSetDevice(c->device));
    double *scr = nullptr;
    const int rc = budget_scratch(c, &scr);
    if (rc) return rc;
    return budgets_with(c, out, scr, scr + (size_t)c->ny * 8, scr + (size_t)c->ny * 8 + 8);
}

static int pop_target(lb2d_ctx *c, int comp, void **buf, double *ref) {
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    const int parity = (int)(c->t & 1);
    if (comp == -1) {
        if (!c->q) return c->fail(LB2D_E_INVAL, "no solute in this lattice");
        *buf = c->g[parity];
        *ref = 0.0;
    } else {
        if (comp < 0 || comp >= c->ncomp) return c->fail(LB2D_E_INVAL, "component %d does not exist", comp);
        *buf = c->f[parity][comp];
        *ref = c->rho_ref[comp];
    }
    return LB2D_OK;
}

// Storage plane of solute direction i (-1: absent from D2Q4).
static int solute_plane(int q, int i) { return q == 9 ? i : ((i >= 1 && i <= 4) ? i - 1 : -1); }

static const double kW[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

int lb2d_get_populations(lb2d_ctx *c, int comp, double *out) {
    if (!c || !out) return LB2D_E_INVAL;
    void *buf;
    double ref;
    int rc = pop_target(c, comp, &buf, &ref);
    if (rc) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    const size_t n = c->n();
    for (int i = 0; i < 9; ++i) {
        const int pl = comp >= 0 ? i : solute_plane(c->q, i);
        if (pl < 0) {  // direction absent from the D2Q4 solute lattice
            std::memset(out + (size_t)i * n, 0, n * 8);
            continue;
        }
        HIPCHK(c, launch_decode_plane(c->storage, buf, c->mask, c->staging, n, pl, i, kW[i] * ref, (unsigned)c->nx,
                                      c->pnx, c->pplane, c->stream));
        HIPCHK(c, hipMemcpyAsync(out + (size_t)i * n, c->staging, n * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return LB2D_OK;
}

int lb2d_set_populations(lb2d_ctx *c, int comp, const double *in) {
    if (!c || !in) return LB2D_E_INVAL;
    void *buf;
    double ref;
    int rc = pop_target(c, comp, &buf, &ref);
    if (rc) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    const size_t n = c->n();
    if (comp < 0)
        for (int i = 0; i < 9; ++i)
            if (solute_plane(c->q, i) < 0)
                for (size_t k = 0; k < n; ++k)
                    if (in[(size_t)i * n + k] != 0.0)
                        return c->fail(LB2D_E_INVAL, "the D2Q4 solute lattice has no population %d", i);
    for (int i = 0; i < 9; ++i) {
        const int pl = comp >= 0 ? i : solute_plane(c->q, i);
        if (pl < 0) continue;
        HIPCHK(c, hipMemcpyAsync(c->staging, in + (size_t)i * n, n * 8, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, launch_encode_plane(c->storage, buf, c->staging, n, pl, i, kW[i] * ref, (unsigned)c->nx,
                                      c->pnx, c->pplane, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return LB2D_OK;
}

int lb2d_get_deposit(lb2d_ctx *c, double *b) {
    if (!c || !b) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    if (!c->reaction) return c->fail(LB2D_E_ORDER, "no surface reaction in this lattice");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(b, c->b, c->n() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LB2D_OK;
}

int lb2d_set_deposit(lb2d_ctx *c, const double *b) {
    if (!c || !b) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    if (!c->reaction) return c->fail(LB2D_E_ORDER, "no surface reaction in this lattice");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(c->b, b, c->n() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LB2D_OK;
}

int lb2d_set_mask(lb2d_ctx *c, const uint8_t *m) {
    if (!c || !m) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(c->mask, m, c->n(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_fill_u8(c->trig, 0, c->n(), c->stream));
    HIPCHK(c, launch_links(c->mask, c->links, c->nx, c->ny, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LB2D_OK;
}

int lb2d_step_count(lb2d_ctx *c, int64_t *t) {
    if (!c || !t) return LB2D_E_INVAL;
    *t = c->t;
    return LB2D_OK;
}

// Checkpoints: a header that identifies the lattice (sizes, components,
// solute, storage, rounding, the population shift, the workspace layout)
// and its step count, followed by the whole bound workspace, byte for byte.
namespace {
struct CkptHeader {
    char magic[8];
    int32_t version, nx, ny, ncomp, q, storage, sr, pad;
    int64_t t;
    uint64_t ws_bytes, layout;
    double rho_ref[2];
};

uint64_t layout_fingerprint(const lb2d_ctx *c) {
    const Layout L = make_layout(c, c->storage);
    const unsigned char *p = (const unsigned char *)&L;
    uint64_t h = 1469598103934665603ull;
    for (size_t k = 0; k < sizeof(L); ++k) h = (h ^ p[k]) * 1099511628211ull;
    return h;
}

CkptHeader ckpt_header(const lb2d_ctx *c) {
    CkptHeader h{};
    std::memcpy(h.magic, "LB2DCKPT", 8);
    h.version = 1;
    h.nx = c->nx;
    h.ny = c->ny;
    h.ncomp = c->ncomp;
    h.q = c->q;
    h.storage = c->storage;
    h.sr = c->sr ? 1 : 0;
    h.t = c->t;
    h.ws_bytes = make_layout(c, c->storage).total;
    h.layout = layout_fingerprint(c);
    h.rho_ref[0] = c->rho_ref[0];
    h.rho_ref[1] = c->rho_ref[1];
    return h;
}
}  // namespace

int lb2d_checkpoint_bytes(lb2d_ctx *c, size_t *bytes) {
    if (!c || !bytes) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    *bytes = sizeof(CkptHeader) + make_layout(c, c->storage).total;
    return LB2D_OK;
}

int lb2d_checkpoint_save(lb2d_ctx *c, void *host, size_t bytes) {
    if (!c || !host) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    const CkptHeader h = ckpt_header(c);
    if (bytes < sizeof(h) + h.ws_bytes)
        return c->fail(LB2D_E_SIZE, "checkpoint needs %zu bytes", (size_t)(sizeof(h) + h.ws_bytes));
    HIPCHK(c, hipSetDevice(c->device));
    std::memcpy(host, &h, sizeof(h));
    HIPCHK(c, hipMemcpyAsync((char *)host + sizeof(h), c->ws, h.ws_bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LB2D_OK;
}

int lb2d_checkpoint_load(lb2d_ctx *c, const void *host, size_t bytes) {
    if (!c || !host) return LB2D_E_INVAL;
    if (!c->bound) return c->fail(LB2D_E_STATE, "not bound");
    CkptHeader h;
    if (bytes < sizeof(h)) return c->fail(LB2D_E_INVAL, "not a checkpoint");
    std::memcpy(&h, host, sizeof(h));
    const CkptHeader mine = ckpt_header(c);
    if (std::memcmp(h.magic, mine.magic, 8) != 0 || h.version != mine.version)
        return c->fail(LB2D_E_INVAL, "not a checkpoint of this library");
    if (h.nx != mine.nx || h.ny != mine.ny || h.ncomp != mine.ncomp || h.q != mine.q || h.storage != mine.storage ||
        h.sr != mine.sr || h.ws_bytes != mine.ws_bytes || h.layout != mine.layout ||
        std::memcmp(h.rho_ref, mine.rho_ref, sizeof(h.rho_ref)) != 0)
        return c->fail(LB2D_E_INVAL, "checkpoint of a lattice set up differently");
    if (bytes < sizeof(h) + h.ws_bytes) return c->fail(LB2D_E_SIZE, "checkpoint truncated");
    if (h.t < 0) return c->fail(LB2D_E_INVAL, "bad step count");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ws, (const char *)host + sizeof(h), h.ws_bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->t = h.t;
    return LB2D_OK;
}

int lb2d_set_timing(lb2d_ctx *c, int on) {
    if (!c) return LB2D_E_INVAL;
    if (on && !c->ev0) {
        HIPCHK(c, hipSetDevice(c->device));
        HIPCHK(c, hipEventCreate(&c->ev0));
        HIPCHK(c, hipEventCreate(&c->ev1));
    }
    c->timing = on != 0;
    c->kernel_ms = 0.0;
    c->kernel_launches = 0;
    return LB2D_OK;
}

int lb2d_kernel_time(lb2d_ctx *c, double *ms, int64_t *launches) {
    if (!c || !ms || !launches) return LB2D_E_INVAL;
    *launches = c->kernel_launches;
    *ms = c->kernel_launches ? c->kernel_ms / (double)c->kernel_launches : 0.0;
    return LB2D_OK;
}

// ------------------------------------------------------------------ batch

int lb2d_batch_create(lb2d_batch **out, int hip_device) {
    if (!out || hip_device < 0) return LB2D_E_INVAL;
    lb2d_batch *b = new lb2d_batch();
    b->device = hip_device;
    *out = b;
    return LB2D_OK;
}

int lb2d_batch_destroy(lb2d_batch *b) {
    if (!b) return LB2D_E_INVAL;
    if (b->ws) {
        (void)hipSetDevice(b->device);
        (void)hipStreamSynchronize(b->stream);
    }
    if (b->graph[0] || b->graph[1] || b->cap_stream) {
        (void)hipSetDevice(b->device);
        for (hipGraphExec_t g : b->graph)
            if (g) (void)hipGraphExecDestroy(g);
        if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    }
    delete b;
    return LB2D_OK;
}

const char *lb2d_batch_last_error(const lb2d_batch *b) { return b ? b->err.c_str() : "null batch"; }

int lb2d_batch_add(lb2d_batch *b, lb2d_ctx *c) {
    if (!b || !c) return LB2D_E_INVAL;
    if (b->final_) return b->fail(LB2D_E_STATE, "batch already finalized");
    if (!c->bound) return b->fail(LB2D_E_STATE, "lattices must be bound before lb2d_batch_add");
    if (!c->plain()) return b->fail(LB2D_E_UNSUPPORTED, "batches hold one-fluid lattices without solute");
    if (c->device != b->device) return b->fail(LB2D_E_INVAL, "lattice on another device");
    if (!b->lat.empty()) {
        if (c->storage != b->storage) return b->fail(LB2D_E_INVAL, "all lattices need the same storage format");
        if ((c->t & 1) != (b->lat[0]->t & 1)) return b->fail(LB2D_E_STATE, "lattices at different step parity");
        if (c->sr != b->sr) return b->fail(LB2D_E_INVAL, "all lattices need the same rounding");
    }
    for (auto *o : b->lat)
        if (o == c) return b->fail(LB2D_E_INVAL, "lattice added twice");
    b->storage = c->storage;
    b->sr = c->sr;
    b->lat.push_back(c);
    return LB2D_OK;
}

static size_t tiles_for(const lb2d_batch *b, int w, int h) {
    size_t n = 0;
    for (auto *c : b->lat) n += (size_t)((c->nx + w - 1) / w) * ((c->ny + h - 1) / h);
    return n;
}

// The multi-step kernel serves a batch whose every lattice satisfies multi_fits.
static bool batch_ms_ok(const lb2d_batch *b) {
    for (auto *c : b->lat)
        if (!multi_fits(b->storage, c->nx, c->ny)) return false;
    return !b->lat.empty();
}

// Tile shapes the autotuner may choose: the one-step shapes of the storage
// format, then the multi-step kernel's tile when the batch allows it.
static int candidate_shapes(const lb2d_batch *b, int *tw, int *th) {
    int n = batch_shapes(b->storage, tw, th, 4);
    if (batch_ms_ok(b)) {
        multi_tile_shape(b->storage, &tw[n], &th[n]);
        ++n;
    }
    return n;
}

static bool is_multi_step_shape(const lb2d_batch *b, int w, int h) {
    int tw, th;
    multi_tile_shape(b->storage, &tw, &th);
    return w == tw && h == th && batch_ms_ok(b);
}

// Largest tile table over the candidate shapes.
static size_t max_tiles_for(const lb2d_batch *b) {
    int tw[5], th[5];
    const int ns = candidate_shapes(b, tw, th);
    size_t m = 0;
    for (int k = 0; k < ns; ++k) m = std::max(m, tiles_for(b, tw[k], th[k]));
    return m;
}

static bool is_batch_shape(const lb2d_batch *b, int w, int h) {
    int tw[5], th[5];
    const int ns = candidate_shapes(b, tw, th);
    for (int k = 0; k < ns; ++k)
        if (tw[k] == w && th[k] == h) return true;
    return false;
}

int lb2d_batch_workspace_bytes(lb2d_batch *b, size_t *bytes) {
    if (!b || !bytes) return LB2D_E_INVAL;
    if (b->lat.empty()) return b->fail(LB2D_E_STATE, "empty batch");
    const size_t tiles = max_tiles_for(b);
    int w1, h1;
    plain_tile(b->storage, &w1, &h1);
    *bytes = align_up(b->lat.size() * sizeof(PlainLattice)) + align_up(tiles * sizeof(Tile)) +
             align_up(tiles_for(b, w1, h1) * sizeof(Tile)) + align_up(8);
    return LB2D_OK;
}


static int batch_upload_tiles(lb2d_batch *b, int w, int h, int sched) {
    std::vector<Tile> t = make_tiles(b, w, h, sched);
    if (t.size() > b->max_tiles) return b->fail(LB2D_E_SIZE, "tile table too large");
    HIPCHK(b, hipMemcpyAsync(b->d_tiles, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    b->ntiles = (int)t.size();
    return LB2D_OK;
}

int lb2d_batch_finalize(lb2d_batch *b, void *dev_ptr, size_t bytes, void *hip_stream, const char *cache) {
    if (!b) return LB2D_E_INVAL;
    if (b->final_) return b->fail(LB2D_E_STATE, "batch already finalized");
    size_t need = 0;
    int rc = lb2d_batch_workspace_bytes(b, &need);
    if (rc) return rc;
    if (!dev_ptr || ((uintptr_t)dev_ptr % kAlign) != 0) return b->fail(LB2D_E_INVAL, "bad workspace pointer");
    if (bytes < need) return b->fail(LB2D_E_SIZE, "workspace of %zu bytes, %zu needed", bytes, need);
    HIPCHK(b, hipSetDevice(b->device));
    b->ws = (char *)dev_ptr;
    b->ws_bytes = bytes;
    b->stream = (hipStream_t)hip_stream;
    b->d_lat = (PlainLattice *)b->ws;
    b->d_tiles = (Tile *)(b->ws + align_up(b->lat.size() * sizeof(PlainLattice)));
    b->max_tiles = max_tiles_for(b);
    plain_tile(b->storage, &b->tile_w1, &b->tile_h1);
    b->d_tiles1 = (Tile *)((char *)b->d_tiles + align_up(b->max_tiles * sizeof(Tile)));
    b->d_step = (unsigned long long *)((char *)b->d_tiles1 +
                                       align_up(tiles_for(b, b->tile_w1, b->tile_h1) * sizeof(Tile)));
    {
        // every lattice of a batch is at the same step, and a lattice that
        // rounds stochastically has its device counter at that step
        const unsigned long long t0 = (unsigned long long)b->lat[0]->t;
        HIPCHK(b, hipMemcpyAsync(b->d_step, &t0, 8, hipMemcpyHostToDevice, (hipStream_t)hip_stream));
        HIPCHK(b, hipStreamSynchronize((hipStream_t)hip_stream));
    }
    plain_tile(b->storage, &b->tile_w, &b->tile_h);
    std::vector<PlainLattice> L;
    b->max_plane = 0;
    size_t pop_bytes = 0;
    for (auto *c : b->lat) {
        L.push_back(plain_lattice(c));
        b->max_plane = std::max(b->max_plane, c->pplane);
        pop_bytes += population_bytes(c);
    }
    b->nt = pop_bytes > kLastLevelCache;
    HIPCHK(b, hipMemcpyAsync(b->d_lat, L.data(), L.size() * sizeof(PlainLattice), hipMemcpyHostToDevice, b->stream));
    {
        const std::vector<Tile> t1 = make_tiles(b, b->tile_w1, b->tile_h1, 0);
        HIPCHK(b, hipMemcpyAsync(b->d_tiles1, t1.data(), t1.size() * sizeof(Tile), hipMemcpyHostToDevice,
                                 b->stream));
        b->ntiles1 = (int)t1.size();
    }
    HIPCHK(b, hipStreamSynchronize(b->stream));
    int cus = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, b->device) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    const std::string key = batch_key(b);
    bool have = false;
    if (cache) {
        FILE *fh = std::fopen(cache, "r");
        if (fh) {
            char k[64] = {0};
            int w, h, s, p;
            if (std::fscanf(fh, "{\"key\": \"%63[0-9a-f]\", \"tile_w\": %d, \"tile_h\": %d, \"schedule\": %d, "
                                "\"blocks_per_cu\": %d}",
                            k, &w, &h, &s, &p) == 5 &&
                key == k && s >= 0 && s <= 2 && p >= 0 && p <= 64 && is_batch_shape(b, w, h)) {
                b->tile_w = w;
                b->tile_h = h;
                b->schedule = s;
                b->bpc = p;
                have = true;
            }
            std::fclose(fh);
        }
    }
    if (!have) {
        // timed trial launches: each writes the lattices' next buffers from
        // the current ones without advancing, so the state is unchanged.
        // Candidates: tile shape (one, two or four brick rows of the
        // one-step kernel, and the multi-step kernel's tile) x schedule
        // (lattice by lattice, largest first, interleaved) x grid (one block
        // per tile, or persistent blocks: 8 or 16 per CU of 256 threads, 1
        // or 2 per CU of the multi-step kernel's 1024 or 512)
        int tws[5], ths[5];
        const int ns = candidate_shapes(b, tws, ths);
        std::vector<TuneCand> cands;
        for (int k = 0; k < ns; ++k) {
            const bool multi = is_multi_step_shape(b, tws[k], ths[k]);
            for (int bpc : {0, multi ? 1 : 8, multi ? 2 : 16})
                for (int sched = 0; sched < 3; ++sched) cands.push_back({tws[k], ths[k], sched, bpc});
        }
        b->trials.clear();
        hipEvent_t e0, e1;
        HIPCHK(b, hipEventCreate(&e0));
        HIPCHK(b, hipEventCreate(&e1));
        const int parity = (int)(b->lat[0]->t & 1);
        float best = 1e30f;
        TuneCand bc = cands[0];
        for (const auto &cd : cands) {
            if ((rc = batch_upload_tiles(b, cd.w, cd.h, cd.sched))) return rc;
            const int grid = batch_grid(b->ntiles, cd.bpc, cus);
            const bool multi = is_multi_step_shape(b, cd.w, cd.h);
            auto launch = [&]() {
                return multi ? launch_batch_ms(b->storage, b->d_lat, b->d_tiles, b->ntiles, parity, grid,
                                               b->max_plane, b->nt, b->sr, 0, b->d_step, b->stream)
                             : launch_batch(b->storage, cd.w, b->d_lat, b->d_tiles, b->ntiles, parity, grid,
                                            b->max_plane, b->nt, b->sr, 0, b->d_step, b->stream);
            };
            HIPCHK(b, launch());
            HIPCHK(b, hipEventRecord(e0, b->stream));
            for (int r = 0; r < 3; ++r) HIPCHK(b, launch());
            HIPCHK(b, hipEventRecord(e1, b->stream));
            HIPCHK(b, hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(b, hipEventElapsedTime(&ms, e0, e1));
            ms /= multi ? (float)multi_steps() : 1.0f;  // per step
            b->trials.push_back({(double)cd.w, (double)cd.h, (double)cd.sched, (double)cd.bpc, ms / 3.0});
            if (ms < best) {
                best = ms;
                bc = cd;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->tile_w = bc.w;
        b->tile_h = bc.h;
        b->schedule = bc.sched;
        b->bpc = bc.bpc;
    }
    if ((rc = batch_upload_tiles(b, b->tile_w, b->tile_h, b->schedule))) return rc;
    b->grid = batch_grid(b->ntiles, b->bpc, cus);
    b->multi = is_multi_step_shape(b, b->tile_w, b->tile_h);
    if (cache) {
        FILE *fh = std::fopen(cache, "w");
        if (fh) {
            std::fprintf(fh,
                         "{\"key\": \"%s\", \"tile_w\": %d, \"tile_h\": %d, \"schedule\": %d, "
                         "\"blocks_per_cu\": %d}\n",
                         key.c_str(), b->tile_w, b->tile_h, b->schedule, b->bpc);
            std::fclose(fh);
        }
    }
    b->t = b->lat[0]->t;
    b->final_ = true;
    return LB2D_OK;
}

// One batched step at offset k of its launch group (with the one-step
// tiles when the multi-step kernel was chosen); tick: steps to add to the
// lattices' step counters after it (stochastic rounding only).
static hipError_t batch_step(lb2d_batch *b, int parity, int k, int tick, hipStream_t s) {
    hipError_t e = b->multi ? launch_batch(b->storage, b->tile_w1, b->d_lat, b->d_tiles1, b->ntiles1, parity,
                                         b->ntiles1, b->max_plane, b->nt, b->sr, k, b->d_step, s)
                          : launch_batch(b->storage, b->tile_w, b->d_lat, b->d_tiles, b->ntiles, parity, b->grid,
                                         b->max_plane, b->nt, b->sr, k, b->d_step, s);
    if (e == hipSuccess && b->sr && tick) e = launch_tick_batch(b->d_lat, (int)b->lat.size(), tick, b->d_step, s);
    return e;
}

// multi_steps() batched steps from a step of parity p as one multi-step
// launch (p -> p^1), at offset k of its launch group; tick as for
// batch_step.
static hipError_t batch_multi(lb2d_batch *b, int p, int k, int tick, hipStream_t s) {
    hipError_t e = launch_batch_ms(b->storage, b->d_lat, b->d_tiles, b->ntiles, p, b->grid, b->max_plane, b->nt,
                                   b->sr, k, b->d_step, s);
    if (e == hipSuccess && b->sr && tick) e = launch_tick_batch(b->d_lat, (int)b->lat.size(), tick, b->d_step, s);
    return e;
}

int lb2d_batch_iteration(lb2d_batch *b, int64_t nsteps) {
    if (!b) return LB2D_E_INVAL;
    if (!b->final_) return b->fail(LB2D_E_STATE, "finalize the batch first");
    if (nsteps < 0) return b->fail(LB2D_E_INVAL, "nsteps must be >= 0");
    for (auto *c : b->lat)
        if (c->t != b->t) return b->fail(LB2D_E_STATE, "a lattice of the batch was advanced on its own");
    HIPCHK(b, hipSetDevice(b->device));
    int64_t left = nsteps;
    // graphs of kGraphSteps (even) steps, captured once per start parity
    const int p0 = (int)(b->t & 1);
    if (left >= kGraphSteps && !b->graph[p0]) {
        if (!b->cap_stream) HIPCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        hipGraph_t gr = nullptr;
        HIPCHK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        const int ms = multi_steps();
        if (b->multi)
            for (int k = 0; k + ms <= kGraphSteps && e == hipSuccess; k += ms)
                e = batch_multi(b, (p0 + k) & 1, k, k + ms == kGraphSteps ? kGraphSteps : 0, b->cap_stream);
        else
            for (int k = 0; k < kGraphSteps && e == hipSuccess; ++k)
                e = batch_step(b, (p0 + k) & 1, k, k == kGraphSteps - 1 ? kGraphSteps : 0, b->cap_stream);
        hipError_t e2 = hipStreamEndCapture(b->cap_stream, &gr);
        if (e != hipSuccess || e2 != hipSuccess) return b->fail(LB2D_E_HIP, "batch graph capture failed");
        HIPCHK(b, hipGraphInstantiate(&b->graph[p0], gr, nullptr, nullptr, 0));
        HIPCHK(b, hipGraphDestroy(gr));
        HIPCHK(b, hipGraphUpload(b->graph[p0], b->stream));
    }
    while (left >= kGraphSteps) {
        HIPCHK(b, hipGraphLaunch(b->graph[p0], b->stream));
        b->t += kGraphSteps;
        left -= kGraphSteps;
    }
    for (; b->multi && left >= multi_steps(); left -= multi_steps()) {
        HIPCHK(b, batch_multi(b, (int)(b->t & 1), 0, multi_steps(), b->stream));
        b->t += multi_steps();
    }
    for (; left > 0; --left) {
        HIPCHK(b, batch_step(b, (int)(b->t & 1), 0, 1, b->stream));
        b->t += 1;
    }
    for (auto *c : b->lat) c->t = b->t;
    return LB2D_OK;
}

int lb2d_batch_config(lb2d_batch *b, int *w, int *h, int *s, int *p) {
    if (!b || !w || !h || !s || !p) return LB2D_E_INVAL;
    if (!b->final_) return b->fail(LB2D_E_STATE, "not finalized");
    *w = b->tile_w;
    *h = b->tile_h;
    *s = b->schedule;
    *p = b->bpc;
    return LB2D_OK;
}

int lb2d_batch_steps_per_launch(lb2d_batch *b, int *steps) {
    if (!b || !steps) return LB2D_E_INVAL;
    if (!b->final_) return b->fail(LB2D_E_STATE, "not finalized");
    *steps = b->multi ? multi_steps() : 1;
    return LB2D_OK;
}

int lb2d_batch_trials(lb2d_batch *b, int max, int *tile_w, int *tile_h, int *schedule, int *blocks_per_cu,
                      double *ms, int *count) {
    if (!b || !count || max < 0) return LB2D_E_INVAL;
    if (!b->final_) return b->fail(LB2D_E_STATE, "not finalized");
    const int n = (int)b->trials.size();
    *count = n;
    if (max > 0 && (!tile_w || !tile_h || !schedule || !blocks_per_cu || !ms)) return LB2D_E_INVAL;
    for (int k = 0; k < n && k < max; ++k) {
        tile_w[k] = (int)b->trials[k][0];
        tile_h[k] = (int)b->trials[k][1];
        schedule[k] = (int)b->trials[k][2];
        blocks_per_cu[k] = (int)b->trials[k][3];
        ms[k] = b->trials[k][4];
    }
    return LB2D_OK;
}

// Measures a plain device-to-device copy of `bytes` (read + write) on the
// stream and returns the average milliseconds per copy over `reps` (not a
// paper command: the practical bandwidth ceiling next to the stencil).
int lb2d_copy_bench(void *src, void *dst, size_t bytes, int reps, void *hip_stream, double *ms) {
    if (!src || !dst || !ms || reps < 1 || bytes == 0 || bytes % 16) return LB2D_E_INVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LB2D_E_HIP;
    if (launch_copy(src, dst, bytes, s) != hipSuccess) return LB2D_E_HIP;
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy(src, dst, bytes, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / reps;
    return e == hipSuccess ? LB2D_OK : LB2D_E_HIP;
}

}  // extern "C"
