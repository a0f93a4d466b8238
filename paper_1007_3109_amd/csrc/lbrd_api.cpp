// Host side of the lbrd C ABI: validation, layout, solver lifecycle, stepping
// (plain launches or replayed HIP graphs), read-outs and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "lbrd.h"
#include "lbrd_internal.h"
#include "lbrd_util.h"

namespace lbrd {

// ------------------------------------------------------------- errors --

static thread_local std::string g_last_error;

void set_error(const char *where, hipError_t e) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
}

// ------------------------------------------------------------- layout --

static int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

std::vector<double> scrambled_densities(size_t n) {
    std::vector<double> rho(n);
    uint64_t z = 0x9e3779b97f4a7c15ull;
    for (double &r : rho) {
        z += 0x9e3779b97f4a7c15ull;   // splitmix64
        uint64_t x = z;
        x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
        x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
        x ^= x >> 31;
        r = 0.5 + 0.5 * (double)(x >> 11) * (1.0 / 9007199254740992.0);
    }
    return rho;
}

// Extra bytes between consecutive planes so that the 9N concurrent streams of
// a step do not start on the same HBM channel.  LBRD_PLANE_SKEW overrides it.
static int64_t plane_skew_bytes() {
    static int64_t v = [] {
        const char *e = std::getenv("LBRD_PLANE_SKEW");
        if (e) return (int64_t)std::max(0L, std::atol(e)) / 256 * 256;
        return (int64_t)768;
    }();
    return v;
}

Layout make_layout(const lbrd_config &c) {
    Layout L;
    L.nx = c.nx;
    L.ny = c.ny;
    L.ns = c.nspecies;
    L.esize = storage_bytes(c.storage);
    L.pitch = round_up(c.nx, 64 / L.esize);
    const int64_t plane = round_up((int64_t)c.ny * L.pitch * L.esize, 256) + plane_skew_bytes();
    L.pstride = plane / L.esize;
    L.buf_bytes = (size_t)round_up(9 * (int64_t)c.nspecies * plane, 4096);
    return L;
}

template <class C>
Params<C> make_params(const lbrd_config &c) {
    Params<C> p;
    std::memset(&p, 0, sizeof(p));
    const int n = c.nspecies;
    const C w[3] = {C(4) / C(9), C(1) / C(9), C(1) / C(36)};
    // equilibrium coefficients: the weights, or the low-Mach Maxwellian
    // c_i = w_i [1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u] evaluated in double
    p.adv = (c.u[0] != 0.0 || c.u[1] != 0.0 || has_shear(c)) ? 1 : 0;
    for (int i = 0; i < 9; ++i) {
        const C wi = i == 0 ? w[0] : (i < 5 ? w[1] : w[2]);
        if (!p.adv) {
            p.ceq[i] = wi;
        } else {
            const double wd = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
            const double eu = kEx[i] * c.u[0] + kEy[i] * c.u[1], uu = c.u[0] * c.u[0] + c.u[1] * c.u[1];
            p.ceq[i] = C(wd * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
        }
    }
    for (int s = 0; s < n; ++s) {
        p.omega[s] = C(1) / C(c.tau[s]);
        p.keep[s] = C(1) - p.omega[s];
        for (int i = 0; i < 9; ++i) {
            const bool shifted = c.storage == LBRD_F16_SHIFTED || c.storage == LBRD_BF16_SHIFTED;
            p.shift[s][i] = shifted ? p.ceq[i] * C(c.rho_ref[s]) : C(0);
        }
        const bool shifted = c.storage == LBRD_F16_SHIFTED || c.storage == LBRD_BF16_SHIFTED;
        p.rho_ref[s] = shifted ? C(c.rho_ref[s]) : C(0);
    }
    if (c.reaction == LBRD_REACT_LINEAR) {
        for (int s = 0; s < n; ++s) {
            for (int j = 0; j < n; ++j) p.K[s * n + j] = C(c.K[s * n + j]);
            p.c[s] = C(c.c[s]);
        }
    }
    if (c.reaction == LBRD_REACT_GRAY_SCOTT) {
        p.F = C(c.F);
        p.k = C(c.k);
        p.Fk = p.F + p.k;
    }
    if (has_shear(c)) {
        p.u0x = C(c.u[0]);
        p.u0y = C(c.u[1]);
        p.amp = C(c.shear[0]);
        p.shear_m = (int32_t)c.shear[1];
        p.shear_ny = c.ny;
    }
    return p;
}
template Params<float> make_params<float>(const lbrd_config &);
template Params<double> make_params<double>(const lbrd_config &);

static int ilog2(int v) {
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

Grid make_grid(const Layout &L, const void *src, void *dst, int vec, int lanes_x) {
    Grid g;
    g.src = src;
    g.dst = dst;
    g.nx = L.nx;
    g.ny = L.ny;
    g.pitch = L.pitch;
    g.pstride = L.pstride;
    g.lanes_x = lanes_x;
    g.lx_shift = ilog2(lanes_x);
    g.nvec = (L.nx + vec - 1) / vec;
    g.nseg = (g.nvec + lanes_x - 1) / lanes_x;
    g.rpw = 64 / lanes_x;
    g.ntiles = (int64_t)g.nseg * ((L.ny + g.rpw - 1) / g.rpw);
    g.blocks = 0;
    g.xcd_order = 1;
    return g;
}

GridT make_gridT(const Layout &L, const void *src, void *dst, int tw, int th, int steps) {
    GridT g;
    g.src = src;
    g.dst = dst;
    g.nx = L.nx;
    g.ny = L.ny;
    g.pitch = L.pitch;
    g.pstride = L.pstride;
    g.tw = tw;
    g.th = th;
    g.ntx = (L.nx + tw - 1) / tw;
    g.nty = (L.ny + th - 1) / th;
    g.ntiles = (int64_t)g.ntx * g.nty;
    g.blocks = 0;
    g.xcd_order = 1;
    g.strip = g.ntx;
    g.steps = steps;
    // a buffer of 4 GiB or more is addressed plane by plane (0: no launch)
    g.bytes = L.buf_bytes < ((size_t)1 << 32) ? (uint32_t)L.buf_bytes : 0;
    const uint64_t plane = (uint64_t)L.pstride * (uint64_t)L.esize;
    g.plane_bytes = plane < ((uint64_t)1 << 32) ? (uint32_t)plane : 0;
    g.nt_store = 0;
    g.march = 0;
    return g;
}

// 16-byte vectors for F64 / F32; 8-byte vectors for the 16-bit forms (half
// the registers of 16-byte ones, measured faster on 4096^2 lattices).
int default_vec(int storage) { return storage == kF64 ? 2 : 4; }

int default_lanes(int nx, int vec) {
    const int nvec = (nx + vec - 1) / vec;
    int l = 1;
    while (l < nvec && l < 64) l <<= 1;
    return l;
}

void fill_batch_inst(BatchInst &bi, const lbrd_config &c, const Layout &L, const void *buf0, const void *buf1,
                     int vec, int lanes_x) {
    std::memset(&bi, 0, sizeof(bi));
    const Grid g = make_grid(L, nullptr, nullptr, vec, lanes_x);
    bi.buf[0] = buf0;
    bi.buf[1] = buf1;
    bi.pitch = L.pitch;
    bi.pstride = L.pstride;
    bi.ntiles = g.ntiles;
    bi.nx = L.nx;
    bi.ny = L.ny;
    bi.lanes_x = lanes_x;
    bi.lx_shift = g.lx_shift;
    bi.nvec = g.nvec;
    bi.nseg = g.nseg;
    bi.rpw = g.rpw;
    bi.storage = c.storage;
    bi.variant = variant_of(c);
    bi.vec = vec;
    if (c.storage == LBRD_F64) bi.pd = make_params<double>(c);
    else bi.pf = make_params<float>(c);
}

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

int validate_config(const lbrd_config *c) {
    if (!c) return LBRD_EINVAL;
    if (c->nspecies < 1 || c->nspecies > LBRD_MAX_SPECIES) return LBRD_EINVAL;
    if (c->nx < 1 || c->ny < 1) return LBRD_EINVAL;
    if ((int64_t)c->nx * c->ny > ((int64_t)1 << 31)) return LBRD_EINVAL;
    if (c->storage < LBRD_F64 || c->storage > LBRD_BF16_SHIFTED) return LBRD_EINVAL;
    if (c->reaction < LBRD_REACT_NONE || c->reaction > LBRD_REACT_GRAY_SCOTT) return LBRD_EINVAL;
    if (c->reaction == LBRD_REACT_GRAY_SCOTT && c->nspecies != 2) return LBRD_EINVAL;
    if (c->reserved != 0) return LBRD_EINVAL;
    for (int s = 0; s < c->nspecies; ++s) {
        if (!(c->tau[s] > 0.5) || !std::isfinite(c->tau[s])) return LBRD_EINVAL;
        if (!std::isfinite(c->rho_ref[s])) return LBRD_EINVAL;
    }
    if (c->reaction == LBRD_REACT_LINEAR) {
        for (int q = 0; q < c->nspecies * c->nspecies; ++q)
            if (!std::isfinite(c->K[q])) return LBRD_EINVAL;
        for (int s = 0; s < c->nspecies; ++s)
            if (!std::isfinite(c->c[s])) return LBRD_EINVAL;
    }
    if (c->reaction == LBRD_REACT_GRAY_SCOTT && (!std::isfinite(c->F) || !std::isfinite(c->k))) return LBRD_EINVAL;
    if (!std::isfinite(c->u[0]) || !std::isfinite(c->u[1])) return LBRD_EINVAL;
    if (c->u[0] != 0.0 || c->u[1] != 0.0) {
        // advective variants: Gray-Scott, or one species with a linear (or no) reaction
        if (!(c->reaction == LBRD_REACT_GRAY_SCOTT || c->nspecies == 1)) return LBRD_EINVAL;
        if (!(c->u[0] * c->u[0] + c->u[1] * c->u[1] < 1.0 / 3.0)) return LBRD_EINVAL;
    }
    if (!std::isfinite(c->shear[0]) || !std::isfinite(c->shear[1])) return LBRD_EINVAL;
    if (c->shear[0] != 0.0) {
        // shear variants: the same reactions, FP64 / FP32 storage, a whole
        // number of periods, |u| below the bound on every row
        if (!(c->reaction == LBRD_REACT_GRAY_SCOTT || c->nspecies == 1)) return LBRD_EINVAL;
        if (c->storage != LBRD_F64 && c->storage != LBRD_F32) return LBRD_EINVAL;
        const double m = c->shear[1];
        if (!(m >= 1.0 && m <= 1e6 && m == std::floor(m))) return LBRD_EINVAL;
        const double umax = std::fabs(c->u[0]) + std::fabs(c->shear[0]);
        if (!(umax * umax + c->u[1] * c->u[1] < 1.0 / 3.0)) return LBRD_EINVAL;
    } else if (c->shear[1] != 0.0) {
        return LBRD_EINVAL;
    }
    return LBRD_OK;
}

// Internal config: NONE runs through the linear kernel with K = 0, c = 0.
lbrd_config normalise(const lbrd_config &c) {
    lbrd_config n = c;
    if (n.reaction == LBRD_REACT_NONE) {
        std::memset(n.K, 0, sizeof(n.K));
        std::memset(n.c, 0, sizeof(n.c));
        n.reaction = LBRD_REACT_LINEAR;
    }
    return n;
}

size_t scratch_bytes() { return (size_t)round_up((kRedBlocks + 1) * kRedSlots * sizeof(double), 4096); }

}  // namespace lbrd

using namespace lbrd;

struct lbrd_solver {
    lbrd_config cfg;       // normalised
    Layout L;
    char *buf[2];
    double *partials;      // kRedBlocks * kRedSlots
    double *result;        // kRedSlots
    hipStream_t stream;
    hipStream_t capture;   // private stream used only to record graphs
    int cur = 0;           // buffer holding the current state
    int64_t t = 0;
    bool initialised = false;
    lbrd_tuning tune;
    alignas(16) unsigned char params[sizeof(Params<double>)];
    hipGraphExec_t graph[2] = {nullptr, nullptr};   // graph_steps steps starting from buf[0] / buf[1]
    int graph_end[2] = {0, 1};                      // buffer holding the state after each graph
    int graph_steps_built = 0;
    int device = 0;
    int cus = 256;
};

namespace {

int fail(const char *where, hipError_t e) {
    set_error(where, e);
    return LBRD_EDEVICE;
}

void drop_graphs(lbrd_solver *h) {
    for (auto &g : h->graph) {
        if (g) hipGraphExecDestroy(g);
        g = nullptr;
    }
    h->graph_steps_built = 0;
}

StepLaunch step_launch(const lbrd_solver *h) {
    return StepLaunch{h->cfg.storage, variant_of(h->cfg), h->tune.vec, h->tune.waves, h->tune.nontemporal != 0};
}

// waves of the one-step launches (the multi-step kernel may use more)
StepLaunch step_launch1(const lbrd_solver *h) {
    StepLaunch sl = step_launch(h);
    if (sl.waves > 4) sl.waves = 4;
    return sl;
}

// Enqueue n steps starting from buf[from]; *end receives the buffer that
// holds the state afterwards.  With fused_steps = T >= 2, launches of T steps
// run while T or more steps remain, then one launch of the 2 .. T-1 left (same
// tiles), then a one-step launch for a single remaining step.
hipError_t enqueue_steps(lbrd_solver *h, int from, int64_t n, hipStream_t st, int *end) {
    const StepLaunch sl = step_launch(h);
    const int T = h->tune.fused_steps;
    int a = from;
    for (int64_t k = 0; k < n;) {
        hipError_t e;
        const int64_t left = n - k;
        if (T >= 2 && left >= 2) {
            const int m = left < T ? (int)left : T;
            if (h->tune.march_rows > 0) {
                // marching wave strips: 64 - 2(m-1) result columns a wave (on
                // buffers of 4 GiB or more the strips of T steps, which the
                // kernel of T steps also runs for m < T)
                const int ts = h->L.buf_bytes >= ((size_t)1 << 32) ? T : m;
                GridT g = make_gridT(h->L, h->buf[a], h->buf[a ^ 1], 64 - 2 * (ts - 1), h->tune.march_rows, m);
                g.march = 1;
                g.xcd_order = h->tune.plain_order == 0 ? 1 : 0;
                g.nt_store = h->tune.nontemporal;
                e = launch_stepT(step_launch1(h), g, h->params, st);
            } else {
                GridT g = make_gridT(h->L, h->buf[a], h->buf[a ^ 1], h->tune.tile_cols, h->tune.tile_rows, m);
                g.blocks = h->tune.blocks_per_cu > 0 ? h->tune.blocks_per_cu * h->cus : 0;
                g.xcd_order = h->tune.plain_order == 0 ? 1 : 0;
                if (h->tune.tile_strip > 0) g.strip = std::min(h->tune.tile_strip, g.ntx);
                g.nt_store = h->tune.nontemporal;
                e = launch_stepT(sl, g, h->params, st);
            }
            k += m;
        } else {
            Grid g = make_grid(h->L, h->buf[a], h->buf[a ^ 1], h->tune.vec, h->tune.lanes_x);
            g.blocks = T == 1 && h->tune.blocks_per_cu > 0 ? h->tune.blocks_per_cu * h->cus : 0;
            g.xcd_order = h->tune.plain_order == 0 ? 1 : 0;
            e = launch_step(step_launch1(h), g, h->params, st);
            k += 1;
        }
        if (e != hipSuccess) return e;
        a ^= 1;
    }
    *end = a;
    return hipSuccess;
}

hipError_t build_graphs(lbrd_solver *h) {
    drop_graphs(h);
    const int n = h->tune.graph_steps;
    for (int from = 0; from < 2; ++from) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t le = enqueue_steps(h, from, n, h->capture, &h->graph_end[from]);
        e = hipStreamEndCapture(h->capture, &graph);
        if (le != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return le;
        }
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&h->graph[from], graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
    }
    h->graph_steps_built = n;
    return hipSuccess;
}

int check_dtype(int dtype) { return (dtype == LBRD_DTYPE_F64 || dtype == LBRD_DTYPE_F32) ? LBRD_OK : LBRD_EINVAL; }

// Stage a host array in the idle ping-pong buffer (large enough: 9 N b >= 8 N
// bytes per site for every storage form).
int stage_host(lbrd_solver *h, const void *host, size_t bytes, const void **dev) {
    char *stage = h->buf[h->cur ^ 1];
    if (bytes > h->L.buf_bytes) return LBRD_ENOMEM;
    hipError_t e = hipMemcpyAsync(stage, host, bytes, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return fail("hipMemcpyAsync", e);
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail("hipStreamSynchronize", e);
    *dev = stage;
    return LBRD_OK;
}

// The multi-step kernel addresses a buffer, or each plane of a buffer of
// 4 GiB or more, with 32-bit byte offsets.
// Row offsets are formed with 24-bit multiplies (row index times row pitch),
// so rows and pitches must also stay below 2^24.
bool big_buffers(const lbrd_solver *h) { return h->L.buf_bytes >= ((size_t)1 << 32); }
bool multi_step_possible(const lbrd_solver *h) {
    return (uint64_t)h->L.pstride * (uint64_t)h->L.esize < ((uint64_t)1 << 32) &&
           (int64_t)h->L.pitch * storage_bytes(h->cfg.storage) < ((int64_t)1 << 24) &&
           h->L.ny <= (1 << 24);
}

// Tile order of multi-step launches.  Row-major over a wide lattice puts
// the tiles above and below a running one a whole tile row away in launch
// order: with fewer workgroups resident on an XCD than tiles in a row, the
// halo rows they share have left the XCD's L2 by then and are fetched again
// (4096^2 FP32 at T = 7 on 32 x 12 tiles reads 2.0x the algorithmic bytes).
// Strips of S tile columns, S = half the workgroups one XCD holds at once
// (LDS-limited, 32 CUs per XCD, at most 32 waves per CU), keep about two
// tile rows of a strip in flight.  Measured per step against row-major:
// 4096^2 FP32 115 against 128 us, 4096^2 FP64 309 against 347 us, 2048^2
// FP64 73 against 84 us; 2048^2 FP32 (64 tiles across, within twice S)
// 2-5 % slower, hence row-major up to 2S tiles across (up to 2S - 1 in
// the 16-bit forms).
int strip_width(const lbrd_solver *h, const lbrd_tuning &t) {
    const size_t lds = stepT_lds_bytes(h->cfg.storage, h->cfg.nspecies, t.tile_cols, t.tile_rows, t.fused_steps);
    if (lds == 0 || t.waves < 1) return 1;
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(kLdsBytes / lds, (size_t)(32 / t.waves)));
    return std::max(1, per_cu * std::max(1, h->cus / 8) / 2);
}
int tiles_across(const lbrd_solver *h, const lbrd_tuning &t) { return (h->cfg.nx + t.tile_cols - 1) / t.tile_cols; }
int default_strip(const lbrd_solver *h, const lbrd_tuning &t) {
    // exactly 2S tiles across: strips measured 1-1.3 % faster for the 16-bit
    // forms (4096^2 on 64 x 20 tiles), 2-5 % slower in FP32 (2048^2, 32 x 12)
    const int strip = strip_width(h, t), across = tiles_across(h, t);
    const bool narrow16 = storage_bytes(h->cfg.storage) == 2 && across == 2 * strip;
    return across > 2 * strip || narrow16 ? strip : 0;
}

struct MarchShape {
    int steps = 0;      // steps per launch; 0: the LDS tiles
    int rows = 0;       // rows per segment; 0: sized for k waves per SIMD
    int waves = 0;      // waves per workgroup
    int k = 1;
};

int max_march_steps(const lbrd_solver *h) { return h->cfg.storage == LBRD_F64 ? kMaxFusedSteps : kMaxMarchSteps; }

// Rows per segment of a marching launch of `steps` steps that make strips x
// segments about k waves per SIMD (k x 4 x CUs in all), with segments as
// long as that allows: each segment reads about 2 x steps rows around it
// again, so longer segments move fewer bytes.  k = 1 is one round of the
// launch where the kernel's registers leave one wave per SIMD.
int march_rows_for(const lbrd_solver *h, int steps, int k) {
    const int u = 64 - 2 * (steps - 1);
    const int64_t strips = (h->cfg.nx + u - 1) / u;
    const int64_t segs = std::max<int64_t>(1, (int64_t)4 * h->cus * k / strips);
    return (int)((h->cfg.ny + segs - 1) / segs);
}

// The default marching shape, or steps 0 where the LDS tiles measured
// faster.  Marching strips recompute only the x-halo and keep no tile in
// LDS; they win wherever the state streams from HBM (beyond the 256 MB
// Infinity Cache, "beyond"), and inside it from 1024^2 sites in FP32 and
// FP64.  Measured per step against the LDS defaults and the shapes these
// replace (64-row segments, at most 8 steps a launch; "big": more than
// 2048^2 sites; k: the segments' waves per SIMD):
//   Gray-Scott and two linear species: FP32 beyond T 10 when big (4096^2:
//     63.5 against 84.5 and 110.8 us), else T 9 (2048^2: 18.1 against 26.7),
//     k 1; FP32 inside from 1024^2 T 7, k 1 (5.80 against 6.54).  F16 beyond
//     T 8 when big (54.3 against 58.3), else T 7 (16.1 against 17.5), BF16
//     one step fewer (57.7 against 57.8; 16.7 against 18.1), k 3.  FP64
//     beyond T 8, k 1 (155.5 against 171.7; 2048^2 39.2 against 59.3; 1024^2
//     11.0 against 16.4; T 7 was best before FP64 strips stored from every
//     lane: 166.4, 42.7, 11.5); inside from 512^2 T 6, 8 rows, one-wave workgroups
//     (4.45 against 4.54).  F16 once its population sums read the packed
//     halves in place: 49.7 us at 4096^2 (T 8), 14.8 at 2048^2 (T 7); and
//     inside the cache from 1024^2, k 2: T 6 (5.43 against 5.57), from
//     1448^2 T 5 (8.24 against 9.10); BF16 inside from 1448^2 T 4, k 3 (9.21
//     against 9.61), below it LDS tiles (1024^2 5.64 against 5.97; F16 at
//     768^2 3.66 against 4.03).
//   One linear species: FP32 beyond T 11, k 2 (29.2 against 40.4; 2048^2 8.54
//     against 10.9), inside from 1024^2 T 7, k 1 (3.01 against 3.49); F16
//     beyond T 7, k 4 when big (30.5 against 30.6), else T 5, k 3 (8.75
//     against 8.96; inside the cache from 1448^2 T 5, k 2, 5.26 against 5.64,
//     and k 3 from 2048^2, 8.64 against 8.98); BF16 beyond and big T 6, k 4
//     (32.9 against 33.0), else LDS tiles (2048^2 inside the cache: 9.01
//     against 9.44 in one run, 9.62 against 9.21 in another); FP64 beyond T
//     8, k 1 (64.7 against 78.7; 2048^2 17.9 against 20.6), inside from
//     1024^2 (4.14 against 4.60).
//   Three species: FP32 beyond T 8, k 3 when big (132.5 against 147.7), else
//     k 1 (33.8 against 42.9), inside from 1024^2 T 6, k 1 (10.5 against
//     15.6); F16 beyond T 6, k 1 when big (109.2 against 123.0), else k 2
//     (28.4 against 29.8); BF16 beyond T 5, 16 rows when big (F16 at the
//     time 123.2; k 1 126.6), else k 2 (F16 30.0 against 34.0).  Four
//     species: FP32 beyond T 5, k 4 when big (271.1 against 278.6), else
//     k 1, one-wave workgroups (68.6 against 72.5); F16 beyond T 5, one-wave
//     workgroups, k 3 when big (195.3 against 205.5), else k 1 (51.2
//     against 52.6).
//   Shear flow, FP32 beyond: T 5, Gray-Scott k 2 when big (134.0 against
//     177.4), else k 1 (2048^2 36.2 against 47.1), one species k 3 (63.8
//     against 80.6; 2048^2 17.9 against 28.9).  Uniform velocity: one
//     species, 16-bit beyond, T 5, k 4 when big (BF16 38.3 against 39.3, F16
//     36.7 against 37.2), else T 6, 64 rows; FP32 T 9, k 2 (33.7 against
//     50.6; 2048^2 9.94 against 14.7); Gray-Scott FP32 beyond T 7, k 2 when
//     big (82.7 against 118.1), else k 1 (22.6 against 31.3), 16-bit beyond
//     T 6, k 3 when big (F16 66.2 against 80.3), else F16 T 6, BF16 T 5, k 3
//     (2048^2 18.5 against 22.0, 19.9 against 22.2).
//   FP64 beyond the cache, once its strips stored from every lane: three
//     species T 5, k 1 (4096^2 336.3 against 997.8; 2048^2 85.3 against
//     211.5); four species T 4, k 1, one-wave workgroups (2048^2 165.4
//     against 288.0); shear flow Gray-Scott T 4, k 4 when big, else k 1
//     (293.1 against 387.3; 75.3 against 93.0), one species T 6, k 1
//     (118.5 against 210.2); uniform velocity Gray-Scott T 8 when big,
//     else 7, k 1 (166.4 against 313.1; 44.8 against 73.8), one species T 8,
//     k 1 (65.4 against 105.5).
// The step counts above 8 trade a wider x-halo (2(T-1) of a wave's 64
// columns) for fewer passes over HBM; where a form's registers run out
// (FP32 with three or four species above T 8) its time jumps.  Forms not
// measured keep the LDS tiles (FP64 inside the cache with three or more
// species or a shear or a velocity, one species inside the cache below
// 1024^2).
MarchShape march_default(const lbrd_solver *h, bool in_cache, int64_t sites) {
    const int st = h->cfg.storage;
    const bool f64 = st == LBRD_F64, f32 = st == LBRD_F32, f16 = st == LBRD_F16_SHIFTED, b16 = !f64 && !f32;
    const bool big = sites > (int64_t)2048 * 2048, mid = sites >= (int64_t)1024 * 1024;
    const int v = variant_of(h->cfg);
    switch (v) {
        case kGS:
        case kLin2:
            if (in_cache) {
                if (f32 && mid) return {7, 0, 4, 1};
                if (f16 && mid) return {sites >= (int64_t)1448 * 1448 ? 5 : 6, 0, 4, 2};
                if (b16 && sites >= (int64_t)1448 * 1448) return {4, 0, 4, 3};
                if (f64 && sites >= (int64_t)512 * 512) return {6, 8, 1, 1};
                return {};
            }
            if (f32) return {big ? 10 : 9, 0, 4, 1};
            if (f64) return {8, 0, 4, 1};
            if (f16) return {big ? 8 : 7, 0, 4, 3};
            return {big ? 7 : 6, 0, 4, 3};
        case kLin1:
            if (in_cache) {
                if (f32 && mid) return {7, 0, 4, 1};
                if (f64 && mid) return {8, 0, 4, 1};
                if (f16 && sites >= (int64_t)1448 * 1448) return {5, 0, 4, sites >= (int64_t)2048 * 2048 ? 3 : 2};
                return {};
            }
            if (f32) return {11, 0, 4, 2};
            if (f64) return {8, 0, 4, 1};
            if (f16) return big ? MarchShape{7, 0, 4, 4} : MarchShape{5, 0, 4, 3};
            return big ? MarchShape{6, 0, 4, 4} : MarchShape{};
        case kLin3:
            if (f64) return in_cache ? MarchShape{} : MarchShape{5, 0, 4, 1};
            if (in_cache) return f32 && mid ? MarchShape{6, 0, 4, 1} : MarchShape{};
            if (f32) return {8, 0, 4, big ? 3 : 1};
            if (f16) return {6, 0, 4, big ? 1 : 2};
            return big ? MarchShape{5, 16, 4, 1} : MarchShape{5, 0, 4, 2};
        case kLin4:
            if (in_cache) return {};
            if (f64) return {4, 0, 1, 1};
            if (f32) return big ? MarchShape{5, 0, 4, 4} : MarchShape{5, 0, 1, 1};
            if (f16) return {5, 0, 1, big ? 3 : 1};
            return {};
        case kShearLin1:
        case kShearGS:
            if (in_cache) return {};
            if (f64) return v == kShearGS ? MarchShape{4, 0, 4, big ? 4 : 1} : MarchShape{6, 0, 4, 1};
            if (!f32) return {};
            return {5, 0, 4, v == kShearGS ? (big ? 2 : 1) : 3};
        case kAdvLin1:
            if (in_cache) return {};
            if (f64) return {8, 0, 4, 1};
            if (f32) return {9, 0, 4, 2};
            return big ? MarchShape{5, 0, 4, 4} : MarchShape{6, 64, 4, 1};
        case kAdvGS:
            if (in_cache) return {};
            if (f32) return {7, 0, 4, big ? 2 : 1};
            if (f64) return {big ? 8 : 7, 0, 4, 1};
            return {big || f16 ? 6 : 5, 0, 4, 3};
        default:
            return {};
    }
}

bool tuning_valid(const lbrd_solver *h, const lbrd_tuning &t) {
    // the one-step shape is used for every one-step launch (also the odd
    // remainder of a fused run)
    if (!step_shape_valid(h->cfg.storage, t.vec, t.lanes_x, std::min(t.waves, 4))) return false;
    if (t.blocks_per_cu < 0 || t.blocks_per_cu > 64) return false;
    if (t.plain_order != 0 && t.plain_order != 1) return false;
    if (t.tile_strip < 0 || t.tile_strip > 65536) return false;
    if (t.march_rows < 0 || t.march_rows > 65536) return false;
    if (t.march_rows > 0 && t.fused_steps >= 2 && big_buffers(h) &&
        !march_big_ok(h->cfg.storage, variant_of(h->cfg), t.fused_steps))
        return false;
    if (t.graph_steps < 0 || (t.graph_steps & 1) || t.graph_steps > 4096) return false;
    if (t.nontemporal != 0 && t.nontemporal != 1) return false;
    if (t.waves < 1 || t.waves > 16) return false;
    if (t.fused_steps == 1) return true;
    if (!multi_step_possible(h)) return false;
    // marching wave strips: no LDS tile
    if (t.march_rows > 0) return t.fused_steps >= 2 && t.fused_steps <= max_march_steps(h);
    if (t.fused_steps < 2 || t.fused_steps > kMaxFusedSteps) return false;
    if (t.tile_rows < 1 || t.tile_rows > 64) return false;
    if (big_buffers(h) && t.tile_cols == 128) return false;   // plane-by-plane launches: 32 or 64 wide
    return stepT_shape_fits(h->cfg.storage, h->cfg.nspecies, t.tile_cols, t.tile_rows, t.fused_steps, t.waves);
}

}  // namespace

extern "C" {

const char *lbrd_strerror(int status) {
    switch (status) {
        case LBRD_OK: return "ok";
        case LBRD_EINVAL: return "invalid argument";
        case LBRD_ENOMEM: return "workspace too small";
        case LBRD_EDEVICE: return g_last_error.empty() ? "HIP runtime error" : g_last_error.c_str();
        case LBRD_ENONFINITE: return "non-finite reduction result";
        case LBRD_ESTATE: return "call out of order (not initialised)";
        case LBRD_ENOTFOUND: return "unknown ticket";
        case LBRD_ETIMEOUT: return "timed out";
        default: return "unknown status";
    }
}

const char *lbrd_version(void) { return "lbrd 0.1 gfx950"; }

int lbrd_validate(const lbrd_config *cfg) { return validate_config(cfg); }

int lbrd_workspace_size(const lbrd_config *cfg, size_t *bytes) {
    int rc = validate_config(cfg);
    if (rc) return rc;
    if (!bytes) return LBRD_EINVAL;
    const Layout L = make_layout(*cfg);
    *bytes = 2 * L.buf_bytes + scratch_bytes();
    return LBRD_OK;
}

int lbrd_create(const lbrd_config *cfg, void *workspace, size_t bytes, void *stream, lbrd_solver **out) {
    int rc = validate_config(cfg);
    if (rc) return rc;
    if (!out || !workspace || ((uintptr_t)workspace & 255)) return LBRD_EINVAL;
    size_t need = 0;
    lbrd_workspace_size(cfg, &need);
    if (bytes < need) return LBRD_ENOMEM;
    lbrd_solver *h = new (std::nothrow) lbrd_solver();
    if (!h) return LBRD_ENOMEM;
    h->cfg = normalise(*cfg);
    h->L = make_layout(h->cfg);
    h->buf[0] = static_cast<char *>(workspace);
    h->buf[1] = h->buf[0] + h->L.buf_bytes;
    h->partials = reinterpret_cast<double *>(h->buf[1] + h->L.buf_bytes);
    h->result = h->partials + (size_t)kRedBlocks * kRedSlots;
    h->stream = static_cast<hipStream_t>(stream);
    hipGetDevice(&h->device);
    h->cus = device_cu_count();
    hipError_t e = hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete h;
        return fail("hipStreamCreateWithFlags", e);
    }
    if (h->cfg.storage == LBRD_F64) {
        Params<double> p = make_params<double>(h->cfg);
        std::memcpy(h->params, &p, sizeof(p));
    } else {
        Params<float> p = make_params<float>(h->cfg);
        std::memcpy(h->params, &p, sizeof(p));
    }
    std::memset(&h->tune, 0, sizeof(h->tune));
    h->tune.vec = default_vec(h->cfg.storage);
    h->tune.lanes_x = default_lanes(h->cfg.nx, h->tune.vec);
    h->tune.waves = 4;
    const int64_t sites = (int64_t)h->cfg.nx * h->cfg.ny;
    if (2 * h->L.buf_bytes > ((size_t)256 << 20)) {
        // one-step launches (odd remainders) beyond the 256 MB Infinity
        // Cache: streaming accesses and the shapes measured fastest on
        // 4096^2 lattices
        h->tune.nontemporal = 1;
        if (h->cfg.storage == LBRD_F32 || h->cfg.storage == LBRD_F64) {
            h->tune.vec = 2;
            h->tune.lanes_x = default_lanes(h->cfg.nx, 2);
        } else if (h->cfg.storage == LBRD_F16_SHIFTED) {
            h->tune.vec = 8;
            h->tune.lanes_x = std::min(32, default_lanes(h->cfg.nx, 8));
        }
    }
    // Several steps per launch on tiles staged in LDS (temporal blocking).
    // The shape is taken from measurements (8 waves per workgroup, T steps
    // per launch, cols x rows tiles), keyed by the bytes B of one site's
    // populations and by whether both buffers fit in the 256 MB Infinity
    // Cache; one species with a linear reaction is cheaper per site and
    // takes more steps per launch:
    //   inside the cache: B <= 18: T 5, 64 x 24; B <= 36: one species T 8,
    //     32 x 32, else T 5, 32 x 24; B <= 72: T 5, 32 x 10; beyond: T 6,
    //     32 x 16;
    //   beyond it: B <= 36: one species T 8, 64 x 14, else T 6, 64 x 20;
    //     B <= 72: T 7, 32 x 12; beyond: T 6, 32 x 16.
    // (1024^2 FP32 Gray-Scott: 6.6 us per step against 7.3 at T = 4; 4096^2:
    // 125 us against 149 in FP32, 76 against 85 in FP16.)  A shape that does
    // not fit in LDS first loses rows (down to 4), then steps per launch.
    // Cached loads, streaming stores beyond the Infinity Cache (4 % faster at
    // 4096^2; 40 % slower inside it), consecutive tiles on one XCD (each
    // measured best).  Buffers of 4 GiB or more are addressed plane by plane
    // (planes below 4 GiB; else one-step launches, 64-bit offsets).
    const bool in_cache = 2 * h->L.buf_bytes <= ((size_t)256 << 20);
    const int site_bytes = 9 * h->cfg.nspecies * storage_bytes(h->cfg.storage);
    const bool cheap = h->cfg.nspecies == 1;
    int ts0, cols, rows0;
    if (site_bytes <= 18) {
        ts0 = in_cache ? 5 : 6; cols = 64; rows0 = in_cache ? 24 : 20;
    } else if (site_bytes <= 36) {
        if (cheap) { ts0 = 8; cols = in_cache ? 32 : 64; rows0 = in_cache ? 32 : 14; }
        else { ts0 = in_cache ? 5 : 6; cols = in_cache ? 32 : 64; rows0 = in_cache ? 24 : 20; }
    } else if (site_bytes <= 72) {
        ts0 = in_cache ? 5 : 7; cols = 32; rows0 = in_cache ? 10 : 12;
    } else {
        ts0 = 6; cols = 32; rows0 = 16;
    }
    // Small lattices are bound by the latency of a launch, not by a
    // throughput: more steps per launch on tiles small enough to give most
    // CUs one (per step against the table above: 64^2 FP64 decay 0.87
    // against 1.17 us, 128^2 FP32 Gray-Scott 1.03 against 1.38, 128^2 FP64
    // Gray-Scott 1.31 against 2.12, 256^2 1.22 against 1.48, 384^2 1.76
    // against 2.20, 512^2 2.32 against 2.65).
    if (in_cache && sites <= 512 * 512) {
        if (sites <= 128 * 128) { ts0 = 8; cols = 32; rows0 = 4; }
        else if (sites <= 256 * 256) { ts0 = 8; cols = 32; rows0 = 8; }
        else if (sites <= 384 * 384) { ts0 = 7; cols = 32; rows0 = 20; }
        else { ts0 = 7; cols = 64; rows0 = 16; }
    }
    h->tune.tile_cols = cols;
    h->tune.tile_rows = rows0;
    h->tune.fused_steps = 1;
    if (multi_step_possible(h)) {
        h->tune.waves = 8;
        h->tune.nontemporal = in_cache ? 0 : 1;
        h->tune.plain_order = 0;
        for (int min_rows : {4, 1})
            for (int ts = ts0; ts >= 2 && h->tune.fused_steps == 1; --ts)
                for (int rows = rows0; rows >= min_rows; rows /= 2)
                    if (stepT_shape_fits(h->cfg.storage, h->cfg.nspecies, cols, rows, ts, 8)) {
                        h->tune.fused_steps = ts;
                        h->tune.tile_rows = rows;
                        break;
                    }
        if (h->tune.fused_steps > 1) h->tune.tile_strip = default_strip(h, h->tune);
    }
    // Marching wave strips replace the LDS tiles where they measured faster.
    MarchShape ms = march_default(h, in_cache, sites);
    if (ms.steps > 0 && big_buffers(h)) {
        // buffers of 4 GiB or more: marching strips with a descriptor per
        // plane (march_big_ok), 8 steps a launch, segments for 3 waves per
        // SIMD (8192^2 FP32 Gray-Scott 317 us per step against 686 on the
        // LDS tiles and 420 with 10 steps in one round; 12288^2 F16 554
        // against 820)
        ms.steps = march_big_ok(h->cfg.storage, variant_of(h->cfg), 8) ? 8 : 0;
        ms.rows = 0;
        ms.k = 3;
        ms.waves = 4;
    }
    if (h->tune.fused_steps > 1 && ms.steps > 0) {
        h->tune.fused_steps = ms.steps;
        h->tune.march_rows = ms.rows > 0 ? ms.rows : march_rows_for(h, ms.steps, ms.k);
        h->tune.waves = ms.waves;
        h->tune.nontemporal = 0;
        h->tune.tile_strip = 0;
    }
    // Captured graphs pay where one-step launches on a small lattice are
    // bound by the host's launch rate; multi-step launches keep the GPU busy
    // longer than a launch takes (plain launches measured 4-10 % faster on
    // 64^2 to 512^2 lattices).
    h->tune.graph_steps = h->tune.fused_steps == 1 && sites <= (1 << 18) ? 32 : 0;
    *out = h;
    return LBRD_OK;
}

int lbrd_destroy(lbrd_solver *h) {
    if (!h) return LBRD_OK;
    drop_graphs(h);
    if (h->capture) hipStreamDestroy(h->capture);
    delete h;
    return LBRD_OK;
}

int lbrd_init(lbrd_solver *h, const void *rho0, int dtype, int on_device) {
    if (!h || !rho0 || check_dtype(dtype)) return LBRD_EINVAL;
    const size_t bytes = (size_t)h->cfg.nspecies * h->cfg.nx * h->cfg.ny * (dtype == LBRD_DTYPE_F64 ? 8 : 4);
    const void *src = rho0;
    if (!on_device) {
        int rc = stage_host(h, rho0, bytes, &src);
        if (rc) return rc;
    }
    hipError_t e = launch_init(h->cfg.storage, h->L, h->params, src, dtype, h->buf[h->cur], h->stream);
    if (e != hipSuccess) return fail("init kernel", e);
    h->t = 0;
    h->initialised = true;
    return LBRD_OK;
}

int lbrd_set_populations(lbrd_solver *h, const void *f, int dtype, int on_device) {
    if (!h || !f || check_dtype(dtype)) return LBRD_EINVAL;
    const int planes = 9 * h->cfg.nspecies;
    const size_t plane_bytes = (size_t)h->cfg.nx * h->cfg.ny * (dtype == LBRD_DTYPE_F64 ? 8 : 4);
    if (on_device) {
        hipError_t e = launch_set_populations(h->cfg.storage, h->L, h->params, f, dtype, 0, planes, h->buf[h->cur],
                                              h->stream);
        if (e != hipSuccess) return fail("set_populations kernel", e);
    } else {
        // host source: staged through the idle buffer, as many planes at a time as fit
        const int per = (int)std::max<size_t>(1, h->L.buf_bytes / plane_bytes);
        for (int p0 = 0; p0 < planes; p0 += per) {
            const int p1 = std::min(planes, p0 + per);
            const void *src = nullptr;
            int rc = stage_host(h, static_cast<const char *>(f) + p0 * plane_bytes, (p1 - p0) * plane_bytes, &src);
            if (rc) return rc;
            hipError_t e = launch_set_populations(h->cfg.storage, h->L, h->params, src, dtype, p0, p1,
                                                  h->buf[h->cur], h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return fail("set_populations kernel", e);
        }
    }
    h->t = 0;
    h->initialised = true;
    return LBRD_OK;
}

int lbrd_get_populations(lbrd_solver *h, void *f_out, int dtype) {
    if (!h || !f_out || check_dtype(dtype)) return LBRD_EINVAL;
    if (!h->initialised) return LBRD_ESTATE;
    hipError_t e = launch_get_populations(h->cfg.storage, h->L, h->params, h->buf[h->cur], f_out, dtype, h->stream);
    return e == hipSuccess ? LBRD_OK : fail("get_populations kernel", e);
}

int lbrd_step(lbrd_solver *h, int64_t nsteps) {
    if (!h || nsteps < 0) return LBRD_EINVAL;
    if (!h->initialised) return LBRD_ESTATE;
    int64_t left = nsteps;
    const int gs = h->tune.graph_steps;
    if (gs > 0 && left >= gs) {
        if (h->graph_steps_built != gs) {
            hipError_t e = build_graphs(h);
            if (e != hipSuccess) {
                drop_graphs(h);
                return fail("graph capture", e);
            }
        }
        while (left >= gs) {
            hipError_t e = hipGraphLaunch(h->graph[h->cur], h->stream);
            if (e != hipSuccess) return fail("hipGraphLaunch", e);
            h->cur = h->graph_end[h->cur];
            left -= gs;
            h->t += gs;
        }
    }
    int end = h->cur;
    hipError_t e = enqueue_steps(h, h->cur, left, h->stream, &end);
    if (e != hipSuccess) return fail("step kernel", e);
    h->cur = end;
    h->t += left;
    return LBRD_OK;
}

int lbrd_moments(lbrd_solver *h, void *rho_out, int dtype, double *mass_out) {
    if (!h || (rho_out && check_dtype(dtype))) return LBRD_EINVAL;
    if (!h->initialised) return LBRD_ESTATE;
    if (!rho_out && !mass_out) return LBRD_OK;
    hipError_t e = launch_moments(h->cfg.storage, h->L, h->params, h->buf[h->cur], rho_out, dtype, nullptr, 0,
                                  h->partials, h->result, h->stream);
    if (e != hipSuccess) return fail("moments kernel", e);
    if (!mass_out) return LBRD_OK;
    double res[kRedSlots];
    e = hipMemcpyAsync(res, h->result, sizeof(res), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail("moments readback", e);
    int rc = LBRD_OK;
    for (int s = 0; s < h->cfg.nspecies; ++s) {
        mass_out[s] = res[s];
        if (!std::isfinite(res[s])) rc = LBRD_ENONFINITE;
    }
    return rc;
}

int lbrd_rel_l2(lbrd_solver *h, const void *ref, int dtype, double *err_out) {
    if (!h || !ref || !err_out || check_dtype(dtype)) return LBRD_EINVAL;
    if (!h->initialised) return LBRD_ESTATE;
    hipError_t e = launch_moments(h->cfg.storage, h->L, h->params, h->buf[h->cur], nullptr, LBRD_DTYPE_F64, ref,
                                  dtype, h->partials, h->result, h->stream);
    if (e != hipSuccess) return fail("moments kernel", e);
    double res[kRedSlots];
    e = hipMemcpyAsync(res, h->result, sizeof(res), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail("rel_l2 readback", e);
    int rc = LBRD_OK;
    for (int s = 0; s < h->cfg.nspecies; ++s) {
        const double num = res[LBRD_MAX_SPECIES + s], den = res[2 * LBRD_MAX_SPECIES + s];
        err_out[s] = den > 0 ? std::sqrt(num / den) : std::sqrt(num);
        if (!std::isfinite(err_out[s])) rc = LBRD_ENONFINITE;
    }
    return rc;
}

int lbrd_spectrum_work_size(int nx, int ny, size_t *bytes) {
    if (nx < 1 || ny < 1 || !bytes) return LBRD_EINVAL;
    *bytes = spectrum_work_bytes(nx, ny);
    return LBRD_OK;
}

int lbrd_spectrum(lbrd_solver *h, int species, void *out, void *work, size_t work_bytes) {
    if (!h || !out || !work || species < 0 || species >= h->cfg.nspecies) return LBRD_EINVAL;
    if (((uintptr_t)work & 255) || ((uintptr_t)out & 7)) return LBRD_EINVAL;
    if (work_bytes < spectrum_work_bytes(h->cfg.nx, h->cfg.ny)) return LBRD_ENOMEM;
    if (!h->initialised) return LBRD_ESTATE;
    hipError_t e = launch_spectrum(h->cfg.storage, h->L, h->params, h->buf[h->cur], species, static_cast<double *>(out),
                                   work, h->partials, h->result, h->stream);
    return e == hipSuccess ? LBRD_OK : fail("spectrum kernels", e);
}

static_assert(LBRD_SPECTRUM_STATIC_MAX_SITES == kStaticSpectrumSites &&
                  LBRD_SPECTRUM_STATIC_BYTES == kStaticSpectrumBytes,
              "the header states the static spectrum scratch's limits");

int lbrd_spectrum_static(lbrd_solver *h, int species, void *out) {
    if (!h || !out || species < 0 || species >= h->cfg.nspecies) return LBRD_EINVAL;
    if ((uintptr_t)out & 7) return LBRD_EINVAL;
    if ((int64_t)h->cfg.nx * h->cfg.ny > kStaticSpectrumSites ||
        spectrum_work_bytes(h->cfg.nx, h->cfg.ny) > kStaticSpectrumBytes)
        return LBRD_ENOMEM;
    if (!h->initialised) return LBRD_ESTATE;
    void *work = nullptr;   // this device's fixed array: nothing is allocated
    hipError_t e = static_spectrum_scratch(h->device, &work);
    if (e != hipSuccess) return fail("hipGetSymbolAddress (spectrum scratch)", e);
    e = launch_spectrum(h->cfg.storage, h->L, h->params, h->buf[h->cur], species, static_cast<double *>(out), work,
                        h->partials, h->result, h->stream);
    return e == hipSuccess ? LBRD_OK : fail("spectrum kernels", e);
}

int lbrd_time(const lbrd_solver *h, int64_t *t) {
    if (!h || !t) return LBRD_EINVAL;
    *t = h->t;
    return LBRD_OK;
}

int lbrd_get_tuning(const lbrd_solver *h, lbrd_tuning *out) {
    if (!h || !out) return LBRD_EINVAL;
    *out = h->tune;
    return LBRD_OK;
}

int lbrd_set_tuning(lbrd_solver *h, const lbrd_tuning *t) {
    if (!h || !t) return LBRD_EINVAL;
    lbrd_tuning n = *t;
    if (n.lanes_x == 0) n.lanes_x = default_lanes(h->cfg.nx, n.vec);
    if (n.fused_steps > 1 && n.tile_cols == 0) n.tile_cols = 64;
    if (!tuning_valid(h, n)) return LBRD_EINVAL;
    const bool rebuild = std::memcmp(&n, &h->tune, sizeof(n)) != 0;
    h->tune = n;
    if (rebuild) drop_graphs(h);
    return LBRD_OK;
}

int lbrd_time_steps(lbrd_solver *h, int64_t nsteps, double *ms) {
    if (!h || !ms || nsteps < 0) return LBRD_EINVAL;
    if (!h->initialised) return LBRD_ESTATE;
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return fail("hipEventCreate", e);
    e = hipEventCreate(&b);
    if (e != hipSuccess) {
        hipEventDestroy(a);
        return fail("hipEventCreate", e);
    }
    int rc = LBRD_OK;
    e = hipEventRecord(a, h->stream);
    if (e == hipSuccess) {
        rc = lbrd_step(h, nsteps);
        if (rc == LBRD_OK) {
            e = hipEventRecord(b, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float f = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
            *ms = f;
        }
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (rc) return rc;
    return e == hipSuccess ? LBRD_OK : fail("event timing", e);
}

int lbrd_autotune(lbrd_solver *h, int steps, const char *cache_path, lbrd_tuning *chosen) {
    if (!h || steps < 2) return LBRD_EINVAL;
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::string arch = "gfx";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    std::ostringstream key;
    key << arch << " st=" << h->cfg.storage << " v=" << variant_of(h->cfg) << " nx=" << h->cfg.nx
        << " ny=" << h->cfg.ny;
    const std::string k = key.str();
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            const size_t bar = line.find('|');
            if (bar == std::string::npos || line.substr(0, bar) != k) continue;
            lbrd_tuning t;
            std::memset(&t, 0, sizeof(t));
            if (std::sscanf(line.c_str() + bar + 1, "%d %d %d %d %d %d %d %d %d %d %d %d", &t.vec, &t.lanes_x,
                            &t.waves, &t.nontemporal, &t.graph_steps, &t.plain_order, &t.blocks_per_cu,
                            &t.fused_steps, &t.tile_rows, &t.tile_cols, &t.tile_strip, &t.march_rows) == 12 &&
                tuning_valid(h, t)) {
                lbrd_set_tuning(h, &t);
                h->initialised = false;
                if (chosen) *chosen = h->tune;
                return LBRD_OK;
            }
        }
    }
    // Candidate shapes: every valid vector width, row-segment width up to the
    // row, waves per workgroup, streaming or cached accesses, tile order,
    // one tile per wave or a persistent grid; and multi-step launches over
    // steps per launch, tile widths and heights and workgroup sizes.
    std::vector<lbrd_tuning> cands;
    const int vecs[3] = {2, 4, 8};
    for (int vec : vecs) {
        const int lmax = default_lanes(h->cfg.nx, vec);
        for (int lx = std::max(1, lmax / 4); lx <= lmax; lx <<= 1)
            for (int w : {1, 2, 4})
                for (int nt = 0; nt < 2; ++nt)
                    for (int order = 0; order < 2; ++order)
                        for (int bpc : {0, 8}) {
                            lbrd_tuning t;
                            std::memset(&t, 0, sizeof(t));
                            t.vec = vec;
                            t.lanes_x = lx;
                            t.waves = w;
                            t.nontemporal = nt;
                            t.plain_order = order;
                            t.blocks_per_cu = bpc;
                            t.fused_steps = 1;
                            t.graph_steps = 0;
                            if (tuning_valid(h, t)) cands.push_back(t);
                        }
    }
    for (int ts = 2; ts <= kMaxFusedSteps; ++ts)
        for (int cols : {32, 64, 128})
            for (int rows : {4, 8, 12, 16, 20, 24, 32})
                for (int w : {4, 8})
                    for (int nt = 0; nt < 2; ++nt)
                        for (int order = 0; order < 1; ++order) {
                            lbrd_tuning t = h->tune;
                            t.vec = default_vec(h->cfg.storage);
                            t.lanes_x = default_lanes(h->cfg.nx, t.vec);
                            t.waves = w;
                            t.nontemporal = nt;
                            t.plain_order = order;
                            t.blocks_per_cu = 0;
                            t.fused_steps = ts;
                            t.tile_rows = rows;
                            t.tile_cols = cols;
                            t.tile_strip = 0;
                            t.march_rows = 0;
                            t.graph_steps = 0;
                            if (!tuning_valid(h, t)) continue;
                            t.tile_strip = default_strip(h, t);
                            cands.push_back(t);
                        }
    // marching wave strips: steps per launch, segment lengths (fixed, or
    // sized for k = 1 .. 4 waves per SIMD), waves per workgroup, streaming
    // stores
    for (int ts = 2; ts <= max_march_steps(h); ++ts)
        for (int r : {16, 32, 64, -1, -2, -3, -4})
            for (int w : {1, 4})
                for (int nt = 0; nt < 2; ++nt) {
                    const int rows = r > 0 ? r : march_rows_for(h, ts, -r);
                    lbrd_tuning t = h->tune;
                    t.vec = default_vec(h->cfg.storage);
                    t.lanes_x = default_lanes(h->cfg.nx, t.vec);
                    t.waves = w;
                    t.nontemporal = nt;
                    t.plain_order = 0;
                    t.blocks_per_cu = 0;
                    t.fused_steps = ts;
                    t.march_rows = rows;
                    t.tile_strip = 0;
                    t.graph_steps = 0;
                    if (tuning_valid(h, t)) cands.push_back(t);
                }
    // the state is scratch from here on.  Timings depend a little on the
    // data (an all-zero field runs faster than real states and favours other
    // shapes), so an initialised solver is timed on its own state and an
    // uninitialised one on a scrambled field of densities in [0.5, 1).
    if (!h->initialised) {
        const std::vector<double> rho = scrambled_densities((size_t)h->cfg.nspecies * h->cfg.nx * h->cfg.ny);
        if (int rc = lbrd_init(h, rho.data(), LBRD_DTYPE_F64, 0)) return rc;
    }
    const lbrd_tuning entry = h->tune;   // the shape in use: always a finalist
    // milliseconds per step of one candidate (whole launches only, running
    // for at least min_ms), or +inf
    auto time_one = [&](const lbrd_tuning &t, double min_ms) {
        if (lbrd_set_tuning(h, &t) != LBRD_OK) return 1e300;
        double ms = 0;
        const int per = std::max(1, (int)t.fused_steps);
        int n = (steps + per - 1) / per * per;
        int rc = lbrd_time_steps(h, per, &ms);   // warm-up
        if (rc == LBRD_OK) rc = lbrd_time_steps(h, n, &ms);
        if (rc == LBRD_OK && ms < min_ms) {
            // short runs are dominated by launch jitter and by clocks that
            // have not settled: grow the run to about min_ms
            const double grow = std::min(256.0, min_ms / std::max(ms, 1e-3));
            n = ((int)(n * grow) + per - 1) / per * per;
            rc = lbrd_time_steps(h, n, &ms);
        }
        return rc == LBRD_OK ? ms / n : 1e300;
    };
    // first pass: every candidate for about 1 ms
    std::vector<std::pair<double, lbrd_tuning>> timed;
    for (const lbrd_tuning &t : cands) timed.emplace_back(time_one(t, 1.0), t);
    std::stable_sort(timed.begin(), timed.end(),
                     [](const auto &a, const auto &b) { return a.first < b.first; });
    // second pass, runs of about 10 ms: the six fastest, the default shape,
    // and the three fastest multi-step shapes with the other tile order
    // (XCD-grouped or the hardware's round-robin; row-major or strips:
    // which one wins depends on the lattice and the shape)
    std::vector<lbrd_tuning> finals;
    for (size_t q = 0; q < timed.size() && finals.size() < 6; ++q)
        if (timed[q].first < 1e300) finals.push_back(timed[q].second);
    finals.push_back(entry);
    int flipped = 0;
    for (size_t q = 0; q < timed.size() && flipped < 3; ++q) {
        if (timed[q].second.fused_steps < 2 || timed[q].first >= 1e300) continue;
        lbrd_tuning t = timed[q].second;
        t.plain_order ^= 1;
        finals.push_back(t);
        t.plain_order ^= 1;
        t.tile_strip = t.tile_strip ? 0 : strip_width(h, t);
        if (t.tile_strip < tiles_across(h, t)) finals.push_back(t);
        ++flipped;
    }
    double best = 1e300;
    lbrd_tuning best_t = entry;
    for (const lbrd_tuning &t : finals) {
        const double ms = time_one(t, 10.0);
        if (ms < best) {
            best = ms;
            best_t = t;
        }
    }
    // the winner with captured graphs of 32 steps, or without them
    lbrd_tuning flip = best_t;
    flip.graph_steps = best_t.graph_steps ? 0 : 32;
    if (time_one(flip, 10.0) < best) best_t = flip;
    lbrd_set_tuning(h, &best_t);
    h->initialised = false;
    h->t = 0;
    if (cache_path) {
        std::ofstream outf(cache_path, std::ios::app);
        outf << k << "|" << best_t.vec << " " << best_t.lanes_x << " " << best_t.waves << " " << best_t.nontemporal
             << " " << best_t.graph_steps << " " << best_t.plain_order << " " << best_t.blocks_per_cu << " "
             << best_t.fused_steps << " " << best_t.tile_rows << " " << best_t.tile_cols << " " << best_t.tile_strip
             << " " << best_t.march_rows
             << "\n";
    }
    if (chosen) *chosen = h->tune;
    return LBRD_OK;
}

const char *lbrd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
