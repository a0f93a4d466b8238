// Host side of batched solving: many independent lattices advanced by one
// persistent launch per step, with the launches of a chunk replayed from a
// captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "lbrd.h"
#include "lbrd_internal.h"
#include "lbrd_util.h"

using namespace lbrd;

namespace {

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

struct BatchPlan {
    size_t hdr_off, inst_off, scratch_off, bufs_off, total;
    std::vector<size_t> buf_off;   // per instance, first of its two buffers
};

BatchPlan plan_batch(const lbrd_config *cfgs, int count) {
    BatchPlan p;
    p.hdr_off = 0;
    p.inst_off = 256;
    p.scratch_off = (size_t)round_up(p.inst_off + sizeof(BatchInst) * (size_t)count, 4096);
    p.bufs_off = p.scratch_off + scratch_bytes();
    size_t off = p.bufs_off;
    for (int i = 0; i < count; ++i) {
        const Layout L = make_layout(normalise(cfgs[i]));
        p.buf_off.push_back(off);
        off += 2 * L.buf_bytes;
    }
    p.total = off;
    return p;
}

int pick_set(const std::vector<lbrd_config> &cfgs) {
    bool gs_f32 = true, serve = true;
    for (const auto &c : cfgs) {
        const int v = variant_of(c);
        if (!(c.storage == LBRD_F32 && v == kGS)) gs_f32 = false;
        if (c.storage == LBRD_F64 || !(v == kGS || v == kLin1)) serve = false;
    }
    return gs_f32 ? kBatchGSF32 : (serve ? kBatchServe : kBatchAny);
}

}  // namespace

struct lbrd_batch {
    int count = 0;
    std::vector<lbrd_config> cfg;   // normalised
    std::vector<Layout> L;
    std::vector<BatchInst> inst;    // host mirror of the device descriptors
    std::vector<char> initialised;
    std::vector<int64_t> tinst;     // steps taken per instance since init
    BatchHeader *d_hdr = nullptr;
    BatchInst *d_inst = nullptr;
    double *partials = nullptr, *result = nullptr;
    hipStream_t stream = nullptr, capture = nullptr;
    int set = kBatchAny;
    int cus = 256;
    int64_t total_tiles = 0;
    lbrd_tuning tune;
    bool dirty = true;              // descriptors need uploading
    hipGraphExec_t graph = nullptr;
    int graph_steps_built = 0;
    int64_t t = 0;
    bool multi_ok = false;          // every instance can take multi-step launches
    int march_mask = 0;             // classes of the batched marching kernel present
    // with several classes, one branch stream per class (forked from the
    // launch stream and joined back, also inside a recorded graph)
    hipStream_t branch[kMarchClasses] = {};
    hipEvent_t fork = nullptr, join[kMarchClasses] = {};
};

namespace {

int fail(const char *where, hipError_t e) {
    set_error(where, e);
    return LBRD_EDEVICE;
}

void release_streams(lbrd_batch *b) {
    for (int c = 0; c < kMarchClasses; ++c) {
        if (b->branch[c]) hipStreamDestroy(b->branch[c]);
        if (b->join[c]) hipEventDestroy(b->join[c]);
    }
    if (b->fork) hipEventDestroy(b->fork);
    if (b->capture) hipStreamDestroy(b->capture);
}

void drop_graph(lbrd_batch *b) {
    if (b->graph) hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_steps_built = 0;
}

int steps_per_launch(const lbrd_batch *b) { return b->tune.fused_steps; }
bool marching(const lbrd_batch *b) { return b->tune.fused_steps > 1 && b->tune.march_rows > 0; }

int64_t blocks_of(const lbrd_batch *b) {
    if (marching(b)) {
        // one wave per strip segment, or a persistent grid of blocks_per_cu
        // workgroups per CU
        const int64_t need = (b->total_tiles + b->tune.waves - 1) / b->tune.waves;
        if (b->tune.blocks_per_cu == 0) return std::max<int64_t>(1, need);
        return std::max<int64_t>(1, std::min<int64_t>((int64_t)b->tune.blocks_per_cu * b->cus, need));
    }
    if (steps_per_launch(b) > 1) {
        // one workgroup per tile, or a persistent grid of blocks_per_cu per CU
        const int64_t need = b->total_tiles;
        if (b->tune.blocks_per_cu == 0) return std::max<int64_t>(1, need);
        return std::max<int64_t>(1, std::min<int64_t>((int64_t)b->tune.blocks_per_cu * b->cus, need));
    }
    int64_t blocks = (int64_t)b->tune.blocks_per_cu * b->cus;
    const int64_t need = (b->total_tiles + b->tune.waves - 1) / b->tune.waves;
    return std::max<int64_t>(1, std::min(blocks, need));
}

// Tile every instance for the current launch kind and lay the tiles out one
// instance after another; the header follows on the batch stream.
hipError_t retile(lbrd_batch *b) {
    int64_t tiles = 0;
    for (int i = 0; i < b->count; ++i) {
        BatchInst &bi = b->inst[i];
        if (marching(b)) set_batch_tiling_march(bi, b->L[i], steps_per_launch(b), b->tune.march_rows);
        else set_batch_tiling(bi, b->L[i], steps_per_launch(b), b->tune.tile_rows, b->tune.tile_cols);
        bi.tile_begin = tiles;
        tiles += bi.ntiles;
    }
    b->total_tiles = tiles;
    b->dirty = true;
    BatchHeader h;
    std::memset(&h, 0, sizeof(h));
    h.count = b->count;
    h.nt_store = steps_per_launch(b) > 1 ? b->tune.nontemporal : 0;
    h.total_tiles = tiles;
    hipError_t e = hipMemcpyAsync(b->d_hdr, &h, sizeof(h), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e;
}

hipError_t upload(lbrd_batch *b, int steps) {
    bool changed = b->dirty;
    for (auto &bi : b->inst) {
        if (bi.steps != steps) changed = true;
        bi.steps = steps;
    }
    if (!changed) return hipSuccess;
    b->dirty = false;
    return hipMemcpyAsync(b->d_inst, b->inst.data(), sizeof(BatchInst) * b->inst.size(), hipMemcpyHostToDevice,
                          b->stream);
}

// Enqueue the launches j = 0 .. launches-1 of a chunk.
hipError_t enqueue(lbrd_batch *b, int64_t launches, hipStream_t st) {
    const int ts = steps_per_launch(b);
    if (marching(b) && b->fork) {
        // several classes: each runs its chain of launches on a branch of its
        // own (they touch disjoint instances), so the classes overlap
        hipError_t e = hipEventRecord(b->fork, st);
        for (int cls = 0; cls < kMarchClasses && e == hipSuccess; ++cls) {
            if (!(b->march_mask & (1 << cls))) continue;
            e = hipStreamWaitEvent(b->branch[cls], b->fork, 0);
            for (int64_t j = 0; j < launches && e == hipSuccess; ++j)
                e = launch_batch_stepW(b->d_hdr, b->d_inst, (int)j, blocks_of(b), b->tune.waves, ts, cls,
                                       b->branch[cls]);
            if (e == hipSuccess) e = hipEventRecord(b->join[cls], b->branch[cls]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, b->join[cls], 0);
        }
        return e;
    }
    for (int64_t j = 0; j < launches; ++j) {
        hipError_t e = hipSuccess;
        if (marching(b)) {
            // one launch per class present (each at its own registers)
            for (int cls = 0; cls < kMarchClasses && e == hipSuccess; ++cls)
                if (b->march_mask & (1 << cls))
                    e = launch_batch_stepW(b->d_hdr, b->d_inst, (int)j, blocks_of(b), b->tune.waves, ts, cls, st);
        } else {
            e = ts > 1 ? launch_batch_stepT(b->d_hdr, b->d_inst, (int)j, blocks_of(b), b->tune.waves, ts,
                                            b->tune.tile_rows, b->tune.tile_cols, b->set, st)
                       : launch_batch_step(b->d_hdr, b->d_inst, (int)j, (int)blocks_of(b), b->tune.waves,
                                           b->tune.nontemporal != 0, b->set, st);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t build_graph(lbrd_batch *b) {
    drop_graph(b);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = enqueue(b, launches_for(b->tune.graph_steps, steps_per_launch(b)), b->capture);
    e = hipStreamEndCapture(b->capture, &g);
    if (le != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e == hipSuccess) b->graph_steps_built = b->tune.graph_steps;
    return e;
}

bool batch_tuning_valid(const lbrd_batch *b, const lbrd_tuning &t) {
    if (t.nontemporal != 0 && t.nontemporal != 1) return false;
    if (t.graph_steps < 0 || t.graph_steps > 4096) return false;
    if (t.fused_steps == 1)
        return (t.waves == 1 || t.waves == 2 || t.waves == 4) && t.blocks_per_cu >= 1 && t.blocks_per_cu <= 32 &&
               !(t.graph_steps & 1);
    // multi-step launches: an even number of launches per captured chunk, so
    // every instance ends a chunk in the buffer it started from
    if (!b->multi_ok || t.fused_steps < 2) return false;
    if (t.fused_steps > (t.march_rows > 0 ? kMaxBatchMarchSteps : kMaxBatchFusedSteps)) return false;
    if (t.graph_steps % (2 * t.fused_steps)) return false;
    if (t.blocks_per_cu < 0 || t.blocks_per_cu > 32) return false;
    if (t.march_rows < 0 || t.march_rows > 65536) return false;
    if (t.march_rows > 0) return t.waves == 1 || t.waves == 2 || t.waves == 4;   // marching strips: no LDS
    return batch_shape_fits(t.fused_steps, t.tile_rows, t.tile_cols, t.waves);
}

const void *params_of(const lbrd_batch *b, int idx) {
    const BatchInst &bi = b->inst[idx];
    return b->cfg[idx].storage == LBRD_F64 ? (const void *)&bi.pd : (const void *)&bi.pf;
}

}  // namespace

extern "C" {

int lbrd_batch_workspace_size(const lbrd_config *cfgs, int count, size_t *bytes) {
    if (!cfgs || count < 1 || !bytes) return LBRD_EINVAL;
    for (int i = 0; i < count; ++i) {
        if (int rc = validate_config(&cfgs[i])) return rc;
        if (has_shear(cfgs[i])) return LBRD_EINVAL;   // single solvers only
    }
    *bytes = plan_batch(cfgs, count).total;
    return LBRD_OK;
}

int lbrd_batch_create(const lbrd_config *cfgs, int count, void *workspace, size_t bytes, void *stream,
                      lbrd_batch **out) {
    size_t need = 0;
    if (int rc = lbrd_batch_workspace_size(cfgs, count, &need)) return rc;
    if (!out || !workspace || ((uintptr_t)workspace & 255)) return LBRD_EINVAL;
    if (bytes < need) return LBRD_ENOMEM;
    lbrd_batch *b = new (std::nothrow) lbrd_batch();
    if (!b) return LBRD_ENOMEM;
    const BatchPlan p = plan_batch(cfgs, count);
    char *base = static_cast<char *>(workspace);
    b->count = count;
    b->stream = static_cast<hipStream_t>(stream);
    b->d_hdr = reinterpret_cast<BatchHeader *>(base + p.hdr_off);
    b->d_inst = reinterpret_cast<BatchInst *>(base + p.inst_off);
    b->partials = reinterpret_cast<double *>(base + p.scratch_off);
    b->result = b->partials + (size_t)kRedBlocks * kRedSlots;
    for (int i = 0; i < count; ++i) {
        const lbrd_config c = normalise(cfgs[i]);
        const Layout L = make_layout(c);
        char *b0 = base + p.buf_off[i];
        const int vec = batch_vec(c.storage);
        BatchInst bi;
        fill_batch_inst(bi, c, L, b0, b0 + L.buf_bytes, vec, default_lanes(c.nx, vec));
        bi.cur = 0;
        b->cfg.push_back(c);
        b->L.push_back(L);
        b->inst.push_back(bi);
    }
    b->initialised.assign(count, 0);
    b->tinst.assign(count, 0);
    b->set = pick_set(b->cfg);
    b->cus = device_cu_count();
    b->multi_ok = b->set != kBatchAny;
    for (const lbrd_config &c : b->cfg) {
        const int cls = march_class(c.storage, variant_of(c));
        if (cls >= 0) b->march_mask |= 1 << cls;
    }
    for (int i = 0; i < count; ++i)
        if (!batch_multi_ok(b->L[i], b->cfg[i].storage)) b->multi_ok = false;
    std::memset(&b->tune, 0, sizeof(b->tune));
    if (b->multi_ok) {
        // while the buffers fit in the Infinity Cache, five steps per launch
        // on 32 x 10 LDS tiles (the LDS of both sets is sized for it), one
        // workgroup of 8 waves per tile; beyond it, marching wave strips
        // (nine steps per launch, segments of 128 rows, one wave per
        // segment, four to a workgroup: on the benchmark's 256-instance
        // Gray-Scott sweep 120.6 us per step, against 129.0 with eight
        // steps, 143.2 with ten, 145.2 with seven on 64 rows, 134.5 with nine
        // on 256); graphs of about 32 steps (an even number of launches)
        size_t bytes = 0;
        for (const Layout &L : b->L) bytes += 2 * L.buf_bytes;
        const bool in_cache = bytes <= ((size_t)256 << 20);
        b->tune.fused_steps = in_cache ? 5 : 9;
        b->tune.tile_rows = in_cache ? 10 : 0;
        b->tune.tile_cols = in_cache ? 32 : 0;
        b->tune.march_rows = in_cache ? 0 : 128;
        b->tune.waves = in_cache ? 8 : 4;
        b->tune.blocks_per_cu = 0;
        const int unit = 2 * b->tune.fused_steps;
        b->tune.graph_steps = std::max(1, (32 + unit / 2) / unit) * unit;
        b->tune.nontemporal = 0;
    } else {
        b->tune.fused_steps = 1;
        b->tune.waves = 4;
        b->tune.blocks_per_cu = 8;
        b->tune.graph_steps = 16;
    }
    hipError_t e = retile(b);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e == hipSuccess && __builtin_popcount(b->march_mask) > 1) {
        e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        for (int c = 0; c < kMarchClasses && e == hipSuccess; ++c)
            if (b->march_mask & (1 << c)) {
                e = hipStreamCreateWithFlags(&b->branch[c], hipStreamNonBlocking);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[c], hipEventDisableTiming);
            }
    }
    if (e != hipSuccess) {
        release_streams(b);
        delete b;
        return fail("batch create", e);
    }
    *out = b;
    return LBRD_OK;
}

int lbrd_batch_destroy(lbrd_batch *b) {
    if (!b) return LBRD_OK;
    drop_graph(b);
    release_streams(b);
    delete b;
    return LBRD_OK;
}

int lbrd_batch_init(lbrd_batch *b, int idx, const void *rho0, int dtype, int on_device) {
    if (!b || idx < 0 || idx >= b->count || !rho0) return LBRD_EINVAL;
    if (dtype != LBRD_DTYPE_F64 && dtype != LBRD_DTYPE_F32) return LBRD_EINVAL;
    BatchInst &bi = b->inst[idx];
    const lbrd_config &c = b->cfg[idx];
    const void *src = rho0;
    char *cur = static_cast<char *>(const_cast<void *>(bi.buf[bi.cur]));
    char *idle = static_cast<char *>(const_cast<void *>(bi.buf[bi.cur ^ 1]));
    if (!on_device) {
        const size_t bytes = (size_t)c.nspecies * c.nx * c.ny * (dtype == LBRD_DTYPE_F64 ? 8 : 4);
        hipError_t e = hipMemcpyAsync(idle, rho0, bytes, hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return fail("batch init copy", e);
        src = idle;
    }
    hipError_t e = launch_init(c.storage, b->L[idx], params_of(b, idx), src, dtype, cur, b->stream);
    if (e != hipSuccess) return fail("batch init kernel", e);
    b->initialised[idx] = 1;
    b->tinst[idx] = 0;
    return LBRD_OK;
}

int lbrd_batch_step(lbrd_batch *b, int64_t nsteps) {
    if (!b || nsteps < 0) return LBRD_EINVAL;
    for (char v : b->initialised)
        if (!v) return LBRD_ESTATE;
    int64_t left = nsteps;
    const int gs = b->tune.graph_steps;
    if (gs > 0 && left >= gs) {
        hipError_t e = upload(b, gs);
        if (e != hipSuccess) return fail("batch descriptors", e);
        if (b->graph_steps_built != gs) {
            e = build_graph(b);
            if (e != hipSuccess) {
                drop_graph(b);
                return fail("batch graph capture", e);
            }
        }
        while (left >= gs) {
            e = hipGraphLaunch(b->graph, b->stream);
            if (e != hipSuccess) return fail("hipGraphLaunch", e);
            left -= gs;
            b->t += gs;
            for (auto &t : b->tinst) t += gs;
        }
    }
    while (left > 0) {
        const int n = (int)std::min<int64_t>(left, 1 << 20);
        const int64_t launches = launches_for(n, steps_per_launch(b));
        hipError_t e = upload(b, n);
        if (e == hipSuccess) e = enqueue(b, launches, b->stream);
        if (e != hipSuccess) return fail("batch step", e);
        if (launches & 1) {
            for (auto &bi : b->inst) bi.cur ^= 1;
            b->dirty = true;
        }
        left -= n;
        b->t += n;
        for (auto &t : b->tinst) t += n;
    }
    return LBRD_OK;
}

int lbrd_batch_advance(lbrd_batch *b, const int64_t *nsteps) {
    if (!b || !nsteps) return LBRD_EINVAL;
    for (int i = 0; i < b->count; ++i) {
        if (nsteps[i] < 0) return LBRD_EINVAL;
        if (nsteps[i] > 0 && !b->initialised[i]) return LBRD_ESTATE;
    }
    std::vector<int64_t> left(nsteps, nsteps + b->count);
    const int ts = steps_per_launch(b);
    const int chunk = b->tune.graph_steps > 0 ? b->tune.graph_steps : 64 * ts;
    for (;;) {
        int most = 0;
        for (int i = 0; i < b->count; ++i) {
            const int n = (int)std::min<int64_t>(left[i], chunk);
            b->inst[i].steps = n;
            most = std::max(most, n);
        }
        if (most == 0) break;
        hipError_t e = hipMemcpyAsync(b->d_inst, b->inst.data(), sizeof(BatchInst) * b->inst.size(),
                                      hipMemcpyHostToDevice, b->stream);
        if (e != hipSuccess) return fail("batch descriptors", e);
        b->dirty = false;
        if (b->tune.graph_steps > 0) {
            // the captured chunk runs graph_steps launches; instances stop at
            // their own step limit inside it
            if (b->graph_steps_built != b->tune.graph_steps) {
                e = build_graph(b);
                if (e != hipSuccess) {
                    drop_graph(b);
                    return fail("batch graph capture", e);
                }
            }
            e = hipGraphLaunch(b->graph, b->stream);
        } else {
            e = enqueue(b, launches_for(most, ts), b->stream);
        }
        if (e != hipSuccess) return fail("batch advance", e);
        for (int i = 0; i < b->count; ++i) {
            const int n = b->inst[i].steps;
            left[i] -= n;
            b->tinst[i] += n;
            b->inst[i].cur ^= (int)(launches_for(n, ts) & 1);
        }
        b->dirty = true;
    }
    return LBRD_OK;
}

int lbrd_batch_spectrum(lbrd_batch *b, int idx, int species, void *out, void *work, size_t work_bytes) {
    if (!b || idx < 0 || idx >= b->count || !out || !work) return LBRD_EINVAL;
    if (species < 0 || species >= b->cfg[idx].nspecies) return LBRD_EINVAL;
    if (((uintptr_t)work & 255) || ((uintptr_t)out & 7)) return LBRD_EINVAL;
    if (work_bytes < spectrum_work_bytes(b->cfg[idx].nx, b->cfg[idx].ny)) return LBRD_ENOMEM;
    if (!b->initialised[idx]) return LBRD_ESTATE;
    const BatchInst &bi = b->inst[idx];
    hipError_t e = launch_spectrum(b->cfg[idx].storage, b->L[idx], params_of(b, idx), bi.buf[bi.cur], species,
                                   static_cast<double *>(out), work, b->partials, b->result, b->stream);
    return e == hipSuccess ? LBRD_OK : fail("batch spectrum", e);
}

int lbrd_batch_time(const lbrd_batch *b, int idx, int64_t *t) {
    if (!b || !t || idx < 0 || idx >= b->count) return LBRD_EINVAL;
    *t = b->tinst[idx];
    return LBRD_OK;
}

int lbrd_batch_rel_l2(lbrd_batch *b, int idx, const void *ref, int dtype, double *err_out) {
    if (!b || idx < 0 || idx >= b->count || !ref || !err_out) return LBRD_EINVAL;
    if (dtype != LBRD_DTYPE_F64 && dtype != LBRD_DTYPE_F32) return LBRD_EINVAL;
    if (!b->initialised[idx]) return LBRD_ESTATE;
    const BatchInst &bi = b->inst[idx];
    hipError_t e = launch_moments(b->cfg[idx].storage, b->L[idx], params_of(b, idx), bi.buf[bi.cur], nullptr,
                                  LBRD_DTYPE_F64, ref, dtype, b->partials, b->result, b->stream);
    if (e != hipSuccess) return fail("batch rel_l2", e);
    double res[kRedSlots];
    e = hipMemcpyAsync(res, b->result, sizeof(res), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail("batch rel_l2 readback", e);
    int rc = LBRD_OK;
    for (int s = 0; s < b->cfg[idx].nspecies; ++s) {
        const double num = res[LBRD_MAX_SPECIES + s], den = res[2 * LBRD_MAX_SPECIES + s];
        err_out[s] = den > 0 ? std::sqrt(num / den) : std::sqrt(num);
        if (!std::isfinite(err_out[s])) rc = LBRD_ENONFINITE;
    }
    return rc;
}

int lbrd_batch_moments(lbrd_batch *b, int idx, void *rho_out, int dtype, double *mass_out) {
    if (!b || idx < 0 || idx >= b->count) return LBRD_EINVAL;
    if (rho_out && dtype != LBRD_DTYPE_F64 && dtype != LBRD_DTYPE_F32) return LBRD_EINVAL;
    if (!b->initialised[idx]) return LBRD_ESTATE;
    if (!rho_out && !mass_out) return LBRD_OK;
    const BatchInst &bi = b->inst[idx];
    hipError_t e = launch_moments(b->cfg[idx].storage, b->L[idx], params_of(b, idx), bi.buf[bi.cur], rho_out, dtype,
                                  nullptr, 0, b->partials, b->result, b->stream);
    if (e != hipSuccess) return fail("batch moments", e);
    if (!mass_out) return LBRD_OK;
    double res[kRedSlots];
    e = hipMemcpyAsync(res, b->result, sizeof(res), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail("batch moments readback", e);
    int rc = LBRD_OK;
    for (int s = 0; s < b->cfg[idx].nspecies; ++s) {
        mass_out[s] = res[s];
        if (!std::isfinite(res[s])) rc = LBRD_ENONFINITE;
    }
    return rc;
}

int lbrd_batch_get_populations(lbrd_batch *b, int idx, void *f_out, int dtype) {
    if (!b || idx < 0 || idx >= b->count || !f_out) return LBRD_EINVAL;
    if (dtype != LBRD_DTYPE_F64 && dtype != LBRD_DTYPE_F32) return LBRD_EINVAL;
    if (!b->initialised[idx]) return LBRD_ESTATE;
    const BatchInst &bi = b->inst[idx];
    hipError_t e = launch_get_populations(b->cfg[idx].storage, b->L[idx], params_of(b, idx), bi.buf[bi.cur], f_out,
                                          dtype, b->stream);
    return e == hipSuccess ? LBRD_OK : fail("batch get_populations", e);
}

int lbrd_batch_get_tuning(const lbrd_batch *b, lbrd_tuning *out) {
    if (!b || !out) return LBRD_EINVAL;
    *out = b->tune;
    return LBRD_OK;
}

int lbrd_batch_set_tuning(lbrd_batch *b, const lbrd_tuning *t) {
    if (!b || !t) return LBRD_EINVAL;
    lbrd_tuning n = *t;
    n.vec = 0;
    n.lanes_x = 0;
    n.plain_order = 0;
    n.tile_strip = 0;
    if (n.fused_steps == 1) n.march_rows = 0;
    if (n.fused_steps == 1 || n.march_rows > 0) n.tile_rows = 0;
    if (n.fused_steps == 1 || n.march_rows > 0) n.tile_cols = 0;
    else if (n.tile_cols == 0) n.tile_cols = 64;
    if (!batch_tuning_valid(b, n)) return LBRD_EINVAL;
    if (std::memcmp(&n, &b->tune, sizeof(n)) == 0) return LBRD_OK;
    const bool tiling = n.fused_steps != b->tune.fused_steps || n.tile_rows != b->tune.tile_rows ||
                        n.tile_cols != b->tune.tile_cols || n.nontemporal != b->tune.nontemporal ||
                        n.march_rows != b->tune.march_rows;
    drop_graph(b);
    b->tune = n;
    if (tiling) {
        hipError_t e = retile(b);
        if (e != hipSuccess) return fail("batch retile", e);
    }
    return LBRD_OK;
}

int lbrd_batch_time_steps(lbrd_batch *b, int64_t nsteps, double *ms) {
    if (!b || !ms || nsteps < 0) return LBRD_EINVAL;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail("hipEventCreate", hipErrorUnknown);
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return fail("hipEventCreate", hipErrorUnknown);
    }
    hipError_t e = hipEventRecord(e0, b->stream);
    int rc = LBRD_OK;
    if (e == hipSuccess) {
        rc = lbrd_batch_step(b, nsteps);
        if (rc == LBRD_OK) {
            e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float f = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
            *ms = f;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    return e == hipSuccess ? LBRD_OK : fail("batch timing", e);
}

int lbrd_batch_autotune(lbrd_batch *b, int steps, lbrd_tuning *chosen) {
    if (!b || steps < 2) return LBRD_EINVAL;
    // The states are scratch from here on.  An all-zero field runs faster
    // than real states and favours other shapes, so instances that have not
    // been initialised are timed on a scrambled field of densities in
    // [0.5, 1); initialised ones on their own state.
    for (int i = 0; i < b->count; ++i) {
        if (b->initialised[i]) continue;
        const lbrd_config &c = b->cfg[i];
        const std::vector<double> rho = scrambled_densities((size_t)c.nspecies * c.nx * c.ny);
        if (int rc = lbrd_batch_init(b, i, rho.data(), LBRD_DTYPE_F64, 0)) return rc;
    }
    const lbrd_tuning keep = b->tune;
    // candidates: persistent one-step launches over blocks per CU, waves and
    // streaming accesses; multi-step launches over steps per launch, tile
    // heights and workgroup sizes (one workgroup per tile)
    std::vector<lbrd_tuning> cands;
    for (int bpc : {1, 2, 4, 8, 16})
        for (int w : {1, 2, 4})
            for (int nt = 0; nt < 2; ++nt) {
                lbrd_tuning t = keep;
                t.fused_steps = 1;
                t.tile_rows = 0;
                t.tile_cols = 0;
                t.blocks_per_cu = bpc;
                t.waves = w;
                t.nontemporal = nt;
                cands.push_back(t);
            }
    if (b->multi_ok)
        for (int ts = 2; ts <= kMaxBatchFusedSteps; ++ts)
            for (int cols : {32, 64})
                for (int rows : {4, 8, 12, 16, 20})
                    for (int w : {4, 8})
                        for (int nt = 0; nt < 2; ++nt) {
                        lbrd_tuning t = keep;
                        t.fused_steps = ts;
                        t.tile_cols = cols;
                        t.tile_rows = rows;
                        t.blocks_per_cu = 0;
                        t.waves = w;
                        t.nontemporal = nt;
                        t.march_rows = 0;
                        cands.push_back(t);
                    }
    if (b->multi_ok)
        for (int ts = 4; ts <= kMaxBatchMarchSteps; ++ts)
            for (int rows : {16, 32, 64, 128, 256})
                for (int w : {1, 4}) {
                    lbrd_tuning t = keep;
                    t.fused_steps = ts;
                    t.march_rows = rows;
                    t.tile_cols = 0;
                    t.tile_rows = 0;
                    t.blocks_per_cu = 0;
                    t.waves = w;
                    t.nontemporal = 0;
                    cands.push_back(t);
                }
    lbrd_tuning best = keep;
    double best_ms = 1e300;
    for (lbrd_tuning t : cands) {
        t.graph_steps = 0;
        if (lbrd_batch_set_tuning(b, &t) != LBRD_OK) continue;
        double ms = 0;
        // whole launches only, compared per step; short runs are dominated by
        // launch jitter, so each candidate runs for about 1 ms at least
        const int per = std::max(1, (int)t.fused_steps);
        int n = (steps + per - 1) / per * per;
        if (lbrd_batch_time_steps(b, per, &ms) != LBRD_OK) continue;
        if (lbrd_batch_time_steps(b, n, &ms) != LBRD_OK) continue;
        if (ms < 1.0) {
            const double grow = std::min(64.0, 1.0 / std::max(ms, 1e-3));
            n = ((int)(n * grow) + per - 1) / per * per;
            if (lbrd_batch_time_steps(b, n, &ms) != LBRD_OK) continue;
        }
        ms /= n;
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
            // the caller's chunk length, rounded up to an even number of launches
            const int unit = best.fused_steps > 1 ? 2 * best.fused_steps : 2;
            best.graph_steps = keep.graph_steps > 0 ? (keep.graph_steps + unit - 1) / unit * unit : 0;
        }
    }
    lbrd_batch_set_tuning(b, &best);
    for (int i = 0; i < b->count; ++i) b->initialised[i] = 0;
    for (auto &t : b->tinst) t = 0;
    for (auto &bi : b->inst) bi.cur = 0;
    b->dirty = true;
    b->t = 0;
    if (chosen) *chosen = b->tune;
    return LBRD_OK;
}

}  // extern "C"
