// Continuous-batching solve server.
//
// A worker thread owns the GPU side.  Each round it
//   1. admits queued requests (FIFO order, skipping ones that do not fit yet)
//      while slots and arena space allow, copies their initial densities and
//      runs the init kernel into their slot;
//   2. advances every resident request by min(chunk, steps left) with a
//      replayed graph of persistent batched launches (per-slot step limits
//      live in device descriptors, so the graph is reused across rounds);
//      rounds of the serving mix advance seven steps per launch, on
//      marching wave strips when the resident buffers exceed the Infinity
//      Cache, else on LDS tiles;
//   3. enqueues the density read-out of requests that finish in this round
//      and records an event;
//   4. while the GPU works on that round, retires the previous round's
//      finished requests: waits for its event, copies densities and FP64
//      masses to host memory, frees their arena blocks and wakes waiters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lbrd.h"
#include "lbrd_internal.h"
#include "lbrd_util.h"

using namespace lbrd;

namespace {

constexpr size_t kAlign = 4096;

size_t align_up(size_t a, size_t b) { return (a + b - 1) / b * b; }

// First-fit allocator over [begin, end) of the arena, coalescing on free.
class Arena {
   public:
    void reset(size_t begin, size_t end) {
        free_.clear();
        if (end > begin) free_[begin] = end - begin;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align_up(bytes, kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes, kAlign);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

   private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, peak_ = 0;
};

struct Request {
    int64_t id = 0;
    lbrd_config cfg;   // normalised
    Layout L;
    std::vector<double> rho0;
    int64_t steps = 0, left = 0;
    int state = 0;     // 0 queued, 1 resident, 2 done, 3 rejected
    double submit_s = 0, admit_s = 0, done_s = 0;
    size_t footprint = 0, off = 0;
    int cur = 0;       // buffer holding the state
    std::vector<double> rho, mass;
    int status = LBRD_OK;
};

size_t request_footprint(const lbrd_config &c, Layout *Lout) {
    const Layout L = make_layout(c);
    if (Lout) *Lout = L;
    const size_t sites = (size_t)c.nx * c.ny;
    return 2 * L.buf_bytes + align_up(sites * c.nspecies * sizeof(double), kAlign) + kAlign;
}

}  // namespace

struct lbrd_server {
    lbrd_server_config sc;
    char *base = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;   // compute (owned)
    hipStream_t copy = nullptr;     // read-back copies
    hipStream_t capture = nullptr;  // graph recording only
    // one branch per marching kernel class in a recorded round (forked from
    // and joined back to the capture stream), so that the classes overlap
    hipStream_t branch[kMarchClasses] = {};
    hipEvent_t fork = nullptr, join[kMarchClasses] = {};
    BatchHeader *d_hdr = nullptr;
    BatchInst *d_inst = nullptr;
    double *partials = nullptr;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Request> reqs;
    std::vector<int64_t> resident;
    std::thread worker;
    bool stop = false;
    bool failed = false;
    int64_t next_id = 1;
    int cus = 256;
    // per kernel set; [3]: multi-step serve on LDS tiles
    hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
    // multi-step serve on marching strips, per set of kernel classes present
    std::map<int, hipGraphExec_t> march_graph;
    std::chrono::steady_clock::time_point t0;
    lbrd_server_stats stats;
    double busy_since = -1;
    double arena_since = 0;   // server clock of the last arena accounting

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void mark_busy(lbrd_server *s) {
    // caller holds the lock
    const double t = s->now();
    if (!s->resident.empty() && s->busy_since < 0) s->busy_since = t;
    if (s->resident.empty() && s->busy_since >= 0) {
        s->stats.busy_s += t - s->busy_since;
        s->busy_since = -1;
    }
}

// Integral of the arena bytes in use over the server clock, brought up to
// now; called (with the lock held) before every change of the bytes in use.
void account_arena(lbrd_server *s) {
    const double t = s->now();
    s->stats.arena_used_byte_s += (double)s->arena.used() * (t - s->arena_since);
    s->arena_since = t;
}

int blocks_for(const lbrd_server *s) { return 8 * s->cus; }

// Multi-step rounds (the serving mix, every request below 4 GiB per buffer):
// seven steps per launch on 32 x 12 tiles, a persistent grid of 8-wave
// workgroups, four per CU.  On the benchmark's request stream (120 requests,
// 16 GB pool), in alternating runs: p50 0.42 s, p99 1.61 s and 238 k
// MLUPS per species while busy, against 0.47 s, 2.0 s and 217 k with five
// steps on 32 x 10, 0.45 s / 1.77 s / 229 k with six on 32 x 12, and worse
// with eight on 32 x 8 or seven on 32 x 16.
constexpr int kServeSteps = 7, kServeRows = 12, kServeCols = 32, kServeWaves = 8, kServeBlocksPerCu = 4;
// Rounds whose resident buffers exceed the 256 MB Infinity Cache run on
// marching wave strips instead: nine steps per launch, segments of 128
// rows, a persistent grid of one workgroup of 4 waves per CU: one wave per
// SIMD, all resident at once (the registers of the Gray-Scott FP32 kernel
// allow one); a second workgroup per CU would wait for the first to finish
// its whole share (on a 4096^2 FP32 lattice: 109 against 93 us per step).
// On the benchmark's 256-instance Gray-Scott sweep with this grid: 122.0 us
// per step, against 135.3 with eight steps and 144.9 with seven on 64 rows.
constexpr int kServeMarchSteps = 9, kServeMarchRows = 128, kServeMarchWaves = 4, kServeMarchBlocksPerCu = 1;

// Round kinds: one step per launch (any mix), multi-step on LDS tiles,
// multi-step on marching strips.
enum RoundKind : int { kRoundOne = 0, kRoundTiles = 1, kRoundMarch = 2 };

int round_steps(int kind) { return kind == kRoundOne ? 1 : kind == kRoundMarch ? kServeMarchSteps : kServeSteps; }

hipError_t enqueue_chunk(lbrd_server *s, int set, int kind, int mask, hipStream_t st) {
    const int64_t launches = launches_for(s->sc.chunk_steps, round_steps(kind));
    if (kind == kRoundMarch) {
        // The classes of a marching round touch disjoint instances: each runs
        // its chain of launches on a branch of its own, forked from st and
        // joined back, so one class's tail overlaps the others' work (their
        // registers let two class kernels share a SIMD).
        hipError_t e = hipEventRecord(s->fork, st);
        for (int cls = 0; cls < kMarchClasses && e == hipSuccess; ++cls) {
            if (!(mask & (1 << cls))) continue;
            e = hipStreamWaitEvent(s->branch[cls], s->fork, 0);
            for (int64_t j = 0; j < launches && e == hipSuccess; ++j)
                e = launch_batch_stepW(s->d_hdr, s->d_inst, (int)j, (int64_t)kServeMarchBlocksPerCu * s->cus,
                                       kServeMarchWaves, kServeMarchSteps, cls, s->branch[cls]);
            if (e == hipSuccess) e = hipEventRecord(s->join[cls], s->branch[cls]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, s->join[cls], 0);
        }
        return e;
    }
    for (int64_t j = 0; j < launches; ++j) {
        hipError_t e = kind == kRoundTiles
                           ? launch_batch_stepT(s->d_hdr, s->d_inst, (int)j, (int64_t)kServeBlocksPerCu * s->cus,
                                                kServeWaves, kServeSteps, kServeRows, kServeCols, set, st)
                           : launch_batch_step(s->d_hdr, s->d_inst, (int)j, blocks_for(s), 4, false, set, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void release_streams(lbrd_server *s) {
    for (int c = 0; c < kMarchClasses; ++c) {
        if (s->branch[c]) hipStreamDestroy(s->branch[c]);
        if (s->join[c]) hipEventDestroy(s->join[c]);
    }
    if (s->fork) hipEventDestroy(s->fork);
    if (s->capture) hipStreamDestroy(s->capture);
    if (s->copy) hipStreamDestroy(s->copy);
    if (s->stream) hipStreamDestroy(s->stream);
}

hipError_t run_chunk(lbrd_server *s, int set, int kind, int mask) {
    hipGraphExec_t &slot = kind == kRoundMarch ? s->march_graph[mask] : s->graph[kind == kRoundTiles ? 3 : set];
    if (!slot) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(s->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t le = enqueue_chunk(s, set, kind, mask, s->capture);
        e = hipStreamEndCapture(s->capture, &g);
        if (le != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return le;
        }
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&slot, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) return e;
    }
    return hipGraphLaunch(slot, s->stream);
}

char *slot_buf(lbrd_server *s, const Request &r, int which) {
    return s->base + r.off + (which ? r.L.buf_bytes : 0);
}
double *slot_rho(lbrd_server *s, const Request &r) {
    return reinterpret_cast<double *>(s->base + r.off + 2 * r.L.buf_bytes);
}
double *slot_result(lbrd_server *s, const Request &r) {
    const size_t sites = (size_t)r.cfg.nx * r.cfg.ny;
    return reinterpret_cast<double *>(s->base + r.off + 2 * r.L.buf_bytes +
                                      align_up(sites * r.cfg.nspecies * sizeof(double), kAlign));
}

const void *params_blob(const Request &r, std::vector<unsigned char> &blob) {
    if (r.cfg.storage == LBRD_F64) {
        Params<double> p = make_params<double>(r.cfg);
        blob.assign(reinterpret_cast<unsigned char *>(&p), reinterpret_cast<unsigned char *>(&p) + sizeof(p));
    } else {
        Params<float> p = make_params<float>(r.cfg);
        blob.assign(reinterpret_cast<unsigned char *>(&p), reinterpret_cast<unsigned char *>(&p) + sizeof(p));
    }
    return blob.data();
}

void worker_loop(lbrd_server *s) {
    std::vector<int64_t> pending_retire;   // finished in the previous round
    hipEvent_t ev_prev = nullptr, ev_cur = nullptr, ev_in = nullptr;
    hipEventCreateWithFlags(&ev_prev, hipEventDisableTiming);
    hipEventCreateWithFlags(&ev_cur, hipEventDisableTiming);
    hipEventCreateWithFlags(&ev_in, hipEventDisableTiming);
    std::vector<BatchInst> inst;
    std::vector<unsigned char> blob;
    hipError_t err = hipSuccess;

    auto retire = [&](std::vector<int64_t> &ids) {
        if (ids.empty()) return;
        // read-back on the copy stream: waits for the previous round only, so
        // the round just enqueued keeps the GPU busy meanwhile
        if (err == hipSuccess) err = hipStreamWaitEvent(s->copy, ev_prev, 0);
        for (int64_t id : ids) {
            Request *r;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                r = &s->reqs.at(id);
            }
            const size_t n = (size_t)r->cfg.nspecies * r->cfg.nx * r->cfg.ny;
            r->rho.resize(n);
            r->mass.resize(kRedSlots);
            if (err == hipSuccess)
                err = hipMemcpyAsync(r->rho.data(), slot_rho(s, *r), n * sizeof(double), hipMemcpyDeviceToHost, s->copy);
            if (err == hipSuccess)
                err = hipMemcpyAsync(r->mass.data(), slot_result(s, *r), kRedSlots * sizeof(double),
                                     hipMemcpyDeviceToHost, s->copy);
        }
        if (err == hipSuccess) err = hipStreamSynchronize(s->copy);
        std::lock_guard<std::mutex> lk(s->mu);
        for (int64_t id : ids) {
            Request *r = &s->reqs.at(id);
            r->mass.resize(r->cfg.nspecies);
            std::vector<double>().swap(r->rho0);
            account_arena(s);
            s->arena.release(r->off, r->footprint);
            r->done_s = s->now();
            r->state = err == hipSuccess ? 2 : 3;
            r->status = err == hipSuccess ? LBRD_OK : LBRD_EDEVICE;
            for (double m : r->mass)
                if (!std::isfinite(m) && r->status == LBRD_OK) r->status = LBRD_ENONFINITE;
            s->stats.completed += 1;
            s->stats.species_site_steps += (int64_t)r->cfg.nspecies * r->cfg.nx * r->cfg.ny * r->steps;
        }
        ids.clear();
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    };

    for (;;) {
        std::vector<Request *> admitted;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                return s->stop || !s->resident.empty() || !pending_retire.empty() || !s->queue.empty();
            });
            if (s->stop && s->resident.empty() && pending_retire.empty()) break;
            // admission by footprint, FIFO with skipping
            if (!s->stop) {
                for (auto it = s->queue.begin(); it != s->queue.end();) {
                    if ((int)s->resident.size() >= s->sc.max_slots) break;
                    Request &r = s->reqs.at(*it);
                    size_t off = 0;
                    account_arena(s);
                    if (s->arena.alloc(r.footprint, &off)) {
                        r.off = off;
                        r.state = 1;
                        r.admit_s = s->now();
                        r.cur = 0;
                        s->resident.push_back(r.id);
                        admitted.push_back(&r);
                        s->stats.admitted += 1;
                        it = s->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            s->stats.arena_peak_used = (int64_t)s->arena.peak();
            mark_busy(s);
        }
        // initial states of the admitted requests: host -> device on the copy
        // stream (not queued behind the running round), then the init kernel
        // on the compute stream after that copy
        for (Request *r : admitted) {
            if (err == hipSuccess)
                err = hipMemcpyAsync(slot_rho(s, *r), r->rho0.data(), r->rho0.size() * sizeof(double),
                                     hipMemcpyHostToDevice, s->copy);
            if (err == hipSuccess) err = hipEventRecord(ev_in, s->copy);
            if (err == hipSuccess) err = hipStreamWaitEvent(s->stream, ev_in, 0);
            if (err == hipSuccess)
                err = launch_init(r->cfg.storage, r->L, params_blob(*r, blob), slot_rho(s, *r), LBRD_DTYPE_F64,
                                  slot_buf(s, *r, 0), s->stream);
        }
        // one round for all resident requests
        std::vector<int64_t> finishing;
        std::vector<int64_t> res;
        std::vector<Request *> resp;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            res = s->resident;
            for (int64_t id : res) resp.push_back(&s->reqs.at(id));
        }
        if (!res.empty() && err == hipSuccess) {
            inst.clear();
            int64_t tiles = 0;
            bool serve = true;
            for (Request *rp : resp) {
                const int v = variant_of(rp->cfg);
                if (rp->cfg.storage == LBRD_F64 || !(v == kGS || v == kLin1)) serve = false;
                if (!batch_multi_ok(rp->L, rp->cfg.storage)) serve = false;
            }
            // the round's launch kind from the resident mix: marching strips
            // once the resident buffers exceed the Infinity Cache, LDS tiles
            // inside it, one step per launch for mixes outside the serving set
            size_t bytes = 0;
            for (Request *rp : resp) bytes += 2 * rp->L.buf_bytes;
            const int kind = !serve ? kRoundOne : bytes > ((size_t)256 << 20) ? kRoundMarch : kRoundTiles;
            int mask = 0;
            if (kind == kRoundMarch)
                for (Request *rp : resp) mask |= 1 << march_class(rp->cfg.storage, variant_of(rp->cfg));
            const int ts = round_steps(kind);
            for (Request *rp : resp) {
                Request &r = *rp;
                const int vec = batch_vec(r.cfg.storage);
                BatchInst bi;
                fill_batch_inst(bi, r.cfg, r.L, slot_buf(s, r, 0), slot_buf(s, r, 1), vec, default_lanes(r.cfg.nx, vec));
                if (kind == kRoundMarch) set_batch_tiling_march(bi, r.L, ts, kServeMarchRows);
                else set_batch_tiling(bi, r.L, ts, kServeRows, kServeCols);
                bi.tile_begin = tiles;
                bi.cur = r.cur;
                bi.steps = (int)std::min<int64_t>(r.left, s->sc.chunk_steps);
                tiles += bi.ntiles;
                inst.push_back(bi);
            }
            BatchHeader h;
            std::memset(&h, 0, sizeof(h));
            h.count = (int)inst.size();
            h.total_tiles = tiles;
            h.nt_store = 0;
            err = hipMemcpyAsync(s->d_inst, inst.data(), sizeof(BatchInst) * inst.size(), hipMemcpyHostToDevice,
                                 s->stream);
            if (err == hipSuccess) err = hipMemcpyAsync(s->d_hdr, &h, sizeof(h), hipMemcpyHostToDevice, s->stream);
            if (err == hipSuccess) err = run_chunk(s, serve ? kBatchServe : kBatchAny, kind, mask);
            for (size_t q = 0; q < res.size() && err == hipSuccess; ++q) {
                Request &r = *resp[q];
                const int taken = inst[q].steps;
                r.left -= taken;
                r.cur ^= (int)(launches_for(taken, ts) & 1);
                if (r.left == 0) {
                    err = launch_moments(r.cfg.storage, r.L, params_blob(r, blob), slot_buf(s, r, r.cur),
                                         slot_rho(s, r), LBRD_DTYPE_F64, nullptr, 0, s->partials, slot_result(s, r),
                                         s->stream);
                    finishing.push_back(r.id);
                }
            }
        }
        if (err == hipSuccess) err = hipEventRecord(ev_cur, s->stream);
        // retire the previous round while this one runs
        retire(pending_retire);
        std::swap(ev_prev, ev_cur);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (int64_t id : finishing)
                s->resident.erase(std::find(s->resident.begin(), s->resident.end(), id));
            mark_busy(s);
        }
        pending_retire = finishing;
        if (err != hipSuccess) {
            set_error("server worker", err);
            std::lock_guard<std::mutex> lk(s->mu);
            s->failed = true;
            for (auto &kv : s->reqs)
                if (kv.second.state < 2) {
                    kv.second.state = 3;
                    kv.second.status = LBRD_EDEVICE;
                }
            s->resident.clear();
            s->queue.clear();
            pending_retire.clear();
            s->cv_done.notify_all();
            break;
        }
    }
    if (!pending_retire.empty()) retire(pending_retire);
    hipEventDestroy(ev_prev);
    hipEventDestroy(ev_cur);
    hipEventDestroy(ev_in);
}

}  // namespace

extern "C" {

int lbrd_server_footprint(const lbrd_config *cfg, size_t *bytes) {
    if (int rc = validate_config(cfg)) return rc;
    if (has_shear(*cfg)) return LBRD_EINVAL;   // single solvers only
    if (!bytes) return LBRD_EINVAL;
    *bytes = request_footprint(normalise(*cfg), nullptr);
    return LBRD_OK;
}

int lbrd_server_create(const lbrd_server_config *sc, void *arena, size_t bytes, void *stream, lbrd_server **out) {
    if (!sc || !out || !arena || ((uintptr_t)arena & 255)) return LBRD_EINVAL;
    if (sc->chunk_steps < 1 || sc->chunk_steps > 100000 || sc->max_slots < 1 || sc->max_slots > 65536 ||
        sc->max_queue < 1)
        return LBRD_EINVAL;
    const size_t inst_off = 256;
    const size_t scratch_off = align_up(inst_off + sizeof(BatchInst) * (size_t)sc->max_slots, kAlign);
    const size_t data_off = scratch_off + scratch_bytes();
    if (bytes < data_off + kAlign) return LBRD_ENOMEM;
    lbrd_server *s = new (std::nothrow) lbrd_server();
    if (!s) return LBRD_ENOMEM;
    s->sc = *sc;
    s->base = static_cast<char *>(arena);
    s->bytes = bytes;
    s->d_hdr = reinterpret_cast<BatchHeader *>(s->base);
    s->d_inst = reinterpret_cast<BatchInst *>(s->base + inst_off);
    s->partials = reinterpret_cast<double *>(s->base + scratch_off);
    s->arena.reset(data_off, bytes / kAlign * kAlign);
    s->cus = device_cu_count();
    s->t0 = std::chrono::steady_clock::now();
    std::memset(&s->stats, 0, sizeof(s->stats));
    s->stats.arena_bytes = (int64_t)(bytes - data_off);
    // the arena may still be in use on the caller's stream: wait once, then
    // run on streams owned by the server
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming);
    for (int c = 0; c < kMarchClasses && e == hipSuccess; ++c) {
        e = hipStreamCreateWithFlags(&s->branch[c], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->join[c], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        set_error("server streams", e);
        release_streams(s);
        delete s;
        return LBRD_EDEVICE;
    }
    int dev = 0;
    hipGetDevice(&dev);
    s->worker = std::thread([s, dev] {
        hipSetDevice(dev);
        worker_loop(s);
    });
    *out = s;
    return LBRD_OK;
}

int lbrd_server_destroy(lbrd_server *s) {
    if (!s) return LBRD_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (int64_t id : s->queue) {
            s->reqs[id].state = 3;
            s->stats.rejected += 1;
        }
        s->queue.clear();
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto &g : s->graph)
        if (g) hipGraphExecDestroy(g);
    for (auto &kv : s->march_graph)
        if (kv.second) hipGraphExecDestroy(kv.second);
    release_streams(s);
    delete s;
    return LBRD_OK;
}

int lbrd_server_submit(lbrd_server *s, const lbrd_config *cfg, const double *rho0_host, int64_t nsteps,
                       int64_t *ticket) {
    if (!s || !rho0_host || !ticket || nsteps < 1) return LBRD_EINVAL;
    if (int rc = validate_config(cfg)) return rc;
    if (has_shear(*cfg)) return LBRD_EINVAL;   // single solvers only
    Request r;
    r.cfg = normalise(*cfg);
    r.footprint = request_footprint(r.cfg, &r.L);
    r.steps = r.left = nsteps;
    const size_t n = (size_t)cfg->nspecies * cfg->nx * cfg->ny;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed) return LBRD_EDEVICE;
    if (s->stop) return LBRD_ESTATE;
    if (r.footprint > (size_t)s->stats.arena_bytes) {
        s->stats.rejected += 1;
        return LBRD_ENOMEM;
    }
    if ((int)s->queue.size() >= s->sc.max_queue) return LBRD_ENOMEM;
    r.rho0.assign(rho0_host, rho0_host + n);
    r.id = s->next_id++;
    r.submit_s = s->now();
    *ticket = r.id;
    s->queue.push_back(r.id);
    s->reqs.emplace(r.id, std::move(r));
    s->stats.submitted += 1;
    s->cv_work.notify_all();
    return LBRD_OK;
}

int lbrd_server_info(lbrd_server *s, int64_t ticket, lbrd_request_info *info) {
    if (!s || !info) return LBRD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return LBRD_ENOTFOUND;
    const Request &r = it->second;
    std::memset(info, 0, sizeof(*info));
    info->state = r.state;
    info->submit_s = r.submit_s;
    info->admit_s = r.admit_s;
    info->done_s = r.done_s;
    info->steps = r.steps;
    info->footprint = (int64_t)r.footprint;
    return LBRD_OK;
}

int lbrd_server_wait(lbrd_server *s, int64_t ticket, double timeout_s) {
    if (!s) return LBRD_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return LBRD_ENOTFOUND;
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(0.0, timeout_s));
    const bool ok = s->cv_done.wait_until(lk, deadline, [&] {
        auto jt = s->reqs.find(ticket);
        return jt == s->reqs.end() || jt->second.state >= 2;
    });
    if (!ok) return LBRD_ETIMEOUT;
    auto jt = s->reqs.find(ticket);
    if (jt == s->reqs.end()) return LBRD_ENOTFOUND;
    return jt->second.state == 2 ? LBRD_OK : (jt->second.status ? jt->second.status : LBRD_EDEVICE);
}

int lbrd_server_take(lbrd_server *s, int64_t ticket, double *rho_out, double *mass_out, lbrd_request_info *info) {
    if (!s) return LBRD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return LBRD_ENOTFOUND;
    Request &r = it->second;
    if (r.state < 2) return LBRD_ESTATE;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->state = r.state;
        info->submit_s = r.submit_s;
        info->admit_s = r.admit_s;
        info->done_s = r.done_s;
        info->steps = r.steps;
        info->footprint = (int64_t)r.footprint;
    }
    const int status = r.state == 2 ? r.status : (r.status ? r.status : LBRD_EDEVICE);
    if (r.state == 2) {
        if (rho_out) std::memcpy(rho_out, r.rho.data(), r.rho.size() * sizeof(double));
        if (mass_out) std::memcpy(mass_out, r.mass.data(), r.mass.size() * sizeof(double));
    }
    s->reqs.erase(it);
    return status;
}

int lbrd_server_stats_get(lbrd_server *s, lbrd_server_stats *out) {
    if (!s || !out) return LBRD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->resident = (int64_t)s->resident.size();
    out->queued = (int64_t)s->queue.size();
    out->arena_peak_used = (int64_t)s->arena.peak();
    account_arena(s);
    out->arena_used = (int64_t)s->arena.used();
    out->arena_used_byte_s = s->stats.arena_used_byte_s;
    out->clock_s = s->now();
    if (s->busy_since >= 0) out->busy_s += out->clock_s - s->busy_since;
    return LBRD_OK;
}

}  // extern "C"
