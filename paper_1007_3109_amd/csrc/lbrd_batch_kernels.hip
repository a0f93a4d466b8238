// Persistent batched step kernel: one launch advances every lattice of a
// batch (of any sizes, parameters and storage forms) by one step.
#include <hip/hip_runtime.h>

#include "lbrd_device.h"

namespace lbrd {

// Vector width used for each storage form inside batches (16-byte vectors
// for F64 / F32; 8-byte vectors for the 16-bit forms keep registers low).
int batch_vec(int storage) { return storage == kF64 ? 2 : 4; }

template <int ST, int V, bool NT>
__device__ __forceinline__ void batch_tile(const BatchInst &bi, int j, int64_t local, int lane) {
    using T = typename Traits<ST>::T;
    constexpr int VEC = ST == kF64 ? 2 : 4;
    const int in = bi.cur ^ (j & 1);
    TileGeom g{bi.nx, bi.ny, bi.pitch, bi.pstride, bi.lx_shift, bi.nvec, bi.nseg, bi.rpw};
    const T *src = static_cast<const T *>(bi.buf[in]);
    T *dst = static_cast<T *>(const_cast<void *>(bi.buf[in ^ 1]));
    if constexpr (ST == kF64) step_tile<ST, V, VEC, NT>(src, dst, g, local, lane, bi.pd);
    else step_tile<ST, V, VEC, NT>(src, dst, g, local, lane, bi.pf);
}

template <int ST, bool NT>
__device__ __forceinline__ void batch_tile_var(const BatchInst &bi, int j, int64_t local, int lane) {
    switch (bi.variant) {
        case kLin1: batch_tile<ST, kLin1, NT>(bi, j, local, lane); break;
        case kLin2: batch_tile<ST, kLin2, NT>(bi, j, local, lane); break;
        case kLin3: batch_tile<ST, kLin3, NT>(bi, j, local, lane); break;
        case kLin4: batch_tile<ST, kLin4, NT>(bi, j, local, lane); break;
        case kAdvLin1: batch_tile<ST, kAdvLin1, NT>(bi, j, local, lane); break;
        case kAdvGS: batch_tile<ST, kAdvGS, NT>(bi, j, local, lane); break;
        default: batch_tile<ST, kGS, NT>(bi, j, local, lane); break;
    }
}

// Serving mix: single-species linear decay or Gray-Scott, in F32 or a
// shifted 16-bit form.
template <int ST, bool NT>
__device__ __forceinline__ void batch_tile_serve(const BatchInst &bi, int j, int64_t local, int lane) {
    if (bi.variant == kGS) batch_tile<ST, kGS, NT>(bi, j, local, lane);
    else batch_tile<ST, kLin1, NT>(bi, j, local, lane);
}

// Persistent step over every tile of every instance.  Each wave walks the
// global tile list with a stride of the whole grid; the instance owning a
// tile is found by binary search over tile_begin (wave-uniform loads).
template <int SET, bool NT>
__global__ __launch_bounds__(256) void k_batch_step(const BatchHeader *__restrict__ hdr,
                                                    const BatchInst *__restrict__ inst, int j) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    const int count = hdr->count;
    const int64_t total = hdr->total_tiles;
    const int64_t stride = (int64_t)gridDim.x * waves;
    int hint = 0;
    for (int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * waves + wave; t < total; t += stride) {
        int lo = inst[hint].tile_begin <= t ? hint : 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (inst[mid].tile_begin <= t) lo = mid;
            else hi = mid - 1;
        }
        hint = lo;
        const BatchInst &bi = inst[lo];
        if (j >= bi.steps) continue;
        const int64_t local = t - bi.tile_begin;
        if constexpr (SET == kBatchGSF32) {
            batch_tile<kF32, kGS, NT>(bi, j, local, lane);
        } else if constexpr (SET == kBatchServe) {
            switch (bi.storage) {
                case kF32: batch_tile_serve<kF32, NT>(bi, j, local, lane); break;
                case kF16: batch_tile_serve<kF16, NT>(bi, j, local, lane); break;
                default: batch_tile_serve<kBF16, NT>(bi, j, local, lane); break;
            }
        } else {
            switch (bi.storage) {
                case kF64: batch_tile_var<kF64, NT>(bi, j, local, lane); break;
                case kF32: batch_tile_var<kF32, NT>(bi, j, local, lane); break;
                case kF16: batch_tile_var<kF16, NT>(bi, j, local, lane); break;
                default: batch_tile_var<kBF16, NT>(bi, j, local, lane); break;
            }
        }
    }
}

// ------------------------------------------- several steps per launch --

template <int ST, int V, int TS, int TW>
__device__ __forceinline__ void batch_tileT(const BatchInst &bi, int j, int64_t local, int m, int nt_store,
                                            unsigned char *smem) {
    using T = typename Traits<ST>::T;
    const int in = bi.cur ^ (j & 1);
    TileT t;
    t.src = buffer_rsrc(bi.buf[in], bi.bytes);
    t.dst = buffer_rsrc(bi.buf[in ^ 1], bi.bytes);
    t.nx = bi.nx;
    t.ny = bi.ny;
    t.th = bi.mt_th;
    t.pitch_b = (uint32_t)bi.pitch * (uint32_t)sizeof(T);
    t.pstride_b = (uint32_t)bi.pstride * (uint32_t)sizeof(T);
    t.nt_store = nt_store;
    const int tx = (int)(local % bi.mt_ntx), ty = (int)(local / bi.mt_ntx);
    if constexpr (ST == kF64)
        stepT_tile<ST, V, TS, TW, true>(t, bi.pd, tx * TW, ty * bi.mt_th, m, reinterpret_cast<T *>(smem));
    else
        stepT_tile<ST, V, TS, TW, true>(t, bi.pf, tx * TW, ty * bi.mt_th, m, reinterpret_cast<T *>(smem));
}

template <int ST, int TS, int TW>
__device__ __forceinline__ void batch_tileT_serve(const BatchInst &bi, int j, int64_t local, int m, int nt_store,
                                                  unsigned char *smem) {
    if (bi.variant == kGS) batch_tileT<ST, kGS, TS, TW>(bi, j, local, m, nt_store, smem);
    else batch_tileT<ST, kLin1, TS, TW>(bi, j, local, m, nt_store, smem);
}

// Launch j of a chunk, TS steps per launch: every workgroup walks the global
// list of TW x rows tiles; the owning instance is found by binary search over
// tile_begin (workgroup-uniform).  Instance i takes m = min(TS, steps_i - j TS)
// steps on its tiles when m > 0; its buffers alternate once per launch.
template <int SET, int TS, int TW>
__global__ __launch_bounds__(1024) void k_batch_stepT(const BatchHeader *__restrict__ hdr,
                                                                        const BatchInst *__restrict__ inst, int j) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int count = hdr->count, nt_store = hdr->nt_store;
    const int64_t total = hdr->total_tiles;
    int hint = 0;
    for (int64_t t = xcd_remap(blockIdx.x, gridDim.x); t < total; t += gridDim.x) {
        int lo = inst[hint].tile_begin <= t ? hint : 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (inst[mid].tile_begin <= t) lo = mid;
            else hi = mid - 1;
        }
        hint = lo;
        const BatchInst &bi = inst[lo];
        const int64_t done = (int64_t)j * TS;
        if (done >= bi.steps) continue;
        const int m = (int)(bi.steps - done < TS ? bi.steps - done : TS);
        const int64_t local = t - bi.tile_begin;
        if constexpr (SET == kBatchGSF32) {
            batch_tileT<kF32, kGS, TS, TW>(bi, j, local, m, nt_store, smem);
        } else {
            switch (bi.storage) {
                case kF32: batch_tileT_serve<kF32, TS, TW>(bi, j, local, m, nt_store, smem); break;
                case kF16: batch_tileT_serve<kF16, TS, TW>(bi, j, local, m, nt_store, smem); break;
                default: batch_tileT_serve<kBF16, TS, TW>(bi, j, local, m, nt_store, smem); break;
            }
        }
    }
}

template <int SET, int TS, int TW>
static hipError_t launch_setT(const BatchHeader *hdr, const BatchInst *inst, int j, int64_t blocks, int waves,
                              size_t lds, hipStream_t st) {
    // per instantiation, once (thread-safe static initialisation): allow more
    // than 64 KB of LDS
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&k_batch_stepT<SET, TS, TW>), hipFuncAttributeMaxDynamicSharedMemorySize,
        160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_batch_stepT<SET, TS, TW>), dim3((unsigned)blocks), dim3(64 * waves), lds, st, hdr, inst,
                       j);
    return hipGetLastError();
}

template <int SET, int TW>
static hipError_t launch_setT_n(const BatchHeader *hdr, const BatchInst *inst, int j, int64_t blocks, int waves,
                                int ts, size_t lds, hipStream_t st) {
    static_assert(kMaxBatchFusedSteps == 8, "instantiate every step count");
    switch (ts) {
        case 2: return launch_setT<SET, 2, TW>(hdr, inst, j, blocks, waves, lds, st);
        case 3: return launch_setT<SET, 3, TW>(hdr, inst, j, blocks, waves, lds, st);
        case 4: return launch_setT<SET, 4, TW>(hdr, inst, j, blocks, waves, lds, st);
        case 5: return launch_setT<SET, 5, TW>(hdr, inst, j, blocks, waves, lds, st);
        case 6: return launch_setT<SET, 6, TW>(hdr, inst, j, blocks, waves, lds, st);
        case 7: return launch_setT<SET, 7, TW>(hdr, inst, j, blocks, waves, lds, st);
        case 8: return launch_setT<SET, 8, TW>(hdr, inst, j, blocks, waves, lds, st);
        default: return hipErrorInvalidValue;
    }
}

template <int SET>
static hipError_t launch_setT_w(const BatchHeader *hdr, const BatchInst *inst, int j, int64_t blocks, int waves,
                                int ts, int cols, size_t lds, hipStream_t st) {
    switch (cols) {
        case 32: return launch_setT_n<SET, 32>(hdr, inst, j, blocks, waves, ts, lds, st);
        case 64: return launch_setT_n<SET, 64>(hdr, inst, j, blocks, waves, ts, lds, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_stepT(const BatchHeader *hdr, const BatchInst *inst, int j, int64_t blocks, int waves, int ts,
                              int rows, int cols, int set, hipStream_t st) {
    // LDS of the largest member of either set: Gray-Scott in FP32
    if (!batch_shape_fits(ts, rows, cols, waves) || blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = stepT_lds_bytes(kF32, 2, cols, rows, ts);
    switch (set) {
        case kBatchGSF32: return launch_setT_w<kBatchGSF32>(hdr, inst, j, blocks, waves, ts, cols, lds, st);
        case kBatchServe: return launch_setT_w<kBatchServe>(hdr, inst, j, blocks, waves, ts, cols, lds, st);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------ marching strips in batches --

template <int ST, int V, int TS>
__device__ __forceinline__ void batch_stripW(const BatchInst &bi, int j, int64_t local, int m, bool nt, int lane) {
    using T = typename Traits<ST>::T;
    constexpr int U = 64 - 2 * (TS - 1);
    const int in = bi.cur ^ (j & 1);
    const int sy = (int)(local / bi.mt_ntx), sx = (int)(local - (int64_t)sy * bi.mt_ntx);
    StripW sw;
    sw.src = buffer_rsrc(bi.buf[in], bi.bytes);
    sw.dst = buffer_rsrc(bi.buf[in ^ 1], bi.bytes);
    sw.nx = bi.nx;
    sw.ny = bi.ny;
    sw.pitch_b = (uint32_t)bi.pitch * (uint32_t)sizeof(T);
    sw.pstride_b = (uint32_t)bi.pstride * (uint32_t)sizeof(T);
    sw.x0 = sx * U;
    sw.y0 = sy * bi.mt_th;
    sw.rows = min(bi.mt_th, bi.ny - sw.y0);
    sw.nt = nt;
    // a launch of all TS steps runs the single-lattice code (its stores at
    // one level only leave the levels in one block for the scheduler); a
    // shorter remainder the code that stores at level m
    const Params<typename Traits<ST>::C> &p = *reinterpret_cast<const Params<typename Traits<ST>::C> *>(
        ST == kF64 ? static_cast<const void *>(&bi.pd) : static_cast<const void *>(&bi.pf));
    if (m == TS) stepW_strip<ST, V, TS>(sw, p, lane);
    else stepW_strip<ST, V, TS, true>(sw, p, lane, m);
}

// Launch j of a chunk on marching strips, TS steps per launch, for the
// instances of one class (storage ST, reaction variant V): each wave walks
// the global list of strip segments of every instance (a persistent grid, so
// that a captured graph serves descriptors that change), finds the owning
// instance by binary search over tile_begin (wave-uniform), skips instances
// of other classes, and advances its own by m = min(TS, steps_i - j TS)
// steps when m > 0; their buffers alternate once per launch.  One kernel per
// class keeps each class at the registers (and waves per SIMD) of its own
// update.  No LDS and no barrier: the waves of a workgroup are independent.
template <int ST, int V, int TS>
__global__ __launch_bounds__(256) void k_batch_stepW(const BatchHeader *__restrict__ hdr,
                                                     const BatchInst *__restrict__ inst, int j) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int waves = blockDim.x >> 6;
    const int count = hdr->count;
    const bool nt = hdr->nt_store != 0;
    const int64_t total = hdr->total_tiles;
    const int64_t stride = (int64_t)gridDim.x * waves;
    int hint = 0;
    for (int64_t t = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * waves + wave; t < total; t += stride) {
        int lo = inst[hint].tile_begin <= t ? hint : 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (inst[mid].tile_begin <= t) lo = mid;
            else hi = mid - 1;
        }
        hint = lo;
        const BatchInst &bi = inst[lo];
        if (bi.storage != ST || bi.variant != V) continue;
        const int64_t done = (int64_t)j * TS;
        if (done >= bi.steps) continue;
        const int m = (int)(bi.steps - done < TS ? bi.steps - done : TS);
        batch_stripW<ST, V, TS>(bi, j, t - bi.tile_begin, m, nt, lane);
    }
}

template <int ST, int V>
static hipError_t launch_classW(const BatchHeader *hdr, const BatchInst *inst, int j, int64_t blocks, int waves,
                                int ts, hipStream_t st) {
    static_assert(kMaxBatchMarchSteps == 12, "instantiate every step count");
    const dim3 grid((unsigned)blocks), block(64 * waves);
    switch (ts) {
        case 2: hipLaunchKernelGGL((k_batch_stepW<ST, V, 2>), grid, block, 0, st, hdr, inst, j); break;
        case 3: hipLaunchKernelGGL((k_batch_stepW<ST, V, 3>), grid, block, 0, st, hdr, inst, j); break;
        case 4: hipLaunchKernelGGL((k_batch_stepW<ST, V, 4>), grid, block, 0, st, hdr, inst, j); break;
        case 5: hipLaunchKernelGGL((k_batch_stepW<ST, V, 5>), grid, block, 0, st, hdr, inst, j); break;
        case 6: hipLaunchKernelGGL((k_batch_stepW<ST, V, 6>), grid, block, 0, st, hdr, inst, j); break;
        case 7: hipLaunchKernelGGL((k_batch_stepW<ST, V, 7>), grid, block, 0, st, hdr, inst, j); break;
        case 8: hipLaunchKernelGGL((k_batch_stepW<ST, V, 8>), grid, block, 0, st, hdr, inst, j); break;
        case 9: hipLaunchKernelGGL((k_batch_stepW<ST, V, 9>), grid, block, 0, st, hdr, inst, j); break;
        case 10: hipLaunchKernelGGL((k_batch_stepW<ST, V, 10>), grid, block, 0, st, hdr, inst, j); break;
        case 11: hipLaunchKernelGGL((k_batch_stepW<ST, V, 11>), grid, block, 0, st, hdr, inst, j); break;
        case 12: hipLaunchKernelGGL((k_batch_stepW<ST, V, 12>), grid, block, 0, st, hdr, inst, j); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int march_class(int storage, int variant) {
    if (variant != kGS && variant != kLin1) return -1;
    const int s = storage == kF32 ? 0 : storage == kF16 ? 1 : storage == kBF16 ? 2 : -1;
    return s < 0 ? -1 : 2 * s + (variant == kGS ? 0 : 1);
}

hipError_t launch_batch_stepW(const BatchHeader *hdr, const BatchInst *inst, int j, int64_t blocks, int waves, int ts,
                              int cls, hipStream_t st) {
    if (ts < 2 || ts > kMaxBatchMarchSteps || !(waves == 1 || waves == 2 || waves == 4) || blocks < 1 ||
        blocks > 0x7fffffff)
        return hipErrorInvalidValue;
    switch (cls) {
        case 0: return launch_classW<kF32, kGS>(hdr, inst, j, blocks, waves, ts, st);
        case 1: return launch_classW<kF32, kLin1>(hdr, inst, j, blocks, waves, ts, st);
        case 2: return launch_classW<kF16, kGS>(hdr, inst, j, blocks, waves, ts, st);
        case 3: return launch_classW<kF16, kLin1>(hdr, inst, j, blocks, waves, ts, st);
        case 4: return launch_classW<kBF16, kGS>(hdr, inst, j, blocks, waves, ts, st);
        case 5: return launch_classW<kBF16, kLin1>(hdr, inst, j, blocks, waves, ts, st);
        default: return hipErrorInvalidValue;
    }
}

void set_batch_tiling_march(BatchInst &bi, const Layout &L, int ts, int rows) {
    const int cols = 64 - 2 * (ts - 1);
    bi.mt_th = rows;
    bi.mt_ntx = (L.nx + cols - 1) / cols;
    bi.ntiles = (int64_t)bi.mt_ntx * ((L.ny + rows - 1) / rows);
    bi.bytes = (uint32_t)L.buf_bytes;
}

bool batch_shape_fits(int ts, int rows, int cols, int waves) {
    return ts >= 2 && ts <= kMaxBatchFusedSteps && (cols == 32 || cols == 64) &&
           stepT_shape_fits(kF32, 2, cols, rows, ts, waves);
}

bool batch_multi_ok(const Layout &L, int storage) {
    // 32-bit byte offsets; row offsets from 24-bit multiplies (row x pitch)
    return L.buf_bytes < ((size_t)1 << 32) && (int64_t)L.pitch * storage_bytes(storage) < ((int64_t)1 << 24) &&
           L.ny <= (1 << 24);
}

void set_batch_tiling(BatchInst &bi, const Layout &L, int ts, int rows, int cols) {
    if (ts > 1) {
        bi.mt_th = rows;
        bi.mt_ntx = (L.nx + cols - 1) / cols;
        bi.ntiles = (int64_t)bi.mt_ntx * ((L.ny + rows - 1) / rows);
        bi.bytes = (uint32_t)L.buf_bytes;
    } else {
        bi.mt_th = 0;
        bi.mt_ntx = 0;
        bi.ntiles = make_grid(L, nullptr, nullptr, bi.vec, bi.lanes_x).ntiles;
        bi.bytes = 0;
    }

}

template <int SET>
static hipError_t launch_set(const BatchHeader *hdr, const BatchInst *inst, int j, int blocks, int waves, bool nt,
                             hipStream_t st) {
    const dim3 grid(blocks), block(64 * waves);
    if (nt) hipLaunchKernelGGL((k_batch_step<SET, true>), grid, block, 0, st, hdr, inst, j);
    else hipLaunchKernelGGL((k_batch_step<SET, false>), grid, block, 0, st, hdr, inst, j);
    return hipGetLastError();
}

hipError_t launch_batch_step(const BatchHeader *hdr, const BatchInst *inst, int j, int blocks, int waves,
                             bool nontemporal, int set, hipStream_t st) {
    switch (set) {
        case kBatchGSF32: return launch_set<kBatchGSF32>(hdr, inst, j, blocks, waves, nontemporal, st);
        case kBatchServe: return launch_set<kBatchServe>(hdr, inst, j, blocks, waves, nontemporal, st);
        default: return launch_set<kBatchAny>(hdr, inst, j, blocks, waves, nontemporal, st);
    }
}

}  // namespace lbrd
