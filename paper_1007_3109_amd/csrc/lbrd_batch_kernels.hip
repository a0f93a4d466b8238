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
