// Host-side launch templates of the step kernel, instantiated once per
// storage form in its own translation unit (parallel compilation).
#pragma once
#include "lbrd_device.h"

namespace lbrd {

template <int ST, int V, int VEC>
inline hipError_t launch_step_t(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st) {
    using C = typename Traits<ST>::C;
    const Params<C> &p = *static_cast<const Params<C> *>(params);
    int64_t nb64 = (g.ntiles + sl.waves - 1) / sl.waves;
    if (g.blocks > 0 && g.blocks < nb64) nb64 = g.blocks;
    if (nb64 > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb64), block(64 * sl.waves);
    const bool row1 = g.lanes_x == 64;
    if (sl.nontemporal) {
        if (row1) hipLaunchKernelGGL((k_step<ST, V, VEC, true, true>), grid, block, 0, st, g, p);
        else hipLaunchKernelGGL((k_step<ST, V, VEC, true, false>), grid, block, 0, st, g, p);
    } else {
        if (row1) hipLaunchKernelGGL((k_step<ST, V, VEC, false, true>), grid, block, 0, st, g, p);
        else hipLaunchKernelGGL((k_step<ST, V, VEC, false, false>), grid, block, 0, st, g, p);
    }
    return hipGetLastError();
}

template <int ST, int V>
inline hipError_t launch_step_v(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st) {
    if constexpr (ST == kF64) {
        return launch_step_t<ST, V, 2>(sl, g, params, st);
    } else if constexpr (ST == kF32) {
        return sl.vec == 2 ? launch_step_t<ST, V, 2>(sl, g, params, st) : launch_step_t<ST, V, 4>(sl, g, params, st);
    } else {
        return sl.vec == 4 ? launch_step_t<ST, V, 4>(sl, g, params, st) : launch_step_t<ST, V, 8>(sl, g, params, st);
    }
}

template <int ST>
inline hipError_t launch_step_s(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st) {
    switch (sl.variant) {
        case kLin1: return launch_step_v<ST, kLin1>(sl, g, params, st);
        case kLin2: return launch_step_v<ST, kLin2>(sl, g, params, st);
        case kLin3: return launch_step_v<ST, kLin3>(sl, g, params, st);
        case kLin4: return launch_step_v<ST, kLin4>(sl, g, params, st);
        case kGS: return launch_step_v<ST, kGS>(sl, g, params, st);
        case kAdvLin1: return launch_step_v<ST, kAdvLin1>(sl, g, params, st);
        case kAdvGS: return launch_step_v<ST, kAdvGS>(sl, g, params, st);
        case kShearLin1:
            if constexpr (ST == kF64 || ST == kF32) return launch_step_v<ST, kShearLin1>(sl, g, params, st);
            return hipErrorInvalidValue;
        case kShearGS:
            if constexpr (ST == kF64 || ST == kF32) return launch_step_v<ST, kShearGS>(sl, g, params, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <int ST, int V, int TS, int TW, bool BIG>
inline hipError_t launch_stepT_t(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st) {
    using C = typename Traits<ST>::C;
    const Params<C> &p = *static_cast<const Params<C> *>(params);
    const size_t lds = stepT_lds_bytes(ST, NSpecies<V>::value, TW, g.th, TS);
    // per instantiation, once (thread-safe static initialisation): allow more
    // than 64 KB of LDS
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&k_stepT<ST, V, TS, TW, BIG>), hipFuncAttributeMaxDynamicSharedMemorySize,
        160 * 1024);
    if (attr != hipSuccess) return attr;
    int64_t nb = g.ntiles;
    if (g.blocks > 0 && g.blocks < nb) nb = g.blocks;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_stepT<ST, V, TS, TW, BIG>), dim3((unsigned)nb), dim3(64 * sl.waves), lds, st, g, p);
    return hipGetLastError();
}

template <int ST, int V, int TW, bool BIG>
inline hipError_t launch_stepT_n(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st) {
    static_assert(kMaxFusedSteps == 8, "instantiate every step count");
    switch (g.steps) {
        case 2: return launch_stepT_t<ST, V, 2, TW, BIG>(sl, g, params, st);
        case 3: return launch_stepT_t<ST, V, 3, TW, BIG>(sl, g, params, st);
        case 4: return launch_stepT_t<ST, V, 4, TW, BIG>(sl, g, params, st);
        case 5: return launch_stepT_t<ST, V, 5, TW, BIG>(sl, g, params, st);
        case 6: return launch_stepT_t<ST, V, 6, TW, BIG>(sl, g, params, st);
        case 7: return launch_stepT_t<ST, V, 7, TW, BIG>(sl, g, params, st);
        case 8: return launch_stepT_t<ST, V, 8, TW, BIG>(sl, g, params, st);
        default: return hipErrorInvalidValue;
    }
}

template <int ST, int V, int TS>
inline hipError_t launch_stepW_t(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st) {
    using C = typename Traits<ST>::C;
    const Params<C> &p = *static_cast<const Params<C> *>(params);
    if (g.tw != 64 - 2 * (TS - 1) || g.th < 1 || sl.waves < 1 || sl.waves > 4) return hipErrorInvalidValue;
    const int64_t nb = (g.ntiles + sl.waves - 1) / sl.waves;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    if (g.bytes == 0) {
        // a buffer of 4 GiB or more: a descriptor per plane; g.steps <= TS
        if constexpr (march_big_ok(ST, V, TS)) {
            if (g.plane_bytes == 0 || g.steps < 2 || g.steps > TS) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_stepW<ST, V, TS, true>), dim3((unsigned)nb), dim3(64 * sl.waves), 0, st, g, p);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_stepW<ST, V, TS>), dim3((unsigned)nb), dim3(64 * sl.waves), 0, st, g, p);
    return hipGetLastError();
}

template <int ST, int V>
inline hipError_t launch_stepW_n(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st) {
    static_assert(kMaxFusedSteps == 8 && kMaxMarchSteps == 12, "instantiate every step count");
    if (g.bytes == 0) {
        // buffers of 4 GiB or more: the kernel of the strips' step count
        // (g.tw) runs g.steps of them
        switch ((64 - g.tw) / 2 + 1) {
            case 8: return launch_stepW_t<ST, V, 8>(sl, g, params, st);
            case 10:
                if constexpr (ST != kF64) return launch_stepW_t<ST, V, 10>(sl, g, params, st);
                return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
    switch (g.steps) {
        case 2: return launch_stepW_t<ST, V, 2>(sl, g, params, st);
        case 3: return launch_stepW_t<ST, V, 3>(sl, g, params, st);
        case 4: return launch_stepW_t<ST, V, 4>(sl, g, params, st);
        case 5: return launch_stepW_t<ST, V, 5>(sl, g, params, st);
        case 6: return launch_stepW_t<ST, V, 6>(sl, g, params, st);
        case 7: return launch_stepW_t<ST, V, 7>(sl, g, params, st);
        case 8: return launch_stepW_t<ST, V, 8>(sl, g, params, st);
        default: break;
    }
    if constexpr (ST != kF64) {
        switch (g.steps) {
            case 9: return launch_stepW_t<ST, V, 9>(sl, g, params, st);
            case 10: return launch_stepW_t<ST, V, 10>(sl, g, params, st);
            case 11: return launch_stepW_t<ST, V, 11>(sl, g, params, st);
            case 12: return launch_stepW_t<ST, V, 12>(sl, g, params, st);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

template <int ST, int V>
inline hipError_t launch_stepT_w(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st) {
    if (g.march) return launch_stepW_n<ST, V>(sl, g, params, st);
    if (!stepT_shape_fits(ST, NSpecies<V>::value, g.tw, g.th, g.steps, sl.waves)) return hipErrorInvalidValue;
    if (g.bytes == 0) {
        // buffers of 4 GiB or more, planes below it: tiles 32 or 64 wide
        if (g.plane_bytes == 0) return hipErrorInvalidValue;
        switch (g.tw) {
            case 32: return launch_stepT_n<ST, V, 32, true>(sl, g, params, st);
            case 64: return launch_stepT_n<ST, V, 64, true>(sl, g, params, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (g.tw) {
        case 32: return launch_stepT_n<ST, V, 32, false>(sl, g, params, st);
        case 64: return launch_stepT_n<ST, V, 64, false>(sl, g, params, st);
        case 128: return launch_stepT_n<ST, V, 128, false>(sl, g, params, st);
        default: return hipErrorInvalidValue;
    }
}

// The multi-step kernel uses cached accesses whatever sl.nontemporal says.
template <int ST>
inline hipError_t launch_stepT_s(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st) {
    switch (sl.variant) {
        case kLin1: return launch_stepT_w<ST, kLin1>(sl, g, params, st);
        case kLin2: return launch_stepT_w<ST, kLin2>(sl, g, params, st);
        case kLin3: return launch_stepT_w<ST, kLin3>(sl, g, params, st);
        case kLin4: return launch_stepT_w<ST, kLin4>(sl, g, params, st);
        case kGS: return launch_stepT_w<ST, kGS>(sl, g, params, st);
        case kAdvLin1: return launch_stepT_w<ST, kAdvLin1>(sl, g, params, st);
        case kAdvGS: return launch_stepT_w<ST, kAdvGS>(sl, g, params, st);
        case kShearLin1:
            if constexpr (ST == kF64 || ST == kF32) return launch_stepT_w<ST, kShearLin1>(sl, g, params, st);
            return hipErrorInvalidValue;
        case kShearGS:
            if constexpr (ST == kF64 || ST == kF32) return launch_stepT_w<ST, kShearGS>(sl, g, params, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lbrd
