// Initialisation, population transfer and read-out kernels, plus the
// storage dispatch of the step launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "lbrd_device.h"

namespace lbrd {

template <int ST>
constexpr bool vec_ok_for(int vec) {
    return ST == kF64 ? vec == 2 : (ST == kF32 ? (vec == 2 || vec == 4) : (vec == 4 || vec == 8));
}

bool step_shape_valid(int storage, int vec, int lanes_x, int waves) {
    bool v = false;
    switch (storage) {
        case kF64: v = vec_ok_for<kF64>(vec); break;
        case kF32: v = vec_ok_for<kF32>(vec); break;
        case kF16: v = vec_ok_for<kF16>(vec); break;
        case kBF16: v = vec_ok_for<kBF16>(vec); break;
        default: return false;
    }
    const bool pow2 = lanes_x >= 1 && lanes_x <= 64 && (lanes_x & (lanes_x - 1)) == 0;
    return v && pow2 && (waves == 1 || waves == 2 || waves == 4);
}

hipError_t launch_stepT(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st) {
    if (g.ntiles <= 0) return hipSuccess;
    if (g.src == g.dst) return hipErrorInvalidValue;   // the step is never in place (ping-pong buffers)
    // 32-bit byte offsets: the whole buffer or each plane below 4 GiB, a row
    // pitch below 16 MiB (24-bit multiplies)
    if ((int64_t)g.pitch * storage_bytes(sl.storage) >= (1 << 24) || (g.bytes == 0 && g.plane_bytes == 0))
        return hipErrorInvalidValue;
    switch (sl.storage) {
        case kF64: return launch_stepT_f64(sl, g, params, st);
        case kF32: return launch_stepT_f32(sl, g, params, st);
        case kF16: return launch_stepT_f16(sl, g, params, st);
        case kBF16: return launch_stepT_bf16(sl, g, params, st);
        default: return hipErrorInvalidValue;
    }
}

size_t stepT_lds_bytes(int storage, int nspecies, int tw, int th, int steps) {
    const int h = steps - 1;
    const int b = storage_bytes(storage);
    return (size_t)(th + 2 * h) * stepT_row_stride(nspecies, tw + 2 * h, b) * b;
}

bool stepT_shape_fits(int storage, int nspecies, int tw, int th, int steps, int waves) {
    if (steps < 2 || steps > kMaxFusedSteps || (tw != 32 && tw != 64 && tw != 128) || th < 1 || waves < 1 || waves > 16)
        return false;
    return stepT_lds_bytes(storage, nspecies, tw, th, steps) <= kLdsBytes;
}

hipError_t launch_step(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st) {
    if (g.ntiles <= 0) return hipSuccess;
    if (g.src == g.dst) return hipErrorInvalidValue;   // the step is never in place (ping-pong buffers)
    switch (sl.storage) {
        case kF64: return launch_step_f64(sl, g, params, st);
        case kF32: return launch_step_f32(sl, g, params, st);
        case kF16: return launch_step_f16(sl, g, params, st);
        case kBF16: return launch_step_bf16(sl, g, params, st);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------- init / populations --

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

template <class C>
__device__ __forceinline__ C load_in(const void *p, int dtype, int64_t k) {
    return dtype == LBRD_DTYPE_F64 ? (C)static_cast<const double *>(p)[k] : (C)static_cast<const float *>(p)[k];
}

// S_{i,s}(y) = w_i rho0_s(y + e_i): the stored form whose pull gives the
// equilibrium f_{i,s}(x, 0) = w_i rho0_s(x).
template <int ST>
__global__ void k_init(Layout L, Params<typename Traits<ST>::C> p, const void *rho0, int dtype,
                       typename Traits<ST>::T *dst) {
    using C = typename Traits<ST>::C;
    const int64_t sites = (int64_t)L.nx * L.ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < sites; k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / L.nx), x = (int)(k % L.nx);
        for (int s = 0; s < L.ns; ++s) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int xs = wrap(x + kEx[i], L.nx), ys = wrap(y + kEy[i], L.ny);
                const C r = load_in<C>(rho0, dtype, ((int64_t)s * L.ny + ys) * L.nx + xs);
                // rest population as r minus the moving ones, so that the
                // nine equilibrium populations of a site sum to r (see
                // collide_site)
                C v;
                if (p.adv) {
                    // the coefficients of the site the population belongs to
                    // (row ys: it streams into (xs, ys) next)
                    C ceq[9];
                    if (p.shear_ny > 0) {
                        shear_ceq<C>(p, ys, ceq);
                    } else {
                        for (int j = 0; j < 9; ++j) ceq[j] = p.ceq[j];
                    }
                    C moving = C(0);
                    for (int j = 1; j < 9; ++j) moving += ceq[j] * r;
                    v = i == 0 ? r - moving : ceq[i] * r;
                } else {
                    v = i == 0 ? r - C(4) * (wgt<C>(1) * r) - C(4) * (wgt<C>(5) * r) : wgt<C>(i) * r;
                }
                dst[(int64_t)(s * 9 + i) * L.pstride + (int64_t)y * L.pitch + x] = encode<ST>(v, p.shift[s][i]);
            }
        }
    }
}

// Planes [p0, p1) of a dense population array f[s][i][y][x] (f holds only
// those planes, plane p0 first) into the stored pull form.
template <int ST>
__global__ void k_set_pop(Layout L, Params<typename Traits<ST>::C> p, const void *f, int dtype, int p0, int p1,
                          typename Traits<ST>::T *dst) {
    using C = typename Traits<ST>::C;
    const int64_t sites = (int64_t)L.nx * L.ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < sites; k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / L.nx), x = (int)(k % L.nx);
        for (int q = p0; q < p1; ++q) {
            const int s = q / 9, i = q % 9;
            const int xs = wrap(x + kEx[i], L.nx), ys = wrap(y + kEy[i], L.ny);
            const C v = load_in<C>(f, dtype, ((int64_t)(q - p0) * L.ny + ys) * L.nx + xs);
            dst[(int64_t)q * L.pstride + (int64_t)y * L.pitch + x] = encode<ST>(v, p.shift[s][i]);
        }
    }
}

template <int ST>
__global__ void k_get_pop(Layout L, Params<typename Traits<ST>::C> p, const typename Traits<ST>::T *src, void *f,
                          int dtype) {
    using C = typename Traits<ST>::C;
    const int64_t sites = (int64_t)L.nx * L.ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < sites; k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / L.nx), x = (int)(k % L.nx);
        for (int s = 0; s < L.ns; ++s) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int xs = wrap(x - kEx[i], L.nx), ys = wrap(y - kEy[i], L.ny);
                const C v = decode<ST>(src[(int64_t)(s * 9 + i) * L.pstride + (int64_t)ys * L.pitch + xs], p.shift[s][i]);
                const int64_t o = (((int64_t)s * 9 + i) * L.ny + y) * L.nx + x;
                if (dtype == LBRD_DTYPE_F64) static_cast<double *>(f)[o] = (double)v;
                else static_cast<float *>(f)[o] = (float)v;
            }
        }
    }
}

// ------------------------------------------------------------ moments --

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// rho_s(x) = sum_i f_{i,s}(x) gathered from the pull neighbours, optionally
// written out, and three FP64 sums per species accumulated per block:
// sum rho, sum (rho - ref)^2, sum ref^2.
template <int ST>
__global__ __launch_bounds__(kRedThreads) void k_moments(Layout L, Params<typename Traits<ST>::C> p,
                                                         const typename Traits<ST>::T *src, void *rho_out,
                                                         int dtype, const void *ref, int ref_dtype,
                                                         double *partials) {
    using C = typename Traits<ST>::C;
    double acc[kRedSlots];
#pragma unroll
    for (int q = 0; q < kRedSlots; ++q) acc[q] = 0.0;
    const int64_t sites = (int64_t)L.nx * L.ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < sites; k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / L.nx), x = (int)(k % L.nx);
#pragma unroll
        for (int s = 0; s < LBRD_MAX_SPECIES; ++s) {
            if (s >= L.ns) break;
            C rho = C(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int xs = wrap(x - kEx[i], L.nx), ys = wrap(y - kEy[i], L.ny);
                rho += decode<ST>(src[(int64_t)(s * 9 + i) * L.pstride + (int64_t)ys * L.pitch + xs], p.shift[s][i]);
            }
            const int64_t o = (int64_t)s * sites + k;
            if (rho_out) {
                if (dtype == LBRD_DTYPE_F64) static_cast<double *>(rho_out)[o] = (double)rho;
                else static_cast<float *>(rho_out)[o] = (float)rho;
            }
            acc[s] += (double)rho;
            if (ref) {
                const double r = ref_dtype == LBRD_DTYPE_F64 ? static_cast<const double *>(ref)[o]
                                                             : (double)static_cast<const float *>(ref)[o];
                const double d = r - (double)rho;
                acc[LBRD_MAX_SPECIES + s] += d * d;
                acc[2 * LBRD_MAX_SPECIES + s] += r * r;
            }
        }
    }
    __shared__ double red[kRedThreads / 64][kRedSlots];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < kRedSlots; ++q) {
        const double w = wave_sum(acc[q]);
        if (lane == 0) red[wave][q] = w;
    }
    __syncthreads();
    if (threadIdx.x < kRedSlots) {
        double t = 0.0;
        for (int w = 0; w < kRedThreads / 64; ++w) t += red[w][threadIdx.x];
        partials[(int64_t)blockIdx.x * kRedSlots + threadIdx.x] = t;
    }
}

// Second pass: one block sums the per-block partials in a fixed order.
__global__ __launch_bounds__(kRedThreads) void k_finalize(const double *partials, int nblocks, double *result) {
    __shared__ double red[kRedThreads / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = 0; q < kRedSlots; ++q) {
        double t = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kRedThreads) t += partials[(int64_t)b * kRedSlots + q];
        t = wave_sum(t);
        if (lane == 0) red[wave] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double u = 0.0;
            for (int w = 0; w < kRedThreads / 64; ++w) u += red[w];
            result[q] = u;
        }
        __syncthreads();
    }
}

template <int ST>
static hipError_t launch_moments_t(const Layout &L, const void *params, const void *src, void *rho_out, int dtype,
                                   const void *ref, int ref_dtype, double *partials, double *result,
                                   hipStream_t st) {
    using C = typename Traits<ST>::C;
    using T = typename Traits<ST>::T;
    const Params<C> &p = *static_cast<const Params<C> *>(params);
    hipLaunchKernelGGL((k_moments<ST>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, L, p,
                       static_cast<const T *>(src), rho_out, dtype, ref, ref_dtype, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, st, partials, kRedBlocks, result);
    return hipGetLastError();
}

static unsigned elementwise_blocks(const Layout &L) {
    const int64_t sites = (int64_t)L.nx * L.ny;
    int64_t b = (sites + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (unsigned)b;
}

#define LBRD_DISPATCH_ST(storage, CALL)              \
    switch (storage) {                               \
        case kF64: { constexpr int ST = kF64; CALL; } \
        case kF32: { constexpr int ST = kF32; CALL; } \
        case kF16: { constexpr int ST = kF16; CALL; } \
        case kBF16: { constexpr int ST = kBF16; CALL; } \
        default: return hipErrorInvalidValue;        \
    }

hipError_t launch_init(int storage, const Layout &L, const void *params, const void *rho0, int dtype, void *dst,
                       hipStream_t st) {
    LBRD_DISPATCH_ST(storage, {
        using C = typename Traits<ST>::C;
        using T = typename Traits<ST>::T;
        hipLaunchKernelGGL((k_init<ST>), dim3(elementwise_blocks(L)), dim3(256), 0, st, L,
                           *static_cast<const Params<C> *>(params), rho0, dtype, static_cast<T *>(dst));
        return hipGetLastError();
    })
}

hipError_t launch_set_populations(int storage, const Layout &L, const void *params, const void *f, int dtype,
                                  int p0, int p1, void *dst, hipStream_t st) {
    LBRD_DISPATCH_ST(storage, {
        using C = typename Traits<ST>::C;
        using T = typename Traits<ST>::T;
        hipLaunchKernelGGL((k_set_pop<ST>), dim3(elementwise_blocks(L)), dim3(256), 0, st, L,
                           *static_cast<const Params<C> *>(params), f, dtype, p0, p1, static_cast<T *>(dst));
        return hipGetLastError();
    })
}

hipError_t launch_get_populations(int storage, const Layout &L, const void *params, const void *src, void *f_out,
                                  int dtype, hipStream_t st) {
    LBRD_DISPATCH_ST(storage, {
        using C = typename Traits<ST>::C;
        using T = typename Traits<ST>::T;
        hipLaunchKernelGGL((k_get_pop<ST>), dim3(elementwise_blocks(L)), dim3(256), 0, st, L,
                           *static_cast<const Params<C> *>(params), static_cast<const T *>(src), f_out, dtype);
        return hipGetLastError();
    })
}

hipError_t launch_moments(int storage, const Layout &L, const void *params, const void *src, void *rho_out,
                          int dtype, const void *ref, int ref_dtype, double *partials, double *result,
                          hipStream_t st) {
    LBRD_DISPATCH_ST(storage, {
        return launch_moments_t<ST>(L, params, src, rho_out, dtype, ref, ref_dtype, partials, result, st);
    })
}

// ------------------------------------------------------------ spectrum --

// rho_s gathered as double [ny][nx] (contiguous).
template <int ST>
__global__ void k_gather_rho(Layout L, Params<typename Traits<ST>::C> p, const typename Traits<ST>::T *src, int s,
                             double *rho) {
    using C = typename Traits<ST>::C;
    const int64_t sites = (int64_t)L.nx * L.ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < sites; k += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(k / L.nx), x = (int)(k % L.nx);
        C r = C(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int xs = wrap(x - kEx[i], L.nx), ys = wrap(y - kEy[i], L.ny);
            r += decode<ST>(src[(int64_t)(s * 9 + i) * L.pstride + (int64_t)ys * L.pitch + xs], p.shift[s][i]);
        }
        rho[k] = (double)r;
    }
}

// Row transform: R[y][kx] = sum_x (rho[y][x] - mean) e^{-2 pi i kx x / nx}.
// One thread per (y, kx); the phase index kx*x is reduced modulo nx exactly.
__global__ void k_dft_rows(const double *rho, const double *mean, int nx, int ny, double2 *R) {
    const int64_t n = (int64_t)nx * ny;
    const double m = mean[0] / (double)n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(q / nx), kx = (int)(q % nx);
        double re = 0.0, im = 0.0;
        int64_t ph = 0;
        for (int x = 0; x < nx; ++x) {
            double sn, cs;
            sincospi(2.0 * (double)ph / (double)nx, &sn, &cs);
            const double g = rho[(int64_t)y * nx + x] - m;
            re += g * cs;
            im -= g * sn;
            ph += kx;
            if (ph >= nx) ph -= nx;
        }
        R[q] = make_double2(re, im);
    }
}

// Column transform and power: P[ky][kx] = |sum_y R[y][kx] e^{-2 pi i ky y / ny}|^2.
__global__ void k_dft_cols(const double2 *R, int nx, int ny, double *P) {
    const int64_t n = (int64_t)nx * ny;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int ky = (int)(q / nx), kx = (int)(q % nx);
        double re = 0.0, im = 0.0;
        int64_t ph = 0;
        for (int y = 0; y < ny; ++y) {
            double sn, cs;
            sincospi(2.0 * (double)ph / (double)ny, &sn, &cs);
            const double2 r = R[(int64_t)y * nx + kx];
            re += r.x * cs + r.y * sn;
            im += r.y * cs - r.x * sn;
            ph += ky;
            if (ph >= ny) ph -= ny;
        }
        P[q] = re * re + im * im;
    }
}

// ----------------------------------------------- FFT of rows and columns --
//
// A line of n complex values (a row of rho minus its mean, or a column of the
// row transform) is transformed by one workgroup in LDS with the Stockham
// autosort formulation: stage s of radix R (the radices, 4, 2, 3 and 5 as
// they divide n, in that order) takes the n/R butterflies j of span Ns (the
// product of the earlier radices), multiplies input r = 0..R-1, read at
// j + r n/R, by e^{-2 pi i (j mod Ns) r / (Ns R)}, takes their R-point DFT
// and writes output r at (j div Ns) Ns R + (j mod Ns) + r Ns of the other
// half of LDS.  Every twiddle's phase is an exact integer fraction.  Lines
// longer than kFftMax or with a prime factor above 5 take the direct sums
// above.

constexpr int kFftMax = 5120;     // 2 x 5120 complex doubles: 160 KB of LDS
constexpr int kFftMaxStages = 32;

struct FftPlan {
    int n, count;
    int r[kFftMaxStages];
};

// The plan of an n-point transform, or count = -1 when it takes the direct sums.
FftPlan fft_plan(int n) {
    FftPlan pl;
    pl.n = n;
    pl.count = 0;
    int m = n;
    for (int r : {4, 2, 3, 5})
        while (m % r == 0 && pl.count < kFftMaxStages) {
            pl.r[pl.count++] = r;
            m /= r;
        }
    if (m != 1 || n > kFftMax) pl.count = -1;
    return pl;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// e^{-2 pi i p / q}, 0 <= p < q
__device__ __forceinline__ double2 cis_neg(int p, int q) {
    double sn, cs;
    sincospi(2.0 * (double)p / (double)q, &sn, &cs);
    return make_double2(cs, -sn);
}

// Transforms the line in a (n values) using b as the other half; returns
// the half that holds the result.  Called by the whole workgroup.
__device__ double2 *fft_line(double2 *a, double2 *b, const FftPlan &pl) {
    const int n = pl.n;
    int ns = 1;
    for (int s = 0; s < pl.count; ++s) {
        const int R = pl.r[s], nr = n / R;
        for (int j = threadIdx.x; j < nr; j += blockDim.x) {
            const int k = j % ns;
            double2 v[5], w[5];
#pragma unroll
            for (int r = 0; r < 5; ++r)
                if (r < R) v[r] = r ? cmul(a[j + r * nr], cis_neg(k * r, ns * R)) : a[j];
#pragma unroll
            for (int kk = 0; kk < 5; ++kk) {
                if (kk >= R) continue;
                double2 acc = v[0];
#pragma unroll
                for (int q = 1; q < 5; ++q)
                    if (q < R) {
                        const double2 t = cmul(v[q], cis_neg((kk * q) % R, R));
                        acc.x += t.x;
                        acc.y += t.y;
                    }
                w[kk] = acc;
            }
            const int d = (j / ns) * ns * R + k;
#pragma unroll
            for (int r = 0; r < 5; ++r)
                if (r < R) b[d + r * ns] = w[r];
        }
        __syncthreads();
        double2 *t = a;
        a = b;
        b = t;
        ns *= R;
    }
    return a;
}

// Row transform by FFT: R[y][kx] as k_dft_rows computes it.
__global__ __launch_bounds__(256) void k_fft_rows(const double *rho, const double *mean, int nx, int ny, double2 *R,
                                                  FftPlan pl) {
    extern __shared__ double2 line[];
    const double m = mean[0] / ((double)nx * ny);
    for (int y = blockIdx.x; y < ny; y += gridDim.x) {
        for (int x = threadIdx.x; x < nx; x += blockDim.x) line[x] = make_double2(rho[(int64_t)y * nx + x] - m, 0.0);
        __syncthreads();
        const double2 *res = fft_line(line, line + nx, pl);
        for (int x = threadIdx.x; x < nx; x += blockDim.x) R[(int64_t)y * nx + x] = res[x];
        __syncthreads();
    }
}

// Column transform and power by FFT: P[ky][kx] as k_dft_cols computes it.
__global__ __launch_bounds__(256) void k_fft_cols(const double2 *R, int nx, int ny, double *P, FftPlan pl) {
    extern __shared__ double2 line[];
    for (int kx = blockIdx.x; kx < nx; kx += gridDim.x) {
        for (int y = threadIdx.x; y < ny; y += blockDim.x) line[y] = R[(int64_t)y * nx + kx];
        __syncthreads();
        const double2 *res = fft_line(line, line + ny, pl);
        for (int y = threadIdx.x; y < ny; y += blockDim.x) P[(int64_t)y * nx + kx] = res[y].x * res[y].x + res[y].y * res[y].y;
        __syncthreads();
    }
}

// Sum of a double array with the deterministic two-pass reduction (slot 0).
__global__ __launch_bounds__(kRedThreads) void k_sum(const double *a, int64_t n, double *partials) {
    double acc = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        acc += a[k];
    __shared__ double red[kRedThreads / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    acc = wave_sum(acc);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x < kRedSlots) {
        double t = 0.0;
        if (threadIdx.x == 0)
            for (int w = 0; w < kRedThreads / 64; ++w) t += red[w];
        partials[(int64_t)blockIdx.x * kRedSlots + threadIdx.x] = t;
    }
}

size_t spectrum_work_bytes(int nx, int ny) {
    const size_t n = (size_t)nx * ny;
    return n * sizeof(double) + n * sizeof(double2) + 256;
}

hipError_t launch_spectrum(int storage, const Layout &L, const void *params, const void *src, int species,
                           double *out, void *work, double *partials, double *result, hipStream_t st) {
    const int64_t n = (int64_t)L.nx * L.ny;
    double *rho = static_cast<double *>(work);
    double2 *R = reinterpret_cast<double2 *>(static_cast<char *>(work) + (((size_t)n * sizeof(double) + 255) / 256) * 256);
    hipError_t e = hipSuccess;
    // rows, then columns: by FFT where the line fits in LDS and factors into
    // 2, 3 and 5, else by the direct sums
    static const hipError_t attr_r = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_rows),
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    static const hipError_t attr_c = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_cols),
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr_r != hipSuccess) return attr_r;
    if (attr_c != hipSuccess) return attr_c;
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    const FftPlan prow = fft_plan(L.nx);
    const FftPlan pcol = fft_plan(L.ny);
    LBRD_DISPATCH_ST(storage, {
        using C = typename Traits<ST>::C;
        using T = typename Traits<ST>::T;
        hipLaunchKernelGGL((k_gather_rho<ST>), dim3(elementwise_blocks(L)), dim3(256), 0, st, L,
                           *static_cast<const Params<C> *>(params), static_cast<const T *>(src), species, rho);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_sum, dim3(kRedBlocks), dim3(kRedThreads), 0, st, rho, n, partials);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedThreads), 0, st, partials, kRedBlocks, result);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (prow.count >= 0)
            hipLaunchKernelGGL(k_fft_rows, dim3((unsigned)std::min(L.ny, 65535)), dim3(256), 2 * L.nx * sizeof(double2),
                               st, rho, result, L.nx, L.ny, R, prow);
        else
            hipLaunchKernelGGL(k_dft_rows, dim3(nb), dim3(256), 0, st, rho, result, L.nx, L.ny, R);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (pcol.count >= 0)
            hipLaunchKernelGGL(k_fft_cols, dim3((unsigned)std::min(L.nx, 65535)), dim3(256), 2 * L.ny * sizeof(double2),
                               st, R, L.nx, L.ny, out, pcol);
        else
            hipLaunchKernelGGL(k_dft_cols, dim3(nb), dim3(256), 0, st, R, L.nx, L.ny, out);
        return hipGetLastError();
    })
}

// Scratch of the spectrum variant that allocates nothing (the gathered
// densities and the row transform of up to kStaticSpectrumSites sites, laid
// out as by launch_spectrum): one fixed array in each GPU's memory, held
// until the process ends.  Host code must use the address that
// hipGetSymbolAddress returns for the current device, never the array's
// name (on the host that is a stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[kStaticSpectrumBytes];

static_assert(kStaticSpectrumBytes >= kStaticSpectrumSites * (sizeof(double) + sizeof(double2)) + 256,
              "the static spectrum scratch holds spectrum_work_bytes of its largest lattice");

hipError_t static_spectrum_scratch(int device, void **ptr) {
    static std::mutex mu;
    static std::vector<void *> addr;   // per device, looked up once
    if (!ptr || device < 0) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(mu);
    if ((size_t)device < addr.size() && addr[device]) {
        *ptr = addr[device];
        return hipSuccess;
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
        const hipError_t back = hipSetDevice(cur);
        if (e == hipSuccess) e = back;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    if (addr.size() <= (size_t)device) addr.resize((size_t)device + 1, nullptr);
    addr[device] = p;
    *ptr = p;
    return hipSuccess;
}

}  // namespace lbrd
