// Internal declarations shared by the lbrd host library and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "lbrd.h"

namespace lbrd {

// Velocity numbering of the public ABI: rest, the four axis directions, the
// four diagonals (the D2Q9 set of Section II.A, Eq. "Weights").
constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Storage traits indices (match LBRD_F64 .. LBRD_BF16_SHIFTED).
enum Storage : int { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

inline int storage_bytes(int st) { return st == kF64 ? 8 : st == kF32 ? 4 : 2; }

// Reaction variants compiled into the step kernel.  NONE runs as LINEAR
// with K = 0, c = 0, which adds exactly +0 to every population.  The
// advective variants carry a uniform equilibrium velocity, the shear
// variants a velocity that varies with the row (one species linear, or
// Gray-Scott; FP64 and FP32 storage).
enum Variant : int {
    kLin1 = 0, kLin2 = 1, kLin3 = 2, kLin4 = 3, kGS = 4, kAdvLin1 = 5, kAdvGS = 6, kShearLin1 = 7, kShearGS = 8,
    kNumVariants = 9
};

inline bool has_shear(const lbrd_config &c) { return c.shear[0] != 0.0; }
inline int variant_of(const lbrd_config &c) {
    const bool adv = c.u[0] != 0.0 || c.u[1] != 0.0;
    if (has_shear(c)) return c.reaction == LBRD_REACT_GRAY_SCOTT ? kShearGS : kShearLin1;
    if (c.reaction == LBRD_REACT_GRAY_SCOTT) return adv ? kAdvGS : kGS;
    return adv ? kAdvLin1 : c.nspecies - 1;
}

// Row-major planes f[s][i] of ny rows x `pitch` elements, `pstride` elements
// apart.  The stored value of plane (s, i) at site y is the post-collision
// population that streams into y + e_i at the next step.
struct Layout {
    int nx = 0, ny = 0, ns = 0, esize = 0;
    int64_t pitch = 0;     // elements per row (64-byte multiple)
    int64_t pstride = 0;   // elements per plane (256-byte multiple + skew)
    size_t buf_bytes = 0;  // one population buffer
};

Layout make_layout(const lbrd_config &c);

// Arithmetic parameters of one lattice, in the compute type C (double for
// F64 storage, float otherwise).  Weighted shifts w_i * rho_ref_s are
// computed on the host in C so host and device agree bit for bit.
template <class C>
struct Params {
    C omega[LBRD_MAX_SPECIES];   // 1 / tau_s
    C keep[LBRD_MAX_SPECIES];    // 1 - 1 / tau_s
    C K[LBRD_MAX_SPECIES * LBRD_MAX_SPECIES];
    C c[LBRD_MAX_SPECIES];
    C F, k, Fk;                  // Fk = F + k
    C rho_ref[LBRD_MAX_SPECIES]; // 16-bit forms: the storage shift density
    C shift[LBRD_MAX_SPECIES][9];   // c_i rho_ref,s
    C ceq[9];                    // equilibrium coefficients c_i (w_i without a velocity)
    int32_t adv;                 // 1: c_i carry an advection velocity
    // shear flow u_x(y) = u0x + amp sin(2 pi m y / ny), u_y = u0y (shear variants)
    C u0x, u0y, amp;
    int32_t shear_m, shear_ny;
};

template <class C>
Params<C> make_params(const lbrd_config &c);

// Geometry of one step launch over one lattice.
struct Grid {
    const void *src;
    void *dst;
    int nx, ny;
    int64_t pitch, pstride;
    int lanes_x;      // lanes per row segment (power of two, <= 64)
    int lx_shift;     // log2(lanes_x)
    int nvec;         // ceil(nx / vec)
    int nseg;         // ceil(nvec / lanes_x)
    int rpw;          // rows per wave = 64 / lanes_x
    int64_t ntiles;   // nseg * ceil(ny / rpw): one tile per wave
    int blocks;       // 0: one tile per wave; else a persistent grid of this many blocks
    int xcd_order;    // 1: consecutive tiles on the same XCD
};

Grid make_grid(const Layout &L, const void *src, void *dst, int vec, int lanes_x);

// Geometry of a launch that advances `steps` time steps (temporal blocking):
// tiles of tw x th sites, one workgroup per tile (or a persistent grid of
// `blocks` workgroups).
struct GridT {
    const void *src;
    void *dst;
    int nx, ny;
    int64_t pitch, pstride;
    int tw, th;
    int ntx, nty;
    int64_t ntiles;
    int blocks;
    int xcd_order;
    int strip;        // tiles in strips of this many tile columns (ntx: row-major order)
    int steps;        // 2 .. kMaxFusedSteps
    uint32_t bytes;   // bytes of one buffer below 4 GiB, else 0 (addressed plane by plane)
    uint32_t plane_bytes;   // bytes of one plane (pstride elements, below 4 GiB)
    int nt_store;     // 1: streaming (non-temporal) stores of the result
    int march;        // 1: marching wave strips (tw = 64 - 2(steps-1) columns, th rows a segment)
};

constexpr int kMaxFusedSteps = 8;
// Marching wave strips of a single solver keep every level in registers and
// no tile in LDS: up to 12 steps a launch in the 32- and 16-bit forms (FP64
// holds 8, its carries take twice the registers).
constexpr int kMaxMarchSteps = 12;
// Marching strips on buffers of 4 GiB or more (a descriptor per plane, each
// plane below 4 GiB): Gray-Scott and one or two linear species, 8 steps a
// launch, or 10 outside FP64.
constexpr bool march_big_ok(int storage, int variant, int steps) {
    return (variant == kGS || variant == kLin1 || variant == kLin2) &&
           (steps == 8 || (steps == 10 && storage != kF64));
}
constexpr int kMaxBatchFusedSteps = 8;
// Batched marching strips (FP32 and 16-bit classes) take up to 12 steps a
// launch, as the single-lattice ones.
constexpr int kMaxBatchMarchSteps = 12;

GridT make_gridT(const Layout &L, const void *src, void *dst, int tw, int th, int steps);
// LDS row stride (elements) of the multi-step region of width ew with 9 N
// planes of `bytes`-byte elements: 9 N ew rounded up so that stride - w is a
// multiple of 256 bytes (64 banks of 4 bytes) for w = ew - 2, the width of
// the first (largest) shrunk middle region.  Consecutive sites of that
// region in row-major order then fall in consecutive banks even where a wave
// wraps to the next row; the later middle phases and phase 1 (width ew) skip
// a few banks at a wrap, the last phase (32 or more lanes to a tile row)
// never wraps inside a half wave.  Measured against padding for ew, ew - 4
// and ew - 6 in alternating runs: 1024^2 FP32 Gray-Scott (T = 5 on 32 x 10)
// 32.9 against 33.6, 33.1 and 33.1 us per launch; 4096^2 FP32 and F16 equal
// or slower with the others.
__host__ __device__ constexpr int stepT_row_stride(int nspecies, int ew, int bytes) {
    const int unit = 256 / bytes;
    const int base = 9 * nspecies * ew;
    const int w = ew - 2;
    return base + ((w - base) % unit + unit) % unit;
}
constexpr size_t kLdsBytes = (size_t)160 * 1024;   // LDS of one CU
// LDS bytes of a launch of `steps` steps on tw x th tiles.
size_t stepT_lds_bytes(int storage, int nspecies, int tw, int th, int steps);
bool stepT_shape_fits(int storage, int nspecies, int tw, int th, int steps, int waves);

// ------------------------------------------------------------ launchers --

struct StepLaunch {
    int storage, variant, vec, waves;
    bool nontemporal;
};

// One time step of one lattice: src -> dst.  launch_step dispatches to the
// per-storage instantiations.
hipError_t launch_step_f64(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st);
hipError_t launch_step_f32(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st);
hipError_t launch_step_f16(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st);
hipError_t launch_step_bf16(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st);
hipError_t launch_step(const StepLaunch &sl, const Grid &g, const void *params, hipStream_t st);
// g.steps time steps src -> dst in one launch.
hipError_t launch_stepT_f64(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st);
hipError_t launch_stepT_f32(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st);
hipError_t launch_stepT_f16(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st);
hipError_t launch_stepT_bf16(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st);
hipError_t launch_stepT(const StepLaunch &sl, const GridT &g, const void *params, hipStream_t st);
bool step_shape_valid(int storage, int vec, int lanes_x, int waves);

hipError_t launch_init(int storage, const Layout &L, const void *params, const void *rho0, int dtype, void *dst,
                       hipStream_t st);
// Planes [p0, p1) (plane = s * 9 + i) of a dense population array that holds
// just those planes.
hipError_t launch_set_populations(int storage, const Layout &L, const void *params, const void *f, int dtype,
                                  int p0, int p1, void *dst, hipStream_t st);
hipError_t launch_get_populations(int storage, const Layout &L, const void *params, const void *src, void *f_out,
                                  int dtype, hipStream_t st);
// Moments read-out plus FP64 per-block partial sums (mass and, when ref is
// given, the two sums of the relative L2 error).  partials holds
// kRedBlocks * kRedSlots doubles; result receives kRedSlots doubles laid out
// as [sum rho_s | sum (ref - rho)_s^2 | sum ref_s^2], LBRD_MAX_SPECIES each.
constexpr int kRedBlocks = 512;
constexpr int kRedSlots = 3 * LBRD_MAX_SPECIES;
constexpr int kRedThreads = 256;
hipError_t launch_moments(int storage, const Layout &L, const void *params, const void *src, void *rho_out,
                          int dtype, const void *ref, int ref_dtype, double *partials, double *result,
                          hipStream_t st);

// Power spectrum of species s: rho gathered into work (double [ny][nx]), its
// mean removed, row DFT into work (complex [ny][nx]), column DFT and |.|^2 into
// out.  work holds spectrum_work_bytes(nx, ny).
size_t spectrum_work_bytes(int nx, int ny);
// The spectrum variant that allocates nothing takes its scratch from a fixed
// device array of kStaticSpectrumBytes (lattices of at most
// kStaticSpectrumSites sites).  static_spectrum_scratch returns that array's
// address on `device` (looked up once per device with the device current).
constexpr int64_t kStaticSpectrumSites = (int64_t)1 << 20;
constexpr size_t kStaticSpectrumBytes = (size_t)kStaticSpectrumSites * 24 + 256;
hipError_t static_spectrum_scratch(int device, void **ptr);
hipError_t launch_spectrum(int storage, const Layout &L, const void *params, const void *src, int species,
                           double *out, void *work, double *partials, double *result, hipStream_t st);

// ------------------------------------------------------------- batching --

// Device descriptor of one lattice of a batch, read by the persistent step
// kernel with wave-uniform loads.  At step j of a chunk the instance reads
// buf[cur ^ (j & 1)] and writes the other buffer, for j < steps.
struct alignas(16) BatchInst {
    const void *buf[2];
    int64_t pitch, pstride;
    int64_t tile_begin;   // first global tile index of this instance
    int64_t ntiles;
    int32_t nx, ny;
    int32_t lanes_x, lx_shift, nvec, nseg, rpw;
    int32_t storage, variant, vec;
    int32_t cur;          // buffer holding the state at the start of the chunk
    int32_t steps;        // steps this instance takes in the chunk
    int32_t mt_ntx, mt_th;   // multi-step tiling: cols x mt_th tiles, mt_ntx per row
    uint32_t bytes;          // bytes of one buffer (multi-step launches: < 4 GiB)
    int32_t pad;
    union {
        Params<float> pf;
        Params<double> pd;
    };
};

struct alignas(16) BatchHeader {
    int32_t count;        // instances
    int32_t nt_store;     // multi-step launches: 1 = streaming stores of the results
    int64_t total_tiles;  // sum of ntiles
};

// Kernel variant sets of the batched step (fewer compiled variants, fewer
// registers): F32 Gray-Scott only; the serving mix (F32 / F16 / BF16 storage,
// single-species linear or Gray-Scott); everything.
enum BatchSet : int { kBatchGSF32 = 0, kBatchServe = 1, kBatchAny = 2 };

// Step j of a chunk for every instance: one persistent launch of `blocks`
// workgroups of `waves` waves that loop over all tiles.  hdr and inst live in
// device memory, so a captured graph stays valid when their contents change.
hipError_t launch_batch_step(const BatchHeader *hdr, const BatchInst *inst, int j, int blocks, int waves,
                             bool nontemporal, int set, hipStream_t st);
// Launch j of a chunk with `ts` steps per launch (2 .. kMaxBatchFusedSteps) on
// cols x rows tiles (cols 32 or 64): instance i advances min(ts, steps_i - j ts)
// steps if that is positive.  Sets kBatchGSF32 and kBatchServe only; the
// descriptors must carry the same multi-step tiling (set_batch_tiling).
// `blocks` workgroups of `waves` waves walk the tiles.
hipError_t launch_batch_stepT(const BatchHeader *hdr, const BatchInst *inst, int j, int64_t blocks, int waves, int ts,
                              int rows, int cols, int set, hipStream_t st);
// Classes of the batched marching kernel, one kernel each: (FP32, F16,
// BF16) x (Gray-Scott, one-species linear), numbered 2 storage + reaction;
// march_class returns -1 for every other instance.
constexpr int kMarchClasses = 6;
int march_class(int storage, int variant);
// Launch j of a chunk with `ts` steps per launch (2 .. kMaxBatchMarchSteps)
// on marching wave strips (64 - 2(ts-1) result columns by mt_th rows each,
// no LDS) for the instances
// of class `cls`: each advances min(ts, steps_i - j ts) steps if that is
// positive; the others are skipped.  The descriptors must carry the marching
// tiling of the same ts (set_batch_tiling_march).  `blocks` workgroups of
// `waves` (1, 2 or 4) waves walk the strips.
hipError_t launch_batch_stepW(const BatchHeader *hdr, const BatchInst *inst, int j, int64_t blocks, int waves, int ts,
                              int cls, hipStream_t st);
// Fill the tiling fields of a descriptor for marching strips of ts steps and
// `rows` rows per segment.
void set_batch_tiling_march(BatchInst &bi, const Layout &L, int ts, int rows);
// Whether a batched multi-step shape fits (LDS of the largest member of either
// set, Gray-Scott in FP32).
bool batch_shape_fits(int ts, int rows, int cols, int waves);
// Whether an instance can take multi-step launches (32-bit byte offsets).
bool batch_multi_ok(const Layout &L, int storage);
// Number of launches that advance `steps` steps at `ts` steps per launch.
inline int64_t launches_for(int64_t steps, int ts) { return ts > 1 ? (steps + ts - 1) / ts : steps; }
// Fill the tiling fields of a descriptor: one-step tiles (ts = 1) or cols x
// rows multi-step tiles.
void set_batch_tiling(BatchInst &bi, const Layout &L, int ts, int rows, int cols);
int batch_vec(int storage);
void fill_batch_inst(BatchInst &bi, const lbrd_config &c, const Layout &L, const void *buf0, const void *buf1,
                     int vec, int lanes_x);

int device_cu_count();

// n densities in [0.5, 1) from a fixed splitmix64 sequence: a stand-in state
// for timing runs (an all-zero field runs faster than real states).
std::vector<double> scrambled_densities(size_t n);

}  // namespace lbrd
