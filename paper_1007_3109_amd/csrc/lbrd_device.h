// Device code of the fused collide-react-stream step (included by the
// per-storage kernel translation units and the batched kernel).
//
// The step is the update of Section II.A (second Eq. "relax"; Appendix Eq.
// "app1") in "pull" form.  The buffer holds, per plane (s, i) and site y, the
// post-collision value S_{i,s}(y) that streams to y + e_i; so the state at t
// is f_{i,s}(x, t) = S_{i,s}(x - e_i).  One step reads, for every site x,
//   f_{i,s}(x) = S_{i,s}(x - e_i)            (streaming, periodic wrap)
//   rho_s = sum_i f_{i,s}                    (ascending i)
//   R_s = R_s(rho_1..rho_N)
//   S'_{i,s}(x) = f_{i,s} (1 - 1/tau_s) + w_i (rho_s / tau_s + R_s)
// and stores S' at x.  Every population is read once and written once: the
// path is bound by HBM bandwidth (about 0.55 flop per byte in FP32), so no
// matrix cores are involved.
//
// Mapping: a wave owns a tile of `rpw` rows x (64 / rpw) lanes; each lane
// owns `VEC` consecutive sites of one row and moves 16 (or 8) bytes per plane
// with one vector load and one vector store.  The +-1 shift in x of six of
// the nine planes is realised in registers: the element that crosses a lane
// boundary comes from the neighbouring lane by a cross-lane shuffle, and only
// lanes at a row-segment edge (or at the periodic wrap) load that one element
// from memory.  Loads stay 16-byte aligned and no LDS staging is needed,
// because no population is used by two sites.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbrd_internal.h"

namespace lbrd {

// ------------------------------------------------------------ storage --

template <int ST>
struct Traits;
template <>
struct Traits<kF64> {
    using T = double;
    using C = double;
};
template <>
struct Traits<kF32> {
    using T = float;
    using C = float;
};
template <>
struct Traits<kF16> {
    using T = uint16_t;
    using C = float;
};
template <>
struct Traits<kBF16> {
    using T = uint16_t;
    using C = float;
};

__device__ __forceinline__ float half_bits_to_float(uint16_t h) {
    _Float16 x;
    __builtin_memcpy(&x, &h, 2);
    return (float)x;
}
__device__ __forceinline__ uint16_t float_to_half_bits(float f) {
    _Float16 x = (_Float16)f;   // round to nearest even
    uint16_t h;
    __builtin_memcpy(&h, &x, 2);
    return h;
}
__device__ __forceinline__ float bf16_bits_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t float_to_bf16_bits(float f) {
    __bf16 h = (__bf16)f;   // round to nearest even (hardware conversion on gfx950)
    uint16_t b;
    __builtin_memcpy(&b, &h, 2);
    return b;
}

template <int ST>
__device__ __forceinline__ typename Traits<ST>::C decode(typename Traits<ST>::T v, typename Traits<ST>::C shift) {
    if constexpr (ST == kF16) return half_bits_to_float(v) + shift;
    else if constexpr (ST == kBF16) return bf16_bits_to_float(v) + shift;
    else return v;
}
template <int ST>
__device__ __forceinline__ typename Traits<ST>::T encode(typename Traits<ST>::C f, typename Traits<ST>::C shift) {
    if constexpr (ST == kF16) return float_to_half_bits(f - shift);
    else if constexpr (ST == kBF16) return float_to_bf16_bits(f - shift);
    else return f;
}

template <int ST>
constexpr bool kShifted = ST == kF16 || ST == kBF16;

// acc + h in FP32 (one rounding; h converts exactly), reading the binary16
// operand directly: one mixed-precision multiply-add by 1.0 instead of a
// conversion and an add.  The population sums of the 16-bit form take it.
// The 1.0 comes from a scalar register the compiler cannot see into, so the
// multiply-add is not folded into an add of a converted value; the compiler
// then selects the mixed multiply-add itself and reads either half of a
// packed register in place.
__device__ __forceinline__ float add_half(float acc, _Float16 h) {
    float one;
    asm("s_mov_b32 %0, 1.0" : "=s"(one));
    return __builtin_fmaf((float)h, one, acc);
}

// Stored value <-> deviation d (= f for F64 / F32, f - w_i rho_ref,s for the
// 16-bit forms).
template <int ST>
__device__ __forceinline__ typename Traits<ST>::C decode_dev(typename Traits<ST>::T v) {
    if constexpr (ST == kF16) return half_bits_to_float(v);
    else if constexpr (ST == kBF16) return bf16_bits_to_float(v);
    else return v;
}
template <int ST>
__device__ __forceinline__ typename Traits<ST>::T encode_dev(typename Traits<ST>::C d) {
    if constexpr (ST == kF16) return float_to_half_bits(d);
    else if constexpr (ST == kBF16) return float_to_bf16_bits(d);
    else return d;
}

// Two FP32 values rounded to the 16-bit form by one packed conversion
// (round to nearest even, as two single conversions).
typedef float float2_v __attribute__((ext_vector_type(2)));
typedef _Float16 half2_v __attribute__((ext_vector_type(2)));
typedef __bf16 bf162_v __attribute__((ext_vector_type(2)));
// The halves are taken from the packed word: bit casts of the vector's
// elements compiled to one conversion stored twice with this compiler.
template <int ST>
__device__ __forceinline__ void encode_pair(float a, float b, uint16_t &oa, uint16_t &ob) {
    uint32_t u;
    if constexpr (ST == kF16) u = __builtin_bit_cast(uint32_t, __builtin_convertvector((float2_v){a, b}, half2_v));
    else u = __builtin_bit_cast(uint32_t, __builtin_convertvector((float2_v){a, b}, bf162_v));
    oa = (uint16_t)u;
    ob = (uint16_t)(u >> 16);
}
// The 9 NS results of one site, paired in species-major order; with PM and
// two species, plane by plane (species 0 and 1 of plane i in one packed
// word, which the marching kernel moves and keeps as one register).  The
// rounding of each value is the same either way.
template <int ST, int NS, bool PM = false>
__device__ __forceinline__ void encode_sites(const float (&r)[NS][9], uint16_t (&o)[NS][9]) {
    if constexpr (PM && NS == 2) {
#pragma unroll
        for (int i = 0; i < 9; ++i) encode_pair<ST>(r[0][i], r[1][i], o[0][i], o[1][i]);
    } else {
#pragma unroll
        for (int k = 0; k + 1 < 9 * NS; k += 2)
            encode_pair<ST>(r[k / 9][k % 9], r[(k + 1) / 9][(k + 1) % 9], o[k / 9][k % 9],
                            o[(k + 1) / 9][(k + 1) % 9]);
        if constexpr ((9 * NS) % 2) o[NS - 1][8] = encode_dev<ST>(r[NS - 1][8]);
    }
}

// D2Q9 weights w_i (Eq. "Weights") in the compute type.
template <class C>
__device__ __forceinline__ constexpr C wgt(int i) {
    return i == 0 ? C(4) / C(9) : (i < 5 ? C(1) / C(9) : C(1) / C(36));
}

template <int BYTES>
struct RawOf;
template <>
struct RawOf<16> {
    typedef uint32_t type __attribute__((ext_vector_type(4)));
};
template <>
struct RawOf<8> {
    typedef uint32_t type __attribute__((ext_vector_type(2)));
};

template <class T, int VEC, bool NT>
__device__ __forceinline__ void load_vec(const T *p, T (&e)[VEC]) {
    using R = typename RawOf<sizeof(T) * VEC>::type;
    R r;
    if constexpr (NT) r = __builtin_nontemporal_load(reinterpret_cast<const R *>(p));
    else r = *reinterpret_cast<const R *>(p);
    __builtin_memcpy(e, &r, sizeof(R));
}
template <class T, int VEC, bool NT>
__device__ __forceinline__ void store_vec(T *p, const T (&e)[VEC]) {
    using R = typename RawOf<sizeof(T) * VEC>::type;
    R r;
    __builtin_memcpy(&r, e, sizeof(R));
    if constexpr (NT) __builtin_nontemporal_store(r, reinterpret_cast<R *>(p));
    else *reinterpret_cast<R *>(p) = r;
}

// The reaction of a variant without its advection, and whether it advects.
template <int V>
constexpr int kReactionOf = (V == kAdvLin1 || V == kShearLin1) ? kLin1 : ((V == kAdvGS || V == kShearGS) ? kGS : V);
template <int V>
constexpr bool kShear = V == kShearLin1 || V == kShearGS;
template <int V>
constexpr bool kAdvective = V == kAdvLin1 || V == kAdvGS || kShear<V>;

template <int V>
struct NSpecies {
    static constexpr int value = kReactionOf<V> == kGS ? 2 : kReactionOf<V> + 1;
};

// a * b + c rounded once.  The site update turns automatic contraction off
// and writes every fused multiply-add out with this, so that each kernel
// that inlines it (one-step, LDS tiles, marching strips, batches) rounds
// exactly alike: a contraction left to the compiler may fuse a different
// product of the same expression in a different kernel.
__device__ __forceinline__ float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Reaction term for one site (Section II.B linear decay; Section III
// Gray-Scott with A_0 = k_1 = 1).
template <int V, class C>
__device__ __forceinline__ void reaction(const Params<C> &p, const C (&rho)[NSpecies<V>::value],
                                         C (&R)[NSpecies<V>::value]) {
#pragma clang fp contract(off)
    constexpr int NS = NSpecies<V>::value;
    if constexpr (kReactionOf<V> == kGS) {
        const C u = rho[0], v = rho[1];
        const C uvv = u * v * v;
        R[0] = fma_c(p.F, C(1) - u, -uvv);
        R[1] = fma_c(-p.Fk, v, uvv);
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            C acc = C(0);
#pragma unroll
            for (int j = 0; j < NS; ++j) acc = fma_c(p.K[s * NS + j], rho[j], acc);
            R[s] = acc + p.c[s];
        }
    }
}

// ------------------------------------------------------- site update --

// Collide and react one site: f holds the nine pulled populations of each
// species in deviation form (d = f for F64 / F32, f - c_i rho_ref,s for the
// 16-bit forms); o receives the encoded post-collision values.  With
// m_s = sum_i d_i (ascending i), rho_s = m_s + rho_ref,s (the c_i sum to
// one) and the update f' = f (1 - 1/tau) + c_i rho / tau + w_i R reads
// d' = d (1 - 1/tau) + c_i m / tau + w_i R; without advection c_i = w_i and
// d' = d (1 - 1/tau) + w_i (m / tau + R).
__device__ __forceinline__ float sinpi_c(float a) { return sinpif(a); }
__device__ __forceinline__ double sinpi_c(double a) { return sinpi(a); }

// Equilibrium coefficients c_i(u) of Eq. "Maxwellian" for the shear flow's
// velocity on row gy: u_x = u0x + amp sin(2 pi m gy / ny), u_y = u0y (the
// phase m gy mod ny is taken in integers).
template <class C>
__device__ __forceinline__ void shear_ceq(const Params<C> &p, int gy, C (&c)[9]) {
#pragma clang fp contract(off)
    const int r = (int)(((int64_t)p.shear_m * gy) % p.shear_ny);
    const C ux = fma_c(p.amp, sinpi_c(C(2 * r) / C(p.shear_ny)), p.u0x);
    const C uy = p.u0y;
    const C uu = fma_c(ux, ux, uy * uy);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const C eu = fma_c(C(kEx[i]), ux, C(kEy[i]) * uy);
        c[i] = wgt<C>(i) * fma_c(C(-1.5), uu, fma_c(C(4.5) * eu, eu, fma_c(C(3), eu, C(1))));
    }
}

// The relaxation f (1 - 1/tau) + e of two species in a 16-bit form, rounded
// plane by plane: species 0 and 1 of plane i in one packed conversion, each
// value computed and rounded as in the species-major order.
template <int ST>
__device__ __forceinline__ void relax_planes(const Params<float> &p, const float (&f)[2][9], const float (&e)[2][9],
                                             uint16_t (&o)[2][9]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        float r0 = fma_c(f[0][i], p.keep[0], e[0][i]);
        float r1 = fma_c(f[1][i], p.keep[1], e[1][i]);
        asm volatile("" : "+v"(r0));
        asm volatile("" : "+v"(r1));
        encode_pair<ST>(r0, r1, o[0][i], o[1][i]);
    }
}

// gy: the site's row (used by the shear variants only).  PM: the 16-bit
// results of two species are rounded plane by plane (encode_sites).
template <int ST, int V, bool PM = false>
__device__ __forceinline__ void collide_site(const Params<typename Traits<ST>::C> &p,
                                             const typename Traits<ST>::C (&f)[NSpecies<V>::value][9],
                                             typename Traits<ST>::T (&o)[NSpecies<V>::value][9], int gy) {
#pragma clang fp contract(off)
    using C = typename Traits<ST>::C;
    constexpr int NS = NSpecies<V>::value;
    C m[NS], rho[NS], R[NS];
    C res[NS][9];   // 16-bit forms: the FP32 results before rounding
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        C acc = f[s][0];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            if constexpr (ST == kF16) acc = add_half(acc, (_Float16)f[s][i]);   // f holds binary16 values
            else acc += f[s][i];
        }
        m[s] = acc;
        rho[s] = kShifted<ST> ? acc + p.rho_ref[s] : acc;
    }
    reaction<V, C>(p, rho, R);
    if constexpr (kAdvective<V>) {
        C ceq[9];
        if constexpr (kShear<V>) {
            shear_ceq<C>(p, gy, ceq);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) ceq[i] = p.ceq[i];
        }
        C e[NS][9];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            // c_i m / tau + w_i R for the moving populations; the rest
            // population takes what makes the nine terms sum to m / tau + R
            const C om = p.omega[s] * m[s];
            const C a = om + R[s];
            C moving = C(0);
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                e[s][i] = fma_c(ceq[i], om, wgt<C>(i) * R[s]);
                moving += e[s][i];
            }
            e[s][0] = a - moving;
        }
        if constexpr (PM && kShifted<ST> && NS == 2) {
            relax_planes<ST>(p, f, e, o);
            return;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                C r = fma_c(f[s][i], p.keep[s], e[s][i]);
                if constexpr (kShifted<ST>) {
                    asm volatile("" : "+v"(r));
                    res[s][i] = r;
                } else {
                    o[s][i] = r;
                }
            }
        }
        if constexpr (kShifted<ST>) encode_sites<ST, NS, PM>(res, o);
        return;
    }
    C ep[NS][9];   // two species in a 16-bit form, plane-major rounding: the e terms
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        // w_i (m / tau + R): the rest weight is taken as 1 - 4/9 - 4/36
        // applied to the value itself, so the nine terms sum to exactly
        // m / tau + R up to unbiased rounding (the rounded weights of a
        // binary format sum to 1 + O(eps), which would add a systematic mass
        // drift every step).
        const C a = fma_c(p.omega[s], m[s], R[s]);
        const C e1 = wgt<C>(1) * a, e5 = wgt<C>(5) * a;
        // (a - 4 e1) - 4 e5: 4 e1 and 4 e5 are exact, so each multiply-add
        // rounds exactly as the subtraction it stands for
        const C e0 = fma_c(C(-4), e5, fma_c(C(-4), e1, a));
        if constexpr (PM && kShifted<ST> && NS == 2) {
#pragma unroll
            for (int i = 0; i < 9; ++i) ep[s][i] = i == 0 ? e0 : (i < 5 ? e1 : e5);
            continue;
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const C e = i == 0 ? e0 : (i < 5 ? e1 : e5);
            C r = fma_c(f[s][i], p.keep[s], e);
            // 16-bit forms: keep the float result as a value of its own so
            // the conversion always rounds the float (the compiler may
            // otherwise fold the multiply-add into a mixed-precision
            // instruction that rounds once, differently in different kernels)
            if constexpr (kShifted<ST>) {
                asm volatile("" : "+v"(r));
                res[s][i] = r;
            } else {
                o[s][i] = r;
            }
        }
    }
    if constexpr (PM && kShifted<ST> && NS == 2) relax_planes<ST>(p, f, ep, o);
    else if constexpr (kShifted<ST>) encode_sites<ST, NS, PM>(res, o);
}

// ---------------------------------------------------------- step tile --

struct TileGeom {
    int nx, ny;
    int64_t pitch, pstride;
    int lx_shift, nvec, nseg, rpw;
};

// One wave advances one tile by one step.  `lane` is 0..63; every lane of the
// wave executes this function (lanes outside the lattice compute on clamped
// addresses and do not store).  ROW1: the tile is one row of 64 lanes
// (lanes_x = 64), so the row and every plane's row base are wave-uniform and
// live in scalar registers; loads then take a scalar base plus one per-lane
// offset.
template <int ST, int V, int VEC, bool NT, bool ROW1 = false>
__device__ __forceinline__ void step_tile(const typename Traits<ST>::T *__restrict__ src,
                                          typename Traits<ST>::T *__restrict__ dst, const TileGeom &g,
                                          int64_t tile, int lane, const Params<typename Traits<ST>::C> &p) {
    using T = typename Traits<ST>::T;
    using C = typename Traits<ST>::C;
    constexpr int NS = NSpecies<V>::value;

    const int lanes_x = ROW1 ? 64 : 1 << g.lx_shift;
    const int sx = (int)(tile % g.nseg);
    const int ry = (int)(tile / g.nseg);
    const int vx = ROW1 ? lane : lane & (lanes_x - 1);
    const int y = ROW1 ? ry : ry * g.rpw + (lane >> g.lx_shift);
    const bool row_ok = y < g.ny;
    const int yc = row_ok ? y : g.ny - 1;
    const int v = sx * lanes_x + vx;
    const bool vec_ok = v < g.nvec;
    const int x0 = (vec_ok ? v : g.nvec - 1) * VEC;
    const int cnt = min(VEC, g.nx - x0);              // valid sites of this vector
    const bool last = x0 + VEC >= g.nx;                // holds site nx - 1
    const bool edge_lo = vx == 0;                      // left neighbour not in this segment
    const bool edge_hi = (vx == lanes_x - 1) || last;  // right neighbour not in this segment
    const int ym = yc == 0 ? g.ny - 1 : yc - 1;
    const int yp = yc + 1 == g.ny ? 0 : yc + 1;
    const int xprev = x0 == 0 ? g.nx - 1 : x0 - 1;
    const int xnext = last ? 0 : x0 + VEC;

    // Pull loads: plane (s, i) at row y - e_iy.
    T raw[NS][9][VEC];
    T e_lo[NS][9], e_hi[NS][9];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int row = kEy[i] == 1 ? ym : (kEy[i] == -1 ? yp : yc);
            const T *rp = src + (int64_t)(s * 9 + i) * g.pstride + (int64_t)row * g.pitch;
            // 32-bit byte offset from a (for ROW1 wave-uniform) row base: lets
            // the compiler use the scalar-base + vector-offset address form
            load_vec<T, VEC, NT>(reinterpret_cast<const T *>(reinterpret_cast<const char *>(rp) +
                                                             (uint32_t)x0 * (uint32_t)sizeof(T)),
                                 raw[s][i]);
            // only the edge lanes issue these single-element loads (exec-masked)
            e_lo[s][i] = T(0);
            e_hi[s][i] = T(0);
            if (kEx[i] == 1) {
                if (edge_lo)
                    e_lo[s][i] = *reinterpret_cast<const T *>(reinterpret_cast<const char *>(rp) +
                                                              (uint32_t)xprev * (uint32_t)sizeof(T));
            }
            if (kEx[i] == -1) {
                if (edge_hi)
                    e_hi[s][i] = *reinterpret_cast<const T *>(reinterpret_cast<const char *>(rp) +
                                                              (uint32_t)xnext * (uint32_t)sizeof(T));
            }
        }
    }

    // Decode and shift along x.  The 16-bit forms are kept in deviation form
    // d = f - w_i rho_ref,s throughout (no shift is added or removed per
    // population); for F64 / F32 storage d = f.
    C f[NS][9][VEC];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            C d[VEC];
#pragma unroll
            for (int j = 0; j < VEC; ++j) d[j] = decode_dev<ST>(raw[s][i][j]);
            if (kEx[i] == 0) {
#pragma unroll
                for (int j = 0; j < VEC; ++j) f[s][i][j] = d[j];
            } else if (kEx[i] == 1) {
                const C nb = __shfl_up(d[VEC - 1], 1);
                const C prev = edge_lo ? decode_dev<ST>(e_lo[s][i]) : nb;
                f[s][i][0] = prev;
#pragma unroll
                for (int j = 1; j < VEC; ++j) f[s][i][j] = d[j - 1];
            } else {
                const C nb = __shfl_down(d[0], 1);
                const C next = edge_hi ? decode_dev<ST>(e_hi[s][i]) : nb;
#pragma unroll
                for (int j = 0; j < VEC - 1; ++j) f[s][i][j] = (last && j == cnt - 1) ? next : d[j + 1];
                f[s][i][VEC - 1] = next;
            }
        }
    }

    // Collide and react, site by site.
    T out[NS][9][VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        C fs[NS][9];
        T os[NS][9];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) fs[s][i] = f[s][i][j];
        collide_site<ST, V>(p, fs, os, yc);
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) out[s][i][j] = os[s][i];
    }

    if (row_ok && vec_ok) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i)
                store_vec<T, VEC, NT>(
                    reinterpret_cast<T *>(reinterpret_cast<char *>(dst + (int64_t)(s * 9 + i) * g.pstride +
                                                                   (int64_t)yc * g.pitch) +
                                          (uint32_t)x0 * (uint32_t)sizeof(T)),
                    out[s][i]);
    }
}

// Block index remap so that consecutive tiles land on the same XCD (blocks
// are dealt to the 8 XCDs round-robin): XCD x gets a contiguous run.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

template <int ST, int V, int VEC, bool NT, bool ROW1>
__global__ __launch_bounds__(256) void k_step(Grid gr, Params<typename Traits<ST>::C> p) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    const int b = gr.xcd_order ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int64_t stride = (int64_t)gridDim.x * waves;
    TileGeom g{gr.nx, gr.ny, gr.pitch, gr.pstride, gr.lx_shift, gr.nvec, gr.nseg, gr.rpw};
    // one tile per wave when the grid covers all tiles; a persistent grid
    // walks the tiles with a stride of the whole grid
    for (int64_t tile = (int64_t)b * waves + wave; tile < gr.ntiles; tile += stride)
        step_tile<ST, V, VEC, NT, ROW1>(static_cast<const typename Traits<ST>::T *>(gr.src),
                                        static_cast<typename Traits<ST>::T *>(gr.dst), g, tile, lane, p);
}

// ------------------------------------------- several steps per launch --

__device__ __forceinline__ int wrap_mod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Raw buffer access with a 32-bit byte offset split into a per-lane part
// (voffset) and a wave-uniform part (soffset, the plane): the hardware adds
// them to the descriptor's base, so no 64-bit address arithmetic is spent per
// population.  Accesses beyond the descriptor's byte range read 0 and do not
// write.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
template <class T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}
// NT: a streaming (non-temporal) store, cache policy bit "nt".
template <class T, bool NT = false>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, T v) {
    constexpr int aux = NT ? 2 : 0;
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(typename RawOf<8>::type, v), r, voff, soff, aux);
    else if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, aux);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, voff, soff, aux);
}

// a * b for a, b below 2^24 (one full-rate multiply)
__device__ __forceinline__ uint32_t mul24(int a, uint32_t b) { return (uint32_t)__umul24((uint32_t)a, b); }

// LDS layout of the multi-step region: row-interleaved planes, element
// (plane P, column x, row y) at y * RS + P * EW + x, with EW the region width
// and RS = stepT_row_stride (9 N EW plus bank padding).  Consecutive lanes
// touch consecutive banks.
//
// The post-collision value leaving site z along e_i is kept in one of two
// forms, alternating phase by phase (the "AA" arrangement):
//   form A: in plane opp(i) at z itself;
//   form B: in plane i at z + e_i, the site it streams to.
// A site x then reads and writes the same cells within one step: from form
// A it pulls plane opp(i) at x - e_i and writes form B into plane i at
// x + e_i (the same cells); from form B it reads plane i at x and writes
// form A into plane opp(i) at x.  No two sites share a cell, so a phase
// updates its region in place with no barrier between its reads and writes.
constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};   // e_opp(i) = -e_i

template <int ST, int NS, int EW, bool FROM_B>
__device__ __forceinline__ void gather_lds(const typename Traits<ST>::T *L, int lx, int ly,
                                           typename Traits<ST>::C (&f)[NS][9]) {
    constexpr int RS = stepT_row_stride(NS, EW, (int)sizeof(typename Traits<ST>::T));
    if constexpr (FROM_B) {
        const typename Traits<ST>::T *b = L + ly * RS + lx;
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) f[s][i] = decode_dev<ST>(b[(s * 9 + i) * EW]);
    } else {
        // from the lower-left neighbour, so every offset is non-negative
        const typename Traits<ST>::T *b = L + (ly - 1) * RS + (lx - 1);
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i)
                f[s][i] = decode_dev<ST>(b[(1 - kEy[i]) * RS + (s * 9 + kOpp[i]) * EW + (1 - kEx[i])]);
    }
}
template <int ST, int NS, int EW, bool TO_B>
__device__ __forceinline__ void put_lds(typename Traits<ST>::T *L, int lx, int ly,
                                        const typename Traits<ST>::T (&o)[NS][9]) {
    constexpr int RS = stepT_row_stride(NS, EW, (int)sizeof(typename Traits<ST>::T));
    if constexpr (TO_B) {
        typename Traits<ST>::T *b = L + (ly - 1) * RS + (lx - 1);
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) b[(1 + kEy[i]) * RS + (s * 9 + i) * EW + (1 + kEx[i])] = o[s][i];
    } else {
        typename Traits<ST>::T *b = L + ly * RS + lx;
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) b[(s * 9 + kOpp[i]) * EW] = o[s][i];
    }
}

// Geometry of one lattice as the multi-step tile reads it.  A buffer below
// 4 GiB is one buffer resource, the plane selected by the wave-uniform
// offset; a larger one (BIG) is addressed plane by plane, each plane below
// 4 GiB its own resource from the 64-bit base pointer.
struct TileT {
    __amdgpu_buffer_rsrc_t src, dst;
    int nx, ny, th;
    uint32_t pitch_b, pstride_b;   // row and plane strides in bytes
    int nt_store;                  // 1: streaming stores of the result (working set beyond the caches)
    const char *src_p;             // BIG: base pointers, plane stride and plane bytes
    char *dst_p;
    uint64_t pstride_64;
    uint32_t plane_b;
};

// Value of plane P at byte offset voff + soff from the plane's origin.
template <class T, bool BIG>
__device__ __forceinline__ T tile_load(const TileT &g, int P, uint32_t voff, uint32_t soff) {
    if constexpr (BIG) return buf_load<T>(buffer_rsrc(g.src_p + (uint64_t)P * g.pstride_64, g.plane_b), voff, soff);
    else return buf_load<T>(g.src, voff, (uint32_t)P * g.pstride_b + soff);
}
template <class T, bool BIG, bool NT = false>
__device__ __forceinline__ void tile_store(const TileT &g, int P, uint32_t voff, T v) {
    if constexpr (BIG) buf_store<T, NT>(buffer_rsrc(g.dst_p + (uint64_t)P * g.pstride_64, g.plane_b), voff, 0u, v);
    else buf_store<T, NT>(g.dst, voff, (uint32_t)P * g.pstride_b, v);
}

// Middle phase J of a multi-step tile: the region shrunk by J-1 on every
// side, read in the form phase J-1 wrote and written in the other one.
template <int ST, int V, int EW, int J>
__device__ __forceinline__ void stepT_middle(const Params<typename Traits<ST>::C> &p, typename Traits<ST>::T *L,
                                             int eh, int nthr, int gy0, int ny) {
    using T = typename Traits<ST>::T;
    using C = typename Traits<ST>::C;
    constexpr int NS = NSpecies<V>::value;
    constexpr bool kFromB = (J - 1) % 2 == 0;   // phase J-1 wrote form B when even
    constexpr int W = EW - 2 * (J - 1);          // width of the shrunk region
    const int rsz = W * (eh - 2 * (J - 1));
    for (int q = threadIdx.x; q < rsz; q += nthr) {
        const int lx = q % W + (J - 1), ly = q / W + (J - 1);
        C f[NS][9];
        gather_lds<ST, NS, EW, kFromB>(L, lx, ly, f);
        T o[NS][9];
        collide_site<ST, V>(p, f, o, kShear<V> ? wrap_mod(gy0 + ly, ny) : 0);
        put_lds<ST, NS, EW, !kFromB>(L, lx, ly, o);
    }
}

// Middle phases J, J+1, .. min(m, TS)-1, each followed by a barrier.
template <int ST, int V, int TS, int EW, int J, bool VARM>
__device__ __forceinline__ void stepT_middles(const Params<typename Traits<ST>::C> &p, typename Traits<ST>::T *L,
                                              int eh, int nthr, int m, int gy0, int ny) {
    if constexpr (J < TS) {
        if (!VARM || m > J) {
            stepT_middle<ST, V, EW, J>(p, L, eh, nthr, gy0, ny);
            __syncthreads();
            stepT_middles<ST, V, TS, EW, J + 1, VARM>(p, L, eh, nthr, m, gy0, ny);
        }
    }
}

// Last phase of a multi-step tile: pull from LDS (form B when the previous
// phase was even), collide on the tile itself, store to the destination.
template <int ST, int V, int TW, int H, bool FROM_B, bool BIG>
__device__ __forceinline__ void stepT_last(const TileT &g, const Params<typename Traits<ST>::C> &p,
                                           const typename Traits<ST>::T *L, int x0, int y0, int nthr) {
    using T = typename Traits<ST>::T;
    using C = typename Traits<ST>::C;
    constexpr int NS = NSpecies<V>::value;
    constexpr int EW = TW + 2 * H;
    const int tsz = TW * g.th;
    for (int q = threadIdx.x; q < tsz; q += nthr) {
        const int lx = q % TW, ly = q / TW;
        const int gx = x0 + lx, gy = y0 + ly;
        C f[NS][9];
        gather_lds<ST, NS, EW, FROM_B>(L, lx + H, ly + H, f);
        T o[NS][9];
        collide_site<ST, V>(p, f, o, kShear<V> ? wrap_mod(gy, g.ny) : 0);
        if (gx < g.nx && gy < g.ny) {
            const uint32_t off = mul24(gy, g.pitch_b) + (uint32_t)gx * sizeof(T);
            if (g.nt_store) {
#pragma unroll
                for (int s = 0; s < NS; ++s)
#pragma unroll
                    for (int i = 0; i < 9; ++i) tile_store<T, BIG, true>(g, s * 9 + i, off, o[s][i]);
            } else {
#pragma unroll
                for (int s = 0; s < NS; ++s)
#pragma unroll
                    for (int i = 0; i < 9; ++i) tile_store<T, BIG>(g, s * 9 + i, off, o[s][i]);
            }
        }
    }
}

// TS time steps on one tile of TW x th sites whose lower-left site is
// (x0, y0) (temporal blocking; called by every thread of the workgroup).
// The workgroup keeps a (TW + 2h) x (th + 2h) region in LDS, h = TS - 1.
// Phase 1 reads step t from the source buffer (pulling across the region's
// edge), collides, and writes the post-collision values of step t+1 on the
// whole region to LDS (form A).  Each middle phase j = 2 .. m-1 advances the
// region shrunk by j-1 sites on every side, in place, alternating the two
// forms so that a site's reads and writes hit cells no other site touches:
// one barrier per phase.  The last phase pulls from LDS, collides on the
// tile itself and stores step t+m.  Per m steps the buffer is read once
// (tile plus a halo) and written once.  Every
// site runs the arithmetic of the one-step kernel on the same encoded inputs,
// so the result is bitwise identical to m one-step launches.  m = TS unless
// VARM, where 1 <= m <= TS is a workgroup-uniform runtime count (m = 1 reads
// and writes the buffers directly).  Byte offsets are 32-bit: within the
// buffer, or within a plane when BIG.
template <int ST, int V, int TS, int TW, bool VARM, bool BIG = false>
__device__ __forceinline__ void stepT_tile(const TileT &g, const Params<typename Traits<ST>::C> &p, int x0, int y0,
                                           int m, typename Traits<ST>::T *L) {
    using T = typename Traits<ST>::T;
    using C = typename Traits<ST>::C;
    constexpr int NS = NSpecies<V>::value;
    constexpr int H = TS - 1;
    constexpr int EW = TW + 2 * H;
    constexpr uint32_t B = sizeof(T);
    const int nx = g.nx, ny = g.ny, th = g.th;
    const int tsz = TW * th;
    const int nthr = blockDim.x;
    if constexpr (!VARM) m = TS;
    if (VARM && m == 1) {
        // a single step: pull from the source buffer, store to the destination
        for (int q = threadIdx.x; q < tsz; q += nthr) {
            const int gx = x0 + q % TW, gy = y0 + q / TW;
            if (gx < nx && gy < ny) {
                const uint32_t cx[3] = {(uint32_t)(gx == 0 ? nx - 1 : gx - 1) * B, (uint32_t)gx * B,
                                        (uint32_t)(gx + 1 == nx ? 0 : gx + 1) * B};
                const uint32_t ry[3] = {mul24(gy == 0 ? ny - 1 : gy - 1, g.pitch_b), mul24(gy, g.pitch_b),
                                        mul24(gy + 1 == ny ? 0 : gy + 1, g.pitch_b)};
                C f[NS][9];
#pragma unroll
                for (int s = 0; s < NS; ++s)
#pragma unroll
                    for (int i = 0; i < 9; ++i)
                        f[s][i] = decode_dev<ST>(tile_load<T, BIG>(g, s * 9 + i, ry[1 - kEy[i]] + cx[1 - kEx[i]], 0u));
                T o[NS][9];
                collide_site<ST, V>(p, f, o, gy);
#pragma unroll
                for (int s = 0; s < NS; ++s)
#pragma unroll
                    for (int i = 0; i < 9; ++i) tile_store<T, BIG>(g, s * 9 + i, ry[1] + cx[1], o[s][i]);
            }
        }
        return;
    }
    const int eh = th + 2 * H, esz = EW * eh;
    // phase 1: step t -> t+1 on the whole region, from the source buffer
    const int dx = nthr % EW, dy = nthr / EW;
    int ex = (int)threadIdx.x % EW, ey = (int)threadIdx.x / EW;
    if (x0 >= H + 1 && x0 + TW + H + 1 <= nx && y0 >= H + 1 && y0 + th + H + 1 <= ny) {
        // Interior tile: the pulled region does not wrap.  The lane's byte
        // offset from the region's lower-left site is advanced incrementally;
        // the plane and the pull shift -e_i go into the wave-uniform offset.
        const uint32_t base = mul24(y0 - H, g.pitch_b) + (uint32_t)(x0 - H) * B;
        const uint32_t step = (uint32_t)dy * g.pitch_b + (uint32_t)dx * B, wrap = g.pitch_b - (uint32_t)EW * B;
        uint32_t rel = mul24(ey, g.pitch_b) + (uint32_t)ex * B;
        for (int q = threadIdx.x; q < esz; q += nthr) {
            C f[NS][9];
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    f[s][i] = decode_dev<ST>(
                        tile_load<T, BIG>(g, s * 9 + i, rel, base - kEy[i] * g.pitch_b - kEx[i] * B));
            T o[NS][9];
            collide_site<ST, V>(p, f, o, y0 - H + ey);
            put_lds<ST, NS, EW, false>(L, ex, ey, o);
            ex += dx;
            ey += dy;
            rel += step;
            if (ex >= EW) {
                ex -= EW;
                ++ey;
                rel += wrap;
            }
        }
    } else {
        const bool one_wrap = nx >= TW + H && ny >= th + H;   // the region wraps at most once per axis
        for (int q = threadIdx.x; q < esz; q += nthr) {
            int gx = x0 - H + ex, gy = y0 - H + ey;
            if (one_wrap) {
                gx += gx < 0 ? nx : 0;
                gx -= gx >= nx ? nx : 0;
                gy += gy < 0 ? ny : 0;
                gy -= gy >= ny ? ny : 0;
            } else {
                gx = wrap_mod(gx, nx);
                gy = wrap_mod(gy, ny);
            }
            // byte offsets of columns x-1, x, x+1 and rows y-1, y, y+1
            const uint32_t cx[3] = {(uint32_t)(gx == 0 ? nx - 1 : gx - 1) * B, (uint32_t)gx * B,
                                    (uint32_t)(gx + 1 == nx ? 0 : gx + 1) * B};
            const uint32_t ry[3] = {mul24(gy == 0 ? ny - 1 : gy - 1, g.pitch_b), mul24(gy, g.pitch_b),
                                    mul24(gy + 1 == ny ? 0 : gy + 1, g.pitch_b)};
            C f[NS][9];
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    f[s][i] = decode_dev<ST>(tile_load<T, BIG>(g, s * 9 + i, ry[1 - kEy[i]] + cx[1 - kEx[i]], 0u));
            T o[NS][9];
            collide_site<ST, V>(p, f, o, gy);
            put_lds<ST, NS, EW, false>(L, ex, ey, o);
            ex += dx;
            ey += dy;
            if (ex >= EW) {
                ex -= EW;
                ++ey;
            }
        }
    }
    __syncthreads();
    // middle phases j = 2 .. m-1: step t+j-1 -> t+j on the region shrunk by
    // j-1, in LDS, in place (phase j reads the form phase j-1 wrote: A after
    // odd phases, B after even ones).  Consecutive threads take consecutive
    // sites of the shrunk region, row by row.
    stepT_middles<ST, V, TS, EW, 2, VARM>(p, L, eh, nthr, m, y0 - H, ny);
    // last phase: step t+m-1 -> t+m on the tile, to the destination buffer
    if (m & 1)
        stepT_last<ST, V, TW, H, true, BIG>(g, p, L, x0, y0, nthr);
    else
        stepT_last<ST, V, TW, H, false, BIG>(g, p, L, x0, y0, nthr);
    __syncthreads();   // LDS is reused by the next tile
}

// TS steps per launch over one lattice: one workgroup per tile (or a
// persistent grid walking the tiles).  BIG: buffers of 4 GiB or more,
// addressed plane by plane.
template <int ST, int V, int TS, int TW, bool BIG>
__global__ __launch_bounds__(1024) void k_stepT(GridT g, Params<typename Traits<ST>::C> p) {
    using T = typename Traits<ST>::T;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    TileT t;
    t.src = buffer_rsrc(g.src, g.bytes);
    t.dst = buffer_rsrc(g.dst, g.bytes);
    t.nx = g.nx;
    t.ny = g.ny;
    t.th = g.th;
    t.pitch_b = (uint32_t)g.pitch * (uint32_t)sizeof(T);
    t.pstride_b = (uint32_t)g.pstride * (uint32_t)sizeof(T);
    t.nt_store = g.nt_store;
    t.src_p = static_cast<const char *>(g.src);
    t.dst_p = static_cast<char *>(g.dst);
    t.pstride_64 = (uint64_t)g.pstride * sizeof(T);
    t.plane_b = g.plane_bytes;
    const int b0 = g.xcd_order ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    // tiles in strips of g.strip tile columns (g.ntx: plain row-major),
    // row-major inside a strip, the last strip possibly narrower; a launch
    // has fewer than 2^31 tiles (each plane is below 4 GiB)
    const int per = g.strip * g.nty;
    for (int tile = b0; tile < (int)g.ntiles; tile += gridDim.x) {
        const int si = tile / per, r = tile - si * per;
        const int sw = min(g.strip, g.ntx - si * g.strip);
        const int ty = r / sw, tx = si * g.strip + (r - ty * sw);
        stepT_tile<ST, V, TS, TW, false, BIG>(t, p, tx * TW, ty * g.th, TS, reinterpret_cast<T *>(smem));
    }
}

// ------------------------------------------------- marching wave strips --
//
// TS time steps per launch without LDS and without barriers.  Each wave owns
// a strip of 64 columns (one per lane; the 2(TS-1) outer columns are halo,
// recomputed by the neighbouring strips) and marches down a segment of rows.
// Level k (the state after k of the launch's steps) is computed one row
// behind level k-1: in iteration j, level 1 computes row r = y0 - h + j from
// the source buffer and level k row r - (k-1) from level k-1, in ascending k,
// so every input of a level is ready when it runs.  Level k at row q pulls,
// from level k-1, the planes with e_y = -1 of row q+1 (computed in the same
// iteration), those with e_y = 0 of row q (the previous iteration) and those
// with e_y = +1 of row q-1 (two iterations back): each level keeps 9 values
// per species of its last two rows in registers.  A pull along x (e_x = +-1)
// takes the neighbouring lane's value by a wavefront shift (DPP).  Level TS
// stores its row; the rows above a segment (its first 2h iterations) only
// fill the pipeline, so a segment of L rows computes L + 2h level-1 rows.
// Only the x-halo is recomputed: 64 / (64 - 2h) per level.  Every site runs
// collide_site on the decoded values the one-step kernel would read, so the
// result is bitwise identical to TS one-step launches.

// v of lane l+1 (wave_shl:1) and of lane l-1 (wave_shr:1); the lanes at the
// wave's edges get their own value back (they hold halo columns).
template <class T>
__device__ __forceinline__ T from_right(T v) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const int lo = __builtin_amdgcn_update_dpp((int)u, (int)u, 0x130, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp((int)(u >> 32), (int)(u >> 32), 0x130, 0xf, 0xf, false);
        return __builtin_bit_cast(T, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    } else if constexpr (sizeof(T) == 4) {
        const int u = __builtin_bit_cast(int, v);
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(u, u, 0x130, 0xf, 0xf, false));
    } else {
        const int u = (int)__builtin_bit_cast(uint16_t, v);
        return __builtin_bit_cast(T, (uint16_t)__builtin_amdgcn_update_dpp(u, u, 0x130, 0xf, 0xf, false));
    }
}
template <class T>
__device__ __forceinline__ T from_left(T v) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const int lo = __builtin_amdgcn_update_dpp((int)u, (int)u, 0x138, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp((int)(u >> 32), (int)(u >> 32), 0x138, 0xf, 0xf, false);
        return __builtin_bit_cast(T, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    } else if constexpr (sizeof(T) == 4) {
        const int u = __builtin_bit_cast(int, v);
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(u, u, 0x138, 0xf, 0xf, false));
    } else {
        const int u = (int)__builtin_bit_cast(uint16_t, v);
        return __builtin_bit_cast(T, (uint16_t)__builtin_amdgcn_update_dpp(u, u, 0x138, 0xf, 0xf, false));
    }
}

// The values a level keeps for the next one, already moved to the column
// that pulls them (planes with e_x = +1 from the left lane, e_x = -1 from the
// right lane): row q-1's planes with e_y = 0 (a: planes 0, 1, 3) and the
// planes with e_y = +1 of the two latest rows (b: planes 2, 5, 6), b[P] for
// the rows of iterations of parity P.  The iteration loop is unrolled by two,
// so a level's new values go to registers of their own and no value is
// copied from one register to another between iterations.
template <class T, int NS>
struct MarchCarry {
    T a[NS][3];
    T b[2][NS][3];
};

// FP64 strips store from every lane: a result lane at its column, a halo
// lane out of range (march_store).  The other forms store from the result
// lanes only, under a branch on the lane.
template <int ST>
constexpr bool kMarchStoreAll = ST == kF64;

// Stores row q of the launch's last level: the 9N populations of each
// result lane.  With kMarchStoreAll every lane stores (nt is not used):
// col_b is the lane's byte column for a result lane and 0xffffffff for a
// halo lane, and the whole byte offset is formed in the lane with a
// saturating add, so a halo lane's stays 0xffffffff, at or past the end of
// every buffer below 4 GiB, and the hardware drops the store (a raw buffer
// access is out of range when its offset reaches the descriptor's byte
// count; the scalar offset is 0, so that holds whether or not the range
// check counts it).  Without the branch the compiler's waits in the FP64
// loop no longer assume the path without stores (measured: 4096^2 FP64
// Gray-Scott at T 8 155.6 against 183.3 us per step).  For FP32 and the
// 16-bit forms the two extra instructions per store cost more than the
// waits (64.9 against 61.7 us at 4096^2 FP32).
// Where a marching launch stores: one descriptor for a buffer below 4 GiB
// (plane P at P * pstride_b bytes), or, with BIG (a buffer of 4 GiB or more,
// each plane below it), a descriptor per plane from the 64-bit base.
struct MarchOut {
    __amdgpu_buffer_rsrc_t dst;
    uint32_t pstride_b;
    char *dst_p;
    uint64_t pstride_64;
    uint32_t plane_b;
};

// Stores v to plane P at byte offset voff + row of its plane (row < the
// plane's bytes).
template <class T, bool NT, bool BIG>
__device__ __forceinline__ void store_plane(const MarchOut &out, int P, uint32_t voff, uint32_t row, T v) {
    if constexpr (BIG) buf_store<T, NT>(buffer_rsrc(out.dst_p + (uint64_t)P * out.pstride_64, out.plane_b), voff, row, v);
    else buf_store<T, NT>(out.dst, voff, (uint32_t)P * out.pstride_b + row, v);
}

template <int ST, int V, bool BIG = false>
__device__ __forceinline__ void march_store(typename Traits<ST>::T (&o)[NSpecies<V>::value][9], int q,
                                            const MarchOut &out, uint32_t pitch_b, uint32_t col_b, bool nt) {
    using T = typename Traits<ST>::T;
    constexpr int NS = NSpecies<V>::value;
    const uint32_t row = (uint32_t)q * pitch_b;
    if constexpr (kMarchStoreAll<ST>) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int P = s * 9 + i;
                if constexpr (BIG)
                    buf_store<T>(buffer_rsrc(out.dst_p + (uint64_t)P * out.pstride_64, out.plane_b),
                                 __builtin_elementwise_add_sat(col_b, row), 0u, o[s][i]);
                else
                    buf_store<T>(out.dst, __builtin_elementwise_add_sat(col_b, (uint32_t)P * out.pstride_b + row), 0u,
                                 o[s][i]);
            }
        return;
    }
    if (nt) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) store_plane<T, true, BIG>(out, s * 9 + i, col_b, row, o[s][i]);
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) store_plane<T, false, BIG>(out, s * 9 + i, col_b, row, o[s][i]);
    }
}

// Level K+1 .. TS of an iteration of parity P, from level K's outputs o (row
// q) and the carry of level K; level K+1 computes row q-1 when it is active
// (iteration j >= 2K).  Level TS stores its row.  With RM (a runtime step
// count m <= TS, the batched launches) level m stores instead, from iteration
// TS - 1 + m - 1 on (its first row of the segment), and the levels above it
// are skipped; the wider x-halo of a TS-step strip covers m steps.  Without
// G (the iterations from 2(TS-1) on, where every level is active) the
// activity tests are left out: the branches they make cost the compiler a
// copy of every carry of the levels they skip.
template <int ST, int V, int TS, int K, int P, bool RM = false, bool G = true, bool BIG = false>
__device__ __forceinline__ void march_levels(const Params<typename Traits<ST>::C> &p,
                                             typename Traits<ST>::T (&o)[NSpecies<V>::value][9],
                                             MarchCarry<typename Traits<ST>::T, NSpecies<V>::value> (&c)[TS - 1],
                                             int j, int q, int ny, const MarchOut &out, uint32_t pitch_b,
                                             uint32_t col_b, bool store_lane, bool nt, int msteps = TS) {
    using T = typename Traits<ST>::T;
    using C = typename Traits<ST>::C;
    constexpr int NS = NSpecies<V>::value;
    if constexpr (RM && K < TS) {
        if (K == msteps && j >= TS - 1 + K - 1 && (kMarchStoreAll<ST> || store_lane))
            march_store<ST, V, BIG>(o, q, out, pitch_b, col_b, nt);
    }
    if constexpr (K == TS) {
        // the last level: row q is the launch's result (active from j >= 2(TS-1))
        if ((!RM || msteps == TS) && (!G || j >= 2 * (TS - 1)) && (kMarchStoreAll<ST> || store_lane))
            march_store<ST, V, BIG>(o, q, out, pitch_b, col_b, nt);
    } else {
        MarchCarry<T, NS> &m = c[K - 1];
        C f[NS][9];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            f[s][4] = decode_dev<ST>(o[s][4]);               // e = ( 0,-1): row q, own column
            f[s][7] = decode_dev<ST>(from_right(o[s][7]));   // e = (-1,-1): row q, column x+1
            f[s][8] = decode_dev<ST>(from_left(o[s][8]));    // e = ( 1,-1): row q, column x-1
            f[s][0] = decode_dev<ST>(m.a[s][0]);             // row q-1
            f[s][1] = decode_dev<ST>(m.a[s][1]);
            f[s][3] = decode_dev<ST>(m.a[s][2]);
            f[s][2] = decode_dev<ST>(m.b[P][s][0]);          // row q-2
            f[s][5] = decode_dev<ST>(m.b[P][s][1]);
            f[s][6] = decode_dev<ST>(m.b[P][s][2]);
            m.a[s][0] = o[s][0];
            m.a[s][1] = from_left(o[s][1]);      // e = ( 1, 0)
            m.a[s][2] = from_right(o[s][3]);     // e = (-1, 0)
            m.b[P][s][0] = o[s][2];              // e = ( 0, 1)
            m.b[P][s][1] = from_left(o[s][5]);   // e = ( 1, 1)
            m.b[P][s][2] = from_right(o[s][6]);  // e = (-1, 1)
        }
        if (!G || j >= 2 * K) {
            T o2[NS][9];
            collide_site<ST, V>(p, f, o2, kShear<V> ? wrap_mod(q - 1, ny) : 0);
            march_levels<ST, V, TS, K + 1, P, RM, G, BIG>(p, o2, c, j, q - 1, ny, out, pitch_b, col_b, store_lane,
                                                       nt, msteps);
        }
    }
}

// Two species in a 16-bit form: the carries hold packed words, species 0 in
// the low half and species 1 in the high half of plane i's word, so one
// lane shift moves both species and a carry takes one register per plane.
struct MarchCarryPk {
    uint32_t a[3];
    uint32_t b[2][3];
};

__device__ __forceinline__ uint32_t pack_planes(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }
__device__ __forceinline__ uint16_t plane_half(uint32_t w, int s) { return s ? (uint16_t)(w >> 16) : (uint16_t)w; }

// march_levels for two species in a 16-bit form on packed words (the same
// values and the same update; the site's results are rounded plane by plane).
template <int ST, int V, int TS, int K, int P, bool RM = false, bool G = true, bool BIG = false>
__device__ __forceinline__ void march_levels_pk(const Params<float> &p, uint16_t (&o)[2][9], MarchCarryPk (&c)[TS - 1],
                                                int j, int q, int ny, const MarchOut &out, uint32_t pitch_b,
                                                uint32_t col_b, bool store_lane, bool nt, int msteps = TS) {
    if constexpr (RM && K < TS) {
        if (K == msteps && j >= TS - 1 + K - 1 && store_lane)
            march_store<ST, V, BIG>(o, q, out, pitch_b, col_b, nt);
    }
    if constexpr (K == TS) {
        if ((!RM || msteps == TS) && (!G || j >= 2 * (TS - 1)) && store_lane)
            march_store<ST, V, BIG>(o, q, out, pitch_b, col_b, nt);
    } else {
        MarchCarryPk &m = c[K - 1];
        uint32_t w[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) w[i] = pack_planes(o[0][i], o[1][i]);
        const uint32_t w7 = from_right(w[7]), w8 = from_left(w[8]);
        float f[2][9];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            f[s][4] = decode_dev<ST>(plane_half(w[4], s));      // e = ( 0,-1): row q, own column
            f[s][7] = decode_dev<ST>(plane_half(w7, s));        // e = (-1,-1): row q, column x+1
            f[s][8] = decode_dev<ST>(plane_half(w8, s));        // e = ( 1,-1): row q, column x-1
            f[s][0] = decode_dev<ST>(plane_half(m.a[0], s));    // row q-1
            f[s][1] = decode_dev<ST>(plane_half(m.a[1], s));
            f[s][3] = decode_dev<ST>(plane_half(m.a[2], s));
            f[s][2] = decode_dev<ST>(plane_half(m.b[P][0], s)); // row q-2
            f[s][5] = decode_dev<ST>(plane_half(m.b[P][1], s));
            f[s][6] = decode_dev<ST>(plane_half(m.b[P][2], s));
        }
        m.a[0] = w[0];
        m.a[1] = from_left(w[1]);      // e = ( 1, 0)
        m.a[2] = from_right(w[3]);     // e = (-1, 0)
        m.b[P][0] = w[2];              // e = ( 0, 1)
        m.b[P][1] = from_left(w[5]);   // e = ( 1, 1)
        m.b[P][2] = from_right(w[6]);  // e = (-1, 1)
        if (!G || j >= 2 * K) {
            uint16_t o2[2][9];
            collide_site<ST, V, true>(p, f, o2, kShear<V> ? wrap_mod(q - 1, ny) : 0);
            march_levels_pk<ST, V, TS, K + 1, P, RM, G, BIG>(p, o2, c, j, q - 1, ny, out, pitch_b, col_b,
                                                          store_lane, nt, msteps);
        }
    }
}

// One wave's strip of a marching launch: columns x0 - (TS-1) .. x0 + 64 -
// TS (the lanes), result columns x0 .. x0 + 63 - 2(TS-1) below nx, rows y0 ..
// y0 + rows - 1; buffers below 4 GiB.
struct StripW {
    __amdgpu_buffer_rsrc_t src, dst;
    int nx, ny;
    uint32_t pitch_b, pstride_b;
    int x0, y0, rows;
    bool nt;
    // BIG (a buffer of 4 GiB or more): base pointers, plane stride and
    // plane bytes, a descriptor per plane
    const char *src_p;
    char *dst_p;
    uint64_t pstride_64;
    uint32_t plane_b;
};

// TS steps (or, with RM, m <= TS steps) on one strip.
template <int ST, int V, int TS, bool RM = false, bool BIG = false>
__device__ __forceinline__ void stepW_strip(const StripW &sw, const Params<typename Traits<ST>::C> &p, int lane,
                                            int m = TS) {
    using T = typename Traits<ST>::T;
    using C = typename Traits<ST>::C;
    constexpr int NS = NSpecies<V>::value;
    constexpr int H = TS - 1;
    constexpr int U = 64 - 2 * H;
    constexpr uint32_t B = sizeof(T);
    const int nx = sw.nx, ny = sw.ny;
    const int x0 = sw.x0, y0 = sw.y0, rows = sw.rows;
    const int xc = x0 - H + lane;   // this lane's column, before the periodic wrap
    const uint32_t cx[3] = {(uint32_t)wrap_mod(xc - 1, nx) * B, (uint32_t)wrap_mod(xc, nx) * B,
                            (uint32_t)wrap_mod(xc + 1, nx) * B};
    const bool store_lane = lane >= H && lane < H + U && xc < nx;
    // the byte column the lane stores at (kMarchStoreAll: out of range for a halo lane)
    const uint32_t col_out = kMarchStoreAll<ST> && !store_lane ? 0xffffffffu : cx[1];
    const __amdgpu_buffer_rsrc_t src = sw.src;
    const uint32_t pitch_b = sw.pitch_b, pstride_b = sw.pstride_b;
    const bool nt = sw.nt;
    MarchOut out;
    out.dst = sw.dst;
    out.pstride_b = pstride_b;
    out.dst_p = sw.dst_p;
    out.pstride_64 = sw.pstride_64;
    out.plane_b = sw.plane_b;
    const int iters = RM ? rows + H + m - 1 : rows + 2 * H;
    // two species in a 16-bit form: packed carries (march_levels_pk)
    constexpr bool PK = kShifted<ST> && NS == 2;
    std::conditional_t<PK, MarchCarryPk, MarchCarry<T, NS>> c[TS - 1];
    // the source values of level 1 for iteration j: plane i at row r - e_iy,
    // column x - e_ix (r = y0 - h + j), loaded two iterations ahead into
    // raw[j & 1] (about two iterations of arithmetic hide the memory latency)
    T raw[2][NS][9];
    auto load_row = [&](auto parity, int r) {
        constexpr int P = decltype(parity)::value;
        const uint32_t ry[3] = {(uint32_t)wrap_mod(r - 1, ny) * pitch_b, (uint32_t)wrap_mod(r, ny) * pitch_b,
                                (uint32_t)wrap_mod(r + 1, ny) * pitch_b};
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if constexpr (BIG)
                    raw[P][s][i] = buf_load<T>(buffer_rsrc(sw.src_p + (uint64_t)(s * 9 + i) * sw.pstride_64, sw.plane_b),
                                               cx[1 - kEx[i]], ry[1 - kEy[i]]);
                else
                    raw[P][s][i] = buf_load<T>(src, cx[1 - kEx[i]], (uint32_t)(s * 9 + i) * pstride_b + ry[1 - kEy[i]]);
            }
    };
    // one iteration of parity P: level 1 at row r = y0 - h + j from the
    // prefetched values, then the values of iteration j + 2 requested, then
    // the levels above (level k from iteration 2(k-1) on; with guarded =
    // false all of them, without testing).
    auto iteration = [&](auto parity, auto guarded, int j) {
        constexpr int P = decltype(parity)::value;
        constexpr bool G = decltype(guarded)::value;
        const int r = y0 - H + j;
        C f[NS][9];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int i = 0; i < 9; ++i) f[s][i] = decode_dev<ST>(raw[P][s][i]);
        T o[NS][9];
        collide_site<ST, V, PK>(p, f, o, kShear<V> ? wrap_mod(r, ny) : 0);
        // requested once level 1 has consumed raw[P], unconditionally (rows
        // wrap, so the two past the segment's end are valid rows): a load
        // under a branch leaves the wait counter unsure at the join, which
        // then waits for every access in flight, the prefetch included
        __builtin_amdgcn_sched_barrier(0);
        load_row(parity, r + 2);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (PK)
            march_levels_pk<ST, V, TS, 1, P, RM, G, BIG>(p, o, c, j, r, ny, out, pitch_b, col_out, store_lane, nt,
                                                         m);
        else
            march_levels<ST, V, TS, 1, P, RM, G, BIG>(p, o, c, j, r, ny, out, pitch_b, col_out, store_lane, nt, m);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using Guarded = std::true_type;
    using Full = std::false_type;
    load_row(I0{}, y0 - H);
    load_row(I1{}, y0 - H + 1);
    int j = 0;
    if constexpr (!RM) {
        // iters = rows + 2h > 2h: the first 2h iterations fill the pipeline,
        // every later one runs all levels
        for (; j < 2 * H; j += 2) {
            iteration(I0{}, Guarded{}, j);
            iteration(I1{}, Guarded{}, j + 1);
        }
        // FP64, once per segment: every access done (vmcnt 0, lgkmcnt 0), so
        // the loop below is entered with nothing in flight and the waits the
        // compiler places in it are set by the loop's own accesses alone, not
        // by the fewer ones in flight on the way in
        if constexpr (kMarchStoreAll<ST>) __builtin_amdgcn_s_waitcnt(0x0070);
        for (; j + 1 < iters; j += 2) {
            iteration(I0{}, Full{}, j);
            iteration(I1{}, Full{}, j + 1);
        }
        if (j < iters) iteration(I0{}, Full{}, j);
    } else {
        for (; j + 1 < iters; j += 2) {
            iteration(I0{}, Guarded{}, j);
            iteration(I1{}, Guarded{}, j + 1);
        }
        if (j < iters) iteration(I0{}, Guarded{}, j);
    }
}

// TS steps per launch (2 .. 12; FP64 2 .. 8) on marching wave strips: g.tw =
// 64 - 2(TS-1) result columns per strip, g.th rows per segment, g.ntx strips
// across and g.nty segments down, one wave each (g.ntiles of them); buffers
// below 4 GiB, or with BIG of 4 GiB or more (g.bytes 0), each plane below it
// (g.plane_bytes), addressed plane by plane; a BIG kernel also runs launches
// of g.steps < TS steps on the strips of TS.
template <int ST, int V, int TS, bool BIG = false>
__global__ __launch_bounds__(256) void k_stepW(GridT g, Params<typename Traits<ST>::C> p) {
    using T = typename Traits<ST>::T;
    constexpr int U = 64 - 2 * (TS - 1);
    constexpr uint32_t B = sizeof(T);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int b = g.xcd_order ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int w = b * (int)(blockDim.x >> 6) + wave;
    if (w >= (int)g.ntiles) return;
    const int sy = w / g.ntx, sx = w - sy * g.ntx;
    StripW sw;
    sw.src = buffer_rsrc(g.src, g.bytes);
    sw.dst = buffer_rsrc(g.dst, g.bytes);
    sw.nx = g.nx;
    sw.ny = g.ny;
    sw.pitch_b = (uint32_t)g.pitch * B;
    sw.pstride_b = (uint32_t)g.pstride * B;
    sw.x0 = sx * U;
    sw.y0 = sy * g.th;
    sw.rows = min(g.th, g.ny - sw.y0);
    sw.nt = g.nt_store != 0;
    sw.src_p = static_cast<const char *>(g.src);
    sw.dst_p = static_cast<char *>(g.dst);
    sw.pstride_64 = (uint64_t)g.pstride * B;
    sw.plane_b = g.plane_bytes;
    if constexpr (BIG) {
        // g.steps = m <= TS: a shorter launch stores at level m (the strip's
        // halo, laid out for TS steps, covers m)
        if (g.steps == TS) stepW_strip<ST, V, TS, false, true>(sw, p, lane);
        else stepW_strip<ST, V, TS, true, true>(sw, p, lane, g.steps);
    } else {
        stepW_strip<ST, V, TS>(sw, p, lane);
    }
}

}  // namespace lbrd
