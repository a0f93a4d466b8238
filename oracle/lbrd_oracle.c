/*
 * Oracle: plain, slow, obviously correct CPU implementation of the reacting-
 * species D2Q9 lattice Boltzmann update of Ayodele, Varnik & Raabe,
 * "Lattice Boltzmann study of pattern formation in reaction-diffusion systems".
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this code.  It shares nothing with the
 * HIP library (no headers, tables, helpers or generators); neither side
 * includes or links the other.
 *
 * The file is compiled twice: with REAL=double (symbols *_f64; the oracle
 * proper) and with REAL=float (symbols *_f32; used only to measure the FP32
 * rounding floor and to emulate the 16-bit shifted storage forms).
 *
 * Layout of a population field: f[s][i][y][x], dense, x fastest,
 * s = species 0..N-1, i = velocity 0..8.  The stored state at time t is the
 * pre-collision f_{i,s}(x, t) of the update equation (Section II.A, the
 * second Eq. "relax"; Appendix, Eq. "app1").
 *
 * The update is written in "push" form, exactly as the paper writes it:
 *     f_{i,s}(x + e_i, t + 1) = f_{i,s}(x, t)
 *                               + (f^eq_{i,s}(x,t) - f_{i,s}(x,t)) / tau_s
 *                               + w_i R_s(rho_1..rho_N)(x, t)
 * with rho_s = sum_i f_{i,s} (Section II.A, the sentence after Eq. "relax"),
 * f^eq_{i,s} = w_i rho_s (Eq. "equili"), periodic wrap in x and y
 * (Section II.B and Section IV), lattice units dx = dt = 1.  With a
 * prescribed velocity u (uniform, or a field given site by site) the
 * equilibrium is the low-Mach Maxwellian of Eq. "Maxwellian",
 * f^eq_{i,s}(x) = c_i(u(x)) rho_s(x) (the paper's runs have u = 0, which gives
 * c_i = w_i exactly).
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef REAL
#define REAL double
#endif
#ifndef SFX
#define SFX(name) name##_f64
#endif

/* Reaction kinds. */
#define ORC_REACT_NONE 0
#define ORC_REACT_LINEAR 1      /* R_s = sum_j K[s][j] rho_j + c_s            */
#define ORC_REACT_GRAY_SCOTT 2  /* R_u = -u v^2 + F (1-u), R_v = u v^2 - (F+k) v */

/* Storage emulation for the 16-bit shifted forms (float build only). */
#define ORC_Q_NONE 0
#define ORC_Q_F16 1
#define ORC_Q_BF16 2

#define ORC_MAX_SPECIES 4

/* D2Q9 velocity set (Section II.A, Eq. "Weights"): rest, the four axis
 * directions and the four diagonals.  The paper fixes the sets, not the
 * numbering; this numbering is the oracle's own. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* Weights w_i: 4/9 for the rest velocity, 1/9 for the axes, 1/36 for the
 * diagonals (Eq. "Weights"), each the correctly rounded quotient in REAL. */
static REAL weight(int i)
{
    if (i == 0) return (REAL)4 / (REAL)9;
    if (i <= 4) return (REAL)1 / (REAL)9;
    return (REAL)1 / (REAL)36;
}

/* Equilibrium coefficient of Eq. "Maxwellian" with c_s^2 = 1/3 (Section
 * II.A): f^eq_i = c_i rho with
 *     c_i = w_i [1 + (e_i.u) / c_s^2 + (e_i.u)^2 / (2 c_s^4) - (u.u) / (2 c_s^2)].
 * u = NULL or u = (0, 0) returns w_i itself (Eq. "equili"). */
static REAL eq_coef(int i, const double *u)
{
    const REAL w = weight(i);
    if (!u || (u[0] == 0.0 && u[1] == 0.0)) return w;
    const REAL ux = (REAL)u[0], uy = (REAL)u[1];
    const REAL cs2 = (REAL)1 / (REAL)3;
    const REAL eu = (REAL)EX[i] * ux + (REAL)EY[i] * uy;
    const REAL uu = ux * ux + uy * uy;
    return w * ((REAL)1 + eu / cs2 + eu * eu / ((REAL)2 * cs2 * cs2) - uu / ((REAL)2 * cs2));
}

/* The velocity at site (x, y): u is NULL (no advection), 2 values (one
 * uniform velocity), or, with u_field != 0, a prescribed field of 2 nx ny
 * values laid out [y][x][component]. */
static const double *site_u(const double *u, int u_field, int nx, int x, int y)
{
    if (!u || !u_field) return u;
    return u + 2 * ((size_t)y * nx + x);
}

/* Expose the equilibrium coefficients c_i(u) (for the tests). */
void SFX(orc_eq_coefs)(const double *u, REAL *c)
{
    for (int i = 0; i < 9; ++i) c[i] = eq_coef(i, u);
}

/* Threads the parallel step uses (1 without OpenMP). */
int SFX(orc_threads)(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Expose the tables so the tests can check the lattice isotropy conditions
 * (Appendix, Eq. "app11") on exactly what the oracle uses. */
void SFX(orc_tables)(REAL *w, int *ex, int *ey)
{
    for (int i = 0; i < 9; ++i) {
        w[i] = weight(i);
        ex[i] = EX[i];
        ey[i] = EY[i];
    }
}

static size_t idx(int nx, int ny, int s, int i, int y, int x)
{
    return (((size_t)s * 9 + (size_t)i) * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x;
}

/* Reaction term R_s(rho_1..rho_N).
 *  LINEAR: params = K[N*N] (row-major, K[s*N+j]) then c[N].  Covers the decay
 *          R_A = -kappa rho_A of Section II.B, Eq. "reac_diff3", and the
 *          A -> B pair (R_B = +kappa rho_A).
 *  GRAY_SCOTT: params = {F, k}; species 0 is u (= A/A_0), species 1 is v.
 *          With A_0 = k_1 = 1 the kinetics of Section III, Eqs. "reac_diff10"
 *          and "reac_diff11", read R_u = -u v^2 + F (1 - u) and
 *          R_v = u v^2 - (F + k) v with F = k_f and k = k_2. */
static void reaction(int kind, int n, const double *params, const REAL *rho, REAL *R)
{
    if (kind == ORC_REACT_LINEAR) {
        for (int s = 0; s < n; ++s) {
            REAL acc = 0;
            for (int j = 0; j < n; ++j) acc += (REAL)params[s * n + j] * rho[j];
            R[s] = acc + (REAL)params[n * n + s];
        }
    } else if (kind == ORC_REACT_GRAY_SCOTT) {
        const REAL F = (REAL)params[0], k = (REAL)params[1];
        const REAL u = rho[0], v = rho[1];
        const REAL uvv = u * v * v;
        R[0] = -uvv + F * ((REAL)1 - u);
        R[1] = uvv - (F + k) * v;
    } else {
        for (int s = 0; s < n; ++s) R[s] = 0;
    }
}

/* Round a float to the nearest binary16 value (ties to even), returned as a
 * float.  Written from the IEEE 754 binary16 format: 1 sign bit, 5 exponent
 * bits (bias 15), 10 fraction bits, subnormals below 2^-14. */
static float round_f16(float x)
{
    if (x != x) return x;
    float a = fabsf(x);
    if (a >= 65520.0f) return copysignf(INFINITY, x);   /* rounds past 65504 */
    if (a < 6.103515625e-05f) {                          /* subnormal: step 2^-24 */
        float q = a / 5.9604644775390625e-08f;           /* exact: power of two */
        float r = nearbyintf(q);                         /* default mode: ties to even */
        return copysignf(r * 5.9604644775390625e-08f, x);
    }
    int e;
    frexpf(a, &e);                                       /* a = m 2^e, m in [0.5,1) */
    float ulp = ldexpf(1.0f, e - 11);                    /* 10 fraction bits */
    float r = nearbyintf(a / ulp) * ulp;                 /* a/ulp exact (power-of-two scale) */
    return copysignf(r, x);
}

/* Round a float to the nearest bfloat16 value (ties to even): keep the upper
 * 16 bits of the binary32 encoding after adding the rounding bias. */
static float round_bf16(float x)
{
    if (x != x) return x;
    uint32_t b;
    memcpy(&b, &x, 4);
    uint32_t lsb = (b >> 16) & 1u;
    b = (b + 0x7fffu + lsb) & 0xffff0000u;
    float r;
    memcpy(&r, &b, 4);
    return r;
}

static REAL quantise(int quant, REAL g)
{
    if (quant == ORC_Q_F16) return (REAL)round_f16((float)g);
    if (quant == ORC_Q_BF16) return (REAL)round_bf16((float)g);
    return g;
}

/* Apply the 16-bit rounding to an array (exported so the tests can check the
 * quantisers against an independent reference). */
void SFX(orc_quantise)(int quant, const float *in, float *out, int64_t n)
{
    for (int64_t j = 0; j < n; ++j) out[j] = (float)quantise(quant, (REAL)in[j]);
}

/* Put populations f [N][9][ny][nx] into the 16-bit shifted storage form in
 * place: f <- c_i rho_ref_s + Q(f - c_i rho_ref_s), Q the 16-bit rounding,
 * c_i the equilibrium coefficient (w_i when u = 0). */
void SFX(orc_encode)(int n, int nx, int ny, int quant, const double *rho_ref, const double *u, REAL *f)
{
    for (int s = 0; s < n; ++s)
        for (int i = 0; i < 9; ++i) {
            const REAL shift = eq_coef(i, u) * (REAL)rho_ref[s];
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    REAL *p = &f[idx(nx, ny, s, i, y, x)];
                    *p = shift + quantise(quant, *p - shift);
                }
        }
}

/* Initial populations: local equilibrium f_{i,s}(x,0) = c_i rho_s(x,0)
 * (Eq. "equili", or Eq. "Maxwellian" with velocity u; the paper does not
 * state the initial populations, this is the reading used throughout).
 * rho0 is [N][ny][nx]; u and u_field as for site_u. */
void SFX(orc_init)(int n, int nx, int ny, const double *rho0, const double *u, int u_field, REAL *f)
{
    for (int s = 0; s < n; ++s)
        for (int i = 0; i < 9; ++i)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    f[idx(nx, ny, s, i, y, x)] =
                        eq_coef(i, site_u(u, u_field, nx, x, y)) * (REAL)rho0[((size_t)s * ny + y) * nx + x];
}

/* One time step t -> t+1 of the update equation, push form, f -> fn. */
static void step_once(int n, int nx, int ny, const double *tau, int kind,
                      const double *params, int quant, const double *rho_ref,
                      const double *u, int u_field, const REAL *f, REAL *fn)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        REAL rho[ORC_MAX_SPECIES], R[ORC_MAX_SPECIES];
        for (int x = 0; x < nx; ++x) {
            /* density moment rho_s = sum_i f_{i,s}, ascending i */
            for (int s = 0; s < n; ++s) {
                REAL acc = 0;
                for (int i = 0; i < 9; ++i) acc += f[idx(nx, ny, s, i, y, x)];
                rho[s] = acc;
            }
            reaction(kind, n, params, rho, R);
            const double *us = site_u(u, u_field, nx, x, y);
            for (int s = 0; s < n; ++s) {
                for (int i = 0; i < 9; ++i) {
                    const REAL fi = f[idx(nx, ny, s, i, y, x)];
                    const REAL wi = weight(i);
                    const REAL ci = eq_coef(i, us);
                    REAL g = fi + (ci * rho[s] - fi) / (REAL)tau[s] + wi * R[s];
                    if (quant != ORC_Q_NONE) {
                        /* storage form: g - c_i rho_ref,s rounded to 16 bits */
                        const REAL shift = ci * (REAL)rho_ref[s];
                        g = shift + quantise(quant, g - shift);
                    }
                    int xd = x + EX[i], yd = y + EY[i];
                    if (xd < 0) xd += nx;
                    if (xd >= nx) xd -= nx;
                    if (yd < 0) yd += ny;
                    if (yd >= ny) yd -= ny;
                    fn[idx(nx, ny, s, i, yd, xd)] = g;
                }
            }
        }
    }
}

/* Advance f (in place, [N][9][ny][nx]) by nsteps.  work is a caller buffer
 * of the same size; u and u_field as for site_u (the equilibrium velocity).
 * Returns 0, or -1 on bad arguments. */
int SFX(orc_run)(int n, int nx, int ny, const double *tau, int kind,
                 const double *params, int quant, const double *rho_ref,
                 const double *u, int u_field, REAL *f, REAL *work, int64_t nsteps)
{
    if (n < 1 || n > ORC_MAX_SPECIES || nx < 1 || ny < 1 || nsteps < 0) return -1;
    if (kind == ORC_REACT_GRAY_SCOTT && n != 2) return -1;
    REAL *a = f, *b = work;
    for (int64_t t = 0; t < nsteps; ++t) {
        step_once(n, nx, ny, tau, kind, params, quant, rho_ref, u, u_field, a, b);
        REAL *tmp = a;
        a = b;
        b = tmp;
    }
    if (a != f) memcpy(f, a, sizeof(REAL) * (size_t)n * 9 * (size_t)nx * (size_t)ny);
    return 0;
}

/* rho_s(x) = sum_i f_{i,s}(x), ascending i.  rho is [N][ny][nx] double. */
void SFX(orc_moments)(int n, int nx, int ny, const REAL *f, double *rho)
{
    for (int s = 0; s < n; ++s)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                REAL acc = 0;
                for (int i = 0; i < 9; ++i) acc += f[idx(nx, ny, s, i, y, x)];
                rho[((size_t)s * ny + y) * nx + x] = (double)acc;
            }
}
