/* Driver for the sanitizer run of the oracle (test infrastructure): calls
 * every oracle entry point on tiny and ragged lattices, every reaction kind,
 * both storage emulations and with a uniform equilibrium velocity or a
 * velocity field, in the FP64 and FP32 builds.  Built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitizers.py; exits 0 when every call succeeds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_tables_f64(double *w, int *ex, int *ey);
void orc_eq_coefs_f64(const double *u, double *c);
void orc_init_f64(int n, int nx, int ny, const double *rho0, const double *u, int u_field, double *f);
int orc_run_f64(int n, int nx, int ny, const double *tau, int kind, const double *params, int quant,
                const double *rho_ref, const double *u, int u_field, double *f, double *work, int64_t nsteps);
void orc_moments_f64(int n, int nx, int ny, const double *f, double *rho);
void orc_init_f32(int n, int nx, int ny, const double *rho0, const double *u, int u_field, float *f);
int orc_run_f32(int n, int nx, int ny, const double *tau, int kind, const double *params, int quant,
                const double *rho_ref, const double *u, int u_field, float *f, float *work, int64_t nsteps);
void orc_encode_f32(int n, int nx, int ny, int quant, const double *rho_ref, const double *u, float *f);
void orc_moments_f32(int n, int nx, int ny, const float *f, double *rho);
void orc_quantise_f32(int quant, const float *in, float *out, int64_t n);

int main(void)
{
    const int shapes[][2] = {{1, 1}, {1, 3}, {3, 3}, {2, 5}, {7, 4}};
    const double tau[4] = {0.7, 1.2, 0.9, 0.6};
    const double rho_ref[4] = {1.0, 0.0, 0.5, 0.25};
    const double u[2] = {0.1, -0.07};
    double w[9], c[9];
    int ex[9], ey[9];
    orc_tables_f64(w, ex, ey);
    orc_eq_coefs_f64(u, c);
    orc_eq_coefs_f64(NULL, c);
    int failures = 0;
    for (size_t k = 0; k < sizeof shapes / sizeof shapes[0]; ++k) {
        const int ny = shapes[k][0], nx = shapes[k][1];
        for (int n = 1; n <= 4; ++n)
            for (int kind = 0; kind <= 2; ++kind) {
                if (kind == 2 && n != 2) continue;
                const size_t sites = (size_t)nx * ny, pops = (size_t)n * 9 * sites;
                double *rho0 = malloc(sizeof(double) * n * sites), *rho = malloc(sizeof(double) * n * sites);
                double *f = malloc(sizeof(double) * pops), *wk = malloc(sizeof(double) * pops);
                double *field = malloc(sizeof(double) * 2 * sites);
                for (size_t j = 0; j < sites; ++j) {
                    field[2 * j] = 0.05 * (double)(j % 3) - 0.05;
                    field[2 * j + 1] = 0.02;
                }
                float *g = malloc(sizeof(float) * pops), *gw = malloc(sizeof(float) * pops);
                double params[4 * 4 + 4];
                for (int q = 0; q < 20; ++q) params[q] = 0.001 * (q % 5) - 0.002;
                if (kind == 2) {
                    params[0] = 0.04;
                    params[1] = 0.06;
                }
                for (size_t j = 0; j < (size_t)n * sites; ++j) rho0[j] = 0.3 + 0.01 * (double)(j % 7);
                for (int adv = 0; adv < 3; ++adv) {
                    /* 0: no velocity; 1: uniform; 2: a field given site by site */
                    const double *uu = adv == 0 ? NULL : (adv == 1 ? u : field);
                    const int uf = adv == 2;
                    orc_init_f64(n, nx, ny, rho0, uu, uf, f);
                    failures += orc_run_f64(n, nx, ny, tau, kind, params, 0, rho_ref, uu, uf, f, wk, 5) != 0;
                    orc_moments_f64(n, nx, ny, f, rho);
                    for (int quant = 0; quant <= (uf ? 0 : 2); ++quant) {
                        orc_init_f32(n, nx, ny, rho0, uu, uf, g);
                        if (quant) orc_encode_f32(n, nx, ny, quant, rho_ref, uu, g);
                        failures += orc_run_f32(n, nx, ny, tau, kind, params, quant, rho_ref, uu, uf, g, gw, 5) != 0;
                        orc_moments_f32(n, nx, ny, g, rho);
                        orc_quantise_f32(quant, g, gw, (int64_t)pops);
                    }
                }
                failures += orc_run_f64(0, nx, ny, tau, kind, params, 0, rho_ref, NULL, 0, f, wk, 1) != -1;
                free(field);
                free(rho0);
                free(rho);
                free(f);
                free(wk);
                free(g);
                free(gw);
            }
    }
    printf("oracle sanitizer driver: %d failures\n", failures);
    return failures != 0;
}
