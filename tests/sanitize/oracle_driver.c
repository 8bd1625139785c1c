/* Drives the FP64 oracle through every command and accessor on small
 * lattices, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py).  Test infrastructure: it calls the oracle's
 * C functions and checks only that they accept valid input and return. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc orc;
orc *orc_create(int nx, int ny);
void orc_destroy(orc *o);
int orc_fluids(orc *o, int ncomp, double tau0, double tau1, double alpha0, double alpha1);
int orc_aveforce(orc *o, int comp, int mode, double value);
int orc_aveacceleration(orc *o, int comp, int mode, double value);
int orc_interforce(orc *o, double G);
int orc_adhesiveforce(orc *o, int comp, double G);
int orc_interforce_psi(orc *o, double G, double psi0, double rho0);
int orc_adhesiveforce_psi(orc *o, double G, double psi0, double rho0);
int orc_momentum_opening(orc *o, int wall, int lo, int hi, int comp, int outlet, int style, double v, double rho);
int orc_solute(orc *o, int q, double tau_s);
int orc_intersolute(orc *o, double G, double psi0, double C0);
int orc_solute_opening_range(orc *o, int wall, int lo, int hi, int outlet, int style, double value, double v);
int orc_surface_reaction(orc *o, double kr, double Cs, double b0, double bmax, uint64_t seed);
int orc_obstacle_circle(orc *o, int xc, int yc, double r);
int orc_obstacle_rect(orc *o, int x0, int x1, int y0, int y1);
int orc_boundary_style(orc *o, int style, double R);
int orc_obstacle_style(orc *o, int comp, double R);
int orc_set_fields(orc *o, int comp, const double *rho, const double *ux, const double *uy);
int orc_set_concentration(orc *o, const double *C, const double *ux, const double *uy);
int orc_step(orc *o, long nsteps);
int orc_moments(orc *o, int comp, double *rho, double *ux, double *uy);
int orc_solute_state(orc *o, double *C, double *b);
int orc_budgets(orc *o, double *out);
int orc_get_f(orc *o, int comp, double *out);
int orc_set_f(orc *o, int comp, const double *in);
int orc_get_g(orc *o, double *out);
int orc_set_g(orc *o, const double *in);
int orc_get_mask(orc *o, uint8_t *out);
int orc_set_mask(orc *o, const uint8_t *in);
int orc_get_b(orc *o, double *out);
int orc_get_bdec(orc *o, double *out);
int orc_set_b(orc *o, const double *in);
int orc_forces(orc *o, int comp, double *Fx, double *Fy);
int orc_set_threads(int n);

static int fails = 0;
#define OK(call) do { if ((call) != 0) { printf("FAILED: %s\n", #call); ++fails; } } while (0)

static void readouts(orc *o, int n, int ncomp) {
    double *a = malloc(sizeof(double) * 9 * n), *b = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n);
    uint8_t *m = malloc(n);
    double bud[16];
    for (int k = -1; k < ncomp; ++k) OK(orc_moments(o, k, a, b, c));
    OK(orc_solute_state(o, a, b));
    OK(orc_budgets(o, bud));
    for (int k = 0; k < ncomp; ++k) {
        OK(orc_get_f(o, k, a));
        OK(orc_set_f(o, k, a));
        OK(orc_forces(o, k, b, c));
    }
    OK(orc_get_g(o, a));
    OK(orc_set_g(o, a));
    OK(orc_get_mask(o, m));
    OK(orc_set_mask(o, m));
    OK(orc_get_b(o, b));
    OK(orc_get_bdec(o, c));
    OK(orc_set_b(o, b));
    free(a); free(b); free(c); free(m);
}

int main(void) {
    orc_set_threads(2);
    /* two fluids, Shan-Chen, adhesion, hybrid solids, momentum openings,
     * D2Q9 solute with openings of every style on every wall, reaction,
     * growth and intersolute */
    const int nx = 41, ny = 37, n = nx * ny;
    double *r0 = malloc(sizeof(double) * n), *r1 = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * n),
           *C = malloc(sizeof(double) * n);
    for (int k = 0; k < n; ++k) {
        r0[k] = 0.5 + 0.3 * ((k * 37) % 11) / 11.0;
        r1[k] = 0.9 - 0.3 * ((k * 17) % 7) / 7.0;
        u[k] = 0.01 * ((k % 5) - 2);
        C[k] = 0.2 + 0.1 * ((k * 13) % 5) / 5.0;
    }
    orc *o = orc_create(nx, ny);
    OK(orc_fluids(o, 2, 0.9, 1.1, 4.0 / 9.0, 0.3));
    OK(orc_aveforce(o, 0, 5, 1e-5));
    OK(orc_aveacceleration(o, 1, 1, 2e-5));
    OK(orc_interforce(o, 0.9));
    OK(orc_adhesiveforce(o, 0, 0.3));
    OK(orc_adhesiveforce(o, 1, -0.3));
    OK(orc_boundary_style(o, 3, 0.0));
    OK(orc_obstacle_style(o, 0, 1.0));
    OK(orc_obstacle_style(o, 1, 0.4));
    OK(orc_obstacle_circle(o, 12, 20, 4.5));
    OK(orc_obstacle_style(o, 0, 0.0));
    OK(orc_obstacle_rect(o, 25, 30, 5, 9));
    OK(orc_obstacle_circle(o, 0, 0, 3.0));
    OK(orc_momentum_opening(o, 2, 3, 20, 0, 0, 2, 0.02, 1.0));
    OK(orc_momentum_opening(o, 3, 3, 20, 0, 1, 4, 0.0, 1.0));
    OK(orc_momentum_opening(o, 2, 22, 38, 1, 0, 3, 0.0, 0.95));
    OK(orc_set_fields(o, 0, r0, u, u));
    OK(orc_set_fields(o, 1, r1, u, u));
    OK(orc_solute(o, 9, 0.8));
    OK(orc_solute_opening_range(o, 0, 2, 30, 0, 3, 1.0, 0.05));
    OK(orc_solute_opening_range(o, 1, 0, 35, 1, 2, 0.0, 0.0));
    OK(orc_solute_opening_range(o, 2, 24, 38, 0, 1, 0.7, 0.0));
    OK(orc_solute_opening_range(o, 3, 24, 38, 1, 3, 0.1, 0.3));
    OK(orc_surface_reaction(o, 0.05, 0.0, 0.01, 0.2, 7));
    OK(orc_intersolute(o, -5e-3, 1.0, 5e-3));
    OK(orc_set_concentration(o, C, u, u));
    OK(orc_step(o, 60));
    readouts(o, n, 2);
    OK(orc_step(o, 3));
    orc_destroy(o);

    /* one fluid with the psi forms, D2Q4 solute, noslip */
    o = orc_create(nx, ny);
    OK(orc_fluids(o, 1, 1.0, 1.0, 4.0 / 9.0, 4.0 / 9.0));
    OK(orc_interforce_psi(o, -120.0, 4.0, 200.0));
    OK(orc_adhesiveforce_psi(o, -100.0, 4.0, 200.0));
    OK(orc_obstacle_rect(o, 0, nx - 1, 0, 0));
    for (int k = 0; k < n; ++k) r0[k] = 200.0 + ((k * 7) % 10) / 10.0;
    OK(orc_set_fields(o, 0, r0, u, u));
    OK(orc_solute(o, 4, 1.0));
    OK(orc_surface_reaction(o, 0.02, 0.5, 0.5, 1.0, 3));
    OK(orc_set_concentration(o, C, u, u));
    OK(orc_step(o, 40));
    readouts(o, n, 1);
    orc_destroy(o);
    free(r0); free(r1); free(u); free(C);
    printf(fails ? "failures: %d\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
