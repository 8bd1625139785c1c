/* Drives the host side of the C ABI (include/lb2d.h) without a GPU, for a
 * build of the host runtime with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py): every command with
 * valid arguments and with the mistakes the library must reject (order
 * rules, bad values, calls before bind), workspace sizes of every storage
 * format with every feature, a bind refused on a host pointer, and batches
 * refused before finalize.  Checks the documented status codes. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lb2d.h"

static int fails = 0;
#define EXPECT(call, code)                                                     \
    do {                                                                       \
        int rc_ = (call);                                                      \
        if (rc_ != (code)) {                                                   \
            printf("FAILED: %s returned %d, expected %d\n", #call, rc_, code); \
            ++fails;                                                           \
        }                                                                      \
    } while (0)

int main(void) {
    const int nx = 45, ny = 38, n = nx * ny;
    double *rho = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * n), *C = malloc(sizeof(double) * n);
    unsigned char *m = calloc(n, 1);
    for (int k = 0; k < n; ++k) {
        rho[k] = 0.8 + 0.01 * (k % 7);
        u[k] = 0.001 * (k % 3);
        C[k] = 0.1;
    }
    m[5 * nx + 7] = 1;
    const double nan = NAN;
    size_t bytes = 0;
    double out[LB2D_NBUDGET], field[3];

    /* order rules and argument checks */
    lb2d_ctx *c = NULL;
    EXPECT(lb2d_create(&c, 0), LB2D_OK);
    EXPECT(lb2d_fluids(c, 1.0, 1.0, nan, nan), LB2D_E_ORDER);
    EXPECT(lb2d_lattice(c, "d2q7", nx, ny, 1.0), LB2D_E_UNSUPPORTED);
    EXPECT(lb2d_lattice(c, "d2q9", 2, ny, 1.0), LB2D_E_INVAL);
    EXPECT(lb2d_lattice(c, "d2q9", nx, ny, 0.5), LB2D_E_INVAL);
    EXPECT(lb2d_lattice(c, "d2q9", nx, ny, 1.0), LB2D_OK);
    EXPECT(lb2d_obstacle_circle(c, 5, 5, 2.0), LB2D_E_ORDER);
    EXPECT(lb2d_solute_opening(c, "xlo", "dirichlet", 1.0), LB2D_E_ORDER);
    EXPECT(lb2d_iteration(c, 5), LB2D_E_STATE);
    EXPECT(lb2d_prepare(c, 5), LB2D_E_STATE);
    EXPECT(lb2d_moments(c, 0, field, field, field), LB2D_E_STATE);
    EXPECT(lb2d_budgets(c, out), LB2D_E_STATE);
    EXPECT(lb2d_budgets_noalloc(c, out), LB2D_E_STATE);
    EXPECT(lb2d_checkpoint_bytes(c, &bytes), LB2D_E_STATE);
    EXPECT(lb2d_checkpoint_save(c, field, sizeof(field)), LB2D_E_STATE);
    EXPECT(lb2d_checkpoint_load(c, field, sizeof(field)), LB2D_E_STATE);
    EXPECT(lb2d_fluids(c, 0.9, 1.1, nan, 0.3), LB2D_OK);
    EXPECT(lb2d_aveforce(c, 5, 1e-5, 0), LB2D_OK);
    EXPECT(lb2d_aveacceleration(c, 1, 2e-5, 1), LB2D_OK);
    EXPECT(lb2d_aveacceleration(c, 9, 2e-5, 1), LB2D_E_INVAL);
    EXPECT(lb2d_interforce(c, 0.9, nan, nan), LB2D_OK);
    EXPECT(lb2d_adhesiveforce(c, 0.3, nan, nan, 0), LB2D_OK);
    EXPECT(lb2d_adhesiveforce(c, -0.3, nan, nan, 1), LB2D_OK);
    EXPECT(lb2d_solute(c, 0.8, 5), LB2D_E_INVAL);
    EXPECT(lb2d_solute(c, 0.8, 9), LB2D_OK);
    EXPECT(lb2d_solute_opening_range(c, "xlo", 2, 30, "inlet", "flux", 1.0, 0.05), LB2D_OK);
    EXPECT(lb2d_solute_opening_range(c, "xhi", 0, ny - 1, "outlet", "adiabatic", 0.0, 0.0), LB2D_OK);
    EXPECT(lb2d_solute_opening_range(c, "ylo", 4, 20, "inlet", "dirichlet", 0.7, 0.0), LB2D_OK);
    EXPECT(lb2d_solute_opening_range(c, "yhi", 10, 30, "outlet", "flux", 0.1, 0.3), LB2D_OK);
    EXPECT(lb2d_solute_opening_range(c, "zlo", 10, 30, "outlet", "flux", 0.1, 0.3), LB2D_E_INVAL);
    EXPECT(lb2d_momentum_opening(c, "ylo", 22, 40, 0, "inlet", "poiseuille", 0.02, 1.0), LB2D_OK);
    EXPECT(lb2d_momentum_opening(c, "yhi", 22, 40, 0, "outlet", "gradient", 0.0, 1.0), LB2D_OK);
    EXPECT(lb2d_boundary_style(c, "hybrid", 0.0), LB2D_OK);
    EXPECT(lb2d_obstacle_style(c, 0, "slip", 0.0), LB2D_OK);
    EXPECT(lb2d_obstacle_style(c, 1, "mixed", 0.4), LB2D_OK);
    EXPECT(lb2d_obstacle_style(c, 2, "mixed", 0.4), LB2D_E_INVAL);
    EXPECT(lb2d_obstacle_circle(c, 12, 20, 4.5), LB2D_OK);
    EXPECT(lb2d_obstacle_rect(c, 25, 30, 5, 9), LB2D_OK);
    EXPECT(lb2d_obstacle_rect(c, 25, nx, 5, 9), LB2D_E_INVAL);
    EXPECT(lb2d_obstacle_mask(c, m), LB2D_OK);
    EXPECT(lb2d_surface_reaction(c, 0.05, 0.0, "growth", 0.01, 0.2, 7), LB2D_OK);
    EXPECT(lb2d_intersolute(c, -5e-3, 1.0, 5e-3), LB2D_OK);
    EXPECT(lb2d_set_fields(c, 0, rho, u, u), LB2D_OK);
    EXPECT(lb2d_set_fields(c, 1, rho, NULL, NULL), LB2D_OK);
    rho[3] = -1.0;
    EXPECT(lb2d_set_fields(c, 1, rho, NULL, NULL), LB2D_E_INVAL);
    rho[3] = 0.8;
    EXPECT(lb2d_set_concentration(c, C, u, NULL), LB2D_OK);
    EXPECT(lb2d_rounding(c, "stochastic", 5), LB2D_OK);
    EXPECT(lb2d_rounding(c, "sideways", 5), LB2D_E_INVAL);
    for (int st = LB2D_F64; st <= LB2D_BF16; ++st) {
        EXPECT(lb2d_workspace_bytes(c, st, &bytes), (st == LB2D_F16 || st == LB2D_BF16) ? LB2D_OK : LB2D_E_UNSUPPORTED);
    }
    EXPECT(lb2d_rounding(c, "nearest", 0), LB2D_OK);
    size_t prev = 0;
    for (int st = LB2D_BF16; st >= LB2D_F64; --st) {
        EXPECT(lb2d_workspace_bytes(c, st, &bytes), LB2D_OK);
        if ((st == LB2D_F32 || st == LB2D_F64) && bytes <= prev) {
            printf("FAILED: workspace of storage %d not larger\n", st);
            ++fails;
        }
        prev = bytes;
    }
    EXPECT(lb2d_workspace_bytes(c, 7, &bytes), LB2D_E_INVAL);
    /* a workspace too small, and a host pointer, which is not device memory */
    EXPECT(lb2d_workspace_bytes(c, LB2D_F32, &bytes), LB2D_OK);
    char *host = malloc(bytes + 256);
    char *aligned = host + (256 - ((size_t)host % 256)) % 256;
    EXPECT(lb2d_bind(c, aligned, 4096, NULL), LB2D_E_SIZE);
    {
        /* LB2D_E_INVAL on a machine with a GPU; LB2D_E_HIP without one */
        const int rc = lb2d_bind(c, aligned, bytes, NULL);
        if (rc != LB2D_E_INVAL && rc != LB2D_E_HIP) {
            printf("FAILED: bind on a host pointer returned %d\n", rc);
            ++fails;
        }
    }
    free(host);
    EXPECT(lb2d_iteration(c, 1), LB2D_E_STATE);
    if (strlen(lb2d_last_error(c)) == 0) {
        printf("FAILED: no message\n");
        ++fails;
    }

    /* one fluid with the psi forms; a D2Q4 solute */
    lb2d_ctx *p = NULL;
    EXPECT(lb2d_create(&p, 0), LB2D_OK);
    EXPECT(lb2d_lattice(p, "d2q9", nx, ny, 1.0), LB2D_OK);
    EXPECT(lb2d_interforce(p, -120.0, 4.0, 200.0), LB2D_OK);
    EXPECT(lb2d_adhesiveforce(p, -100.0, 4.0, 200.0, 0), LB2D_OK);
    EXPECT(lb2d_interforce(p, 0.9, nan, nan), LB2D_E_INVAL);
    EXPECT(lb2d_solute(p, 1.0, 4), LB2D_OK);
    EXPECT(lb2d_workspace_bytes(p, LB2D_F32, &bytes), LB2D_OK);

    /* batches hold bound lattices only */
    lb2d_batch *b = NULL;
    EXPECT(lb2d_batch_create(&b, 0), LB2D_OK);
    EXPECT(lb2d_batch_add(b, p), LB2D_E_STATE);
    EXPECT(lb2d_batch_workspace_bytes(b, &bytes), LB2D_E_STATE);
    EXPECT(lb2d_batch_iteration(b, 1), LB2D_E_STATE);
    EXPECT(lb2d_batch_destroy(b), LB2D_OK);

    EXPECT(lb2d_destroy(p), LB2D_OK);
    EXPECT(lb2d_destroy(c), LB2D_OK);
    EXPECT(lb2d_destroy(NULL), LB2D_E_INVAL);
    free(rho); free(u); free(C); free(m);
    printf(fails ? "failures: %d\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
