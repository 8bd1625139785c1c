/*
 * lb2d_oracle.c -- plain, slow, FP64 CPU oracle for the 2-D lattice Boltzmann
 * method of "Introduction to Perl module lb2d.pm 0.1 for basic Lattice
 * Boltzmann simulations" (D. Sergi, arXiv:1202.0442).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the HIP library against an
 * independent, obviously correct implementation.  It shares no code, header,
 * table or helper with the HIP library.
 *
 * Everything is FP64 and written as plain loops over nodes, in the order the
 * paper gives the steps (Sec. "Model and algorithm", Fig. "algorithm"):
 *   stream (with the obstacle rule applied in the same loop)
 *   -> moments -> forces -> equilibrium + BGK collision
 *   -> solute stream (+ reactive / opening rules) -> solute collision
 *   -> deposit on the solid surface -> surface growth.
 *
 * Readings of points the paper leaves open (each one is listed with its
 * justification in the design notes of the repository):
 *   - nodes are given as counts nx, ny (the paper's lattice(d2q9,Nx,Ny)
 *     has Nx+1, Ny+1 nodes; the caller adds the 1);
 *   - velocity numbering e0=(0,0), e1=(1,0), e2=(0,1), e3=(-1,0), e4=(0,-1),
 *     e5=(1,1), e6=(-1,1), e7=(-1,-1), e8=(1,-1): it is the one for which the
 *     unknowns at an xlo opening are f1,f5,f8 and for which the slip rule of
 *     the boundary_style command sends f5 at (i,j) towards (i+1,j+1);
 *   - body forces enter through the Shan-Chen velocity shift
 *     u_eq = u' + tau F / rho (fluids command, "equilibrium velocity as
 *     explained in Refs.");
 *   - Shan-Chen forces use the densities of the same step, after streaming;
 *     solid neighbours carry zero density (two components) or zero psi (one
 *     component, psi = psi0 exp(-rho0 / rho)) in the cohesion sum;
 *   - the solute lattice is D2Q9 (g_eq = w C (1 + 3 e.u)) or the paper's
 *     D2Q4 (g_eq = C/4 (1 + 2 e.u)); Q is a run parameter;
 *   - the reactive surface rule is applied per link (generalises the D2Q4
 *     rule of the surface_reaction command and App. C to any Q, and reduces
 *     to it exactly for Q = 4);
 *   - growth candidates are the 4 direct fluid neighbours E,N,W,S, picked by
 *     a counter-based SplitMix64 hash (Steele, Lea & Flood, OOPSLA 2014);
 *   - the intersolute force uses the concentrations of the same step after
 *     streaming (as interforce does); psi is 0 on solids, where C <= 0 and
 *     across a wall of a non-periodic solute axis, and the velocity term
 *     tau_s F / C is added only where C > 0.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads used by the row loops (1 without OpenMP). */
int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ---------------------------------------------------------------- lattice */

/* D2Q9 velocities and weights, Eq. (eq): w0 = 4/9, w1..4 = 1/9, w5..8 = 1/36. */
static const int EX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Index of the velocity opposite to i (e_opp = -e_i). */
static int opposite(int i) {
    for (int k = 0; k < 9; ++k)
        if (EX9[k] == -EX9[i] && EY9[k] == -EY9[i]) return k;
    return -1;
}

/* Index of the velocity mirrored in x (ex -> -ex, ey kept). */
static int mirror_x(int i) {
    for (int k = 0; k < 9; ++k)
        if (EX9[k] == -EX9[i] && EY9[k] == EY9[i]) return k;
    return -1;
}

/* Solute lattice: Q = 9 uses all nine D2Q9 velocities with the D2Q9 weights;
 * Q = 4 uses e1..e4 only, each with weight 1/4 (solute command, D2Q4). */
static int solute_has(int q, int i) { return q == 9 ? 1 : (i >= 1 && i <= 4); }
static double solute_w(int q, int i) {
    if (q == 9) return W9[i];
    return (i >= 1 && i <= 4) ? 0.25 : 0.0;
}
/* Squared sound speed of the solute lattice: sum_i w_i e_ix^2. */
static double solute_cs2(int q) { return q == 9 ? 1.0 / 3.0 : 0.5; }
/* Sum of the weights of the links that cross one flat wall (normal along
 * x or y): 1/9 + 2/36 for D2Q9, 1/4 for D2Q4. */
static double solute_wall_w(int q) { return q == 9 ? 1.0 / 6.0 : 0.25; }

/* ------------------------------------------------------------------ state */

typedef struct orc {
    int nx, ny;
    long n;                      /* nx * ny */
    int ncomp;                   /* 1 or 2 fluid components */
    double tau[2], alpha[2];
    double force[2][2];          /* aveforce: summed force vector per comp */
    double accel[2][2];          /* aveacceleration: summed vector per comp */
    int has_inter;
    double G;                    /* interforce strength */
    int has_ads[2];
    double Gads[2];              /* adhesiveforce per component */
    int psi_inter, psi_ads;      /* one component: forces act through
                                    psi(rho) = psi0 exp(-rho0 / rho) */
    double psi0_i, rho0_i;       /* psi of interforce */
    double psi0_a, rho0_a;       /* psi of adhesiveforce */
    int q;                       /* solute lattice: 0 = off, 4 or 9 */
    double tau_s;
    int isol;                    /* intersolute command */
    double G_s, psi0_s, C0_s;    /* its strength and psi = psi0 exp(-C0/C) */
    int nsopen;                  /* solute openings (inlet_solute/outlet_solute) */
    struct {
        int wall;                /* 0 xlo, 1 xhi, 2 ylo, 3 yhi */
        int lo, hi;              /* node range along the wall */
        int outlet;              /* 0 inlet, 1 outlet */
        int style;               /* 1 dirichlet, 2 adiabatic, 3 flux */
        double value;            /* dirichlet: imposed C; flux: C0 */
        double v;                /* flux: velocity of the injected solution */
    } sopen[16];
    int reaction;
    double kr, Cs, b0, bmax;
    uint64_t seed;
    int b_ready;                 /* b initialised to b0 on solids */

    /* momentum openings (inlet_momentum / outlet_momentum) */
    int nopen;
    struct {
        int wall;                /* 0 xlo, 1 xhi, 2 ylo, 3 yhi */
        int lo, hi;              /* node range along the wall */
        int comp;
        int outlet;              /* 0 inlet, 1 outlet */
        int style;               /* 1 poiseuille, 2 uniform, 3 dirichlet, 4 gradient */
        double v, rho;
    } open[16];
    int open_ready;              /* opening nodes set to their initial state */

    double *f[2], *ftmp[2];      /* [9][n] populations, post-collision */
    double *g, *gtmp;            /* [9][n] solute populations */
    uint8_t *mask;               /* 1 = solid */
    double *refl[2];             /* per node and component: share R of a
                                    diagonal mode hitting this solid that
                                    is reflected (0 noslip, 1 slip, R mixed) */
    double style_R[2];           /* R given to the next obstacles */
    double grow_R[2];            /* R of solids made by growth */
    double *b;                   /* deposited mass on solid nodes */
    double *bacc;                /* per-step deposit scratch */
    double *bdec;                /* deposits the growth decisions of the last
                                    step were taken from (after its deposit,
                                    before any reset); a record for tests */
    uint8_t *grow;               /* per-step growth marks */
    double *rho[2], *jx[2], *jy[2], *Fx[2], *Fy[2]; /* per-step scratch */

    long t;                      /* completed steps */
    double removed_rho[2], removed_C, inflow, outflow;
    double consumed_b;           /* deposits reset to zero by growth */
    long grown_nodes;
} orc;

static long idx(const orc *o, int x, int y) { return (long)y * o->nx + x; }
static int wrap(int a, int n) { return ((a % n) + n) % n; }

orc *orc_create(int nx, int ny) {
    if (nx < 1 || ny < 1) return NULL;
    orc *o = (orc *)calloc(1, sizeof(orc));
    o->nx = nx;
    o->ny = ny;
    o->n = (long)nx * ny;
    o->ncomp = 1;
    o->tau[0] = o->tau[1] = 1.0;
    o->alpha[0] = o->alpha[1] = 4.0 / 9.0;
    for (int c = 0; c < 2; ++c) {
        o->refl[c] = (double *)calloc(o->n, sizeof(double));
        o->f[c] = (double *)calloc(9 * o->n, sizeof(double));
        o->ftmp[c] = (double *)calloc(9 * o->n, sizeof(double));
        o->rho[c] = (double *)calloc(o->n, sizeof(double));
        o->jx[c] = (double *)calloc(o->n, sizeof(double));
        o->jy[c] = (double *)calloc(o->n, sizeof(double));
        o->Fx[c] = (double *)calloc(o->n, sizeof(double));
        o->Fy[c] = (double *)calloc(o->n, sizeof(double));
    }
    o->g = (double *)calloc(9 * o->n, sizeof(double));
    o->gtmp = (double *)calloc(9 * o->n, sizeof(double));
    o->mask = (uint8_t *)calloc(o->n, 1);
    o->grow = (uint8_t *)calloc(o->n, 1);
    o->b = (double *)calloc(o->n, sizeof(double));
    o->bacc = (double *)calloc(o->n, sizeof(double));
    o->bdec = (double *)calloc(o->n, sizeof(double));
    return o;
}

void orc_destroy(orc *o) {
    if (!o) return;
    for (int c = 0; c < 2; ++c) {
        free(o->refl[c]);
        free(o->f[c]); free(o->ftmp[c]); free(o->rho[c]); free(o->jx[c]);
        free(o->jy[c]); free(o->Fx[c]); free(o->Fy[c]);
    }
    free(o->g); free(o->gtmp); free(o->mask); free(o->grow); free(o->b);
    free(o->bacc);
    free(o->bdec);
    free(o);
}

/* --------------------------------------------------------------- commands */

/* lattice(d2q9, ., ., tau) for one fluid; fluids(tau1, tau2, a1, a2) for two.
 * alpha = 4/9 gives A_i = 1 and the plain Eq. (eq). */
int orc_fluids(orc *o, int ncomp, double tau0, double tau1, double alpha0,
               double alpha1) {
    if (ncomp < 1 || ncomp > 2 || tau0 <= 0.5 || (ncomp == 2 && tau1 <= 0.5))
        return -1;
    o->ncomp = ncomp;
    o->tau[0] = tau0;
    o->tau[1] = tau1;
    o->alpha[0] = alpha0;
    o->alpha[1] = alpha1;
    return 0;
}

/* aveforce(mode, value, fluid): value * e_mode added to the force; calls with
 * the same or other modes sum component-wise. */
int orc_aveforce(orc *o, int comp, int mode, double value) {
    if (comp < 0 || comp > 1 || mode < 0 || mode > 8) return -1;
    o->force[comp][0] += value * EX9[mode];
    o->force[comp][1] += value * EY9[mode];
    return 0;
}

/* aveacceleration(mode, value, fluid): acceleration added on fluid sites;
 * the force on component c is rho_c times the summed acceleration. */
int orc_aveacceleration(orc *o, int comp, int mode, double value) {
    if (comp < 0 || comp > 1 || mode < 0 || mode > 8) return -1;
    o->accel[comp][0] += value * EX9[mode];
    o->accel[comp][1] += value * EY9[mode];
    return 0;
}

/* interforce(G) in the two-component form. */
int orc_interforce(orc *o, double G) {
    o->has_inter = 1;
    o->G = G;
    return 0;
}

/* interforce(G, psi0, rho0), one component (interforce command):
 * F = -G psi(x) sum_i w_i psi(x + e_i) e_i, psi = psi0 exp(-rho0 / rho),
 * with psi = 0 on solid neighbours (the force acts between fluid sites). */
int orc_interforce_psi(orc *o, double G, double psi0, double rho0) {
    if (o->ncomp != 1 || !(rho0 > 0.0)) return -1;
    o->has_inter = 1;
    o->psi_inter = 1;
    o->G = G;
    o->psi0_i = psi0;
    o->rho0_i = rho0;
    return 0;
}

/* adhesiveforce(G, psi0, rho0), one component (adhesiveforce command):
 * F = -G psi(x) sum_i w_i s(x + e_i) e_i. */
int orc_adhesiveforce_psi(orc *o, double G, double psi0, double rho0) {
    if (o->ncomp != 1 || !(rho0 > 0.0)) return -1;
    o->has_ads[0] = 1;
    o->psi_ads = 1;
    o->Gads[0] = G;
    o->psi0_a = psi0;
    o->rho0_a = rho0;
    return 0;
}

static double psi_of(double psi0, double rho0, double rho) { return psi0 * exp(-rho0 / rho); }

/* adhesiveforce(G_c, fluid) in the two-component form. */
int orc_adhesiveforce(orc *o, int comp, double G) {
    if (comp < 0 || comp > 1) return -1;
    o->has_ads[comp] = 1;
    o->Gads[comp] = G;
    return 0;
}

/* solute(tau_s) on a D2Q9 (q = 9) or D2Q4 (q = 4) lattice. */
int orc_solute(orc *o, int q, double tau_s) {
    if ((q != 4 && q != 9) || tau_s <= 0.5) return -1;
    o->q = q;
    o->tau_s = tau_s;
    return 0;
}

/* inlet_solute / outlet_solute: nodes lo..hi of wall 0 xlo, 1 xhi, 2 ylo,
 * 3 yhi are a solute opening; style 1 dirichlet (value = imposed C),
 * 2 adiabatic, 3 flux (value = C0 of the injected solution, v its
 * velocity).  An opening on a wall makes the solute non-periodic across
 * that axis; nodes of the two walls of the axis outside the openings are
 * then impermeable to the solute (bounce-back).  The fluid stays periodic. */
int orc_solute_opening_range(orc *o, int wall, int lo, int hi, int outlet, int style, double value,
                             double v) {
    if (o->nsopen >= 16 || wall < 0 || wall > 3 || style < 1 || style > 3) return -1;
    int len = wall < 2 ? o->ny : o->nx;
    if (lo < 0 || hi < lo || hi >= len) return -1;
    o->sopen[o->nsopen].wall = wall;
    o->sopen[o->nsopen].lo = lo;
    o->sopen[o->nsopen].hi = hi;
    o->sopen[o->nsopen].outlet = outlet ? 1 : 0;
    o->sopen[o->nsopen].style = style;
    o->sopen[o->nsopen].value = value;
    o->sopen[o->nsopen].v = v;
    o->nsopen++;
    return 0;
}

/* The whole x wall (wall 0 xlo, 1 xhi) as a dirichlet (1) or adiabatic (2)
 * solute opening. */
int orc_solute_opening(orc *o, int wall, int style, double value) {
    if (wall < 0 || wall > 1 || style < 1 || style > 2) return -1;
    return orc_solute_opening_range(o, wall, 0, o->ny - 1, wall, style, value, 0.0);
}

/* surface_reaction(kr, Cs, "growth", b0, bmax) plus the seed of the growth
 * choice. */
int orc_surface_reaction(orc *o, double kr, double Cs, double b0, double bmax,
                         uint64_t seed) {
    o->reaction = 1;
    o->kr = kr;
    o->Cs = Cs;
    o->b0 = b0;
    o->bmax = bmax;
    o->seed = seed;
    o->b_ready = 0;
    return 0;
}

/* obstacle(circle, xc, yc, r): a node is solid when its squared distance to
 * the centre, measured with the minimum image on the periodic box, is at
 * most r^2. */
static void circle_node(orc *o, int x, int y, int xc, int yc, double r) {
    long dx = wrap(x - xc, o->nx), dy = wrap(y - yc, o->ny);
    if (o->nx - dx < dx) dx = o->nx - dx;
    if (o->ny - dy < dy) dy = o->ny - dy;
    double d2 = (double)(dx * dx + dy * dy);
    if (d2 <= r * r) {
        o->mask[idx(o, x, y)] = 1;
        o->refl[0][idx(o, x, y)] = o->style_R[0];
        o->refl[1][idx(o, x, y)] = o->style_R[1];
    }
}

int orc_obstacle_circle(orc *o, int xc, int yc, double r) {
    /* only nodes within the bounding box can be inside; a circle that spans
     * half the box or more is tested against every node */
    int h = (r < (double)(o->nx + o->ny)) ? (int)r + 1 : o->nx + o->ny;
    if (2 * h + 1 >= o->nx || 2 * h + 1 >= o->ny) {
        for (int y = 0; y < o->ny; ++y)
            for (int x = 0; x < o->nx; ++x) circle_node(o, x, y, xc, yc, r);
        return 0;
    }
    for (int dy = -h; dy <= h; ++dy)
        for (int dx = -h; dx <= h; ++dx)
            circle_node(o, wrap(xc + dx, o->nx), wrap(yc + dy, o->ny), xc, yc, r);
    return 0;
}

/* obstacle(rectangle, x0, x1, y0, y1), bounds inclusive. */
int orc_obstacle_rect(orc *o, int x0, int x1, int y0, int y1) {
    if (x0 > x1 || y0 > y1 || x0 < 0 || y0 < 0 || x1 >= o->nx || y1 >= o->ny)
        return -1;
    for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) {
            o->mask[idx(o, x, y)] = 1;
            o->refl[0][idx(o, x, y)] = o->style_R[0];
            o->refl[1][idx(o, x, y)] = o->style_R[1];
        }
    return 0;
}

/* intersolute(G, psi0, C0): adds tau_s F / C to the solvent velocity in
 * the solute equilibrium, F = -G psi(x) sum_{i=1..4} psi(x + e_i) e_i over
 * the four axis neighbours (no weights), psi = psi0 exp(-C0 / C)
 * (intersolute command). */
int orc_intersolute(orc *o, double G, double psi0, double C0) {
    if (!o->q || !(C0 > 0.0)) return -1;
    o->isol = 1;
    o->G_s = G;
    o->psi0_s = psi0;
    o->C0_s = C0;
    return 0;
}

/* boundary_style(style, R): 0 noslip, 1 slip, 2 mixed with reflected
 * share R, 3 hybrid (each obstacle carries its own style, see
 * orc_obstacle_style; solids made by growth are noslip).  Sets the style
 * of the obstacles that follow and of grown solids. */
int orc_boundary_style(orc *o, int style, double R) {
    if (style < 0 || style > 3 || (style == 2 && !(R >= 0.0 && R <= 1.0))) return -1;
    double v = style == 1 ? 1.0 : style == 2 ? R : 0.0;
    for (int c = 0; c < 2; ++c) o->style_R[c] = o->grow_R[c] = v;
    return 0;
}

/* Hybrid style: the style of component comp for the obstacles that follow
 * (obstacle command's extra arguments): R = 0 noslip, 1 slip, else mixed. */
int orc_obstacle_style(orc *o, int comp, double R) {
    if (comp < 0 || comp > 1 || !(R >= 0.0 && R <= 1.0)) return -1;
    o->style_R[comp] = R;
    return 0;
}

/* ------------------------------------------------------------ equilibrium */

/* Equilibrium of the fluids command:
 * f_i = w_i rho [A_i + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u],
 * A_0 = (9/4) alpha, A_i = (9/5)(1 - alpha) for i = 1..8. */
static double feq(int i, double rho, double ux, double uy, double alpha) {
    double A = (i == 0) ? 2.25 * alpha : 1.8 * (1.0 - alpha);
    double eu = EX9[i] * ux + EY9[i] * uy;
    double uu = ux * ux + uy * uy;
    return W9[i] * rho * (A + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

/* Solute equilibrium, linear in u: g_i = w_i C (1 + e.u / cs^2); this is
 * Eq. (ueq) for Q = 4 (w = 1/4, cs^2 = 1/2). */
static double geq(int q, int i, double C, double ux, double uy) {
    double eu = EX9[i] * ux + EY9[i] * uy;
    return solute_w(q, i) * C * (1.0 + eu / solute_cs2(q));
}

double orc_feq(int i, double rho, double ux, double uy, double alpha) {
    return feq(i, rho, ux, uy, alpha);
}

double orc_geq(int q, int i, double C, double ux, double uy) {
    return geq(q, i, C, ux, uy);
}

/* position0 / momentum0: every population set to its equilibrium value. */
int orc_set_fields(orc *o, int comp, const double *rho, const double *ux,
                   const double *uy) {
    if (comp < 0 || comp > 1) return -1;
    o->open_ready = 0;  /* opening nodes are set again before the next use */
    for (long s = 0; s < o->n; ++s)
        for (int i = 0; i < 9; ++i)
            o->f[comp][i * o->n + s] =
                feq(i, rho[s], ux ? ux[s] : 0.0, uy ? uy[s] : 0.0,
                    o->alpha[comp]);
    return 0;
}

/* concentration0: solute populations set to their equilibrium value at the
 * given velocity (NULL = at rest). */
int orc_set_concentration(orc *o, const double *C, const double *ux,
                          const double *uy) {
    if (!o->q) return -1;
    for (long s = 0; s < o->n; ++s)
        for (int i = 0; i < 9; ++i)
            o->g[i * o->n + s] =
                solute_has(o->q, i)
                    ? geq(o->q, i, C[s], ux ? ux[s] : 0.0, uy ? uy[s] : 0.0)
                    : 0.0;
    return 0;
}

/* -------------------------------------------------- momentum openings */

/* inlet/outlet + inlet_momentum/outlet_momentum: nodes lo..hi of a wall of
 * the box carry an opening for component comp.  Styles (inlet_momentum
 * command): poiseuille (v = v_max of the parabolic profile), uniform (v),
 * dirichlet (density rho held), gradient (extrapolation after collision).
 * rho is the density the opening nodes start with. */
int orc_momentum_opening(orc *o, int wall, int lo, int hi, int comp, int outlet, int style, double v,
                         double rho) {
    if (o->nopen >= 16 || wall < 0 || wall > 3 || comp < 0 || comp >= o->ncomp) return -1;
    if (style < 1 || style > 4 || !(rho > 0.0)) return -1;
    int len = wall < 2 ? o->ny : o->nx;
    if (lo < 0 || hi < lo || hi >= len) return -1;
    o->open[o->nopen].wall = wall;
    o->open[o->nopen].lo = lo;
    o->open[o->nopen].hi = hi;
    o->open[o->nopen].comp = comp;
    o->open[o->nopen].outlet = outlet ? 1 : 0;
    o->open[o->nopen].style = style;
    o->open[o->nopen].v = v;
    o->open[o->nopen].rho = rho;
    o->nopen++;
    return 0;
}

/* Inward unit normal (nx_, ny_) of a wall and the node at coordinate k
 * along it. */
static void wall_geom(const orc *o, int wall, int k, int *x, int *y, int *nxw, int *nyw) {
    switch (wall) {
        case 0: *x = 0; *y = k; *nxw = 1; *nyw = 0; break;
        case 1: *x = o->nx - 1; *y = k; *nxw = -1; *nyw = 0; break;
        case 2: *x = k; *y = 0; *nxw = 0; *nyw = 1; break;
        default: *x = k; *y = o->ny - 1; *nxw = 0; *nyw = -1; break;
    }
}

/* Normal velocity u.n (n inward) imposed at coordinate k of a velocity
 * opening: the speed into the domain for an inlet, out of it for an
 * outlet; poiseuille: v(k) = 4 v_max / L^2 [(L/2)^2 - ((2k - lo - hi)/2)^2],
 * L = hi - lo + 1 (inlet_momentum command). */
static double opening_un(int outlet, int style, double v, int lo, int hi, int k) {
    double sp = v;
    if (style == 1) {
        double L = hi - lo + 1.0, h = (2.0 * k - lo - hi) / 2.0;
        sp = 4.0 * v / (L * L) * (L * L / 4.0 - h * h);
    }
    return outlet ? -sp : sp;
}

/* Zou-He closure at an opening node (inlet_momentum command, App. A), for
 * the inward normal n and zero tangential velocity: with T the populations
 * along the wall (e.n = 0) and O those leaving the domain (e.n = -1),
 *   rho (1 - u.n) = sum_T f + 2 sum_O f;
 * the entering populations (e.n = +1) are the opposite ones plus
 *   (2/3) rho u.n  (axial),
 *   -(1/2) (e.t) (f_t - f_-t) + (1/6) rho u.n  (diagonal),
 * t the tangent.  Velocity styles give u.n and yield rho; dirichlet gives
 * rho and yields u.n.  f holds the nine populations of the node. */
static void zou_he(double *f, long n, long s, int nxw, int nyw, int pressure, double given) {
    int txw = nyw != 0 ? 1 : 0, tyw = nxw != 0 ? 1 : 0;  /* tangent */
    double sT = 0.0, sO = 0.0, ftp = 0.0, ftm = 0.0;
    for (int i = 0; i < 9; ++i) {
        int en = EX9[i] * nxw + EY9[i] * nyw, et = EX9[i] * txw + EY9[i] * tyw;
        double v = f[i * n + s];
        if (en == 0) {
            sT += v;
            if (et == 1) ftp = v;
            if (et == -1) ftm = v;
        } else if (en < 0) {
            sO += v;
        }
    }
    double rho, un;
    if (pressure) {
        rho = given;
        un = 1.0 - (sT + 2.0 * sO) / rho;
    } else {
        un = given;
        rho = (sT + 2.0 * sO) / (1.0 - un);
    }
    for (int i = 0; i < 9; ++i) {
        int en = EX9[i] * nxw + EY9[i] * nyw, et = EX9[i] * txw + EY9[i] * tyw;
        if (en != 1) continue;
        double fo = f[opposite(i) * n + s];
        f[i * n + s] = (et == 0) ? fo + 2.0 / 3.0 * rho * un
                                 : fo - 0.5 * et * (ftp - ftm) + 1.0 / 6.0 * rho * un;
    }
}

/* Opening nodes start at equilibrium with the opening's density and
 * velocity (the inlet/outlet commands override earlier settings). */
static void init_openings(orc *o) {
    if (o->open_ready) return;
    o->open_ready = 1;
    for (int k = 0; k < o->nopen; ++k)
        for (int j = o->open[k].lo; j <= o->open[k].hi; ++j) {
            int x, y, nxw, nyw;
            wall_geom(o, o->open[k].wall, j, &x, &y, &nxw, &nyw);
            long s = idx(o, x, y);
            double un = (o->open[k].style <= 2)
                            ? opening_un(o->open[k].outlet, o->open[k].style, o->open[k].v, o->open[k].lo,
                                         o->open[k].hi, j)
                            : 0.0;
            for (int i = 0; i < 9; ++i)
                o->f[o->open[k].comp][i * o->n + s] =
                    o->mask[s] ? 0.0 : feq(i, o->open[k].rho, un * nxw, un * nyw, o->alpha[o->open[k].comp]);
        }
}

/* ---------------------------------------------------- reactive link rule */

/* Reactive half-way link.  g_out is the population that streamed from the
 * fluid node into the wall along the link of direction i (weight w_i).
 * The surface_reaction command imposes D dC/dn = kr (C - Cs); per link the
 * rate is k_i = kr w_i / W (W = weight of one flat wall, so the links of a
 * flat wall add up to kr).  The link concentration and returning population
 *   C_i = (2 g_out + k_i Cs) / (2 w_i + k_i),   g_i = 2 w_i C_i - g_out
 * make the flux into the wall, g_out - g_i, equal to k_i (C_i - Cs).  For
 * Q = 4 (w = 1/4, k_i = kr) this is exactly the rule of the command:
 * C = (2 g_chi + kr Cs) / (kr + 1/2), g_i = -g_chi + C/2.
 * Mass deposits only when the flux is positive ("if Delta b > 0"); a
 * non-positive flux leaves the plain bounce-back.  Returns the deposit. */
double orc_reactive_link(int q, int i, double kr, double Cs, double g_out,
                         double *g_in) {
    double w = solute_w(q, i);
    double k = kr * w / solute_wall_w(q);
    double Ci = (2.0 * g_out + k * Cs) / (2.0 * w + k);
    double gi = 2.0 * w * Ci - g_out;
    double db = g_out - gi;
    if (!(db > 0.0)) {
        gi = g_out;
        db = 0.0;
    }
    if (g_in) *g_in = gi;
    return db;
}

/* ------------------------------------------------------------------- RNG */

/* One output of SplitMix64 for the state x: add the golden gamma, then the
 * variant-13 finaliser (Steele, Lea & Flood 2014). */
uint64_t orc_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Uniform pick of one of m candidates from hash h. */
int orc_pick(uint64_t h, int m) {
    return (int)(((h >> 32) * (uint64_t)m) >> 32);
}

/* ------------------------------------------------------------------ step */

/* The solute is periodic along axis 0 (x) / 1 (y) unless a solute opening
 * lies on one of that axis' walls. */
static int solute_periodic(const orc *o, int axis) {
    for (int k = 0; k < o->nsopen; ++k)
        if ((o->sopen[k].wall < 2) == (axis == 0)) return 0;
    return 1;
}

/* Node (x,y) lies on a wall of a non-periodic solute axis. */
static int solute_on_closed_wall(const orc *o, int x, int y) {
    return (!solute_periodic(o, 0) && (x == 0 || x == o->nx - 1)) ||
           (!solute_periodic(o, 1) && (y == 0 || y == o->ny - 1));
}

/* Index of the solute opening holding node (x,y) whose wall the pull along
 * direction i crosses, or -1. */
static int solute_opening_at(const orc *o, int x, int y, int i) {
    for (int k = 0; k < o->nsopen; ++k) {
        int w = o->sopen[k].wall, pos = w < 2 ? y : x;
        int on = (w == 0 && x == 0) || (w == 1 && x == o->nx - 1) || (w == 2 && y == 0) ||
                 (w == 3 && y == o->ny - 1);
        if (!on || pos < o->sopen[k].lo || pos > o->sopen[k].hi) continue;
        int sx = x - EX9[i], sy = y - EY9[i];
        int cross = (w == 0 && sx < 0) || (w == 1 && sx >= o->nx) || (w == 2 && sy < 0) || (w == 3 && sy >= o->ny);
        if (cross) return k;
    }
    return -1;
}

/* Index of the velocity mirrored across a wall of axis 0 (x) or 1 (y). */
static int mirror_axis(int i, int axis) {
    for (int k = 0; k < 9; ++k)
        if (axis == 0 ? (EX9[k] == -EX9[i] && EY9[k] == EY9[i]) : (EX9[k] == EX9[i] && EY9[k] == -EY9[i]))
            return k;
    return -1;
}

/* Source of the pull along direction i into node (x,y) on the fluid lattice
 * (periodic on both axes). */
static long fluid_src(const orc *o, int x, int y, int i) {
    return idx(o, wrap(x - EX9[i], o->nx), wrap(y - EY9[i], o->ny));
}

/* ------------------------------------------- slip / mixed boundaries */

static int solid_at(const orc *o, int x, int y) { return o->mask[idx(o, wrap(x, o->nx), wrap(y, o->ny))]; }

/* Fate of the diagonal mode k of fluid node P = (px, py) heading into the
 * solid T = P + e_k (boundary_style command, slip rule): 1 if it reflects
 * off a horizontal wall (P + (0, ky) solid, P + (kx, 0) fluid) and lands on
 * P + (2kx, 0), 2 if it reflects off a vertical wall (P + (kx, 0) solid,
 * P + (0, ky) fluid) and lands on P + (0, 2ky), 0 if it bounces back (a
 * corner, or the landing node is solid). */
static int slip_branch(const orc *o, int px, int py, int k) {
    int kx = EX9[k], ky = EY9[k];
    int sy = solid_at(o, px, py + ky), sx = solid_at(o, px + kx, py);
    if (sy && !sx && !solid_at(o, px + 2 * kx, py)) return 1;
    if (sx && !sy && !solid_at(o, px, py + 2 * ky)) return 2;
    return 0;
}

/* Population of diagonal direction i arriving at fluid node X = (x, y)
 * whose source T = X - e_i is solid, with the reflected share R of T (0
 * noslip, 1 slip, else mixed): X's own mode opp(i) that hit T comes back
 * with weight 1 - R when it has a slip branch (1 otherwise), and modes
 * mirrored off the wall at T arrive with weight R: from X - (2 ex_i, 0) by
 * a horizontal reflection (mode (ex_i, -ey_i)) and from X - (0, 2 ey_i) by
 * a vertical one (mode (-ex_i, ey_i)). */
static double diagonal_at_wall(const orc *o, int c, int x, int y, int i) {
    const long n = o->n;
    int ax = EX9[i], ay = EY9[i];
    double R = o->refl[c][idx(o, wrap(x - ax, o->nx), wrap(y - ay, o->ny))];
    long s = idx(o, x, y);
    int own = opposite(i);
    double v = (R > 0.0 && slip_branch(o, x, y, own) ? 1.0 - R : 1.0) * o->f[c][own * n + s];
    if (R > 0.0) {
        int hx = x - 2 * ax, hy = y, kh = -1, vx = x, vy = y - 2 * ay, kv = -1;
        for (int k = 5; k < 9; ++k) {
            if (EX9[k] == ax && EY9[k] == -ay) kh = k;
            if (EX9[k] == -ax && EY9[k] == ay) kv = k;
        }
        if (!solid_at(o, hx, hy) && slip_branch(o, wrap(hx, o->nx), hy, kh) == 1)
            v += R * o->f[c][kh * n + idx(o, wrap(hx, o->nx), hy)];
        if (!solid_at(o, vx, vy) && slip_branch(o, vx, wrap(vy, o->ny), kv) == 2)
            v += R * o->f[c][kv * n + idx(o, vx, wrap(vy, o->ny))];
    }
    return v;
}

/* Forces on the fluid nodes from the densities in o->rho (which must hold
 * the post-streaming densities of the current step; equal to the
 * post-collision ones since BGK conserves each component's mass).
 *   F_c = aveforce_c + rho_c aveacceleration_c
 *         - G rho_c(x) sum_{i=1..8} w_i rho_cbar(x+e_i) e_i   (interforce)
 *         - G_c rho_c(x) sum_{i=1..8} w_i s(x+e_i) e_i          (adhesion)
 * with rho_cbar = 0 on solid neighbours and s = 1 on solids. */
static void compute_forces(orc *o) {
    for (int c = 0; c < o->ncomp; ++c)
#pragma omp parallel for schedule(static)
        for (int y = 0; y < o->ny; ++y)
            for (int x = 0; x < o->nx; ++x) {
                long s = idx(o, x, y);
                double Fx = 0.0, Fy = 0.0;
                if (!o->mask[s]) {
                    double r = o->rho[c][s];
                    Fx = o->force[c][0] + r * o->accel[c][0];
                    Fy = o->force[c][1] + r * o->accel[c][1];
                    if (o->has_inter && o->ncomp == 2) {
                        double sx = 0.0, sy = 0.0;
                        for (int i = 1; i < 9; ++i) {
                            long nb = idx(o, wrap(x + EX9[i], o->nx),
                                          wrap(y + EY9[i], o->ny));
                            double rb = o->mask[nb] ? 0.0 : o->rho[1 - c][nb];
                            sx += W9[i] * rb * EX9[i];
                            sy += W9[i] * rb * EY9[i];
                        }
                        Fx += -o->G * r * sx;
                        Fy += -o->G * r * sy;
                    }
                    if (o->has_inter && o->psi_inter) {
                        double sx = 0.0, sy = 0.0;
                        for (int i = 1; i < 9; ++i) {
                            long nb = idx(o, wrap(x + EX9[i], o->nx),
                                          wrap(y + EY9[i], o->ny));
                            double pb = o->mask[nb] ? 0.0 : psi_of(o->psi0_i, o->rho0_i, o->rho[0][nb]);
                            sx += W9[i] * pb * EX9[i];
                            sy += W9[i] * pb * EY9[i];
                        }
                        double ps = psi_of(o->psi0_i, o->rho0_i, r);
                        Fx += -o->G * ps * sx;
                        Fy += -o->G * ps * sy;
                    }
                    if (o->has_ads[c]) {
                        double sx = 0.0, sy = 0.0;
                        for (int i = 1; i < 9; ++i) {
                            long nb = idx(o, wrap(x + EX9[i], o->nx),
                                          wrap(y + EY9[i], o->ny));
                            double sv = o->mask[nb] ? 1.0 : 0.0;
                            sx += W9[i] * sv * EX9[i];
                            sy += W9[i] * sv * EY9[i];
                        }
                        /* two components: rho_c; one component: psi(rho) */
                        double a = o->psi_ads ? psi_of(o->psi0_a, o->rho0_a, r) : r;
                        Fx += -o->Gads[c] * a * sx;
                        Fy += -o->Gads[c] * a * sy;
                    }
                }
                o->Fx[c][s] = Fx;
                o->Fy[c][s] = Fy;
            }
}

/* Densities and momenta of the populations in arrays f[c]. */
static void compute_moments(orc *o, double *const *f) {
    for (int c = 0; c < o->ncomp; ++c)
#pragma omp parallel for schedule(static)
        for (long s = 0; s < o->n; ++s) {
            double r = 0.0, mx = 0.0, my = 0.0;
            if (!o->mask[s])
                for (int i = 0; i < 9; ++i) {
                    double v = f[c][i * o->n + s];
                    r += v;
                    mx += v * EX9[i];
                    my += v * EY9[i];
                }
            o->rho[c][s] = r;
            o->jx[c][s] = mx;
            o->jy[c][s] = my;
        }
}

static void init_b(orc *o) {
    if (o->b_ready) return;
    for (long s = 0; s < o->n; ++s) o->b[s] = o->mask[s] ? o->b0 : 0.0;
    o->b_ready = 1;
}


/* Rank of node s among the growth candidates of solid node sd: the direct
 * neighbours E, N, W, S (e1..e4) that are fluid, inside the domain and not
 * on an open solute column. Fills cand[] and returns their number. */
static int growth_candidates(const orc *o, int x, int y, long *cand) {
    int m = 0;
    for (int i = 1; i <= 4; ++i) {
        int cx = x + EX9[i], cy = y + EY9[i];
        if ((cx < 0 || cx >= o->nx) && !solute_periodic(o, 0)) continue;
        if ((cy < 0 || cy >= o->ny) && !solute_periodic(o, 1)) continue;
        cx = wrap(cx, o->nx);
        cy = wrap(cy, o->ny);
        if (solute_on_closed_wall(o, cx, cy)) continue;
        long c = idx(o, cx, cy);
        if (!o->mask[c]) cand[m++] = c;
    }
    return m;
}

static void one_step(orc *o) {
    const long n = o->n;
    const int nx = o->nx, ny = o->ny;
    if (o->reaction) init_b(o);
    init_openings(o);

    /* 1. Fluid streaming (pull): the population arriving at x along e_i left
     * x - e_i; if that node is solid, the population that x itself sent
     * towards the wall comes back reversed (noslip, half-way bounce-back). */
    for (int c = 0; c < o->ncomp; ++c)
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long s = idx(o, x, y);
                for (int i = 0; i < 9; ++i) {
                    double v = 0.0;
                    if (!o->mask[s]) {
                        long src = fluid_src(o, x, y, i);
                        if (!o->mask[src])
                            v = o->f[c][i * n + src];
                        else if (i <= 4)
                            v = o->f[c][opposite(i) * n + s];
                        else
                            v = diagonal_at_wall(o, c, x, y, i);
                    }
                    o->ftmp[c][i * n + s] = v;
                }
            }

    /* 1b. Zou-He closure of the velocity and pressure openings. */
    for (int k = 0; k < o->nopen; ++k) {
        if (o->open[k].style > 3) continue;
        for (int j = o->open[k].lo; j <= o->open[k].hi; ++j) {
            int x, y, nxw, nyw;
            wall_geom(o, o->open[k].wall, j, &x, &y, &nxw, &nyw);
            long s = idx(o, x, y);
            if (o->mask[s]) continue;
            int pressure = o->open[k].style == 3;
            double given = pressure ? o->open[k].rho
                                    : opening_un(o->open[k].outlet, o->open[k].style, o->open[k].v,
                                                 o->open[k].lo, o->open[k].hi, j);
            zou_he(o->ftmp[o->open[k].comp], n, s, nxw, nyw, pressure, given);
        }
    }

    /* 2. Moments after streaming. */
    compute_moments(o, o->ftmp);

    /* 3. Forces from those densities. */
    compute_forces(o);

    /* 4.+5. Equilibrium velocity and BGK collision.
     * u' = sum_c (j_c / tau_c) / sum_c (rho_c / tau_c),
     * u_c^eq = u' + tau_c F_c / rho_c, f <- f - (f - f_eq(rho_c, u_c^eq))/tau_c.
     * The solvent velocity of Eq. (u_solvent),
     * u_s = sum_c (j_c + F_c/2) / sum_c rho_c, is kept for the solute. */
    double *usx = (double *)calloc(n, sizeof(double));
    double *usy = (double *)calloc(n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; ++s) {
        if (o->mask[s]) {
            for (int c = 0; c < o->ncomp; ++c)
                for (int i = 0; i < 9; ++i) o->f[c][i * n + s] = 0.0;
            continue;
        }
        double num_x = 0.0, num_y = 0.0, den = 0.0;
        double sjx = 0.0, sjy = 0.0, srho = 0.0;
        for (int c = 0; c < o->ncomp; ++c) {
            num_x += o->jx[c][s] / o->tau[c];
            num_y += o->jy[c][s] / o->tau[c];
            den += o->rho[c][s] / o->tau[c];
            sjx += o->jx[c][s] + 0.5 * o->Fx[c][s];
            sjy += o->jy[c][s] + 0.5 * o->Fy[c][s];
            srho += o->rho[c][s];
        }
        double upx = num_x / den, upy = num_y / den;
        usx[s] = sjx / srho;
        usy[s] = sjy / srho;
        for (int c = 0; c < o->ncomp; ++c) {
            double r = o->rho[c][s];
            double ux = upx + o->tau[c] * o->Fx[c][s] / r;
            double uy = upy + o->tau[c] * o->Fy[c][s] / r;
            for (int i = 0; i < 9; ++i) {
                double fi = o->ftmp[c][i * n + s];
                double fe = feq(i, r, ux, uy, o->alpha[c]);
                o->f[c][i * n + s] = fi - (fi - fe) / o->tau[c];
            }
        }
    }

    /* 5b. Gradient openings: after collision each population of an opening
     * node is extrapolated from the next two nodes inward,
     * f(wall) = 2 f(wall + n) - f(wall + 2n) (inlet_momentum command). */
    for (int k = 0; k < o->nopen; ++k) {
        if (o->open[k].style != 4) continue;
        double *fc = o->f[o->open[k].comp];
        for (int j = o->open[k].lo; j <= o->open[k].hi; ++j) {
            int x, y, nxw, nyw;
            wall_geom(o, o->open[k].wall, j, &x, &y, &nxw, &nyw);
            long s = idx(o, x, y), s1 = idx(o, x + nxw, y + nyw), s2 = idx(o, x + 2 * nxw, y + 2 * nyw);
            if (o->mask[s] || o->mask[s1] || o->mask[s2]) continue;
            for (int i = 0; i < 9; ++i) fc[i * n + s] = 2.0 * fc[i * n + s1] - fc[i * n + s2];
        }
    }

    o->t += 1;
    if (!o->q) {
        free(usx);
        free(usy);
        return;
    }

    /* 6. Solute streaming (pull) with bounce-back on solids (or the reactive
     * link rule when the surface reaction is on), bounce-back on the closed
     * walls of a non-periodic axis and the opening rules at opening nodes.
     * o->g still holds the post-collision values of the previous step. */
    const int q = o->q;
    const int xper = solute_periodic(o, 0), yper = solute_periodic(o, 1);
    const double Dsol = solute_cs2(q) * (o->tau_s - 0.5);
    /* flux openings set the whole node to equilibrium at C (after the
     * solvent velocity is known): C per node, or NAN */
    double *Cflux = (double *)malloc(sizeof(double) * n);
    /* opening fluxes are summed per row, then over rows in order, so the
     * result does not depend on how rows are shared among threads */
    double *in_row = (double *)calloc(ny, sizeof(double));
    double *out_row = (double *)calloc(ny, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long s = idx(o, x, y);
            Cflux[s] = NAN;
            for (int i = 0; i < 9; ++i) o->gtmp[i * n + s] = 0.0;
            if (o->mask[s]) continue;
            int unknown[9] = {0};
            int kopen = -1;
            for (int i = 0; i < 9; ++i) {
                if (!solute_has(q, i)) continue;
                int sxr = x - EX9[i], syr = y - EY9[i];
                int cross = ((sxr < 0 || sxr >= nx) && !xper) || ((syr < 0 || syr >= ny) && !yper);
                double g_out = o->g[opposite(i) * n + s];
                if (cross) {
                    int k = solute_opening_at(o, x, y, i);
                    if (k >= 0) {
                        unknown[i] = 1;
                        kopen = k;
                    } else {
                        o->gtmp[i * n + s] = g_out; /* closed wall: bounce-back */
                    }
                    continue;
                }
                long src = idx(o, wrap(sxr, nx), wrap(syr, ny));
                double gi;
                if (o->mask[src]) {
                    gi = g_out;
                    if (o->reaction)
                        orc_reactive_link(q, i, o->kr, o->Cs, g_out, &gi);
                } else {
                    gi = o->g[i * n + src];
                }
                o->gtmp[i * n + s] = gi;
            }
            if (kopen >= 0) {
                double known = 0.0, wu = 0.0;
                for (int i = 0; i < 9; ++i) {
                    if (!solute_has(q, i)) continue;
                    if (unknown[i])
                        wu += solute_w(q, i);
                    else
                        known += o->gtmp[i * n + s];
                }
                int st = o->sopen[kopen].style, w = o->sopen[kopen].wall;
                if (st == 1) {
                    /* dirichlet: C = Cbar after streaming; the deficit
                     * Cbar - C' (C' = sum of the known populations) is shared
                     * by the unknowns in proportion to their weights (a single
                     * unknown takes all of it, as in the command's rule). */
                    double deficit = o->sopen[kopen].value - known;
                    for (int i = 0; i < 9; ++i)
                        if (unknown[i]) {
                            double gi = solute_w(q, i) / wu * deficit;
                            o->gtmp[i * n + s] = gi;
                            in_row[y] += gi;
                        }
                } else if (st == 2) {
                    /* adiabatic: zero normal flux; each unknown takes the
                     * value of its mirror across the wall (g3 = g1 on xhi). */
                    for (int i = 0; i < 9; ++i)
                        if (unknown[i]) {
                            double gi = o->gtmp[mirror_axis(i, w < 2 ? 0 : 1) * n + s];
                            o->gtmp[i * n + s] = gi;
                            in_row[y] += gi;
                        }
                } else {
                    /* flux: C = (v C0 + D C1)/(D + v) at an inlet,
                     * (v C0 - D C1)/(v - D) at an outlet (App. B), C1 the
                     * concentration of the next node inward (previous time
                     * level; 0 if that node is solid); all populations go to
                     * equilibrium at C. */
                    int nxw = w == 0 ? 1 : w == 1 ? -1 : 0, nyw = w == 2 ? 1 : w == 3 ? -1 : 0;
                    long s1 = idx(o, x + nxw, y + nyw);
                    double C1 = 0.0;
                    if (!o->mask[s1])
                        for (int i = 0; i < 9; ++i) C1 += o->g[i * n + s1];
                    double v = o->sopen[kopen].v, C0 = o->sopen[kopen].value;
                    double C = o->sopen[kopen].outlet ? (v * C0 - Dsol * C1) / (v - Dsol)
                                                      : (v * C0 + Dsol * C1) / (Dsol + v);
                    Cflux[s] = C;
                    in_row[y] += C - known;
                }
            }
            /* Populations of the previous step that left through an opening. */
            for (int i = 0; i < 9; ++i) {
                if (!solute_has(q, i)) continue;
                int dx = x + EX9[i], dy = y + EY9[i];
                int cross = ((dx < 0 || dx >= nx) && !xper) || ((dy < 0 || dy >= ny) && !yper);
                if (cross && solute_opening_at(o, x, y, opposite(i)) >= 0) out_row[y] += o->g[i * n + s];
            }
        }
    for (int y = 0; y < ny; ++y) {
        o->inflow += in_row[y];
        o->outflow += out_row[y];
    }
    free(in_row);
    free(out_row);

    /* 7. Deposit (surface_reaction command): each solid node collects the
     * flux of every reactive link that ends on it, recomputed from the
     * population that entered the wall, i.e. the value the fluid side used. */
    if (o->reaction) {
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long sd = idx(o, x, y);
                if (!o->mask[sd]) continue;
                double dep = 0.0;
                for (int i = 1; i < 9; ++i) {
                    if (!solute_has(q, i)) continue;
                    int fx = x + EX9[i], fy = y + EY9[i];
                    if ((fx < 0 || fx >= nx) && !xper) continue;
                    if ((fy < 0 || fy >= ny) && !yper) continue;
                    long fl = idx(o, wrap(fx, nx), wrap(fy, ny));
                    if (o->mask[fl]) continue;
                    double g_out = o->g[opposite(i) * n + fl];
                    dep += orc_reactive_link(q, i, o->kr, o->Cs, g_out, NULL);
                }
                o->b[sd] += dep;
            }
    }

    /* 7b. intersolute force from the concentrations after streaming (the
     * ones the collision uses, as for interforce): psi = psi0 exp(-C0/C)
     * on fluid nodes with C > 0, 0 on solids, where C <= 0 and across a
     * wall of a non-periodic solute axis. */
    double *Fsx = NULL, *Fsy = NULL;
    if (o->isol) {
        double *psi = (double *)malloc(sizeof(double) * n);
        Fsx = (double *)calloc(n, sizeof(double));
        Fsy = (double *)calloc(n, sizeof(double));
#pragma omp parallel for schedule(static)
        for (long s = 0; s < n; ++s) {
            double C = 0.0;
            for (int i = 0; i < 9; ++i) C += o->gtmp[i * n + s];
            if (!isnan(Cflux[s])) C = Cflux[s];
            psi[s] = (!o->mask[s] && C > 0.0) ? o->psi0_s * exp(-o->C0_s / C) : 0.0;
        }
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long s = idx(o, x, y);
                if (o->mask[s]) continue;
                double sx = 0.0, sy = 0.0;
                for (int i = 1; i <= 4; ++i) {
                    int cx = x + EX9[i], cy = y + EY9[i];
                    if (((cx < 0 || cx >= nx) && !xper) || ((cy < 0 || cy >= ny) && !yper)) continue;
                    double pn = psi[idx(o, wrap(cx, nx), wrap(cy, ny))];
                    sx += EX9[i] * pn;
                    sy += EY9[i] * pn;
                }
                Fsx[s] = -o->G_s * psi[s] * sx;
                Fsy[s] = -o->G_s * psi[s] * sy;
            }
        free(psi);
    }

    /* 8. Solute collision towards g_eq(C, u_s), u_s the solvent velocity
     * plus tau_s F / C of intersolute. */
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; ++s) {
        if (o->mask[s]) {
            for (int i = 0; i < 9; ++i) o->g[i * n + s] = 0.0;
            continue;
        }
        double C = 0.0;
        for (int i = 0; i < 9; ++i) C += o->gtmp[i * n + s];
        const int flux = !isnan(Cflux[s]);
        if (flux) C = Cflux[s];
        double ux = usx[s], uy = usy[s];
        if (o->isol && C > 0.0) {
            ux = ux + o->tau_s * Fsx[s] / C;
            uy = uy + o->tau_s * Fsy[s] / C;
        }
        for (int i = 0; i < 9; ++i) {
            if (!solute_has(q, i)) {
                o->g[i * n + s] = 0.0;
                continue;
            }
            double ge = geq(q, i, C, ux, uy);
            double gi = o->gtmp[i * n + s];
            o->g[i * n + s] = flux ? ge : gi - (gi - ge) / o->tau_s;
        }
    }
    free(usx);
    free(usy);
    free(Cflux);
    free(Fsx);
    free(Fsy);

    /* 9. Surface growth: every solid node whose deposit exceeds bmax turns
     * one of its direct fluid neighbours into solid, each candidate equally
     * likely, and its own deposit is reset to zero (App. C, item 5).  All
     * decisions use the mask and deposits of this step before any change;
     * a node chosen twice grows once. */
    if (o->reaction) {
        memset(o->grow, 0, n);
        memcpy(o->bdec, o->b, sizeof(double) * n);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long sd = idx(o, x, y);
                if (!o->mask[sd] || !(o->b[sd] > o->bmax)) continue;
                long cand[4];
                int m = growth_candidates(o, x, y, cand);
                if (m == 0) continue;
                uint64_t h = orc_splitmix64(o->seed ^
                                            ((uint64_t)o->t * (uint64_t)n +
                                             (uint64_t)sd));
                o->grow[cand[orc_pick(h, m)]] = 1;
                o->consumed_b += o->b[sd];
                o->b[sd] = 0.0;
            }
        for (long s = 0; s < n; ++s) {
            if (!o->grow[s]) continue;
            for (int c = 0; c < o->ncomp; ++c) {
                double r = 0.0;
                for (int i = 0; i < 9; ++i) {
                    r += o->f[c][i * n + s];
                    o->f[c][i * n + s] = 0.0;
                }
                o->removed_rho[c] += r;
            }
            double C = 0.0;
            for (int i = 0; i < 9; ++i) {
                C += o->g[i * n + s];
                o->g[i * n + s] = 0.0;
            }
            o->removed_C += C;
            o->refl[0][s] = o->grow_R[0];
            o->refl[1][s] = o->grow_R[1];
            o->mask[s] = 1;
            o->b[s] = o->b0;
            o->grown_nodes += 1;
        }
    }
}

int orc_step(orc *o, long nsteps) {
    for (long k = 0; k < nsteps; ++k) one_step(o);
    return 0;
}

/* ---------------------------------------------------------------- readout */

/* Output command: density and velocity after collision, the velocity with
 * the applied forces taken into account (output command).  From the stored post-collision
 * state the velocity is (j_post - F/2)/rho, which equals the half-force
 * velocity (j + F/2)/rho of the streamed state for one fluid, and for the
 * mixture (comp = -1) equals Eq. (u_solvent).  Solid nodes read rho = -11
 * and zero velocity (write_restart convention). */
int orc_moments(orc *o, int comp, double *rho, double *ux, double *uy) {
    if (comp < -1 || comp >= o->ncomp) return -1;
    init_openings(o);
    compute_moments(o, o->f);
    compute_forces(o);
    for (long s = 0; s < o->n; ++s) {
        if (o->mask[s]) {
            rho[s] = -11.0;
            ux[s] = uy[s] = 0.0;
            continue;
        }
        double r = 0.0, mx = 0.0, my = 0.0;
        for (int c = 0; c < o->ncomp; ++c) {
            if (comp >= 0 && c != comp) continue;
            r += o->rho[c][s];
            mx += o->jx[c][s] - 0.5 * o->Fx[c][s];
            my += o->jy[c][s] - 0.5 * o->Fy[c][s];
        }
        rho[s] = r;
        ux[s] = mx / r;
        uy[s] = my / r;
    }
    return 0;
}

/* Solute output: C on fluid nodes (0 on solids), deposit b on solids (0 on
 * fluid nodes). */
int orc_solute_state(orc *o, double *C, double *b) {
    if (!o->q) return -1;
    if (o->reaction) init_b(o);
    for (long s = 0; s < o->n; ++s) {
        double c = 0.0;
        if (!o->mask[s])
            for (int i = 0; i < 9; ++i) c += o->g[i * o->n + s];
        if (C) C[s] = c;
        if (b) b[s] = (o->mask[s] && o->reaction) ? o->b[s] : 0.0;
    }
    return 0;
}

/* Budgets (thermo command, in FP64): see the index list in the Python
 * wrapper. */
int orc_budgets(orc *o, double *out) {
    if (o->reaction) init_b(o);
    init_openings(o);
    for (int k = 0; k < 16; ++k) out[k] = 0.0;
    long nfluid = 0;
    for (long s = 0; s < o->n; ++s) {
        if (o->mask[s]) {
            if (o->reaction) out[5] += o->b[s];
            continue;
        }
        nfluid++;
        for (int c = 0; c < o->ncomp; ++c)
            for (int i = 0; i < 9; ++i) {
                double v = o->f[c][i * o->n + s];
                out[c] += v;
                out[2] += v * EX9[i];
                out[3] += v * EY9[i];
            }
        if (o->q)
            for (int i = 0; i < 9; ++i) out[4] += o->g[i * o->n + s];
    }
    out[6] = o->removed_rho[0];
    out[7] = o->removed_rho[1];
    out[8] = o->removed_C;
    out[9] = o->inflow;
    out[10] = o->outflow;
    out[11] = (double)o->t;
    out[12] = (double)o->grown_nodes;
    out[13] = (double)nfluid;
    out[14] = o->consumed_b;
    return 0;
}

/* ------------------------------------------------------ raw state access */

long orc_step_count(const orc *o) { return o->t; }
void orc_set_step_count(orc *o, long t) { o->t = t; }

int orc_get_f(orc *o, int comp, double *out) {
    if (comp < 0 || comp > 1) return -1;
    init_openings(o);
    memcpy(out, o->f[comp], sizeof(double) * 9 * o->n);
    return 0;
}
int orc_set_f(orc *o, int comp, const double *in) {
    if (comp < 0 || comp > 1) return -1;
    o->open_ready = 1;  /* raw populations are taken as given */
    memcpy(o->f[comp], in, sizeof(double) * 9 * o->n);
    return 0;
}
int orc_get_g(const orc *o, double *out) {
    memcpy(out, o->g, sizeof(double) * 9 * o->n);
    return 0;
}
int orc_set_g(orc *o, const double *in) {
    memcpy(o->g, in, sizeof(double) * 9 * o->n);
    return 0;
}
int orc_get_mask(const orc *o, uint8_t *out) {
    memcpy(out, o->mask, o->n);
    return 0;
}
int orc_set_mask(orc *o, const uint8_t *in) {
    memcpy(o->mask, in, o->n);
    return 0;
}
int orc_get_b(orc *o, double *out) {
    if (o->reaction) init_b(o);
    memcpy(out, o->b, sizeof(double) * o->n);
    return 0;
}
/* Deposits at the growth decisions of the last step (after its deposit,
 * before the triggering deposits were reset). */
int orc_get_bdec(orc *o, double *out) {
    memcpy(out, o->bdec, sizeof(double) * o->n);
    return 0;
}
int orc_set_b(orc *o, const double *in) {
    memcpy(o->b, in, sizeof(double) * o->n);
    o->b_ready = 1;
    return 0;
}
/* Forces of the current (post-collision) state, for tests. */
int orc_forces(orc *o, int comp, double *Fx, double *Fy) {
    if (comp < 0 || comp >= o->ncomp) return -1;
    init_openings(o);
    compute_moments(o, o->f);
    compute_forces(o);
    memcpy(Fx, o->Fx[comp], sizeof(double) * o->n);
    memcpy(Fy, o->Fy[comp], sizeof(double) * o->n);
    return 0;
}
