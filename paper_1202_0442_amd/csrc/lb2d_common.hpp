// lb2d_common.hpp -- parameter blocks shared by the host runtime and the
// gfx950 kernels of the D2Q9 lattice Boltzmann library.  Plain structs only.
#pragma once
#include <cstddef>
#include <cstdint>

namespace lb2d {

// Storage formats (same values as LB2D_F64 ... in include/lb2d.h).
enum Storage : int { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

// Brick layout of every population plane (fluid components and solute):
// each plane is cut into bricks of BW x BH nodes stored contiguously, in
// row-major brick order over the plane padded to whole bricks: 4x4 for
// 4-byte values (64 bytes), 4x8 for 2-byte values (64 bytes) and 8x4 for
// 8-byte values (256 bytes).  A brick covers a compact 2-D patch, so bricks
// that lie entirely inside obstacles are never read or written; the
// 64-byte bricks skip more of the solid area next to obstacle boundaries
// than 128-byte ones (measured faster on the porous workload, while 32-byte
// bricks lose to the shorter memory segments).
inline constexpr int brick_w_for(int value_bytes) { return value_bytes == 8 ? 8 : 4; }
inline constexpr int brick_h_for(int value_bytes) { return value_bytes == 2 ? 8 : 4; }

// One single-fluid lattice for the plain fused step (and for one entry of
// the batched step).  Populations live in two buffers (two-lattice pull
// scheme); f[p] holds 9 brick-layout planes of deviations f_i - w_i rho_ref
// (zero, and never read, at solid nodes).
struct PlainLattice {
    void *f[2];
    const uint16_t *links; // bit 0: node solid; bit i (1..8): node + e_i solid
                           // (row-major [ny][nx])
    int nx, ny;
    unsigned pnx;          // nx padded to whole bricks
    size_t plane;          // elements per population plane (padded)
    double omega;         // 1 / tau
    double tau;
    double Fx, Fy;        // aveforce (summed vector)
    double ax, ay;        // aveacceleration (summed vector)
    double rho_ref;       // shift of the stored populations
    // the same seven coefficients rounded to FP32, for the formats whose
    // collision runs in FP32 (FP32 and the 16-bit formats)
    float omega_f, tau_f, Fx_f, Fy_f, ax_f, ay_f, rho_ref_f;
    const unsigned long long *step;  // completed steps (device; read only by
                                     // the stochastically rounded step)
    unsigned seed;        // key of the stochastic-rounding stream
};

// Steps per launch of the multi-step one-fluid kernel, and its tile (FP64:
// kMultiTW / 2 x kMultiTH).  Measured on the porous 4096^2 lattice, FP32,
// microseconds per step for 1 .. 6 steps per launch: 168, 112, 90.5, 77.9,
// 71.9, 72.5.
constexpr int kMultiSteps = 5;
constexpr int kMultiTW = 64;
constexpr int kMultiTH = 16;
static_assert(kMultiSteps % 2 == 1, "an odd number of steps per launch keeps the buffer convention");

// Tile of the batched step: lattice index and lower-left node.
struct Tile {
    int lattice;
    int x0, y0;
    int pad;
};

// Physical coefficients of the general step in its arithmetic type (the
// host fills an FP64 and an FP32 copy, so no kernel converts them).
template <typename R>
struct StepCoef {
    R tau[2], omega[2];
    R A0[2], A1[2];        // equilibrium coefficients A_0, A_{1..8}
    R rho_ref[2];          // shift of the stored populations
    R force[2][2], accel[2][2];
    R G;                   // interforce strength
    R Gads[2];             // adhesiveforce per component (0 = off)
    R psi0, rho0;          // one component: interforce psi = psi0 exp(-rho0/rho)
    R psi0a, rho0a;        // one component: adhesiveforce psi
    R omega_s;             // 1 / tau_s
    R Dsol;                // solute diffusivity c_s^2 (tau_s - 1/2)
    R Cs;                  // saturation concentration
    R rlink[2];            // reactive links: 2 k_i / (2 w_i + k_i), axial and diagonal
    R rlink_cs[2];         // the same times w_i Cs
};

// One momentum opening (inlet/outlet + inlet_momentum/outlet_momentum
// commands): nodes lo..hi of a wall of the box, for one fluid component.
struct OpenSpec {
    int wall;             // 0 xlo, 1 xhi, 2 ylo, 3 yhi
    int lo, hi;           // node range along the wall
    int comp;
    int outlet;           // 0 inlet, 1 outlet
    int style;            // 1 poiseuille, 2 uniform, 3 dirichlet, 4 gradient
    double v, rho;        // speed (v_max for poiseuille) and density
};
constexpr int kMaxOpen = 8;

// One solute opening (inlet_solute / outlet_solute commands): nodes lo..hi
// of a wall.  An opening makes the solute non-periodic across its axis; the
// rest of that axis' two walls is impermeable to the solute.
struct SoluteOpen {
    int wall;             // 0 xlo, 1 xhi, 2 ylo, 3 yhi
    int lo, hi;           // node range along the wall
    int outlet;           // 0 inlet, 1 outlet
    int style;            // 1 dirichlet, 2 adiabatic, 3 flux
    double value;         // dirichlet: imposed C; flux: C0 of the injected solution
    double v;             // flux: velocity of the injected solution
};

// Everything the general fused step needs: up to two fluid components with
// Shan-Chen cohesion / adhesion and an optional solute (D2Q9 or D2Q4) with
// openings, a reactive surface, FP64 deposits and growth triggers.
struct FullParams {
    void *f[2][2];        // [parity][component] fluid populations
    void *g[2];           // [parity] solute populations, sq planes
    uint8_t *mask;        // 1 = solid
    uint16_t *links;      // bit 0: node solid; bit i: node + e_i solid
    uint8_t *trig;        // growth trigger: 0 or 1..4 = direction to grow
    double *b;            // deposits, FP64, [ny][nx]
    double *partial;      // running per-wavefront tallies of the step kernel [slots][4]
    double *gpartial;     // running per-block tallies of the growth kernel [nblk][4]
    double *totals;       // fixed-order sums of the tallies (LB2D_B_* indices)
    long long *dstep;     // completed steps (device copy)
    unsigned *gflag;      // [2]: a growth trigger fired in the step of that parity
    uint8_t *gseg[2];     // [parity][y * ((nx + 255) / 256) + x / 256]: 1 = that
                          // row segment of 256 nodes holds the target of a growth
                          // trigger fired in the step of that parity
    unsigned pnx;         // padded nx of the brick layout
    size_t pplane;        // elements per population plane
    int nx, ny;
    int ncomp;
    int psi;              // one component: interforce acts through psi(rho)
    int has_ads;
    int ads_psi;          // one component: adhesion acts through psi(rho)
    int sq;               // solute lattice: 9 (D2Q9, plane i = direction i) or
                          // 4 (D2Q4, plane i-1 = direction i = 1..4); 0 = none
    int sxper, syper;     // 1: solute periodic along x / y (no opening on that axis' walls)
    int nsopen;           // solute openings
    SoluteOpen sopen[kMaxOpen];
    double b0, bmax;
    unsigned long long seed;
    int nblk_main;        // tally slots of the step kernel (one per wavefront)
    int nblk_grow;        // blocks (tally slots) of the growth kernel
    int nopen;            // momentum openings
    OpenSpec open[kMaxOpen];
    int slip;             // some solid reflects diagonal modes (slip/mixed/hybrid)
    double *refl[2];      // per node and component: reflected share R of a
                          // diagonal mode hitting this solid (0 noslip, 1 slip)
    double grow_R[2];     // R of solids made by growth
    int isol;             // intersolute force on the solute
    double is_G, is_psi0, is_C0;  // its strength and psi = psi0 exp(-C0 / C)
    double tau_s;         // solute relaxation time
    int sr;               // 16-bit storage rounds stochastically
    unsigned sr_seed;     // its key
    StepCoef<double> cd;  // FP64 coefficients
    StepCoef<float> cf;   // the same rounded to FP32
};

}  // namespace lb2d
