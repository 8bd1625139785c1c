// lb2d_device.hpp -- device code of the gfx950 kernels of the D2Q9 lattice
// Boltzmann library: lattice constants, storage codecs, the fused step
// kernels and the set-up / read-out kernels.  Included by the translation
// units that instantiate and launch them (lb2d_kernels.hip and the
// lb2d_full_*.hip units of the general step); everything here has internal
// linkage.
//
// Method: "Introduction to Perl module lb2d.pm 0.1 for basic Lattice
// Boltzmann simulations" (D. Sergi, arXiv:1202.0442), Sec. "Model and
// algorithm" (Eq. (lb), Eq. (eq), Fig. "algorithm") and the commands
// fluids, solute, boundary_style (noslip), obstacle, surface_reaction,
// inlet_solute/outlet_solute, aveforce, aveacceleration, interforce,
// adhesiveforce, thermo and output.
//
// Design (bandwidth-bound stencil, no matrix cores):
//  * populations are nine planes per buffer, each plane stored as bricks of
//    4x4 (FP32), 4x8 (16-bit) or 8x4 (FP64) nodes, in two buffers; a step
//    pulls f_i from x - e_i in buffer p and writes buffer p^1; the lanes of
//    a wavefront cover whole bricks, and a brick is written only if it
//    holds a fluid node;
//  * half-way bounce-back is a per-lane address select: when x - e_i is
//    solid the lane reads its own opposite population instead;
//  * one fused pass per step does stream, moments, forces, equilibrium and
//    BGK relaxation (and, in the general kernel, the solute step, reactive
//    links and deposit gathering); solid nodes are skipped entirely; the
//    one-fluid step runs five steps per launch, the first four kept in LDS
//    for a tile and the rings around it;
//  * Shan-Chen cohesion needs the post-stream densities of the 8
//    neighbours: the general kernel computes a (TX+2) x (TY+2) density tile
//    in LDS, pulling the halo nodes' populations again (they come from L2),
//    and maps tiles to XCDs in contiguous bands so neighbouring tiles share
//    an L2;
//  * deposits are gathered by the solid node's own thread (no atomics);
//    growth is decided there and applied by a separate gather kernel over
//    the row segments that hold a trigger's target;
//  * every FP64 tally is a fixed-order block reduction followed by a
//    fixed-order sum of the block partials, so results are bitwise
//    reproducible.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lb2d_common.hpp"
#include "lb2d_kernels.hpp"

namespace lb2d {
namespace {

// ----------------------------------------------------------------- lattice

__host__ __device__ constexpr int ex(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) {
    return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 5 + 2) % 4) + 5);
}
static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp");
// x-mirror (ex -> -ex): 1<->3, 5<->6, 7<->8.
__host__ __device__ constexpr int mirx(int i) {
    return i == 1 ? 3 : i == 3 ? 1 : i == 5 ? 6 : i == 6 ? 5 : i == 7 ? 8 : i == 8 ? 7 : i;
}
// Eq. (eq) weights.
template <typename R>
__host__ __device__ constexpr R wgt(int i) {
    return i == 0 ? R(4.0 / 9.0) : (i <= 4 ? R(1.0 / 9.0) : R(1.0 / 36.0));
}

// Solute lattices (solute command): D2Q9 with the weights above and
// c_s^2 = 1/3, or the paper's D2Q4 (directions 1..4, weight 1/4 each,
// c_s^2 = 1/2).  SQ = 0 means no solute.
template <int SQ>
__host__ __device__ constexpr bool shas(int i) {
    return SQ == 9 ? true : (SQ == 4 ? (i >= 1 && i <= 4) : false);
}
template <int SQ, typename R>
__host__ __device__ constexpr R swgt(int i) {
    return SQ == 9 ? wgt<R>(i) : R(0.25);
}
// 1 / c_s^2 of the solute lattice
template <int SQ, typename R>
__host__ __device__ constexpr R sics2() {
    return SQ == 9 ? R(3) : R(2);
}
// storage plane of solute direction i
template <int SQ>
__host__ __device__ constexpr int spl(int i) {
    return SQ == 9 ? i : i - 1;
}
// Direction stored in solute plane k (the inverse of spl): D2Q4 keeps
// directions 1..4 in planes 0..3.
__host__ __device__ constexpr int splane_dir(int sq, int k) { return sq == 4 ? k + 1 : k; }

// Reciprocal: the hardware's (1 ulp) in FP32, exact division in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// ----------------------------------------------------------------- storage

// bfloat16 bits (a distinct scalar type, so it can be read through any
// address space)
enum class bf16s : uint16_t {};

template <typename S>
struct Codec;

template <>
struct Codec<double> {
    using R = double;
    __device__ static double dec(double v, int) { return v; }
    __device__ static double enc(double v, int) { return v; }
};
template <>
struct Codec<float> {
    using R = float;
    __device__ static float dec(float v, int) { return v; }
    __device__ static float enc(float v, int) { return v; }
};
// 16-bit formats: deviation times 2 (rest), 8 (axis), 32 (diagonal), which
// brings all nine to a similar magnitude, then rounded to nearest even.
__host__ __device__ constexpr float scale16(int i) { return i == 0 ? 2.0f : (i <= 4 ? 8.0f : 32.0f); }
__host__ __device__ constexpr float iscale16(int i) { return i == 0 ? 0.5f : (i <= 4 ? 0.125f : 0.03125f); }
// enc_sr rounds stochastically with the hardware converts of gfx950: the
// value rounds away from zero with probability equal to the discarded
// fraction of an ulp, decided by the high bits of the random word r (13 bits
// for FP16, 16 bits for BF16).
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf162_t __attribute__((ext_vector_type(2)));
template <>
struct Codec<_Float16> {
    using R = float;
    // one mixed-precision multiply-add (v_fma_mix_f32) instead of a convert
    // and a multiply; exact, the scale being a power of two
    __device__ static float dec(_Float16 v, int i) { return __builtin_fmaf((float)v, iscale16(i), 0.0f); }
    __device__ static _Float16 enc(float d, int i) { return (_Float16)(d * scale16(i)); }
    __device__ static _Float16 enc_sr(float d, int i, unsigned r) {
        half2_t h = {};
        h = __builtin_amdgcn_cvt_sr_f16_f32(h, d * scale16(i), r, false);
        return h[0];
    }
};
template <>
struct Codec<bf16s> {
    using R = float;
    __device__ static float dec(bf16s v, int i) {
        return __uint_as_float((uint32_t)(uint16_t)v << 16) * iscale16(i);
    }
    __device__ static bf16s enc(float d, int i) {
        // round to nearest even: the gfx950 convert (v_cvt_pk_bf16_f32)
        return (bf16s)__builtin_bit_cast(uint16_t, (__bf16)(d * scale16(i)));
    }
    __device__ static bf16s enc_sr(float d, int i, unsigned r) {
        bf162_t h = {};
        h = __builtin_amdgcn_cvt_sr_bf16_f32(h, d * scale16(i), r, false);
        return (bf16s)__builtin_bit_cast(uint16_t, h[0]);
    }
};

// Counter-based random words for stochastic rounding: the 32-bit integer
// hash "lowbias32" (C. Wellons, hash-prospector, 2018) of the node and the
// step, extended to five words per node by Marsaglia's xorshift32
// recurrence (J. Stat. Softw. 8(14), 2003).  Each word serves two
// populations: itself and itself shifted left by 16 bits.
__device__ __forceinline__ unsigned lowbias32(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ unsigned xorshift32(unsigned x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

__device__ __forceinline__ int wrapi(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}

// Element index of node (x, y) in a brick-layout plane of padded width pnx.
template <typename S>
__host__ __device__ __forceinline__ size_t brick_index(unsigned x, unsigned y, unsigned pnx) {
    constexpr unsigned W = brick_w_for(sizeof(S)), H = brick_h_for(sizeof(S));
    return ((size_t)(y / H) * (pnx / W) + (x / W)) * (W * H) + (y % H) * W + (x % W);
}


// Byte offset of node (x, y) in a brick-layout plane, computed in O
// (32-bit when the population arrays are below 4 GiB: a uniform base
// pointer plus a 32-bit lane offset needs no 64-bit lane arithmetic).
template <typename S, typename O>
__device__ __forceinline__ O brick_off(unsigned x, unsigned y, unsigned pnx) {
    constexpr unsigned W = brick_w_for(sizeof(S)), H = brick_h_for(sizeof(S));
    return (((O)(y / H) * (O)(pnx / W) + (O)(x / W)) * (O)(W * H) + (O)((y % H) * W + (x % W))) * (O)sizeof(S);
}

// The same offset split into a row part and a column part (their sum), so
// that the eight neighbours of a node cost one add each.
template <typename S, typename O>
__device__ __forceinline__ O brick_row(unsigned y, unsigned pnx) {
    constexpr unsigned W = brick_w_for(sizeof(S)), H = brick_h_for(sizeof(S));
    return ((O)(y / H) * (O)(pnx / W) * (O)(W * H) + (O)((y % H) * W)) * (O)sizeof(S);
}
template <typename S, typename O>
__device__ __forceinline__ O brick_col(unsigned x) {
    constexpr unsigned W = brick_w_for(sizeof(S)), H = brick_h_for(sizeof(S));
    return ((O)(x / W) * (O)(W * H) + (O)(x % W)) * (O)sizeof(S);
}

// Offsets of node (x, y) (src[0]) and of node - e_i for each direction,
// given the periodic neighbour coordinates xm = x - 1, xp = x + 1, ym, yp.
template <typename S, typename O>
__device__ __forceinline__ void brick_pulls(unsigned x, unsigned y, unsigned xm, unsigned xp, unsigned ym,
                                            unsigned yp, unsigned pnx, O (&src)[9]) {
    const O r0 = brick_row<S, O>(y, pnx), rm = brick_row<S, O>(ym, pnx), rp = brick_row<S, O>(yp, pnx);
    const O c0 = brick_col<S, O>(x), cm = brick_col<S, O>(xm), cp = brick_col<S, O>(xp);
    src[0] = r0 + c0;
    src[1] = r0 + cm;
    src[2] = rm + c0;
    src[3] = r0 + cp;
    src[4] = rp + c0;
    src[5] = rm + cm;
    src[6] = rm + cp;
    src[7] = rp + cp;
    src[8] = rp + cm;
}

// Deterministic block sum of K doubles per thread into out[0..K) (valid in
// thread 0).  `sh` must hold blockDim.x * blockDim.y * K doubles... to keep
// LDS small the reduction goes through wavefront shuffles first.
template <int K>
__device__ void block_sum(double (&v)[K], double *sh, double *out) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nthr = blockDim.x * blockDim.y;
    const int lane = tid & 63, wid = tid >> 6, nw = (nthr + 63) >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double a = v[k];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        v[k] = a;
    }
    if (lane == 0)
        for (int k = 0; k < K; ++k) sh[wid * K + k] = v[k];
    __syncthreads();
    if (tid == 0) {
        for (int k = 0; k < K; ++k) {
            double a = 0.0;
            for (int w = 0; w < nw; ++w) a += sh[w * K + k];
            out[k] = a;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------- plain fused step

// One node of the single-fluid step: pull with half-way bounce-back,
// moments, velocity-shift forcing, BGK relaxation to Eq. (eq), store.
// Populations are deviations d_i = f_i - w_i rho_ref, so
// rho = rho_ref + sum d_i and j = sum d_i e_i; the equilibrium deviation is
// w_i [drho + rho (3 e.u + 9/2 (e.u)^2 - 3/2 u.u)].
//
// Memory behaviour:
//  * one 16-bit link word per node says which of the 8 neighbours are
//    solid, so the nine population addresses (own opposite population when
//    the source is solid: noslip bounce-back) are known after one load and
//    the nine loads are issued together;
//  * a brick with at least one fluid node stores all its nodes (solid
//    nodes store zeros, which nothing ever reads), so every store writes
//    whole bricks -- partial segments along obstacle edges would make the
//    memory read-modify-write them; bricks that are entirely solid are
//    never written, and wavefronts that are entirely solid do no memory
//    work at all;
//  * the stores are streaming (non-temporal) when the populations exceed
//    the last-level cache: nothing reads the new populations in the same
//    step.
// Pointers known to address global memory (so the compiler emits global_*
// rather than flat_* instructions for pointers read from device tables).
#define LB2D_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ LB2D_GLOBAL T *gbl(T *p) {
    return (LB2D_GLOBAL T *)p;
}

// Streaming store of one population value (a vector global store with the
// non-temporal hint): the new populations are not read again in the same
// step, so they need not stay in the caches.  Used when a lattice's
// populations exceed the 256 MB last-level cache (Infinity Cache) of the
// MI355X; smaller lattices keep plain stores, so that the next step finds
// its populations in that cache.  16-bit values are stored through their
// bit pattern.
template <typename S>
__device__ __forceinline__ void st_stream(LB2D_GLOBAL S *p, S v) {
    if constexpr (sizeof(S) == 2) {
        uint16_t bits;
        __builtin_memcpy(&bits, &v, 2);
        __builtin_nontemporal_store(bits, (LB2D_GLOBAL uint16_t *)p);
    } else {
        __builtin_nontemporal_store(v, p);
    }
}

// Wavefront-uniform copy of one step's lattice parameters (scalar
// registers); the collision coefficients in the arithmetic type.
template <typename S>
struct PlainArgs {
    using R = typename Codec<S>::R;
    const S *fin;
    S *fout;
    const uint16_t *links;
    unsigned nx, ny, pnx;
    size_t plane;
    R omega, tau, Fx, Fy, ax, ay, rho_ref;
};

__device__ __forceinline__ unsigned ufl(unsigned v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long ufl64(unsigned long long v) {
    return ((unsigned long long)ufl((unsigned)(v >> 32)) << 32) | ufl((unsigned)v);
}
__device__ __forceinline__ double ufld(double v) { return __longlong_as_double((long long)ufl64((unsigned long long)__double_as_longlong(v))); }
__device__ __forceinline__ float ufld(float v) { return __uint_as_float(ufl(__float_as_uint(v))); }
template <typename T>
__device__ __forceinline__ T *uflp(T *p) { return (T *)ufl64((unsigned long long)p); }

// Parameters of lattice L at the given parity; `uniform` forces them into
// scalar registers when L was read from memory.
template <typename S>
__device__ __forceinline__ PlainArgs<S> plain_args(const PlainLattice &L, int parity) {
    PlainArgs<S> a;
    a.fin = (const S *)(parity ? L.f[1] : L.f[0]);
    a.fout = (S *)(parity ? L.f[0] : L.f[1]);
    a.links = L.links;
    a.nx = (unsigned)L.nx;
    a.ny = (unsigned)L.ny;
    a.pnx = L.pnx;
    a.plane = L.plane;
    if constexpr (sizeof(typename PlainArgs<S>::R) == 4) {
        a.omega = L.omega_f;
        a.tau = L.tau_f;
        a.Fx = L.Fx_f;
        a.Fy = L.Fy_f;
        a.ax = L.ax_f;
        a.ay = L.ay_f;
        a.rho_ref = L.rho_ref_f;
    } else {
        a.omega = L.omega;
        a.tau = L.tau;
        a.Fx = L.Fx;
        a.Fy = L.Fy;
        a.ax = L.ax;
        a.ay = L.ay;
        a.rho_ref = L.rho_ref;
    }
    return a;
}

template <typename S>
__device__ __forceinline__ PlainArgs<S> uniform_args(PlainArgs<S> a) {
    a.fin = uflp(a.fin);
    a.fout = uflp(a.fout);
    a.links = uflp(a.links);
    a.nx = ufl(a.nx);
    a.ny = ufl(a.ny);
    a.pnx = ufl(a.pnx);
    a.plane = (size_t)ufl64((unsigned long long)a.plane);
    a.omega = ufld(a.omega);
    a.tau = ufld(a.tau);
    a.Fx = ufld(a.Fx);
    a.Fy = ufld(a.Fy);
    a.ax = ufld(a.ax);
    a.ay = ufld(a.ay);
    a.rho_ref = ufld(a.rho_ref);
    return a;
}

// Multiply-add with one rounding, in the arithmetic type.
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Pull of one fluid node (x, y) with link word lk: d_i from x - e_i in the
// input buffer, or the node's own opposite population where x - e_i is
// solid (noslip bounce-back).
template <typename S, typename O>
__device__ __forceinline__ void plain_pull(const PlainArgs<S> &L, unsigned xx, unsigned yy, unsigned lk,
                                           typename Codec<S>::R (&d)[9]) {
    using C = Codec<S>;
    const unsigned nx = L.nx, ny = L.ny, pnx = L.pnx;
    const O pl = (O)L.plane * (O)sizeof(S);  // bytes per plane
    const LB2D_GLOBAL char *__restrict__ fin = (const LB2D_GLOBAL char *)gbl(L.fin);
    const unsigned xm = (xx == 0) ? nx - 1 : xx - 1;
    const unsigned xp = (xx == nx - 1) ? 0 : xx + 1;
    const unsigned ym = (yy == 0) ? ny - 1 : yy - 1;
    const unsigned yp = (yy == ny - 1) ? 0 : yy + 1;
    O src[9];  // the node, then node - e_i for each direction
    brick_pulls<S, O>(xx, yy, xm, xp, ym, yp, pnx, src);
    const O s = src[0];
    d[0] = C::dec(*(const LB2D_GLOBAL S *)(fin + s), 0);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        // node - e_i is node + e_opp(i): solid -> bounce-back
        const bool wall = (lk >> opp(i)) & 1u;
        const O a = wall ? (O)opp(i) * pl + s : (O)i * pl + src[i];
        d[i] = C::dec(*(const LB2D_GLOBAL S *)(fin + a), i);
    }
}

// Collision of one node from its pulled deviations: moments, velocity-shift
// forcing, Eq. (eq), BGK relaxation; d receives the post-collision
// deviations (zero at solid nodes).  Every multiply-add is written out and
// implicit contraction is off, so the rounding is the same in every kernel
// this is inlined into (the one-step, multi-step and batched kernels give the
// same bits).  The order of operations and the fused products are those the
// compiler chose for the FP32 and FP64 one-step kernels with contraction
// on (the diagonal projections e.u fuse the product of 1/rho with the x
// momentum, and the u.u term enters the bracket as one multiply-add),
// except that the sums start from their first term rather than from zero.
template <typename S, typename R>
__device__ __forceinline__ void plain_relax(const PlainArgs<S> &L, R (&d)[9], bool fluid) {
#pragma clang fp contract(off)
    R drho = d[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) drho = drho + d[i];
    const R jx = (((d[1] - d[3]) + d[5]) - d[6] - d[7]) + d[8];
    const R jy = (((d[2] - d[4]) + d[5]) + d[6] - d[7]) - d[8];
    const R rho = drho + L.rho_ref;
    const R tau = L.tau, omega = L.omega;
    const R Fx = fmar(rho, L.ax, L.Fx);
    const R Fy = fmar(rho, L.ay, L.Fy);
    const R mx = fmar(Fx, tau, jx);  // j + tau F
    const R my = fmar(Fy, tau, jy);
    const R inv = rcp(rho);
    const R ux = inv * mx, uy = inv * my;
    const R u2 = fmar(ux, ux, uy * uy);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        R eu;
        if (i == 0) eu = R(0);
        else if (i == 1) eu = ux;
        else if (i == 2) eu = uy;
        else if (i == 3) eu = -ux;
        else if (i == 4) eu = -uy;
        else eu = fmar(ex(i) > 0 ? inv : -inv, mx, ey(i) > 0 ? uy : -uy);
        // 3 e.u + 9/2 (e.u)^2 - 3/2 u.u, then f_eq - w_i rho_ref - d_i
        R t = (R(4.5) * eu) * eu;
        t = fmar(R(3), eu, t);
        t = fmar(R(-1.5), u2, t);
        const R dd = fmar(fmar(rho, t, drho), wgt<R>(i), -d[i]);
        d[i] = fluid ? fmar(dd, omega, d[i]) : R(0);
    }
}

// Random words of node (x, y) for stochastic rounding under step key tkey.
__device__ __forceinline__ void sr_words(unsigned node, unsigned tkey, unsigned (&w)[5]) {
    w[0] = lowbias32(node ^ tkey);
#pragma unroll
    for (int k = 1; k < 5; ++k) w[k] = xorshift32(w[k - 1]);
}

// Population i of a node in the storage format (rounded stochastically with
// the node's words when SR).
template <typename S, bool SR>
__device__ __forceinline__ S plain_enc(typename Codec<S>::R v, int i, const unsigned (&w)[5]) {
    if constexpr (SR) return Codec<S>::enc_sr(v, i, (i & 1) ? (w[i >> 1] << 16) : w[i >> 1]);
    else return Codec<S>::enc(v, i);
}

template <typename S, typename O, bool SR, bool NT>
__device__ __forceinline__ void plain_node(const PlainArgs<S> &L, int x, int y, bool inside, unsigned tkey) {
    using C = Codec<S>;
    using R = typename C::R;
    constexpr unsigned kGroup = brick_w_for(sizeof(S)) * brick_h_for(sizeof(S));  // lanes per brick
    const unsigned nx = L.nx, pnx = L.pnx;
    const unsigned s_row = inside ? (unsigned)y * nx + (unsigned)x : 0u;
    const unsigned lk = inside ? (unsigned)gbl(L.links)[s_row] : 1u;
    const bool fluid = (lk & 1u) == 0u;
    const unsigned long long bal = __ballot(fluid);
    if (bal == 0ull) return;
    if (!inside) return;
    // a brick (one 64- to 256-byte segment) is written iff it holds a fluid node
    const unsigned lane = __lane_id();
    const unsigned long long gmask =
        (kGroup >= 64) ? ~0ull : (((1ull << (kGroup & 63)) - 1ull) << ((lane / kGroup) * kGroup));
    if ((bal & gmask) == 0ull) return;
    R d[9];
    if (fluid) {
        plain_pull<S, O>(L, (unsigned)x, (unsigned)y, lk, d);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = R(0);
    }
    plain_relax(L, d, fluid);
    unsigned w[5] = {0u, 0u, 0u, 0u, 0u};
    if constexpr (SR) sr_words((unsigned)(y * (int)nx + x), tkey, w);
    const O pl = (O)L.plane * (O)sizeof(S);
    LB2D_GLOBAL char *__restrict__ fout = (LB2D_GLOBAL char *)gbl(L.fout);
    const O s = brick_off<S, O>((unsigned)x, (unsigned)y, pnx);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const S e = plain_enc<S, SR>(d[i], i, w);
        if constexpr (NT) st_stream((LB2D_GLOBAL S *)(fout + (O)i * pl + s), e);
        else *(LB2D_GLOBAL S *)(fout + (O)i * pl + s) = e;
    }
}

// Node of a TX-wide tile handled by thread t: BW x BH consecutive threads
// cover one brick, the tile's bricks in row-major order, so a wavefront's
// loads and stores of one plane touch whole bricks (four 64-byte FP32
// bricks, two 64-byte 16-bit bricks, two 256-byte FP64 bricks).
template <int TX, int BW, int BH>
__device__ __forceinline__ void tile_thread(int t, int &lx, int &ly) {
    constexpr int BPR = TX / BW;
    const int b = t / (BW * BH), k = t % (BW * BH);
    lx = (b % BPR) * BW + k % BW;
    ly = (b / BPR) * BH + k / BW;
}

// Thread t of a 256-thread block of the one-fluid step -> node of a tile of
// (256 / (BW*BH)) bricks side by side (64x4 nodes for 4-byte values, 32x8
// for 2-byte values, 64x4 for 8-byte values).
template <typename S>
__device__ __forceinline__ void brick_thread(int t, int &lx, int &ly) {
    constexpr int W = brick_w_for(sizeof(S)), H = brick_h_for(sizeof(S));
    tile_thread<256 / (W * H) * W, W, H>(t, lx, ly);
}

// k: offset of this step in its launch group (the step computed is the
// device step count + k + 1; only stochastic rounding reads it).
template <typename S, typename O, bool SR, bool NT>
__global__ void __launch_bounds__(256) k_plain(PlainLattice L, int parity, int k) {
    constexpr int TW = 256 / (brick_w_for(sizeof(S)) * brick_h_for(sizeof(S))) * brick_w_for(sizeof(S)),
                  TH = brick_h_for(sizeof(S));
    int lx, ly;
    brick_thread<S>(threadIdx.x, lx, ly);
    const int x = blockIdx.x * TW + lx;
    const int y = blockIdx.y * TH + ly;
    unsigned tkey = 0u;
    if constexpr (SR) tkey = lowbias32((unsigned)(*L.step + (unsigned long long)k + 1ull) ^ L.seed);
    plain_node<S, O, SR, NT>(plain_args<S>(L, parity), x, y, x < L.nx && y < L.ny, tkey);
}

// NS steps in one pass (temporal blocking, NS = kMultiSteps).  A block of
// TW x TH threads owns a tile of whole bricks; one LDS region holds the tile
// and NS - 1 rings of nodes around it, in the storage format (every value
// rounded exactly as a store would round it):
//  * step 1 for the tile and all the rings, pulled from the input buffer as
//    in the one-step kernel, into LDS;
//  * step s = 2 .. NS-1 for the tile and rings 1 .. NS-s, pulled from LDS
//    into registers and, after a barrier, written back to the same slots;
//  * step NS for the tile, pulled from LDS and written to the output buffer
//    as whole bricks.
// So the populations cross HBM once per NS steps, and the results are those
// of NS one-step launches bit for bit.  NS is odd: a launch reads buffer p
// and writes p^1, so after every launch the state lies in the buffer its
// step count names.  Ring nodes wrap periodically with one conditional add
// or subtract; the host requires the lattice to hold the whole region
// (nx >= TW + 2(NS-1), ny >= TH + 2(NS-1)).  Thread t below the total ring
// size owns one ring node (inner rings first) for every step that needs it.
// k: offset of the first of the NS steps in its launch group, as in k_plain.
// (kMultiSteps, kMultiTW and kMultiTH are in lb2d_common.hpp.)

// The first step of node (x, y) into LDS slot `slot` (planes of PL
// elements); returns the node's link word.
template <typename S, typename O, bool SR, int PL>
__device__ __forceinline__ unsigned plain_stage(const PlainArgs<S> &L, unsigned x, unsigned y, int slot, S *sf,
                                                unsigned tkey) {
    using R = typename Codec<S>::R;
    const unsigned lk = (unsigned)gbl(L.links)[y * L.nx + x];
    const bool fluid = (lk & 1u) == 0u;
    if (__ballot(fluid) == 0ull || !fluid) return lk;
    R d[9];
    plain_pull<S, O>(L, x, y, lk, d);
    plain_relax(L, d, true);
    unsigned w[5] = {0u, 0u, 0u, 0u, 0u};
    if constexpr (SR) sr_words(y * L.nx + x, tkey, w);
#pragma unroll
    for (int i = 0; i < 9; ++i) sf[i * PL + slot] = plain_enc<S, SR>(d[i], i, w);
    return lk;
}

// LDS region of the NS-step kernel for a TW x TH tile: (TW + 2(NS-1)) x
// (TH + 2(NS-1)) slots per plane, rows padded to 8 slots; the tile sits at
// offset (NS-1, NS-1).  Ring r (r = 1 .. NS-1) surrounds the tile at
// distance r.
template <int TW, int TH, int NS>
struct MultiTile {
    static constexpr int O = NS - 1, AW = TW + 2 * O, AH = TH + 2 * O, PITCH = (AW + 7) / 8 * 8, PL = AH * PITCH;
    static constexpr int ring(int r) { return 2 * (TW + 2 * r) + 2 * (TH + 2 * r - 2); }
    static constexpr int rings(int m) { return m <= 0 ? 0 : rings(m - 1) + ring(m); }
    static constexpr int NR = rings(NS - 1);  // ring slots in all
};

// Slot s of ring r in region coordinates: the ring's first row, its last
// row, then its first and last columns without their corners.
template <int TW, int TH, int NS>
__device__ __forceinline__ void ring_slot(int s, int r, int &ax, int &ay) {
    const int w = TW + 2 * r, h = TH + 2 * r, o = NS - 1 - r;
    if (s < w) {
        ax = o + s;
        ay = o;
    } else if (s < 2 * w) {
        ax = o + s - w;
        ay = o + h - 1;
    } else if (s < 2 * w + h - 2) {
        ax = o;
        ay = o + 1 + s - 2 * w;
    } else {
        ax = o + w - 1;
        ay = o + 1 + s - 2 * w - (h - 2);
    }
}

// Pull of a node whose populations sit in LDS (slot c; rows of P slots,
// planes of PL), then its collision; d receives the post-collision
// deviations.  The slot of node - e_i in plane i, or (solid source) the
// node's own slot in plane opp(i), is c + K + wall * (opposite - K), so that
// the constant part folds into the LDS instruction's offset.  Solid lanes
// read one of the two slots too (inside the region, whatever it holds):
// plain_relax zeroes their output.
template <typename S, int P, int PL>
__device__ __forceinline__ void lds_pull_relax(const PlainArgs<S> &a, const S *sf, int c, unsigned lk, bool fluid,
                                               typename Codec<S>::R (&d)[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int K = i * PL - ey(i) * P - ex(i);
        const int wall = (int)((lk >> opp(i)) & 1u);
        d[i] = Codec<S>::dec(sf[c + wall * (opp(i) * PL - K) + K], i);
    }
    plain_relax(a, d, fluid);
}

// The NS steps of the tile at (x0, y0) by a block of TW x TH threads; key:
// stochastic-rounding keys of the NS steps; sf: the block's LDS region (9
// planes).  No thread leaves before the last barrier, so a block may run
// several tiles in a row (the caller separates them by a barrier).
// A value held in a vector register: a multiply-add may take one scalar
// operand, so a uniform force term kept in a vector register spares the
// copy into one that every collision would otherwise need.
template <typename R>
__device__ __forceinline__ R in_vgpr(R v) {
    asm("" : "=v"(v) : "0"(v));
    return v;
}

template <typename S, typename O, bool SR, bool NT, int TW, int TH, int NS>
__device__ __forceinline__ void multi_tile(const PlainArgs<S> &a0, int x0, int y0, const unsigned (&key)[NS], S *sf) {
    PlainArgs<S> a = a0;
    a.Fx = in_vgpr(a0.Fx);
    a.Fy = in_vgpr(a0.Fy);
    using C = Codec<S>;
    using R = typename C::R;
    using T = MultiTile<TW, TH, NS>;
    constexpr int W = brick_w_for(sizeof(S)), H = brick_h_for(sizeof(S)), G = W * H;
    constexpr int P = T::PITCH, PL = T::PL, OF = T::O;
    static_assert(TW % W == 0 && TH % H == 0 && T::NR <= TW * TH, "tile of whole bricks");
    const int nx = (int)a.nx, ny = (int)a.ny;
    const int t = threadIdx.x;
    int lx, ly;
    tile_thread<TW, W, H>(t, lx, ly);
    // the thread's own node (wrapped when the tile overhangs the lattice:
    // such slots hold the nodes past the lattice's last row or column)
    const int gx = x0 + lx, gy = y0 + ly;
    const unsigned ux = (unsigned)(gx < nx ? gx : gx - nx), uy = (unsigned)(gy < ny ? gy : gy - ny);
    const int c = (ly + OF) * P + lx + OF;
    // step 1: the own node, and the thread's ring node (ring rr, slot rc)
    const unsigned lk = plain_stage<S, O, SR, PL>(a, ux, uy, c, sf, key[0]);
    int rc = -1, rr = NS;
    unsigned rlk = 1u, rx = 0u, ry = 0u;
    if (t < T::NR) {
        int q = t, r = 1;
        while (q >= T::ring(r)) {
            q -= T::ring(r);
            ++r;
        }
        int ax, ay;
        ring_slot<TW, TH, NS>(q, r, ax, ay);
        int qx = x0 - OF + ax, qy = y0 - OF + ay;
        qx = qx < 0 ? qx + nx : (qx >= nx ? qx - nx : qx);
        qy = qy < 0 ? qy + ny : (qy >= ny ? qy - ny : qy);
        rlk = plain_stage<S, O, SR, PL>(a, (unsigned)qx, (unsigned)qy, ay * P + ax, sf, key[0]);
        rc = ay * P + ax;
        rr = r;
        rx = (unsigned)qx;
        ry = (unsigned)qy;
    }
    __syncthreads();
    // steps 2 .. NS-1: the own node and (while its ring is still needed)
    // the ring node into registers; then, once every thread has read, back
    // to their LDS slots
    const bool fl = (lk & 1u) == 0u;
    R d[9], e[9];
    unsigned w[5] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll 1
    for (int st = 1; st < NS - 1; ++st) {
        const bool rfl = rr <= NS - 1 - st && (rlk & 1u) == 0u;
        if (fl) lds_pull_relax<S, P, PL>(a, sf, c, lk, true, d);
        if (rfl) lds_pull_relax<S, P, PL>(a, sf, rc, rlk, true, e);
        __syncthreads();
        if (fl) {
            if constexpr (SR) sr_words(uy * a.nx + ux, key[st], w);
#pragma unroll
            for (int i = 0; i < 9; ++i) sf[i * PL + c] = plain_enc<S, SR>(d[i], i, w);
        }
        if (rfl) {
            if constexpr (SR) sr_words(ry * a.nx + rx, key[st], w);
#pragma unroll
            for (int i = 0; i < 9; ++i) sf[i * PL + rc] = plain_enc<S, SR>(e[i], i, w);
        }
        __syncthreads();
    }
    // step NS: the tile's nodes from LDS; a brick is written iff it holds a
    // fluid node
    const bool inside = gx < nx && gy < ny;
    const bool fluid = inside && fl;
    const unsigned long long bal = __ballot(fluid);
    const unsigned lane = __lane_id();
    const unsigned long long gmask = (G >= 64) ? ~0ull : (((1ull << (G & 63)) - 1ull) << ((lane / G) * G));
    if (inside && (bal & gmask) != 0ull) {
        lds_pull_relax<S, P, PL>(a, sf, c, lk, fluid, d);
        if constexpr (SR) sr_words((unsigned)(gy * nx + gx), key[NS - 1], w);
        const O pl = (O)a.plane * (O)sizeof(S);
        LB2D_GLOBAL char *__restrict__ fout = (LB2D_GLOBAL char *)gbl(a.fout);
        const O s = brick_off<S, O>((unsigned)gx, (unsigned)gy, a.pnx);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const S v = plain_enc<S, SR>(d[i], i, w);
            if constexpr (NT) st_stream((LB2D_GLOBAL S *)(fout + (O)i * pl + s), v);
            else *(LB2D_GLOBAL S *)(fout + (O)i * pl + s) = v;
        }
    }
}

// Keys of the stochastic rounding of steps st + 1 .. st + NS.
template <int NS>
__device__ __forceinline__ void sr_keys(unsigned long long st, unsigned seed, unsigned (&key)[NS]) {
#pragma unroll
    for (int j = 0; j < NS; ++j) key[j] = lowbias32((unsigned)(st + 1ull + (unsigned long long)j) ^ seed);
}

template <typename S, typename O, bool SR, bool NT, int TW, int TH, int NS>
__global__ void __launch_bounds__(TW *TH) k_plain_ms(PlainLattice L, int parity, int k) {
    __shared__ S sf[9 * MultiTile<TW, TH, NS>::PL];
    unsigned key[NS] = {};
    if constexpr (SR) sr_keys<NS>(*L.step + (unsigned long long)k, L.seed, key);
    multi_tile<S, O, SR, NT, TW, TH, NS>(plain_args<S>(L, parity), blockIdx.x * TW, blockIdx.y * TH, key, sf);
}

// Batched NS-step kernel: blocks walk a table of TW x TH tiles of many
// lattices, as k_batch does, each tile as in k_plain_ms (every lattice of
// the batch holds the whole region).
template <typename S, typename O, bool SR, bool NT, int TW, int TH, int NS>
__global__ void __launch_bounds__(TW *TH) k_batch_ms(const PlainLattice *__restrict__ lat,
                                                    const Tile *__restrict__ tiles, int ntiles, int parity, int k,
                                                    const unsigned long long *__restrict__ bstep) {
    __shared__ S sf[9 * MultiTile<TW, TH, NS>::PL];
    unsigned long long step = 0ull;
    if constexpr (SR) step = *bstep + (unsigned long long)k;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int li = (int)ufl((unsigned)tiles[t].lattice);
        const int x0 = (int)ufl((unsigned)tiles[t].x0), y0 = (int)ufl((unsigned)tiles[t].y0);
        const PlainArgs<S> a = uniform_args(plain_args<S>(lat[li], parity));
        unsigned key[NS] = {};
        if constexpr (SR) {
            sr_keys<NS>(step, lat[li].seed, key);
#pragma unroll
            for (int j = 0; j < NS; ++j) key[j] = ufl(key[j]);
        }
        if (t != (int)blockIdx.x) __syncthreads();  // the previous tile's LDS reads are done
        multi_tile<S, O, SR, NT, TW, TH, NS>(a, x0, y0, key, sf);
    }
}

// Batched step: blocks walk a table of tiles (lattice, x0, y0) of many
// independent lattices; `persistent` grids stride over the table.  A tile
// is TX nodes wide and 256 / TX nodes high (whole bricks; the autotuner
// picks TX).  With stochastic rounding each lattice draws the random words
// it would draw stepped alone (its seed and node numbering, and the step
// count, which all lattices of a batch share: `bstep`, read once per
// block); k is the step's offset in its launch group, as in k_plain.
template <typename S, typename O, bool SR, bool NT, int TX>
__global__ void __launch_bounds__(256) k_batch(const PlainLattice *__restrict__ lat,
                                              const Tile *__restrict__ tiles, int ntiles,
                                              int parity, int k,
                                              const unsigned long long *__restrict__ bstep) {
    constexpr int W = brick_w_for(sizeof(S)), H = brick_h_for(sizeof(S));
    static_assert(TX % W == 0 && (256 / (W * H)) % (TX / W) == 0, "tile of whole bricks");
    int lx, ly;
    tile_thread<TX, W, H>(threadIdx.x, lx, ly);
    unsigned long long step = 0ull;
    if constexpr (SR) step = *bstep + (unsigned long long)k + 1ull;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int li = (int)ufl((unsigned)tiles[t].lattice);
        const int x0 = (int)ufl((unsigned)tiles[t].x0), y0 = (int)ufl((unsigned)tiles[t].y0);
        const PlainArgs<S> a = uniform_args(plain_args<S>(lat[li], parity));
        unsigned tkey = 0u;
        if constexpr (SR) tkey = ufl(lowbias32((unsigned)step ^ lat[li].seed));
        const int x = x0 + lx;
        const int y = y0 + ly;
        plain_node<S, O, SR, NT>(a, x, y, x < (int)a.nx && y < (int)a.ny, tkey);
    }
}

// --------------------------------------------------------- general step

constexpr int kTX = 32;   // tile width (nodes, whole bricks)
constexpr int kTY = 8;    // tile height (nodes, whole 4-node bricks); measured:
                          // 32x8 and 16x16 beat 64x4, 32x4, 64x8, 128x4, 128x8

template <typename S>
__device__ __forceinline__ typename Codec<S>::R ldpop(const S *__restrict__ f, size_t a, int i) {
    return Codec<S>::dec(f[a], i);
}

// Reactive half-way link (surface_reaction command, App. C, applied per
// link): k_i = kr w_i / W (W = 1/6 for D2Q9, 1/4 for D2Q4, so the links of
// a flat wall add up to kr); the link concentration
// C_i = (2 g_out + k_i Cs) / (2 w_i + k_i), the returning population
// g_in = 2 w_i C_i - g_out, and the deposit g_out - g_in if positive,
// otherwise plain bounce-back.  For D2Q4 this is the rule as printed.
// Eliminating C_i and g_in gives the deposit as one multiply-add,
// g_out - g_in = 2 k_i / (2 w_i + k_i) (g_out - w_i Cs) = a g_out - a w_i Cs,
// with a (rlink) and a w_i Cs (rlink_cs) passed by the host for axial and
// diagonal links; g_in = g_out - deposit.
template <int SQ, typename R>
__device__ __forceinline__ R link_deposit(int i, const StepCoef<R> &q, R g_out) {
    const int k = i <= 4 ? 0 : 1;
    const R db = q.rlink[k] * g_out - q.rlink_cs[k];
    return db > R(0) ? db : R(0);
}

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Maps the linear block id to a tile so that each XCD (blocks are dealt
// round-robin over 8 XCDs) works on one contiguous band of tile rows.
__device__ __forceinline__ int xcd_band(int b, int nblk) {
    const int per = nblk / 8, rem = nblk % 8;
    const int xcd = b % 8, k = b / 8;
    // the first `rem` XCDs take one extra tile
    const int start = xcd * per + (xcd < rem ? xcd : rem);
    const int len = per + (xcd < rem ? 1 : 0);
    return (k < len) ? start + k : -1;
}


// psi(rho) = psi0 exp(-rho0 / rho) of the one-component interforce and
// adhesiveforce commands.
__device__ __forceinline__ float psi_of(float psi0, float rho0, float rho) { return psi0 * expf(-rho0 / rho); }
__device__ __forceinline__ double psi_of(double psi0, double rho0, double rho) { return psi0 * exp(-rho0 / rho); }

// Zou-He closure at a node of a momentum opening on wall W (inlet_momentum
// command, App. A), in deviation form d_i = f_i - w_i rho_ref.  With n the
// inward normal, t the tangent, T the populations along the wall and O
// those leaving the domain, rho (1 - u.n) = rho_ref + sum_T d + 2 sum_O d
// (the weights of T and twice O add up to 1); each entering population is
// its opposite plus (2/3) rho u.n (axial) or
// -(1/2) (e.t)(d_t - d_-t) + (1/6) rho u.n (diagonal); zero tangential
// velocity.  Velocity styles give u.n, dirichlet gives rho.
template <int W>
__host__ __device__ constexpr int wall_en(int i) {
    return W == 0 ? ex(i) : W == 1 ? -ex(i) : W == 2 ? ey(i) : -ey(i);
}
template <int W>
__host__ __device__ constexpr int wall_et(int i) {
    return W < 2 ? ey(i) : ex(i);
}
template <int W, typename R>
__device__ __forceinline__ void zou_he(R (&d)[9], bool pressure, R given, R rho_ref) {
    R sT = R(0), sO = R(0), tp = R(0), tm = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (wall_en<W>(i) == 0) {
            sT += d[i];
            if (wall_et<W>(i) == 1) tp = d[i];
            if (wall_et<W>(i) == -1) tm = d[i];
        } else if (wall_en<W>(i) < 0) {
            sO += d[i];
        }
    }
    const R known = rho_ref + sT + R(2) * sO;
    R rho, un;
    if (pressure) {
        rho = given;
        un = R(1) - known / rho;
    } else {
        un = given;
        rho = known / (R(1) - un);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (wall_en<W>(i) != 1) continue;
        d[i] = (wall_et<W>(i) == 0) ? d[opp(i)] + R(2.0 / 3.0) * rho * un
                                    : d[opp(i)] - R(0.5) * R(wall_et<W>(i)) * (tp - tm) + R(1.0 / 6.0) * rho * un;
    }
}

// Normal velocity u.n (n inward) of a velocity opening at coordinate k
// along its wall: the speed into the domain for an inlet, out of it for an
// outlet; poiseuille: v(k) = 4 v_max / L^2 [(L/2)^2 - ((2k - lo - hi)/2)^2],
// L = hi - lo + 1.
template <typename R>
__host__ __device__ __forceinline__ R opening_un(const OpenSpec &o, int k) {
    R sp = R(o.v);
    if (o.style == 1) {
        const R L = R(o.hi - o.lo + 1), h = R(2 * k - o.lo - o.hi) / R(2);
        sp = R(4) * R(o.v) / (L * L) * (L * L / R(4) - h * h);
    }
    return o.outlet ? -sp : sp;
}

// Population loads and stores at byte offsets from an array base.
template <typename S, typename O>
__device__ __forceinline__ typename Codec<S>::R ldb(const S *__restrict__ base, O off, int i) {
    return Codec<S>::dec(*(const S *)((const char *)base + off), i);
}
// The general step always stores streaming: a uniform run-time choice
// between streaming and plain stores measured 7% slower on the two-fluid +
// solute workload than either form alone, and streaming stores won on
// every general-step workload measured.
template <typename S, typename O>
__device__ __forceinline__ void stb(S *__restrict__ base, O off, S v) {
    st_stream((LB2D_GLOBAL S *)((LB2D_GLOBAL char *)gbl(base) + off), v);
}

// Slip rule of the boundary_style command at diagonal mode k of node
// (lx, ly) of the tile (mask tile sm with a kSlipRing-node ring): 1 if
// the mode, heading into a solid, reflects off a horizontal wall (cell
// across y solid, cell across x fluid) and lands two nodes along x, 2 if it
// reflects off a vertical wall and lands two nodes along y, 0 if it bounces
// back (a corner, or a solid landing node).  Reads the mask at most two
// nodes from (lx, ly) on each axis.
constexpr int kSlipRing = 3;
template <int MH, int MW>
__device__ __forceinline__ int slip_branch(const uint8_t (&sm)[MH][MW], int lx, int ly, int k) {
    const int kx = ex(k), ky = ey(k);
    const int cx = lx + kSlipRing, cy = ly + kSlipRing;
    const bool sy = sm[cy + ky][cx] != 0, sx = sm[cy][cx + kx] != 0;
    if (sy && !sx && !sm[cy][cx + 2 * kx]) return 1;
    if (sx && !sy && !sm[cy + 2 * ky][cx]) return 2;
    return 0;
}

// Diagonal population i arriving at fluid node (x, y) (tile position
// lx, ly) whose source T = node - e_i is solid with reflected share R:
// the node's own mode opp(i) that hit T returns with weight 1 - R when it
// has a slip branch (1 otherwise); modes mirrored off the wall at T arrive
// with weight R from node - (2 ex_i, 0) (horizontal wall, mode
// (ex_i, -ey_i)) and from node - (0, 2 ey_i) (vertical wall, mode
// (-ex_i, ey_i)).  own = the bounce-back value d_opp(i)(node).  Values are
// stored shifted by w rho_ref (the same w = 1/36 for every diagonal), so
// the weights' sum minus one times w rho_ref is added back: the rule moves
// mass between nodes and its weights need not sum to one at a node.
template <typename S, typename O, typename R, int MH, int MW>
__device__ __forceinline__ R slip_diagonal(const FullParams &p, int c, const S *__restrict__ fin, O pl,
                                           const uint8_t (&sm)[MH][MW], int lx, int ly, int x, int y, int i,
                                           R own, R rho_ref) {
    const int ax = ex(i), ay = ey(i);
    const double Rt = p.refl[c][(size_t)wrapi(y - ay, p.ny) * p.nx + wrapi(x - ax, p.nx)];
    if (!(Rt > 0.0)) return own;
    const R RR = R(Rt);
    const bool mine = slip_branch(sm, lx, ly, opp(i)) != 0;
    R v = mine ? (R(1) - RR) * own : own;
    R extra = mine ? -RR : R(0);
    const int cx = lx + kSlipRing, cy = ly + kSlipRing;
    // partner across x (horizontal wall): mode kh = (ax, -ay)
    const int kh = ax > 0 ? (ay > 0 ? 8 : 5) : (ay > 0 ? 7 : 6);
    if (!sm[cy][cx - 2 * ax] && slip_branch(sm, lx - 2 * ax, ly, kh) == 1) {
        const O a = brick_off<S, O>((unsigned)wrapi(x - 2 * ax, p.nx), (unsigned)y, p.pnx);
        v += RR * ldb(fin, (O)kh * pl + a, kh);
        extra += RR;
    }
    // partner across y (vertical wall): mode kv = (-ax, ay)
    const int kv = ax > 0 ? (ay > 0 ? 6 : 7) : (ay > 0 ? 5 : 8);
    if (!sm[cy - 2 * ay][cx] && slip_branch(sm, lx, ly - 2 * ay, kv) == 2) {
        const O a = brick_off<S, O>((unsigned)x, (unsigned)wrapi(y - 2 * ay, p.ny), p.pnx);
        v += RR * ldb(fin, (O)kv * pl + a, kv);
        extra += RR;
    }
    return v + R(1.0 / 36.0) * rho_ref * extra;
}

// Applies the openings of component c that hold node (x, y) (Zou-He styles
// only; gradient openings act after the collision, in k_open_gradient).
template <typename R>
__device__ __forceinline__ void apply_openings(const FullParams &p, int c, int x, int y, R (&d)[9], R rho_ref) {
    for (int k = 0; k < p.nopen; ++k) {
        const OpenSpec &o = p.open[k];
        if (o.comp != c || o.style > 3) continue;
        const int pos = o.wall < 2 ? y : x;
        const bool on = (o.wall == 0 ? x == 0 : o.wall == 1 ? x == p.nx - 1 : o.wall == 2 ? y == 0 : y == p.ny - 1) &&
                        pos >= o.lo && pos <= o.hi;
        if (!on) continue;
        const bool pressure = o.style == 3;
        const R given = pressure ? R(o.rho) : opening_un<R>(o, pos);
        switch (o.wall) {
            case 0: zou_he<0>(d, pressure, given, rho_ref); break;
            case 1: zou_he<1>(d, pressure, given, rho_ref); break;
            case 2: zou_he<2>(d, pressure, given, rho_ref); break;
            default: zou_he<3>(d, pressure, given, rho_ref); break;
        }
    }
}

// Solute openings.  Node (cx, cy) lies outside the box across a wall of a
// non-periodic solute axis.
__device__ __forceinline__ bool across_closed(const FullParams &p, int cx, int cy) {
    return (!p.sxper && (cx < 0 || cx >= p.nx)) || (!p.syper && (cy < 0 || cy >= p.ny));
}
// Population i of a node on wall w enters the domain across that wall
// (its source lies outside): e_i . n > 0, n the inward normal.
template <int SQ>
__device__ __forceinline__ bool enters_across(int w, int i) {
    return shas<SQ>(i) && (w == 0 ? ex(i) > 0 : w == 1 ? ex(i) < 0 : w == 2 ? ey(i) > 0 : ey(i) < 0);
}
// y-mirror (ey -> -ey): 2<->4, 5<->8, 6<->7.
__host__ __device__ constexpr int miry(int i) {
    return i == 2 ? 4 : i == 4 ? 2 : i == 5 ? 8 : i == 8 ? 5 : i == 6 ? 7 : i == 7 ? 6 : i;
}
// The solute opening that holds node (x, y), or -1.
__device__ __forceinline__ int find_solute_opening(const FullParams &p, int x, int y) {
    int k = -1;
    for (int j = 0; j < p.nsopen; ++j) {
        const SoluteOpen &o = p.sopen[j];
        const int pos = o.wall < 2 ? y : x;
        const bool on = o.wall == 0 ? x == 0 : o.wall == 1 ? x == p.nx - 1 : o.wall == 2 ? y == 0 : y == p.ny - 1;
        if (on && pos >= o.lo && pos <= o.hi) k = j;
    }
    return k;
}

// Halo slot j of a TX x TY tile's density ring -> position in the
// (TX+2) x (TY+2) tile: bottom row, top row, then left/right columns.
template <int TX, int TY>
__device__ __forceinline__ void halo_slot(int j, int &hx, int &hy) {
    if (j < TX + 2) {
        hx = j;
        hy = 0;
    } else if (j < 2 * (TX + 2)) {
        hx = j - (TX + 2);
        hy = TY + 1;
    } else {
        const int k = j - 2 * (TX + 2);
        hx = (k & 1) ? TX + 1 : 0;
        hy = 1 + k / 2;
    }
}

// Sum of three doubles over a wavefront (fixed butterfly order).
__device__ __forceinline__ void wave_sum3(double (&v)[4]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double a = v[k];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        v[k] = a;
    }
}

// General fused step on the brick layout.  One thread per node of a
// TX x TY tile:
//  1. one 16-bit link word per node (bit 0: solid; bit i: node + e_i
//     solid) gives every bounce-back, adhesion and surface decision;
//  2. pull both components (fluid lanes), with the slip/mixed rule for
//     diagonal modes that hit such solids and the Zou-He closure at
//     momentum openings; solute pull with bounce-back or reactive link at
//     walls and the opening rules on open walls;
//     solid lanes next to fluid gather the deposit of their reactive links;
//  3. densities of the tile plus a one-node halo in LDS -- the halo nodes'
//     populations are pulled again (from L2) so that the Shan-Chen force
//     sees the post-stream densities of this step;
//  4. forces (aveforce, aveacceleration, cohesion, adhesion), the common
//     velocity u' and each component's equilibrium velocity, collision;
//  5. solute collision at the solvent velocity of Eq. (u_solvent), plus
//     tau_s F / C of the intersolute force (psi(C) of the tile and its ring
//     in LDS, from the concentrations after streaming);
//  6. deposits and growth decisions of solid lanes next to fluid.
// A brick is stored iff it holds a fluid node (solid lanes store zeros),
// so every store writes whole lines and all-solid bricks move no data.
// EXT instantiations carry the features most lattices lack (momentum
// openings, slip/mixed solids, intersolute), each switched on at run time.
// Population addresses are byte offsets of type O from the array base:
// 32-bit when the arrays are below 4 GiB (a uniform base plus a 32-bit
// lane offset, no 64-bit lane arithmetic), 64-bit otherwise.
// Tallies (inflow, outflow, consumed deposit) go to one running slot per
// wavefront, summed in a fixed order only when budgets are read.
template <typename R>
__device__ __forceinline__ const StepCoef<R> &coef(const FullParams &p);
template <>
__device__ __forceinline__ const StepCoef<double> &coef<double>(const FullParams &p) { return p.cd; }
template <>
__device__ __forceinline__ const StepCoef<float> &coef<float>(const FullParams &p) { return p.cf; }

// Solute populations arriving at fluid node (x, y) (inside the box) after
// streaming (solute command): bounce-back, or the reactive link rule, at
// solid sources; bounce-back across a closed wall of a non-periodic solute
// axis; and the rules of the solute opening that holds the node
// (inlet_solute/outlet_solute, App. B).  lk is the node's link word, s and
// src the brick offsets of the node and of node - e_i.  Adds the opening's
// inflow to tal[0] and the populations that left through it to tal[1]; a
// node of a flux opening returns flux = true and its concentration Cf.
template <typename S, typename O, int SQ, bool REACT, typename R>
__device__ __forceinline__ void solute_pull(const FullParams &p, const StepCoef<R> &q, const S *__restrict__ gin,
                                            O pl, int x, int y, unsigned lk, O s, const O (&src)[9], R (&g)[9],
                                            double (&tal)[4], bool &flux, R &Cf) {
    const int nx = p.nx, ny = p.ny;
    const unsigned pnx = p.pnx;
    // nodes on a wall of a non-periodic solute axis
    const bool edge = (!p.sxper && (x == 0 || x == nx - 1)) || (!p.syper && (y == 0 || y == ny - 1));
    const int kop = edge ? find_solute_opening(p, x, y) : -1;
    const int kw = kop >= 0 ? p.sopen[kop].wall : -1;
    bool unk[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        unk[i] = false;
        if (!shas<SQ>(i)) continue;
        // a pull across a closed wall bounces back; across the wall of this
        // node's opening the population is unknown
        const int sxr = x - ex(i), syr = y - ey(i);
        const bool cross = edge && ((!p.sxper && (sxr < 0 || sxr >= nx)) || (!p.syper && (syr < 0 || syr >= ny)));
        unk[i] = kw >= 0 && enters_across<SQ>(kw, i);
        const bool solid_src = ((lk >> opp(i)) & 1u) && !cross;
        const bool bb = solid_src || cross;
        const O a = bb ? (O)spl<SQ>(opp(i)) * pl + s : (O)spl<SQ>(i) * pl + src[i];
        R v = ldb(gin, a, i);
        if constexpr (REACT) {
            // a select, not a branch: the nine loads stay issued together
            const R gi = v - link_deposit<SQ, R>(i, q, v);
            v = solid_src ? gi : v;
        }
        g[i] = v;
    }
    if (kop >= 0) {
        const SoluteOpen &o = p.sopen[kop];
        R known = R(0), wu = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if (!shas<SQ>(i)) continue;
            if (unk[i]) wu += swgt<SQ, R>(i);
            else known += g[i];
        }
        if (o.style == 1) {
            // dirichlet: the unknowns share Cbar - C' by weight
            const R deficit = (R(o.value) - known) * rcp(wu);
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (unk[i]) {
                    g[i] = swgt<SQ, R>(i) * deficit;
                    tal[0] += (double)g[i];
                }
        } else if (o.style == 2) {
            // adiabatic: each unknown copies its mirror across the wall
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (unk[i]) {
                    g[i] = kw < 2 ? g[mirx(i)] : g[miry(i)];
                    tal[0] += (double)g[i];
                }
        } else {
            // flux (App. B): C = (v C0 + D C1)/(D + v) at an inlet,
            // (v C0 - D C1)/(v - D) at an outlet, C1 the concentration of
            // the next node inward at the previous time level (0 if it is
            // solid)
            const int nxw = kw == 0 ? 1 : kw == 1 ? -1 : 0, nyw = kw == 2 ? 1 : kw == 3 ? -1 : 0;
            const int in_dir = kw == 0 ? 1 : kw == 1 ? 3 : kw == 2 ? 2 : 4;  // e_in = n
            const O s1 = brick_off<S, O>((unsigned)(x + nxw), (unsigned)(y + nyw), pnx);
            R C1 = R(0);
            if (!((lk >> in_dir) & 1u)) {
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    if (shas<SQ>(i)) C1 += ldb(gin, (O)spl<SQ>(i) * pl + s1, i);
            }
            const R v = R(o.v), C0 = R(o.value), D = q.Dsol;
            Cf = o.outlet ? (v * C0 - D * C1) / (v - D) : (v * C0 + D * C1) / (D + v);
            flux = true;
            tal[0] += (double)(Cf - known);
        }
        // populations of the previous step that left through the opening
#pragma unroll
        for (int i = 1; i < 9; ++i)
            if (shas<SQ>(i) && enters_across<SQ>(kw, opp(i)))
                tal[1] += (double)ldb(gin, (O)spl<SQ>(i) * pl + s, i);
    }
}

template <typename S, typename O, int NC, bool SC, int SQ, bool REACT, bool EXT, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_full(FullParams p, int parity) {
    using C = Codec<S>;
    using R = typename C::R;
    constexpr bool SOL = SQ != 0;
    constexpr O SB = (O)sizeof(S);
    constexpr int BW = brick_w_for(sizeof(S)), BH = brick_h_for(sizeof(S));
    static_assert(TX % BW == 0 && TY % BH == 0, "tile of whole bricks");
    __shared__ R srho[SC ? NC : 1][SC ? TY + 2 : 1][SC ? TX + 2 : 1];
    // mask tile with a kSlipRing-node ring for the slip rules: the rule
    // reads two nodes around a node, and the density halo lies one node out
    __shared__ uint8_t smask[EXT ? TY + 2 * kSlipRing : 1][EXT ? TX + 2 * kSlipRing : 1];
    // psi(C) of the intersolute force with a one-node ring
    __shared__ R spsi[EXT && SOL ? TY + 2 : 1][EXT && SOL ? TX + 2 : 1];
    const StepCoef<R> &q = coef<R>(p);

    const int nx = p.nx, ny = p.ny;
    const unsigned pnx = p.pnx;
    const O pl = (O)p.pplane * SB;  // bytes per plane
    const uint16_t *__restrict__ links = p.links;
    const int tiles_x = (nx + TX - 1) / TX;
    int tile = xcd_band(blockIdx.x, gridDim.x);
    if (tile < 0) tile = blockIdx.x;
    const int tx0 = (tile % tiles_x) * TX, ty0 = (tile / tiles_x) * TY;
    const int tid = threadIdx.x;
    int lx, ly;
    tile_thread<TX, BW, BH>(tid, lx, ly);
    const int x = tx0 + lx, y = ty0 + ly;
    const bool valid = (x < nx) && (y < ny);
    // lanes past a ragged lattice edge stand for the periodic image of their
    // position: the density tile needs its density, nothing else of theirs
    // is loaded or stored
    const unsigned ux_ = (unsigned)(x % nx), uy_ = (unsigned)(y % ny);
    const size_t srow = (size_t)uy_ * nx + ux_;
    const unsigned lk = links[srow];
    const bool solid = (lk & 1u) != 0u;
    const bool fluid = !solid;
    const bool pull = fluid && (valid || SC);
    // a brick is stored iff it holds a fluid node
    const unsigned long long bal = __ballot(valid && fluid);
    const unsigned lane = __lane_id();
    constexpr unsigned kG = BW * BH;  // lanes per brick
    const bool store = valid && ((bal >> ((lane / kG) * kG)) & ((1ull << kG) - 1ull)) != 0ull;

    if constexpr (EXT) {
        if (p.slip) {
            constexpr int MW = TX + 2 * kSlipRing, MH = TY + 2 * kSlipRing;
            for (int k = tid; k < MW * MH; k += TX * TY) {
                const int mx = k % MW, my = k / MW;
                smask[my][mx] = p.mask[(size_t)wrapi(ty0 + my - kSlipRing, ny) * nx + wrapi(tx0 + mx - kSlipRing, nx)];
            }
            __syncthreads();
        }
    }

    // the ring of the density tile: the NH halo slots are dealt to the
    // wavefronts in equal contiguous runs (lane l < PER of wavefront w owns
    // slot w * PER + l); a slot's link word is loaded with the own one and
    // its populations are pulled before the own ones, so that all loads of
    // the step are in flight together and the halo sums free their
    // registers first
    constexpr int NH = SC ? 2 * (TX + 2) + 2 * TY : 0;
    constexpr int NWV = TX * TY / 64, PER = (NH + NWV - 1) / NWV;
    static_assert(PER <= 64, "halo run fits a wavefront");
    const int hj = (tid & 63) < PER ? (tid >> 6) * PER + (tid & 63) : NH;  // NH: none
    int hx = 0, hy = 0;
    bool hpull = false;
    R hrho[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) hrho[c] = R(0);
    if constexpr (SC) {
        if (hj < NH) {
            halo_slot<TX, TY>(hj, hx, hy);
            const unsigned gx = (unsigned)wrapi(tx0 + hx - 1, nx), gy = (unsigned)wrapi(ty0 + hy - 1, ny);
            const unsigned hl = links[(size_t)gy * nx + gx];
            hpull = !(hl & 1u);
            if (hpull) {
                const unsigned gxm = (gx == 0) ? nx - 1 : gx - 1, gxp = (gx + 1 == (unsigned)nx) ? 0 : gx + 1;
                const unsigned gym = (gy == 0) ? ny - 1 : gy - 1, gyp = (gy + 1 == (unsigned)ny) ? 0 : gy + 1;
                O hsrc[9];
                brick_pulls<S, O>(gx, gy, gxm, gxp, gym, gyp, pnx, hsrc);
                const O hs = hsrc[0];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const S *__restrict__ fin = (const S *)p.f[parity][c];
                    R acc = ldb(fin, hs, 0);
#pragma unroll
                    for (int i = 1; i < 9; ++i) {
                        const bool wall = (hl >> opp(i)) & 1u;
                        const O a = wall ? (O)opp(i) * pl + hs : (O)i * pl + hsrc[i];
                        R v = ldb(fin, a, i);
                        if constexpr (EXT) {
                            if (p.slip && i >= 5 && wall)
                                v = slip_diagonal<S, O, R>(p, c, fin, pl, smask, hx - 1, hy - 1, (int)gx, (int)gy, i,
                                                           v, q.rho_ref[c]);
                        }
                        acc += v;
                    }
                    hrho[c] = q.rho_ref[c] + acc;
                }
            }
        }
    }

    // byte offsets of the node and of node - e_i (periodic) in a plane
    const unsigned xm = (ux_ == 0) ? nx - 1 : ux_ - 1, xp = (ux_ + 1 >= (unsigned)nx) ? 0 : ux_ + 1;
    const unsigned ym = (uy_ == 0) ? ny - 1 : uy_ - 1, yp = (uy_ + 1 >= (unsigned)ny) ? 0 : uy_ + 1;
    O src[9];
    brick_pulls<S, O>(ux_, uy_, xm, xp, ym, yp, pnx, src);
    const O s = src[0];

    // 1. pull both components at the own node
    R d[NC][9];
    R drho[NC], jx[NC], jy[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int i = 0; i < 9; ++i) d[c][i] = R(0);
        if (pull) {
            const S *__restrict__ fin = (const S *)p.f[parity][c];
            d[c][0] = ldb(fin, s, 0);
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const bool wall = (lk >> opp(i)) & 1u;
                const O a = wall ? (O)opp(i) * pl + s : (O)i * pl + src[i];
                d[c][i] = ldb(fin, a, i);
            }
        }
        if constexpr (EXT) {
            // slip / mixed solids: diagonal modes reflected off flat walls
            if (p.slip && pull) {
                const S *__restrict__ fin = (const S *)p.f[parity][c];
#pragma unroll
                for (int i = 5; i < 9; ++i)
                    if ((lk >> opp(i)) & 1u)
                        d[c][i] = slip_diagonal<S, O, R>(p, c, fin, pl, smask, lx, ly, (int)ux_, (int)uy_, i,
                                                         d[c][i], q.rho_ref[c]);
            }
            // momentum openings (only lanes on the box edge can hold one)
            if (p.nopen > 0 && valid && fluid && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1))
                apply_openings<R>(p, c, x, y, d[c], q.rho_ref[c]);
        }
        drho[c] = jx[c] = jy[c] = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            drho[c] += d[c][i];
            if (ex(i)) jx[c] += ex(i) > 0 ? d[c][i] : -d[c][i];
            if (ey(i)) jy[c] += ey(i) > 0 ? d[c][i] : -d[c][i];
        }
    }

    // 2. solute pull (issued before the density-tile barrier so that its
    // latency overlaps the halo pulls): bounce-back or reactive link at
    // walls, the opening rules on open walls
    R g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = R(0);
    double tal[4] = {0.0, 0.0, 0.0, 0.0};  // inflow, outflow, consumed deposit
    bool flux = false;   // node of a flux opening: all populations to g_eq(Cf)
    R Cf = R(0);
    if constexpr (SOL) {
        const S *__restrict__ gin = (const S *)p.g[parity];
        // lanes past a ragged edge pull too when the intersolute stencil
        // needs their concentration (their tallies are dropped)
        if ((valid || (EXT && p.isol)) && fluid)
            solute_pull<S, O, SQ, REACT, R>(p, q, gin, pl, (int)ux_, (int)uy_, lk, s, src, g, tal, flux, Cf);
        if constexpr (EXT) {
            if (!valid) tal[0] = tal[1] = 0.0;
        }
    }
    // intersolute: psi(C) of the tile and of its one-node ring, from the
    // concentrations after streaming (the ring nodes' solute populations are
    // pulled again); 0 on solids, where C <= 0 and across a wall of a
    // non-periodic solute axis
    if constexpr (EXT && SOL) {
        if (p.isol) {
            const R psi0 = R(p.is_psi0), C0 = R(p.is_C0);
            R Cn = R(0);
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (shas<SQ>(i)) Cn += g[i];
            if (flux) Cn = Cf;
            spsi[ly + 1][lx + 1] = (fluid && !across_closed(p, x, y) && Cn > R(0)) ? psi_of(psi0, C0, Cn) : R(0);
            const S *__restrict__ gin = (const S *)p.g[parity];
            for (int j = tid; j < 2 * (TX + 2) + 2 * TY; j += TX * TY) {
                int rx, ry;
                halo_slot<TX, TY>(j, rx, ry);
                const int cx = tx0 + rx - 1, cy = ty0 + ry - 1;
                R ps = R(0);
                if (!across_closed(p, cx, cy)) {
                    const unsigned gx = (unsigned)wrapi(cx, nx), gy = (unsigned)wrapi(cy, ny);
                    const unsigned hl = links[(size_t)gy * nx + gx];
                    if (!(hl & 1u)) {
                        const unsigned gxm = (gx == 0) ? nx - 1 : gx - 1, gxp = (gx + 1 == (unsigned)nx) ? 0 : gx + 1;
                        const unsigned gym = (gy == 0) ? ny - 1 : gy - 1, gyp = (gy + 1 == (unsigned)ny) ? 0 : gy + 1;
                        O hsrc[9];
                        brick_pulls<S, O>(gx, gy, gxm, gxp, gym, gyp, pnx, hsrc);
                        const O hs = hsrc[0];
                        R gh[9];
#pragma unroll
                        for (int i = 0; i < 9; ++i) gh[i] = R(0);
                        double th[4] = {0.0, 0.0, 0.0, 0.0};
                        bool fh = false;
                        R Ch = R(0);
                        solute_pull<S, O, SQ, REACT, R>(p, q, gin, pl, (int)gx, (int)gy, hl, hs, hsrc, gh, th, fh, Ch);
                        R Cr = R(0);
#pragma unroll
                        for (int i = 0; i < 9; ++i)
                            if (shas<SQ>(i)) Cr += gh[i];
                        if (fh) Cr = Ch;
                        if (Cr > R(0)) ps = psi_of(psi0, C0, Cr);
                    }
                }
                spsi[ry][rx] = ps;
            }
            __syncthreads();
        }
    }
    // deposit gathered by solid nodes next to fluid (loads issued early too):
    // the fluid neighbour node + e_i is node - e_opp(i)
    bool fluid8 = false, fluid4 = false;
    double dep = 0.0;
    if constexpr (REACT) {
        if (valid && solid) {
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                if (across_closed(p, x + ex(i), y + ey(i))) continue;
                if (!((lk >> i) & 1u)) {
                    fluid8 = true;
                    if (i <= 4) fluid4 = true;
                }
            }
            if (fluid8) {
                // the links' deposits are summed in the arithmetic type, then
                // added to the FP64 deposit
                const S *__restrict__ gin = (const S *)p.g[parity];
                R sum = R(0);
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    if (!shas<SQ>(i)) continue;
                    if (across_closed(p, x + ex(i), y + ey(i))) continue;
                    if ((lk >> i) & 1u) continue;
                    const R g_out = ldb(gin, (O)spl<SQ>(opp(i)) * pl + src[opp(i)], opp(i));
                    sum += link_deposit<SQ, R>(i, q, g_out);
                }
                dep = (double)sum;
            }
        }
    }

    // 3. density tile for the cohesion stencil: own nodes (and periodic
    // images past a ragged edge) and the pulled halo ring; one component
    // keeps psi(rho) instead of rho.  Solids hold 0.
    if constexpr (SC) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const R r = q.rho_ref[c] + drho[c];
            srho[c][ly + 1][lx + 1] = solid ? R(0) : (NC == 1 ? psi_of(q.psi0, q.rho0, r) : r);
        }
        if (hj < NH) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                srho[c][hy][hx] = hpull ? (NC == 1 ? psi_of(q.psi0, q.rho0, hrho[c]) : hrho[c]) : R(0);
        }
        __syncthreads();
    }

    // 4.-7. only wavefronts with a fluid node of the lattice collide and store
    // (all-solid wavefronts have nothing to store; all barriers are behind)
    if (bal != 0ull) {
        // 4. forces (solid lanes compute throw-away values from zero populations)
        R rho[NC], Fx[NC], Fy[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            rho[c] = q.rho_ref[c] + drho[c];
            Fx[c] = q.force[c][0] + rho[c] * q.accel[c][0];
            Fy[c] = q.force[c][1] + rho[c] * q.accel[c][1];
        }
        if constexpr (SC && NC == 2) {
            if (valid) {
                R sx[2] = {R(0), R(0)}, sy[2] = {R(0), R(0)};
#pragma unroll
                for (int i = 1; i < 9; ++i) {
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const R rb = srho[1 - c][ly + 1 + ey(i)][lx + 1 + ex(i)];
                        if (ex(i)) sx[c] += wgt<R>(i) * (ex(i) > 0 ? rb : -rb);
                        if (ey(i)) sy[c] += wgt<R>(i) * (ey(i) > 0 ? rb : -rb);
                    }
                }
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    Fx[c] += -q.G * rho[c] * sx[c];
                    Fy[c] += -q.G * rho[c] * sy[c];
                }
            }
        }
        if constexpr (SC && NC == 1) {
            // one component: F = -G psi(x) sum_i w_i psi(x + e_i) e_i
            if (valid) {
                R sx = R(0), sy = R(0);
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const R pb = srho[0][ly + 1 + ey(i)][lx + 1 + ex(i)];
                    if (ex(i)) sx += wgt<R>(i) * (ex(i) > 0 ? pb : -pb);
                    if (ey(i)) sy += wgt<R>(i) * (ey(i) > 0 ? pb : -pb);
                }
                const R ps = srho[0][ly + 1][lx + 1];
                Fx[0] += -q.G * ps * sx;
                Fy[0] += -q.G * ps * sy;
            }
        }
        if (p.has_ads) {
            R ax = R(0), ay = R(0);
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const R sv = ((lk >> i) & 1u) ? R(1) : R(0);
                if (ex(i)) ax += wgt<R>(i) * (ex(i) > 0 ? sv : -sv);
                if (ey(i)) ay += wgt<R>(i) * (ey(i) > 0 ? sv : -sv);
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                // two components: rho_c; one component: psi(rho) of adhesiveforce
                const R a = (NC == 1 && p.ads_psi) ? psi_of(q.psi0a, q.rho0a, rho[c]) : rho[c];
                Fx[c] += -q.Gads[c] * a * ax;
                Fy[c] += -q.Gads[c] * a * ay;
            }
        }
        // 5. common velocity u' and per-component equilibrium velocities
        R nux = R(0), nuy = R(0), den = R(0), sjx = R(0), sjy = R(0), srh = R(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const R om = q.omega[c];
            nux += jx[c] * om;
            nuy += jy[c] * om;
            den += rho[c] * om;
            sjx += jx[c] + R(0.5) * Fx[c];
            sjy += jy[c] + R(0.5) * Fy[c];
            srh += rho[c];
        }
        const R iden = rcp(den);
        const R upx = nux * iden, upy = nuy * iden;
        // 6. collide (in place)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const R tau = q.tau[c], om = q.omega[c];
            const R irho = rcp(rho[c]);
            const R ux = upx + tau * Fx[c] * irho;
            const R uy = upy + tau * Fy[c] * irho;
            const R usq = R(1.5) * (ux * ux + uy * uy);
            const R rr = q.rho_ref[c];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const R eu = R(ex(i)) * ux + R(ey(i)) * uy;
                const R A = (i == 0) ? q.A0[c] : q.A1[c];
                const R deq = wgt<R>(i) * (rho[c] * A - rr + rho[c] * (R(3) * eu + R(4.5) * eu * eu - usq));
                d[c][i] = fluid ? d[c][i] + om * (deq - d[c][i]) : R(0);
            }
        }
        // 7. solute collision at the solvent velocity (in place)
        if constexpr (SOL) {
            const R isrh = rcp(srh);
            R usx = sjx * isrh, usy = sjy * isrh;
            R Cc = R(0);
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (shas<SQ>(i)) Cc += g[i];
            if (flux) Cc = Cf;
            if constexpr (EXT) {
                // intersolute: u_s + tau_s F / C, F = -G psi(x) sum_{i=1..4}
                // psi(x + e_i) e_i over the four axis neighbours
                if (p.isol && Cc > R(0)) {
                    const R ps = spsi[ly + 1][lx + 1];
                    const R sx = spsi[ly + 1][lx + 2] - spsi[ly + 1][lx];
                    const R sy = spsi[ly + 2][lx + 1] - spsi[ly][lx + 1];
                    const R G = R(p.is_G), ts = R(p.tau_s);
                    usx = usx + ts * (-G * ps * sx) / Cc;
                    usy = usy + ts * (-G * ps * sy) / Cc;
                }
            }
            // flux-opening nodes take the equilibrium itself (relaxation 1)
            const R oms = flux ? R(1) : q.omega_s;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (!shas<SQ>(i)) continue;
                const R eu = R(ex(i)) * usx + R(ey(i)) * usy;
                const R geq = swgt<SQ, R>(i) * Cc * (R(1) + sics2<SQ, R>() * eu);
                g[i] = fluid ? g[i] + oms * (geq - g[i]) : R(0);
            }
        }
        // all stores of the lane in one region (streaming stores)
        if (store) {
            bool rne = true;
            if constexpr (sizeof(S) == 2) {
                if (p.sr) {
                    rne = false;
                    // stochastic rounding: five random words per node and plane
                    // group (component 0, component 1, solute), keyed on the node,
                    // the step being computed and the group
                    const unsigned tkey = lowbias32((unsigned)(*p.dstep + 1ll) ^ p.sr_seed);
#pragma unroll
                    for (int c = 0; c < NC + (SOL ? 1 : 0); ++c) {
                        unsigned w[5];
                        w[0] = lowbias32((unsigned)srow ^ tkey ^ (0x9E3779B9u * (unsigned)(c + 1)));
#pragma unroll
                        for (int k = 1; k < 5; ++k) w[k] = xorshift32(w[k - 1]);
                        const bool sol = c == NC;
                        S *__restrict__ out = sol ? (S *)p.g[parity ^ 1] : (S *)p.f[parity ^ 1][c < NC ? c : 0];
#pragma unroll
                        for (int i = 0; i < 9; ++i) {
                            const unsigned r = (i & 1) ? (w[i >> 1] << 16) : w[i >> 1];
                            if (!sol) stb(out, (O)i * pl + s, C::enc_sr(d[c < NC ? c : 0][i], i, r));
                            else if (shas<SQ>(i)) stb(out, (O)spl<SQ>(i) * pl + s, C::enc_sr(g[i], i, r));
                        }
                    }
                }
            }
            if (rne) {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    S *__restrict__ fout = (S *)p.f[parity ^ 1][c];
#pragma unroll
                    for (int i = 0; i < 9; ++i) stb(fout, (O)i * pl + s, C::enc(d[c][i], i));
                }
                if constexpr (SOL) {
                    S *__restrict__ gout = (S *)p.g[parity ^ 1];
#pragma unroll
                    for (int i = 0; i < 9; ++i)
                        if (shas<SQ>(i)) stb(gout, (O)spl<SQ>(i) * pl + s, C::enc(g[i], i));
                }
            }
        }
    }
    if (valid && solid && REACT && fluid8) {
        // 8. solid node next to fluid: add the gathered deposit, then decide
        // growth from the post-deposit value
        double bn = p.b[srow] + dep;
        if (fluid4) {
            // candidates: E, N, W, S that are fluid, inside the solute
            // domain and not on an open solute column
            unsigned candbits = 0;
            int m = 0;
#pragma unroll
            for (int i = 1; i <= 4; ++i) {
                const int cx = x + ex(i), cy = y + ey(i);
                // not across or on a wall of a non-periodic solute axis
                if ((!p.sxper && (cx <= 0 || cx >= nx - 1)) || (!p.syper && (cy <= 0 || cy >= ny - 1))) continue;
                if (!((lk >> i) & 1u)) {
                    candbits |= 1u << i;
                    ++m;
                }
            }
            uint8_t code = 0;
            if (bn > p.bmax && m > 0) {
                const unsigned long long t = (unsigned long long)(*p.dstep) + 1ull;
                const unsigned long long h = splitmix64(
                    p.seed ^ (t * (unsigned long long)nx * (unsigned long long)ny + (unsigned long long)srow));
                const int k = (int)(((h >> 32) * (unsigned long long)m) >> 32);
                // the k-th candidate in E, N, W, S order
                int seen = 0;
#pragma unroll
                for (int i = 1; i <= 4; ++i)
                    if (candbits & (1u << i)) {
                        if (seen == k) code = (uint8_t)i;
                        ++seen;
                    }
                tal[2] += bn;
                bn = 0.0;
                p.gflag[parity] = 1u;
                // the growth kernel visits only the row segments so marked
                const int gx = wrapi(x + ex(code), nx), gy = wrapi(y + ey(code), ny);
                p.gseg[parity][(size_t)gy * ((nx + 255) / 256) + gx / 256] = 1u;
            }
            p.trig[srow] = code;
        }
        p.b[srow] = bn;
    }

    if constexpr (SOL) {
        // running per-wavefront tallies: each wavefront owns one slot and
        // adds its step's sum in step order
        const bool has = tal[0] != 0.0 || tal[1] != 0.0 || tal[2] != 0.0;
        if (__any(has)) {
            wave_sum3(tal);
            if (lane == 0) {
                double *dst = p.partial + ((size_t)blockIdx.x * (TX * TY / 64) + (tid >> 6)) * 4;
                dst[0] += tal[0];
                dst[1] += tal[1];
                dst[2] += tal[2];
            }
        }
    }
}

// Gradient openings: after the collision each population of an opening
// node is extrapolated from the next two nodes inward,
// f(wall) = 2 f(wall + n) - f(wall + 2n) (inlet_momentum command); the
// same holds for the deviations.  One thread per opening node
// (blockIdx.y = opening).
template <typename S>
__global__ void __launch_bounds__(256) k_open_gradient(FullParams p, int parity_new) {
    using C = Codec<S>;
    const OpenSpec &o = p.open[blockIdx.y];
    const int j = o.lo + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (o.style != 4 || j > o.hi) return;
    const int nxw = o.wall == 0 ? 1 : o.wall == 1 ? -1 : 0;
    const int nyw = o.wall == 2 ? 1 : o.wall == 3 ? -1 : 0;
    const int x = o.wall == 0 ? 0 : o.wall == 1 ? p.nx - 1 : j;
    const int y = o.wall == 2 ? 0 : o.wall == 3 ? p.ny - 1 : j;
    const int x1 = x + nxw, y1 = y + nyw, x2 = x + 2 * nxw, y2 = y + 2 * nyw;
    const size_t nx = (size_t)p.nx;
    if (p.mask[y * nx + x] || p.mask[y1 * nx + x1] || p.mask[y2 * nx + x2]) return;
    S *f = (S *)p.f[parity_new][o.comp];
    const size_t s0 = brick_index<S>(x, y, p.pnx), s1 = brick_index<S>(x1, y1, p.pnx),
                 s2 = brick_index<S>(x2, y2, p.pnx);
    for (int i = 0; i < 9; ++i) {
        const auto a = C::dec(f[(size_t)i * p.pplane + s1], i), b = C::dec(f[(size_t)i * p.pplane + s2], i);
        f[(size_t)i * p.pplane + s0] = C::enc(a + a - b, i);
    }
}

// Growth: a fluid node turns solid when a direct neighbour's trigger points
// at it; its populations' mass is tallied as removed, it gets deposit b0,
// and the link words of the node and of its eight neighbours are updated
// (atomic OR on the 32-bit word holding each 16-bit link word: neighbours
// of two new solids are shared).  A fixed grid strides over row segments,
// so each block's running tally slot sees the same nodes in the same order
// every step.  Block 0 advances the device step counter (read by the next
// step's growth decisions).
constexpr int kGrowBlocks = 1024;

// One row segment of the growth kernel: the thread's node (x = 256 * (seg %
// segs_x) + threadIdx.x of row seg / segs_x) turns solid if a direct
// neighbour's trigger points at it; its removed fluid and solute are added
// to tal and any is set.
template <typename S, int NC>
__device__ __forceinline__ void grow_segment(const FullParams &p, int parity_new, int seg, int segs_x,
                                             double (&tal)[4], bool &any) {
    using C = Codec<S>;
    const int nx = p.nx, ny = p.ny;
    const size_t plane = p.pplane;
    const int x = (seg % segs_x) * 256 + threadIdx.x;
    const int y = seg / segs_x;
    if (x >= nx) return;
    const size_t s = (size_t)y * nx + x;
    if (p.mask[s]) return;
    bool grow = false;
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
        const int sx = x + ex(k), sy = y + ey(k);
        if (across_closed(p, sx, sy)) continue;
        const size_t sn = (size_t)wrapi(sy, ny) * nx + wrapi(sx, nx);
        if (p.trig[sn] == (uint8_t)opp(k)) grow = true;
    }
    if (!grow) return;
    any = true;
    const size_t ps = brick_index<S>((unsigned)x, (unsigned)y, p.pnx);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const S *__restrict__ f = (const S *)p.f[parity_new][c];
        double r = 0.0;
        for (int i = 0; i < 9; ++i)
            r += wgt<double>(i) * p.cd.rho_ref[c] + (double)C::dec(f[(size_t)i * plane + ps], i);
        tal[c] += r;
    }
    const S *__restrict__ g = (const S *)p.g[parity_new];
    double cc = 0.0;
    for (int k = 0; k < p.sq; ++k) cc += (double)C::dec(g[(size_t)k * plane + ps], splane_dir(p.sq, k));
    tal[2] += cc;
    tal[3] += 1.0;
    // the node's fluid and solute are removed: its stored values are
    // cleared as the step clears every solid node (deviation 0 for the
    // fluid, 0 for the solute)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        S *__restrict__ f = (S *)p.f[parity_new][c];
        for (int i = 0; i < 9; ++i) f[(size_t)i * plane + ps] = C::enc(0.0, i);
    }
    for (int k = 0; k < p.sq; ++k) ((S *)p.g[parity_new])[(size_t)k * plane + ps] = C::enc(0.0, k);
    if (p.slip)
        for (int c = 0; c < NC; ++c) p.refl[c][s] = p.grow_R[c];
    p.mask[s] = 1;
    p.b[s] = p.b0;
    // link words: own bit 0; neighbour s + e_j sees s at e_opp(j)
    unsigned *lw = (unsigned *)p.links;
    atomicOr(lw + (s >> 1), 1u << (16u * (unsigned)(s & 1)));
#pragma unroll
    for (int j = 1; j < 9; ++j) {
        const size_t n = (size_t)wrapi(y + ey(j), ny) * nx + wrapi(x + ex(j), nx);
        atomicOr(lw + (n >> 1), (1u << opp(j)) << (16u * (unsigned)(n & 1)));
    }
}

template <typename S, int NC, bool REACT>
__global__ void __launch_bounds__(256) k_growth(FullParams p, int parity_new) {
    __shared__ double sred[4 * 4];
    const int nx = p.nx, ny = p.ny;
    const bool first = blockIdx.x == 0 && threadIdx.x == 0;
    if (!REACT) {
        if (first) {
            *p.dstep += 1;
            p.gflag[parity_new] = 0u;
        }
        return;
    }
    // only the row segments that the step kernel marked can hold a node to
    // grow (the targets of this step's triggers), so the others are skipped,
    // all of them in a step without any trigger; the marks of the other
    // parity (read by the previous step's launch) are cleared for the next
    // step.  The block's segments are blockIdx.x + k * gridDim.x in
    // increasing k; their marks are read 256 at a time, one per thread.
    const bool fired = p.gflag[parity_new ^ 1] != 0u;
    const uint8_t *__restrict__ marked = p.gseg[parity_new ^ 1];
    __shared__ uint8_t slive[256];
    double tal[4] = {0.0, 0.0, 0.0, 0.0};
    bool any = false;
    if constexpr (REACT) {
        const int segs_x = (nx + 255) / 256;
        const int nseg = segs_x * ny;
        const int stride = (int)gridDim.x;
        for (int base = blockIdx.x; base < nseg; base += 256 * stride) {
            const int mine = base + (int)threadIdx.x * stride;
            bool lv = false;
            if (mine < nseg) {
                lv = fired && marked[mine] != 0u;
                p.gseg[parity_new][mine] = 0u;
            }
            slive[threadIdx.x] = lv ? 1u : 0u;
            if (__syncthreads_or(lv)) {
                for (int k = 0; k < 256; ++k) {
                    const int seg = base + k * stride;
                    if (seg >= nseg) break;
                    if (slive[k]) grow_segment<S, NC>(p, parity_new, seg, segs_x, tal, any);
                }
            }
            __syncthreads();
        }
    }
    if (__syncthreads_or(any)) {
        double out[4];
        block_sum<4>(tal, sred, out);
        if (threadIdx.x == 0) {
            double *dst = p.gpartial + (size_t)blockIdx.x * 4;
            for (int k = 0; k < 4; ++k) dst[k] += out[k];
        }
    }
    if (first) {
        *p.dstep += 1;
        p.gflag[parity_new] = 0u;
    }
}

// Fixed-order sums of the running tally slots into totals[] (LB2D_B_*
// indices).
__global__ void __launch_bounds__(256) k_tally_final(FullParams p) {
    __shared__ double sred[4 * 8];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < p.nblk_main; k += 256) {
        const double *q = p.partial + (size_t)k * 4;
        acc[0] += q[0];
        acc[1] += q[1];
        acc[2] += q[2];
    }
    for (int k = threadIdx.x; k < p.nblk_grow; k += 256) {
        const double *q = p.gpartial + (size_t)k * 4;
        acc[3] += q[0];
        acc[4] += q[1];
        acc[5] += q[2];
        acc[6] += q[3];
    }
    double tot[8];
    block_sum<8>(acc, sred, tot);
    if (threadIdx.x == 0) {
        p.totals[9] = tot[0];   // inflow
        p.totals[10] = tot[1];  // outflow
        p.totals[14] = tot[2];  // consumed deposit
        p.totals[6] = tot[3];   // removed mass 0
        p.totals[7] = tot[4];   // removed mass 1
        p.totals[8] = tot[5];   // removed solute
        p.totals[12] = tot[6];  // grown nodes
    }
}

// ------------------------------------------------- plain-step geometry

// Link word of every node: bit 0 = node solid, bit i = node + e_i solid.
__global__ void k_links(const uint8_t *__restrict__ mask, uint16_t *__restrict__ links, int nx, int ny) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    unsigned v = mask[(size_t)y * nx + x] ? 1u : 0u;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int gx = wrapi(x + ex(i), nx), gy = wrapi(y + ey(i), ny);
        if (mask[(size_t)gy * nx + gx]) v |= 1u << i;
    }
    links[(size_t)y * nx + x] = (uint16_t)v;
}

// ---------------------------------------------------------- set-up kernels

__global__ void k_fill_u8(uint8_t *p, uint8_t v, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        p[k] = v;
}

__global__ void k_fill_f64(double *p, double v, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        p[k] = v;
}

__global__ void k_or_mask(uint8_t *mask, const uint8_t *src, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        if (src[k]) mask[k] = 1;
}

// obstacle(circle): one block per circle sweeps its bounding box; a node is
// solid when its squared minimum-image distance (integers, exact in FP64)
// is at most r^2.  Stores are idempotent, so overlapping circles are fine.
__global__ void k_raster_circles(uint8_t *mask, int nx, int ny, const int *cxy, const double *cr) {
    const int xc = cxy[2 * blockIdx.x], yc = cxy[2 * blockIdx.x + 1];
    const double r = cr[blockIdx.x];
    const double r2 = r * r;
    // half-width of the bounding box (a radius beyond the box sweeps it all)
    const int h = (r < (double)(nx + ny)) ? (int)r + 1 : nx + ny;
    const int wx = (2 * h + 1 < nx) ? 2 * h + 1 : nx;
    const int wy = (2 * h + 1 < ny) ? 2 * h + 1 : ny;
    const int x0 = (2 * h + 1 < nx) ? xc - h : 0;
    const int y0 = (2 * h + 1 < ny) ? yc - h : 0;
    for (int k = threadIdx.x; k < wx * wy; k += blockDim.x) {
        const int gx = wrapi(x0 + k % wx, nx), gy = wrapi(y0 + k / wx, ny);
        long long dx = wrapi(gx - xc, nx), dy = wrapi(gy - yc, ny);
        if (nx - dx < dx) dx = nx - dx;
        if (ny - dy < dy) dy = ny - dy;
        const double d2 = (double)(dx * dx + dy * dy);
        if (d2 <= r2) mask[(size_t)gy * nx + gx] = 1;
    }
}

__global__ void k_raster_rects(uint8_t *mask, int nx, const int *rects) {
    const int x0 = rects[4 * blockIdx.x], x1 = rects[4 * blockIdx.x + 1];
    const int y0 = rects[4 * blockIdx.x + 2], y1 = rects[4 * blockIdx.x + 3];
    const int w = x1 - x0 + 1, h = y1 - y0 + 1;
    for (long long k = threadIdx.x; k < (long long)w * h; k += blockDim.x)
        mask[(size_t)(y0 + k / w) * nx + (x0 + k % w)] = 1;
}

// Populations at the equilibrium of (rho, u) from FP64 staging arrays
// (computed in FP64, then shifted and encoded).
template <typename S>
__global__ void k_init_fluid(S *f, const double *rho, const double *ux, const double *uy, size_t n,
                             double A0, double A1, double rho_ref, unsigned nx, unsigned pnx,
                             size_t pplane) {
    using C = Codec<S>;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        const size_t dst = brick_index<S>((unsigned)(k % nx), (unsigned)(k / nx), pnx);
        const double r = rho[k], u = ux[k], v = uy[k];
        const double usq = 1.5 * (u * u + v * v);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double eu = ex(i) * u + ey(i) * v;
            const double A = (i == 0) ? A0 : A1;
            const double fe = wgt<double>(i) * r * (A + 3.0 * eu + 4.5 * eu * eu - usq);
            f[(size_t)i * pplane + dst] = C::enc((typename C::R)(fe - wgt<double>(i) * rho_ref), i);
        }
    }
}

template <typename S, int SQ>
__global__ void k_init_solute(S *g, const double *Cc, const double *ux, const double *uy, size_t n, unsigned nx,
                              unsigned pnx, size_t pplane) {
    using C = Codec<S>;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        const double c = Cc[k], u = ux[k], v = uy[k];
        const size_t dst = brick_index<S>((unsigned)(k % nx), (unsigned)(k / nx), pnx);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if (!shas<SQ>(i)) continue;
            const double eu = ex(i) * u + ey(i) * v;
            const double ge = swgt<SQ, double>(i) * c * (1.0 + sics2<SQ, double>() * eu);
            g[(size_t)spl<SQ>(i) * pplane + dst] = C::enc((typename C::R)ge, i);
        }
    }
}

__global__ void k_init_b(double *b, const uint8_t *mask, double b0, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        b[k] = mask[k] ? b0 : 0.0;
}

// Raw state <-> FP64 row-major staging (one plane at a time);
// `shift` = w_i rho_ref.
template <typename S>
__global__ void k_decode_plane(const S *f, const uint8_t *mask, double *out, size_t n, int i, int dir, double shift,
                               unsigned nx, unsigned pnx, size_t pplane) {
    using C = Codec<S>;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        const size_t a = brick_index<S>((unsigned)(k % nx), (unsigned)(k / nx), pnx);
        out[k] = mask[k] ? 0.0 : shift + (double)C::dec(f[(size_t)i * pplane + a], dir);
    }
}
template <typename S>
__global__ void k_encode_plane(S *f, const double *in, size_t n, int i, int dir, double shift, unsigned nx,
                               unsigned pnx, size_t pplane) {
    using C = Codec<S>;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        const size_t a = brick_index<S>((unsigned)(k % nx), (unsigned)(k / nx), pnx);
        f[(size_t)i * pplane + a] = C::enc((typename C::R)(in[k] - shift), dir);
    }
}

// ---------------------------------------------------------------- read-out

template <typename S>
__device__ double node_rho(const FullParams &p, const S *f, int x, int y, double rho_ref) {
    using C = Codec<S>;
    const size_t plane = p.pplane;
    const size_t s = brick_index<S>((unsigned)x, (unsigned)y, p.pnx);
    double r = rho_ref;
    for (int i = 0; i < 9; ++i) r += (double)C::dec(f[(size_t)i * plane + s], i);
    return r;
}

// Density and velocity (j_post - F/2)/rho of component `comp` (or the
// mixture for comp < 0), in FP64 from the stored state; -11 at solids.
template <typename S>
__global__ void k_moments(FullParams p, int parity, int comp, double *orho, double *oux, double *ouy) {
    using C = Codec<S>;
    const int nx = p.nx, ny = p.ny;
    const size_t plane = p.pplane;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= nx) return;
    const size_t s = (size_t)y * nx + x;
    const size_t ps = brick_index<S>((unsigned)x, (unsigned)y, p.pnx);
    if (p.mask[s]) {
        orho[s] = -11.0;
        oux[s] = ouy[s] = 0.0;
        return;
    }
    double rho[2] = {0, 0}, jx[2] = {0, 0}, jy[2] = {0, 0};
    for (int c = 0; c < p.ncomp; ++c) {
        const S *f = (const S *)p.f[parity][c];
        double r = p.cd.rho_ref[c], mx = 0, my = 0;
        for (int i = 0; i < 9; ++i) {
            const double v = (double)C::dec(f[(size_t)i * plane + ps], i);
            r += v;
            mx += ex(i) * v;
            my += ey(i) * v;
        }
        rho[c] = r;
        jx[c] = mx;
        jy[c] = my;
    }
    double R = 0, MX = 0, MY = 0;
    for (int c = 0; c < p.ncomp; ++c) {
        if (comp >= 0 && c != comp) continue;
        double Fx = p.cd.force[c][0] + rho[c] * p.cd.accel[c][0];
        double Fy = p.cd.force[c][1] + rho[c] * p.cd.accel[c][1];
        if (p.ncomp == 2 && p.cd.G != 0.0) {
            double sx = 0, sy = 0;
            const S *fo = (const S *)p.f[parity][1 - c];
            for (int i = 1; i < 9; ++i) {
                const int gx = wrapi(x + ex(i), nx), gy = wrapi(y + ey(i), ny);
                if (p.mask[(size_t)gy * nx + gx]) continue;
                const double rb = node_rho<S>(p, fo, gx, gy, p.cd.rho_ref[1 - c]);
                sx += wgt<double>(i) * rb * ex(i);
                sy += wgt<double>(i) * rb * ey(i);
            }
            Fx += -p.cd.G * rho[c] * sx;
            Fy += -p.cd.G * rho[c] * sy;
        }
        if (p.ncomp == 1 && p.psi) {
            // one-component cohesion through psi(rho)
            double sx = 0, sy = 0;
            const S *fo = (const S *)p.f[parity][0];
            for (int i = 1; i < 9; ++i) {
                const int gx = wrapi(x + ex(i), nx), gy = wrapi(y + ey(i), ny);
                if (p.mask[(size_t)gy * nx + gx]) continue;
                const double pb = psi_of(p.cd.psi0, p.cd.rho0, node_rho<S>(p, fo, gx, gy, p.cd.rho_ref[0]));
                sx += wgt<double>(i) * pb * ex(i);
                sy += wgt<double>(i) * pb * ey(i);
            }
            const double ps = psi_of(p.cd.psi0, p.cd.rho0, rho[0]);
            Fx += -p.cd.G * ps * sx;
            Fy += -p.cd.G * ps * sy;
        }
        if (p.has_ads) {
            double sx = 0, sy = 0;
            for (int i = 1; i < 9; ++i) {
                const int gx = wrapi(x + ex(i), nx), gy = wrapi(y + ey(i), ny);
                const double sv = p.mask[(size_t)gy * nx + gx] ? 1.0 : 0.0;
                sx += wgt<double>(i) * sv * ex(i);
                sy += wgt<double>(i) * sv * ey(i);
            }
            const double a = p.ads_psi ? psi_of(p.cd.psi0a, p.cd.rho0a, rho[c]) : rho[c];
            Fx += -p.cd.Gads[c] * a * sx;
            Fy += -p.cd.Gads[c] * a * sy;
        }
        R += rho[c];
        MX += jx[c] - 0.5 * Fx;
        MY += jy[c] - 0.5 * Fy;
    }
    orho[s] = R;
    oux[s] = MX / R;
    ouy[s] = MY / R;
}

template <typename S>
__global__ void k_solute_state(FullParams p, int parity, int reaction, double *oc, double *ob) {
    using C = Codec<S>;
    const size_t n = (size_t)p.nx * p.ny;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        double c = 0.0;
        const bool sol = p.mask[k] != 0;
        if (!sol) {
            const S *g = (const S *)p.g[parity];
            const size_t a = brick_index<S>((unsigned)(k % p.nx), (unsigned)(k / p.nx), p.pnx);
            for (int j = 0; j < p.sq; ++j) c += (double)C::dec(g[(size_t)j * p.pplane + a], splane_dir(p.sq, j));
        }
        oc[k] = c;
        ob[k] = (sol && reaction) ? p.b[k] : 0.0;
    }
}

// Budgets: per-block FP64 partials over rows, then one block sums them.
template <typename S>
__global__ void __launch_bounds__(256) k_budget_partial(FullParams p, int parity, int has_solute,
                                                        int reaction, double *part) {
    using C = Codec<S>;
    __shared__ double sred[4 * 8];
    const int nx = p.nx;
    const size_t plane = p.pplane;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // m0 m1 jx jy C b nfluid -
    const int y = blockIdx.x;
    for (int x = threadIdx.x; x < nx; x += 256) {
        const size_t s = (size_t)y * nx + x;
        if (p.mask[s]) {
            if (reaction) v[5] += p.b[s];
            continue;
        }
        v[6] += 1.0;
        const size_t ps = brick_index<S>((unsigned)x, (unsigned)y, p.pnx);
        for (int c = 0; c < p.ncomp; ++c) {
            const S *f = (const S *)p.f[parity][c];
            for (int i = 0; i < 9; ++i) {
                const double fv = wgt<double>(i) * p.cd.rho_ref[c] + (double)C::dec(f[(size_t)i * plane + ps], i);
                v[c] += fv;
                v[2] += ex(i) * fv;
                v[3] += ey(i) * fv;
            }
        }
        if (has_solute) {
            const S *g = (const S *)p.g[parity];
            for (int j = 0; j < p.sq; ++j) v[4] += (double)C::dec(g[(size_t)j * plane + ps], splane_dir(p.sq, j));
        }
    }
    double out[8];
    block_sum<8>(v, sred, out);
    if (threadIdx.x == 0)
        for (int k = 0; k < 8; ++k) part[(size_t)blockIdx.x * 8 + k] = out[k];
}

__global__ void __launch_bounds__(256) k_budget_final(const double *part, int nblk, double *out8) {
    __shared__ double sred[4 * 8];
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < nblk; k += 256)
        for (int j = 0; j < 8; ++j) v[j] += part[(size_t)k * 8 + j];
    double out[8];
    block_sum<8>(v, sred, out);
    if (threadIdx.x == 0)
        for (int j = 0; j < 8; ++j) out8[j] = out[j];
}

// Plain copy kernel (read + write n floats) used to measure the practical
// HBM ceiling next to the stencil.  Streaming (non-temporal) loads and
// stores: the fastest plain copy measured on the MI355X.
__global__ void __launch_bounds__(256) k_copy(const float4 *__restrict__ a, float4 *__restrict__ b, size_t n4) {
    // each block copies 4 consecutive chunks of 256 float4: four loads in
    // flight per thread before the stores
    const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
    const LB2D_GLOBAL float *ga = (const LB2D_GLOBAL float *)gbl(a);
    LB2D_GLOBAL float *gb = (LB2D_GLOBAL float *)gbl(b);
    float v[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + 256 * k < n4)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[k][c] = __builtin_nontemporal_load(ga + 4 * (base + 256 * k) + c);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + 256 * k < n4)
#pragma unroll
            for (int c = 0; c < 4; ++c) __builtin_nontemporal_store(v[k][c], gb + 4 * (base + 256 * k) + c);
}

inline int grid1d(size_t n, int bs = 256) {
    size_t g = (n + bs - 1) / bs;
    if (g > 65536) g = 65536;
    return (int)(g ? g : 1);
}


#define LB2D_DISPATCH(st, CALL)                             \
    do {                                                    \
        switch (st) {                                       \
            case kF64: { using S = double; CALL; break; }   \
            case kF32: { using S = float; CALL; break; }    \
            case kF16: { using S = _Float16; CALL; break; } \
            default: { using S = bf16s; CALL; break; }      \
        }                                                   \
    } while (0)

// Nine planes of `plane` values of `bytes` each are addressable with 32-bit
// byte offsets.
inline bool fits32(size_t plane, size_t bytes) { return (unsigned long long)plane * 9ull * bytes < (1ull << 32); }

}  // namespace
}  // namespace lb2d
