// lb2d_kernels.hip -- launchers of the gfx950 kernels of the D2Q9 lattice
// Boltzmann library (the kernels themselves are in lb2d_device.hpp; the
// general step's instantiations are in the lb2d_full_*.hip units).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lb2d_device.hpp"

namespace lb2d {
// --------------------------------------------------------------- launchers

size_t storage_bytes(int st) { return st == kF64 ? 8 : st == kF32 ? 4 : 2; }


void plain_tile(int st, int *tw, int *th) {
    const int h = brick_h_for((int)storage_bytes(st));
    const int bw = brick_w_for((int)storage_bytes(st));
    *tw = 256 / (bw * h) * bw;
    *th = h;
}

template <bool NT>
static void plain_dispatch(int st, const PlainLattice &L, int parity, bool sr, int k, hipStream_t stream) {
    int tw, th;
    plain_tile(st, &tw, &th);
    const dim3 blk(256), grd((L.nx + tw - 1) / tw, (L.ny + th - 1) / th);
    if (sr && st == kF16)
        hipLaunchKernelGGL((k_plain<_Float16, uint32_t, true, NT>), grd, blk, 0, stream, L, parity, k);
    else if (sr && st == kBF16)
        hipLaunchKernelGGL((k_plain<bf16s, uint32_t, true, NT>), grd, blk, 0, stream, L, parity, k);
    else if (fits32(L.plane, storage_bytes(st)))
        LB2D_DISPATCH(st, hipLaunchKernelGGL((k_plain<S, uint32_t, false, NT>), grd, blk, 0, stream, L, parity, k));
    else
        LB2D_DISPATCH(st, hipLaunchKernelGGL((k_plain<S, size_t, false, NT>), grd, blk, 0, stream, L, parity, k));
}

hipError_t launch_plain(int st, const PlainLattice &L, int parity, bool sr, bool nt, int k, hipStream_t stream) {
    if (nt) plain_dispatch<true>(st, L, parity, sr, k, stream);
    else plain_dispatch<false>(st, L, parity, sr, k, stream);
    return hipGetLastError();
}

// Tile of the multi-step kernel: 64 x 16 nodes (1024 threads), 32 x 16 for
// 8-byte values (whose LDS region then takes 69 KB).
void multi_tile_shape(int st, int *tw, int *th) {
    *tw = st == kF64 ? kMultiTW / 2 : kMultiTW;
    *th = kMultiTH;
}

int multi_steps() { return kMultiSteps; }

bool multi_fits(int st, int nx, int ny) {
    int tw, th;
    multi_tile_shape(st, &tw, &th);
    return nx >= tw + 2 * (kMultiSteps - 1) && ny >= th + 2 * (kMultiSteps - 1);
}

template <typename S, typename O, bool SR, bool NT>
static void multi_launch(const PlainLattice &L, int parity, int k, hipStream_t stream) {
    constexpr int TW = sizeof(S) == 8 ? kMultiTW / 2 : kMultiTW, TH = kMultiTH;
    const dim3 blk(TW * TH), grd((L.nx + TW - 1) / TW, (L.ny + TH - 1) / TH);
    hipLaunchKernelGGL((k_plain_ms<S, O, SR, NT, TW, TH, kMultiSteps>), grd, blk, 0, stream, L, parity, k);
}

template <bool NT>
static void multi_dispatch(int st, const PlainLattice &L, int parity, bool sr, int k, hipStream_t stream) {
    if (sr && st == kF16)
        multi_launch<_Float16, uint32_t, true, NT>(L, parity, k, stream);
    else if (sr && st == kBF16)
        multi_launch<bf16s, uint32_t, true, NT>(L, parity, k, stream);
    else if (fits32(L.plane, storage_bytes(st)))
        LB2D_DISPATCH(st, (multi_launch<S, uint32_t, false, NT>(L, parity, k, stream)));
    else
        LB2D_DISPATCH(st, (multi_launch<S, size_t, false, NT>(L, parity, k, stream)));
}

hipError_t launch_plain_ms(int st, const PlainLattice &L, int parity, bool sr, bool nt, int k, hipStream_t stream) {
    if (!multi_fits(st, L.nx, L.ny)) return hipErrorInvalidValue;
    if (nt) multi_dispatch<true>(st, L, parity, sr, k, stream);
    else multi_dispatch<false>(st, L, parity, sr, k, stream);
    return hipGetLastError();
}

__global__ void k_tick(unsigned long long *step, int n) { *step += (unsigned long long)n; }

hipError_t launch_tick(unsigned long long *step, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(1), 0, s, step, n);
    return hipGetLastError();
}

// Tile widths of the batched step for a storage format: tiles of 1, 2 or 4
// brick rows (64x4, 32x8, 16x16 nodes for 4- and 8-byte values; 32x8,
// 16x16, 8x32 for 2-byte values).
int batch_shapes(int st, int *tw, int *th, int max) {
    const int vb = (int)storage_bytes(st);
    const int W = brick_w_for(vb), H = brick_h_for(vb), bricks = 256 / (W * H);
    int n = 0;
    for (int rows = 1; rows <= 4 && n < max; rows *= 2) {
        tw[n] = bricks / rows * W;
        th[n] = rows * H;
        ++n;
    }
    return n;
}

template <typename S, typename O, bool SR, bool NT>
static void batch_shape(int tw, const PlainLattice *lat, const Tile *tiles, int ntiles, int parity, int grid, int k,
                        const unsigned long long *bstep, hipStream_t stream) {
    constexpr int W = brick_w_for(sizeof(S)), H = brick_h_for(sizeof(S)), B = 256 / (W * H);
#define LB2D_BATCH(TX_) \
    hipLaunchKernelGGL((k_batch<S, O, SR, NT, TX_>), dim3(grid), dim3(256), 0, stream, lat, tiles, ntiles, parity, k, bstep)
    if (tw == B * W) LB2D_BATCH(B * W);
    else if (tw == B / 2 * W) LB2D_BATCH(B / 2 * W);
    else LB2D_BATCH(B / 4 * W);
#undef LB2D_BATCH
}

template <bool NT>
static void batch_dispatch(int st, int tw, const PlainLattice *lat, const Tile *tiles, int ntiles, int parity,
                           int grid, size_t max_plane, bool sr, int k, const unsigned long long *bstep,
                           hipStream_t stream) {
    // stochastic rounding: every lattice's arrays are below 4 GiB (checked at bind)
    if (sr && st == kF16)
        batch_shape<_Float16, uint32_t, true, NT>(tw, lat, tiles, ntiles, parity, grid, k, bstep, stream);
    else if (sr && st == kBF16)
        batch_shape<bf16s, uint32_t, true, NT>(tw, lat, tiles, ntiles, parity, grid, k, bstep, stream);
    else if (fits32(max_plane, storage_bytes(st)))
        LB2D_DISPATCH(st, (batch_shape<S, uint32_t, false, NT>(tw, lat, tiles, ntiles, parity, grid, k, bstep,
                                                                stream)));
    else
        LB2D_DISPATCH(st, (batch_shape<S, size_t, false, NT>(tw, lat, tiles, ntiles, parity, grid, k, bstep,
                                                              stream)));
}

hipError_t launch_batch(int st, int tile_w, const PlainLattice *lat, const Tile *tiles, int ntiles, int parity,
                        int grid, size_t max_plane, bool nt, bool sr, int k, const unsigned long long *bstep,
                        hipStream_t stream) {
    if (nt) batch_dispatch<true>(st, tile_w, lat, tiles, ntiles, parity, grid, max_plane, sr, k, bstep, stream);
    else batch_dispatch<false>(st, tile_w, lat, tiles, ntiles, parity, grid, max_plane, sr, k, bstep, stream);
    return hipGetLastError();
}

template <typename S, typename O, bool SR, bool NT>
static void batch_ms_launch(const PlainLattice *lat, const Tile *tiles, int ntiles, int parity, int grid, int k,
                            const unsigned long long *bstep, hipStream_t stream) {
    constexpr int TW = sizeof(S) == 8 ? kMultiTW / 2 : kMultiTW, TH = kMultiTH;
    hipLaunchKernelGGL((k_batch_ms<S, O, SR, NT, TW, TH, kMultiSteps>), dim3(grid), dim3(TW * TH), 0, stream, lat,
                       tiles, ntiles, parity, k, bstep);
}

template <bool NT>
static void batch_ms_dispatch(int st, const PlainLattice *lat, const Tile *tiles, int ntiles, int parity, int grid,
                              size_t max_plane, bool sr, int k, const unsigned long long *bstep, hipStream_t stream) {
    if (sr && st == kF16)
        batch_ms_launch<_Float16, uint32_t, true, NT>(lat, tiles, ntiles, parity, grid, k, bstep, stream);
    else if (sr && st == kBF16)
        batch_ms_launch<bf16s, uint32_t, true, NT>(lat, tiles, ntiles, parity, grid, k, bstep, stream);
    else if (fits32(max_plane, storage_bytes(st)))
        LB2D_DISPATCH(st,
                      (batch_ms_launch<S, uint32_t, false, NT>(lat, tiles, ntiles, parity, grid, k, bstep, stream)));
    else
        LB2D_DISPATCH(st, (batch_ms_launch<S, size_t, false, NT>(lat, tiles, ntiles, parity, grid, k, bstep, stream)));
}

hipError_t launch_batch_ms(int st, const PlainLattice *lat, const Tile *tiles, int ntiles, int parity, int grid,
                           size_t max_plane, bool nt, bool sr, int k, const unsigned long long *bstep,
                           hipStream_t stream) {
    if (nt) batch_ms_dispatch<true>(st, lat, tiles, ntiles, parity, grid, max_plane, sr, k, bstep, stream);
    else batch_ms_dispatch<false>(st, lat, tiles, ntiles, parity, grid, max_plane, sr, k, bstep, stream);
    return hipGetLastError();
}

// Advances the batch's step counter and that of every lattice of the batch
// (which each lattice reads when stepped alone) by n.
__global__ void k_tick_batch(const PlainLattice *__restrict__ lat, int nlat, int n, unsigned long long *bstep) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nlat) *(unsigned long long *)lat[i].step += (unsigned long long)n;
    if (i == 0) *bstep += (unsigned long long)n;
}

hipError_t launch_tick_batch(const PlainLattice *lat, int nlat, int n, unsigned long long *bstep, hipStream_t s) {
    hipLaunchKernelGGL(k_tick_batch, dim3((nlat + 255) / 256), dim3(256), 0, s, lat, nlat, n, bstep);
    return hipGetLastError();
}

int full_tiles(int nx, int ny) { return ((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY); }
int full_slots(int nx, int ny) { return full_tiles(nx, ny) * (kTX * kTY / 64); }
int growth_segments(int nx, int ny) { return ((nx + 255) / 256) * ny; }
int growth_blocks(int nx, int ny) {
    const int segs = growth_segments(nx, ny);
    return segs < kGrowBlocks ? segs : kGrowBlocks;
}

hipError_t launch_full(int st, const FullParams &p, int parity, bool sc, bool react, hipStream_t stream) {
    // the instantiations of the general step live in one translation unit
    // per storage format and feature set (lb2d_full_*.hip)
    const bool ext = p.nopen > 0 || p.slip || p.isol;
    switch (st) {
        case kF64: return ext ? launch_full_f64_ext(p, parity, sc, react, stream)
                              : launch_full_f64(p, parity, sc, react, stream);
        case kF32: return ext ? launch_full_f32_ext(p, parity, sc, react, stream)
                              : launch_full_f32(p, parity, sc, react, stream);
        case kF16: return ext ? launch_full_f16_ext(p, parity, sc, react, stream)
                              : launch_full_f16(p, parity, sc, react, stream);
        default: return ext ? launch_full_bf16_ext(p, parity, sc, react, stream)
                            : launch_full_bf16(p, parity, sc, react, stream);
    }
}

double opening_normal_velocity(const OpenSpec &o, int k) { return opening_un<double>(o, k); }

hipError_t launch_open_gradient(int st, const FullParams &p, int parity_new, hipStream_t stream) {
    int len = 0;
    for (int k = 0; k < p.nopen; ++k)
        if (p.open[k].style == 4) len = std::max(len, p.open[k].hi - p.open[k].lo + 1);
    if (len == 0) return hipSuccess;
    const dim3 g((len + 255) / 256, p.nopen), b(256);
    LB2D_DISPATCH(st, hipLaunchKernelGGL(k_open_gradient<S>, g, b, 0, stream, p, parity_new));
    return hipGetLastError();
}

template <typename S>
static void growth_dispatch(const FullParams &p, int parity_new, bool react, dim3 g, dim3 b, hipStream_t stream) {
    if (p.ncomp == 2) {
        if (react) hipLaunchKernelGGL((k_growth<S, 2, true>), g, b, 0, stream, p, parity_new);
        else hipLaunchKernelGGL((k_growth<S, 2, false>), g, b, 0, stream, p, parity_new);
    } else {
        if (react) hipLaunchKernelGGL((k_growth<S, 1, true>), g, b, 0, stream, p, parity_new);
        else hipLaunchKernelGGL((k_growth<S, 1, false>), g, b, 0, stream, p, parity_new);
    }
}

hipError_t launch_growth(int st, const FullParams &p, int parity_new, bool react, hipStream_t stream) {
    const dim3 g = react ? dim3(growth_blocks(p.nx, p.ny)) : dim3(1), b(256);
    LB2D_DISPATCH(st, growth_dispatch<S>(p, parity_new, react, g, b, stream));
    return hipGetLastError();
}

hipError_t launch_tally_final(const FullParams &p, hipStream_t s) {
    hipLaunchKernelGGL(k_tally_final, dim3(1), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u8, dim3(grid1d(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f64, dim3(grid1d(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_or_mask(uint8_t *mask, const uint8_t *src, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_or_mask, dim3(grid1d(n)), dim3(256), 0, s, mask, src, n);
    return hipGetLastError();
}
hipError_t launch_raster_circles(uint8_t *mask, int nx, int ny, const int *cxy, const double *cr, int count,
                                 hipStream_t s) {
    if (count > 0) hipLaunchKernelGGL(k_raster_circles, dim3(count), dim3(256), 0, s, mask, nx, ny, cxy, cr);
    return hipGetLastError();
}
hipError_t launch_raster_rects(uint8_t *mask, int nx, const int *rects, int count, hipStream_t s) {
    if (count > 0) hipLaunchKernelGGL(k_raster_rects, dim3(count), dim3(256), 0, s, mask, nx, rects);
    return hipGetLastError();
}
hipError_t launch_init_fluid(int st, void *f, const double *rho, const double *ux, const double *uy, size_t n,
                             double A0, double A1, double rho_ref, unsigned nx, unsigned pnx,
                             size_t pplane, hipStream_t s) {
    LB2D_DISPATCH(st, hipLaunchKernelGGL(k_init_fluid<S>, dim3(grid1d(n)), dim3(256), 0, s, (S *)f, rho, ux, uy, n,
                                         A0, A1, rho_ref, nx, pnx, pplane));
    return hipGetLastError();
}
hipError_t launch_init_solute(int st, void *g, const double *C, const double *ux, const double *uy, size_t n,
                              int sq, unsigned nx, unsigned pnx, size_t pplane, hipStream_t s) {
    if (sq == 4)
        LB2D_DISPATCH(st, hipLaunchKernelGGL((k_init_solute<S, 4>), dim3(grid1d(n)), dim3(256), 0, s, (S *)g, C, ux,
                                             uy, n, nx, pnx, pplane));
    else
        LB2D_DISPATCH(st, hipLaunchKernelGGL((k_init_solute<S, 9>), dim3(grid1d(n)), dim3(256), 0, s, (S *)g, C, ux,
                                             uy, n, nx, pnx, pplane));
    return hipGetLastError();
}
hipError_t launch_init_b(double *b, const uint8_t *mask, double b0, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_init_b, dim3(grid1d(n)), dim3(256), 0, s, b, mask, b0, n);
    return hipGetLastError();
}
hipError_t launch_decode_plane(int st, const void *f, const uint8_t *mask, double *out, size_t n, int i, int dir,
                               double shift, unsigned nx, unsigned pnx, size_t pplane, hipStream_t s) {
    LB2D_DISPATCH(st, hipLaunchKernelGGL(k_decode_plane<S>, dim3(grid1d(n)), dim3(256), 0, s, (const S *)f, mask,
                                         out, n, i, dir, shift, nx, pnx, pplane));
    return hipGetLastError();
}
hipError_t launch_links(const uint8_t *mask, uint16_t *links, int nx, int ny, hipStream_t s) {
    hipLaunchKernelGGL(k_links, dim3((nx + 255) / 256, ny), dim3(256), 0, s, mask, links, nx, ny);
    return hipGetLastError();
}
hipError_t launch_encode_plane(int st, void *f, const double *in, size_t n, int i, int dir, double shift,
                               unsigned nx, unsigned pnx, size_t pplane, hipStream_t s) {
    LB2D_DISPATCH(st, hipLaunchKernelGGL(k_encode_plane<S>, dim3(grid1d(n)), dim3(256), 0, s, (S *)f, in, n, i,
                                         dir, shift, nx, pnx, pplane));
    return hipGetLastError();
}
hipError_t launch_moments(int st, const FullParams &p, int parity, int comp, double *rho, double *ux, double *uy,
                          hipStream_t s) {
    const dim3 g((p.nx + 255) / 256, p.ny), b(256);
    LB2D_DISPATCH(st, hipLaunchKernelGGL(k_moments<S>, g, b, 0, s, p, parity, comp, rho, ux, uy));
    return hipGetLastError();
}
hipError_t launch_solute_state(int st, const FullParams &p, int parity, int reaction, double *C, double *b,
                               hipStream_t s) {
    const size_t n = (size_t)p.nx * p.ny;
    LB2D_DISPATCH(st, hipLaunchKernelGGL(k_solute_state<S>, dim3(grid1d(n)), dim3(256), 0, s, p, parity, reaction, C,
                                         b));
    return hipGetLastError();
}
hipError_t launch_budgets(int st, const FullParams &p, int parity, int has_solute, int reaction, double *part,
                          double *out8, hipStream_t s) {
    LB2D_DISPATCH(st, hipLaunchKernelGGL(k_budget_partial<S>, dim3(p.ny), dim3(256), 0, s, p, parity, has_solute,
                                         reaction, part));
    hipLaunchKernelGGL(k_budget_final, dim3(1), dim3(256), 0, s, part, p.ny, out8);
    return hipGetLastError();
}
hipError_t launch_copy(const void *a, void *b, size_t bytes, hipStream_t s) {
    const size_t n4 = bytes / 16;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)((n4 + 1023) / 1024)), dim3(256), 0, s, (const float4 *)a,
                       (float4 *)b, n4);
    return hipGetLastError();
}

}  // namespace lb2d
