// lb2d_kernels.hpp -- host-side launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "lb2d_common.hpp"

namespace lb2d {

size_t storage_bytes(int st);
int full_tiles(int nx, int ny);
// Running tally slots of the general step (one per wavefront) and blocks
// (= tally slots) of the growth kernel.
int full_slots(int nx, int ny);
// Row segments of 256 nodes (((nx + 255) / 256) per row) that the growth
// kernel walks, and its block count.
int growth_segments(int nx, int ny);
int growth_blocks(int nx, int ny);

// Tile (in nodes) covered by one 256-thread block of the one-fluid step.
void plain_tile(int st, int *tw, int *th);
// One-fluid step; sr: stochastic rounding (16-bit storage, 32-bit offsets),
// nt: streaming stores, k: offset of the step in its launch group.
hipError_t launch_plain(int st, const PlainLattice &L, int parity, bool sr, bool nt, int k, hipStream_t s);
// multi_steps() (an odd number of) steps in one launch (buffer parity ->
// parity^1), for lattices that hold the kernel's tile with multi_steps() - 1
// rings of nodes around it (multi_fits).  Arguments as for launch_plain (k:
// offset of the first of the steps).
int multi_steps();
void multi_tile_shape(int st, int *tw, int *th);
bool multi_fits(int st, int nx, int ny);
hipError_t launch_plain_ms(int st, const PlainLattice &L, int parity, bool sr, bool nt, int k, hipStream_t s);
// Adds n to the device step counter.
hipError_t launch_tick(unsigned long long *step, int n, hipStream_t s);
// Tile shapes (width, height in nodes) of the batched step for a storage
// format, widest first; returns their number (at most max).
int batch_shapes(int st, int *tw, int *th, int max);
// tile_w: one of the widths of batch_shapes; max_plane: largest population
// plane (elements) of the batch's lattices; sr, nt, k as for launch_plain;
// bstep: the batch's device step counter (equal to every lattice's; read
// only with sr).
hipError_t launch_batch(int st, int tile_w, const PlainLattice *lat, const Tile *tiles, int ntiles, int parity,
                        int grid, size_t max_plane, bool nt, bool sr, int k, const unsigned long long *bstep,
                        hipStream_t s);
// Batched multi-step kernel over a table of multi_tile_shape-sized tiles of
// lattices that each satisfy multi_fits; arguments as for launch_batch (k:
// offset of the first of the steps).
hipError_t launch_batch_ms(int st, const PlainLattice *lat, const Tile *tiles, int ntiles, int parity, int grid,
                         size_t max_plane, bool nt, bool sr, int k, const unsigned long long *bstep,
                         hipStream_t s);
// Adds n to the batch's step counter and to that of each of its nlat lattices.
hipError_t launch_tick_batch(const PlainLattice *lat, int nlat, int n, unsigned long long *bstep, hipStream_t s);
// Streaming stores pay off once the populations (all buffers) no longer
// fit in the last-level cache.
constexpr size_t kLastLevelCache = 256ull << 20;
// General step; the solute lattice (none, D2Q9, D2Q4) is p.sq.
hipError_t launch_full(int st, const FullParams &p, int parity, bool sc, bool react, hipStream_t s);
// The general step per storage format, for lattices without (plain name)
// and with (_ext) momentum openings, slip solids or intersolute; one
// translation unit each (lb2d_full_*.hip).
hipError_t launch_full_f64(const FullParams &p, int parity, bool sc, bool react, hipStream_t s);
hipError_t launch_full_f64_ext(const FullParams &p, int parity, bool sc, bool react, hipStream_t s);
hipError_t launch_full_f32(const FullParams &p, int parity, bool sc, bool react, hipStream_t s);
hipError_t launch_full_f32_ext(const FullParams &p, int parity, bool sc, bool react, hipStream_t s);
hipError_t launch_full_f16(const FullParams &p, int parity, bool sc, bool react, hipStream_t s);
hipError_t launch_full_f16_ext(const FullParams &p, int parity, bool sc, bool react, hipStream_t s);
hipError_t launch_full_bf16(const FullParams &p, int parity, bool sc, bool react, hipStream_t s);
hipError_t launch_full_bf16_ext(const FullParams &p, int parity, bool sc, bool react, hipStream_t s);
hipError_t launch_growth(int st, const FullParams &p, int parity_new, bool react, hipStream_t s);
// Normal velocity (inward) of velocity opening o at coordinate k along its
// wall (poiseuille profile or uniform; negative for outlets).
double opening_normal_velocity(const OpenSpec &o, int k);
// Gradient-style momentum openings (after the step); no-op without them.
hipError_t launch_open_gradient(int st, const FullParams &p, int parity_new, hipStream_t s);
hipError_t launch_tally_final(const FullParams &p, hipStream_t s);

hipError_t launch_fill_u8(uint8_t *p, uint8_t v, size_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s);
hipError_t launch_or_mask(uint8_t *mask, const uint8_t *src, size_t n, hipStream_t s);
hipError_t launch_raster_circles(uint8_t *mask, int nx, int ny, const int *cxy, const double *cr, int count,
                                 hipStream_t s);
hipError_t launch_raster_rects(uint8_t *mask, int nx, const int *rects, int count, hipStream_t s);
hipError_t launch_init_fluid(int st, void *f, const double *rho, const double *ux, const double *uy, size_t n,
                             double A0, double A1, double rho_ref, unsigned nx, unsigned pnx,
                             size_t pplane, hipStream_t s);
// Solute populations at equilibrium on a D2Q9 (sq = 9) or D2Q4 (sq = 4)
// lattice, sq brick-layout planes of pplane elements.
hipError_t launch_init_solute(int st, void *g, const double *C, const double *ux, const double *uy, size_t n,
                              int sq, unsigned nx, unsigned pnx, size_t pplane, hipStream_t s);
hipError_t launch_init_b(double *b, const uint8_t *mask, double b0, size_t n, hipStream_t s);
// Plane i of a population array <-> FP64 row-major values; dir: the
// direction stored in that plane (it sets the 16-bit scale).
hipError_t launch_decode_plane(int st, const void *f, const uint8_t *mask, double *out, size_t n, int i, int dir,
                               double shift, unsigned nx, unsigned pnx, size_t pplane, hipStream_t s);
hipError_t launch_links(const uint8_t *mask, uint16_t *links, int nx, int ny, hipStream_t s);
hipError_t launch_encode_plane(int st, void *f, const double *in, size_t n, int i, int dir, double shift,
                               unsigned nx, unsigned pnx, size_t pplane, hipStream_t s);
hipError_t launch_moments(int st, const FullParams &p, int parity, int comp, double *rho, double *ux, double *uy,
                          hipStream_t s);
hipError_t launch_solute_state(int st, const FullParams &p, int parity, int reaction, double *C, double *b,
                               hipStream_t s);
hipError_t launch_budgets(int st, const FullParams &p, int parity, int has_solute, int reaction, double *part,
                          double *out8, hipStream_t s);
hipError_t launch_copy(const void *a, void *b, size_t bytes, hipStream_t s);

}  // namespace lb2d
