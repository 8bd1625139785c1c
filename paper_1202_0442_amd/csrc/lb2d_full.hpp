// lb2d_full.hpp -- instantiations of the general fused step k_full for one
// storage format S, one per feature set: number of fluid components,
// Shan-Chen forces, solute lattice (none, D2Q9, D2Q4), reaction, and EXT
// (momentum openings, slip solids, intersolute), with 32- or 64-bit
// population offsets.  Each lb2d_full_*.hip unit instantiates one S and
// one EXT, so the build compiles them in parallel.
#pragma once
#include "lb2d_device.hpp"

namespace lb2d {
namespace {

template <typename S, typename O, int SQ, bool EXT>
static void full_dispatch_sq(const FullParams &p, int parity, bool sc, bool react, hipStream_t st) {
    const int nblk = full_tiles(p.nx, p.ny);
    const dim3 g(nblk), b(kTX * kTY);
#define LB2D_FULL(NC_, SC_, REACT_) \
    hipLaunchKernelGGL((k_full<S, O, NC_, SC_, SQ, REACT_, EXT, kTX, kTY>), g, b, 0, st, p, parity)
    if (p.ncomp == 2) {
        if (sc) {
            if (react) LB2D_FULL(2, true, true);
            else LB2D_FULL(2, true, false);
        } else {
            if (react) LB2D_FULL(2, false, true);
            else LB2D_FULL(2, false, false);
        }
    } else {
        if (sc) {
            if (react) LB2D_FULL(1, true, true);
            else LB2D_FULL(1, true, false);
        } else {
            if (react) LB2D_FULL(1, false, true);
            else LB2D_FULL(1, false, false);
        }
    }
#undef LB2D_FULL
}

template <typename S, int SQ, bool EXT>
static void full_dispatch_off(const FullParams &p, int parity, bool sc, bool react, hipStream_t st) {
    // 32-bit byte offsets when every population array (9 planes) is below 4 GiB
    if (fits32(p.pplane, sizeof(S))) full_dispatch_sq<S, uint32_t, SQ, EXT>(p, parity, sc, react, st);
    else full_dispatch_sq<S, size_t, SQ, EXT>(p, parity, sc, react, st);
}

// The reaction needs a solute; the solute lattice is p.sq (0, 9 or 4).
template <typename S, bool EXT>
static hipError_t full_dispatch(const FullParams &p, int parity, bool sc, bool react, hipStream_t st) {
    if (p.sq == 9) full_dispatch_off<S, 9, EXT>(p, parity, sc, react, st);
    else if (p.sq == 4) full_dispatch_off<S, 4, EXT>(p, parity, sc, react, st);
    else full_dispatch_off<S, 0, EXT>(p, parity, sc, false, st);
    return hipGetLastError();
}

}  // namespace
}  // namespace lb2d
