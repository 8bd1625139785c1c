// General fused step, bf16 storage, lattices with momentum openings, slip solids or intersolute.
#include "lb2d_full.hpp"

namespace lb2d {
hipError_t launch_full_bf16_ext(const FullParams &p, int parity, bool sc, bool react, hipStream_t s) {
    return full_dispatch<bf16s, true>(p, parity, sc, react, s);
}
}  // namespace lb2d
