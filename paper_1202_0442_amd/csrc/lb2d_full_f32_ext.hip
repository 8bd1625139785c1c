// General fused step, f32 storage, lattices with momentum openings, slip solids or intersolute.
#include "lb2d_full.hpp"

namespace lb2d {
hipError_t launch_full_f32_ext(const FullParams &p, int parity, bool sc, bool react, hipStream_t s) {
    return full_dispatch<float, true>(p, parity, sc, react, s);
}
}  // namespace lb2d
