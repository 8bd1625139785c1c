// General fused step, f64 storage, lattices with momentum openings, slip solids or intersolute.
#include "lb2d_full.hpp"

namespace lb2d {
hipError_t launch_full_f64_ext(const FullParams &p, int parity, bool sc, bool react, hipStream_t s) {
    return full_dispatch<double, true>(p, parity, sc, react, s);
}
}  // namespace lb2d
