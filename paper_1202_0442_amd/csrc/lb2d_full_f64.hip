// General fused step, f64 storage, lattices without the extended features.
#include "lb2d_full.hpp"

namespace lb2d {
hipError_t launch_full_f64(const FullParams &p, int parity, bool sc, bool react, hipStream_t s) {
    return full_dispatch<double, false>(p, parity, sc, react, s);
}
}  // namespace lb2d
