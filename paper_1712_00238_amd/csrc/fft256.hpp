// Lines of the 2x oversampled grids of the nonequispaced route that the
// fused sizes do not cover: 192 points (N = 96) and 256 points (N = 128).
#pragma once

#include "fft.hpp"

namespace sdf {

template <>
struct DefaultPlan<192> {
    using type = Radices<8, 8, 3>;
};

template <>
struct DefaultPlan<256> {
    using type = Radices<8, 8, 4>;
};

}  // namespace sdf
