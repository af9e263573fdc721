// 256-point lines: the 2x oversampled grid of the nonequispaced route.
#pragma once

#include "fft.hpp"

namespace sdf {

template <>
struct DefaultPlan<256> {
    using type = Radices<8, 8, 4>;
};

}  // namespace sdf
