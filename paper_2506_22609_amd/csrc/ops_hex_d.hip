// Kernel instantiations: Hex N x N for N = 14 .. 16.
#include "kernels.hpp"

namespace lx {
const GameOps *ops_hex_d(int n) { return ops_range<Hex, 14, 16>(n); }
} // namespace lx
