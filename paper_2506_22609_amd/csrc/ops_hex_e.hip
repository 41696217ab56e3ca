// Kernel instantiations: Hex N x N for N = 17 .. 19.
#include "kernels.hpp"

namespace lx {
const GameOps *ops_hex_e(int n) { return ops_range<Hex, 17, 19>(n); }
} // namespace lx
