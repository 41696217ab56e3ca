// Kernel instantiations: Hex N x N for N = 1 .. 6.
#include "kernels.hpp"

namespace lx {
const GameOps *ops_hex_a(int n) { return ops_range<Hex, 1, 6>(n); }
} // namespace lx
