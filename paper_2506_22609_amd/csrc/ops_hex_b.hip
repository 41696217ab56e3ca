// Kernel instantiations: Hex N x N for N = 7 .. 10.
#include "kernels.hpp"

namespace lx {
const GameOps *ops_hex_b(int n) { return ops_range<Hex, 7, 10>(n); }
} // namespace lx
