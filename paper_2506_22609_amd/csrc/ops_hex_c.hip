// Kernel instantiations: Hex N x N for N = 11 .. 13.
#include "kernels.hpp"

namespace lx {
const GameOps *ops_hex_c(int n) { return ops_range<Hex, 11, 13>(n); }
} // namespace lx
