// Kernel instantiations: Gomoku N x N for N = 5 .. 8.
#include "kernels.hpp"

namespace lx {
const GameOps *ops_gomoku_a(int n) { return ops_range<Gomoku, 5, 8>(n); }
} // namespace lx
