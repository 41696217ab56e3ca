// Kernel instantiations: Gomoku N x N for N = 9 .. 12.
#include "kernels.hpp"

namespace lx {
const GameOps *ops_gomoku_b(int n) { return ops_range<Gomoku, 9, 12>(n); }
} // namespace lx
