// Kernel instantiations: Gomoku N x N for N = 16 .. 17.
#include "kernels.hpp"

namespace lx {
const GameOps *ops_gomoku_d(int n) { return ops_range<Gomoku, 16, 17>(n); }
} // namespace lx
