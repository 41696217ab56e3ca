// Kernel instantiations: Gomoku N x N for N = 13 .. 15.
#include "kernels.hpp"

namespace lx {
const GameOps *ops_gomoku_c(int n) { return ops_range<Gomoku, 13, 15>(n); }
} // namespace lx
