// Kernel instantiations: Gomoku N x N for N = 18 .. 19.
#include "kernels.hpp"

namespace lx {
const GameOps *ops_gomoku_e(int n) { return ops_range<Gomoku, 18, 19>(n); }
} // namespace lx
