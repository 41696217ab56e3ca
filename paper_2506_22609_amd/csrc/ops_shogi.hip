// Kernel instantiations: Dai Hasami Shogi on the 9x9 board.
#include "shogi.hpp"

namespace lx {

const GameOps *ops_hasami_shogi(int rows, int cols)
{
    static const GameOps o = ShogiLaunch::ops();
    return rows == 9 && cols == 9 ? &o : nullptr;
}

} // namespace lx
