// Kernel instantiations: the movement games, Wolf and Sheep and English
// Draughts on the 8x8 board.
#include "moves.hpp"

namespace lx {

const GameOps *ops_wolf_sheep(int rows, int cols)
{
    static const GameOps o = MoveLaunch<DiagGame<8>>::ops();
    return rows == 8 && cols == 8 ? &o : nullptr;
}

const GameOps *ops_draughts(int rows, int cols)
{
    static const GameOps o = MoveLaunch<DiagGame<9>>::ops();
    return rows == 8 && cols == 8 ? &o : nullptr;
}

} // namespace lx
