// Kernel instantiations: Tic-Tac-Toe 3x3, Connect Four 6x7, Reversi 8x8.
#include "kernels.hpp"

namespace lx {

const GameOps *ops_tictactoe(int rows, int cols)
{
    static const GameOps o = Launch<TicTacToe>::ops();
    return (rows == 3 && cols == 3) ? &o : nullptr;
}

const GameOps *ops_connect_four(int rows, int cols)
{
    static const GameOps o = Launch<ConnectFour>::ops();
    return (rows == 6 && cols == 7) ? &o : nullptr;
}

const GameOps *ops_reversi(int rows, int cols)
{
    static const GameOps o = Launch<Reversi>::ops();
    return (rows == 8 && cols == 8) ? &o : nullptr;
}

} // namespace lx
