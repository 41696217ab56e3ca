// Kernel instantiations: Pente on 7x7, 9x9 and 19x19.
#include "kernels.hpp"

namespace lx {

const GameOps *ops_pente(int rows, int cols)
{
    static const GameOps o7 = Launch<Pente<7>>::ops(), o9 = Launch<Pente<9>>::ops(),
                         o19 = Launch<Pente<19>>::ops();
    if (rows != cols) return nullptr;
    switch (rows) {
    case 7: return &o7;
    case 9: return &o9;
    case 19: return &o19;
    default: return nullptr;
    }
}

} // namespace lx
