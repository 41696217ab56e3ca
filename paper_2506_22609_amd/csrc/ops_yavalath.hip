// Kernel instantiations: Yavalath on hexagons of diameter 3, 5, 7 and 9.
#include "kernels.hpp"

namespace lx {

const GameOps *ops_yavalath(int rows, int cols)
{
    static const GameOps o3 = Launch<Yavalath<3>>::ops(), o5 = Launch<Yavalath<5>>::ops(),
                         o7 = Launch<Yavalath<7>>::ops(), o9 = Launch<Yavalath<9>>::ops();
    if (rows != cols) return nullptr;
    switch (rows) {
    case 3: return &o3;
    case 5: return &o5;
    case 7: return &o7;
    case 9: return &o9;
    default: return nullptr;
    }
}

} // namespace lx
