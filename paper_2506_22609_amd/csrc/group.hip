// Kernel instantiations: the batch-group playout (Tic-Tac-Toe, Connect Four
// and Hex 11x11 batches in one launch) and the one-grid mixed batch
// (Tic-Tac-Toe, Connect Four, Reversi, Hex 11x11, Gomoku 15x15).
#include "kernels.hpp"

namespace lx {

hipError_t launch_playout_group(const GroupArgs &a, bool from_start, hipStream_t s)
{
    const unsigned blocks = (unsigned)a.first_block[a.nb];
    if (from_start)
        hipLaunchKernelGGL((k_playout_group<true, PlayoutGroup>), dim3(blocks), dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL((k_playout_group<false, PlayoutGroup>), dim3(blocks), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mixed_group(const MixedGroupArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_persist_group<PersistGroup>), dim3((unsigned)a.first_block[a.n]), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

} // namespace lx
