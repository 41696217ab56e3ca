// Kernel instantiations: the batch-group playout (Tic-Tac-Toe, Connect Four
// and Hex 11x11 batches in one launch).
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

} // namespace lx
