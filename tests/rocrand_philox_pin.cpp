// Test helper: exposes rocRAND's host-side Philox4x32-10 engine (a library
// implementation independent of the oracle) so a test can pin the oracle's
// Philox block function to it.  Built host-only by the test that uses it.
#include <rocrand/rocrand_philox4x32_10.h>
#include <stdint.h>

extern "C" void pin_philox(uint64_t seed, uint64_t subsequence, uint64_t offset, uint32_t out[4])
{
    rocrand_device::philox4x32_10_engine e(seed, subsequence, offset);
    for (int i = 0; i < 4; i++) out[i] = e();
}
