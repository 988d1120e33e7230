// mm_fused2d.hip -- fused phase-space pass (x-transport, y-transport, G-hat,
// relaxation and heat-flux tensor in one read of G^n and one write of G^{n+1}).
#include "mm_device.h"
#include "mm_launch.h"

namespace mm {

bool fused_supported(const Params &, int) { return false; }

void launch_micro_fused2d(const void *, void *, double *, const double *, const double *, const Params &, int,
                          hipStream_t)
{
}

} // namespace mm
