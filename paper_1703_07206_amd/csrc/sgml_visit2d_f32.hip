// sgml_visit2d_f32.hip -- the 2D row-marching visit and cycle-end pass in
// float, axis stencil (the kernels are in sgml_visit2d_impl.h; one precision
// and stencil per file so that the four compile in parallel).
#include "sgml_visit2d_impl.h"

namespace sgml {

bool fused_visit_supported(int sweeps) { return sweeps == 1 || sweeps == 2 || sweeps == 4 || sweeps == 6; }

template void launch_cycle_end2d<float>(const Variant &, const CycleEndArgs &, hipStream_t);
template void launch_visit2d<float>(const Variant &, const VisitArgs &, hipStream_t);
template void launch_visit2d_r<float, 0>(const VisitArgs &, bool, hipStream_t);
template void launch_restrict2d<float>(int, const float *, float *, hipStream_t);
template void launch_restrict2d2<float>(int, const float *, float *, float *, hipStream_t);

template void launch_visit_end2d<float>(const Variant &, const VisitArgs &, const CycleEndArgs &, hipStream_t);
template void launch_visit_end2d_r<float, 0>(const VisitArgs &, const CycleEndArgs &, hipStream_t);
// by default fused where level 0 is large: on smaller levels one wavefront's
// longer row pipeline, not memory traffic, sets the time of the fused pass
bool visit_end_supported(int sweeps, int m, bool any_size)
{
    if (!(sweeps == 1 || sweeps == 2 || sweeps == 4 || sweeps == 6)) return false;
    if (any_size) return true;
    const int W = 128 - 2 * ((sweeps + 2) / 2 * 2 + 2);
    return (long long)((m + W - 1) / W) * m >= kLargeLevelRows;
}

}  // namespace sgml
