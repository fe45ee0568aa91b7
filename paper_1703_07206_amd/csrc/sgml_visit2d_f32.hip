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

template void launch_visit_end2d<float>(const Variant &, const VisitArgs &, const CycleEndArgs &, hipStream_t);
template void launch_visit_end2d_r<float, 0>(const VisitArgs &, const CycleEndArgs &, hipStream_t);
bool visit_end_supported(int sweeps) { return sweeps == 1 || sweeps == 2 || sweeps == 4 || sweeps == 6; }

}  // namespace sgml
