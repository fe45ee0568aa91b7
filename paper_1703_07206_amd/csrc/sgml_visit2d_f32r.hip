// sgml_visit2d_f32r.hip -- the 2D row-marching visit in float, radial
// stencil (kernels in sgml_visit2d_impl.h).
#include "sgml_visit2d_impl.h"

namespace sgml {

template void launch_visit2d_r<float, 1>(const VisitArgs &, bool, hipStream_t);

template void launch_visit_end2d_r<float, 1>(const VisitArgs &, const CycleEndArgs &, hipStream_t);

}  // namespace sgml
