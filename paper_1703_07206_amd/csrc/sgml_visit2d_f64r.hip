// sgml_visit2d_f64r.hip -- the 2D row-marching visit in double, radial
// stencil (kernels in sgml_visit2d_impl.h).
#include "sgml_visit2d_impl.h"

namespace sgml {

template void launch_visit2d_r<double, 1>(const VisitArgs &, bool, hipStream_t);

}  // namespace sgml
