// sgml_visit2d_f64.hip -- the 2D row-marching visit and cycle-end pass in
// double, axis stencil (the kernels are in sgml_visit2d_impl.h; one precision
// and stencil per file so that the four compile in parallel).
#include "sgml_visit2d_impl.h"

namespace sgml {

template void launch_cycle_end2d<double>(const Variant &, const CycleEndArgs &, hipStream_t);
template void launch_visit2d<double>(const Variant &, const VisitArgs &, hipStream_t);
template void launch_visit2d_r<double, 0>(const VisitArgs &, bool, hipStream_t);
template void launch_restrict2d<double>(int, const double *, double *, hipStream_t);
template void launch_restrict2d2<double>(int, const double *, double *, double *, hipStream_t);

}  // namespace sgml
