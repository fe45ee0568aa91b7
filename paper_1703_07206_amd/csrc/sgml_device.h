// sgml_device.h -- device helpers shared by the SGML kernels.
#pragma once

#include "sgml_internal.h"

namespace sgml {

__device__ __forceinline__ size_t lin(int i, int j, int k, int m)
{
    return ((size_t)k * (size_t)m + (size_t)j) * (size_t)m + (size_t)i;
}

// Image of a coordinate across a face (node reflection).  For unknown nodes
// it only triggers at Neumann faces: an unknown is never on a Dirichlet face.
__device__ __forceinline__ int mir(int c, int m)
{
    c = c < 0 ? -c : c;
    return c > m - 1 ? 2 * (m - 1) - c : c;
}

template <int DIM>
__device__ __forceinline__ bool is_dir(int i, int j, int k, int m, unsigned dir)
{
    bool d = ((dir & 1u) && i == 0) || ((dir & 2u) && i == m - 1) || ((dir & 4u) && j == 0) ||
             ((dir & 8u) && j == m - 1);
    if (DIM == 3) d = d || ((dir & 16u) && k == 0) || ((dir & 32u) && k == m - 1);
    return d;
}

// Order-independent max of non-negative doubles (and NaN, whose bit pattern
// with a clear sign bit exceeds that of +inf): integer max of the bits,
// accumulated per block and then into one slot of a reduction target.
__device__ __forceinline__ unsigned long long dbits(double x)
{
    return (unsigned long long)__double_as_longlong(fabs(x));
}

}  // namespace sgml
