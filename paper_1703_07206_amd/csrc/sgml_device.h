// sgml_device.h -- device helpers shared by the SGML kernels.
#pragma once

#include "sgml_internal.h"

namespace sgml {

// Linear index of node (i, j, k) of an m^d array, in index type I (int where
// the array is known to be small, as in LDS).
template <typename I>
__device__ __forceinline__ I lin_as(int i, int j, int k, int m)
{
    return ((I)k * (I)m + (I)j) * (I)m + (I)i;
}

__device__ __forceinline__ size_t lin(int i, int j, int k, int m) { return lin_as<size_t>(i, j, k, m); }

// Image of a coordinate across a face (node reflection).  For unknown nodes
// it only triggers at Neumann faces: an unknown is never on a Dirichlet face.
__device__ __forceinline__ int mir(int c, int m)
{
    c = c < 0 ? -c : c;
    return c > m - 1 ? 2 * (m - 1) - c : c;
}

// Whether node (i, j, k) lies on a Dirichlet face (bit f of dir: face f of
// x-, x+, y-, y+, z-, z+).  Bitwise, so that it compiles without branches.
template <int DIM>
__device__ __forceinline__ bool is_dir(int i, int j, int k, int m, unsigned dir)
{
    bool d = (((dir & 1u) != 0) & (i == 0)) | (((dir & 2u) != 0) & (i == m - 1)) |
             (((dir & 4u) != 0) & (j == 0)) | (((dir & 8u) != 0) & (j == m - 1));
    if (DIM == 3) d = d | (((dir & 16u) != 0) & (k == 0)) | (((dir & 32u) != 0) & (k == m - 1));
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
