// Layout of the edge-prep records (device code only; included by the kernel
// sources).
#pragma once

#include <hip/hip_runtime.h>

namespace fblts {

// Edge-prep records of the n = E * nm edge items of a state (item = edge * nm
// + member), stored split by use in 4n doubles: (l F, q_e) as a double2 at
// [0, 2n) -- gathered for every edges_on_edge neighbour --, l u at [2n, 3n)
// -- neighbours' tangential velocity, with drag or wind --, and h_e at
// [3n, 4n) -- the edge's own, with drag or wind.
__device__ __forceinline__ double2 rec_fq(const double* P, long k) { return reinterpret_cast<const double2*>(P)[k]; }
__device__ __forceinline__ double rec_q(const double* P, long k) { return P[2 * k + 1]; }
__device__ __forceinline__ double rec_lu(const double* P, long n, long k) { return P[2 * n + k]; }
__device__ __forceinline__ double rec_he(const double* P, long n, long k) { return P[3 * n + k]; }

}  // namespace fblts
