// The edge-prep records: their layout and their computation (device code
// only; included by the forward and the adjoint kernel sources).
#pragma once

#include <hip/hip_runtime.h>

#include "fblts_internal.h"

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

// q at an edge's two vertices v0, v1 from the per-edge copies of their lists:
// the same operations, in the same order, as vertex_q.
__device__ __forceinline__ void edge_vertices_q(const MeshDev& m, int e, int v0, int v1, const double* __restrict__ Usrc,
                                                const double* __restrict__ hs, int nm, int mem, double& q0,
                                                double& q1) {
  int code[6], cell[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    code[k] = m.e_vq_edge[k * m.es + e];
    cell[k] = m.e_vq_cell[k * m.es + e];
  }
  double q[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int v = side ? v1 : v0;
    double circ = 0.0, hv = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int k = 3 * side + j;
      const int ed = code[k] >> 1;
      const double c = m.e_dc[ed] * Usrc[(long)ed * nm + mem];
      circ = (code[k] & 1) ? circ - c : circ + c;
      hv = fma(m.v_kite[j * m.vs + v], hs[(long)cell[k] * nm + mem], hv);
    }
    const double ia = m.v_invA[v];
    q[side] = (circ * ia + m.v_f[v]) / (hv * ia);
  }
  q0 = q[0];
  q1 = q[1];
}

// The record of edge e, member mem of nm (np = E * nm items), at the point
// (Usrc, hs): l F with F = h_e u (h_e = H_e when LINEAR, the mean of the two
// cells' h* otherwise), q_e = (q_v0 + q_v1) / 2 (q_v read from q, or with
// FUSE_Q evaluated from u and h* at the edge's two vertices), l u and h_e.
template <bool LINEAR, bool FUSE_Q>
__device__ __forceinline__ void prep_record(const MeshDev& m, int e, int mem, int nm, long np, const double* Usrc,
                                            const double* hs, const double* q, double* P) {
  const int c0 = m.e_cell[e], c1 = m.e_cell[m.es + e];
  const int v0 = m.e_vert[e], v1 = m.e_vert[m.es + e];
  const double u = Usrc[(long)e * nm + mem];
  const double dv = m.e_dv[e];
  double he, qe;
  if constexpr (LINEAR) {
    he = m.e_He[e];
    qe = 0.5 * (q[v0] + q[v1]);
  } else {
    he = 0.5 * (hs[(long)c0 * nm + mem] + hs[(long)c1 * nm + mem]);
    if (FUSE_Q) {
      double q0, q1;
      edge_vertices_q(m, e, v0, v1, Usrc, hs, nm, mem, q0, q1);
      qe = 0.5 * (q0 + q1);
    } else {
      qe = 0.5 * (q[(long)v0 * nm + mem] + q[(long)v1 * nm + mem]);
    }
  }
  const long k = (long)e * nm + mem;
  reinterpret_cast<double2*>(P)[k] = make_double2(dv * (he * u), qe);
  P[2 * np + k] = dv * u;
  P[3 * np + k] = he;
}

}  // namespace fblts
