// gfx950 kernels of the FB-LTS hot path.
//
// One stage of FB-RK(3,2) (paper Section 2.1, eq. fbrk32) -- and therefore of
// the coarse advancement and of every fine substep of FB-LTS (Section 2.2) --
// runs as four gather passes over contiguous index ranges:
//   cell pass   : Psi (eq. trisk_thickness), the FB stage update of h, the
//                 FB-averaged thickness h*, and B = K + g(h* - H);
//   vertex pass : potential vorticity q_v = (zeta_v + f_v) / h*_v;
//   prep pass   : per-edge (l F, q_e, l u, h_e), stored split by use (the
//                 (l F, q_e) pair, then l u, then h_e: neighbours read 16 or
//                 24 bytes of it, not 32);
//   edge pass   : Phi (PV flux through the TRiSK weights, eq. trisk_vorticity,
//                 Bernoulli gradient, quadratic drag and wind stress of
//                 eq. hurricane_model), the FB stage update of u.
// The work is HBM/L2-gather bound (well below one FP64 flop per byte), so
// there is no matrix-core path: lanes map to (entity, member) pairs with the
// member index fastest, blocks are remapped so that each XCD works on a
// contiguous slice of the range (its L2 then holds that slice's neighbours),
// and every value has exactly one writer (no atomics; bitwise deterministic).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fblts_internal.h"
#include "prep_record.h"

namespace fblts {

// Blocks are dispatched round-robin over the 8 XCDs; give XCD x the
// contiguous tile run [start(x), start(x)+count(x)).
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int X = 8;
  const int q = n / X, r = n % X;
  const int x = b % X, k = b / X;
  return x * q + (x < r ? x : r) + k;
}

// Segment of block b.  ONE: the launch has a single segment (every solver,
// and ensembles of one mesh), so the segment's fields sit at fixed argument
// offsets and their scalar loads issue in the kernel's first round instead
// of after the lookup.
template <bool ONE, class S>
__device__ __forceinline__ int find_seg(const Launch<S>& L, int b) {
  if constexpr (ONE) {
    return 0;
  } else {
    int s = 0;
#pragma unroll
    for (int k = 1; k < kMaxSeg; ++k)
      if (k < L.nseg && b >= L.blk_start[k]) s = k;
    return s;
  }
}

// First block of segment s (segment 0 starts at block 0).
template <bool ONE, class S>
__device__ __forceinline__ int seg_block(const Launch<S>& L, int s) {
  if constexpr (ONE) return 0;
  else return L.blk_start[s];
}

// Force kernel-argument values into scalar registers at this point.  Placed
// before a kernel's range check, it makes the segment's pointers load in the
// same scalar round as its bounds, ahead of the first gather; left alone, the
// compiler sinks each load next to its first use and the kernel waits for
// several dependent rounds.  The asm is empty: it only consumes the values.
template <typename T>
__device__ __forceinline__ void sgpr_ready1(const T& v) {
  asm volatile("" ::"s"(v));
}
template <typename... T>
__device__ __forceinline__ void sgpr_ready(const T&... v) {
  (sgpr_ready1(v), ...);
}

// ------------------------------------------------- prediction arithmetic
// Interface-one prediction (eq. preds) at fine substep k from the values at
// t^n (yn) and the coarse stage values (y_s, y3): each product rounded, then
// summed left to right (the library is built without contraction).  At k = 0
// the y3 term is a zero product, and adding it changes nothing, so the k = 0
// values are formed without it while y3 does not exist yet.
__device__ __forceinline__ double pred_n(double a, double y3, double one_minus_a, double yn) {
  return a * y3 + one_minus_a * yn;
}
__device__ __forceinline__ double pred_s(double a, double y3, double invM, double ys, double c, double yn) {
  return a * y3 + invM * ys + c * yn;
}
__device__ __forceinline__ double pred_3(double ap, double y3, double c, double yn) { return ap * y3 + c * yn; }

// A coarse stage's hand-over of item i (flat index ii) to the fine arrays.
__device__ __forceinline__ void mirror_store(const Mirror& M, int i, long ii, double y, double y0, int nm_log2) {
  if (M.dst == nullptr || i < M.b || i >= M.e) return;
  if (i < M.p) {
    M.dst[ii] = M.a * y + M.c * y0;
    if (M.sv != nullptr) M.sv[ii - ((long)M.b << nm_log2)] = y0;
  } else {
    M.dst[ii] = y;
  }
}

// The folded prediction / assembly of an edge by its own thread (after its
// own update and accumulation; afin = the accumulated tendency).
__device__ __forceinline__ void tail_own_edge(const StepTail& T, int e, long ee, int nm_log2, double afin) {
  if (e < T.e_b) return;
  const long t = ee - ((long)T.e_b << nm_log2);
  if (T.kind == 1) {
    if (e >= T.e_p) return;
    const double un = T.sv_u[t], u3 = T.D3[ee];
    const double u1 = T.D1[ee], u2 = T.D2[ee];
    T.U0[ee] = pred_n(T.a, u3, T.one_minus_a, un);
    T.U1[ee] = pred_s(T.a, u3, T.invM, u1, T.c, un);
    T.U2[ee] = pred_s(T.a, u3, T.invM, u2, T.c, un);
  } else {
    if (e >= T.e_q) return;
    double base;
    if (e < T.e_p) base = T.sv_u[t];
    else base = T.U0[ee];
    T.U0[ee] = fma(T.delta, afin, base);
  }
}

// The folded work's extra items: t counts from 0 after the pass's edges.
__device__ __forceinline__ void tail_item(const StepTail& T, long t, int nm_log2) {
  if (T.kind == 1) {
    if (t >= ((long)(T.c_p - T.c_b) << nm_log2)) return;
    const long i = ((long)T.c_b << nm_log2) + t;
    const double hn = T.sv_h[t], h3 = T.C3[i];
    const double h1 = T.C1[i], h2 = T.C2[i];
    T.H0[i] = pred_n(T.a, h3, T.one_minus_a, hn);
    T.H1[i] = pred_s(T.a, h3, T.invM, h1, T.c, hn);
    T.H2[i] = pred_s(T.a, h3, T.invM, h2, T.c, hn);
    T.H3[i] = pred_3(T.ap, h3, T.c, hn);
  } else {
    const long nc = (long)(T.c_e - T.c_b) << nm_log2;
    if (t < nc) {
      const long i = ((long)T.c_b << nm_log2) + t;
      const int c = (int)(i >> nm_log2);
      if (c < T.c_p) T.H0[i] = fma(T.delta, T.acc_h[i], T.sv_h[t]);
      else if (c < T.c_q) T.H0[i] = fma(T.delta, T.acc_h[i], T.H0[i]);
      else T.H0[i] = T.C3[i];
    } else if (t - nc < ((long)(T.e_e - T.e_q) << nm_log2)) {
      const long i = ((long)T.e_q << nm_log2) + (t - nc);
      T.U0[i] = T.D3[i];
    }
  }
}

// ---------------------------------------------------------------- cell pass
// MODE 0: linear TRiSK (flux H_e u, B = g(h* - H)); 1: nonlinear (flux h_e u,
// B = K + g(h* - H)); 2: fast terms of the operator splitting, eq. fast_terms
// (flux h_e u, B = g(h* - H), no kinetic energy).
template <int MODE, bool ONE>
__device__ __forceinline__ void cell_body(const Launch<CellSeg>& L, const int b) {
  constexpr bool NONLINEAR = MODE != 0;   // thickness flux with h_e
  constexpr bool KE = MODE == 1;          // kinetic energy in B
  const int s = find_seg<ONE>(L, b);
  const CellSeg& S = L.seg[s];
  if constexpr (ONE) sgpr_ready(L.block, S.m.c_edge, S.m.c_nbr, S.m.cs, S.m.c_nedge, S.Hsrc, S.Usrc, S.m.e_dv, S.m.e_dc);
  const int nm_log2 = S.nm_log2;
  const long item = (long)S.begin * (1L << nm_log2) + (long)(b - seg_block<ONE>(L, s)) * L.block + threadIdx.x;
  const int i = (int)(item >> nm_log2);
  if (i >= S.end) return;
  const int mem = (int)(item & ((1 << nm_log2) - 1));
  const int nm = 1 << nm_log2;
  const MeshDev& m = S.m;

  const bool in_upd = i >= S.upd_begin && i < S.upd_end;
  const bool in_acc = i >= S.acc_begin && i < S.acc_end;
  const bool need_psi = in_upd || in_acc;
  const long ii = (long)i * nm + mem;
  const double h_i = S.Hsrc[ii];
  // the cell's own operands, loaded ahead of the gathers
  const double h0 = S.H0[ii];
  const double invA = m.c_invA[i];
  const double Hrest = m.c_H[i];
  const double hnew_src = in_upd ? 0.0 : S.Hnew_src[ii];
  const double acc0 = (in_acc && !S.acc_first) ? S.acc[ii] : 0.0;
  double flux = 0.0, ke = 0.0;
  const int ne = m.c_nedge[i];
  // Phase 1: the first kUnrollCell slots exist for every cell (padded lists),
  // so all their index loads issue together; phase 2 issues every value
  // gather; phase 3 accumulates with padded slots masked out.  The flux is
  // formed for every cell (it is only used where Psi is needed) so that no
  // branch separates the loads.
  int code[kUnrollCell], nb[kUnrollCell];
#pragma unroll
  for (int j = 0; j < kUnrollCell; ++j) {
    code[j] = m.c_edge[j * m.cs + i];
    nb[j] = m.c_nbr[j * m.cs + i];
  }
  double ue[kUnrollCell], dv[kUnrollCell], dc[kUnrollCell], hx[kUnrollCell];
#pragma unroll
  for (int j = 0; j < kUnrollCell; ++j) {
    const int e = code[j] >> 1;
    ue[j] = S.Usrc[(long)e * nm + mem];
    dv[j] = m.e_dv[e];
    if (NONLINEAR) {
      dc[j] = KE ? m.e_dc[e] : 0.0;
      hx[j] = S.Hsrc[(long)nb[j] * nm + mem];
    } else {
      hx[j] = m.e_He[e];
    }
  }
  // one slot: flux term n_{e,i} l_e h_e u_e, kinetic-energy term l_e d_e u_e^2
  auto acc_slot = [&](int c, double u, double l, double d, double hnb, bool valid) {
    const double he = NONLINEAR ? 0.5 * (h_i + hnb) : hnb;
    double f = l * (he * u);
    f = (c & 1) ? -f : f;
    flux += valid ? f : 0.0;
    if (KE) ke += valid ? l * d * (u * u) : 0.0;
  };
#pragma unroll
  for (int j = 0; j < kUnrollCell; ++j) acc_slot(code[j], ue[j], dv[j], dc[j], hx[j], j < ne);
  for (int j = kUnrollCell; j < ne; ++j) {
    const int c = m.c_edge[j * m.cs + i];
    const int e = c >> 1;
    const double u = S.Usrc[(long)e * nm + mem];
    const double hnb = NONLINEAR ? S.Hsrc[(long)m.c_nbr[j * m.cs + i] * nm + mem] : m.e_He[e];
    acc_slot(c, u, m.e_dv[e], KE ? m.e_dc[e] : 0.0, hnb, true);
  }
  (void)need_psi;
  const double psi = -flux * invA;
  double hnew;
  if (in_upd) {
    hnew = fma(S.c_dt, psi, h0);
    S.Hdst[ii] = hnew;
    mirror_store(S.mir, i, ii, hnew, h0, nm_log2);
  } else {
    hnew = hnew_src;
  }
  if (in_acc) {
    const double a = S.acc_w * psi;
    S.acc[ii] = S.acc_first ? a : acc0 + a;
  }
  const double hs = S.wn * hnew + S.ws * h_i + S.wb * h0;
  S.hs[ii] = hs;
  const double K = KE ? 0.25 * ke * invA : 0.0;
  S.B[ii] = K + S.g * (hs - Hrest);
}

template <int MODE, bool ONE>
__global__ void __launch_bounds__(kBlock) k_cell(const Launch<CellSeg> L) {
  cell_body<MODE, ONE>(L, xcd_tile(blockIdx.x, gridDim.x));
}

// -------------------------------------------------------------- vertex pass
// q_v = (zeta_v + f_v) / h_v with zeta_v = (1/A_v) sum s_{e,v} d_e u_e and
// h_v = (1/A_v) sum kite_{i,v} h*_i.  Shared by the vertex pass and the fused
// prep pass, so both produce the same bits.
__device__ __forceinline__ double vertex_q(const MeshDev& m, int v, const double* __restrict__ Usrc,
                                           const double* __restrict__ hs, int nm, int mem) {
  int code[3], cell[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    code[j] = m.v_edge[j * m.vs + v];
    cell[j] = m.v_cell[j * m.vs + v];
  }
  double circ = 0.0, hv = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int e = code[j] >> 1;
    const double c = m.e_dc[e] * Usrc[(long)e * nm + mem];
    circ = (code[j] & 1) ? circ - c : circ + c;
    hv = fma(m.v_kite[j * m.vs + v], hs[(long)cell[j] * nm + mem], hv);
  }
  const double ia = m.v_invA[v];
  return (circ * ia + m.v_f[v]) / (hv * ia);
}

template <bool ONE>
__device__ __forceinline__ void vertex_body(const Launch<VertSeg>& L, const int b) {
  const int s = find_seg<ONE>(L, b);
  const VertSeg& S = L.seg[s];
  if constexpr (ONE) sgpr_ready(L.block, S.m.v_edge, S.m.v_cell, S.m.vs, S.Usrc, S.hs, S.m.e_dc, S.q);
  const int nm_log2 = S.nm_log2;
  const long item = (long)S.begin * (1L << nm_log2) + (long)(b - seg_block<ONE>(L, s)) * L.block + threadIdx.x;
  const int v = (int)(item >> nm_log2);
  if (v >= S.end) return;
  const int mem = (int)(item & ((1 << nm_log2) - 1));
  const int nm = 1 << nm_log2;
  S.q[(long)v * nm + mem] = vertex_q(S.m, v, S.Usrc, S.hs, nm, mem);
}

template <bool ONE>
__global__ void __launch_bounds__(kBlock) k_vertex(const Launch<VertSeg> L) {
  vertex_body<ONE>(L, xcd_tile(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------- prep pass
// FUSE_Q: evaluate q at the edge's two vertices here instead of reading the
// vertex pass's output (one launch fewer per stage, each vertex evaluated by
// its three edges).
template <bool LINEAR, bool FUSE_Q, bool ONE>
__device__ __forceinline__ void prep_body(const Launch<PrepSeg>& L, const int b) {
  const int s = find_seg<ONE>(L, b);
  const PrepSeg& S = L.seg[s];
  if constexpr (ONE) {
    sgpr_ready(L.block, S.m.e_cell, S.m.e_vert, S.m.es, S.m.E, S.Usrc, S.m.e_dv, S.hs, S.P);
    if constexpr (FUSE_Q) sgpr_ready(S.m.e_vq_edge, S.m.e_vq_cell, S.m.e_dc, S.m.v_kite, S.m.vs);
  }
  const int nm_log2 = S.nm_log2;
  const long item = (long)S.begin * (1L << nm_log2) + (long)(b - seg_block<ONE>(L, s)) * L.block + threadIdx.x;
  const int e = (int)(item >> nm_log2);
  if (e >= S.end) return;
  const int mem = (int)(item & ((1 << nm_log2) - 1));
  const int nm = 1 << nm_log2;
  const MeshDev& m = S.m;
  prep_record<LINEAR, FUSE_Q>(m, e, mem, nm, (long)m.E << nm_log2, S.Usrc, S.hs, S.q, S.P);
}

template <bool LINEAR, bool FUSE_Q, bool ONE>
__global__ void __launch_bounds__(kBlock) k_prep(const Launch<PrepSeg> L) {
  prep_body<LINEAR, FUSE_Q, ONE>(L, xcd_tile(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------- edge pass
// PV flux through one cell's edge list (CELLS variant of the momentum pass):
// walk the cell's other edges counter-clockwise starting after e and form the
// TRiSK weight w = n_{e,i} n_{e',i} (1/2 - sum of the kite fractions passed),
// the same weights, in the same order, as the cell's part of e's
// edges_on_edge list.  w = (slot << 0) | (degree << 4) of e in this cell.
template <bool NEED_U>
__device__ __forceinline__ void walk_cell(const MeshDev& m, const double* __restrict__ P, long np, int i, int w,
                                          double pey, int nm, int mem, double& sq, double& su) {
  constexpr int U = kUnrollCell - 1;   // walk positions whose loads issue together
  const int j0 = w & 15, n = (w >> 4) & 15;
  const int se = m.c_edge[j0 * m.cs + i] & 1;
  int code[U];
  double R[U];
#pragma unroll
  for (int t = 0; t < U; ++t) {
    // position t + 1: previous slot (j0 + t) mod n, slot (j0 + t + 1) mod n;
    // positions past the degree load valid slots and are masked below
    int jp = j0 + t;
    jp -= jp >= n ? n : 0;
    jp -= jp >= n ? n : 0;
    int j = jp + 1;
    j -= j >= n ? n : 0;
    R[t] = m.c_R[jp * m.cs + i];
    code[t] = m.c_edge[j * m.cs + i];
  }
  double2 p2[U];
  double lu[U];
#pragma unroll
  for (int t = 0; t < U; ++t) {
    const long k = (long)(code[t] >> 1) * nm + mem;
    p2[t] = rec_fq(P, k);
    lu[t] = NEED_U ? rec_lu(P, np, k) : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < U; ++t) {
    if (t + 1 < n) {
      acc = acc + R[t];
      double wt = 0.5 - acc;
      wt = (code[t] & 1) != se ? -wt : wt;
      sq = fma(wt * p2[t].x, pey + p2[t].y, sq);
      if (NEED_U) su = fma(wt, lu[t], su);
    }
  }
  int j = j0 + U;
  while (j >= n) j -= n;
  for (int mm = U + 1; mm < n; ++mm) {
    const int jp = j;
    j = j + 1 == n ? 0 : j + 1;
    acc = acc + m.c_R[jp * m.cs + i];
    const int c = m.c_edge[j * m.cs + i];
    double wt = 0.5 - acc;
    wt = (c & 1) != se ? -wt : wt;
    const long k = (long)(c >> 1) * nm + mem;
    const double2 q = rec_fq(P, k);
    sq = fma(wt * q.x, pey + q.y, sq);
    if (NEED_U) su = fma(wt, rec_lu(P, np, k), su);
  }
}

// CELLS: the PV flux through the two cells' edge lists and kite fractions
// (walk_cell) instead of the edges_on_edge list and stored weights; only for
// meshes whose stored weights are exactly those walks (the planner checks).
// GROUP (every segment has at least 16 members and at most 16 edges_on_edge
// slots): the members of an edge fill whole 16-lane groups of the wavefront,
// so lane r of each group loads slot r's index and weight once and the group
// shares them through cross-lane permutes instead of every lane loading every
// slot; all maxEOE slots are taken (the padding slots are exact no-ops), so
// every lane of the group takes part in every permute.
template <bool DRAG, bool WIND, bool CELLS, bool ONE, bool GROUP>
__device__ __forceinline__ void edge_body(const Launch<EdgeSeg>& L, const int b) {
  const int s = find_seg<ONE>(L, b);
  const EdgeSeg& S = L.seg[s];
  if constexpr (ONE) {
    sgpr_ready(L.block, S.P, S.B, S.m.es, S.m.E, S.m.e_cell, S.m.e_invdc);
    if constexpr (CELLS) sgpr_ready(S.m.e_cs, S.m.c_edge, S.m.c_R, S.m.cs);
    else sgpr_ready(S.m.e_eoe, S.m.e_w, S.m.e_neoe, S.m.maxEOE);
  }
  const int nm_log2 = S.nm_log2;
  const long item = (long)S.begin * (1L << nm_log2) + (long)(b - seg_block<ONE>(L, s)) * L.block + threadIdx.x;
  const int e = (int)(item >> nm_log2);
  if (e >= S.end) {
    if (S.tail.kind != 0) tail_item(S.tail, item - ((long)S.end << nm_log2), nm_log2);
    return;
  }
  const int mem = (int)(item & ((1 << nm_log2) - 1));
  const int nm = 1 << nm_log2;
  const MeshDev& m = S.m;
  const double* P = S.P;
  const long np = (long)m.E << nm_log2;
  const long ee = (long)e * nm + mem;
  // the edge's own operands, loaded ahead of the neighbour gathers so that
  // they share the gathers' rounds instead of following them
  const int c0 = m.e_cell[e], c1 = m.e_cell[m.es + e];
  const double idc = m.e_invdc[e];
  const double B0 = S.B[(long)c0 * nm + mem], B1 = S.B[(long)c1 * nm + mem];
  const double pey = rec_q(P, ee);
  const double he = (DRAG || WIND) ? rec_he(P, np, ee) : 1.0;
  const double u = (DRAG || WIND) ? S.Usrc[ee] : 0.0;
  const double cde = DRAG ? 0.5 * (S.cd[(long)c0 * nm + mem] + S.cd[(long)c1 * nm + mem]) : 0.0;
  const double wn = WIND ? S.wind_n[ee] : 0.0, wt = WIND ? S.wind_t[ee] : 0.0;
  const double cw = WIND ? S.wind_c[ee] : 0.0;
  const bool upd = e >= S.upd_begin && e < S.upd_end, acc = e >= S.acc_begin && e < S.acc_end;
  const double u0 = upd ? S.U0[ee] : 0.0;
  const double acc0 = (acc && !S.acc_first) ? S.acc[ee] : 0.0;
  double sq = 0.0, su = 0.0;
  if (CELLS) {
    const int w = m.e_cs[e];
    walk_cell<DRAG || WIND>(m, P, np, m.e_cell[e], w & 0xff, pey, nm, mem, sq, su);
    walk_cell<DRAG || WIND>(m, P, np, m.e_cell[m.es + e], (w >> 8) & 0xff, pey, nm, mem, sq, su);
  } else if (GROUP) {
    const int lane = threadIdx.x & 63, base = lane & ~15, r = lane & 15;
    const int n = m.e_neoe[e];
    int idx_r = e;
    double w_r = 0.0;
    if (r < m.maxEOE) {
      idx_r = m.e_eoe[r * m.es + e];
      w_r = m.e_w[r * m.es + e];
    }
    // a padded slot (past the edge's list) only takes part in the permutes:
    // its term would add an exact zero (sq and su are never -0), so its
    // gathers are not issued
    auto slot = [&](int j) {
      const int e2 = __shfl(idx_r, base + j);
      const double w = __shfl(w_r, base + j);
      if (j < kEOEFull || j < n) {
        const long k2 = (long)e2 * nm + mem;
        const double2 p2 = rec_fq(P, k2);
        sq = fma(w * p2.x, pey + p2.y, sq);
        if (DRAG || WIND) su = fma(w, rec_lu(P, np, k2), su);
      }
    };
#pragma unroll
    for (int j = 0; j < kUnrollEOE; ++j) slot(j);
    for (int j = kUnrollEOE; j < m.maxEOE; ++j) slot(j);
  } else {
    const int n = m.e_neoe[e];
    auto slot = [&](int j) {
      const int e2 = m.e_eoe[j * m.es + e];
      const bool real = j < kEOEFull || j < n;
      const double w0 = m.e_w[(real ? j * m.es : 0) + e];
      const double w = real ? w0 : 0.0;
      const long k2 = (long)e2 * nm + mem;
      const double2 p2 = rec_fq(P, k2);
      sq = fma(w * p2.x, pey + p2.y, sq);
      if (DRAG || WIND) su = fma(w, rec_lu(P, np, k2), su);
    };
    // the first kUnrollEOE slots exist for every edge (padded with the edge
    // itself at weight 0, an exact no-op): their index loads issue together;
    // a padded slot past kEOEFull loads the edge's slot-0 weight instead of
    // its own and takes +0 (the stored value, so the same bits) with no line
    // of padding fetched; the loop covers the rare longer lists
#pragma unroll
    for (int j = 0; j < kUnrollEOE; ++j) slot(j);
    for (int j = kUnrollEOE; j < n; ++j) slot(j);
  }
  double phi = 0.5 * sq * idc - (B1 - B0) * idc;
  if (DRAG || WIND) {
    const double up = su * idc;
    if (DRAG) phi -= cde * sqrt(u * u + up * up) * u / he;
    if (WIND) {
      const double rn = wn - u, rt = wt - up;
      phi += cw * sqrt(rn * rn + rt * rt) * rn / he;
    }
  }
  if (upd) {
    const double unew = fma(S.c_dt, phi, u0);
    S.Udst[ee] = unew;
    mirror_store(S.mir, e, ee, unew, u0, nm_log2);
  }
  double afin = 0.0;
  if (acc) {
    const double a = S.acc_w * phi;
    afin = S.acc_first ? a : acc0 + a;
    S.acc[ee] = afin;
  }
  if (S.tail.kind != 0) tail_own_edge(S.tail, e, ee, nm_log2, afin);
}

// Block index of a momentum-pass launch: the edge blocks XCD by XCD, the
// blocks of folded work (if any) after them in dispatch order.
__device__ __forceinline__ int edge_tile(const Launch<EdgeSeg>& L) {
  const int n = L.xcd_n;
  if (n > 0 && (int)blockIdx.x >= n) return blockIdx.x;
  return xcd_tile(blockIdx.x, n > 0 ? n : gridDim.x);
}

template <bool DRAG, bool WIND, bool CELLS, bool ONE, bool GROUP>
__global__ void __launch_bounds__(kBlock) k_edge(const Launch<EdgeSeg> L) {
  edge_body<DRAG, WIND, CELLS, ONE, GROUP>(L, edge_tile(L));
}

// ----------------------------------------------------- fast momentum pass
// Fast momentum tendency of the operator splitting (eq. fast_terms):
// Phi = -(B_c1 - B_c0) / d_e with B = g(h* - H), plus (SLOW) the slow tendency
// frozen at the start of the step or substep (eq. splitting).
template <bool SLOW, bool ONE>
__device__ __forceinline__ void edge_fast_body(const Launch<EdgeSeg>& L, const int b) {
  const int s = find_seg<ONE>(L, b);
  const EdgeSeg& S = L.seg[s];
  if constexpr (ONE) sgpr_ready(L.block, S.B, S.m.es, S.m.e_cell, S.m.e_invdc, S.Udst, S.U0);
  const int nm_log2 = S.nm_log2;
  const long item = (long)S.begin * (1L << nm_log2) + (long)(b - seg_block<ONE>(L, s)) * L.block + threadIdx.x;
  const int e = (int)(item >> nm_log2);
  if (e >= S.end) {
    if (S.tail.kind != 0) tail_item(S.tail, item - ((long)S.end << nm_log2), nm_log2);
    return;
  }
  const int mem = (int)(item & ((1 << nm_log2) - 1));
  const int nm = 1 << nm_log2;
  const MeshDev& m = S.m;
  const long ee = (long)e * nm + mem;
  const int c0 = m.e_cell[e], c1 = m.e_cell[m.es + e];
  double phi = -(S.B[(long)c1 * nm + mem] - S.B[(long)c0 * nm + mem]) * m.e_invdc[e];
  if (SLOW) phi += S.slow[ee];
  if (e >= S.upd_begin && e < S.upd_end) {
    const double u0 = S.U0[ee];
    const double unew = fma(S.c_dt, phi, u0);
    S.Udst[ee] = unew;
    mirror_store(S.mir, e, ee, unew, u0, nm_log2);
  }
  double afin = 0.0;
  if (e >= S.acc_begin && e < S.acc_end) {
    const double a = S.acc_w * phi;
    afin = S.acc_first ? a : S.acc[ee] + a;
    S.acc[ee] = afin;
  }
  if (S.tail.kind != 0) tail_own_edge(S.tail, e, ee, nm_log2, afin);
}

template <bool SLOW, bool ONE>
__global__ void __launch_bounds__(kBlock) k_edge_fast(const Launch<EdgeSeg> L) {
  edge_fast_body<SLOW, ONE>(L, edge_tile(L));
}

// ---------------------------------------------------------- prediction pass
template <bool ONE>
__device__ __forceinline__ void predict_body(const Launch<PredSeg>& L, const int b) {
  const int s = find_seg<ONE>(L, b);
  const PredSeg& S = L.seg[s];
  if constexpr (ONE) sgpr_ready(L.block, S.save, S.c_begin, S.c_end, S.e_begin, S.e_end, S.a, S.invM);
  const int nm_log2 = S.nm_log2;
  const int nm = 1 << nm_log2;
  const long nc = (long)(S.c_end - S.c_begin) * nm;
  const long ne = (long)(S.e_end - S.e_begin) * nm;
  const long t = (long)(b - seg_block<ONE>(L, s)) * L.block + threadIdx.x;
  if (t < nc) {
    const long i = (long)S.c_begin * nm + t;
    double hn, h1, h2, h3;
    if (S.save) {
      hn = S.H0[i]; h1 = S.H1[i]; h2 = S.H2[i]; h3 = S.H3[i];
      S.sv_h[t] = hn; S.sv_h[nc + t] = h1; S.sv_h[2 * nc + t] = h2; S.sv_h[3 * nc + t] = h3;
    } else {
      hn = S.sv_h[t]; h1 = S.sv_h[nc + t]; h2 = S.sv_h[2 * nc + t]; h3 = S.sv_h[3 * nc + t];
    }
    S.H0[i] = pred_n(S.a, h3, S.one_minus_a, hn);
    S.H1[i] = pred_s(S.a, h3, S.invM, h1, S.c, hn);
    S.H2[i] = pred_s(S.a, h3, S.invM, h2, S.c, hn);
    S.H3[i] = pred_3(S.ap, h3, S.c, hn);
  } else if (t < nc + ne) {
    const long tt = t - nc;
    const long i = (long)S.e_begin * nm + tt;
    double un, u1, u2, u3;
    if (S.save) {
      un = S.U0[i]; u1 = S.U1[i]; u2 = S.U2[i]; u3 = S.U3[i];
      S.sv_u[tt] = un; S.sv_u[ne + tt] = u1; S.sv_u[2 * ne + tt] = u2; S.sv_u[3 * ne + tt] = u3;
    } else {
      un = S.sv_u[tt]; u1 = S.sv_u[ne + tt]; u2 = S.sv_u[2 * ne + tt]; u3 = S.sv_u[3 * ne + tt];
    }
    S.U0[i] = pred_n(S.a, u3, S.one_minus_a, un);
    S.U1[i] = pred_s(S.a, u3, S.invM, u1, S.c, un);
    S.U2[i] = pred_s(S.a, u3, S.invM, u2, S.c, un);
  }
}

template <bool ONE>
__global__ void __launch_bounds__(kBlock) k_predict(const Launch<PredSeg> L) {
  predict_body<ONE>(L, blockIdx.x);
}

// ------------------------------------------------------------ assembly pass
template <bool ONE>
__device__ __forceinline__ void assemble_body(const Launch<AsmSeg>& L, const int b) {
  const int s = find_seg<ONE>(L, b);
  const AsmSeg& S = L.seg[s];
  if constexpr (ONE) sgpr_ready(L.block, S.if1_c_begin, S.if1_c_end, S.if2_c_end, S.N, S.if1_e_begin, S.if1_e_end,
                                S.if2_e_end, S.E);
  const int nm = 1 << S.nm_log2;
  const long ncell = (long)(S.N - S.if1_c_begin) * nm;
  const long nedge = (long)(S.E - S.if1_e_begin) * nm;
  const long t = (long)(b - seg_block<ONE>(L, s)) * L.block + threadIdx.x;
  if (t < ncell) {
    const long i = (long)S.if1_c_begin * nm + t;
    const long c = i >> S.nm_log2;
    if (c < S.if1_c_end) {
      S.H0[i] = fma(S.delta, S.acc_h[i], S.sv_h[t]);
    } else if (c < S.if2_c_end) {
      S.H0[i] = fma(S.delta, S.acc_h[i], S.H0[i]);
    } else {
      S.H0[i] = S.H3[i];
    }
  } else if (t < ncell + nedge) {
    const long tt = t - ncell;
    const long i = (long)S.if1_e_begin * nm + tt;
    const long e = i >> S.nm_log2;
    if (e < S.if1_e_end) {
      S.U0[i] = fma(S.delta, S.acc_u[i], S.sv_u[tt]);
    } else if (e < S.if2_e_end) {
      S.U0[i] = fma(S.delta, S.acc_u[i], S.U0[i]);
    } else {
      S.U0[i] = S.U3[i];
    }
  }
}

template <bool ONE>
__global__ void __launch_bounds__(kBlock) k_assemble(const Launch<AsmSeg> L) {
  assemble_body<ONE>(L, blockIdx.x);
}

// -------------------------------------------------------- persistent launch
// A run of passes in one cooperative launch: every block walks the passes in
// order, takes its share of each pass's blocks (each XCD a contiguous slice,
// as xcd_tile does for a separate launch), and waits at a grid barrier before
// the next pass.  Each pass evaluates exactly what its own launch would
// (the same body, item by item), so the results are bitwise those of the
// separate launches.

// Two-level grid barrier: the blocks of group g = blockIdx.x % 8 arrive at
// their group's counter, the last of each group at the top counter, and the
// last group leader advances the generation, which everyone polls.  Device-
// scope atomics are relaxed; fences order the data: a release fence before
// arriving, an acquire-release fence on each leader's path, an acquire fence
// after the wait.  A wait gives up after kSpinLimit polls (seconds) and sets
// the abort flag, which also releases every other waiting block; the launch's
// results are then invalid and the host reports it.
constexpr long kSpinLimit = 1L << 22;

__device__ bool grid_barrier(const GridBar& B) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    const unsigned X = 8, G = gridDim.x, g = blockIdx.x % X;
    const unsigned members = G / X + (g < G % X ? 1u : 0u);
    const unsigned groups = G < X ? G : X;
    unsigned* gen = B.ctr + 400;
    unsigned* grp = B.ctr + 32 * (g + 1);
    const unsigned cur = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    bool last = false;
    if (__hip_atomic_fetch_add(grp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == members - 1) {
      __hip_atomic_store(grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      if (__hip_atomic_fetch_add(B.ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == groups - 1) {
        __hip_atomic_store(B.ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_store(gen, cur + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = true;
      }
    }
    if (!last) {
      long spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == cur) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit || __hip_atomic_load(B.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_store(B.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok != 0;
}

__device__ __forceinline__ void run_pass(const PassDesc& D, int b) {
  switch (D.kind) {
    case PK_CELL:
      if (D.variant == 1) cell_body<1, false>(D.u.cell, b);
      else if (D.variant == 2) cell_body<2, false>(D.u.cell, b);
      else cell_body<0, false>(D.u.cell, b);
      break;
    case PK_VERT: vertex_body<false>(D.u.vert, b); break;
    case PK_PREP:
      if (D.variant == 0) prep_body<true, false, false>(D.u.prep, b);
      else if (D.variant == 1) prep_body<false, false, false>(D.u.prep, b);
      else prep_body<false, true, false>(D.u.prep, b);
      break;
    case PK_EDGE:
      switch (D.variant) {
        case 0: edge_body<false, false, false, false, false>(D.u.edge, b); break;
        case 1: edge_body<true, false, false, false, false>(D.u.edge, b); break;
        case 2: edge_body<false, true, false, false, false>(D.u.edge, b); break;
        case 3: edge_body<true, true, false, false, false>(D.u.edge, b); break;
        case 4: edge_body<false, false, false, false, true>(D.u.edge, b); break;
        case 5: edge_body<true, false, false, false, true>(D.u.edge, b); break;
        case 6: edge_body<false, true, false, false, true>(D.u.edge, b); break;
        default: edge_body<true, true, false, false, true>(D.u.edge, b); break;
      }
      break;
    case PK_EDGE_FAST:
      if (D.variant) edge_fast_body<true, false>(D.u.edge, b);
      else edge_fast_body<false, false>(D.u.edge, b);
      break;
    case PK_PRED: predict_body<false>(D.u.pred, b); break;
    case PK_ASM: assemble_body<false>(D.u.asmb, b); break;
    default: break;
  }
}

__global__ void __launch_bounds__(kBlock) k_persistent(const PassDesc* __restrict__ D, int n, GridBar B) {
  __shared__ PassDesc sd;
  const int G = (int)gridDim.x;
  for (int p = 0; p < n; ++p) {
    // the pass's descriptor, staged in LDS for the whole block
    {
      const unsigned long long* src = reinterpret_cast<const unsigned long long*>(D + p);
      unsigned long long* dst = reinterpret_cast<unsigned long long*>(&sd);
      for (int k = threadIdx.x; k < (int)(sizeof(PassDesc) / 8); k += kBlock) dst[k] = src[k];
    }
    __syncthreads();
    const int nvb = sd.nvb;
    if (nvb > 0) {
      const int X = 8, x = blockIdx.x % X, k = blockIdx.x / X, per = G / X;
      const int lo = (int)((long)nvb * x / X), hi = (int)((long)nvb * (x + 1) / X);
      for (int vb = lo + k; vb < hi; vb += per) run_pass(sd, vb);
    }
    __syncthreads();
    if (nvb > 0 && p + 1 < n && !grid_barrier(B)) return;
  }
}

// RK4 final combination: y <- y + (dt/6) acc over [0,n*nm).
__global__ void __launch_bounds__(kBlock) k_axpy_final(double* y, const double* acc, double c, long n) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) y[t] = fma(c, acc[t], y[t]);
}

// Member scatter/gather between caller numbering and the library's numbering:
// dst[new*nm + member] = src[old(new)] (to_lib) or the reverse.
__global__ void __launch_bounds__(kBlock) k_permute(double* dst, const double* src, const int* perm_new_to_old,
                                                    int n, int nm_log2, int member, int to_lib) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const long lib = ((long)i << nm_log2) + member;
  const int usr = perm_new_to_old[i];
  if (to_lib) dst[lib] = src[usr];
  else dst[usr] = src[lib];
}

__global__ void __launch_bounds__(kBlock) k_copy(double* dst, const double* src, long n) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

__global__ void __launch_bounds__(kBlock) k_fill(double* dst, double v, long n) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) dst[t] = v;
}

// ------------------------------------------------------------- diagnostics
// Per (block, member) partial sums in a fixed tree, then one block per
// member sums the partials in block order: the result does not depend on
// scheduling.  Quantities (kDiagQ): mass, abs vorticity, |abs vorticity|,
// cell energy, edge energy, min h, non-finite count, h <= 0 count.
constexpr int kDiagQ = 8;

// Reduce over the block the values of lanes with equal (tid % nm), nm a power
// of two; the results land in sh[0..nm).  A butterfly inside each 64-lane
// wavefront first (lanes l and l ^ s hold the same member when s >= nm), then
// the per-wavefront results in wavefront order through LDS.  Fixed order, so
// the result is deterministic.  Every thread of the block must call it.
__device__ __forceinline__ void block_reduce(double* sh, double v, int nm, bool is_min) {
  constexpr int kWaves = kBlock / 64;
  if (nm >= 64) {
    // one lane per member in each wavefront: a tree over LDS only
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int stride = kBlock / 2; stride >= nm; stride >>= 1) {
      if (threadIdx.x < stride) {
        const double a = sh[threadIdx.x], c = sh[threadIdx.x + stride];
        sh[threadIdx.x] = is_min ? fmin(a, c) : a + c;
      }
      __syncthreads();
    }
    return;
  }
  for (int s = 32; s >= nm; s >>= 1) {
    const double o = __shfl_xor(v, s);
    v = is_min ? fmin(v, o) : v + o;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane < nm) sh[wave * nm + lane] = v;
  __syncthreads();
  if (threadIdx.x < nm) {
    double r = sh[threadIdx.x];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) {
      const double x = sh[w * nm + threadIdx.x];
      r = is_min ? fmin(r, x) : r + x;
    }
    sh[threadIdx.x] = r;
  }
  __syncthreads();
}

struct DiagArgs {
  MeshDev m;
  int nm_log2;
  int linear;
  const double* h;
  const double* u;
  double g;
  double* partial;    // [kDiagQ][nblocks][nm]
  int nblocks;
};

__global__ void __launch_bounds__(kBlock) k_diag(const DiagArgs A) {
  __shared__ double sh[kBlock];
  const int nm = 1 << A.nm_log2;
  const MeshDev& m = A.m;
  const int mem = threadIdx.x & (nm - 1);
  const int lane_ent = threadIdx.x >> A.nm_log2;
  const int ents_per_pass = kBlock >> A.nm_log2;
  const int nmax = m.N > m.E ? (m.N > m.V ? m.N : m.V) : (m.E > m.V ? m.E : m.V);
  const int chunk = (nmax + A.nblocks - 1) / A.nblocks;
  const int lo = blockIdx.x * chunk;
  const int hi = lo + chunk;
  double q[kDiagQ] = {0, 0, 0, 0, 0, 1e300, 0, 0};
  for (int i = lo + lane_ent; i < hi; i += ents_per_pass) {
    if (i < m.N) {
      const double h = A.h[(long)i * nm + mem];
      const double H = m.c_H[i];
      q[0] += m.c_A[i] * h;
      if (A.linear) q[3] += 0.5 * A.g * m.c_A[i] * (h - H) * (h - H);
      else q[3] += m.c_A[i] * A.g * h * (0.5 * h - H);
      q[5] = fmin(q[5], h);
      if (!isfinite(h)) q[6] += 1.0;
      if (!(h > 0.0)) q[7] += 1.0;
    }
    if (i < m.E) {
      const double u = A.u[(long)i * nm + mem];
      const double he = A.linear ? m.e_He[i]
                                 : 0.5 * (A.h[(long)m.e_cell[i] * nm + mem] + A.h[(long)m.e_cell[m.es + i] * nm + mem]);
      q[4] += 0.5 * m.e_dv[i] * m.e_dc[i] * he * u * u;
      if (!isfinite(u)) q[6] += 1.0;
    }
    if (i < m.V) {
      double circ = 0.0;
      for (int j = 0; j < 3; ++j) {
        const int code = m.v_edge[j * m.vs + i];
        const int e = code >> 1;
        const double c = m.e_dc[e] * A.u[(long)e * nm + mem];
        circ = (code & 1) ? circ - c : circ + c;
      }
      const double eta = circ + m.v_A[i] * m.v_f[i];
      q[1] += eta;
      q[2] += fabs(eta);
    }
  }
  for (int k = 0; k < kDiagQ; ++k) {
    block_reduce(sh, q[k], nm, k == 5);
    if (threadIdx.x < nm) A.partial[((long)k * A.nblocks + blockIdx.x) * nm + threadIdx.x] = sh[threadIdx.x];
    __syncthreads();
  }
}

// One block per member: sum partials over blocks in order (tree over a fixed
// assignment of blocks to threads).
__global__ void __launch_bounds__(kBlock) k_diag_final(const double* partial, int nblocks, int nm, double* out) {
  __shared__ double sh[kBlock];
  const int mem = blockIdx.x;
  for (int k = 0; k < kDiagQ; ++k) {
    const bool is_min = k == 5;
    double v = is_min ? 1e300 : 0.0;
    for (int bb = threadIdx.x; bb < nblocks; bb += kBlock) {
      const double x = partial[((long)k * nblocks + bb) * nm + mem];
      v = is_min ? fmin(v, x) : v + x;
    }
    block_reduce(sh, v, 1, is_min);
    if (threadIdx.x == 0) out[(long)mem * kDiagQ + k] = sh[0];
    __syncthreads();
  }
}

// ------------------------------------------------------------- host launchers
template <class S>
static int blocks_for(Launch<S>& L, long (*items)(const S&), int bs) {
  L.block = bs;
  int acc = 0;
  for (int s = 0; s < L.nseg; ++s) {
    L.blk_start[s] = acc;
    acc += (int)((items(L.seg[s]) + bs - 1) / bs);
  }
  for (int s = L.nseg; s <= kMaxSeg; ++s) L.blk_start[s] = acc;
  return acc;
}

static long cell_items(const CellSeg& s) { return s.end > s.begin ? (long)(s.end - s.begin) << s.nm_log2 : 0; }
static long vert_items(const VertSeg& s) { return s.end > s.begin ? (long)(s.end - s.begin) << s.nm_log2 : 0; }
static long prep_items(const PrepSeg& s) { return s.end > s.begin ? (long)(s.end - s.begin) << s.nm_log2 : 0; }
static long tail_items(const StepTail& t, int nm_log2) {
  if (t.kind == 1) return (long)(t.c_p - t.c_b) << nm_log2;
  if (t.kind == 2) return ((long)(t.c_e - t.c_b) + (long)(t.e_e - t.e_q)) << nm_log2;
  return 0;
}
static long edge_items(const EdgeSeg& s) {
  return (s.end > s.begin ? (long)(s.end - s.begin) << s.nm_log2 : 0) + tail_items(s.tail, s.nm_log2);
}
static long pred_items(const PredSeg& s) {
  return ((long)(s.c_end - s.c_begin) + (long)(s.e_end - s.e_begin)) << s.nm_log2;
}
static long asm_items(const AsmSeg& s) {
  return ((long)(s.N - s.if1_c_begin) + (long)(s.E - s.if1_e_begin)) << s.nm_log2;
}

// Kernel timing: when a pair of events is armed, the next stencil-pass launch
// records them from its own dispatch (start and end timestamps of the kernel,
// no marker packets in between), then the pair is disarmed.
static thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

void arm_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_ev_start = start;
  g_ev_stop = stop;
}

template <typename F, typename... A>
static void launch_timed(F kernel, int nb, int bs, hipStream_t st, A... args) {
  if (g_ev_start) {
    hipExtLaunchKernelGGL(kernel, dim3(nb), dim3(bs), 0, st, g_ev_start, g_ev_stop, 0, args...);
    g_ev_start = g_ev_stop = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, dim3(nb), dim3(bs), 0, st, args...);
  }
}

// Launch the one-segment instance of a kernel when the table has a single
// segment, the general one otherwise.
template <typename K1, typename KN, class S>
static void launch_segs(K1 one, KN many, int nb, int bs, hipStream_t st, const Launch<S>& L) {
  if (L.nseg == 1) launch_timed(one, nb, bs, st, L);
  else launch_timed(many, nb, bs, st, L);
}

// Each launcher returns the number of blocks launched (0: nothing to do).
int launch_cell(Launch<CellSeg> L, int mode, int bs, hipStream_t st) {
  const int nb = blocks_for(L, cell_items, bs);
  if (nb == 0) return 0;
  if (mode == 1) launch_segs(k_cell<1, true>, k_cell<1, false>, nb, bs, st, L);
  else if (mode == 2) launch_segs(k_cell<2, true>, k_cell<2, false>, nb, bs, st, L);
  else launch_segs(k_cell<0, true>, k_cell<0, false>, nb, bs, st, L);
  return nb;
}

int launch_vertex(Launch<VertSeg> L, int bs, hipStream_t st) {
  const int nb = blocks_for(L, vert_items, bs);
  if (nb == 0) return 0;
  launch_segs(k_vertex<true>, k_vertex<false>, nb, bs, st, L);
  return nb;
}

// Every segment of a launch has the same physics (linear or not).
int launch_prep(Launch<PrepSeg> L, bool fuse_q, int bs, hipStream_t st) {
  const int nb = blocks_for(L, prep_items, bs);
  if (nb == 0) return 0;
  if (L.seg[0].linear) launch_segs(k_prep<true, false, true>, k_prep<true, false, false>, nb, bs, st, L);
  else if (fuse_q) launch_segs(k_prep<false, true, true>, k_prep<false, true, false>, nb, bs, st, L);
  else launch_segs(k_prep<false, false, true>, k_prep<false, false, false>, nb, bs, st, L);
  return nb;
}

template <bool CELLS, bool GROUP>
static void launch_edge_t(const Launch<EdgeSeg>& L, bool drag, bool wind, int nb, int bs, hipStream_t st) {
  if (drag && wind)
    launch_segs(k_edge<true, true, CELLS, true, GROUP>, k_edge<true, true, CELLS, false, GROUP>, nb, bs, st, L);
  else if (drag)
    launch_segs(k_edge<true, false, CELLS, true, GROUP>, k_edge<true, false, CELLS, false, GROUP>, nb, bs, st, L);
  else if (wind)
    launch_segs(k_edge<false, true, CELLS, true, GROUP>, k_edge<false, true, CELLS, false, GROUP>, nb, bs, st, L);
  else
    launch_segs(k_edge<false, false, CELLS, true, GROUP>, k_edge<false, false, CELLS, false, GROUP>, nb, bs, st, L);
}

// Slot sharing within 16-lane groups: every segment has >= 16 members (an
// edge's members then fill whole, aligned 16-lane groups) and <= 16 slots.
static bool group_slots(const Launch<EdgeSeg>& L) {
  for (int s = 0; s < L.nseg; ++s)
    if (L.seg[s].nm_log2 < 4 || L.seg[s].m.maxEOE > 16) return false;
  return true;
}

// A one-segment momentum pass with folded work: its edge blocks keep the
// XCD layout, the folded work's blocks follow round-robin.
static void tail_layout(Launch<EdgeSeg>& L, int bs) {
  L.xcd_n = 0;
  const EdgeSeg& s = L.seg[0];
  if (L.nseg != 1 || s.tail.kind == 0) return;
  const long ne = s.end > s.begin ? (long)(s.end - s.begin) << s.nm_log2 : 0;
  L.xcd_n = (int)((ne + bs - 1) / bs);
}

int launch_edge(Launch<EdgeSeg> L, bool drag, bool wind, int bs, hipStream_t st, bool cells) {
  const int nb = blocks_for(L, edge_items, bs);
  if (nb == 0) return 0;
  tail_layout(L, bs);
  if (cells) launch_edge_t<true, false>(L, drag, wind, nb, bs, st);
  else if (group_slots(L)) launch_edge_t<false, true>(L, drag, wind, nb, bs, st);
  else launch_edge_t<false, false>(L, drag, wind, nb, bs, st);
  return nb;
}

int launch_edge_fast(Launch<EdgeSeg> L, bool slow, int bs, hipStream_t st) {
  const int nb = blocks_for(L, edge_items, bs);
  if (nb == 0) return 0;
  tail_layout(L, bs);
  if (slow) launch_segs(k_edge_fast<true, true>, k_edge_fast<true, false>, nb, bs, st, L);
  else launch_segs(k_edge_fast<false, true>, k_edge_fast<false, false>, nb, bs, st, L);
  return nb;
}

int launch_predict(Launch<PredSeg> L, hipStream_t st) {
  const int nb = blocks_for(L, pred_items, kBlock);
  if (nb == 0) return 0;
  if (L.nseg == 1) hipLaunchKernelGGL(k_predict<true>, dim3(nb), dim3(kBlock), 0, st, L);
  else hipLaunchKernelGGL(k_predict<false>, dim3(nb), dim3(kBlock), 0, st, L);
  return nb;
}

int launch_assemble(Launch<AsmSeg> L, hipStream_t st) {
  const int nb = blocks_for(L, asm_items, kBlock);
  if (nb == 0) return 0;
  if (L.nseg == 1) hipLaunchKernelGGL(k_assemble<true>, dim3(nb), dim3(kBlock), 0, st, L);
  else hipLaunchKernelGGL(k_assemble<false>, dim3(nb), dim3(kBlock), 0, st, L);
  return nb;
}

// Descriptors of the passes a persistent launch can run (laid out for
// kBlock-thread blocks); false for a pass kind it cannot run.
bool desc_cell(PassDesc& d, Launch<CellSeg> L, int mode) {
  d.kind = PK_CELL;
  d.variant = mode;
  d.nvb = blocks_for(L, cell_items, kBlock);
  d.u.cell = L;
  return true;
}

bool desc_vert(PassDesc& d, Launch<VertSeg> L) {
  d.kind = PK_VERT;
  d.variant = 0;
  d.nvb = blocks_for(L, vert_items, kBlock);
  d.u.vert = L;
  return true;
}

bool desc_prep(PassDesc& d, Launch<PrepSeg> L, bool fuse_q) {
  d.kind = PK_PREP;
  d.variant = L.seg[0].linear ? 0 : (fuse_q ? 2 : 1);
  d.nvb = blocks_for(L, prep_items, kBlock);
  d.u.prep = L;
  return true;
}

bool desc_edge(PassDesc& d, Launch<EdgeSeg> L, bool drag, bool wind, bool fast, bool cells) {
  if (cells) return false;
  d.nvb = blocks_for(L, edge_items, kBlock);
  if (fast) {
    d.kind = PK_EDGE_FAST;
    d.variant = L.seg[0].slow != nullptr ? 1 : 0;
  } else {
    d.kind = PK_EDGE;
    d.variant = (drag ? 1 : 0) | (wind ? 2 : 0) | (group_slots(L) ? 4 : 0);
  }
  d.u.edge = L;
  return true;
}

bool desc_pred(PassDesc& d, Launch<PredSeg> L) {
  d.kind = PK_PRED;
  d.variant = 0;
  d.nvb = blocks_for(L, pred_items, kBlock);
  d.u.pred = L;
  return true;
}

bool desc_asm(PassDesc& d, Launch<AsmSeg> L) {
  d.kind = PK_ASM;
  d.variant = 0;
  d.nvb = blocks_for(L, asm_items, kBlock);
  d.u.asmb = L;
  return true;
}

// Blocks of one cooperative launch of k_persistent: per_cu blocks per
// compute unit, at most as many as stay resident (a multiple of 8, the XCD
// count).
int persistent_grid(int per_cu, hipError_t* err) {
  int dev = 0, cus = 0, occ = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_persistent, kBlock, 0);
  *err = e;
  if (e != hipSuccess) return 0;
  return ((per_cu < occ ? per_cu : occ) * cus) / 8 * 8;
}

hipError_t launch_persistent(const PassDesc* dev_desc, int n, int grid, GridBar B, hipStream_t st) {
  void* args[] = {(void*)&dev_desc, (void*)&n, (void*)&B};
  return hipLaunchCooperativeKernel((const void*)k_persistent, dim3(grid), dim3(kBlock), args, 0, st);
}

void launch_axpy_final(double* y, const double* acc, double c, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpy_final, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, y, acc, c, n);
}

void launch_permute(double* dst, const double* src, const int* perm, int n, int nm_log2, int member, int to_lib,
                    hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_permute, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, dst, src, perm, n, nm_log2,
                     member, to_lib);
}

void launch_copy(double* dst, const double* src, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, dst, src, n);
}

void launch_fill(double* dst, double v, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, dst, v, n);
}

int diag_blocks(const MeshDev& m) {
  int nmax = m.N > m.E ? (m.N > m.V ? m.N : m.V) : (m.E > m.V ? m.E : m.V);
  int nb = (nmax + 4095) / 4096;
  return nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
}

void launch_diag(const MeshDev& m, int nm_log2, int linear, const double* h, const double* u, double g,
                 double* partial, double* out, hipStream_t st) {
  DiagArgs A;
  A.m = m;
  A.nm_log2 = nm_log2;
  A.linear = linear;
  A.h = h;
  A.u = u;
  A.g = g;
  A.partial = partial;
  A.nblocks = diag_blocks(m);
  hipLaunchKernelGGL(k_diag, dim3(A.nblocks), dim3(kBlock), 0, st, A);
  hipLaunchKernelGGL(k_diag_final, dim3(1 << nm_log2), dim3(kBlock), 0, st, (const double*)partial, A.nblocks,
                     1 << nm_log2, out);
}

}  // namespace fblts
