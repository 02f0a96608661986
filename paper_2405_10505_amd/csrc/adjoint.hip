// Reverse-mode (adjoint) kernels of the TRiSK tendencies, gfx950.
//
// For a tendency evaluated at a point (u, h) and a cotangent on its output,
// these kernels accumulate the cotangents of the inputs (vector-Jacobian
// products).  Every transpose is written as a gather, so each output has one
// writer: no atomics, and the result is bitwise reproducible.
//   * cellsOnEdge <-> edgesOnCell, verticesOnEdge <-> edgesOnVertex and
//     cellsOnVertex <-> verticesOnCell are each other's transposes;
//   * edgesOnEdge is a symmetric relation, and the transposed weight w_{e',e}
//     is stored beside w_{e,e'} (exact, no reliance on antisymmetry rounding).
// Thickness tendency (eq. trisk_thickness): Psi_i = -(1/A_i) sum n_{e,i} l_e F_e,
// F_e = h_e u_e.  Momentum tendency (eq. trisk_vorticity with eq.
// nonlinear_swe and the quadratic drag of eq. hurricane_model):
// Phi_e = (1/d_e) sum w_{e,e'} (lF)_e' (q_e+q_e')/2 - (B_c1-B_c0)/d_e - C_D |u| u / h_e.
// The edge records at the point (lF, q_e, l u, h_e) are computed as the
// forward's prep pass computes them (q_v evaluated inside), in the first
// launch of the Phi transpose; the vertex transpose forms q_v itself.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fblts_internal.h"
#include "lincomb.h"
#include "prep_record.h"

namespace fblts {

namespace {
__device__ __forceinline__ int tid_global() { return blockIdx.x * blockDim.x + threadIdx.x; }
}  // namespace

// y[i] = b*y[i] + a0*x0[i] + a1*x1[i] + a2*x2[i] over [begin,end) (null inputs skipped).
__global__ void __launch_bounds__(kBlock) k_lincomb(double* y, double b, const double* x0, double a0,
                                                    const double* x1, double a1, const double* x2, double a2,
                                                    int begin, int end) {
  const int i = begin + tid_global();
  if (i >= end) return;
  // plain multiply-add in a fixed order (matches the forward passes' FB averages)
  double v = b == 0.0 ? 0.0 : b * y[i];
  if (x0) v = v + a0 * x0[i];
  if (x1) v = v + a1 * x1[i];
  if (x2) v = v + a2 * x2[i];
  y[i] = v;
}

// A run of elementwise combinations: index i of every descriptor whose range
// holds i, in order.  Each combination reads and writes only index i of its
// arrays, so applying the run index by index equals launching the
// combinations one after another.
__device__ __forceinline__ void lin_apply(const LinBatch& B, int i) {
  for (int k = 0; k < B.n; ++k) {
    const LinDesc& D = B.d[k];
    if (i < D.begin || i >= D.end) continue;
    double v = D.b == 0.0 ? 0.0 : D.b * D.y[i];
    if (D.x0) v = v + D.a0 * D.x0[i];
    if (D.x1) v = v + D.a1 * D.x1[i];
    if (D.x2) v = v + D.a2 * D.x2[i];
    D.y[i] = v;
  }
}

__global__ void __launch_bounds__(kBlock) k_lincomb_batch(const LinBatch B) { lin_apply(B, tid_global()); }

// Cell-slot loops: the first kUnrollCell slots exist for every cell (padded
// lists), so their loads issue together; slots past the cell's degree are
// skipped (the sums are the plain in-order sums).

// ------------------------------------------------------------ Psi transpose
// Fbar_e = l_e (-pb_c0/A_c0 + pb_c1/A_c1); ub_e += Fbar_e h_e; T_e = Fbar_e u_e.
__global__ void __launch_bounds__(kBlock) k_psi_vjp_edge(MeshDev m, int n_e, int linear, const double* u,
                                                         const double* h, const double* pb, double* ub, double* T) {
  const int e = tid_global();
  if (e >= n_e) return;
  const int c0 = m.e_cell[e], c1 = m.e_cell[m.es + e];
  const double fb = m.e_dv[e] * (pb[c1] * m.c_invA[c1] - pb[c0] * m.c_invA[c0]);
  const double he = linear ? m.e_He[e] : 0.5 * (h[c0] + h[c1]);
  ub[e] = fma(fb, he, ub[e]);
  if (!linear) T[e] = fb * u[e];
}

// hb_i += (1/2) sum_{e in E_i} T_e.
__device__ __forceinline__ void psi_vjp_cell(const MeshDev& m, int i, const double* T, double* hb) {
  const int n = m.c_nedge[i];
  const double hb0 = hb[i];
  double t[kUnrollCell];
#pragma unroll
  for (int j = 0; j < kUnrollCell; ++j) t[j] = T[m.c_edge[j * m.cs + i] >> 1];
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kUnrollCell; ++j)
    if (j < n) s += t[j];
  for (int j = kUnrollCell; j < n; ++j) s += T[m.c_edge[j * m.cs + i] >> 1];
  hb[i] = fma(0.5, s, hb0);
}

// The Psi transpose's cell pass on cells [0, n_c), thread i on cell i, then
// the combinations B at index i (an epilogue: the caller folds in only runs
// that leave T alone, so no thread's epilogue touches what another reads).
__global__ void __launch_bounds__(kBlock) k_psi_vjp_cell(MeshDev m, int n_c, const double* T, double* hb,
                                                         const LinBatch B) {
  const int i = tid_global();
  if (i < n_c) psi_vjp_cell(m, i, T, hb);
  lin_apply(B, i);
}

// ------------------------------------------------------------ Phi transpose
// Pass 1 (edges): G_e = fb_e/d_e; drag terms of d/du_e, d/du_perp_e, d/dh_e, d/dC_D.
// h_e and the neighbours' l u are formed from u and h* as the edge records
// form them (the same operations), so this pass does not wait for the records.
__device__ __forceinline__ void phi_vjp_e1(const MeshDev& m, int e, bool linear, int drag, const double* u,
                                           const double* hs, const double* cd, const double* fb, double* G,
                                           double* R, double* HD, double* CDB, double* ub) {
  const double g = fb[e] * m.e_invdc[e];
  G[e] = g;
  if (!drag) return;
  const int n = m.e_neoe[e];
  // the edge's own operands first, then every slot's loads together
  const double ue = u[e];
  const int c0 = m.e_cell[e], c1 = m.e_cell[m.es + e];
  const double he = linear ? m.e_He[e] : 0.5 * (hs[c0] + hs[c1]);
  const double cde = 0.5 * (cd[c0] + cd[c1]);
  const double ub0 = ub[e];
  double w[kUnrollEOE], lu[kUnrollEOE];
#pragma unroll
  for (int j = 0; j < kUnrollEOE; ++j) {
    const int e2 = m.e_eoe[j * m.es + e];
    w[j] = m.e_w[j * m.es + e];
    lu[j] = m.e_dv[e2] * u[e2];
  }
  double su = 0.0;
#pragma unroll
  for (int j = 0; j < kUnrollEOE; ++j)
    if (j < n) su = fma(w[j], lu[j], su);
  for (int j = kUnrollEOE; j < n; ++j) {
    const int e2 = m.e_eoe[j * m.es + e];
    su = fma(m.e_w[j * m.es + e], m.e_dv[e2] * u[e2], su);
  }
  const double up = su * m.e_invdc[e];
  const double sp = sqrt(ue * ue + up * up);
  // D = C_D |u| u / h_e, Phi -= D; |u| u is C^1 with zero derivative at |u| = 0
  const double dDdu = sp > 0.0 ? cde * (sp + ue * ue / sp) / he : 0.0;
  const double dDdup = sp > 0.0 ? cde * ue * up / (sp * he) : 0.0;
  ub[e] = fma(-fb[e], dDdu, ub0);
  R[e] = -fb[e] * dDdup * m.e_invdc[e];
  HD[e] = fb[e] * cde * sp * ue / (he * he);
  CDB[e] = -fb[e] * sp * ue / he;
}

// Pass 2 (cells): Bbar_i = sum n_{e,i} G_e; hsb_i += g Bbar_i (G_e formed
// from fb as pass 1 forms it, so this pass does not wait for pass 1).
__device__ __forceinline__ void phi_vjp_c1(const MeshDev& m, int i, double g, const double* fb, double* BB,
                                           double* hsb) {
  const int n = m.c_nedge[i];
  const double hsb0 = hsb[i];
  int code[kUnrollCell];
  double x[kUnrollCell];
#pragma unroll
  for (int j = 0; j < kUnrollCell; ++j) {
    code[j] = m.c_edge[j * m.cs + i];
    const int e = code[j] >> 1;
    x[j] = fb[e] * m.e_invdc[e];
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kUnrollCell; ++j)
    if (j < n) s = (code[j] & 1) ? s - x[j] : s + x[j];
  for (int j = kUnrollCell; j < n; ++j) {
    const int c = m.c_edge[j * m.cs + i];
    const double y = fb[c >> 1] * m.e_invdc[c >> 1];
    s = (c & 1) ? s - y : s + y;
  }
  BB[i] = s;
  hsb[i] = fma(g, s, hsb0);
}

// The edge records at the point (the forward's prep pass, q_v evaluated
// inside unless LINEAR) and passes 1 and 2, independent of each other, in one
// launch: threads [0, n_p) take the records of edges [0, n_p), the next n_e
// threads pass 1 on edges [0, n_e), the next n_c pass 2 on cells [0, n_c).
template <bool LINEAR>
__global__ void __launch_bounds__(kBlock) k_phi_vjp_a(MeshDev m, int n_p, int n_e, int n_c, int drag, double g,
                                                      const double* u, const double* hs, double* P,
                                                      const double* cd, const double* fb, double* G, double* R,
                                                      double* HD, double* CDB, double* ub, double* BB, double* hsb) {
  const int t = tid_global();
  if (t < n_p)
    prep_record<LINEAR, !LINEAR>(m, t, 0, 1, m.E, u, hs, m.v_q0, P);
  else if (t < n_p + n_e)
    phi_vjp_e1(m, t - n_p, LINEAR, drag, u, hs, cd, fb, G, R, HD, CDB, ub);
  else if (t < n_p + n_e + n_c)
    phi_vjp_c1(m, t - n_p - n_e, g, fb, BB, hsb);
}

// Pass 3 (edges, edges_on_edge gathers): PV-flux transpose, drag perp transpose,
// kinetic-energy transpose; writes qbar_e, and h_e's cotangent HE_e.
__global__ void __launch_bounds__(kBlock) k_phi_vjp_e2(MeshDev m, int n_e, int linear, int drag, const double* u,
                                                       const double* P, const double* G, const double* R,
                                                       const double* HD, const double* BB, double* QB, double* HE,
                                                       double* ub) {
  const int e = tid_global();
  if (e >= n_e) return;
  const double2 pe = rec_fq(P, e);
  const int n = m.e_neoe[e];
  // the edge's own operands first, then every slot's loads together
  const double ue = u[e];
  const double le = m.e_dv[e];
  const double ub0 = ub[e];
  const double Ge = G[e];
  const int c0 = m.e_cell[e], c1 = m.e_cell[m.es + e];
  const double kb = linear ? 0.0 : BB[c0] * m.c_invA[c0] + BB[c1] * m.c_invA[c1];
  const double hde = (!linear && drag) ? HD[e] : 0.0;
  const double heown = linear ? m.e_He[e] : rec_he(P, m.E, e);
  const double dce = m.e_dc[e];
  double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  auto slot = [&](int e2, double wT, double w, const double2& p2, double g2, double r2) {
    s1 = fma(wT * g2, p2.y + pe.y, s1);   // d/d(lF)_e of the neighbours' Q_perp
    s2 = fma(w, p2.x, s2);                 // d Q_perp_e / d q_e (own sum)
    s3 = fma(wT, g2, s3);                  // d Q_perp_e2 / d q_e (neighbours)
    if (drag) s4 = fma(wT, r2, s4);        // neighbours' |u| through u_perp
  };
  int e2[kUnrollEOE];
  double wT[kUnrollEOE], w[kUnrollEOE], g2[kUnrollEOE], r2[kUnrollEOE];
  double2 p2[kUnrollEOE];
#pragma unroll
  for (int j = 0; j < kUnrollEOE; ++j) {
    e2[j] = m.e_eoe[j * m.es + e];
    wT[j] = m.e_wT[j * m.es + e];
    w[j] = m.e_w[j * m.es + e];
  }
#pragma unroll
  for (int j = 0; j < kUnrollEOE; ++j) {
    p2[j] = rec_fq(P, e2[j]);
    g2[j] = G[e2[j]];
    r2[j] = drag ? R[e2[j]] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < kUnrollEOE; ++j)
    if (j < n) slot(e2[j], wT[j], w[j], p2[j], g2[j], r2[j]);
  for (int j = kUnrollEOE; j < n; ++j) {
    const int f = m.e_eoe[j * m.es + e];
    slot(f, m.e_wT[j * m.es + e], m.e_w[j * m.es + e], rec_fq(P, f), G[f], drag ? R[f] : 0.0);
  }
  const double lFb = 0.5 * s1;
  const double Fb = le * lFb;
  double acc = ub0;
  if (!linear) {
    QB[e] = 0.5 * (Ge * s2 + pe.x * s3);
    acc = fma(Fb, heown, acc);                                 // F = h_e u
    HE[e] = Fb * ue + (drag ? hde : 0.0);                      // h_e's cotangent
    acc = fma(0.5 * le * dce * ue, kb, acc);                   // K_i = (1/A_i) sum l d u^2 / 4
    if (drag) acc = fma(le, s4, acc);
  } else {
    acc = fma(Fb, heown, acc);                                 // F = H_e u
  }
  ub[e] = acc;
}

// Pass 4 (vertices): qbar_v = (1/2) sum_{e in E_v} QB_e; zeta and h_v cotangents
// (scaled by 1/A_v): ZA_v = qbar_v / (h_v A_v), HV_v = -qbar_v q_v / (h_v A_v).
// q_v = (zeta_v + f_v) / h_v is formed here from u and hs with the operations,
// in the order, of the forward's vertex PV.
__global__ void __launch_bounds__(kBlock) k_phi_vjp_v1(MeshDev m, int n_v, const double* u, const double* hs,
                                                       const double* QB, double* ZA, double* HV) {
  const int v = tid_global();
  if (v >= n_v) return;
  int code[3], cell[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    code[j] = m.v_edge[j * m.vs + v];
    cell[j] = m.v_cell[j * m.vs + v];
  }
  double qb = 0.0, circ = 0.0, hv = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int e = code[j] >> 1;
    qb += QB[e];
    const double c = m.e_dc[e] * u[e];
    circ = (code[j] & 1) ? circ - c : circ + c;
    hv = fma(m.v_kite[j * m.vs + v], hs[cell[j]], hv);
  }
  qb *= 0.5;
  const double ia = m.v_invA[v];
  const double hvv = hv * ia;   // h_v
  const double q = (circ * ia + m.v_f[v]) / hvv;
  ZA[v] = qb / hvv * ia;
  HV[v] = -qb * q / hvv * ia;
}

// Passes 5 and 6, independent of each other, in one launch: threads [0, n_c)
// take the cells [0, n_c), threads [n_c, n_c + n_e) the edges [0, n_e); then
// every thread i applies the combinations B at index i (an epilogue: the
// caller folds in only runs that leave ZA, HE, HV, CDB and ub alone, so no
// thread's epilogue touches what another thread reads or writes).
// Edges: ub_e += d_e (ZA_{v1} - ZA_{v0})  (circulation sign +1 at v1).
// Cells: hsb_i += (1/2) sum_{e in E_i} HE_e + sum_{v in V_i} kite_{i,v} HV_v;
// cdb_i += (1/2) sum_{e in E_i} CDB_e.
__device__ __forceinline__ void phi_vjp_e3(const MeshDev& m, int e, const double* ZA, double* ub) {
  const int v0 = m.e_vert[e], v1 = m.e_vert[m.es + e];
  ub[e] = fma(m.e_dc[e], ZA[v1] - ZA[v0], ub[e]);
}

__device__ __forceinline__ void phi_vjp_c2(const MeshDev& m, int i, int drag, const double* HE, const double* HV,
                                           const double* CDB, double* hsb, double* cdb) {
  const int n = m.c_nedge[i];
  const double hsb0 = hsb[i];
  const double cdb0 = drag ? cdb[i] : 0.0;
  double he[kUnrollCell], kv[kUnrollCell], hv[kUnrollCell], cb[kUnrollCell];
#pragma unroll
  for (int j = 0; j < kUnrollCell; ++j) {
    const int e = m.c_edge[j * m.cs + i] >> 1;
    he[j] = HE[e];
    kv[j] = m.c_kite[j * m.cs + i];
    hv[j] = HV[m.c_vert[j * m.cs + i]];
    cb[j] = drag ? CDB[e] : 0.0;
  }
  double se = 0.0, sv = 0.0, sc = 0.0;
#pragma unroll
  for (int j = 0; j < kUnrollCell; ++j)
    if (j < n) {
      se += he[j];
      sv = fma(kv[j], hv[j], sv);
      if (drag) sc += cb[j];
    }
  for (int j = kUnrollCell; j < n; ++j) {
    const int e = m.c_edge[j * m.cs + i] >> 1;
    se += HE[e];
    sv = fma(m.c_kite[j * m.cs + i], HV[m.c_vert[j * m.cs + i]], sv);
    if (drag) sc += CDB[e];
  }
  hsb[i] = hsb0 + 0.5 * se + sv;
  if (drag) cdb[i] = fma(0.5, sc, cdb0);
}

__global__ void __launch_bounds__(kBlock) k_phi_vjp_ec(MeshDev m, int n_e, int n_c, int drag, const double* ZA,
                                                       const double* HE, const double* HV, const double* CDB,
                                                       double* ub, double* hsb, double* cdb, const LinBatch B) {
  const int t = tid_global();
  if (t < n_c)
    phi_vjp_c2(m, t, drag, HE, HV, CDB, hsb, cdb);
  else if (t < n_c + n_e)
    phi_vjp_e3(m, t - n_c, ZA, ub);
  lin_apply(B, t);
}

// ----------------------------------------------------------------- launchers
static dim3 grid_for(long n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

void launch_lincomb(double* y, double b, const double* x0, double a0, const double* x1, double a1, const double* x2,
                    double a2, int begin, int end, hipStream_t st) {
  if (end <= begin) return;
  hipLaunchKernelGGL(k_lincomb, grid_for(end - begin), dim3(kBlock), 0, st, y, b, x0, a0, x1, a1, x2, a2, begin, end);
}

void launch_lincomb_batch(const LinBatch& B, hipStream_t st) {
  if (B.n == 0 || B.end_max <= 0) return;
  hipLaunchKernelGGL(k_lincomb_batch, grid_for(B.end_max), dim3(kBlock), 0, st, B);
}

// The Psi transpose up to its cell pass, which launch_psi_vjp_cells runs.
void launch_psi_vjp(const MeshDev& m, int linear, const double* u, const double* h, const double* pb, double* ub,
                    double* T, const PsiRange& r, hipStream_t st) {
  if (r.ne > 0)
    hipLaunchKernelGGL(k_psi_vjp_edge, grid_for(r.ne), dim3(kBlock), 0, st, m, r.ne, linear, u, h, pb, ub, T);
}

// The cell pass (nonlinear only) with the combinations B as its epilogue.
void launch_psi_vjp_cells(const MeshDev& m, int n_c, const double* T, double* hb, const LinBatch& B,
                          hipStream_t st) {
  const long n = std::max<long>(n_c, B.n > 0 ? B.end_max : 0);
  if (n > 0) hipLaunchKernelGGL(k_psi_vjp_cell, grid_for(n), dim3(kBlock), 0, st, m, n_c, T, hb, B);
}

// Passes 0-4 of the Phi transpose (passes 5 and 6: launch_phi_vjp_ec).
// Scratch: P (edge records), G, R, HD, CDB, HE, QB (edges), BB (cells), ZA, HV (vertices).
void launch_phi_vjp(const MeshDev& m, int linear, int drag, double g, const double* u, const double* hs,
                    double* P, const double* cd, const double* fb, double* ub, double* hsb, double* G, double* R,
                    double* HD, double* CDB, double* HE, double* QB, double* BB, double* ZA, double* HV,
                    const VjpRange& r, hipStream_t st) {
  const long na = (long)r.pe + r.e1 + r.c1;
  if (na > 0) {
    if (linear)
      hipLaunchKernelGGL(k_phi_vjp_a<true>, grid_for(na), dim3(kBlock), 0, st, m, r.pe, r.e1, r.c1, drag, g, u, hs,
                         P, cd, fb, G, R, HD, CDB, ub, BB, hsb);
    else
      hipLaunchKernelGGL(k_phi_vjp_a<false>, grid_for(na), dim3(kBlock), 0, st, m, r.pe, r.e1, r.c1, drag, g, u, hs,
                         P, cd, fb, G, R, HD, CDB, ub, BB, hsb);
  }
  if (r.e2 > 0)
    hipLaunchKernelGGL(k_phi_vjp_e2, grid_for(r.e2), dim3(kBlock), 0, st, m, r.e2, linear, drag, u,
                       (const double*)P, (const double*)G, (const double*)R, (const double*)HD, (const double*)BB, QB,
                       HE, ub);
  if (!linear && r.v1 > 0)
    hipLaunchKernelGGL(k_phi_vjp_v1, grid_for(r.v1), dim3(kBlock), 0, st, m, r.v1, u, hs, (const double*)QB, ZA, HV);
}

// Passes 5 and 6 (nonlinear only) with the combinations B as their epilogue.
void launch_phi_vjp_ec(const MeshDev& m, int n_e, int n_c, int drag, const double* ZA, const double* HE,
                       const double* HV, const double* CDB, double* ub, double* hsb, double* cdb, const LinBatch& B,
                       hipStream_t st) {
  const long n = std::max<long>((long)n_e + n_c, B.n > 0 ? B.end_max : 0);
  if (n > 0)
    hipLaunchKernelGGL(k_phi_vjp_ec, grid_for(n), dim3(kBlock), 0, st, m, n_e, n_c, drag, ZA, HE, HV, CDB, ub, hsb,
                       cdb, B);
}

}  // namespace fblts
