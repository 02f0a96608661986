// Internal types shared by the host planner and the gfx950 kernels.
//
// Device layout (all in the library's region-contiguous numbering):
//   * per-entity scalars: one value per cell / edge / vertex;
//   * fixed-degree incidence lists in slot-major ("ELL") order, list[j*stride + i],
//     so the lanes of a wavefront read consecutive addresses for slot j;
//   * state and scratch arrays carry nm members innermost: x[i*nm + member].
#pragma once
#include <cstdint>

namespace fblts {

constexpr int kMaxSeg = 4;       // meshes (segments) one launch can cover
constexpr int kBlock = 256;      // threads per block for the stencil passes
// Gather loops issue the first slots' loads together (no loop-carried
// address dependence): cells unroll 7 edge slots (heptagons included), edges
// 12 edges_on_edge slots (an edge between two heptagons); longer lists, rare
// on Voronoi meshes, finish in a loop.
constexpr int kUnrollCell = 7;
constexpr int kUnrollEOE = 12;
// Of those, the momentum pass fetches the weights of slots from kEOEFull on
// only where the edge's list reaches them: a padded slot's load re-reads the
// edge's slot-0 weight (a line already being fetched) and +0 replaces the
// value.  On a mostly hexagonal mesh nearly every list fills 10 slots and few
// fill 11, so most lines of those slots' weights are never fetched.
constexpr int kEOEFull = 10;

// Permuted mesh, device pointers.  Edge codes carry a sign bit:
// code = 2*e + (sign < 0 ? 1 : 0).
struct MeshDev {
  int N, E, V;
  int cs, es, vs;          // slot strides (cell, edge, vertex lists)
  int maxE, maxEOE;
  // cells
  const int* c_nedge;      // [N]
  const int* c_edge;       // [maxE][cs]  edge code, sign = n_{e,i}
  const int* c_nbr;        // [maxE][cs]  cell across that edge
  const double* c_invA;    // [N]
  const double* c_A;       // [N]
  const double* c_H;       // [N]
  // edges
  const int* e_cell;       // [2][es]  c0, c1 (n_e points c0 -> c1)
  const int* e_vert;       // [2][es]  v0, v1 (t_e points v0 -> v1)
  const double* e_dc;      // [E] d_e
  const double* e_dv;      // [E] l_e
  const double* e_invdc;   // [E]
  const double* e_He;      // [E] resting depth at the edge (linear flux)
  const int* e_neoe;       // [E]
  const int* e_eoe;        // [maxEOE][es]
  const double* e_w;       // [maxEOE][es]
  // vertices
  const int* v_edge;       // [3][vs]  edge code, sign = circulation sign s_{e,v}
  const int* v_cell;       // [3][vs]
  const double* v_kite;    // [3][vs]
  const double* v_invA;    // [V]
  const double* v_A;       // [V]
  const double* v_f;       // [V]
  const double* v_q0;      // [V] f_v / H_v (linear PV about rest)
  // transposes used by the adjoint kernels
  const double* e_wT;      // [maxEOE][es]  w_{e2,e} for e2 = e_eoe[j][e] (0 on padding)
  const int* c_vert;       // [maxE][cs]    vertices of the cell (ccw; padding repeats slot 0)
  const double* c_kite;    // [maxE][cs]    kite area of the cell at that vertex (0 on padding)
  // momentum pass through the cells' edge lists
  const double* c_R;       // [maxE][cs]    kite fraction R_{i,v} = kite / A_i (0 on padding)
  const int* e_cs;         // [E] slot0 | deg0 << 4 | slot1 << 8 | deg1 << 12
  // the lists of each edge's two vertices, copied per edge (fused q_v)
  const int* e_vq_edge;    // [6][es]  v0's three edge codes, then v1's
  const int* e_vq_cell;    // [6][es]  v0's three cells, then v1's
};

// Coarse stages of the pipelined FB-LTS step (fine substep 0 overlapping the
// coarse advancement) hand their stage values to the fine substeps' own
// arrays as they are formed: on [b, p) (interface one) the k = 0 prediction
// a * y + c * y0, on [p, e) the value itself, where y is the updated value
// and y0 the FB base value of the item; with sv, y0 is also saved on [b, p)
// (compact, members innermost).  dst == nullptr: nothing.
struct Mirror {
  double* dst;
  double* sv;
  int b, p, e;
  double a, c;
};

// Thickness pass: Psi, FB stage update, FB-averaged thickness and Bernoulli
// function over cells [begin,end).  Psi is evaluated on [upd_begin,upd_end)
// (written as H0 + c_dt*Psi to Hdst) and on [acc_begin,acc_end) (added to acc
// with weight acc_w; acc_first overwrites instead of adding).  Everywhere in
// [begin,end): Hnew = updated value or Hnew_src[i]; hs = wn*Hnew + ws*Hsrc +
// wb*H0; B = K(Usrc) + g (hs - H).
struct CellSeg {
  MeshDev m;
  int nm_log2;
  int begin, end, upd_begin, upd_end, acc_begin, acc_end, acc_first;
  const double* Hsrc;
  const double* Usrc;
  const double* H0;
  const double* Hnew_src;
  double* Hdst;
  double* hs;
  double* B;
  double* acc;
  double c_dt, wn, ws, wb, acc_w, g;
  Mirror mir;
};

// Vertex pass: q_v = (zeta_v(Usrc) + f_v) / h_v(hs) over vertices [begin,end).
struct VertSeg {
  MeshDev m;
  int nm_log2;
  int begin, end;
  const double* Usrc;
  const double* hs;
  double* q;
};

// Edge-prep pass: P_e = (l_e h_e u_e, q_e, l_e u_e, h_e) over edges [begin,end).
struct PrepSeg {
  MeshDev m;
  int nm_log2;
  int begin, end;
  int linear;
  const double* Usrc;
  const double* hs;
  const double* q;         // per member (nonlinear) or the static q0 (linear)
  double* P;               // 4 doubles per edge and member, split by use (prep_record.h)
};

// Work folded into the last momentum pass of a fine substep (pipelined
// FB-LTS step), in place of a separate launch after it:
//  kind 1, the interface-one prediction for the next substep (eq. preds):
//    edges [e_b, e_p) by the edge's own thread after its own work, cells
//    [c_b, c_p) by extra items after the edges;
//  kind 2, the correction and assembly of t^{n+1}: edges [e_b, e_q)
//    (interface one and two, whose accumulated tendency the thread has just
//    formed) by their own thread, cells [c_b, c_e) and interior edges
//    [e_q, e_e) by extra items.
// H* / U* are the fine substeps' arrays (H0, U0 the state), C* / D* the coarse
// stage values, sv_* the saved h^n, u^n on interface one.
struct StepTail {
  int kind;
  int c_b, c_p, c_q, c_e;
  int e_b, e_p, e_q, e_e;
  double* H0; double* H1; double* H2; double* H3;
  const double* C1; const double* C2; const double* C3;
  double* U0; double* U1; double* U2;
  const double* D1; const double* D2; const double* D3;
  const double* sv_h; const double* sv_u; const double* acc_h;
  double a, one_minus_a, invM, c, ap, delta;
};

// Momentum pass: Phi_e from P, B, drag and wind over edges; update
// [upd_begin,upd_end) as U0 + c_dt*Phi into Udst, accumulate on
// [acc_begin,acc_end).
struct EdgeSeg {
  MeshDev m;
  int nm_log2;
  int begin, end, upd_begin, upd_end, acc_begin, acc_end, acc_first;
  const double* P;
  const double* B;
  const double* Usrc;
  const double* U0;
  double* Udst;
  double* acc;
  const double* cd;        // per cell and member, or nullptr
  const double* wind_n;    // per edge and member, or nullptr
  const double* wind_t;
  const double* wind_c;    // wind-stress coefficient C_W per edge and member
  const double* slow;      // fast pass: frozen slow tendency per edge and member, or nullptr
  double c_dt, acc_w;
  Mirror mir;
  StepTail tail;
};

// Interface-one prediction (eq. preds) over cells [c_begin,c_end) and edges
// [e_begin,e_end); on k == 0 the coarse data is first saved to the compact
// arrays sv_h[4][nc*nm], sv_u[4][ne*nm].
struct PredSeg {
  int nm_log2;
  int c_begin, c_end, e_begin, e_end;
  double* H0; double* H1; double* H2; double* H3;
  double* U0; double* U1; double* U2; const double* U3;
  double* sv_h; double* sv_u;
  int save;
  double a, one_minus_a, invM, c, ap;
};

// Interface correction and assembly of t^{n+1}: IF-1 from the saved h^n,
// IF-2 from H0 (= h^n there), interior from the coarse stage 3.
struct AsmSeg {
  int nm_log2;
  int if1_c_begin, if1_c_end, if2_c_end, N;
  int if1_e_begin, if1_e_end, if2_e_end, E;
  double* H0; const double* H3; const double* acc_h; const double* sv_h;
  double* U0; const double* U3; const double* acc_u; const double* sv_u;
  double delta;
};

// Cyclone wind at edges for the wind-stress term: per member a Holland
// vortex on a great-circle track, evaluated at t = t0 + clock[0] * dt, or calm
// air (zero wind) for a member without a storm.
struct CycloneParams {
  double c0[3], axis[3];
  double v_trans, dp, rm, b, rho_air, radius, omega, t0, omega_track;
  int enabled;              // 0: calm air
  int pad;
};
struct CycloneArgs {
  const double* x;          // [3][E] unit edge positions (may be null when no member has a storm)
  const double* n;          // [3][E] unit edge normals
  double* wn;               // [E*nm] W . n_e, members innermost
  double* wt;               // [E*nm] W . (x cross n_e)
  double* wc;               // [E*nm] wind-stress coefficient C_W(|W|)
  const long long* clock;   // coarse steps since the storms were set
  const CycloneParams* p;   // [nm]
  int E, nm_log2;
  double dt;
  double rho_ratio;         // rho_air / rho_water of the C_W law
};

template <class S>
struct Launch {
  int nseg;
  int block;                 // threads per block of the launch
  int blk_start[kMaxSeg + 1];
  // > 0: only the first xcd_n blocks are laid out XCD by XCD; the blocks
  // after them (work folded into a momentum pass) go round-robin over the
  // XCDs, so that every XCD gets its share of both kinds of block
  int xcd_n;
  S seg[kMaxSeg];
};

// One pass of a persistent launch: a run of consecutive stencil and
// elementwise passes executed by one cooperative kernel, with a grid-wide
// barrier between passes.  The pass's launch table is laid out for blocks of
// kBlock threads; nvb is its number of such (virtual) blocks.
enum PassKind { PK_CELL = 0, PK_VERT, PK_PREP, PK_EDGE, PK_EDGE_FAST, PK_PRED, PK_ASM };
struct PassDesc {
  int kind;       // PassKind
  int variant;    // CELL: MODE; PREP: 0 linear, 1 nonlinear, 2 nonlinear with q_v fused;
                  // EDGE: drag | wind << 1 | group << 2; EDGE_FAST: slow
  int nvb;
  int pad;
  union U {
    Launch<CellSeg> cell;
    Launch<VertSeg> vert;
    Launch<PrepSeg> prep;
    Launch<EdgeSeg> edge;
    Launch<PredSeg> pred;
    Launch<AsmSeg> asmb;
  } u;
};

// Grid barrier state of a persistent launch (device memory, zero before the
// first launch and zero again after every completed launch): ctr[0] counts
// the group leaders, ctr[32 * (g + 1)] the blocks of group g (g < 8), ctr[400]
// is the generation; abort is set when a wait gave up (the launch is then
// abandoned and its results are invalid).
struct GridBar {
  unsigned* ctr;
  int* abort;
};
constexpr int kBarWords = 512;

}  // namespace fblts
