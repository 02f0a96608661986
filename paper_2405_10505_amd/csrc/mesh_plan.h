// Host-side mesh copy, validation, region layering and the per-solver plan
// (permutation, pass ranges, byte model).  No device code here.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fblts.h"

namespace fblts {

struct HostMesh {
  int N = 0, E = 0, V = 0;
  std::vector<int> coe, voe;                 // [2E]
  std::vector<int> eoc_off, eoc, voc_off, voc;
  std::vector<int> eoe_off, eoe;
  std::vector<double> woe;
  std::vector<int> eov, cov;                 // [3V]
  std::vector<double> kite;                  // [3V]
  std::vector<double> dc, dv, A, Av, fv, fe, H;
};

// Throws std::runtime_error with a message naming the violated property.
void validate_and_copy(const fblts_mesh_desc* d, HostMesh& m);

// 4-level labels from binary or 4-level input; throws on invalid input.
// layer[i]: fine cells -(hops to coarse set), coarse cells +(hops to fine set);
// +big / -big when the other set is empty.
void layer_regions(const HostMesh& m, const int8_t* labels, bool binary, int r, std::vector<int8_t>& lab4,
                   std::vector<int>& layer);

struct Range {
  int b = 0, e = 0;
  int size() const { return e > b ? e - b : 0; }
};

// One stage's four passes.
struct StageRanges {
  Range cell, cell_upd, cell_acc;
  Range vert, prep;
  Range edge, edge_upd, edge_acc;
};

struct Plan {
  // permutations: new -> old (caller) index
  std::vector<int> cell_new2old, edge_new2old, vert_new2old;
  std::vector<int> cell_old2new, edge_old2new, vert_old2new;
  std::vector<int8_t> cell_lab, edge_lab;    // in new numbering
  int nF = 0, nIF1 = 0, nIF2 = 0, nINT = 0;  // cells per region (contiguous in this order)
  int nFE = 0, nIF1E = 0, nIF2E = 0, nINTE = 0;
  StageRanges coarse[3];   // coarse advancement (suffix ranges)
  StageRanges fine[3];     // fine substep (prefix ranges)
  int fine_depth_max = 0;  // deepest fine layer touched by the coarse sweep (hops)
  // one past the largest cell / edge whose stage-input value (h, u) the third
  // fine stage reads: interface two and the interior cells within its
  // stencils hold the coarse stage values there (Sec. 2.2, step 4)
  int fine3_cell_end = 0, fine3_edge_end = 0;
};

// Build the plan for FB-LTS (4-level labels) or for a global scheme (all
// coarse).  nonlinear selects the vertex passes.  Throws std::runtime_error
// (message starting with "region:") when the stencil condition fails.
void build_plan(const HostMesh& m, const std::vector<int8_t>& lab4, const std::vector<int>& layer, bool fblts,
                bool nonlinear, int r, Plan& p, bool full_coarse = false);

// Reordered mesh in the device layout (host staging before upload).
struct PermMesh {
  int N, E, V, cs, es, vs, maxE, maxEOE;
  std::vector<int> c_nedge, c_edge, c_nbr;
  std::vector<double> c_invA, c_A, c_H;
  std::vector<int> e_cell, e_vert, e_neoe, e_eoe;
  std::vector<double> e_dc, e_dv, e_invdc, e_He, e_w;
  std::vector<int> v_edge, v_cell;
  std::vector<double> v_kite, v_invA, v_A, v_f, v_q0;
  std::vector<double> e_wT, c_kite;
  std::vector<int> c_vert;
  // momentum pass through the cells' edge lists: kite fraction R_{i,v} per
  // cell slot, and per edge the slot of the edge in each of its two cells and
  // those cells' degrees (4 bits each: slot0 | deg0<<4 | slot1<<8 | deg1<<12)
  std::vector<double> c_R;
  std::vector<int> e_cs;
  // 2: the mesh's edges_on_edge lists and weights are exactly the cell walks
  // with w = n_{e,i} n_{e',i} (1/2 - sum R) (bitwise); 1: within 1e-13; 0: not
  int kite_weights = 0;
};
void permute_mesh(const HostMesh& m, const Plan& p, PermMesh& pm);

// Per-pass byte model of each pass kind over a range: every mesh array
// element, state element and intermediate (h*, B, q_v, the edge-prep records)
// the pass reads or writes, each once per launch.  nm = members; state and
// intermediate bytes scale with nm, mesh bytes do not.
double bytes_cell_pass(const PermMesh& pm, const StageRanges& r, bool nonlinear, int nm, bool ke = true);
double bytes_vert_pass(const PermMesh& pm, const Range& r, int nm);
double bytes_prep_pass(const PermMesh& pm, const Range& r, bool nonlinear, int nm, bool fuse_q = false);
double bytes_edge_pass(const PermMesh& pm, const StageRanges& r, bool drag, bool wind, int nm);
// momentum pass walking the two cells' edge lists (weights from kite fractions)
double bytes_edge_cells_pass(const PermMesh& pm, const StageRanges& r, bool drag, bool wind, int nm);
// fast momentum pass of the operator splitting (pressure gradient + frozen slow tendency)
double bytes_edge_fast_pass(const PermMesh& pm, const StageRanges& r, bool slow, int nm);

// Compulsory (algorithmic) bytes of each pass kind: the mesh arrays and the
// state arrays (h, u, their stage and time-level copies, accumulators, drag
// and wind) that the pass's mathematics references, each element once per
// launch; intermediates that a pass could keep on chip -- the thickness flux,
// q, K, B, h* and the edge-prep records -- cost nothing in either direction.
// The momentum pass through the cells' edge lists computes the same
// mathematics and has the same compulsory bytes as compulsory_edge_pass.
double compulsory_cell_pass(const PermMesh& pm, const StageRanges& r, bool nonlinear, int nm, bool ke = true);
double compulsory_vert_pass(const PermMesh& pm, const Range& r, int nm);
double compulsory_prep_pass(const PermMesh& pm, const Range& r, bool nonlinear, int nm);
double compulsory_edge_pass(const PermMesh& pm, const StageRanges& r, bool drag, bool wind, int nm);
double compulsory_edge_fast_pass(const PermMesh& pm, const StageRanges& r, bool slow, int nm);

}  // namespace fblts
