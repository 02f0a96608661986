// Solver, ensemble and the C ABI of include/fblts.h.
//
// Step orchestration (one coarse step of FB-LTS, paper Section 2.2):
//   coarse advancement: 3 FB-RK(3,2) stages with dt over suffix ranges of the
//     region-ordered mesh (the coarse region plus the fine layers its
//     stencils reach), writing H1..H3 / U1..U3;
//   for k = 0..M-1: interface-one prediction (eq. preds), then 3 stages with
//     dt/M over prefix ranges (fine region plus the halo its stencils read);
//     stage 3 updates the fine region in place and accumulates Psi / Phi on
//     interface one and two (eq. if_correction);
//   assembly: interface correction and interior copy.
// Global FB-RK(3,2) runs the three stages over whole ranges; RK4 runs four
// stages with accumulation.  All launches go to one stream; a coarse step can
// be captured once in a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <tuple>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fblts.h"
#include "fblts_internal.h"
#include "lincomb.h"
#include "mesh_plan.h"

namespace fblts {
int launch_cell(Launch<CellSeg> L, int mode, int bs, hipStream_t st);
int launch_vertex(Launch<VertSeg> L, int bs, hipStream_t st);
int launch_prep(Launch<PrepSeg> L, bool fuse_q, int bs, hipStream_t st);
int launch_edge(Launch<EdgeSeg> L, bool drag, bool wind, int bs, hipStream_t st, bool cells);
int launch_edge_fast(Launch<EdgeSeg> L, bool slow, int bs, hipStream_t st);
int launch_predict(Launch<PredSeg> L, hipStream_t st);
int launch_assemble(Launch<AsmSeg> L, hipStream_t st);
void launch_axpy_final(double* y, const double* acc, double c, long n, hipStream_t st);
void launch_permute(double* dst, const double* src, const int* perm, int n, int nm_log2, int member, int to_lib,
                    hipStream_t st);
void launch_copy(double* dst, const double* src, long n, hipStream_t st);
void launch_fill(double* dst, double v, long n, hipStream_t st);
void launch_cyclone(const CycloneArgs& a, hipStream_t st);
void arm_launch_events(hipEvent_t start, hipEvent_t stop);
void launch_clock_tick(long long* clock, hipStream_t st);
int diag_blocks(const MeshDev& m);
void launch_diag(const MeshDev& m, int nm_log2, int linear, const double* h, const double* u, double g,
                 double* partial, double* out, hipStream_t st);
constexpr int kDiagQ = 8;
bool desc_cell(PassDesc& d, Launch<CellSeg> L, int mode);
bool desc_vert(PassDesc& d, Launch<VertSeg> L);
bool desc_prep(PassDesc& d, Launch<PrepSeg> L, bool fuse_q);
bool desc_edge(PassDesc& d, Launch<EdgeSeg> L, bool drag, bool wind, bool fast, bool cells);
bool desc_pred(PassDesc& d, Launch<PredSeg> L);
bool desc_asm(PassDesc& d, Launch<AsmSeg> L);
int persistent_grid(int per_cu, hipError_t* err);
hipError_t launch_persistent(const PassDesc* dev_desc, int n, int grid, GridBar B, hipStream_t st);
}  // namespace fblts

using namespace fblts;

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

namespace {

struct Err : std::runtime_error {
  int code;
  Err(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Err(FBLTS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
int guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const Err& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "out of host memory";
    return FBLTS_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    const std::string s = g_err;
    if (s.rfind("region:", 0) == 0) return FBLTS_EREGION;
    return FBLTS_EINVAL;
  } catch (...) {
    g_err = "unknown error";
    return FBLTS_EINVAL;
  }
}

// ----------------------------------------------------------- device buffers

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 8;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) throw Err(FBLTS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    bytes = b;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

template <class T>
void upload(DevBuf& d, const std::vector<T>& v) {
  d.alloc(v.size() * sizeof(T));
  if (!v.empty()) hip_check(hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy H2D");
}

// Device copy of the permuted mesh.
struct DevMesh {
  DevBuf c_nedge, c_edge, c_nbr, c_invA, c_A, c_H;
  DevBuf e_cell, e_vert, e_dc, e_dv, e_invdc, e_He, e_neoe, e_eoe, e_w;
  DevBuf v_edge, v_cell, v_kite, v_invA, v_A, v_f, v_q0;
  DevBuf e_wT, c_vert, c_kite, c_R, e_cs, e_vq_edge, e_vq_cell;
  DevBuf cell_n2o, edge_n2o, vert_n2o;
  MeshDev md{};
  void upload_from(const PermMesh& pm, const Plan& p) {
    upload(c_nedge, pm.c_nedge);
    upload(c_edge, pm.c_edge);
    upload(c_nbr, pm.c_nbr);
    upload(c_invA, pm.c_invA);
    upload(c_A, pm.c_A);
    upload(c_H, pm.c_H);
    upload(e_cell, pm.e_cell);
    upload(e_vert, pm.e_vert);
    upload(e_dc, pm.e_dc);
    upload(e_dv, pm.e_dv);
    upload(e_invdc, pm.e_invdc);
    upload(e_He, pm.e_He);
    upload(e_neoe, pm.e_neoe);
    upload(e_eoe, pm.e_eoe);
    upload(e_w, pm.e_w);
    upload(v_edge, pm.v_edge);
    upload(v_cell, pm.v_cell);
    upload(v_kite, pm.v_kite);
    upload(v_invA, pm.v_invA);
    upload(v_A, pm.v_A);
    upload(v_f, pm.v_f);
    upload(v_q0, pm.v_q0);
    upload(e_wT, pm.e_wT);
    upload(c_vert, pm.c_vert);
    upload(c_kite, pm.c_kite);
    upload(c_R, pm.c_R);
    upload(e_cs, pm.e_cs);
    {
      // each edge's two vertex lists, slot-major per edge: the prep pass with
      // fused q_v then finds the vertices' edges and cells in its first round
      std::vector<int> vqe((size_t)6 * pm.es, 0), vqc((size_t)6 * pm.es, 0);
      for (int e = 0; e < pm.E; ++e)
        for (int side = 0; side < 2; ++side) {
          const int v = pm.e_vert[(size_t)side * pm.es + e];
          for (int j = 0; j < 3; ++j) {
            vqe[(size_t)(3 * side + j) * pm.es + e] = pm.v_edge[(size_t)j * pm.vs + v];
            vqc[(size_t)(3 * side + j) * pm.es + e] = pm.v_cell[(size_t)j * pm.vs + v];
          }
        }
      upload(e_vq_edge, vqe);
      upload(e_vq_cell, vqc);
    }
    upload(cell_n2o, p.cell_new2old);
    upload(edge_n2o, p.edge_new2old);
    upload(vert_n2o, p.vert_new2old);
    md.N = pm.N;
    md.E = pm.E;
    md.V = pm.V;
    md.cs = pm.cs;
    md.es = pm.es;
    md.vs = pm.vs;
    md.maxE = pm.maxE;
    md.maxEOE = pm.maxEOE;
    md.c_nedge = c_nedge.as<int>();
    md.c_edge = c_edge.as<int>();
    md.c_nbr = c_nbr.as<int>();
    md.c_invA = c_invA.as<double>();
    md.c_A = c_A.as<double>();
    md.c_H = c_H.as<double>();
    md.e_cell = e_cell.as<int>();
    md.e_vert = e_vert.as<int>();
    md.e_dc = e_dc.as<double>();
    md.e_dv = e_dv.as<double>();
    md.e_invdc = e_invdc.as<double>();
    md.e_He = e_He.as<double>();
    md.e_neoe = e_neoe.as<int>();
    md.e_eoe = e_eoe.as<int>();
    md.e_w = e_w.as<double>();
    md.v_edge = v_edge.as<int>();
    md.v_cell = v_cell.as<int>();
    md.v_kite = v_kite.as<double>();
    md.v_invA = v_invA.as<double>();
    md.v_A = v_A.as<double>();
    md.v_f = v_f.as<double>();
    md.v_q0 = v_q0.as<double>();
    md.e_wT = e_wT.as<double>();
    md.c_vert = c_vert.as<int>();
    md.c_kite = c_kite.as<double>();
    md.c_R = c_R.as<double>();
    md.e_cs = e_cs.as<int>();
    md.e_vq_edge = e_vq_edge.as<int>();
    md.e_vq_cell = e_vq_cell.as<int>();
  }
};

// State and scratch of nm members on one mesh.
struct DevState {
  int nm = 1, nm_log2 = 0;
  DevBuf H[4], hs, B, acc_h, sv_h, cd;
  DevBuf U[4], acc_u, sv_u, P, q;
  DevBuf wind_n, wind_t, wind_c;   // wind forcing: components and C_W per edge and member
  bool has_wind = false;
  DevBuf slow;   // operator splitting: frozen slow momentum tendency [E*nm]
  // moving cyclone: wind evaluated on the device once per coarse step
  DevBuf cyc_x, cyc_n, cyc_clock, cyc_p;
  bool cyclone = false;
  CycloneArgs cyc{};
  void alloc(const PermMesh& pm, const Plan& p, int nm_) {
    nm = nm_;
    nm_log2 = 0;
    while ((1 << nm_log2) < nm) ++nm_log2;
    const size_t Nc = (size_t)pm.N * nm, Ne = (size_t)pm.E * nm, Nv = (size_t)pm.V * nm;
    for (int k = 0; k < 4; ++k) {
      H[k].alloc(Nc * 8);
      U[k].alloc(Ne * 8);
    }
    hs.alloc(Nc * 8);
    B.alloc(Nc * 8);
    acc_h.alloc(Nc * 8);
    cd.alloc(Nc * 8);
    acc_u.alloc(Ne * 8);
    P.alloc(Ne * 32);
    q.alloc(Nv * 8);
    sv_h.alloc((size_t)4 * std::max(1, p.nIF1) * nm * 8);
    sv_u.alloc((size_t)4 * std::max(1, p.nIF1E) * nm * 8);
  }
  // The fine substeps' own stage arrays and scratch (pipelined FB-LTS step:
  // fine substep 0 runs beside the coarse stages 2 and 3, so neither may
  // overwrite what the other reads); allocated on first use, zeroed once.
  DevBuf Hf[4], Uf[3], hs_f, B_f, P_f, q_f;
  void alloc_fine(const PermMesh& pm, hipStream_t st) {
    const size_t Nc = (size_t)pm.N * nm, Ne = (size_t)pm.E * nm, Nv = (size_t)pm.V * nm;
    if (hs_f.bytes >= Nc * 8 && P_f.bytes >= Ne * 32 && q_f.bytes >= Nv * 8) return;
    DevBuf* cells[] = {&Hf[1], &Hf[2], &Hf[3], &hs_f, &B_f};
    DevBuf* edges[] = {&Uf[1], &Uf[2]};
    for (DevBuf* b : cells) b->alloc(Nc * 8);
    for (DevBuf* b : edges) b->alloc(Ne * 8);
    P_f.alloc(Ne * 32);
    q_f.alloc(Nv * 8);
    for (DevBuf* b : {&Hf[1], &Hf[2], &Hf[3], &hs_f, &B_f, &Uf[1], &Uf[2], &P_f, &q_f})
      hip_check(hipMemsetAsync(b->p, 0, b->bytes, st), "hipMemsetAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  }
};

struct Pass {
  enum Kind { CELL, VERT, PREP, EDGE, PRED, ASM, RK4FIN, COPY, WIND, TICK } kind;
  // position in the step: 100*phase + 10*substep + stage (phase 0 coarse, 1 fine,
  // 2 prediction, 3 assembly); used to place the adjoint's tape snapshots
  int tag = 0;
  double* cdst = nullptr;          // COPY
  const double* csrc = nullptr;
  long cn = 0;
  Launch<CellSeg> cell{};
  Launch<VertSeg> vert{};
  Launch<PrepSeg> prep{};
  Launch<EdgeSeg> edge{};
  Launch<PredSeg> pred{};
  Launch<AsmSeg> asmb{};
  std::vector<CycloneArgs> cycs;   // WIND (one per mesh)
  std::vector<long long*> clocks;  // TICK (one per mesh)
  // RK4 final: per segment (y, acc, n)
  std::vector<std::tuple<double*, const double*, long>> fin;
  double fin_c = 0.0;
  double model_bytes = 0.0;   // per-pass model (intermediates included)
  double comp_bytes = 0.0;    // compulsory model (intermediates free)
  bool fuse_q = false;   // PREP: evaluate q_v in the prep pass (no vertex pass)
  int cell_mode = 1;     // CELL: 0 linear, 1 nonlinear, 2 fast terms (k_cell<MODE>)
  bool edge_fast = false;   // EDGE: fast momentum pass (k_edge_fast)
  bool edge_cells = false;  // EDGE: PV flux through the cells' edge lists (k_edge<., ., true>)
  int bs = kBlock;       // threads per block of the stencil passes
};

struct MeshUnit {
  // one mesh with nm members: plan, device mesh, state, pass list
  const HostMesh* hm = nullptr;
  std::vector<int8_t> lab4;
  std::vector<int> layer;
  Plan plan;
  PermMesh pm;
  DevMesh dm;
  DevState st;
  std::vector<Pass> passes;
  uint64_t version = 0;   // advanced whenever the pass list is rebuilt
  int64_t cell_substeps = 0;
  double bytes_edge = 0.0, bytes_cell = 0.0;   // per-pass model of the momentum / thickness passes
  double comp_edge = 0.0, comp_cell = 0.0;     // compulsory model of the same passes
  int64_t edge_items = 0;
};

struct Params {
  fblts_params p;
  bool nonlinear() const { return p.physics == FBLTS_PHYS_NONLINEAR; }
  bool gravity_wave() const { return p.physics == FBLTS_PHYS_GRAVITY_WAVE; }
  // stencils reach neighbour thicknesses (nonlinear flux): nonlinear and fast terms
  bool wide() const { return p.physics != FBLTS_PHYS_LINEAR; }
  // stages evaluate only the fast terms (plus a frozen slow tendency when split)
  bool fast() const { return gravity_wave() || p.split > 0; }
};

void check_params(const fblts_params* p) {
  if (!p) throw Err(FBLTS_EINVAL, "params is NULL");
  if (!(p->dt > 0) || !std::isfinite(p->dt)) throw Err(FBLTS_EINVAL, "dt must be positive");
  if (!(p->g > 0)) throw Err(FBLTS_EINVAL, "g must be positive");
  if (p->M < 1 || p->M > 1024) throw Err(FBLTS_EINVAL, "M must be in 1..1024");
  if (p->scheme < 0 || p->scheme > 2) throw Err(FBLTS_EINVAL, "unknown scheme");
  if (p->physics < 0 || p->physics > 2) throw Err(FBLTS_EINVAL, "unknown physics");
  if (p->split < 0 || p->split > 2) throw Err(FBLTS_EINVAL, "split must be 0, 1 or 2");
  if (p->split && p->physics != FBLTS_PHYS_NONLINEAR)
    throw Err(FBLTS_EINVAL, "operator splitting needs nonlinear physics");
  if (p->split && p->scheme == FBLTS_SCHEME_RK4) throw Err(FBLTS_EINVAL, "operator splitting applies to FB schemes");
  if (p->split == 2 && p->scheme != FBLTS_SCHEME_FBLTS)
    throw Err(FBLTS_EINVAL, "per-substep slow terms (split 2) need the FB-LTS scheme");
  if (p->r_layers < 1 || p->r_layers > 64) throw Err(FBLTS_EINVAL, "r_layers must be in 1..64");
}

// Build the pass list of one mesh unit (segments are merged by the caller).
// Launch-structure options (results are bitwise identical across them).
struct LaunchOpts {
  bool fuse_q = true;        // q_v evaluated inside the prep pass
  int block = kBlock;        // threads per block of the stencil passes
  bool edge_cells = false;   // momentum pass through the cells' edge lists
  int graph_steps = 8;       // coarse steps per replayed hipGraph
  int persistent = 0;        // > 0: runs of passes in one cooperative launch each, with
                             // this many blocks per compute unit
  bool pipeline = true;      // FB-LTS: fine substep 0 beside the coarse stages, prediction
                             // and assembly folded into momentum passes
};

// Pipelined FB-LTS step: the same passes and arithmetic as the sequential
// list (Sec. 2.2 steps 1-4), arranged into fewer dependent launches.
//  * Fine substep 0 depends on the coarse advancement only through the
//    interface-one predictions, and its stage j needs the coarse stage j
//    values only: it runs on its own arrays (Hf, Uf) and scratch, as a second
//    segment of the launches of coarse stage j + 1.  The coarse stages hand
//    their values over as they form them (Mirror): the k = 0 prediction on
//    interface one, and on stage 2 and 3 the values themselves where the
//    third fine stage reads interface two and the interior.
//  * The prediction for substep k + 1, and after the last substep the
//    correction and assembly, are folded into the last momentum pass of
//    substep k (StepTail) instead of launching on their own.
// A coarse step is then 9M + 3 stencil launches instead of 10M + 10 (q_v
// fused).  emit(which, k) appends one stage's passes: which 0..2 the coarse
// stages, 3..5 the fine stages of substep k, 6 the per-substep slow terms.
template <class Emit>
void build_pipelined(MeshUnit& u, const Params& P, const Plan& pl, Emit emit, hipStream_t st) {
  const fblts_params& p = P.p;
  DevState& s = u.st;
  s.alloc_fine(u.pm, st);
  const int M = p.M, N = u.pm.N, E = u.pm.E, nm = s.nm;
  auto take = [&](int which, int k) {
    std::vector<Pass> keep;
    keep.swap(u.passes);
    emit(which, k);
    std::vector<Pass> got;
    got.swap(u.passes);
    u.passes.swap(keep);
    return got;
  };
  const int if1b = pl.nF, if1e = pl.nF + pl.nIF1, if2e = if1e + pl.nIF2;
  const int if1eb = pl.nFE, if1ee = pl.nFE + pl.nIF1E, if2ee = if1ee + pl.nIF2E;
  const int cend = std::max(pl.fine3_cell_end, if1e), eend = std::max(pl.fine3_edge_end, if1ee);
  // the k = 0 prediction coefficients, formed as the prediction pass forms them
  const double invM = 1.0 / M, c0 = (double)(M - 1) / (double)M, ap0 = (double)1 / (double)M;
  auto internal = [](const char* what) { throw Err(FBLTS_EINVAL, std::string("internal: pipelined step: ") + what); };
  auto add_bytes = [&](Pass& ps, double b) {
    ps.model_bytes += b;
    ps.comp_bytes += b;
    if (ps.kind == Pass::EDGE) {
      u.bytes_edge += b;
      u.comp_edge += b;
    } else if (ps.kind == Pass::CELL) {
      u.bytes_cell += b;
      u.comp_cell += b;
    }
  };
  auto set_mirror = [&](std::vector<Pass>& v, Pass::Kind kind, Mirror m) {
    if (m.e <= m.b) return;
    for (Pass& ps : v) {
      if (ps.kind != kind) continue;
      int ub, ue, b, e;
      if (kind == Pass::CELL) {
        const CellSeg& c = ps.cell.seg[0];
        ub = c.upd_begin, ue = c.upd_end, b = c.begin, e = c.end;
      } else {
        const EdgeSeg& c = ps.edge.seg[0];
        ub = c.upd_begin, ue = c.upd_end, b = c.begin, e = c.end;
      }
      if (m.b < std::max(ub, b) || m.e > std::min(ue, e)) internal("hand-over range outside the coarse update");
      if (kind == Pass::CELL) ps.cell.seg[0].mir = m;
      else ps.edge.seg[0].mir = m;
      add_bytes(ps, 8.0 * nm * ((double)(m.e - m.b) + (m.sv ? (double)(m.p - m.b) : 0.0)));
      return;
    }
    internal("no pass to hand over from");
  };
  auto set_tail = [&](std::vector<Pass>& v, int k) {
    for (Pass& ps : v) {
      if (ps.kind != Pass::EDGE) continue;
      EdgeSeg& e = ps.edge.seg[0];
      StepTail t{};
      t.c_b = if1b, t.c_p = if1e, t.c_q = if2e, t.c_e = N;
      t.e_b = if1eb, t.e_p = if1ee, t.e_q = if2ee, t.e_e = E;
      t.H0 = s.H[0].as<double>();
      t.H1 = s.Hf[1].as<double>();
      t.H2 = s.Hf[2].as<double>();
      t.H3 = s.Hf[3].as<double>();
      t.C1 = s.H[1].as<double>();
      t.C2 = s.H[2].as<double>();
      t.C3 = s.H[3].as<double>();
      t.U0 = s.U[0].as<double>();
      t.U1 = s.Uf[1].as<double>();
      t.U2 = s.Uf[2].as<double>();
      t.D1 = s.U[1].as<double>();
      t.D2 = s.U[2].as<double>();
      t.D3 = s.U[3].as<double>();
      t.sv_h = s.sv_h.as<double>();
      t.sv_u = s.sv_u.as<double>();
      t.acc_h = s.acc_h.as<double>();
      double b;
      if (k + 1 < M) {
        const int kk = k + 1;
        t.kind = 1;
        t.a = (double)kk / (double)M;
        t.one_minus_a = (double)(M - kk) / (double)M;
        t.invM = 1.0 / M;
        t.c = (double)(M - kk - 1) / (double)M;
        t.ap = (double)(kk + 1) / (double)M;
        if (if1ee > if1eb && (e.begin > if1eb || e.end < if1ee)) internal("interface-one edges outside the pass");
        b = 64.0 * (if1e - if1b) + 56.0 * (if1ee - if1eb);
      } else {
        t.kind = 2;
        t.delta = p.dt / M;
        if (if2ee > if1eb && (e.acc_begin > if1eb || e.acc_end < if2ee))
          internal("interface edges outside the accumulation");
        b = 24.0 * (if1e - if1b) + 24.0 * (if2e - if1e) + 16.0 * (N - if2e) + 16.0 * (if2ee - if1eb) +
            16.0 * (E - if2ee);
      }
      if (e.end < e.begin) e.end = e.begin;
      e.tail = t;
      add_bytes(ps, b * nm);
      return;
    }
    internal("no momentum pass to fold into");
  };
  // one launch for two stages' passes of a kind (segments of one launch)
  auto rank = [](const Pass& q) {
    switch (q.kind) {
      case Pass::CELL: return 0;
      case Pass::VERT: return 1;
      case Pass::PREP: return 2;
      case Pass::EDGE: return 3;
      default: return 4;
    }
  };
  auto nonempty = [](const Pass& q) {
    switch (q.kind) {
      case Pass::CELL: return q.cell.seg[0].end > q.cell.seg[0].begin;
      case Pass::VERT: return q.vert.seg[0].end > q.vert.seg[0].begin;
      case Pass::PREP: return q.prep.seg[0].end > q.prep.seg[0].begin;
      case Pass::EDGE: return q.edge.seg[0].end > q.edge.seg[0].begin || q.edge.seg[0].tail.kind != 0;
      default: return true;
    }
  };
  auto merge2 = [&](const std::vector<Pass>& a, const std::vector<Pass>& b) {
    std::vector<Pass> out;
    size_t i = 0, j = 0;
    while (i < a.size() || j < b.size()) {
      if (j == b.size() || (i < a.size() && rank(a[i]) < rank(b[j]))) {
        out.push_back(a[i++]);
        continue;
      }
      if (i == a.size() || rank(b[j]) < rank(a[i])) {
        out.push_back(b[j++]);
        continue;
      }
      const Pass& x = a[i++];
      const Pass& y = b[j++];
      if (rank(x) > 3) internal("unexpected pass kind in a stage");
      if (!nonempty(y)) {
        out.push_back(x);
        continue;
      }
      if (!nonempty(x)) {
        out.push_back(y);
        continue;
      }
      Pass m = x;
      switch (m.kind) {
        case Pass::CELL: m.cell.seg[m.cell.nseg++] = y.cell.seg[0]; break;
        case Pass::VERT: m.vert.seg[m.vert.nseg++] = y.vert.seg[0]; break;
        case Pass::PREP: m.prep.seg[m.prep.nseg++] = y.prep.seg[0]; break;
        default: m.edge.seg[m.edge.nseg++] = y.edge.seg[0]; break;
      }
      m.model_bytes += y.model_bytes;
      m.comp_bytes += y.comp_bytes;
      out.push_back(m);
    }
    return out;
  };
  auto append = [&](const std::vector<Pass>& v) { u.passes.insert(u.passes.end(), v.begin(), v.end()); };

  std::vector<Pass> C[3];
  for (int j = 0; j < 3; ++j) C[j] = take(j, 0);
  set_mirror(C[0], Pass::CELL, Mirror{s.Hf[1].as<double>(), s.sv_h.as<double>(), if1b, if1e, if1e, invM, c0});
  set_mirror(C[0], Pass::EDGE, Mirror{s.Uf[1].as<double>(), s.sv_u.as<double>(), if1eb, if1ee, if1ee, invM, c0});
  set_mirror(C[1], Pass::CELL, Mirror{s.Hf[2].as<double>(), nullptr, if1b, if1e, cend, invM, c0});
  set_mirror(C[1], Pass::EDGE, Mirror{s.Uf[2].as<double>(), nullptr, if1eb, if1ee, eend, invM, c0});
  set_mirror(C[2], Pass::CELL, Mirror{s.Hf[3].as<double>(), nullptr, if1b, if1e, cend, ap0, c0});
  for (int k = 0; k < M; ++k) {
    if (p.split == 2 && k > 0) append(take(6, k));
    std::vector<Pass> F[3];
    for (int j = 0; j < 3; ++j) F[j] = take(3 + j, k);
    set_tail(F[2], k);
    if (k == 0) {
      append(C[0]);
      append(merge2(C[1], F[0]));
      append(merge2(C[2], F[1]));
      append(F[2]);
    } else {
      for (auto& f : F) append(f);
    }
  }
  u.cell_substeps = ((int64_t)(N - pl.nF) + (int64_t)M * pl.nF) * nm;
}

void build_passes_impl(MeshUnit& u, const Params& P, bool drag_on, bool fuse_q, const Plan* plan = nullptr,
                       bool edge_cells = false, bool pipeline = false, hipStream_t st = nullptr) {
  const fblts_params& p = P.p;
  const bool nl = P.nonlinear();
  const MeshDev& md = u.dm.md;
  DevState& s = u.st;
  auto H = [&](int k) { return s.H[k].as<double>(); };
  auto U = [&](int k) { return s.U[k].as<double>(); };
  // stage scratch (h*, B, edge records, q_v): the fine substeps of a
  // pipelined step switch to their own set
  double* sc_hs = s.hs.as<double>();
  double* sc_B = s.B.as<double>();
  double* sc_P = s.P.as<double>();
  double* sc_q = s.q.as<double>();
  u.passes.clear();
  int cur_tag = 0;
  u.bytes_edge = 0;
  u.bytes_cell = 0;
  u.comp_edge = 0;
  u.comp_cell = 0;
  u.edge_items = 0;
  const int nm = s.nm;

  const bool fast = P.fast();
  const int stage_cell_mode = fast ? 2 : (nl ? 1 : 0);
  if (p.split && s.slow.bytes < (size_t)md.E * nm * 8) s.slow.alloc((size_t)md.E * nm * 8);
  const double* slow = p.split ? s.slow.as<double>() : nullptr;
  auto cell_pass = [&](const StageRanges& r, const double* Hsrc, const double* Usrc, const double* H0,
                       const double* Hnew_src, double* Hdst, double c_dt, double wn, double ws, double wb,
                       double* acc, double acc_w, int acc_first, int mode, double g) {
    Pass ps;
    ps.kind = Pass::CELL;
    ps.cell_mode = mode;
    ps.cell.nseg = 1;
    CellSeg& c = ps.cell.seg[0];
    c.m = md;
    c.nm_log2 = s.nm_log2;
    c.begin = r.cell.b;
    c.end = r.cell.e;
    c.upd_begin = r.cell_upd.b;
    c.upd_end = r.cell_upd.e;
    c.acc_begin = r.cell_acc.b;
    c.acc_end = r.cell_acc.e;
    c.acc_first = acc_first;
    c.Hsrc = Hsrc;
    c.Usrc = Usrc;
    c.H0 = H0;
    c.Hnew_src = Hnew_src;
    c.Hdst = Hdst;
    c.hs = sc_hs;
    c.B = sc_B;
    c.acc = acc;
    c.c_dt = c_dt;
    c.wn = wn;
    c.ws = ws;
    c.wb = wb;
    c.acc_w = acc_w;
    c.g = g;
    ps.model_bytes = bytes_cell_pass(u.pm, r, mode != 0, nm, mode == 1);
    ps.comp_bytes = compulsory_cell_pass(u.pm, r, mode != 0, nm, mode == 1);
    u.bytes_cell += ps.model_bytes;
    u.comp_cell += ps.comp_bytes;
    ps.tag = cur_tag;
    u.passes.push_back(ps);
  };
  auto vert_pass = [&](const StageRanges& r, const double* Usrc) {
    if (!nl || fuse_q || r.vert.size() == 0) return;
    Pass ps;
    ps.kind = Pass::VERT;
    ps.vert.nseg = 1;
    VertSeg& v = ps.vert.seg[0];
    v.m = md;
    v.nm_log2 = s.nm_log2;
    v.begin = r.vert.b;
    v.end = r.vert.e;
    v.Usrc = Usrc;
    v.hs = sc_hs;
    v.q = sc_q;
    ps.model_bytes = bytes_vert_pass(u.pm, r.vert, nm);
    ps.comp_bytes = compulsory_vert_pass(u.pm, r.vert, nm);
    ps.tag = cur_tag;
    u.passes.push_back(ps);
  };
  auto prep_pass = [&](const StageRanges& r, const double* Usrc) {
    Pass ps;
    ps.kind = Pass::PREP;
    ps.prep.nseg = 1;
    PrepSeg& q = ps.prep.seg[0];
    q.m = md;
    q.nm_log2 = s.nm_log2;
    q.begin = r.prep.b;
    q.end = r.prep.e;
    q.linear = nl ? 0 : 1;
    q.Usrc = Usrc;
    q.hs = sc_hs;
    q.q = nl ? sc_q : md.v_q0;
    q.P = sc_P;
    ps.fuse_q = nl && fuse_q;
    ps.model_bytes = bytes_prep_pass(u.pm, r.prep, nl, nm, ps.fuse_q);
    // with q_v fused the prep pass references the vertex pass's arrays too
    ps.comp_bytes = compulsory_prep_pass(u.pm, r.prep, nl, nm) +
                    (ps.fuse_q ? compulsory_vert_pass(u.pm, r.vert, nm) : 0.0);
    ps.tag = cur_tag;
    u.passes.push_back(ps);
  };
  auto edge_pass = [&](const StageRanges& r, const double* Usrc, const double* U0, double* Udst, double c_dt,
                       double* acc, double acc_w, int acc_first, bool fast_pass) {
    Pass ps;
    ps.kind = Pass::EDGE;
    ps.edge_fast = fast_pass;
    ps.edge_cells = edge_cells && !fast_pass;
    ps.edge.nseg = 1;
    EdgeSeg& e = ps.edge.seg[0];
    e.m = md;
    e.nm_log2 = s.nm_log2;
    e.begin = r.edge.b;
    e.end = r.edge.e;
    e.upd_begin = r.edge_upd.b;
    e.upd_end = r.edge_upd.e;
    e.acc_begin = r.edge_acc.b;
    e.acc_end = r.edge_acc.e;
    e.acc_first = acc_first;
    e.P = sc_P;
    e.B = sc_B;
    e.Usrc = Usrc;
    e.U0 = U0;
    e.Udst = Udst;
    e.acc = acc;
    e.cd = drag_on ? s.cd.as<double>() : nullptr;
    e.wind_n = s.has_wind ? s.wind_n.as<double>() : nullptr;
    e.wind_t = s.has_wind ? s.wind_t.as<double>() : nullptr;
    e.wind_c = s.has_wind ? s.wind_c.as<double>() : nullptr;
    e.c_dt = c_dt;
    e.acc_w = acc_w;
    e.slow = fast_pass ? slow : nullptr;
    ps.model_bytes = fast_pass ? bytes_edge_fast_pass(u.pm, r, slow != nullptr, nm)
                     : ps.edge_cells ? bytes_edge_cells_pass(u.pm, r, drag_on, s.has_wind, nm)
                                     : bytes_edge_pass(u.pm, r, drag_on, s.has_wind, nm);
    ps.comp_bytes = fast_pass ? compulsory_edge_fast_pass(u.pm, r, slow != nullptr, nm)
                              : compulsory_edge_pass(u.pm, r, drag_on, s.has_wind, nm);
    u.bytes_edge += ps.model_bytes;
    u.comp_edge += ps.comp_bytes;
    u.edge_items += (int64_t)r.edge.size() * nm;
    ps.tag = cur_tag;
    u.passes.push_back(ps);
  };
  auto stage = [&](const StageRanges& r, const double* Hsrc, const double* Usrc, const double* H0,
                   const double* Hnew_src, double* Hdst, double c_dt, double wn, double ws, double wb, double* acch,
                   const double* U0, double* Udst, double* accu, double acc_w, int acc_first) {
    cell_pass(r, Hsrc, Usrc, H0, Hnew_src, Hdst, c_dt, wn, ws, wb, acch, acc_w, acc_first, stage_cell_mode, p.g);
    if (!fast) {
      vert_pass(r, Usrc);
      prep_pass(r, Usrc);
    }
    edge_pass(r, Usrc, U0, Udst, c_dt, accu, acc_w, acc_first, fast);
  };
  // Operator splitting (Section 3.2, eq. splitting): the slow momentum
  // tendency (PV flux, -grad K, drag, wind) at the state (Hs, Us), written to
  // `slow` on the edge range of r.  Cell pass with g = 0 (B = K) and h* = Hs,
  // then the full vertex / prep / momentum passes with the result accumulated
  // (first write) into `slow`; nothing is updated.
  auto slow_eval = [&](const StageRanges& r, const double* Hs, const double* Us) {
    StageRanges q = r;
    q.cell_upd = q.cell_acc = Range{0, 0};
    q.edge_upd = Range{0, 0};
    q.edge_acc = q.edge;
    cell_pass(q, Hs, Us, Hs, Hs, nullptr, 0.0, 0.0, 1.0, 0.0, nullptr, 1.0, 1, 1, 0.0);
    vert_pass(q, Us);
    prep_pass(q, Us);
    edge_pass(q, Us, Us, nullptr, 0.0, s.slow.as<double>(), 1.0, 1, false);
  };
  StageRanges full{};
  full.cell = Range{0, md.N};
  full.vert = Range{0, md.V};
  full.prep = Range{0, md.E};
  full.edge = Range{0, md.E};

  const double dt = p.dt, b1 = p.beta1, b2 = p.beta2, b3 = p.beta3;
  const Plan& pl = plan ? *plan : u.plan;
  const int N = md.N, E = md.E;
  if (p.scheme == FBLTS_SCHEME_FBRK32) {
    const StageRanges* R = pl.coarse;
    if (p.split) slow_eval(full, H(0), U(0));
    stage(R[0], H(0), U(0), H(0), H(1), H(1), dt / 3, b1, 0.0, 1 - b1, nullptr, U(0), U(1), nullptr, 1, 1);
    stage(R[1], H(1), U(1), H(0), H(2), H(2), dt / 2, b2, 0.0, 1 - b2, nullptr, U(0), U(2), nullptr, 1, 1);
    // stage 3 updates the state in place
    stage(R[2], H(2), U(2), H(0), H(0), H(0), dt, b3, 1 - 2 * b3, b3, nullptr, U(0), U(0), nullptr, 1, 1);
    u.cell_substeps = (int64_t)N * nm;
    return;
  }
  if (p.scheme == FBLTS_SCHEME_RK4) {
    StageRanges R = pl.coarse[0];
    StageRanges Racc = R;
    Racc.cell_acc = {0, N};
    Racc.edge_acc = {0, E};
    StageRanges Rlast = Racc;
    Rlast.cell_upd = {0, 0};
    Rlast.edge_upd = {0, 0};
    double* ah = s.acc_h.as<double>();
    double* au = s.acc_u.as<double>();
    // y2 = y + dt/2 k1 -> slot 1; y3 = y + dt/2 k2 -> slot 2; y4 = y + dt k3 -> slot 1
    stage(Racc, H(0), U(0), H(0), H(1), H(1), dt / 2, 0.0, 1.0, 0.0, ah, U(0), U(1), au, 1.0, 1);
    stage(Racc, H(1), U(1), H(0), H(2), H(2), dt / 2, 0.0, 1.0, 0.0, ah, U(0), U(2), au, 2.0, 0);
    stage(Racc, H(2), U(2), H(0), H(1), H(1), dt, 0.0, 1.0, 0.0, ah, U(0), U(1), au, 2.0, 0);
    stage(Rlast, H(1), U(1), H(0), H(3), H(3), 0.0, 0.0, 1.0, 0.0, ah, U(0), U(3), au, 1.0, 0);
    Pass fin;
    fin.kind = Pass::RK4FIN;
    fin.fin_c = dt / 6.0;
    fin.fin.emplace_back(H(0), ah, (long)N * nm);
    fin.fin.emplace_back(U(0), au, (long)E * nm);
    fin.model_bytes = 3.0 * 8.0 * ((double)N + E) * nm;
    u.passes.push_back(fin);
    u.cell_substeps = (int64_t)N * nm;
    return;
  }
  // ---- FB-LTS
  const int M = p.M;
  const double delta = dt / M;
  const StageRanges* C = pl.coarse;
  if (p.split) {
    cur_tag = 0;
    slow_eval(full, H(0), U(0));
  }
  if (pipeline) {
    build_pipelined(u, P, pl, [&](int which, int k) {
      // which: 0..2 coarse stage, 3..5 fine stage of substep k, 6 the
      // per-substep slow terms (split 2); the fine ones on the fine arrays
      // and scratch
      DevState& d = u.st;
      auto Hf = [&](int j) { return j == 0 ? H(0) : d.Hf[j].as<double>(); };
      auto Uf = [&](int j) { return j == 0 ? U(0) : d.Uf[j].as<double>(); };
      const bool fine = which >= 3;
      sc_hs = fine ? d.hs_f.as<double>() : d.hs.as<double>();
      sc_B = fine ? d.B_f.as<double>() : d.B.as<double>();
      sc_P = fine ? d.P_f.as<double>() : d.P.as<double>();
      sc_q = fine ? d.q_f.as<double>() : d.q.as<double>();
      double* ahp = d.acc_h.as<double>();
      double* aup = d.acc_u.as<double>();
      const double dl = dt / M;
      switch (which) {
        case 0:
          cur_tag = 1;
          stage(C[0], H(0), U(0), H(0), H(1), H(1), dt / 3, b1, 0.0, 1 - b1, nullptr, U(0), U(1), nullptr, 1, 1);
          break;
        case 1:
          cur_tag = 2;
          stage(C[1], H(1), U(1), H(0), H(2), H(2), dt / 2, b2, 0.0, 1 - b2, nullptr, U(0), U(2), nullptr, 1, 1);
          break;
        case 2:
          cur_tag = 3;
          stage(C[2], H(2), U(2), H(0), H(3), H(3), dt, b3, 1 - 2 * b3, b3, nullptr, U(0), U(3), nullptr, 1, 1);
          break;
        case 3:
          cur_tag = 100 + 10 * k + 1;
          stage(pl.fine[0], H(0), U(0), H(0), Hf(1), Hf(1), dl / 3, b1, 0.0, 1 - b1, nullptr, U(0), Uf(1), nullptr,
                1, 1);
          break;
        case 4:
          cur_tag = 100 + 10 * k + 2;
          stage(pl.fine[1], Hf(1), Uf(1), H(0), Hf(2), Hf(2), dl / 2, b2, 0.0, 1 - b2, nullptr, U(0), Uf(2), nullptr,
                1, 1);
          break;
        case 5:
          cur_tag = 100 + 10 * k + 3;
          stage(pl.fine[2], Hf(2), Uf(2), H(0), Hf(3), H(0), dl, b3, 1 - 2 * b3, b3, ahp, U(0), U(0), aup, 1.0,
                k == 0);
          break;
        case 6:
          cur_tag = 100 + 10 * k;
          slow_eval(pl.fine[2], H(0), U(0));
          break;
      }
    }, st);
    return;
  }
  cur_tag = 1;
  stage(C[0], H(0), U(0), H(0), H(1), H(1), dt / 3, b1, 0.0, 1 - b1, nullptr, U(0), U(1), nullptr, 1, 1);
  cur_tag = 2;
  stage(C[1], H(1), U(1), H(0), H(2), H(2), dt / 2, b2, 0.0, 1 - b2, nullptr, U(0), U(2), nullptr, 1, 1);
  cur_tag = 3;
  stage(C[2], H(2), U(2), H(0), H(3), H(3), dt, b3, 1 - 2 * b3, b3, nullptr, U(0), U(3), nullptr, 1, 1);
  const int if1b = pl.nF, if1e = pl.nF + pl.nIF1, if2e = if1e + pl.nIF2;
  const int if1eb = pl.nFE, if1ee = pl.nFE + pl.nIF1E, if2ee = if1ee + pl.nIF2E;
  const StageRanges* F = pl.fine;
  if (p.split == 2)
    for (int j = 0; j < 2; ++j)
      if (F[j].edge.size() > 0 && (F[j].edge.b < F[2].edge.b || F[j].edge.e > F[2].edge.e))
        throw Err(FBLTS_EINVAL, "fine stage edge ranges are not nested (per-substep slow terms)");
  double* ah = s.acc_h.as<double>();
  double* au = s.acc_u.as<double>();
  for (int k = 0; k < M; ++k) {
    Pass pr;
    pr.kind = Pass::PRED;
    pr.pred.nseg = 1;
    PredSeg& q = pr.pred.seg[0];
    q.nm_log2 = s.nm_log2;
    q.c_begin = if1b;
    q.c_end = if1e;
    q.e_begin = if1eb;
    q.e_end = if1ee;
    q.H0 = H(0);
    q.H1 = H(1);
    q.H2 = H(2);
    q.H3 = H(3);
    q.U0 = U(0);
    q.U1 = U(1);
    q.U2 = U(2);
    q.U3 = U(3);
    q.sv_h = s.sv_h.as<double>();
    q.sv_u = s.sv_u.as<double>();
    q.save = k == 0;
    q.a = (double)k / (double)M;
    q.one_minus_a = (double)(M - k) / (double)M;
    q.invM = 1.0 / M;
    q.c = (double)(M - k - 1) / (double)M;
    q.ap = (double)(k + 1) / (double)M;
    pr.model_bytes = ((double)(if1e - if1b) * 8 + (double)(if1ee - if1eb) * 7) * 8.0 * nm;
    pr.tag = 200 + 10 * k;
    u.passes.push_back(pr);
    if (p.split == 2 && k > 0) {
      // Section 4.2's variant: slow terms at t^{n,k} from the substep's starting
      // state, on every edge the substep's stages compute (stage 3's range)
      cur_tag = 100 + 10 * k;
      slow_eval(F[2], H(0), U(0));
    }
    cur_tag = 100 + 10 * k + 1;
    stage(F[0], H(0), U(0), H(0), H(1), H(1), delta / 3, b1, 0.0, 1 - b1, nullptr, U(0), U(1), nullptr, 1, 1);
    cur_tag = 100 + 10 * k + 2;
    stage(F[1], H(1), U(1), H(0), H(2), H(2), delta / 2, b2, 0.0, 1 - b2, nullptr, U(0), U(2), nullptr, 1, 1);
    cur_tag = 100 + 10 * k + 3;
    stage(F[2], H(2), U(2), H(0), H(3), H(0), delta, b3, 1 - 2 * b3, b3, ah, U(0), U(0), au, 1.0, k == 0);
  }
  Pass as;
  as.kind = Pass::ASM;
  as.asmb.nseg = 1;
  AsmSeg& a = as.asmb.seg[0];
  a.nm_log2 = s.nm_log2;
  a.if1_c_begin = if1b;
  a.if1_c_end = if1e;
  a.if2_c_end = if2e;
  a.N = N;
  a.if1_e_begin = if1eb;
  a.if1_e_end = if1ee;
  a.if2_e_end = if2ee;
  a.E = E;
  a.H0 = H(0);
  a.H3 = H(3);
  a.acc_h = ah;
  a.sv_h = s.sv_h.as<double>();
  a.U0 = U(0);
  a.U3 = U(3);
  a.acc_u = au;
  a.sv_u = s.sv_u.as<double>();
  a.delta = delta;
  as.model_bytes = (((double)(N - if1b) * 3) + ((double)(E - if1eb) * 3)) * 8.0 * nm;
  as.tag = 300;
  u.passes.push_back(as);
  u.cell_substeps = ((int64_t)(N - pl.nF) + (int64_t)M * pl.nF) * nm;
}

// With a moving cyclone, each coarse step starts by evaluating the wind at
// the step's time and ends by advancing the device step clock.
void add_forcing_passes(MeshUnit& u) {
  if (!u.st.cyclone) return;
  Pass w;
  w.kind = Pass::WIND;
  w.tag = -1;
  w.cycs = {u.st.cyc};
  w.model_bytes = (double)u.pm.E * 8.0 * 8.0;
  Pass t;
  t.kind = Pass::TICK;
  t.tag = -2;
  t.clocks = {u.st.cyc_clock.as<long long>()};
  u.passes.insert(u.passes.begin(), w);
  u.passes.push_back(t);
}

void build_passes(MeshUnit& u, const Params& P, bool drag_on, const LaunchOpts& o, hipStream_t st) {
  const int bs = o.block;
  if (o.edge_cells && u.pm.kite_weights == 0)
    throw Err(FBLTS_EINVAL, "the mesh's edges_on_edge weights are not the kite-fraction walks of its cells");
  build_passes_impl(u, P, drag_on, o.fuse_q, nullptr, o.edge_cells, o.pipeline, st);
  add_forcing_passes(u);
  for (Pass& p : u.passes) p.bs = bs;
  ++u.version;
}

// Merge per-mesh pass lists into multi-segment launches.
std::vector<Pass> merge_passes(const std::vector<MeshUnit*>& units) {
  std::vector<Pass> out;
  if (units.empty()) return out;
  const size_t n = units[0]->passes.size();
  for (auto* u : units)
    if (u->passes.size() != n) throw Err(FBLTS_EINVAL, "ensemble meshes have different pass sequences");
  if ((int)units.size() > kMaxSeg) throw Err(FBLTS_EINVAL, "too many meshes in one ensemble (max 4)");
  for (size_t k = 0; k < n; ++k) {
    Pass ps = units[0]->passes[k];
    for (size_t m = 1; m < units.size(); ++m) {
      const Pass& q = units[m]->passes[k];
      if (q.kind != ps.kind) throw Err(FBLTS_EINVAL, "ensemble pass kinds differ");
      const int j = (int)m;
      switch (ps.kind) {
        case Pass::CELL: ps.cell.seg[j] = q.cell.seg[0]; ps.cell.nseg = j + 1; break;
        case Pass::VERT: ps.vert.seg[j] = q.vert.seg[0]; ps.vert.nseg = j + 1; break;
        case Pass::PREP: ps.prep.seg[j] = q.prep.seg[0]; ps.prep.nseg = j + 1; break;
        case Pass::EDGE: ps.edge.seg[j] = q.edge.seg[0]; ps.edge.nseg = j + 1; break;
        case Pass::PRED: ps.pred.seg[j] = q.pred.seg[0]; ps.pred.nseg = j + 1; break;
        case Pass::ASM: ps.asmb.seg[j] = q.asmb.seg[0]; ps.asmb.nseg = j + 1; break;
        case Pass::RK4FIN:
          for (auto& t : q.fin) ps.fin.push_back(t);
          break;
        case Pass::WIND: ps.cycs.insert(ps.cycs.end(), q.cycs.begin(), q.cycs.end()); break;
        case Pass::TICK: ps.clocks.insert(ps.clocks.end(), q.clocks.begin(), q.clocks.end()); break;
        case Pass::COPY: break;
      }
      ps.model_bytes += q.model_bytes;
      ps.comp_bytes += q.comp_bytes;
    }
    out.push_back(ps);
  }
  return out;
}

struct Timing {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[4];
  size_t used[4] = {0, 0, 0, 0};
  ~Timing() {
    for (auto& v : ev)
      for (auto& p : v) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
      }
  }
  std::pair<hipEvent_t, hipEvent_t> get(int cls) {
    if (used[cls] == ev[cls].size()) {
      hipEvent_t a, b;
      hip_check(hipEventCreate(&a), "hipEventCreate");
      hip_check(hipEventCreate(&b), "hipEventCreate");
      ev[cls].emplace_back(a, b);
    }
    return ev[cls][used[cls]++];
  }
  void unget(int cls) { --used[cls]; }
  void reset() { std::fill(used, used + 4, 0); }
};

// Launch the passes [first, last) on a stream.
void run_pass_range(const Pass* first, const Pass* last, bool drag, bool wind, hipStream_t st, Timing* tm) {
  for (const Pass* pp = first; pp != last; ++pp) {
    const Pass& ps = *pp;
    int cls = -1;
    switch (ps.kind) {
      case Pass::EDGE: cls = 0; break;
      case Pass::CELL: cls = 1; break;
      case Pass::VERT: cls = 2; break;
      case Pass::PREP: cls = 3; break;
      default: break;
    }
    // timed passes: the launch records the pair from its own dispatch timestamps
    std::pair<hipEvent_t, hipEvent_t> evp{nullptr, nullptr};
    if (tm && tm->on && cls >= 0) {
      evp = tm->get(cls);
      arm_launch_events(evp.first, evp.second);
    }
    int nb = -1;
    switch (ps.kind) {
      case Pass::CELL: nb = launch_cell(ps.cell, ps.cell_mode, ps.bs, st); break;
      case Pass::VERT: nb = launch_vertex(ps.vert, ps.bs, st); break;
      case Pass::PREP: nb = launch_prep(ps.prep, ps.fuse_q, ps.bs, st); break;
      case Pass::EDGE:
        nb = ps.edge_fast ? launch_edge_fast(ps.edge, ps.edge.seg[0].slow != nullptr, ps.bs, st)
                          : launch_edge(ps.edge, drag, wind, ps.bs, st, ps.edge_cells);
        break;
      case Pass::PRED: launch_predict(ps.pred, st); break;
      case Pass::ASM: launch_assemble(ps.asmb, st); break;
      case Pass::RK4FIN:
        for (auto& t : ps.fin) launch_axpy_final(std::get<0>(t), std::get<1>(t), ps.fin_c, std::get<2>(t), st);
        break;
      case Pass::COPY: launch_copy(ps.cdst, ps.csrc, ps.cn, st); break;
      case Pass::WIND:
        for (const CycloneArgs& a : ps.cycs) launch_cyclone(a, st);
        break;
      case Pass::TICK:
        for (long long* c : ps.clocks) launch_clock_tick(c, st);
        break;
    }
    if (evp.first) {
      arm_launch_events(nullptr, nullptr);
      if (nb == 0) tm->unget(cls);   // empty range: nothing was launched or recorded
    }
  }
  hip_check(hipGetLastError(), "kernel launch");
}

void run_passes(const std::vector<Pass>& passes, bool drag, bool wind, hipStream_t st, Timing* tm) {
  run_pass_range(passes.data(), passes.data() + passes.size(), drag, wind, st, tm);
}

// The step program in persistent form: maximal runs of consecutive passes
// that the persistent kernel can run, each one cooperative launch (grid-wide
// barriers between its passes), and the other passes (forcing, the RK4
// combination) launched on their own in between.
struct PersistProg {
  struct Item {
    int first = 0, count = 0;   // passes [first, first + count)
    bool coop = false;
    int desc = 0, grid = 0;     // first descriptor and grid of a cooperative run
  };
  std::vector<Item> items;
  DevBuf desc, bar;             // descriptors; barrier counters + abort flag
  uint64_t version = ~0ull;     // the pass list it was built from
  int per_cu = 0;               // and the blocks per compute unit
  void reset() { version = ~0ull; }
};

void build_persist(const std::vector<Pass>& passes, bool drag, bool wind, int per_cu, PersistProg& pp,
                   hipStream_t st) {
  hipError_t err = hipSuccess;
  const int gmax = persistent_grid(per_cu, &err);
  hip_check(err, "cooperative launch occupancy");
  if (gmax < 8) throw Err(FBLTS_EDEVICE, "the persistent kernel cannot keep 8 blocks resident");
  std::vector<PassDesc> host;
  pp.items.clear();
  for (size_t i = 0; i < passes.size(); ++i) {
    const Pass& p = passes[i];
    PassDesc d;
    bool ok = false;
    switch (p.kind) {
      case Pass::CELL: ok = desc_cell(d, p.cell, p.cell_mode); break;
      case Pass::VERT: ok = desc_vert(d, p.vert); break;
      case Pass::PREP: ok = desc_prep(d, p.prep, p.fuse_q); break;
      case Pass::EDGE: ok = desc_edge(d, p.edge, drag, wind, p.edge_fast, p.edge_cells); break;
      case Pass::PRED: ok = desc_pred(d, p.pred); break;
      case Pass::ASM: ok = desc_asm(d, p.asmb); break;
      default: break;
    }
    if (!ok) {
      PersistProg::Item it;
      it.first = (int)i;
      it.count = 1;
      pp.items.push_back(it);
      continue;
    }
    if (pp.items.empty() || !pp.items.back().coop) {
      PersistProg::Item it;
      it.first = (int)i;
      it.coop = true;
      it.desc = (int)host.size();
      it.grid = 8;
      pp.items.push_back(it);
    }
    PersistProg::Item& it = pp.items.back();
    ++it.count;
    it.grid = std::min(gmax, std::max(it.grid, (d.nvb + 7) / 8 * 8));
    host.push_back(d);
  }
  if (!host.empty()) {
    pp.desc.alloc(host.size() * sizeof(PassDesc));
    hip_check(hipMemcpyAsync(pp.desc.p, host.data(), host.size() * sizeof(PassDesc), hipMemcpyHostToDevice, st),
              "hipMemcpyAsync");
  }
  if (!pp.bar.p) {
    pp.bar.alloc(kBarWords * sizeof(unsigned) + 64);
    hip_check(hipMemsetAsync(pp.bar.p, 0, kBarWords * sizeof(unsigned) + 64, st), "hipMemsetAsync");
  }
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

void run_persist(const std::vector<Pass>& passes, const PersistProg& pp, bool drag, bool wind, hipStream_t st) {
  GridBar B;
  B.ctr = static_cast<unsigned*>(pp.bar.p);
  B.abort = reinterpret_cast<int*>(static_cast<char*>(pp.bar.p) + kBarWords * sizeof(unsigned));
  for (const PersistProg::Item& it : pp.items) {
    if (it.coop)
      hip_check(launch_persistent(pp.desc.as<PassDesc>() + it.desc, it.count, it.grid, B, st),
                "hipLaunchCooperativeKernel");
    else
      run_pass_range(passes.data() + it.first, passes.data() + it.first + it.count, drag, wind, st, nullptr);
  }
}

// A grid barrier that gave up (the launch could not keep its blocks
// resident) leaves results that are invalid: report it, and clear the
// counters for the next launch.
void check_persist(PersistProg& pp, hipStream_t st) {
  if (!pp.bar.p) return;
  int abort_flag = 0;
  hip_check(hipMemcpyAsync(&abort_flag, static_cast<char*>(pp.bar.p) + kBarWords * sizeof(unsigned), sizeof(int),
                           hipMemcpyDeviceToHost, st),
            "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (abort_flag) {
    hip_check(hipMemsetAsync(pp.bar.p, 0, kBarWords * sizeof(unsigned) + 64, st), "hipMemsetAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    throw Err(FBLTS_EDEVICE, "a grid barrier of the persistent launch gave up waiting: the state is invalid");
  }
}

}  // namespace

// ------------------------------------------------------------------ adjoint
//
// Reverse mode of the FB-LTS step (paper Section 2.2) in definition mode: the
// recording forward evaluates the coarse advancement on every cell and edge
// (so every primal value the transposed operators read is valid), the fine
// substeps as usual, and snapshots the stage arrays into a per-step tape.  The
// reverse sweep then walks the step backwards, statement by statement, using
// the transposed tendency kernels.  Checkpoints of (h, u) every K steps bound
// the tape to K steps.

namespace fblts {
void launch_lincomb_batch(const LinBatch& B, hipStream_t st);
void launch_lincomb(double* y, double b, const double* x0, double a0, const double* x1, double a1, const double* x2,
                    double a2, int begin, int end, hipStream_t st);
void launch_psi_vjp(const MeshDev& m, int linear, const double* u, const double* h, const double* pb, double* ub,
                    double* T, const PsiRange& r, hipStream_t st);
void launch_psi_vjp_cells(const MeshDev& m, int n_c, const double* T, double* hb, const LinBatch& B,
                          hipStream_t st);
void launch_phi_vjp(const MeshDev& m, int linear, int drag, double g, const double* u, const double* hs,
                    double* P, const double* cd, const double* fb, double* ub, double* hsb, double* G, double* R,
                    double* HD, double* CDB, double* HE, double* QB, double* BB, double* ZA, double* HV,
                    const VjpRange& r, hipStream_t st);
void launch_phi_vjp_ec(const MeshDev& m, int n_e, int n_c, int drag, const double* ZA, const double* HE,
                       const double* HV, const double* CDB, double* ub, double* hsb, double* cdb, const LinBatch& B,
                       hipStream_t st);
}  // namespace fblts

namespace {

enum CellArr { hNb, hb, h1b, h2b, h3b, H0b, H1b, H2b, H3b, ahb, pb, hsb, hspt, BBa, cdb, kNCellArr };
enum EdgeArr { uNb, ub, u1b, u2b, u3b, U0b, U1b, U2b, U3Fb, aub, fb, Ta, Ga, Ra, HDa, CDBa, HEa, QBa, kNEdgeArr };

}  // namespace

struct AdjointState {
  int n_steps = 0, ckpt_every = 0, M = 0;
  bool recorded = false;
  uint64_t gen = 0;   // the solver's generation the recording belongs to
  Plan plan_full;
  size_t tape_c = 0, tape_e = 0;   // doubles per step of the cell / edge tape
  DevBuf ckpt, final_state, step_tape, seg_tape;
  DevBuf cells, edges, verts, Pf;
  std::vector<Pass> rec;
};

namespace {

struct Rev {
  // views of one solver's arrays for the reverse sweep
  const MeshDev* m;
  int N, E, V, nF, if1e, if2e, nFE, if1ee, if2ee, M;
  double dt, b1, b2, b3, g;
  bool linear, drag;
  const double* cd;
  double* C[kNCellArr];
  double* Ed[kNEdgeArr];
  double* ZA;
  double* HV;
  double* P;
  hipStream_t st;
  // transpose ranges: the whole mesh (coarse stages), and the fine stages'
  // cotangent supports (stages 1-2: fine rows; stage 3: with the interfaces)
  VjpRange phi_all, phi_f12, phi_f3;
  PsiRange psi_all, psi_f12, psi_f3;
  // Inside a reverse step the elementwise combinations between two tendency
  // transposes are collected and launched as one batch (same arithmetic per
  // element, in the same order); elsewhere each launches at once.  The last
  // kernel of a transpose (Psi's cell pass, Phi's passes 5-6) waits for the
  // next flush, which hands it the collected batch as an epilogue (thread i
  // applies the batch at index i after its own item) when no combination
  // writes an array that kernel reads at other indices or reads or writes
  // one it writes from another thread; otherwise the batch follows it.
  bool batching = false;
  LinBatch pending;
  struct Tail {
    int kind = 0;   // 0 none, 1 Psi cell pass, 2 Phi passes 5-6
    int n_e = 0, n_c = 0;
    const double* T = nullptr;   // Psi: gathered
    double* hb = nullptr;        // Psi: written by thread i at index i
    // Phi: ZA, HE, HV, CDB gathered; hsb, cdb written by thread i at index i
    // (cells first); ub written by thread n_c + e at index e
    const double *ZA = nullptr, *HE = nullptr, *HV = nullptr, *CDB = nullptr;
    double *ub = nullptr, *hsb = nullptr, *cdb = nullptr;
  } tail;
  bool foldable() const {
    const void* gathered[4] = {tail.T, nullptr, nullptr, nullptr};
    const void* other = nullptr;   // written from another thread than its index
    if (tail.kind == 2) {
      gathered[0] = tail.ZA;
      gathered[1] = tail.HE;
      gathered[2] = tail.HV;
      gathered[3] = tail.CDB;
      other = tail.ub;
    }
    auto in = [&](const void* p) {
      if (!p) return false;
      for (const void* q : gathered)
        if (q == p) return true;
      return p == other;
    };
    for (int k = 0; k < pending.n; ++k) {
      const LinDesc& d = pending.d[k];
      if (in(d.y)) return false;
      for (const void* x : {(const void*)d.x0, (const void*)d.x1, (const void*)d.x2})
        if (x && x == other) return false;
    }
    return true;
  }
  void launch_tail(const LinBatch& B) {
    if (tail.kind == 1) launch_psi_vjp_cells(*m, tail.n_c, tail.T, tail.hb, B, st);
    else launch_phi_vjp_ec(*m, tail.n_e, tail.n_c, drag ? 1 : 0, tail.ZA, tail.HE, tail.HV, tail.CDB, tail.ub,
                           tail.hsb, tail.cdb, B, st);
    tail.kind = 0;
  }
  void flush() {
    if (tail.kind != 0) {
      if (pending.n > 0 && foldable()) {
        launch_tail(pending);
        pending.n = 0;
        pending.end_max = 0;
        return;
      }
      launch_tail(LinBatch{});
    }
    launch_lincomb_batch(pending, st);
    pending.n = 0;
    pending.end_max = 0;
  }
  void lin(double* y, double b, const double* x0, double a0, const double* x1, double a1, const double* x2, double a2,
           int lo, int hi) {
    if (hi <= lo) return;
    if (!batching) {
      launch_lincomb(y, b, x0, a0, x1, a1, x2, a2, lo, hi, st);
      return;
    }
    if (pending.n == kLinBatch) flush();
    pending.d[pending.n++] = LinDesc{y, x0, x1, x2, b, a0, a1, a2, lo, hi};
    pending.end_max = std::max(pending.end_max, hi);
  }
  void zero(double* y, int lo, int hi) { lin(y, 0.0, nullptr, 0, nullptr, 0, nullptr, 0, lo, hi); }
  void set(double* y, double a, const double* x, int lo, int hi) { lin(y, 0.0, x, a, nullptr, 0, nullptr, 0, lo, hi); }
  void axpy(double* y, double a, const double* x, int lo, int hi) { lin(y, 1.0, x, a, nullptr, 0, nullptr, 0, lo, hi); }
  // cotangent pbar of Psi(u, h) (zero past the range's support) -> ubar, hbar (accumulated)
  void psi_vjp(const double* u, const double* h, const double* pbar, double* ubar, double* hbar,
               const PsiRange& r) {
    zero(Ed[Ta], r.ne, r.zT);
    flush();
    launch_psi_vjp(*m, linear ? 1 : 0, u, h, pbar, ubar, Ed[Ta], r, st);
    if (!linear && r.nc > 0) {
      tail = Tail{};
      tail.kind = 1;
      tail.n_c = r.nc;
      tail.T = Ed[Ta];
      tail.hb = hbar;
      if (!batching) flush();
    }
  }
  // cotangent fbar of Phi(u, hs) (zero past the range's support) -> ubar
  // (accumulated), hsbar (overwritten), C_D (accumulated)
  void phi_vjp(const double* u, const double* hs, const double* fbar, double* ubar, double* hsbar,
               const VjpRange& r) {
    zero(hsbar, 0, N);
    zero(Ed[Ga], r.e1, r.zG);
    zero(Ed[Ra], r.e1, r.zR);
    zero(Ed[HDa], r.e1, r.zHD);
    zero(Ed[CDBa], r.e1, r.zCDB);
    zero(C[BBa], r.c1, r.zBB);
    zero(Ed[QBa], r.e2, r.zQB);
    zero(Ed[HEa], r.e2, r.zHE);
    zero(ZA, r.v1, r.zZA);
    zero(HV, r.v1, r.zHV);
    flush();
    // the first launch also writes the forward intermediates at the point:
    // the edge records the later passes read (q_v evaluated inside)
    launch_phi_vjp(*m, linear ? 1 : 0, drag ? 1 : 0, g, u, hs, P, cd, fbar, ubar, hsbar, Ed[Ga], Ed[Ra], Ed[HDa],
                   Ed[CDBa], Ed[HEa], Ed[QBa], C[BBa], ZA, HV, r, st);
    if (!linear && r.e3 + r.c3 > 0) {
      tail = Tail{};
      tail.kind = 2;
      tail.n_e = r.e3;
      tail.n_c = r.c3;
      tail.ZA = ZA;
      tail.HE = Ed[HEa];
      tail.HV = HV;
      tail.CDB = Ed[CDBa];
      tail.ub = ubar;
      tail.hsb = hsbar;
      tail.cdb = C[cdb];
      if (!batching) flush();
    }
  }
  // One reverse step: (hNb, uNb) = cotangent of the step's output -> (hb, ub)
  // = cotangent of its input; C_D's cotangent accumulates.  tc / te: tape.
  void step(const double* tc, const double* te) {
    auto TC = [&](int slot) { return tc + (size_t)slot * N; };
    auto TE = [&](int slot) { return te + (size_t)slot * E; };
    const double* h = TC(0);
    const double* h1 = TC(1);
    const double* h2 = TC(2);
    const double* h3 = TC(3);
    const double* u = TE(0);
    const double* u1 = TE(1);
    const double* u2 = TE(2);
    double** c = C;
    double** e = Ed;
    batching = true;
    for (int k : {hb, h1b, h2b, h3b, H0b, H1b, H2b, H3b, ahb}) zero(c[k], 0, N);
    for (int k : {ub, u1b, u2b, u3b, U0b, U1b, U2b, U3Fb, aub}) zero(e[k], 0, E);
    const double delta = dt / M;
    // assembly: h^{n+1} = h3 (interior), H0 (fine), h + delta acc_h (interface)
    set(c[h3b], 1.0, c[hNb], if2e, N);
    set(c[H0b], 1.0, c[hNb], 0, nF);
    set(c[hb], 1.0, c[hNb], nF, if2e);
    set(c[ahb], delta, c[hNb], nF, if2e);
    set(e[u3b], 1.0, e[uNb], if2ee, E);
    set(e[U0b], 1.0, e[uNb], 0, nFE);
    set(e[ub], 1.0, e[uNb], nFE, if2ee);
    set(e[aub], delta, e[uNb], nFE, if2ee);
    for (int k = M - 1; k >= 0; --k) {
      const double* H0k = TC(4 + 4 * k);
      const double* H1k = TC(5 + 4 * k);
      const double* H2k = TC(6 + 4 * k);
      const double* H3k = TC(7 + 4 * k);
      const double* U0k = TE(4 + 3 * k);
      const double* U1k = TE(5 + 3 * k);
      const double* U2k = TE(6 + 3 * k);
      // H0[F] <- H3[F]; U0[Fe] <- U3F[Fe]
      axpy(c[H3b], 1.0, c[H0b], 0, nF);
      zero(c[H0b], 0, nF);
      set(e[U3Fb], 1.0, e[U0b], 0, nFE);
      zero(e[U0b], 0, nFE);
      // stage 3, momentum: U3F = U0 + delta Phi(U2, hs3) on Fe; acc_u += Phi on IFe
      zero(e[fb], 0, E);
      set(e[fb], delta, e[U3Fb], 0, nFE);
      set(e[fb], 1.0, e[aub], nFE, if2ee);
      axpy(e[U0b], 1.0, e[U3Fb], 0, nFE);
      lin(c[hspt], 0.0, H3k, b3, H2k, 1.0 - 2.0 * b3, H0k, b3, 0, N);
      phi_vjp(U2k, c[hspt], e[fb], e[U2b], c[hsb], phi_f3);
      lin(c[H3b], 1.0, c[hsb], b3, nullptr, 0, nullptr, 0, 0, N);
      lin(c[H2b], 1.0, c[hsb], 1.0 - 2.0 * b3, nullptr, 0, nullptr, 0, 0, N);
      lin(c[H0b], 1.0, c[hsb], b3, nullptr, 0, nullptr, 0, 0, N);
      // stage 3, thickness: H3[F] = H0 + delta Psi(U2, H2); acc_h += Psi on IF
      zero(c[pb], 0, N);
      set(c[pb], delta, c[H3b], 0, nF);
      set(c[pb], 1.0, c[ahb], nF, if2e);
      axpy(c[H0b], 1.0, c[H3b], 0, nF);
      zero(c[H3b], 0, nF);
      psi_vjp(U2k, H2k, c[pb], e[U2b], c[H2b], psi_f3);
      // stage 2, momentum: U2[Fe] = U0 + delta/2 Phi(U1, hs2)
      zero(e[fb], 0, E);
      set(e[fb], delta / 2, e[U2b], 0, nFE);
      axpy(e[U0b], 1.0, e[U2b], 0, nFE);
      zero(e[U2b], 0, nFE);
      lin(c[hspt], 0.0, H2k, b2, H0k, 1.0 - b2, nullptr, 0, 0, N);
      phi_vjp(U1k, c[hspt], e[fb], e[U1b], c[hsb], phi_f12);
      lin(c[H2b], 1.0, c[hsb], b2, nullptr, 0, nullptr, 0, 0, N);
      lin(c[H0b], 1.0, c[hsb], 1.0 - b2, nullptr, 0, nullptr, 0, 0, N);
      // stage 2, thickness: H2[F] = H0 + delta/2 Psi(U1, H1)
      zero(c[pb], 0, N);
      set(c[pb], delta / 2, c[H2b], 0, nF);
      axpy(c[H0b], 1.0, c[H2b], 0, nF);
      zero(c[H2b], 0, nF);
      psi_vjp(U1k, H1k, c[pb], e[U1b], c[H1b], psi_f12);
      // stage 1, momentum: U1[Fe] = U0 + delta/3 Phi(U0, hs1)
      zero(e[fb], 0, E);
      set(e[fb], delta / 3, e[U1b], 0, nFE);
      axpy(e[U0b], 1.0, e[U1b], 0, nFE);
      zero(e[U1b], 0, nFE);
      lin(c[hspt], 0.0, H1k, b1, H0k, 1.0 - b1, nullptr, 0, 0, N);
      phi_vjp(U0k, c[hspt], e[fb], e[U0b], c[hsb], phi_f12);
      lin(c[H1b], 1.0, c[hsb], b1, nullptr, 0, nullptr, 0, 0, N);
      lin(c[H0b], 1.0, c[hsb], 1.0 - b1, nullptr, 0, nullptr, 0, 0, N);
      // stage 1, thickness: H1[F] = H0 + delta/3 Psi(U0, H0)
      zero(c[pb], 0, N);
      set(c[pb], delta / 3, c[H1b], 0, nF);
      axpy(c[H0b], 1.0, c[H1b], 0, nF);
      zero(c[H1b], 0, nF);
      psi_vjp(U0k, H0k, c[pb], e[U0b], c[H0b], psi_f12);
      // interface-one prediction (eq. preds) of substep k
      const double a = (double)k / (double)M, oma = (double)(M - k) / (double)M;
      const double cc = (double)(M - k - 1) / (double)M, ap = (double)(k + 1) / (double)M, iM = 1.0 / M;
      lin(c[h3b], 1.0, c[H0b], a, c[H1b], a, c[H2b], a, nF, if1e);
      lin(c[h3b], 1.0, c[H3b], ap, nullptr, 0, nullptr, 0, nF, if1e);
      lin(c[hb], 1.0, c[H0b], oma, c[H1b], cc, c[H2b], cc, nF, if1e);
      lin(c[hb], 1.0, c[H3b], cc, nullptr, 0, nullptr, 0, nF, if1e);
      axpy(c[h1b], iM, c[H1b], nF, if1e);
      axpy(c[h2b], iM, c[H2b], nF, if1e);
      for (int q : {H0b, H1b, H2b, H3b}) zero(c[q], nF, if1e);
      lin(e[u3b], 1.0, e[U0b], a, e[U1b], a, e[U2b], a, nFE, if1ee);
      lin(e[ub], 1.0, e[U0b], oma, e[U1b], cc, e[U2b], cc, nFE, if1ee);
      axpy(e[u1b], iM, e[U1b], nFE, if1ee);
      axpy(e[u2b], iM, e[U2b], nFE, if1ee);
      for (int q : {U0b, U1b, U2b}) zero(e[q], nFE, if1ee);
    }
    // the fine arrays start as copies of the coarse stage values
    axpy(c[hb], 1.0, c[H0b], 0, N);
    axpy(c[h1b], 1.0, c[H1b], 0, N);
    axpy(c[h2b], 1.0, c[H2b], 0, N);
    axpy(c[h3b], 1.0, c[H3b], 0, N);
    axpy(e[ub], 1.0, e[U0b], 0, E);
    axpy(e[u1b], 1.0, e[U1b], 0, E);
    axpy(e[u2b], 1.0, e[U2b], 0, E);
    // coarse advancement (eq. fbrk32), stage 3 to 1
    axpy(e[ub], 1.0, e[u3b], 0, E);
    set(e[fb], dt, e[u3b], 0, E);
    lin(c[hspt], 0.0, h3, b3, h2, 1.0 - 2.0 * b3, h, b3, 0, N);
    phi_vjp(u2, c[hspt], e[fb], e[u2b], c[hsb], phi_all);
    lin(c[h3b], 1.0, c[hsb], b3, nullptr, 0, nullptr, 0, 0, N);
    lin(c[h2b], 1.0, c[hsb], 1.0 - 2.0 * b3, nullptr, 0, nullptr, 0, 0, N);
    lin(c[hb], 1.0, c[hsb], b3, nullptr, 0, nullptr, 0, 0, N);
    axpy(c[hb], 1.0, c[h3b], 0, N);
    set(c[pb], dt, c[h3b], 0, N);
    psi_vjp(u2, h2, c[pb], e[u2b], c[h2b], psi_all);
    axpy(e[ub], 1.0, e[u2b], 0, E);
    set(e[fb], dt / 2, e[u2b], 0, E);
    lin(c[hspt], 0.0, h2, b2, h, 1.0 - b2, nullptr, 0, 0, N);
    phi_vjp(u1, c[hspt], e[fb], e[u1b], c[hsb], phi_all);
    lin(c[h2b], 1.0, c[hsb], b2, nullptr, 0, nullptr, 0, 0, N);
    lin(c[hb], 1.0, c[hsb], 1.0 - b2, nullptr, 0, nullptr, 0, 0, N);
    axpy(c[hb], 1.0, c[h2b], 0, N);
    set(c[pb], dt / 2, c[h2b], 0, N);
    psi_vjp(u1, h1, c[pb], e[u1b], c[h1b], psi_all);
    axpy(e[ub], 1.0, e[u1b], 0, E);
    set(e[fb], dt / 3, e[u1b], 0, E);
    lin(c[hspt], 0.0, h1, b1, h, 1.0 - b1, nullptr, 0, 0, N);
    phi_vjp(u, c[hspt], e[fb], e[ub], c[hsb], phi_all);
    lin(c[h1b], 1.0, c[hsb], b1, nullptr, 0, nullptr, 0, 0, N);
    lin(c[hb], 1.0, c[hsb], 1.0 - b1, nullptr, 0, nullptr, 0, 0, N);
    axpy(c[hb], 1.0, c[h1b], 0, N);
    set(c[pb], dt / 3, c[h1b], 0, N);
    psi_vjp(u, h, c[pb], e[ub], c[hb], psi_all);
    flush();
    batching = false;
  }
};

}  // namespace

// ------------------------------------------------------------------ objects

// The step program captured as hipGraphs: one coarse step, and `G` coarse
// steps back to back (each graph launch has a fixed cost at its boundary, so
// longer runs replay the G-step graph and finish with single steps).
struct StepGraphs {
  hipGraph_t g1 = nullptr, gG = nullptr;
  hipGraphExec_t x1 = nullptr, xG = nullptr;
  int G = 0;
  StepGraphs() = default;
  StepGraphs(const StepGraphs&) = delete;
  StepGraphs& operator=(const StepGraphs&) = delete;
  ~StepGraphs() { reset(); }
  void reset() {
    if (x1) (void)hipGraphExecDestroy(x1);
    if (g1) (void)hipGraphDestroy(g1);
    if (xG) (void)hipGraphExecDestroy(xG);
    if (gG) (void)hipGraphDestroy(gG);
    x1 = xG = nullptr;
    g1 = gG = nullptr;
    G = 0;
  }
  template <class F>
  static void capture(hipStream_t st, int steps, F&& run_one, hipGraph_t& g, hipGraphExec_t& x) {
    hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
      for (int k = 0; k < steps; ++k) run_one();
    } catch (...) {
      hipGraph_t bad = nullptr;
      (void)hipStreamEndCapture(st, &bad);
      if (bad) (void)hipGraphDestroy(bad);
      throw;
    }
    hip_check(hipStreamEndCapture(st, &g), "hipStreamEndCapture");
    hip_check(hipGraphInstantiate(&x, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  }
  // replay n coarse steps, capturing first when needed
  template <class F>
  void run(hipStream_t st, int n, int steps_per_graph, F&& run_one) {
    if (!x1 || G != steps_per_graph) {
      reset();
      capture(st, 1, run_one, g1, x1);
      if (steps_per_graph > 1) capture(st, steps_per_graph, run_one, gG, xG);
      G = steps_per_graph;
    }
    int k = 0;
    if (G > 1)
      for (; k + G <= n; k += G) hip_check(hipGraphLaunch(xG, st), "hipGraphLaunch");
    for (; k < n; ++k) hip_check(hipGraphLaunch(x1, st), "hipGraphLaunch");
  }
};

struct fblts_mesh {
  HostMesh hm;
};

struct fblts_solver {
  const fblts_mesh* mesh = nullptr;
  Params P;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  std::unique_ptr<MeshUnit> unit;
  bool have_regions = false, have_state = false, drag_on = false;
  LaunchOpts opt;
  bool graph_on = false;
  StepGraphs graphs;
  PersistProg persist;
  Timing timing;
  DevBuf diag_partial, diag_out;
  DevBuf stage_h, stage_u;   // caller-order staging
  DevBuf dbg_h, dbg_u, dbg_out;
  double time = 0.0;
  int64_t step = 0;
  // Generation: advanced by every call that changes the trajectory (regions,
  // state, drag, wind, storm, steps).  An adjoint recording is valid only for
  // the generation it ended in.
  uint64_t gen = 0;
  std::unique_ptr<AdjointState> adj;
  ~fblts_solver() {
    drop_graph();
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
  void drop_graph() { graphs.reset(); }
};

struct fblts_ensemble {
  Params P;
  // ensemble launches hold one segment per mesh: the sequential step
  LaunchOpts opt = [] {
    LaunchOpts o;
    o.pipeline = false;
    return o;
  }();
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<std::unique_ptr<MeshUnit>> units;
  std::vector<Pass> passes;
  uint64_t version = 0;   // advanced whenever the merged pass list is rebuilt
  bool graph_on = false;
  StepGraphs graphs;
  PersistProg persist;
  DevBuf diag_partial, diag_out, stage_h, stage_u;
  int64_t step = 0;
  ~fblts_ensemble() {
    graphs.reset();
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

// ------------------------------------------------------------------ helpers

static void setup_unit(MeshUnit& u, const HostMesh& hm, const Params& P, const int8_t* labels, bool binary, int nm) {
  u.hm = &hm;
  const bool fblts_scheme = P.p.scheme == FBLTS_SCHEME_FBLTS;
  if (fblts_scheme) {
    if (!labels) throw Err(FBLTS_EINVAL, "labels is NULL");
    layer_regions(hm, labels, binary, P.p.r_layers, u.lab4, u.layer);
  } else {
    u.lab4.assign(hm.N, 3);
    u.layer.assign(hm.N, 1 << 20);
  }
  build_plan(hm, u.lab4, u.layer, fblts_scheme, P.wide(), P.p.r_layers, u.plan);
  permute_mesh(hm, u.plan, u.pm);
  u.dm.upload_from(u.pm, u.plan);
  u.st.alloc(u.pm, u.plan, nm);
}

static void init_scratch(MeshUnit& u, hipStream_t st) {
  // every scratch array starts as a copy of the state (finite everywhere)
  const long Nc = (long)u.pm.N * u.st.nm, Ne = (long)u.pm.E * u.st.nm;
  for (int k = 1; k < 4; ++k) {
    launch_copy(u.st.H[k].as<double>(), u.st.H[0].as<double>(), Nc, st);
    launch_copy(u.st.U[k].as<double>(), u.st.U[0].as<double>(), Ne, st);
  }
  launch_copy(u.st.hs.as<double>(), u.st.H[0].as<double>(), Nc, st);
  launch_fill(u.st.B.as<double>(), 0.0, Nc, st);
  launch_fill(u.st.acc_h.as<double>(), 0.0, Nc, st);
  launch_fill(u.st.acc_u.as<double>(), 0.0, Ne, st);
  launch_fill(u.st.P.as<double>(), 0.0, Ne * 4, st);
  launch_fill(u.st.q.as<double>(), 0.0, (long)u.pm.V * u.st.nm, st);
}

static hipStream_t make_stream(void* s, bool& own) {
  if (s) {
    own = false;
    return static_cast<hipStream_t>(s);
  }
  hipStream_t st;
  hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
  own = true;
  return st;
}

static void state_in(MeshUnit& u, DevBuf& sh, DevBuf& su, const double* h, const double* uu, int member,
                     bool on_device, hipStream_t st) {
  const int N = u.pm.N, E = u.pm.E;
  const double* dh = h;
  const double* du = uu;
  if (!on_device) {
    if (sh.bytes < (size_t)N * 8) sh.alloc((size_t)N * 8);
    if (su.bytes < (size_t)E * 8) su.alloc((size_t)E * 8);
    if (h) hip_check(hipMemcpyAsync(sh.p, h, (size_t)N * 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    if (uu) hip_check(hipMemcpyAsync(su.p, uu, (size_t)E * 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    dh = sh.as<double>();
    du = su.as<double>();
  }
  if (h) launch_permute(u.st.H[0].as<double>(), dh, u.dm.cell_n2o.as<int>(), N, u.st.nm_log2, member, 1, st);
  if (uu) launch_permute(u.st.U[0].as<double>(), du, u.dm.edge_n2o.as<int>(), E, u.st.nm_log2, member, 1, st);
}

static void state_out(MeshUnit& u, DevBuf& sh, DevBuf& su, double* h, double* uu, int member, bool on_device,
                      hipStream_t st) {
  const int N = u.pm.N, E = u.pm.E;
  double* dh = h;
  double* du = uu;
  if (!on_device) {
    if (sh.bytes < (size_t)N * 8) sh.alloc((size_t)N * 8);
    if (su.bytes < (size_t)E * 8) su.alloc((size_t)E * 8);
    dh = sh.as<double>();
    du = su.as<double>();
  }
  if (h) launch_permute(dh, u.st.H[0].as<double>(), u.dm.cell_n2o.as<int>(), N, u.st.nm_log2, member, 0, st);
  if (uu) launch_permute(du, u.st.U[0].as<double>(), u.dm.edge_n2o.as<int>(), E, u.st.nm_log2, member, 0, st);
  if (!on_device) {
    if (h) hip_check(hipMemcpyAsync(h, sh.p, (size_t)N * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    if (uu) hip_check(hipMemcpyAsync(uu, su.p, (size_t)E * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  }
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

static void diag_of(MeshUnit& u, const Params& P, DevBuf& part, DevBuf& out, hipStream_t st, std::vector<double>& res) {
  const int nb = diag_blocks(u.dm.md);
  const size_t need = (size_t)kDiagQ * nb * u.st.nm * 8;
  if (part.bytes < need) part.alloc(need);
  if (out.bytes < (size_t)kDiagQ * u.st.nm * 8) out.alloc((size_t)kDiagQ * u.st.nm * 8);
  launch_diag(u.dm.md, u.st.nm_log2, P.wide() ? 0 : 1, u.st.H[0].as<double>(), u.st.U[0].as<double>(), P.p.g,
              part.as<double>(), out.as<double>(), st);
  hip_check(hipGetLastError(), "diagnostics launch");
  res.resize((size_t)kDiagQ * u.st.nm);
  hip_check(hipMemcpyAsync(res.data(), out.p, res.size() * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

// ------------------------------------------- allocation-free diagnostics
// fblts_diagnostics_noalloc keeps the reduction's per-block partial sums and
// its results in this file-scope device array instead of buffers the solver
// allocates.  Every GPU the library runs on holds its own copy until the
// process ends.  The diagnostics of a one-member solver launch at most
// kDiagMaxBlocks blocks (diag_blocks), so every solver fits.
constexpr int kDiagMaxBlocks = 1024;
constexpr size_t kScratchDoubles = (size_t)kDiagQ * kDiagMaxBlocks + kDiagQ;
static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` on each device, taken once per device with that
// device current (the array's name in host code is only a stand-in).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxDevices] = {};

static void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Err(FBLTS_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev]) return;
  void* p = nullptr;
  hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  if (!p) throw Err(FBLTS_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
  g_scratch_dev[dev] = static_cast<double*>(p);
}

static int fill_diag(const double* q, double time, int64_t step, fblts_diag* o) {
  o->mass = q[0];
  o->abs_vorticity = q[1];
  o->abs_vorticity_scale = q[2];
  o->energy = q[3] + q[4];
  o->min_h = q[5];
  o->n_nonfinite = (int64_t)q[6];
  o->time = time;
  o->step = step;
  return (q[6] > 0 || q[7] > 0) ? FBLTS_ENONFINITE : FBLTS_OK;
}

// ------------------------------------------------------------ step drivers

static void solver_run(fblts_solver* s, int n) {
  MeshUnit& u = *s->unit;
  if (s->opt.persistent && !s->timing.on) {
    // one cooperative launch per run of passes (timing launches every pass on
    // its own); the program is built before any capture
    if (s->persist.version != u.version || s->persist.per_cu != s->opt.persistent) {
      build_persist(u.passes, s->drag_on, u.st.has_wind, s->opt.persistent, s->persist, s->stream);
      s->persist.version = u.version;
      s->persist.per_cu = s->opt.persistent;
      s->drop_graph();
    }
    auto one = [&] { run_persist(u.passes, s->persist, s->drag_on, u.st.has_wind, s->stream); };
    if (s->graph_on) s->graphs.run(s->stream, n, s->opt.graph_steps, one);
    else
      for (int k = 0; k < n; ++k) one();
  } else if (s->graph_on && !s->timing.on) {
    s->graphs.run(s->stream, n, s->opt.graph_steps,
                  [&] { run_passes(u.passes, s->drag_on, u.st.has_wind, s->stream, nullptr); });
  } else {
    if (s->timing.on) s->timing.reset();
    for (int k = 0; k < n; ++k) run_passes(u.passes, s->drag_on, u.st.has_wind, s->stream, &s->timing);
  }
  s->step += n;
  s->time += n * s->P.p.dt;
  ++s->gen;
}

static void ensemble_run(fblts_ensemble* e, int n) {
  const bool nl = e->P.nonlinear();
  if (e->opt.persistent) {
    if (e->persist.version != e->version || e->persist.per_cu != e->opt.persistent) {
      build_persist(e->passes, nl, e->units[0]->st.has_wind, e->opt.persistent, e->persist, e->stream);
      e->persist.version = e->version;
      e->persist.per_cu = e->opt.persistent;
      e->graphs.reset();
    }
    auto one = [&] { run_persist(e->passes, e->persist, nl, e->units[0]->st.has_wind, e->stream); };
    if (e->graph_on) e->graphs.run(e->stream, n, e->opt.graph_steps, one);
    else
      for (int k = 0; k < n; ++k) one();
  } else if (e->graph_on) {
    e->graphs.run(e->stream, n, e->opt.graph_steps,
                  [&] { run_passes(e->passes, nl, e->units[0]->st.has_wind, e->stream, nullptr); });
  } else {
    for (int k = 0; k < n; ++k) run_passes(e->passes, nl, e->units[0]->st.has_wind, e->stream, nullptr);
  }
  e->step += n;
}

// Rebuild the pass lists after a change of launch options (drops the graphs).
static void solver_rebuild(fblts_solver* s) {
  s->drop_graph();
  if (s->have_regions) build_passes(*s->unit, s->P, s->drag_on, s->opt, s->stream);
}

static void ensemble_rebuild(fblts_ensemble* e) {
  std::vector<MeshUnit*> units;
  for (auto& u : e->units) {
    build_passes(*u, e->P, e->P.nonlinear(), e->opt, e->stream);
    units.push_back(u.get());
  }
  e->passes = merge_passes(units);
  ++e->version;
  e->graphs.reset();
}

// ------------------------------------------------------------- autotuning
// Everything a coarse step changes besides the counters, per mesh unit: the
// state, and with a moving storm its step clock and the wind it evaluated.
struct SnapUnit {
  DevBuf h, u, wn, wt, wc;
  long long clock = 0;
  bool cyclone = false;
};

static std::vector<std::unique_ptr<SnapUnit>> snapshot_take(const std::vector<MeshUnit*>& units, hipStream_t st) {
  std::vector<std::unique_ptr<SnapUnit>> snap;
  for (MeshUnit* u : units) {
    auto q = std::make_unique<SnapUnit>();
    const long Nc = (long)u->pm.N * u->st.nm, Ne = (long)u->pm.E * u->st.nm;
    q->h.alloc((size_t)Nc * 8);
    q->u.alloc((size_t)Ne * 8);
    launch_copy(q->h.as<double>(), u->st.H[0].as<double>(), Nc, st);
    launch_copy(q->u.as<double>(), u->st.U[0].as<double>(), Ne, st);
    if (u->st.cyclone) {
      q->cyclone = true;
      q->wn.alloc((size_t)Ne * 8);
      q->wt.alloc((size_t)Ne * 8);
      q->wc.alloc((size_t)Ne * 8);
      launch_copy(q->wn.as<double>(), u->st.wind_n.as<double>(), Ne, st);
      launch_copy(q->wt.as<double>(), u->st.wind_t.as<double>(), Ne, st);
      launch_copy(q->wc.as<double>(), u->st.wind_c.as<double>(), Ne, st);
      hip_check(hipMemcpyAsync(&q->clock, u->st.cyc_clock.p, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    }
    snap.push_back(std::move(q));
  }
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  return snap;
}

static void snapshot_restore(const std::vector<MeshUnit*>& units, const std::vector<std::unique_ptr<SnapUnit>>& snap,
                             hipStream_t st) {
  for (size_t k = 0; k < units.size(); ++k) {
    MeshUnit& u = *units[k];
    const SnapUnit& q = *snap[k];
    const long Nc = (long)u.pm.N * u.st.nm, Ne = (long)u.pm.E * u.st.nm;
    launch_copy(u.st.H[0].as<double>(), q.h.as<double>(), Nc, st);
    launch_copy(u.st.U[0].as<double>(), q.u.as<double>(), Ne, st);
    init_scratch(u, st);
    if (q.cyclone) {
      launch_copy(u.st.wind_n.as<double>(), q.wn.as<double>(), Ne, st);
      launch_copy(u.st.wind_t.as<double>(), q.wt.as<double>(), Ne, st);
      launch_copy(u.st.wind_c.as<double>(), q.wc.as<double>(), Ne, st);
      hip_check(hipMemcpyAsync(u.st.cyc_clock.p, &q.clock, 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    }
  }
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

struct Schedule {
  int fuse = 1, block = kBlock, cells = 0;
  double ms = 0.0;
  int persistent = 0;
};
using ScheduleCache = std::vector<std::pair<std::string, Schedule>>;

static std::string trim(const char* c) {
  std::string s(c);
  const size_t a = s.find_first_not_of(" \t\r\n");
  if (a == std::string::npos) return std::string();
  const size_t b = s.find_last_not_of(" \t\r\n");
  return s.substr(a, b - a + 1);
}

// The schedule cache is a JSON object with one workload per line,
//   "<key>": {"fuse_vertex": F, "block": B, "edge_cells": C, "ms_per_step": T}
// and is read and written only in that form.
static ScheduleCache cache_read(const char* path) {
  ScheduleCache v;
  std::FILE* f = std::fopen(path, "r");
  if (!f) return v;  // no cache yet
  char buf[1024];
  bool ok = true;
  while (ok && std::fgets(buf, sizeof buf, f)) {
    std::string s = trim(buf);
    if (s.empty() || s == "{" || s == "}") continue;
    if (s.back() == ',') s.pop_back();
    const size_t q = (s.size() > 1 && s[0] == '"') ? s.find('"', 1) : std::string::npos;
    Schedule t;
    int end = 0;
    ok = q != std::string::npos &&
         std::sscanf(s.c_str() + q + 1,
                     " : {\"fuse_vertex\": %d, \"block\": %d, \"edge_cells\": %d, \"persistent\": %d, "
                     "\"ms_per_step\": %lf }%n",
                     &t.fuse, &t.block, &t.cells, &t.persistent, &t.ms, &end) == 5 &&
         end > 0 && s.c_str()[q + 1 + end] == '\0' && (t.fuse == 0 || t.fuse == 1) &&
         (t.block == 64 || t.block == 128 || t.block == 256) && (t.cells == 0 || t.cells == 1) &&
         t.persistent >= 0 && t.persistent <= 16 && std::isfinite(t.ms) && t.ms >= 0.0;
    if (ok) v.emplace_back(s.substr(1, q - 1), t);
  }
  std::fclose(f);
  if (!ok) throw Err(FBLTS_EINVAL, std::string("autotune cache ") + path + " is not a schedule cache of this library");
  return v;
}

static void cache_write(const char* path, const ScheduleCache& v) {
  const std::string tmp = std::string(path) + ".tmp";
  std::FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) throw Err(FBLTS_EINVAL, "autotune cache: cannot write " + tmp);
  std::fprintf(f, "{\n");
  for (size_t k = 0; k < v.size(); ++k) {
    const Schedule& t = v[k].second;
    std::fprintf(f,
                 "\"%s\": {\"fuse_vertex\": %d, \"block\": %d, \"edge_cells\": %d, \"persistent\": %d, "
                 "\"ms_per_step\": %.6f}%s\n",
                 v[k].first.c_str(), t.fuse, t.block, t.cells, t.persistent, t.ms, k + 1 < v.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  const bool closed = std::fclose(f) == 0;
  if (!closed || std::rename(tmp.c_str(), path) != 0) throw Err(FBLTS_EINVAL, std::string("autotune cache: cannot write ") + path);
}

// Workload keys: everything that changes the pass program or its sizes.
static int wind_kind(const MeshUnit& u) { return u.st.cyclone ? 2 : (u.st.has_wind ? 1 : 0); }

static std::string solver_key(const fblts_solver& s) {
  const MeshUnit& u = *s.unit;
  char b[256];
  std::snprintf(b, sizeof b, "solver:N%d:E%d:F%d:IF%d:scheme%d:M%d:phys%d:split%d:drag%d:wind%d:G%d", u.pm.N, u.pm.E,
                u.plan.nF, u.plan.nIF1, s.P.p.scheme, s.P.p.M, s.P.p.physics, s.P.p.split, s.drag_on ? 1 : 0,
                wind_kind(u), s.opt.graph_steps);
  return b;
}

static std::string ensemble_key(const fblts_ensemble& e) {
  std::string k = "ensemble";
  char b[160];
  for (const auto& u : e.units) {
    std::snprintf(b, sizeof b, ":N%dF%dm%d", u->pm.N, u->plan.nF, u->st.nm);
    k += b;
  }
  std::snprintf(b, sizeof b, ":scheme%d:M%d:phys%d:split%d:wind%d:G%d", e.P.p.scheme, e.P.p.M, e.P.p.physics,
                e.P.p.split, wind_kind(*e.units[0]), e.opt.graph_steps);
  return k + b;
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    hip_check(hipEventCreate(&a), "hipEventCreate");
    hip_check(hipEventCreate(&b), "hipEventCreate");
  }
  EventPair(const EventPair&) = delete;
  EventPair& operator=(const EventPair&) = delete;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Two warm-up steps (they capture the graphs), then `repeats` runs of `steps`
// steps between stream events; the best run's time per step in ms.
template <class Run>
static double time_schedule(hipStream_t st, int steps, int repeats, Run&& run) {
  run(2);
  hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
  EventPair ev;
  double best = std::numeric_limits<double>::infinity();
  for (int r = 0; r < repeats; ++r) {
    hip_check(hipEventRecord(ev.a, st), "hipEventRecord");
    run(steps);
    hip_check(hipEventRecord(ev.b, st), "hipEventRecord");
    hip_check(hipEventSynchronize(ev.b), "hipEventSynchronize");
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, ev.a, ev.b), "hipEventElapsedTime");
    best = std::min(best, (double)ms / steps);
  }
  return best;
}

// ------------------------------------------------------------------- C ABI

extern "C" {

const char* fblts_last_error(void) { return g_err.c_str(); }
int fblts_version(void) { return 100; }

int fblts_mesh_create(const fblts_mesh_desc* desc, fblts_mesh** out) {
  return guarded([&] {
    if (!out) throw Err(FBLTS_EINVAL, "out is NULL");
    auto m = std::make_unique<fblts_mesh>();
    validate_and_copy(desc, m->hm);
    *out = m.release();
    return FBLTS_OK;
  });
}

void fblts_mesh_destroy(fblts_mesh* mesh) { delete mesh; }

int fblts_layer_regions(const fblts_mesh* mesh, const int8_t* labels, int32_t binary, int32_t r, int8_t* out_labels,
                        int32_t* out_layer) {
  return guarded([&] {
    if (!mesh || !out_labels) throw Err(FBLTS_EINVAL, "NULL argument");
    std::vector<int8_t> lab4;
    std::vector<int> layer;
    layer_regions(mesh->hm, labels, binary != 0, r, lab4, layer);
    std::memcpy(out_labels, lab4.data(), lab4.size());
    if (out_layer)
      for (size_t i = 0; i < layer.size(); ++i) out_layer[i] = layer[i];
    return FBLTS_OK;
  });
}

int fblts_plan(const fblts_mesh* mesh, const int8_t* labels, int32_t binary, int32_t r, int32_t nonlinear,
               fblts_plan_info* out) {
  return guarded([&] {
    if (!mesh || !out) throw Err(FBLTS_EINVAL, "NULL argument");
    if (r < 1 || r > 64) throw Err(FBLTS_EINVAL, "r must be in 1..64");
    std::vector<int8_t> lab4;
    std::vector<int> layer;
    layer_regions(mesh->hm, labels, binary != 0, r, lab4, layer);
    Plan p;
    build_plan(mesh->hm, lab4, layer, true, nonlinear != 0, r, p);
    std::memset(out, 0, sizeof(*out));
    out->n_cells = mesh->hm.N;
    out->n_edges = mesh->hm.E;
    out->n_fine = p.nF;
    out->n_if1 = p.nIF1;
    out->n_if2 = p.nIF2;
    out->n_int = p.nINT;
    out->n_fine_e = p.nFE;
    out->n_if1_e = p.nIF1E;
    out->n_if2_e = p.nIF2E;
    out->n_int_e = p.nINTE;
    for (int s = 0; s < 3; ++s) {
      out->coarse_cell_begin[s] = p.coarse[s].cell.b;
      out->coarse_edge_begin[s] = p.coarse[s].edge.b;
      out->fine_cell_end[s] = p.fine[s].cell.e;
      out->fine_edge_end[s] = p.fine[s].edge.e;
    }
    return FBLTS_OK;
  });
}

int fblts_solver_create(const fblts_mesh* mesh, const fblts_params* params, void* hip_stream, fblts_solver** out) {
  return guarded([&] {
    if (!mesh || !out) throw Err(FBLTS_EINVAL, "NULL argument");
    check_params(params);
    auto s = std::make_unique<fblts_solver>();
    s->mesh = mesh;
    s->P.p = *params;
    hip_check(hipGetDevice(&s->device), "hipGetDevice");
    s->stream = make_stream(hip_stream, s->own_stream);
    scratch_setup(s->device);   // the solver's device is current here
    *out = s.release();
    return FBLTS_OK;
  });
}

void fblts_solver_destroy(fblts_solver* s) {
  if (s && s->stream) (void)hipStreamSynchronize(s->stream);
  delete s;
}

int fblts_set_regions(fblts_solver* s, const int8_t* labels, int32_t binary) {
  return guarded([&] {
    if (!s) throw Err(FBLTS_EINVAL, "solver is NULL");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->drop_graph();
    ++s->gen;
    s->have_regions = false;
    s->have_state = false;
    auto u = std::make_unique<MeshUnit>();
    setup_unit(*u, s->mesh->hm, s->P, labels, binary != 0, 1);
    s->unit = std::move(u);
    s->drag_on = false;
    build_passes(*s->unit, s->P, s->drag_on, s->opt, s->stream);
    s->have_regions = true;
    return FBLTS_OK;
  });
}

int fblts_set_state(fblts_solver* s, const double* h, const double* u, int32_t on_device) {
  return guarded([&] {
    if (!s || !h || !u) throw Err(FBLTS_EINVAL, "NULL argument");
    if (!s->have_regions) throw Err(FBLTS_ESTATE, "set_regions must come first");
    if (on_device) hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    ++s->gen;
    MeshUnit& un = *s->unit;
    state_in(un, s->stage_h, s->stage_u, h, u, 0, on_device != 0, s->stream);
    init_scratch(un, s->stream);
    if (un.st.cyclone) {
      // a new trajectory starts at model time zero: so does the storm
      static const long long zero = 0;
      hip_check(hipMemcpyAsync(un.st.cyc_clock.p, &zero, 8, hipMemcpyHostToDevice, s->stream), "hipMemcpyAsync");
      launch_cyclone(un.st.cyc, s->stream);
    }
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->have_state = true;
    s->time = 0.0;
    s->step = 0;
    return FBLTS_OK;
  });
}

int fblts_get_state(fblts_solver* s, double* h, double* u, int32_t on_device) {
  return guarded([&] {
    if (!s || (!h && !u)) throw Err(FBLTS_EINVAL, "NULL argument");
    if (!s->have_state) throw Err(FBLTS_ESTATE, "no state");
    check_persist(s->persist, s->stream);
    state_out(*s->unit, s->stage_h, s->stage_u, h, u, 0, on_device != 0, s->stream);
    return FBLTS_OK;
  });
}

int fblts_set_drag(fblts_solver* s, const double* cd, int32_t on_device) {
  return guarded([&] {
    if (!s) throw Err(FBLTS_EINVAL, "solver is NULL");
    if (!s->have_regions) throw Err(FBLTS_ESTATE, "set_regions must come first");
    MeshUnit& u = *s->unit;
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->drop_graph();
    ++s->gen;
    if (!cd) {
      s->drag_on = false;
    } else {
      if (!s->P.nonlinear()) throw Err(FBLTS_EINVAL, "drag needs nonlinear physics");
      if (on_device) hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
      const double* src = cd;
      if (!on_device) {
        if (s->stage_h.bytes < (size_t)u.pm.N * 8) s->stage_h.alloc((size_t)u.pm.N * 8);
        hip_check(hipMemcpyAsync(s->stage_h.p, cd, (size_t)u.pm.N * 8, hipMemcpyHostToDevice, s->stream), "memcpy");
        src = s->stage_h.as<double>();
      }
      launch_permute(u.st.cd.as<double>(), src, u.dm.cell_n2o.as<int>(), u.pm.N, 0, 0, 1, s->stream);
      hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
      s->drag_on = true;
    }
    build_passes(u, s->P, s->drag_on, s->opt, s->stream);
    return FBLTS_OK;
  });
}

int fblts_set_wind(fblts_solver* s, const double* wn, const double* wt, const double* wc, int32_t on_device) {
  return guarded([&] {
    if (!s) throw Err(FBLTS_EINVAL, "solver is NULL");
    if (!s->have_regions) throw Err(FBLTS_ESTATE, "set_regions must come first");
    MeshUnit& u = *s->unit;
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->drop_graph();
    ++s->gen;
    u.st.cyclone = false;
    if (!wn || !wt || !wc) {
      if (wn || wt || wc) throw Err(FBLTS_EINVAL, "set_wind takes all three arrays or none");
      u.st.has_wind = false;
    } else {
      if (!s->P.nonlinear()) throw Err(FBLTS_EINVAL, "wind stress needs nonlinear physics");
      if (on_device) hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
      const int E = u.pm.E;
      if (u.st.wind_n.bytes < (size_t)E * 8) {
        u.st.wind_n.alloc((size_t)E * 8);
        u.st.wind_t.alloc((size_t)E * 8);
        u.st.wind_c.alloc((size_t)E * 8);
      }
      const double* a = wn;
      const double* b = wt;
      const double* c = wc;
      DevBuf ta, tb, tc;
      if (!on_device) {
        ta.alloc((size_t)E * 8);
        tb.alloc((size_t)E * 8);
        tc.alloc((size_t)E * 8);
        hip_check(hipMemcpy(ta.p, wn, (size_t)E * 8, hipMemcpyHostToDevice), "memcpy");
        hip_check(hipMemcpy(tb.p, wt, (size_t)E * 8, hipMemcpyHostToDevice), "memcpy");
        hip_check(hipMemcpy(tc.p, wc, (size_t)E * 8, hipMemcpyHostToDevice), "memcpy");
        a = ta.as<double>();
        b = tb.as<double>();
        c = tc.as<double>();
      }
      launch_permute(u.st.wind_n.as<double>(), a, u.dm.edge_n2o.as<int>(), E, 0, 0, 1, s->stream);
      launch_permute(u.st.wind_t.as<double>(), b, u.dm.edge_n2o.as<int>(), E, 0, 0, 1, s->stream);
      launch_permute(u.st.wind_c.as<double>(), c, u.dm.edge_n2o.as<int>(), E, 0, 0, 1, s->stream);
      hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
      u.st.has_wind = true;
    }
    build_passes(u, s->P, s->drag_on, s->opt, s->stream);
    return FBLTS_OK;
  });
}

// ---------------------------------------------------------- cyclone forcing

static void unit3(const double* v, double* o, const char* what) {
  const double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  if (!(l > 0) || !std::isfinite(l)) throw Err(FBLTS_EINVAL, std::string("cyclone: zero or non-finite ") + what);
  for (int k = 0; k < 3; ++k) o[k] = v[k] / l;
}

// Validated device parameters of one storm (NULL: calm air).
static CycloneParams cyclone_params(const fblts_cyclone* c) {
  CycloneParams q{};
  if (!c) return q;
  const double vals[] = {c->v_trans, c->dp, c->rm, c->b, c->rho_air, c->radius, c->omega, c->t0};
  for (double v : vals)
    if (!std::isfinite(v)) throw Err(FBLTS_EINVAL, "cyclone parameters must be finite");
  if (!(c->rm > 0) || !(c->b > 0) || !(c->rho_air > 0) || !(c->radius > 0) || !(c->dp >= 0))
    throw Err(FBLTS_EINVAL, "cyclone: rm, b, rho_air, radius must be positive and dp non-negative");
  unit3(c->center, q.c0, "centre");
  unit3(c->axis, q.axis, "track axis");
  q.v_trans = c->v_trans;
  q.dp = c->dp;
  q.rm = c->rm;
  q.b = c->b;
  q.rho_air = c->rho_air;
  q.radius = c->radius;
  q.omega = c->omega;
  q.t0 = c->t0;
  q.omega_track = c->v_trans / c->radius;
  q.enabled = 1;
  return q;
}

// Wind arrays [E*nm], per-member parameters (calm air) and a zero step clock.
static void cyclone_install(MeshUnit& u, double dt, double rho_ratio) {
  const int E = u.pm.E, nm = u.st.nm;
  if (u.st.wind_n.bytes < (size_t)E * nm * 8) {
    u.st.wind_n.alloc((size_t)E * nm * 8);
    u.st.wind_t.alloc((size_t)E * nm * 8);
    u.st.wind_c.alloc((size_t)E * nm * 8);
  }
  std::vector<CycloneParams> calm(nm);
  u.st.cyc_p.alloc(calm.size() * sizeof(CycloneParams));
  hip_check(hipMemcpy(u.st.cyc_p.p, calm.data(), calm.size() * sizeof(CycloneParams), hipMemcpyHostToDevice),
            "memcpy");
  u.st.cyc_clock.alloc(8);
  const long long zero = 0;
  hip_check(hipMemcpy(u.st.cyc_clock.p, &zero, 8, hipMemcpyHostToDevice), "memcpy");
  CycloneArgs a{};
  a.x = u.st.cyc_x.bytes ? u.st.cyc_x.as<double>() : nullptr;
  a.n = u.st.cyc_n.bytes ? u.st.cyc_n.as<double>() : nullptr;
  a.wn = u.st.wind_n.as<double>();
  a.wt = u.st.wind_t.as<double>();
  a.wc = u.st.wind_c.as<double>();
  a.rho_ratio = rho_ratio;
  a.clock = u.st.cyc_clock.as<long long>();
  a.p = static_cast<const CycloneParams*>(u.st.cyc_p.p);
  a.E = E;
  a.nm_log2 = u.st.nm_log2;
  a.dt = dt;
  u.st.cyc = a;
  u.st.cyclone = true;
  u.st.has_wind = true;
}

// Unit edge positions and normals (caller order, [E][3]) in the library's SoA layout.
static void cyclone_positions(MeshUnit& u, const double* x_edge, const double* n_edge) {
  if (!x_edge || !n_edge) throw Err(FBLTS_EINVAL, "edge positions and normals are required");
  const int E = u.pm.E;
  std::vector<double> hx((size_t)3 * E), hn((size_t)3 * E);
  for (int i = 0; i < E; ++i) {
    const int o = u.plan.edge_new2old[i];
    double xu[3];
    unit3(x_edge + 3 * (size_t)o, xu, "edge position");
    const double* nv = n_edge + 3 * (size_t)o;
    const double nl = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    const double nx = nv[0] * xu[0] + nv[1] * xu[1] + nv[2] * xu[2];
    if (!(std::fabs(nl - 1.0) < 1e-6) || !(std::fabs(nx) < 1e-6))
      throw Err(FBLTS_EINVAL, "cyclone: edge normals must be unit vectors tangent to the sphere");
    for (int k = 0; k < 3; ++k) {
      hx[(size_t)k * E + i] = xu[k];
      hn[(size_t)k * E + i] = nv[k];
    }
  }
  if (u.st.cyc_x.bytes != hx.size() * 8) {
    u.st.cyc_x.alloc(hx.size() * 8);
    u.st.cyc_n.alloc(hn.size() * 8);
  }
  hip_check(hipMemcpy(u.st.cyc_x.p, hx.data(), hx.size() * 8, hipMemcpyHostToDevice), "memcpy");
  hip_check(hipMemcpy(u.st.cyc_n.p, hn.data(), hn.size() * 8, hipMemcpyHostToDevice), "memcpy");
  u.st.cyc.x = u.st.cyc_x.as<double>();
  u.st.cyc.n = u.st.cyc_n.as<double>();
}

static void cyclone_member(MeshUnit& u, int member, const CycloneParams& q) {
  hip_check(hipMemcpy(static_cast<char*>(u.st.cyc_p.p) + (size_t)member * sizeof(CycloneParams), &q,
                      sizeof(CycloneParams), hipMemcpyHostToDevice),
            "memcpy");
}

int fblts_set_cyclone(fblts_solver* s, const fblts_cyclone* c, const double* x_edge, const double* n_edge) {
  return guarded([&] {
    if (!s) throw Err(FBLTS_EINVAL, "solver is NULL");
    if (!s->have_regions) throw Err(FBLTS_ESTATE, "set_regions must come first");
    MeshUnit& u = *s->unit;
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->drop_graph();
    ++s->gen;
    if (!c) {
      u.st.cyclone = false;
      u.st.has_wind = false;
    } else {
      if (!s->P.nonlinear()) throw Err(FBLTS_EINVAL, "wind stress needs nonlinear physics");
      const CycloneParams q = cyclone_params(c);
      cyclone_positions(u, x_edge, n_edge);
      cyclone_install(u, s->P.p.dt, s->P.p.rho_air / s->P.p.rho_water);
      cyclone_member(u, 0, q);
      // wind of the first step, so that the state is complete before any step
      launch_cyclone(u.st.cyc, s->stream);
      hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    }
    build_passes(u, s->P, s->drag_on, s->opt, s->stream);
    return FBLTS_OK;
  });
}

int fblts_get_wind(fblts_solver* s, double* wn, double* wt, double* wc) {
  return guarded([&] {
    if (!s || !wn || !wt) throw Err(FBLTS_EINVAL, "NULL argument");
    if (!s->have_regions || !s->unit->st.has_wind) throw Err(FBLTS_ESTATE, "no wind is set");
    MeshUnit& u = *s->unit;
    const int E = u.pm.E;
    std::vector<double> a(E), b(E), c(E);
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    hip_check(hipMemcpy(a.data(), u.st.wind_n.p, (size_t)E * 8, hipMemcpyDeviceToHost), "memcpy");
    hip_check(hipMemcpy(b.data(), u.st.wind_t.p, (size_t)E * 8, hipMemcpyDeviceToHost), "memcpy");
    hip_check(hipMemcpy(c.data(), u.st.wind_c.p, (size_t)E * 8, hipMemcpyDeviceToHost), "memcpy");
    for (int i = 0; i < E; ++i) {
      const int o = u.plan.edge_new2old[i];
      wn[o] = a[i];
      wt[o] = b[i];
      if (wc) wc[o] = c[i];
    }
    return FBLTS_OK;
  });
}

// An on/off option's value: 0 or 1, anything else is refused.
static bool on_off(int32_t value, const char* name) {
  if (value != 0 && value != 1) throw Err(FBLTS_EINVAL, std::string(name) + ": 0 (off) or 1 (on)");
  return value == 1;
}

int fblts_set_option(fblts_solver* s, int32_t option, int32_t value) {
  return guarded([&] {
    if (!s) throw Err(FBLTS_EINVAL, "solver is NULL");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->drop_graph();
    if (option == FBLTS_OPT_FUSE_VERTEX) {
      s->opt.fuse_q = on_off(value, "fuse_vertex");
    } else if (option == FBLTS_OPT_BLOCK) {
      if (value != 64 && value != 128 && value != 256) throw Err(FBLTS_EINVAL, "block size must be 64, 128 or 256");
      s->opt.block = value;
    } else if (option == FBLTS_OPT_GRAPH_STEPS) {
      if (value < 1 || value > 64) throw Err(FBLTS_EINVAL, "steps per graph must be in 1..64");
      s->opt.graph_steps = value;
    } else if (option == FBLTS_OPT_EDGE_CELLS) {
      if (value && (!s->have_regions || s->unit->pm.kite_weights == 0))
        throw Err(FBLTS_EINVAL, "edge-via-cells needs set_regions first and kite-derived TRiSK weights");
      s->opt.edge_cells = on_off(value, "edge_cells");
    } else if (option == FBLTS_OPT_PERSISTENT) {
      if (value < 0 || value > 16) throw Err(FBLTS_EINVAL, "persistent: 0 (off) or blocks per compute unit, 1..16");
      s->opt.persistent = value;
    } else if (option == FBLTS_OPT_PIPELINE) {
      s->opt.pipeline = on_off(value, "pipeline");
    } else {
      throw Err(FBLTS_EINVAL, "unknown option");
    }
    solver_rebuild(s);
    return FBLTS_OK;
  });
}

int fblts_set_graph(fblts_solver* s, int32_t enable) {
  return guarded([&] {
    if (!s) throw Err(FBLTS_EINVAL, "solver is NULL");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->drop_graph();
    s->graph_on = enable != 0;
    return FBLTS_OK;
  });
}

int fblts_step(fblts_solver* s, int32_t n) {
  return guarded([&] {
    if (!s) throw Err(FBLTS_EINVAL, "solver is NULL");
    if (n < 0) throw Err(FBLTS_EINVAL, "negative step count");
    if (!s->have_state) throw Err(FBLTS_ESTATE, "set_state must come first");
    solver_run(s, n);
    return FBLTS_OK;
  });
}

int fblts_diagnostics(fblts_solver* s, fblts_diag* out) {
  return guarded([&] {
    if (!s || !out) throw Err(FBLTS_EINVAL, "NULL argument");
    if (!s->have_state) throw Err(FBLTS_ESTATE, "no state");
    check_persist(s->persist, s->stream);
    std::vector<double> q;
    diag_of(*s->unit, s->P, s->diag_partial, s->diag_out, s->stream, q);
    const int rc = fill_diag(q.data(), s->time, s->step, out);
    if (rc != FBLTS_OK) g_err = "state holds non-finite values or h <= 0";
    return rc;
  });
}

int fblts_diagnostics_noalloc(fblts_solver* s, fblts_diag* out) {
  return guarded([&] {
    if (!s || !out) throw Err(FBLTS_EINVAL, "NULL argument");
    if (!s->have_state) throw Err(FBLTS_ESTATE, "no state");
    if (s->device < 0 || s->device >= kMaxDevices || !g_scratch_dev[s->device])
      throw Err(FBLTS_EDEVICE, "the scratch array is not set up on the solver's device");
    check_persist(s->persist, s->stream);
    MeshUnit& u = *s->unit;
    const int nb = diag_blocks(u.dm.md);
    const size_t part = (size_t)kDiagQ * nb * u.st.nm;
    if (part + (size_t)kDiagQ * u.st.nm > kScratchDoubles)
      throw Err(FBLTS_EINVAL, "the diagnostics need more than the " + std::to_string(kScratchDoubles) +
                                  " doubles of the allocation-free scratch");
    double* sp = g_scratch_dev[s->device];
    // every partial and result is written before it is read: nothing to clear
    launch_diag(u.dm.md, u.st.nm_log2, s->P.wide() ? 0 : 1, u.st.H[0].as<double>(), u.st.U[0].as<double>(),
                s->P.p.g, sp, sp + part, s->stream);
    hip_check(hipGetLastError(), "diagnostics launch");
    double q[kDiagQ];
    hip_check(hipMemcpyAsync(q, sp + part, sizeof(q), hipMemcpyDeviceToHost, s->stream), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    const int rc = fill_diag(q, s->time, s->step, out);
    if (rc != FBLTS_OK) g_err = "state holds non-finite values or h <= 0";
    return rc;
  });
}

int fblts_get_info(fblts_solver* s, fblts_info* o) {
  return guarded([&] {
    if (!s || !o) throw Err(FBLTS_EINVAL, "NULL argument");
    if (!s->have_regions) throw Err(FBLTS_ESTATE, "set_regions must come first");
    const MeshUnit& u = *s->unit;
    std::memset(o, 0, sizeof(*o));
    o->n_cells = u.pm.N;
    o->n_edges = u.pm.E;
    o->n_vertices = u.pm.V;
    o->n_fine = u.plan.nF;
    o->n_if1 = u.plan.nIF1;
    o->n_if2 = u.plan.nIF2;
    o->n_int = u.plan.nINT;
    o->n_fine_e = u.plan.nFE;
    o->n_if1_e = u.plan.nIF1E;
    o->n_if2_e = u.plan.nIF2E;
    o->n_int_e = u.plan.nINTE;
    o->max_edges = u.pm.maxE;
    o->max_eoe = u.pm.maxEOE;
    o->cell_substeps_per_step = u.cell_substeps;
    int64_t launches = 0;
    double bytes = 0, comp = 0;
    for (const Pass& p : u.passes) {
      launches += p.kind == Pass::RK4FIN ? (int64_t)p.fin.size() : 1;
      bytes += p.model_bytes;
      comp += p.comp_bytes;
    }
    o->launches_per_step = launches;
    o->model_bytes_per_step = bytes;
    o->model_bytes_edge_pass = u.bytes_edge;
    o->edge_pass_items_per_step = u.edge_items;
    o->model_bytes_cell_pass = u.bytes_cell;
    o->compulsory_bytes_per_step = comp;
    o->compulsory_bytes_edge_pass = u.comp_edge;
    o->compulsory_bytes_cell_pass = u.comp_cell;
    return FBLTS_OK;
  });
}

int fblts_set_timing(fblts_solver* s, int32_t enable) {
  return guarded([&] {
    if (!s) throw Err(FBLTS_EINVAL, "solver is NULL");
    s->timing.on = enable != 0;
    s->timing.reset();
    return FBLTS_OK;
  });
}

int fblts_kernel_time(fblts_solver* s, int32_t cls, double* avg_ms, int64_t* launches) {
  return guarded([&] {
    if (!s || !avg_ms || cls < 0 || cls > 3) throw Err(FBLTS_EINVAL, "bad argument");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    double tot = 0;
    const size_t n = s->timing.used[cls];
    for (size_t k = 0; k < n; ++k) {
      float ms = 0;
      hip_check(hipEventElapsedTime(&ms, s->timing.ev[cls][k].first, s->timing.ev[cls][k].second), "hipEventElapsedTime");
      tot += ms;
    }
    *avg_ms = n ? tot / n : 0.0;
    if (launches) *launches = (int64_t)n;
    return FBLTS_OK;
  });
}

int fblts_time_kernels(fblts_solver* s, int32_t cls, int32_t repeats, double* avg_ms, int64_t* launches) {
  return guarded([&] {
    if (!s || !avg_ms || cls < 0 || cls > 3 || repeats < 1) throw Err(FBLTS_EINVAL, "bad argument");
    if (!s->have_state) throw Err(FBLTS_ESTATE, "set_state must come first");
    MeshUnit& u = *s->unit;
    const Pass::Kind kinds[4] = {Pass::EDGE, Pass::CELL, Pass::VERT, Pass::PREP};
    std::vector<Pass> sel;
    for (const Pass& p : u.passes)
      if (p.kind == kinds[cls]) sel.push_back(p);
    if (launches) *launches = (int64_t)sel.size() * repeats;
    *avg_ms = 0.0;
    if (sel.empty()) return FBLTS_OK;
    hipEvent_t a, b;
    hip_check(hipEventCreate(&a), "hipEventCreate");
    hip_check(hipEventCreate(&b), "hipEventCreate");
    std::vector<Pass> one(1);
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    hip_check(hipEventRecord(a, s->stream), "hipEventRecord");
    for (const Pass& p : sel) {
      one[0] = p;
      for (int r = 0; r < repeats; ++r) run_passes(one, s->drag_on, u.st.has_wind, s->stream, nullptr);
    }
    hip_check(hipEventRecord(b, s->stream), "hipEventRecord");
    hip_check(hipEventSynchronize(b), "hipEventSynchronize");
    float ms = 0;
    hip_check(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *avg_ms = ms / ((double)sel.size() * repeats);
    return FBLTS_OK;
  });
}

int fblts_debug_tendency(fblts_solver* s, int32_t which, const double* h, const double* u, double* out,
                         int32_t on_device) {
  return guarded([&] {
    if (!s || !h || !u || !out) throw Err(FBLTS_EINVAL, "NULL argument");
    if (which < 0 || which > 2) throw Err(FBLTS_EINVAL, "which must be 0 (Psi), 1 (Phi) or 2 (slow part of Phi)");
    if (which == 2 && !s->P.nonlinear()) throw Err(FBLTS_EINVAL, "the slow tendency needs nonlinear physics");
    if (!s->have_regions) throw Err(FBLTS_ESTATE, "set_regions must come first");
    MeshUnit& U = *s->unit;
    const int N = U.pm.N, E = U.pm.E, V = U.pm.V;
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    if (on_device) hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (s->dbg_h.bytes < (size_t)N * 8) s->dbg_h.alloc((size_t)N * 8);
    if (s->dbg_u.bytes < (size_t)E * 8) s->dbg_u.alloc((size_t)E * 8);
    if (s->dbg_out.bytes < (size_t)std::max(N, E) * 8) s->dbg_out.alloc((size_t)std::max(N, E) * 8);
    // stage the inputs in library order (member slot 0 of a one-member layout)
    const double* sh = h;
    const double* su = u;
    DevBuf th, tu;
    if (!on_device) {
      th.alloc((size_t)N * 8);
      tu.alloc((size_t)E * 8);
      hip_check(hipMemcpy(th.p, h, (size_t)N * 8, hipMemcpyHostToDevice), "memcpy");
      hip_check(hipMemcpy(tu.p, u, (size_t)E * 8, hipMemcpyHostToDevice), "memcpy");
      sh = th.as<double>();
      su = tu.as<double>();
    }
    double* Hin = s->dbg_h.as<double>();
    double* Uin = s->dbg_u.as<double>();
    double* acc = s->dbg_out.as<double>();
    launch_permute(Hin, sh, U.dm.cell_n2o.as<int>(), N, 0, 0, 1, s->stream);
    launch_permute(Uin, su, U.dm.edge_n2o.as<int>(), E, 0, 0, 1, s->stream);
    const bool nl = s->P.nonlinear();
    StageRanges R;
    R.cell = {0, N};
    R.vert = {0, nl ? V : 0};
    R.prep = {0, E};
    R.edge = {0, E};
    R.cell_upd = {0, 0};
    R.edge_upd = {0, 0};
    Launch<CellSeg> c{};
    c.nseg = 1;
    CellSeg& cs = c.seg[0];
    cs.m = U.dm.md;
    cs.nm_log2 = 0;
    cs.begin = 0;
    cs.end = N;
    cs.upd_begin = cs.upd_end = 0;
    cs.acc_begin = 0;
    cs.acc_end = which == 0 ? N : 0;
    cs.acc_first = 1;
    cs.Hsrc = Hin;
    cs.Usrc = Uin;
    cs.H0 = Hin;
    cs.Hnew_src = Hin;
    cs.Hdst = nullptr;
    cs.hs = U.st.hs.as<double>();
    cs.B = U.st.B.as<double>();
    cs.acc = acc;
    cs.c_dt = 0;
    cs.wn = 0;
    cs.ws = 1;
    cs.wb = 0;
    cs.acc_w = 1;
    cs.g = which == 2 ? 0.0 : s->P.p.g;   // slow part: B = K only
    if (U.st.nm != 1) throw Err(FBLTS_EINVAL, "debug tendency needs a one-member solver");
    const bool gw = s->P.gravity_wave();
    launch_cell(c, gw ? 2 : (nl ? 1 : 0), kBlock, s->stream);
    if (which >= 1 && gw) {
      Launch<EdgeSeg> ee{};
      ee.nseg = 1;
      EdgeSeg& es = ee.seg[0];
      es.m = U.dm.md;
      es.begin = 0;
      es.end = E;
      es.upd_begin = es.upd_end = 0;
      es.acc_begin = 0;
      es.acc_end = E;
      es.acc_first = 1;
      es.B = U.st.B.as<double>();
      es.acc = acc;
      es.acc_w = 1;
      launch_edge_fast(ee, false, kBlock, s->stream);
    } else if (which >= 1) {
      if (nl) {
        Launch<VertSeg> v{};
        v.nseg = 1;
        v.seg[0] = VertSeg{U.dm.md, 0, 0, V, Uin, U.st.hs.as<double>(), U.st.q.as<double>()};
        launch_vertex(v, kBlock, s->stream);
      }
      Launch<PrepSeg> pp{};
      pp.nseg = 1;
      pp.seg[0] = PrepSeg{U.dm.md, 0, 0, E, nl ? 0 : 1, Uin, U.st.hs.as<double>(),
                          nl ? U.st.q.as<double>() : U.dm.md.v_q0, U.st.P.as<double>()};
      launch_prep(pp, false, kBlock, s->stream);
      Launch<EdgeSeg> ee{};
      ee.nseg = 1;
      EdgeSeg& es = ee.seg[0];
      es.m = U.dm.md;
      es.nm_log2 = 0;
      es.begin = 0;
      es.end = E;
      es.upd_begin = es.upd_end = 0;
      es.acc_begin = 0;
      es.acc_end = E;
      es.acc_first = 1;
      es.P = U.st.P.as<double>();
      es.B = U.st.B.as<double>();
      es.Usrc = Uin;
      es.U0 = Uin;
      es.Udst = nullptr;
      es.acc = acc;
      es.cd = s->drag_on ? U.st.cd.as<double>() : nullptr;
      es.wind_n = U.st.has_wind ? U.st.wind_n.as<double>() : nullptr;
      es.wind_t = U.st.has_wind ? U.st.wind_t.as<double>() : nullptr;
      es.wind_c = U.st.has_wind ? U.st.wind_c.as<double>() : nullptr;
      es.c_dt = 0;
      es.acc_w = 1;
      launch_edge(ee, s->drag_on, U.st.has_wind, kBlock, s->stream, false);
    }
    const int n = which == 0 ? N : E;
    const int* perm = which == 0 ? U.dm.cell_n2o.as<int>() : U.dm.edge_n2o.as<int>();
    double* dst = out;
    DevBuf to;
    if (!on_device) {
      to.alloc((size_t)n * 8);
      dst = to.as<double>();
    }
    launch_permute(dst, acc, perm, n, 0, 0, 0, s->stream);
    hip_check(hipGetLastError(), "kernel launch");
    if (!on_device) hip_check(hipMemcpyAsync(out, dst, (size_t)n * 8, hipMemcpyDeviceToHost, s->stream), "memcpy");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    // the debug pass overwrote shared scratch: restore the stage invariants
    s->drop_graph();
    if (s->have_state) init_scratch(U, s->stream);
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    return FBLTS_OK;
  });
}

// ------------------------------------------------------------------ ensemble

int fblts_ensemble_create(const fblts_mesh* const* meshes, const int8_t* const* cell_labels, int32_t binary,
                          const int32_t* members_per_mesh, int32_t n_meshes, const fblts_params* params,
                          void* hip_stream, fblts_ensemble** out) {
  return guarded([&] {
    if (!meshes || !members_per_mesh || !out) throw Err(FBLTS_EINVAL, "NULL argument");
    if (n_meshes < 1 || n_meshes > kMaxSeg) throw Err(FBLTS_EINVAL, "n_meshes must be in 1..4");
    check_params(params);
    auto e = std::make_unique<fblts_ensemble>();
    e->P.p = *params;
    e->stream = make_stream(hip_stream, e->own_stream);
    std::vector<MeshUnit*> units;
    for (int k = 0; k < n_meshes; ++k) {
      const int nm = members_per_mesh[k];
      if (nm < 1 || nm > 64 || (nm & (nm - 1))) throw Err(FBLTS_EINVAL, "members per mesh must be a power of two <= 64");
      if (!meshes[k]) throw Err(FBLTS_EINVAL, "mesh is NULL");
      auto u = std::make_unique<MeshUnit>();
      setup_unit(*u, meshes[k]->hm, e->P, cell_labels ? cell_labels[k] : nullptr, binary != 0, nm);
      build_passes(*u, e->P, e->P.nonlinear(), e->opt, e->stream);
      units.push_back(u.get());
      e->units.push_back(std::move(u));
    }
    e->passes = merge_passes(units);
    ++e->version;
    // zero drag until set
    for (auto& u : e->units) launch_fill(u->st.cd.as<double>(), 0.0, (long)u->pm.N * u->st.nm, e->stream);
    hip_check(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    *out = e.release();
    return FBLTS_OK;
  });
}

void fblts_ensemble_destroy(fblts_ensemble* e) {
  if (e && e->stream) (void)hipStreamSynchronize(e->stream);
  delete e;
}

int fblts_ensemble_set_member(fblts_ensemble* e, int32_t mesh, int32_t member, const double* h, const double* u,
                              const double* cd, int32_t on_device) {
  return guarded([&] {
    if (!e || mesh < 0 || mesh >= (int)e->units.size()) throw Err(FBLTS_EINVAL, "bad mesh index");
    MeshUnit& U = *e->units[mesh];
    if (member < 0 || member >= U.st.nm) throw Err(FBLTS_EINVAL, "bad member index");
    if (!h || !u) throw Err(FBLTS_EINVAL, "NULL state");
    if (on_device) hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    state_in(U, e->stage_h, e->stage_u, h, u, member, on_device != 0, e->stream);
    if (cd) {
      const double* src = cd;
      DevBuf t;
      if (!on_device) {
        t.alloc((size_t)U.pm.N * 8);
        hip_check(hipMemcpy(t.p, cd, (size_t)U.pm.N * 8, hipMemcpyHostToDevice), "memcpy");
        src = t.as<double>();
      }
      launch_permute(U.st.cd.as<double>(), src, U.dm.cell_n2o.as<int>(), U.pm.N, U.st.nm_log2, member, 1, e->stream);
      hip_check(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    }
    init_scratch(U, e->stream);
    hip_check(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    return FBLTS_OK;
  });
}

int fblts_ensemble_get_member(fblts_ensemble* e, int32_t mesh, int32_t member, double* h, double* u,
                              int32_t on_device) {
  return guarded([&] {
    if (!e || mesh < 0 || mesh >= (int)e->units.size()) throw Err(FBLTS_EINVAL, "bad mesh index");
    MeshUnit& U = *e->units[mesh];
    if (member < 0 || member >= U.st.nm) throw Err(FBLTS_EINVAL, "bad member index");
    check_persist(e->persist, e->stream);
    state_out(U, e->stage_h, e->stage_u, h, u, member, on_device != 0, e->stream);
    return FBLTS_OK;
  });
}

int fblts_ensemble_set_cyclone(fblts_ensemble* e, int32_t mesh, int32_t member, const fblts_cyclone* c,
                               const double* x_edge, const double* n_edge) {
  return guarded([&] {
    if (!e || mesh < 0 || mesh >= (int)e->units.size()) throw Err(FBLTS_EINVAL, "bad mesh index");
    MeshUnit& U = *e->units[mesh];
    if (member < 0 || member >= U.st.nm) throw Err(FBLTS_EINVAL, "bad member index");
    if (!e->P.nonlinear()) throw Err(FBLTS_EINVAL, "wind stress needs nonlinear physics");
    const CycloneParams q = cyclone_params(c);
    hip_check(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    if (c || x_edge) cyclone_positions(U, x_edge, n_edge);
    // first storm: every member of every mesh gets the atmosphere (calm air
    // until given a storm), so that all meshes share one pass sequence
    if (!e->units[0]->st.cyclone)
      for (auto& u : e->units) cyclone_install(*u, e->P.p.dt, e->P.p.rho_air / e->P.p.rho_water);
    if (q.enabled && !U.st.cyc.x) throw Err(FBLTS_EINVAL, "edge positions and normals are required");
    cyclone_member(U, member, q);
    std::vector<MeshUnit*> units;
    for (auto& u : e->units) {
      build_passes(*u, e->P, e->P.nonlinear(), e->opt, e->stream);
      units.push_back(u.get());
    }
    e->passes = merge_passes(units);
    ++e->version;
    e->graphs.reset();
    launch_cyclone(U.st.cyc, e->stream);
    hip_check(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    return FBLTS_OK;
  });
}

int fblts_ensemble_set_graph(fblts_ensemble* e, int32_t enable) {
  return guarded([&] {
    if (!e) throw Err(FBLTS_EINVAL, "ensemble is NULL");
    hip_check(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    e->graphs.reset();
    e->graph_on = enable != 0;
    return FBLTS_OK;
  });
}

int fblts_ensemble_set_option(fblts_ensemble* e, int32_t option, int32_t value) {
  return guarded([&] {
    if (!e) throw Err(FBLTS_EINVAL, "ensemble is NULL");
    hip_check(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    if (option == FBLTS_OPT_FUSE_VERTEX) {
      e->opt.fuse_q = on_off(value, "fuse_vertex");
    } else if (option == FBLTS_OPT_BLOCK) {
      if (value != 64 && value != 128 && value != 256) throw Err(FBLTS_EINVAL, "block size must be 64, 128 or 256");
      e->opt.block = value;
    } else if (option == FBLTS_OPT_GRAPH_STEPS) {
      if (value < 1 || value > 64) throw Err(FBLTS_EINVAL, "steps per graph must be in 1..64");
      e->opt.graph_steps = value;
    } else if (option == FBLTS_OPT_EDGE_CELLS) {
      for (auto& u : e->units)
        if (value && u->pm.kite_weights == 0)
          throw Err(FBLTS_EINVAL, "edge-via-cells needs kite-derived TRiSK weights on every mesh");
      e->opt.edge_cells = on_off(value, "edge_cells");
    } else if (option == FBLTS_OPT_PERSISTENT) {
      if (value < 0 || value > 16) throw Err(FBLTS_EINVAL, "persistent: 0 (off) or blocks per compute unit, 1..16");
      e->opt.persistent = value;
    } else if (option == FBLTS_OPT_PIPELINE) {
      if (on_off(value, "pipeline")) throw Err(FBLTS_EINVAL, "ensembles run the sequential step (pipeline 0)");
    } else {
      throw Err(FBLTS_EINVAL, "unknown option");
    }
    ensemble_rebuild(e);
    return FBLTS_OK;
  });
}

int fblts_ensemble_step(fblts_ensemble* e, int32_t n) {
  return guarded([&] {
    if (!e) throw Err(FBLTS_EINVAL, "ensemble is NULL");
    if (n < 0) throw Err(FBLTS_EINVAL, "negative step count");
    ensemble_run(e, n);
    return FBLTS_OK;
  });
}

int fblts_ensemble_diagnostics(fblts_ensemble* e, fblts_diag* out) {
  return guarded([&] {
    if (!e || !out) throw Err(FBLTS_EINVAL, "NULL argument");
    check_persist(e->persist, e->stream);
    int rc = FBLTS_OK;
    size_t k = 0;
    for (auto& u : e->units) {
      std::vector<double> q;
      diag_of(*u, e->P, e->diag_partial, e->diag_out, e->stream, q);
      for (int m = 0; m < u->st.nm; ++m, ++k) {
        const int r = fill_diag(&q[(size_t)m * kDiagQ], e->step * e->P.p.dt, e->step, &out[k]);
        if (r != FBLTS_OK) rc = r;
      }
    }
    if (rc != FBLTS_OK) g_err = "a member holds non-finite values or h <= 0";
    return rc;
  });
}

int fblts_ensemble_info(fblts_ensemble* e, int64_t* member_cells, int64_t* cell_substeps, double* model_bytes) {
  return guarded([&] {
    if (!e) throw Err(FBLTS_EINVAL, "ensemble is NULL");
    int64_t mc = 0, cs = 0;
    for (auto& u : e->units) {
      mc += (int64_t)u->pm.N * u->st.nm;
      cs += u->cell_substeps;
    }
    double b = 0;
    for (auto& p : e->passes) b += p.model_bytes;
    if (member_cells) *member_cells = mc;
    if (cell_substeps) *cell_substeps = cs;
    if (model_bytes) *model_bytes = b;
    return FBLTS_OK;
  });
}

int fblts_autotune(void* handle, int32_t handle_kind, int32_t steps, int32_t repeats, const char* cache_json_path,
                   fblts_schedule* out, fblts_schedule* tried, int32_t max_tried, int32_t* n_tried) {
  return guarded([&] {
    if (!handle) throw Err(FBLTS_EINVAL, "handle is NULL");
    if (steps < 1 || steps > 10000 || repeats < 1 || repeats > 100)
      throw Err(FBLTS_EINVAL, "steps must be in 1..10000 and repeats in 1..100");
    if (max_tried < 0 || (max_tried > 0 && !tried)) throw Err(FBLTS_EINVAL, "bad candidate output array");
    fblts_solver* s = handle_kind == FBLTS_HANDLE_SOLVER ? static_cast<fblts_solver*>(handle) : nullptr;
    fblts_ensemble* e = handle_kind == FBLTS_HANDLE_ENSEMBLE ? static_cast<fblts_ensemble*>(handle) : nullptr;
    if (!s && !e) throw Err(FBLTS_EINVAL, "unknown handle kind");
    if (s && !s->have_state) throw Err(FBLTS_ESTATE, "set_state must come first");
    hipStream_t st = s ? s->stream : e->stream;
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    std::vector<MeshUnit*> units;
    if (s) units.push_back(s->unit.get());
    else
      for (auto& u : e->units) units.push_back(u.get());
    LaunchOpts& opt = s ? s->opt : e->opt;
    bool& graph_on = s ? s->graph_on : e->graph_on;
    bool cells_ok = true;
    for (MeshUnit* u : units) cells_ok = cells_ok && u->pm.kite_weights != 0;
    auto rebuild = [&] {
      if (s) solver_rebuild(s);
      else ensemble_rebuild(e);
    };
    auto run = [&](int n) {
      if (s) solver_run(s, n);
      else ensemble_run(e, n);
    };
    const std::string key = s ? solver_key(*s) : ensemble_key(*e);

    ScheduleCache cache;
    if (cache_json_path) cache = cache_read(cache_json_path);
    Schedule best;
    bool hit = false;
    for (const auto& kv : cache)
      if (kv.first == key && (!kv.second.cells || cells_ok)) {
        best = kv.second;
        hit = true;
      }
    int ntried = 0;
    if (!hit) {
      const bool graph_was = graph_on, timing_was = s && s->timing.on;
      const double time0 = s ? s->time : 0.0;
      const int64_t step0 = s ? s->step : e->step;
      const auto snap = snapshot_take(units, st);
      auto restore = [&] {
        snapshot_restore(units, snap, st);
        if (s) {
          s->time = time0;
          s->step = step0;
          s->timing.on = timing_was;
        } else {
          e->step = step0;
        }
        graph_on = graph_was;
      };
      if (s) s->timing.on = false;
      best.ms = std::numeric_limits<double>::infinity();
      // search order: the graph-replayed per-pass schedules, then the
      // persistent launch (fused q_v or not; its blocks are kBlock threads),
      // then the momentum pass through the cells' edge lists
      struct Cand {
        int fuse, bs, cells, persistent;
      };
      std::vector<Cand> cands;
      for (int fuse = 1; fuse >= 0; --fuse)
        for (int bs : {256, 128, 64}) cands.push_back({fuse, bs, 0, 0});
      int coop = 0;
      hip_check(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, s ? s->device : 0),
                "hipDeviceGetAttribute");
      if (coop)
        for (int fuse = 1; fuse >= 0; --fuse)
          for (int per_cu : {1, 4}) cands.push_back({fuse, kBlock, 0, per_cu});
      if (cells_ok)
        for (int fuse = 1; fuse >= 0; --fuse)
          for (int bs : {256, 128, 64}) cands.push_back({fuse, bs, 1, 0});
      try {
        for (const Cand& c : cands) {
          opt.fuse_q = c.fuse != 0;
          opt.block = c.bs;
          opt.edge_cells = c.cells != 0;
          opt.persistent = c.persistent;
          graph_on = true;
          rebuild();
          const double ms = time_schedule(st, steps, repeats, run);
          if (s) check_persist(s->persist, st);
          else check_persist(e->persist, st);
          if (ntried < max_tried) tried[ntried] = fblts_schedule{c.fuse, c.bs, c.cells, 0, ms, c.persistent};
          ++ntried;
          if (ms < best.ms) best = Schedule{c.fuse, c.bs, c.cells, ms, c.persistent};
        }
      } catch (...) {
        try {
          hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
          restore();
        } catch (...) {
        }
        throw;
      }
      restore();
    }
    opt.fuse_q = best.fuse != 0;
    opt.block = best.block;
    opt.edge_cells = best.cells != 0;
    opt.persistent = best.persistent;
    rebuild();
    if (!hit && cache_json_path) {
      bool replaced = false;
      for (auto& kv : cache)
        if (kv.first == key) {
          kv.second = best;
          replaced = true;
        }
      if (!replaced) cache.emplace_back(key, best);
      cache_write(cache_json_path, cache);
    }
    if (out) *out = fblts_schedule{best.fuse, best.block, best.cells, hit ? 1 : 0, best.ms, best.persistent};
    if (n_tried) *n_tried = ntried;
    return FBLTS_OK;
  });
}

}  // extern "C"

// ------------------------------------------------------------- adjoint ABI

static void adj_check(fblts_solver* s) {
  if (!s) throw Err(FBLTS_EINVAL, "solver is NULL");
  if (!s->have_state) throw Err(FBLTS_ESTATE, "set_state must come first");
  if (s->P.p.scheme != FBLTS_SCHEME_FBLTS) throw Err(FBLTS_EINVAL, "the adjoint covers the FB-LTS scheme");
  if (s->unit->st.has_wind) throw Err(FBLTS_EINVAL, "the adjoint does not cover the wind-stress term");
  if (s->P.fast()) throw Err(FBLTS_EINVAL, "the adjoint covers the unsplit linear and nonlinear systems only");
}

static Rev make_rev(fblts_solver* s, AdjointState& A) {
  MeshUnit& u = *s->unit;
  Rev r;
  r.m = &u.dm.md;
  r.N = u.pm.N;
  r.E = u.pm.E;
  r.V = u.pm.V;
  r.nF = u.plan.nF;
  r.if1e = r.nF + u.plan.nIF1;
  r.if2e = r.if1e + u.plan.nIF2;
  r.nFE = u.plan.nFE;
  r.if1ee = r.nFE + u.plan.nIF1E;
  r.if2ee = r.if1ee + u.plan.nIF2E;
  r.M = s->P.p.M;
  r.dt = s->P.p.dt;
  r.b1 = s->P.p.beta1;
  r.b2 = s->P.p.beta2;
  r.b3 = s->P.p.beta3;
  r.g = s->P.p.g;
  r.linear = !s->P.nonlinear();
  r.drag = s->drag_on;
  r.cd = u.st.cd.as<double>();
  for (int k = 0; k < kNCellArr; ++k) r.C[k] = A.cells.as<double>() + (size_t)k * r.N;
  for (int k = 0; k < kNEdgeArr; ++k) r.Ed[k] = A.edges.as<double>() + (size_t)k * r.E;
  r.ZA = A.verts.as<double>();
  r.HV = r.ZA + r.V;
  r.P = A.Pf.as<double>();
  r.st = s->stream;
  // Prefix closures through the permuted mesh's incidence lists: one past
  // the largest index a range of entities reaches.
  const PermMesh& pm = u.pm;
  auto cells_of_edges = [&](int ne) {
    int x = 0;
    for (int e = 0; e < ne; ++e) x = std::max({x, pm.e_cell[e] + 1, pm.e_cell[(size_t)pm.es + e] + 1});
    return x;
  };
  auto edges_of_cells = [&](int nc) {
    int x = 0;
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < pm.c_nedge[i]; ++j) x = std::max(x, (pm.c_edge[(size_t)j * pm.cs + i] >> 1) + 1);
    return x;
  };
  auto eoe_of_edges = [&](int ne) {
    int x = ne;
    for (int e = 0; e < ne; ++e)
      for (int j = 0; j < pm.e_neoe[e]; ++j) x = std::max(x, pm.e_eoe[(size_t)j * pm.es + e] + 1);
    return x;
  };
  auto verts_of_edges = [&](int ne) {
    int x = 0;
    for (int e = 0; e < ne; ++e) x = std::max({x, pm.e_vert[e] + 1, pm.e_vert[(size_t)pm.es + e] + 1});
    return x;
  };
  auto edges_of_verts = [&](int nv) {
    int x = 0;
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < 3; ++j) x = std::max(x, (pm.v_edge[(size_t)j * pm.vs + v] >> 1) + 1);
    return x;
  };
  auto cells_of_verts = [&](int nv) {
    int x = 0;
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < 3; ++j) x = std::max(x, pm.v_cell[(size_t)j * pm.vs + v] + 1);
    return x;
  };
  auto verts_of_cells = [&](int nc) {
    int x = 0;
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < pm.c_nedge[i]; ++j) x = std::max(x, pm.c_vert[(size_t)j * pm.cs + i] + 1);
    return x;
  };
  // Phi with its cotangent on edges [0, fe): pass 1 forms G (and the drag
  // terms) there; pass 2 sums G over cells; pass 3 gathers G, R and the
  // records over edges_on_edge and B-bar at the edge's cells; pass 4 sums
  // q-bar over vertices; passes 5-6 spread the vertex terms to edges and
  // cells.  Each z bound is the reach of the readers of an intermediate.
  auto phi_range = [&](int fe) {
    VjpRange q;
    q.e1 = fe;
    q.c1 = cells_of_edges(fe);
    q.e2 = std::max({fe, eoe_of_edges(fe), edges_of_cells(q.c1)});
    q.v1 = verts_of_edges(q.e2);
    q.e3 = edges_of_verts(q.v1);
    q.c3 = std::max(cells_of_edges(q.e2), cells_of_verts(q.v1));
    q.pe = eoe_of_edges(q.e2);
    q.zG = std::max(edges_of_cells(q.c1), q.pe);
    q.zR = q.pe;
    q.zHD = q.e2;
    q.zCDB = edges_of_cells(q.c3);
    q.zBB = cells_of_edges(q.e2);
    q.zQB = edges_of_verts(q.v1);
    q.zHE = q.zCDB;
    q.zZA = verts_of_edges(q.e3);
    q.zHV = verts_of_cells(q.c3);
    return q;
  };
  // Psi with its cotangent on cells [0, pc): the edge pass over the cells'
  // edges, the cell pass over those edges' cells.
  auto psi_range = [&](int pc) {
    PsiRange q;
    q.ne = edges_of_cells(pc);
    q.nc = cells_of_edges(q.ne);
    q.zT = edges_of_cells(q.nc);
    return q;
  };
  r.phi_all = VjpRange{r.E, r.N, r.E, r.V, r.E, r.N, r.E, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  r.psi_all = PsiRange{r.E, r.N, 0};
  r.phi_f12 = phi_range(r.nFE);
  r.phi_f3 = phi_range(r.if2ee);
  r.psi_f12 = psi_range(r.nF);
  r.psi_f3 = psi_range(r.if2e);
  return r;
}

static void adj_alloc(fblts_solver* s, AdjointState& A) {
  const MeshUnit& u = *s->unit;
  const size_t N = u.pm.N, E = u.pm.E, V = u.pm.V;
  if (A.cells.bytes < kNCellArr * N * 8) A.cells.alloc(kNCellArr * N * 8);
  if (A.edges.bytes < kNEdgeArr * E * 8) A.edges.alloc(kNEdgeArr * E * 8);
  if (A.verts.bytes < 2 * V * 8) A.verts.alloc(2 * V * 8);
  if (A.Pf.bytes < 4 * E * 8) A.Pf.alloc(4 * E * 8);
}

// Recording forward: the definition-mode pass list with tape snapshots.
static void build_recording(fblts_solver* s, AdjointState& A) {
  MeshUnit& u = *s->unit;
  const int N = u.pm.N, E = u.pm.E, M = s->P.p.M;
  build_plan(*u.hm, u.lab4, u.layer, true, s->P.nonlinear(), s->P.p.r_layers, A.plan_full, true);
  if (A.plan_full.cell_new2old != u.plan.cell_new2old || A.plan_full.edge_new2old != u.plan.edge_new2old)
    throw Err(FBLTS_EINVAL, "internal: definition-mode plan reordered the mesh");
  // build the definition-mode pass list without disturbing the solver's own
  std::vector<Pass> keep = u.passes;
  const double kb[4] = {u.bytes_edge, u.bytes_cell, u.comp_edge, u.comp_cell};
  const int64_t ki = u.edge_items, kc = u.cell_substeps;
  build_passes_impl(u, s->P, s->drag_on, s->opt.fuse_q, &A.plan_full);
  std::vector<Pass> def = u.passes;
  u.passes = keep;
  u.bytes_edge = kb[0];
  u.bytes_cell = kb[1];
  u.comp_edge = kb[2];
  u.comp_cell = kb[3];
  u.edge_items = ki;
  u.cell_substeps = kc;
  A.tape_c = (size_t)(4 + 4 * M) * N;
  A.tape_e = (size_t)(4 + 3 * M) * E;
  if (A.step_tape.bytes < (A.tape_c + A.tape_e) * 8) A.step_tape.alloc((A.tape_c + A.tape_e) * 8);
  double* tc = A.step_tape.as<double>();
  double* te = tc + A.tape_c;
  auto H = [&](int k) { return u.st.H[k].as<double>(); };
  auto U = [&](int k) { return u.st.U[k].as<double>(); };
  auto copy = [&](double* dst, const double* src, long n) {
    Pass c;
    c.kind = Pass::COPY;
    c.cdst = dst;
    c.csrc = src;
    c.cn = n;
    A.rec.push_back(c);
  };
  A.rec.clear();
  copy(tc, H(0), N);
  copy(te, U(0), E);
  for (size_t i = 0; i < def.size(); ++i) {
    const Pass& p = def[i];
    A.rec.push_back(p);
    const bool last_of_tag = i + 1 == def.size() || def[i + 1].tag != p.tag;
    if (p.tag == 3 && last_of_tag) {
      for (int k = 1; k <= 3; ++k) {
        copy(tc + (size_t)k * N, H(k), N);
        copy(te + (size_t)k * E, U(k), E);
      }
    }
    if (p.kind == Pass::PRED) {
      const int k = (p.tag - 200) / 10;
      copy(tc + (size_t)(4 + 4 * k) * N, H(0), N);
      copy(te + (size_t)(4 + 3 * k) * E, U(0), E);
    }
    if (p.tag >= 100 && p.tag < 200) {
      const int k = (p.tag - 100) / 10, st = (p.tag - 100) % 10;
      if (p.kind == Pass::EDGE && st == 1) {
        copy(tc + (size_t)(5 + 4 * k) * N, H(1), N);
        copy(te + (size_t)(5 + 3 * k) * E, U(1), E);
      }
      if (p.kind == Pass::EDGE && st == 2) {
        copy(tc + (size_t)(6 + 4 * k) * N, H(2), N);
        copy(te + (size_t)(6 + 3 * k) * E, U(2), E);
      }
      if (p.kind == Pass::CELL && st == 3) {   // H3: fine cells were written into H0
        copy(tc + (size_t)(7 + 4 * k) * N, H(3), N);
        copy(tc + (size_t)(7 + 4 * k) * N, H(0), u.plan.nF);
      }
    }
  }
}

extern "C" {

int fblts_adjoint_forward(fblts_solver* s, int32_t n_steps, int32_t ckpt_every) {
  return guarded([&] {
    adj_check(s);
    if (n_steps < 1 || ckpt_every < 1) throw Err(FBLTS_EINVAL, "n_steps and ckpt_every must be positive");
    if (s->unit->st.nm != 1) throw Err(FBLTS_EINVAL, "the adjoint needs a one-member solver");
    if (!s->adj) s->adj = std::make_unique<AdjointState>();
    AdjointState& A = *s->adj;
    MeshUnit& u = *s->unit;
    const int N = u.pm.N, E = u.pm.E;
    A.recorded = false;
    A.n_steps = n_steps;
    A.ckpt_every = ckpt_every;
    A.M = s->P.p.M;
    const int nck = (n_steps + ckpt_every - 1) / ckpt_every;
    if (A.ckpt.bytes < (size_t)nck * (N + E) * 8) A.ckpt.alloc((size_t)nck * (N + E) * 8);
    if (A.final_state.bytes < (size_t)(N + E) * 8) A.final_state.alloc((size_t)(N + E) * 8);
    for (int t = 0; t < n_steps; ++t) {
      if (t % ckpt_every == 0) {
        double* c = A.ckpt.as<double>() + (size_t)(t / ckpt_every) * (N + E);
        launch_copy(c, u.st.H[0].as<double>(), N, s->stream);
        launch_copy(c + N, u.st.U[0].as<double>(), E, s->stream);
      }
      run_passes(u.passes, s->drag_on, false, s->stream, nullptr);
    }
    launch_copy(A.final_state.as<double>(), u.st.H[0].as<double>(), N, s->stream);
    launch_copy(A.final_state.as<double>() + N, u.st.U[0].as<double>(), E, s->stream);
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->step += n_steps;
    s->time += n_steps * s->P.p.dt;
    A.gen = ++s->gen;
    A.recorded = true;
    return FBLTS_OK;
  });
}

int fblts_adjoint_recording(fblts_solver* s, uint64_t* id) {
  return guarded([&] {
    if (!s || !id) throw Err(FBLTS_EINVAL, "NULL argument");
    *id = (s->adj && s->adj->recorded && s->adj->gen == s->gen) ? s->adj->gen : 0;
    return FBLTS_OK;
  });
}

int fblts_adjoint_backward(fblts_solver* s, const double* gh_final, const double* gu_final, double* gh0, double* gu0,
                           double* gcd, int32_t on_device) {
  return guarded([&] {
    adj_check(s);
    if (!s->adj || !s->adj->recorded) throw Err(FBLTS_ESTATE, "fblts_adjoint_forward must come first");
    if (s->adj->gen != s->gen)
      throw Err(FBLTS_ESTATE, "the solver's regions, state, forcing or step count changed after "
                              "fblts_adjoint_forward: record the forward run again");
    if (!gh_final || !gu_final) throw Err(FBLTS_EINVAL, "NULL seed");
    AdjointState& A = *s->adj;
    MeshUnit& u = *s->unit;
    const int N = u.pm.N, E = u.pm.E;
    if (on_device) hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    adj_alloc(s, A);
    build_recording(s, A);
    const int K = A.ckpt_every;
    if (A.seg_tape.bytes < (size_t)K * (A.tape_c + A.tape_e) * 8) A.seg_tape.alloc((size_t)K * (A.tape_c + A.tape_e) * 8);
    Rev r = make_rev(s, A);
    // seeds into the library's numbering
    DevBuf th, tu;
    const double* sh = gh_final;
    const double* su = gu_final;
    if (!on_device) {
      th.alloc((size_t)N * 8);
      tu.alloc((size_t)E * 8);
      hip_check(hipMemcpy(th.p, gh_final, (size_t)N * 8, hipMemcpyHostToDevice), "memcpy");
      hip_check(hipMemcpy(tu.p, gu_final, (size_t)E * 8, hipMemcpyHostToDevice), "memcpy");
      sh = th.as<double>();
      su = tu.as<double>();
    }
    launch_permute(r.C[hNb], sh, u.dm.cell_n2o.as<int>(), N, 0, 0, 1, s->stream);
    launch_permute(r.Ed[uNb], su, u.dm.edge_n2o.as<int>(), E, 0, 0, 1, s->stream);
    r.zero(r.C[cdb], 0, N);
    const int nseg = (A.n_steps + K - 1) / K;
    const size_t per = A.tape_c + A.tape_e;
    for (int seg = nseg - 1; seg >= 0; --seg) {
      const int t0 = seg * K, t1 = std::min(A.n_steps, t0 + K);
      const double* c = A.ckpt.as<double>() + (size_t)seg * (N + E);
      launch_copy(u.st.H[0].as<double>(), c, N, s->stream);
      launch_copy(u.st.U[0].as<double>(), c + N, E, s->stream);
      for (int t = t0; t < t1; ++t) {
        run_passes(A.rec, s->drag_on, false, s->stream, nullptr);
        launch_copy(A.seg_tape.as<double>() + (size_t)(t - t0) * per, A.step_tape.as<double>(), (long)per, s->stream);
      }
      for (int t = t1 - 1; t >= t0; --t) {
        const double* tc = A.seg_tape.as<double>() + (size_t)(t - t0) * per;
        r.step(tc, tc + A.tape_c);
        // the input cotangent of this step is the output cotangent of the previous one
        launch_copy(r.C[hNb], r.C[hb], N, s->stream);
        launch_copy(r.Ed[uNb], r.Ed[ub], E, s->stream);
      }
    }
    hip_check(hipGetLastError(), "adjoint launches");
    // outputs in the caller's numbering
    auto out = [&](double* dst, const double* src, const int* perm, int n) {
      if (!dst) return;
      if (on_device) {
        launch_permute(dst, src, perm, n, 0, 0, 0, s->stream);
      } else {
        DevBuf t;
        t.alloc((size_t)n * 8);
        launch_permute(t.as<double>(), src, perm, n, 0, 0, 0, s->stream);
        hip_check(hipMemcpyAsync(dst, t.p, (size_t)n * 8, hipMemcpyDeviceToHost, s->stream), "memcpy");
        hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
      }
    };
    out(gh0, r.C[hNb], u.dm.cell_n2o.as<int>(), N);
    out(gu0, r.Ed[uNb], u.dm.edge_n2o.as<int>(), E);
    out(gcd, r.C[cdb], u.dm.cell_n2o.as<int>(), N);
    // leave the solver at the final state of the forward run
    launch_copy(u.st.H[0].as<double>(), A.final_state.as<double>(), N, s->stream);
    launch_copy(u.st.U[0].as<double>(), A.final_state.as<double>() + N, E, s->stream);
    init_scratch(u, s->stream);
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    return FBLTS_OK;
  });
}

int fblts_debug_vjp(fblts_solver* s, int32_t which, const double* h, const double* u, const double* cot, double* hbar,
                    double* ubar, double* cdbar) {
  return guarded([&] {
    if (!s || !h || !u || !cot || !hbar || !ubar) throw Err(FBLTS_EINVAL, "NULL argument");
    if (!s->have_regions) throw Err(FBLTS_ESTATE, "set_regions must come first");
    if (which != 0 && which != 1) throw Err(FBLTS_EINVAL, "which must be 0 (Psi) or 1 (Phi)");
    if (!s->adj) s->adj = std::make_unique<AdjointState>();
    AdjointState& A = *s->adj;
    MeshUnit& U = *s->unit;
    const int N = U.pm.N, E = U.pm.E;
    adj_alloc(s, A);
    Rev r = make_rev(s, A);
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    DevBuf th, tu, tc, dh, du;
    th.alloc((size_t)N * 8);
    tu.alloc((size_t)E * 8);
    tc.alloc((size_t)std::max(N, E) * 8);
    dh.alloc((size_t)N * 8);
    du.alloc((size_t)E * 8);
    hip_check(hipMemcpy(th.p, h, (size_t)N * 8, hipMemcpyHostToDevice), "memcpy");
    hip_check(hipMemcpy(tu.p, u, (size_t)E * 8, hipMemcpyHostToDevice), "memcpy");
    hip_check(hipMemcpy(tc.p, cot, (size_t)(which == 0 ? N : E) * 8, hipMemcpyHostToDevice), "memcpy");
    // inputs into library order: h -> hspt, u -> U3Fb, cotangent -> pb / fb
    launch_permute(r.C[hspt], th.as<double>(), U.dm.cell_n2o.as<int>(), N, 0, 0, 1, s->stream);
    launch_permute(r.Ed[U3Fb], tu.as<double>(), U.dm.edge_n2o.as<int>(), E, 0, 0, 1, s->stream);
    r.zero(r.Ed[ub], 0, E);
    r.zero(r.C[hb], 0, N);
    r.zero(r.C[cdb], 0, N);
    if (which == 0) {
      launch_permute(r.C[pb], tc.as<double>(), U.dm.cell_n2o.as<int>(), N, 0, 0, 1, s->stream);
      r.psi_vjp(r.Ed[U3Fb], r.C[hspt], r.C[pb], r.Ed[ub], r.C[hb], r.psi_all);
    } else {
      launch_permute(r.Ed[fb], tc.as<double>(), U.dm.edge_n2o.as<int>(), E, 0, 0, 1, s->stream);
      r.phi_vjp(r.Ed[U3Fb], r.C[hspt], r.Ed[fb], r.Ed[ub], r.C[hb], r.phi_all);
    }
    launch_permute(dh.as<double>(), r.C[hb], U.dm.cell_n2o.as<int>(), N, 0, 0, 0, s->stream);
    launch_permute(du.as<double>(), r.Ed[ub], U.dm.edge_n2o.as<int>(), E, 0, 0, 0, s->stream);
    hip_check(hipMemcpyAsync(hbar, dh.p, (size_t)N * 8, hipMemcpyDeviceToHost, s->stream), "memcpy");
    hip_check(hipMemcpyAsync(ubar, du.p, (size_t)E * 8, hipMemcpyDeviceToHost, s->stream), "memcpy");
    if (cdbar) {
      launch_permute(dh.as<double>(), r.C[cdb], U.dm.cell_n2o.as<int>(), N, 0, 0, 0, s->stream);
      hip_check(hipMemcpyAsync(cdbar, dh.p, (size_t)N * 8, hipMemcpyDeviceToHost, s->stream), "memcpy");
    }
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    return FBLTS_OK;
  });
}

}  // extern "C"
