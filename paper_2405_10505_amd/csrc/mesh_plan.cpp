// Host-side mesh validation, region layering (paper Section 2.2), the
// region-contiguous reordering and the dependency-closure pass ranges.
#include "mesh_plan.h"
#include "fblts_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <numeric>
#include <stdexcept>

namespace fblts {

namespace {

[[noreturn]] void fail(const std::string& msg) { throw std::runtime_error(msg); }

template <class T>
std::vector<T> copy_arr(const T* p, size_t n, const char* name) {
  if (n > 0 && p == nullptr) fail(std::string("mesh: ") + name + " is NULL");
  return std::vector<T>(p, p + n);
}

std::string at(const char* what, long i) { return std::string(what) + " " + std::to_string(i); }

}  // namespace

void validate_and_copy(const fblts_mesh_desc* d, HostMesh& m) {
  if (!d) fail("mesh: descriptor is NULL");
  if (d->n_cells < 3 || d->n_edges < 3 || d->n_vertices < 2) fail("mesh: too few cells, edges or vertices");
  const int N = d->n_cells, E = d->n_edges, V = d->n_vertices;
  m.N = N;
  m.E = E;
  m.V = V;
  m.coe = copy_arr(d->cells_on_edge, 2 * (size_t)E, "cells_on_edge");
  m.voe = copy_arr(d->vertices_on_edge, 2 * (size_t)E, "vertices_on_edge");
  m.eoc_off = copy_arr(d->edges_on_cell_off, (size_t)N + 1, "edges_on_cell_off");
  m.voc_off = copy_arr(d->vertices_on_cell_off, (size_t)N + 1, "vertices_on_cell_off");
  if (m.eoc_off[0] != 0) fail("mesh: edges_on_cell_off[0] != 0");
  for (int i = 0; i < N; ++i) {
    if (m.eoc_off[i + 1] - m.eoc_off[i] < 3) fail("mesh: cell with fewer than 3 edges: " + at("cell", i));
    if (m.eoc_off[i + 1] - m.eoc_off[i] > 16) fail("mesh: cell with more than 16 edges: " + at("cell", i));
    if (m.voc_off[i] != m.eoc_off[i] || m.voc_off[i + 1] != m.eoc_off[i + 1])
      fail("mesh: vertices_on_cell_off differs from edges_on_cell_off at " + at("cell", i));
  }
  const size_t nce = (size_t)m.eoc_off[N];
  if (nce != 2 * (size_t)E) fail("mesh: sum of cell degrees != 2 * n_edges");
  m.eoc = copy_arr(d->edges_on_cell, nce, "edges_on_cell");
  m.voc = copy_arr(d->vertices_on_cell, nce, "vertices_on_cell");
  m.eoe_off = copy_arr(d->edges_on_edge_off, (size_t)E + 1, "edges_on_edge_off");
  if (m.eoe_off[0] != 0) fail("mesh: edges_on_edge_off[0] != 0");
  for (int e = 0; e < E; ++e)
    if (m.eoe_off[e + 1] < m.eoe_off[e]) fail("mesh: edges_on_edge_off not monotone at " + at("edge", e));
  const size_t neoe = (size_t)m.eoe_off[E];
  m.eoe = copy_arr(d->edges_on_edge, neoe, "edges_on_edge");
  m.woe = copy_arr(d->weights_on_edge, neoe, "weights_on_edge");
  m.eov = copy_arr(d->edges_on_vertex, 3 * (size_t)V, "edges_on_vertex");
  m.cov = copy_arr(d->cells_on_vertex, 3 * (size_t)V, "cells_on_vertex");
  m.kite = copy_arr(d->kite_areas_on_vertex, 3 * (size_t)V, "kite_areas_on_vertex");
  m.dc = copy_arr(d->dc_edge, E, "dc_edge");
  m.dv = copy_arr(d->dv_edge, E, "dv_edge");
  m.A = copy_arr(d->area_cell, N, "area_cell");
  m.Av = copy_arr(d->area_triangle, V, "area_triangle");
  m.fv = copy_arr(d->f_vertex, V, "f_vertex");
  m.fe = copy_arr(d->f_edge, E, "f_edge");
  m.H = copy_arr(d->bottom_depth, N, "bottom_depth");

  // index ranges and incidence
  for (int e = 0; e < E; ++e) {
    const int c0 = m.coe[2 * e], c1 = m.coe[2 * e + 1], v0 = m.voe[2 * e], v1 = m.voe[2 * e + 1];
    if (c0 < 0 || c0 >= N || c1 < 0 || c1 >= N || c0 == c1) fail("mesh: bad cells_on_edge at " + at("edge", e));
    if (v0 < 0 || v0 >= V || v1 < 0 || v1 >= V || v0 == v1) fail("mesh: bad vertices_on_edge at " + at("edge", e));
    if (!(m.dc[e] > 0) || !(m.dv[e] > 0) || !std::isfinite(m.dc[e]) || !std::isfinite(m.dv[e]))
      fail("mesh: non-positive dc_edge/dv_edge at " + at("edge", e));
    if (!std::isfinite(m.fe[e])) fail("mesh: non-finite f_edge at " + at("edge", e));
  }
  std::vector<int> seen(E, 0);
  for (int i = 0; i < N; ++i) {
    if (!(m.A[i] > 0) || !std::isfinite(m.A[i])) fail("mesh: non-positive area_cell at " + at("cell", i));
    if (!(m.H[i] > 0) || !std::isfinite(m.H[i])) fail("mesh: non-positive bottom_depth at " + at("cell", i));
    for (int k = m.eoc_off[i]; k < m.eoc_off[i + 1]; ++k) {
      const int e = m.eoc[k], v = m.voc[k];
      if (e < 0 || e >= E) fail("mesh: edges_on_cell out of range at " + at("cell", i));
      if (v < 0 || v >= V) fail("mesh: vertices_on_cell out of range at " + at("cell", i));
      if (m.coe[2 * e] != i && m.coe[2 * e + 1] != i)
        fail("mesh: edge " + std::to_string(e) + " listed on " + at("cell", i) + " does not touch it");
      seen[e]++;
    }
  }
  for (int e = 0; e < E; ++e)
    if (seen[e] != 2) fail("mesh: " + at("edge", e) + " appears on " + std::to_string(seen[e]) + " cells");
  for (int v = 0; v < V; ++v) {
    if (!(m.Av[v] > 0) || !std::isfinite(m.Av[v])) fail("mesh: non-positive area_triangle at " + at("vertex", v));
    if (!std::isfinite(m.fv[v])) fail("mesh: non-finite f_vertex at " + at("vertex", v));
    for (int j = 0; j < 3; ++j) {
      const int c = m.cov[3 * v + j], e = m.eov[3 * v + j];
      if (c < 0 || c >= N) fail("mesh: cells_on_vertex out of range at " + at("vertex", v));
      if (e < 0 || e >= E) fail("mesh: edges_on_vertex out of range at " + at("vertex", v));
      const int cn = m.cov[3 * v + (j + 1) % 3];
      const int a = m.coe[2 * e], b = m.coe[2 * e + 1];
      if (!((a == c && b == cn) || (a == cn && b == c)))
        fail("mesh: edges_on_vertex[j] does not join cells_on_vertex j and j+1 at " + at("vertex", v));
      if (m.voe[2 * e] != v && m.voe[2 * e + 1] != v)
        fail("mesh: vertices_on_edge does not contain " + at("vertex", v));
      if (!(m.kite[3 * v + j] > 0) || !std::isfinite(m.kite[3 * v + j]))
        fail("mesh: non-positive kite area at " + at("vertex", v));
    }
  }
  // orientation: traversing c0 -> c1 is counter-clockwise about v1, i.e. c1
  // follows c0 in the counter-clockwise cells_on_vertex list of v1.
  for (int e = 0; e < E; ++e) {
    const int c0 = m.coe[2 * e], c1 = m.coe[2 * e + 1];
    for (int side = 0; side < 2; ++side) {
      const int v = m.voe[2 * e + side];
      const int a = side ? c0 : c1, b = side ? c1 : c0;   // at v1: c0 then c1; at v0: c1 then c0
      bool ok = false;
      for (int j = 0; j < 3; ++j)
        if (m.cov[3 * v + j] == a && m.cov[3 * v + (j + 1) % 3] == b) ok = true;
      if (!ok) fail("mesh: vertices_on_edge orientation inconsistent with cells_on_vertex at " + at("edge", e));
    }
  }
  // cells: vertex j lies between edge j and edge j+1 (counter-clockwise)
  std::vector<double> kite_sum(N, 0.0);
  for (int v = 0; v < V; ++v)
    for (int j = 0; j < 3; ++j) kite_sum[m.cov[3 * v + j]] += m.kite[3 * v + j];
  for (int i = 0; i < N; ++i) {
    const int a = m.eoc_off[i], n = m.eoc_off[i + 1] - a;
    for (int j = 0; j < n; ++j) {
      const int v = m.voc[a + j], e0 = m.eoc[a + j], e1 = m.eoc[a + (j + 1) % n];
      const bool t0 = m.voe[2 * e0] == v || m.voe[2 * e0 + 1] == v;
      const bool t1 = m.voe[2 * e1] == v || m.voe[2 * e1 + 1] == v;
      if (!t0 || !t1) fail("mesh: vertex j is not between edges j and j+1 at " + at("cell", i));
      // counter-clockwise: edge j is shared with the cell that follows i around v
      int pos = -1;
      for (int k = 0; k < 3; ++k)
        if (m.cov[3 * v + k] == i) pos = k;
      if (pos < 0) fail("mesh: vertices_on_cell / cells_on_vertex mismatch at " + at("cell", i));
      const int next = m.cov[3 * v + (pos + 1) % 3];
      const int nb0 = m.coe[2 * e0] == i ? m.coe[2 * e0 + 1] : m.coe[2 * e0];
      if (nb0 != next) fail("mesh: edges_on_cell is not counter-clockwise at " + at("cell", i));
    }
    if (std::fabs(kite_sum[i] - m.A[i]) > 1e-9 * m.A[i]) fail("mesh: kite areas do not sum to area_cell at " + at("cell", i));
  }
  for (int v = 0; v < V; ++v) {
    const double s = m.kite[3 * v] + m.kite[3 * v + 1] + m.kite[3 * v + 2];
    if (std::fabs(s - m.Av[v]) > 1e-9 * m.Av[v]) fail("mesh: kite areas do not sum to area_triangle at " + at("vertex", v));
  }
  // edges_on_edge: the other edges of c0 then the other edges of c1
  for (int e = 0; e < E; ++e) {
    const int c0 = m.coe[2 * e], c1 = m.coe[2 * e + 1];
    const int n0 = m.eoc_off[c0 + 1] - m.eoc_off[c0], n1 = m.eoc_off[c1 + 1] - m.eoc_off[c1];
    if (m.eoe_off[e + 1] - m.eoe_off[e] != n0 - 1 + n1 - 1)
      fail("mesh: edges_on_edge count != deg(c0)+deg(c1)-2 at " + at("edge", e));
    for (int k = m.eoe_off[e]; k < m.eoe_off[e + 1]; ++k) {
      const int e2 = m.eoe[k];
      if (e2 < 0 || e2 >= E || e2 == e) fail("mesh: bad edges_on_edge entry at " + at("edge", e));
      const int a = m.coe[2 * e2], b = m.coe[2 * e2 + 1];
      if (a != c0 && b != c0 && a != c1 && b != c1) fail("mesh: edges_on_edge entry shares no cell at " + at("edge", e));
      if (!std::isfinite(m.woe[k])) fail("mesh: non-finite weight at " + at("edge", e));
    }
  }
}

// ------------------------------------------------------------------ layering

static std::vector<int> bfs_hops(const HostMesh& m, const std::vector<std::vector<int>>& nb,
                                 const std::vector<char>& src) {
  std::vector<int> d(m.N, -1);
  std::deque<int> q;
  for (int i = 0; i < m.N; ++i)
    if (src[i]) {
      d[i] = 0;
      q.push_back(i);
    }
  while (!q.empty()) {
    const int x = q.front();
    q.pop_front();
    for (int y : nb[x])
      if (d[y] < 0) {
        d[y] = d[x] + 1;
        q.push_back(y);
      }
  }
  return d;
}

static std::vector<std::vector<int>> cell_nbrs(const HostMesh& m) {
  std::vector<std::vector<int>> nb(m.N);
  for (int e = 0; e < m.E; ++e) {
    nb[m.coe[2 * e]].push_back(m.coe[2 * e + 1]);
    nb[m.coe[2 * e + 1]].push_back(m.coe[2 * e]);
  }
  return nb;
}

void layer_regions(const HostMesh& m, const int8_t* labels, bool binary, int r, std::vector<int8_t>& lab4,
                   std::vector<int>& layer) {
  if (!labels) fail("labels is NULL");
  if (r < 1 || r > 64) fail("r_layers must be in 1..64");
  const int N = m.N;
  lab4.assign(N, 3);
  std::vector<char> fine(N, 0), coarse(N, 0);
  for (int i = 0; i < N; ++i) {
    const int l = labels[i];
    if (binary) {
      if (l != 0 && l != 1) fail("binary labels must be 0 (fine) or 1 (coarse)");
      fine[i] = l == 0;
    } else {
      if (l < 0 || l > 3) fail("labels must be in 0..3 (F, IF-1, IF-2, interior)");
      fine[i] = l == 0;
    }
    coarse[i] = !fine[i];
  }
  const auto nb = cell_nbrs(m);
  const auto dF = bfs_hops(m, nb, fine);     // hops from the fine set
  const auto dC = bfs_hops(m, nb, coarse);   // hops from the coarse set
  layer.assign(N, 0);
  const int big = 1 << 20;
  for (int i = 0; i < N; ++i) {
    if (fine[i]) layer[i] = dC[i] < 0 ? -big : -dC[i];
    else layer[i] = dF[i] < 0 ? big : dF[i];
  }
  if (binary) {
    for (int i = 0; i < N; ++i) {
      if (fine[i]) lab4[i] = 0;
      else if (layer[i] <= r) lab4[i] = 1;
      else if (layer[i] <= 2 * r) lab4[i] = 2;
      else lab4[i] = 3;
    }
  } else {
    for (int i = 0; i < N; ++i) lab4[i] = labels[i];
  }
  // only neighbouring regions may touch (Section 2.2)
  for (int e = 0; e < m.E; ++e) {
    const int a = lab4[m.coe[2 * e]], b = lab4[m.coe[2 * e + 1]];
    if (std::abs(a - b) > 1)
      fail("region: cells " + std::to_string(m.coe[2 * e]) + " and " + std::to_string(m.coe[2 * e + 1]) +
           " are adjacent but " + std::to_string(std::abs(a - b)) + " regions apart");
  }
}

// -------------------------------------------------------------------- plan

namespace {

struct NewAdj {
  // new-numbered incidence, flattened
  std::vector<int> eoc_off, eoc, nbr;  // cells -> edges, neighbour across
  std::vector<int> coe, voe;           // edges -> cells, vertices
  std::vector<int> eoe_off, eoe;       // edges -> edges
  std::vector<int> eov, cov;           // vertices -> edges, cells
};

NewAdj new_adjacency(const HostMesh& m, const Plan& p) {
  NewAdj a;
  const int N = m.N, E = m.E, V = m.V;
  a.eoc_off.assign(N + 1, 0);
  for (int in = 0; in < N; ++in) {
    const int io = p.cell_new2old[in];
    a.eoc_off[in + 1] = a.eoc_off[in] + (m.eoc_off[io + 1] - m.eoc_off[io]);
  }
  a.eoc.resize(a.eoc_off[N]);
  a.nbr.resize(a.eoc_off[N]);
  for (int in = 0; in < N; ++in) {
    const int io = p.cell_new2old[in];
    int k = a.eoc_off[in];
    for (int t = m.eoc_off[io]; t < m.eoc_off[io + 1]; ++t, ++k) {
      const int eo = m.eoc[t];
      a.eoc[k] = p.edge_old2new[eo];
      const int other = m.coe[2 * eo] == io ? m.coe[2 * eo + 1] : m.coe[2 * eo];
      a.nbr[k] = p.cell_old2new[other];
    }
  }
  a.coe.resize(2 * (size_t)E);
  a.voe.resize(2 * (size_t)E);
  a.eoe_off.assign(E + 1, 0);
  for (int en = 0; en < E; ++en) {
    const int eo = p.edge_new2old[en];
    a.coe[2 * en] = p.cell_old2new[m.coe[2 * eo]];
    a.coe[2 * en + 1] = p.cell_old2new[m.coe[2 * eo + 1]];
    a.voe[2 * en] = p.vert_old2new[m.voe[2 * eo]];
    a.voe[2 * en + 1] = p.vert_old2new[m.voe[2 * eo + 1]];
    a.eoe_off[en + 1] = a.eoe_off[en] + (m.eoe_off[eo + 1] - m.eoe_off[eo]);
  }
  a.eoe.resize(a.eoe_off[E]);
  for (int en = 0; en < E; ++en) {
    const int eo = p.edge_new2old[en];
    int k = a.eoe_off[en];
    for (int t = m.eoe_off[eo]; t < m.eoe_off[eo + 1]; ++t, ++k) a.eoe[k] = p.edge_old2new[m.eoe[t]];
  }
  a.eov.resize(3 * (size_t)V);
  a.cov.resize(3 * (size_t)V);
  for (int vn = 0; vn < V; ++vn) {
    const int vo = p.vert_new2old[vn];
    for (int j = 0; j < 3; ++j) {
      a.eov[3 * vn + j] = p.edge_old2new[m.eov[3 * vo + j]];
      a.cov[3 * vn + j] = p.cell_old2new[m.cov[3 * vo + j]];
    }
  }
  return a;
}

// What one stage's four passes read, given their ranges.  Used to grow the
// preceding stage's ranges (suffix) or to size a stage's own auxiliary
// passes (prefix).
struct Reads {
  int min_cell = INT32_MAX, max_cell = -1;   // cells whose previous-stage h is read
  int min_edge = INT32_MAX, max_edge = -1;   // edges whose previous-stage u is read
  void cell(int c) {
    min_cell = std::min(min_cell, c);
    max_cell = std::max(max_cell, c);
  }
  void edge(int e) {
    min_edge = std::min(min_edge, e);
    max_edge = std::max(max_edge, e);
  }
};

// Reads of the stage-input arrays (Hsrc / Usrc) by one stage with the given ranges.
Reads stage_input_reads(const NewAdj& a, const StageRanges& s, bool nonlinear) {
  Reads r;
  for (int i = s.cell.b; i < s.cell.e; ++i) {
    r.cell(i);  // hs uses Hsrc of the cell itself
    const bool psi = (i >= s.cell_upd.b && i < s.cell_upd.e) || (i >= s.cell_acc.b && i < s.cell_acc.e);
    for (int k = a.eoc_off[i]; k < a.eoc_off[i + 1]; ++k) {
      if (nonlinear || psi) r.edge(a.eoc[k]);           // K and Psi read u of the cell's edges
      if (psi && nonlinear) r.cell(a.nbr[k]);           // Psi reads h of neighbours
    }
  }
  if (nonlinear)
    for (int v = s.vert.b; v < s.vert.e; ++v)
      for (int j = 0; j < 3; ++j) r.edge(a.eov[3 * v + j]);
  for (int e = s.prep.b; e < s.prep.e; ++e) r.edge(e);
  for (int e = s.edge.b; e < s.edge.e; ++e) r.edge(e);  // drag reads u of the edge
  return r;
}

// Auxiliary pass ranges (prep, vertex, cell-derive) implied by an edge pass
// over edges [eb, ee): returns the min and max index each pass must cover.
struct Aux {
  int pmin = INT32_MAX, pmax = -1, vmin = INT32_MAX, vmax = -1, cmin = INT32_MAX, cmax = -1;
};

Aux aux_for_edges(const NewAdj& a, int eb, int ee, bool nonlinear) {
  Aux x;
  auto pe = [&](int e) {
    x.pmin = std::min(x.pmin, e);
    x.pmax = std::max(x.pmax, e);
  };
  for (int e = eb; e < ee; ++e) {
    pe(e);
    for (int k = a.eoe_off[e]; k < a.eoe_off[e + 1]; ++k) pe(a.eoe[k]);
    for (int j = 0; j < 2; ++j) {   // B at the edge's cells
      x.cmin = std::min(x.cmin, a.coe[2 * e + j]);
      x.cmax = std::max(x.cmax, a.coe[2 * e + j]);
    }
  }
  if (x.pmax < 0) return x;
  for (int e = x.pmin; e <= x.pmax; ++e)
    for (int j = 0; j < 2; ++j) {
      if (nonlinear) {
        x.cmin = std::min(x.cmin, a.coe[2 * e + j]);   // h_e from h* of both cells
        x.cmax = std::max(x.cmax, a.coe[2 * e + j]);
        x.vmin = std::min(x.vmin, a.voe[2 * e + j]);   // q at both vertices
        x.vmax = std::max(x.vmax, a.voe[2 * e + j]);
      }
    }
  if (nonlinear && x.vmax >= 0)
    for (int v = x.vmin; v <= x.vmax; ++v)
      for (int j = 0; j < 3; ++j) {
        x.cmin = std::min(x.cmin, a.cov[3 * v + j]);
        x.cmax = std::max(x.cmax, a.cov[3 * v + j]);
      }
  return x;
}

}  // namespace

void build_plan(const HostMesh& m, const std::vector<int8_t>& lab4, const std::vector<int>& layer, bool fblts,
                bool nonlinear, int r, Plan& p, bool full_coarse) {
  const int N = m.N, E = m.E, V = m.V;
  // ---- cell order: region, then hop distance to the other region (clamped so
  // deep cells keep the caller's locality order), then caller index.
  const int fine_clamp = 6 * r, coarse_clamp = 2 * r + 3;
  std::vector<long> ckey(N);
  for (int i = 0; i < N; ++i) {
    int l = fblts ? layer[i] : 0;
    l = std::max(-fine_clamp, std::min(coarse_clamp, l));
    const int lab = fblts ? lab4[i] : 3;
    ckey[i] = (long)lab * 1000 + (l + 500);
  }
  p.cell_new2old.resize(N);
  std::iota(p.cell_new2old.begin(), p.cell_new2old.end(), 0);
  std::stable_sort(p.cell_new2old.begin(), p.cell_new2old.end(), [&](int a, int b) { return ckey[a] < ckey[b]; });
  p.cell_old2new.resize(N);
  for (int i = 0; i < N; ++i) p.cell_old2new[p.cell_new2old[i]] = i;
  // ---- edges by their lower new cell (then the other); vertices likewise
  std::vector<std::pair<long, int>> ek(E);
  for (int e = 0; e < E; ++e) {
    const int a = p.cell_old2new[m.coe[2 * e]], b = p.cell_old2new[m.coe[2 * e + 1]];
    ek[e] = {(long)std::min(a, b) * N + std::max(a, b), e};
  }
  std::sort(ek.begin(), ek.end());
  p.edge_new2old.resize(E);
  p.edge_old2new.resize(E);
  for (int en = 0; en < E; ++en) {
    p.edge_new2old[en] = ek[en].second;
    p.edge_old2new[ek[en].second] = en;
  }
  std::vector<std::pair<long, int>> vk(V);
  for (int v = 0; v < V; ++v) {
    int c[3];
    for (int j = 0; j < 3; ++j) c[j] = p.cell_old2new[m.cov[3 * v + j]];
    std::sort(c, c + 3);
    vk[v] = {((long)c[0] * N + c[1]) * 4 + (c[2] % 4), v};
  }
  std::sort(vk.begin(), vk.end());
  p.vert_new2old.resize(V);
  p.vert_old2new.resize(V);
  for (int vn = 0; vn < V; ++vn) {
    p.vert_new2old[vn] = vk[vn].second;
    p.vert_old2new[vk[vn].second] = vn;
  }
  // ---- labels and region counts in new numbering
  p.cell_lab.resize(N);
  p.edge_lab.resize(E);
  int cnt[4] = {0, 0, 0, 0}, ecnt[4] = {0, 0, 0, 0};
  for (int in = 0; in < N; ++in) {
    p.cell_lab[in] = fblts ? lab4[p.cell_new2old[in]] : 3;
    cnt[p.cell_lab[in]]++;
  }
  for (int en = 0; en < E; ++en) {
    const int eo = p.edge_new2old[en];
    const int l = std::min(fblts ? lab4[m.coe[2 * eo]] : 3, fblts ? lab4[m.coe[2 * eo + 1]] : 3);
    p.edge_lab[en] = (int8_t)l;
    ecnt[l]++;
  }
  for (int en = 1; en < E; ++en)
    if (p.edge_lab[en] < p.edge_lab[en - 1]) fail("internal: edge order is not region-contiguous");
  p.nF = cnt[0];
  p.nIF1 = cnt[1];
  p.nIF2 = cnt[2];
  p.nINT = cnt[3];
  p.nFE = ecnt[0];
  p.nIF1E = ecnt[1];
  p.nIF2E = ecnt[2];
  p.nINTE = ecnt[3];
  const NewAdj a = new_adjacency(m, p);
  const int nIF = p.nF + p.nIF1 + p.nIF2, nIFE = p.nFE + p.nIF1E + p.nIF2E;

  if (!fblts) {
    for (int s = 0; s < 3; ++s) {
      StageRanges& R = p.coarse[s];
      R.cell = R.cell_upd = {0, N};
      R.cell_acc = {0, 0};
      R.vert = {0, nonlinear ? V : 0};
      R.prep = {0, E};
      R.edge = R.edge_upd = {0, E};
      R.edge_acc = {0, 0};
      p.fine[s] = StageRanges();
    }
    return;
  }

  // ---- stencil condition (Section 2.2): the fine updates must read only fine
  // and interface-one data; interface-two updates must not read fine data.
  {
    Aux xf = aux_for_edges(a, 0, p.nFE, nonlinear);
    std::vector<int> cells, edges;
    if (xf.pmax >= 0) {
      for (int e = 0; e < p.nFE; ++e) {
        edges.push_back(e);
        for (int k = a.eoe_off[e]; k < a.eoe_off[e + 1]; ++k) {
          const int e2 = a.eoe[k];
          edges.push_back(e2);
          for (int j = 0; j < 2; ++j) {
            if (nonlinear) {
              cells.push_back(a.coe[2 * e2 + j]);
              const int v = a.voe[2 * e2 + j];
              for (int t = 0; t < 3; ++t) {
                cells.push_back(a.cov[3 * v + t]);
                edges.push_back(a.eov[3 * v + t]);
              }
            }
          }
        }
        for (int j = 0; j < 2; ++j) {
          const int c = a.coe[2 * e + j];
          cells.push_back(c);
          for (int k = a.eoc_off[c]; k < a.eoc_off[c + 1]; ++k) edges.push_back(a.eoc[k]);
        }
      }
    }
    for (int c : cells)
      if (p.cell_lab[c] > 1)
        fail("region: the fine-edge stencil reaches interface two (cell " + std::to_string(p.cell_new2old[c]) +
             "); interface one must be thicker (Section 2.2 stencil condition)");
    for (int e : edges)
      if (p.edge_lab[e] > 1)
        fail("region: the fine-edge stencil reaches an interface-two edge (edge " + std::to_string(p.edge_new2old[e]) +
             "); interface one must be thicker");
    // interface-two edges must not see the fine region
    for (int e = p.nFE + p.nIF1E; e < nIFE; ++e)
      for (int k = a.eoe_off[e]; k < a.eoe_off[e + 1]; ++k) {
        const int e2 = a.eoe[k];
        for (int j = 0; j < 2; ++j) {
          if (p.cell_lab[a.coe[2 * e2 + j]] == 0)
            fail("region: an interface-two edge stencil reaches the fine region; interface two must be thicker");
          const int v = a.voe[2 * e2 + j];
          for (int t = 0; t < 3; ++t)
            if (nonlinear && p.cell_lab[a.cov[3 * v + t]] == 0)
              fail("region: an interface-two edge stencil reaches the fine region; interface two must be thicker");
        }
      }
  }

  // ---- fine substep: prefix ranges
  for (int s = 0; s < 3; ++s) {
    StageRanges& R = p.fine[s];
    const int ee = (s < 2) ? p.nFE : nIFE;
    R.edge = {0, ee};
    R.edge_upd = {0, p.nFE};
    R.edge_acc = (s == 2) ? Range{p.nFE, nIFE} : Range{0, 0};
    const Aux x = aux_for_edges(a, 0, ee, nonlinear);
    R.prep = {0, x.pmax + 1};
    R.vert = {0, nonlinear ? x.vmax + 1 : 0};
    int ce = std::max(x.cmax + 1, (s < 2) ? p.nF : nIF);
    R.cell = {0, ce};
    R.cell_upd = {0, p.nF};
    R.cell_acc = (s == 2) ? Range{p.nF, nIF} : Range{0, 0};
  }
  {
    const Reads rd = stage_input_reads(a, p.fine[2], nonlinear);
    p.fine3_cell_end = std::max(rd.max_cell + 1, p.fine[2].cell.e);
    p.fine3_edge_end = std::max(rd.max_edge + 1, p.fine[2].edge.e);
  }

  // ---- coarse advancement: suffix ranges by backward closure.  Every coarse
  // stage value is kept on the whole coarse region (the fine substeps read the
  // interface-two and interior values as aliases, interface one as prediction
  // input, the interior as the final value).
  int need_c = p.nF, need_e = p.nFE;      // coarse cells / edges: [nF,N), [nFE,E)
  int cell_min_next = need_c, edge_min_next = need_e;
  for (int s = 2; s >= 0; --s) {
    StageRanges& R = p.coarse[s];
    const int eb = std::min(need_e, edge_min_next);
    R.edge = R.edge_upd = {eb, E};
    R.edge_acc = {0, 0};
    const Aux x = aux_for_edges(a, eb, E, nonlinear);
    R.prep = {x.pmax >= 0 ? x.pmin : E, E};
    R.vert = {nonlinear && x.vmax >= 0 ? x.vmin : V, nonlinear ? V : V};
    const int cb = std::min({need_c, cell_min_next, x.cmax >= 0 ? x.cmin : N});
    R.cell = R.cell_upd = {cb, N};
    R.cell_acc = {0, 0};
    const Reads rd = stage_input_reads(a, R, nonlinear);
    cell_min_next = std::min(need_c, rd.min_cell);
    edge_min_next = std::min(need_e, rd.min_edge);
  }
  // definition mode (used by the adjoint's recording forward): the coarse
  // advancement is evaluated on every cell, edge and vertex
  if (full_coarse)
    for (int s = 0; s < 3; ++s) {
      StageRanges& R = p.coarse[s];
      R.cell = R.cell_upd = {0, N};
      R.vert = {0, nonlinear ? V : 0};
      R.prep = {0, E};
      R.edge = R.edge_upd = {0, E};
    }
  // deepest fine layer reached by the coarse sweep (for reporting against F^5)
  int deepest = 0;
  for (int i = p.coarse[0].cell.b; i < p.nF; ++i)
    deepest = std::max(deepest, -layer[p.cell_new2old[i]]);
  p.fine_depth_max = deepest;
}

// --------------------------------------------------------------- permutation

static int round_up(int x, int a) { return (x + a - 1) / a * a; }

void permute_mesh(const HostMesh& m, const Plan& p, PermMesh& pm) {
  const int N = m.N, E = m.E, V = m.V;
  pm.N = N;
  pm.E = E;
  pm.V = V;
  pm.cs = round_up(N, 64);
  pm.es = round_up(E, 64);
  pm.vs = round_up(V, 64);
  int maxE = 0, maxEOE = 0;
  for (int i = 0; i < N; ++i) maxE = std::max(maxE, m.eoc_off[i + 1] - m.eoc_off[i]);
  for (int e = 0; e < E; ++e) maxEOE = std::max(maxEOE, m.eoe_off[e + 1] - m.eoe_off[e]);
  // the gather kernels unroll the first kUnrollCell / kUnrollEOE slots with no
  // bounds test: pad the lists to at least that width with harmless entries
  maxE = std::max(maxE, kUnrollCell);
  maxEOE = std::max(maxEOE, kUnrollEOE);
  pm.maxE = maxE;
  pm.maxEOE = maxEOE;
  pm.c_nedge.assign(N, 0);
  pm.c_edge.assign((size_t)maxE * pm.cs, 0);
  pm.c_nbr.assign((size_t)maxE * pm.cs, 0);
  pm.c_invA.resize(N);
  pm.c_A.resize(N);
  pm.c_H.resize(N);
  for (int in = 0; in < N; ++in) {
    const int io = p.cell_new2old[in];
    const int b = m.eoc_off[io], n = m.eoc_off[io + 1] - b;
    pm.c_nedge[in] = n;
    for (int j = n; j < maxE; ++j) {   // padding repeats slot 0; the kernel masks it out
      const int eo = m.eoc[b];
      const bool outward = m.coe[2 * eo] == io;
      pm.c_edge[(size_t)j * pm.cs + in] = 2 * p.edge_old2new[eo] + (outward ? 0 : 1);
      pm.c_nbr[(size_t)j * pm.cs + in] = p.cell_old2new[outward ? m.coe[2 * eo + 1] : m.coe[2 * eo]];
    }
    for (int j = 0; j < n; ++j) {
      const int eo = m.eoc[b + j];
      const int en = p.edge_old2new[eo];
      const bool outward = m.coe[2 * eo] == io;   // n_{e,i} = +1 when n_e points out of i
      pm.c_edge[(size_t)j * pm.cs + in] = 2 * en + (outward ? 0 : 1);
      const int other = outward ? m.coe[2 * eo + 1] : m.coe[2 * eo];
      pm.c_nbr[(size_t)j * pm.cs + in] = p.cell_old2new[other];
    }
    pm.c_A[in] = m.A[io];
    pm.c_invA[in] = 1.0 / m.A[io];
    pm.c_H[in] = m.H[io];
  }
  pm.e_cell.assign(2 * (size_t)pm.es, 0);
  pm.e_vert.assign(2 * (size_t)pm.es, 0);
  pm.e_dc.resize(E);
  pm.e_dv.resize(E);
  pm.e_invdc.resize(E);
  pm.e_He.resize(E);
  pm.e_neoe.resize(E);
  pm.e_eoe.assign((size_t)maxEOE * pm.es, 0);
  pm.e_w.assign((size_t)maxEOE * pm.es, 0.0);
  for (int en = 0; en < E; ++en) {
    const int eo = p.edge_new2old[en];
    pm.e_cell[en] = p.cell_old2new[m.coe[2 * eo]];
    pm.e_cell[pm.es + en] = p.cell_old2new[m.coe[2 * eo + 1]];
    pm.e_vert[en] = p.vert_old2new[m.voe[2 * eo]];
    pm.e_vert[pm.es + en] = p.vert_old2new[m.voe[2 * eo + 1]];
    pm.e_dc[en] = m.dc[eo];
    pm.e_dv[en] = m.dv[eo];
    pm.e_invdc[en] = 1.0 / m.dc[eo];
    pm.e_He[en] = 0.5 * (m.H[m.coe[2 * eo]] + m.H[m.coe[2 * eo + 1]]);
    const int b = m.eoe_off[eo], n = m.eoe_off[eo + 1] - b;
    pm.e_neoe[en] = n;
    for (int j = n; j < maxEOE; ++j) {   // padding: the edge itself with weight 0
      pm.e_eoe[(size_t)j * pm.es + en] = en;
      pm.e_w[(size_t)j * pm.es + en] = 0.0;
    }
    for (int j = 0; j < n; ++j) {
      pm.e_eoe[(size_t)j * pm.es + en] = p.edge_old2new[m.eoe[b + j]];
      pm.e_w[(size_t)j * pm.es + en] = m.woe[b + j];
    }
  }
  // transposed weights: w_{e2,e} where e2 is slot j of e's list
  pm.e_wT.assign((size_t)maxEOE * pm.es, 0.0);
  {
    std::vector<std::pair<long, double>> wl;   // key e*E+e2 -> w_{e,e2}
    wl.reserve(m.eoe.size());
    for (int eo = 0; eo < E; ++eo)
      for (int t = m.eoe_off[eo]; t < m.eoe_off[eo + 1]; ++t) wl.push_back({(long)eo * E + m.eoe[t], m.woe[t]});
    std::sort(wl.begin(), wl.end());
    for (int en = 0; en < E; ++en) {
      const int eo = p.edge_new2old[en];
      for (int j = 0; j < pm.e_neoe[en]; ++j) {
        const int e2o = m.eoe[m.eoe_off[eo] + j];
        const long key = (long)e2o * E + eo;
        auto it = std::lower_bound(wl.begin(), wl.end(), std::make_pair(key, -1e300));
        if (it == wl.end() || it->first != key) fail("mesh: edges_on_edge is not symmetric (needed by the adjoint)");
        pm.e_wT[(size_t)j * pm.es + en] = it->second;
      }
    }
  }
  // cell -> vertex list with the cell's kite at each vertex
  pm.c_vert.assign((size_t)maxE * pm.cs, 0);
  pm.c_kite.assign((size_t)maxE * pm.cs, 0.0);
  {
    std::vector<std::pair<long, double>> kl;   // key cell*V+vertex -> kite
    kl.reserve(3 * (size_t)V);
    for (int v = 0; v < V; ++v)
      for (int j = 0; j < 3; ++j) kl.push_back({(long)m.cov[3 * v + j] * V + v, m.kite[3 * v + j]});
    std::sort(kl.begin(), kl.end());
    for (int in = 0; in < N; ++in) {
      const int io = p.cell_new2old[in];
      const int b = m.voc_off[io], n = m.voc_off[io + 1] - b;
      for (int j = 0; j < maxE; ++j) {
        const int vo = m.voc[b + (j < n ? j : 0)];
        pm.c_vert[(size_t)j * pm.cs + in] = p.vert_old2new[vo];
        if (j < n) {
          const long key = (long)io * V + vo;
          auto it = std::lower_bound(kl.begin(), kl.end(), std::make_pair(key, -1e300));
          pm.c_kite[(size_t)j * pm.cs + in] = it->second;
        }
      }
    }
  }
  // kite fractions per cell slot and the per-edge slot/degree word; then check
  // that the mesh's edges_on_edge lists and weights are the cell walks
  pm.c_R.assign((size_t)maxE * pm.cs, 0.0);
  for (int in = 0; in < N; ++in) {
    const int n = pm.c_nedge[in];
    for (int j = 0; j < n; ++j) pm.c_R[(size_t)j * pm.cs + in] = pm.c_kite[(size_t)j * pm.cs + in] / pm.c_A[in];
  }
  pm.e_cs.assign(E, 0);
  pm.kite_weights = maxE <= 15 ? 2 : 0;
  for (int in = 0; in < N && pm.kite_weights; ++in) {
    const int n = pm.c_nedge[in];
    if (n < 3) pm.kite_weights = 0;
    for (int j = 0; j < n; ++j) {
      const int en = pm.c_edge[(size_t)j * pm.cs + in] >> 1;
      const int side = pm.e_cell[en] == in ? 0 : 1;
      pm.e_cs[en] |= (j | (n << 4)) << (8 * side);
    }
  }
  for (int en = 0; en < E && pm.kite_weights; ++en) {
    int k = 0;
    for (int side = 0; side < 2 && pm.kite_weights; ++side) {
      const int in = pm.e_cell[(size_t)side * pm.es + en];
      const int w = (pm.e_cs[en] >> (8 * side)) & 0xff, j0 = w & 15, n = w >> 4;
      if (n != pm.c_nedge[in] || j0 >= n || (pm.c_edge[(size_t)j0 * pm.cs + in] >> 1) != en) {
        pm.kite_weights = 0;   // e.g. an edge whose two cells coincide
        break;
      }
      const int se = pm.c_edge[(size_t)j0 * pm.cs + in] & 1;
      double acc = 0.0;
      int j = j0;
      for (int mm = 1; mm < n; ++mm, ++k) {
        const int jp = j;
        j = j + 1 == n ? 0 : j + 1;
        acc = acc + pm.c_R[(size_t)jp * pm.cs + in];
        const int code = pm.c_edge[(size_t)j * pm.cs + in];
        double wt = 0.5 - acc;
        if ((code & 1) != se) wt = -wt;
        if (k >= pm.e_neoe[en] || pm.e_eoe[(size_t)k * pm.es + en] != (code >> 1)) {
          pm.kite_weights = 0;
          break;
        }
        const double d = std::fabs(wt - pm.e_w[(size_t)k * pm.es + en]);
        if (d != 0.0) pm.kite_weights = d <= 1e-13 ? std::min(pm.kite_weights, 1) : 0;
      }
    }
    if (k != pm.e_neoe[en]) pm.kite_weights = 0;
  }
  pm.v_edge.assign(3 * (size_t)pm.vs, 0);
  pm.v_cell.assign(3 * (size_t)pm.vs, 0);
  pm.v_kite.assign(3 * (size_t)pm.vs, 0.0);
  pm.v_invA.resize(V);
  pm.v_A.resize(V);
  pm.v_f.resize(V);
  pm.v_q0.resize(V);
  for (int vn = 0; vn < V; ++vn) {
    const int vo = p.vert_new2old[vn];
    double Hv = 0.0;
    for (int j = 0; j < 3; ++j) {
      const int eo = m.eov[3 * vo + j];
      // circulation sign: +1 at v1 (c0 -> c1 is counter-clockwise about v1)
      const bool pos = m.voe[2 * eo + 1] == vo;
      pm.v_edge[(size_t)j * pm.vs + vn] = 2 * p.edge_old2new[eo] + (pos ? 0 : 1);
      pm.v_cell[(size_t)j * pm.vs + vn] = p.cell_old2new[m.cov[3 * vo + j]];
      pm.v_kite[(size_t)j * pm.vs + vn] = m.kite[3 * vo + j];
      Hv += m.kite[3 * vo + j] * m.H[m.cov[3 * vo + j]];
    }
    pm.v_A[vn] = m.Av[vo];
    pm.v_invA[vn] = 1.0 / m.Av[vo];
    pm.v_f[vn] = m.fv[vo];
    pm.v_q0[vn] = m.fv[vo] / (Hv / m.Av[vo]);
  }
}

// ---------------------------------------------------------------- byte model

namespace {
struct Stamp {
  std::vector<int> s;
  int gen = 0;
  explicit Stamp(size_t n) : s(n, 0) {}
  void next() { ++gen; }
  bool mark(int i) {
    if (s[i] == gen) return false;
    s[i] = gen;
    return true;
  }
};
}  // namespace

double bytes_cell_pass(const PermMesh& pm, const StageRanges& r, bool nonlinear, int nm, bool ke) {
  const double S = 8.0 * nm;
  double b = 0;
  Stamp se(pm.E), sc(pm.N);
  se.next();
  sc.next();
  for (int i = r.cell.b; i < r.cell.e; ++i) sc.mark(i);
  for (int i = r.cell.b; i < r.cell.e; ++i) {
    const bool upd = i >= r.cell_upd.b && i < r.cell_upd.e;
    const bool acc = i >= r.cell_acc.b && i < r.cell_acc.e;
    const bool psi = upd || acc;
    const int n = pm.c_nedge[i];
    b += 4 + 8 + 8;                                // nedge, 1/A, H
    if (nonlinear || psi) b += 4.0 * n;            // edge codes
    if (psi && nonlinear) b += 4.0 * n;            // neighbour codes
    b += S * 5;                                    // Hsrc, H0, Hnew (read or write), hs, B
    if (acc) b += 2 * S;
    for (int j = 0; j < n; ++j) {
      const int e = pm.c_edge[(size_t)j * pm.cs + i] >> 1;
      if ((nonlinear || psi) && se.mark(e)) b += S + 8 + ((nonlinear && !ke) ? 0 : 8);  // u, l, d (or He)
      if (psi && nonlinear) {
        const int nb = pm.c_nbr[(size_t)j * pm.cs + i];
        if (sc.mark(nb)) b += S;
      }
    }
  }
  return b;
}

double bytes_vert_pass(const PermMesh& pm, const Range& r, int nm) {
  const double S = 8.0 * nm;
  double b = 0;
  Stamp se(pm.E), sc(pm.N);
  se.next();
  sc.next();
  for (int v = r.b; v < r.e; ++v) {
    b += 3 * (4 + 4 + 8) + 8 + 8 + S;   // edge codes, cells, kites, 1/A_v, f_v, q write
    for (int j = 0; j < 3; ++j) {
      if (se.mark(pm.v_edge[(size_t)j * pm.vs + v] >> 1)) b += 8 + S;   // d_e, u
      if (sc.mark(pm.v_cell[(size_t)j * pm.vs + v])) b += S;            // h*
    }
  }
  return b;
}

double bytes_prep_pass(const PermMesh& pm, const Range& r, bool nonlinear, int nm, bool fuse_q) {
  const double S = 8.0 * nm;
  double b = 0;
  Stamp sc(pm.N), sv(pm.V), se(pm.E);
  sc.next();
  sv.next();
  se.next();
  for (int e = r.b; e < r.e; ++e) {
    b += 8 + 8 + 8 + S + 4 * S;   // cells, vertices, l_e, u, P write
    if (!nonlinear) b += 8;       // H_e
    if (nonlinear && fuse_q) b += 6 * (4 + 4);   // the vertices' edge codes and cells, copied per edge
    if (fuse_q) se.mark(e);
    for (int j = 0; j < 2; ++j) {
      const int c = pm.e_cell[(size_t)j * pm.es + e];
      if (nonlinear && sc.mark(c)) b += S;
      const int v = pm.e_vert[(size_t)j * pm.es + e];
      if (sv.mark(v)) {
        if (!nonlinear) {
          b += 8;   // static q0
        } else if (!fuse_q) {
          b += S;   // q from the vertex pass
        } else {
          // the vertex's own data: codes, cells, kites, 1/A_v, f_v; and its
          // edges' d_e, u and cells' h* when not already counted
          b += 3 * 8 + 8 + 8;   // kites, 1/A_v, f_v
          for (int t = 0; t < 3; ++t) {
            const int e2 = pm.v_edge[(size_t)t * pm.vs + v] >> 1;
            if (se.mark(e2)) b += 8 + S;    // d_e, u
            else b += 8;                    // d_e of an edge in the range
            if (sc.mark(pm.v_cell[(size_t)t * pm.vs + v])) b += S;
          }
        }
      }
    }
  }
  return b;
}

// Prep-record components a momentum pass references, each counted once per
// launch: the edge's own q_e (and h_e with drag or wind), each neighbour's
// l F and q_e (and l u with drag or wind).
struct RecordStamps {
  Stamp F, q, lu, he;
  explicit RecordStamps(int E) : F(E), q(E), lu(E), he(E) {
    F.next();
    q.next();
    lu.next();
    he.next();
  }
  double own(int e, bool need_u, double S) { return (q.mark(e) ? S : 0) + (need_u && he.mark(e) ? S : 0); }
  double nbr(int e, bool need_u, double S) {
    return (F.mark(e) ? S : 0) + (q.mark(e) ? S : 0) + (need_u && lu.mark(e) ? S : 0);
  }
};

double bytes_edge_pass(const PermMesh& pm, const StageRanges& r, bool drag, bool wind, int nm) {
  const double S = 8.0 * nm;
  double b = 0;
  RecordStamps rs(pm.E);
  Stamp sc(pm.N);
  sc.next();
  for (int e = r.edge.b; e < r.edge.e; ++e) {
    const int n = pm.e_neoe[e];
    b += 4 + n * (4.0 + 8.0) + 8 + 8;       // count, edges_on_edge, weights, cells, 1/d_e
    const bool upd = e >= r.edge_upd.b && e < r.edge_upd.e;
    const bool acc = e >= r.edge_acc.b && e < r.edge_acc.e;
    if (upd) b += 2 * S;                     // U0, Udst
    if (acc) b += 2 * S;
    if (drag || wind) b += S;                // u of the edge
    if (wind) b += 3 * S;                    // wind components and C_W (per member)
    b += rs.own(e, drag || wind, S);
    for (int j = 0; j < n; ++j) b += rs.nbr(pm.e_eoe[(size_t)j * pm.es + e], drag || wind, S);
    for (int j = 0; j < 2; ++j)
      if (sc.mark(pm.e_cell[(size_t)j * pm.es + e])) b += S + (drag ? S : 0);   // B (+ C_D)
  }
  return b;
}

double bytes_edge_cells_pass(const PermMesh& pm, const StageRanges& r, bool drag, bool wind, int nm) {
  const double S = 8.0 * nm;
  double b = 0;
  RecordStamps rs(pm.E);
  Stamp sc(pm.N);
  sc.next();
  for (int e = r.edge.b; e < r.edge.e; ++e) {
    b += 8 + 4 + 8;                          // cells, slot/degree word, 1/d_e
    const bool upd = e >= r.edge_upd.b && e < r.edge_upd.e;
    const bool acc = e >= r.edge_acc.b && e < r.edge_acc.e;
    if (upd) b += 2 * S;                     // U0, Udst
    if (acc) b += 2 * S;
    if (drag || wind) b += S;                // u of the edge
    if (wind) b += 3 * S;                    // wind components and C_W (per member)
    b += rs.own(e, drag || wind, S);
    for (int j = 0; j < 2; ++j) {
      const int c = pm.e_cell[(size_t)j * pm.es + e];
      if (sc.mark(c)) {
        const int n = pm.c_nedge[c];
        b += S + (drag ? S : 0) + 4 + n * (4.0 + 8.0);   // B (+ C_D), degree, edge codes, R
        for (int k = 0; k < n; ++k) {   // the walk reads the cell's other edges
          const int e2 = pm.c_edge[(size_t)k * pm.cs + c] >> 1;
          if (e2 != e) b += rs.nbr(e2, drag || wind, S);
        }
      }
    }
  }
  return b;
}

double bytes_edge_fast_pass(const PermMesh& pm, const StageRanges& r, bool slow, int nm) {
  const double S = 8.0 * nm;
  double b = 0;
  Stamp sc(pm.N);
  sc.next();
  for (int e = r.edge.b; e < r.edge.e; ++e) {
    b += 8 + 8;                              // cells, 1/d_e
    const bool upd = e >= r.edge_upd.b && e < r.edge_upd.e;
    const bool acc = e >= r.edge_acc.b && e < r.edge_acc.e;
    if (upd) b += 2 * S;                     // U0, Udst
    if (acc) b += 2 * S;
    if (slow) b += S;
    for (int j = 0; j < 2; ++j)
      if (sc.mark(pm.e_cell[(size_t)j * pm.es + e])) b += S;   // B
  }
  return b;
}

// ------------------------------------------------- compulsory byte model

double compulsory_cell_pass(const PermMesh& pm, const StageRanges& r, bool nonlinear, int nm, bool ke) {
  const double S = 8.0 * nm;
  double b = 0;
  Stamp se(pm.E), sc(pm.N);
  se.next();
  sc.next();
  for (int i = r.cell.b; i < r.cell.e; ++i) sc.mark(i);
  for (int i = r.cell.b; i < r.cell.e; ++i) {
    const bool upd = i >= r.cell_upd.b && i < r.cell_upd.e;
    const bool acc = i >= r.cell_acc.b && i < r.cell_acc.e;
    const bool psi = upd || acc;
    const int n = pm.c_nedge[i];
    b += 4 + 8 + 8;                                // degree, 1/A, resting depth
    if (nonlinear || psi) b += 4.0 * n;            // edges (with their orientation signs)
    if (psi && nonlinear) b += 4.0 * n;            // neighbour cells
    b += 3 * S;                                    // h of the stage, h^n, the new h (read or written)
    if (acc) b += 2 * S;
    for (int j = 0; j < n; ++j) {
      const int e = pm.c_edge[(size_t)j * pm.cs + i] >> 1;
      if ((nonlinear || psi) && se.mark(e)) b += S + 8 + ((nonlinear && !ke) ? 0 : 8);  // u, l, d (or H_e)
      if (psi && nonlinear) {
        const int nb = pm.c_nbr[(size_t)j * pm.cs + i];
        if (sc.mark(nb)) b += S;                   // neighbour h
      }
    }
  }
  return b;
}

double compulsory_vert_pass(const PermMesh& pm, const Range& r, int nm) {
  const double S = 8.0 * nm;
  double b = 0;
  Stamp se(pm.E);
  se.next();
  for (int v = r.b; v < r.e; ++v) {
    b += 3 * (4 + 4 + 8) + 8 + 8;   // edges, cells, kites, 1/A_v, f_v
    for (int j = 0; j < 3; ++j)
      if (se.mark(pm.v_edge[(size_t)j * pm.vs + v] >> 1)) b += 8 + S;   // d_e, u
  }
  return b;
}

double compulsory_prep_pass(const PermMesh& pm, const Range& r, bool nonlinear, int nm) {
  const double S = 8.0 * nm;
  double b = 0;
  for (int e = r.b; e < r.e; ++e) {
    b += 8 + 8 + 8 + S;             // cells, vertices, l_e, u
    if (!nonlinear) b += 8;         // H_e
  }
  return b;
}

double compulsory_edge_pass(const PermMesh& pm, const StageRanges& r, bool drag, bool wind, int nm) {
  const double S = 8.0 * nm;
  const bool tang = drag || wind;   // the tangential velocity reads the neighbours' u
  double b = 0;
  Stamp se(pm.E), sc(pm.N);
  se.next();
  sc.next();
  for (int e = r.edge.b; e < r.edge.e; ++e) {
    const int n = pm.e_neoe[e];
    b += 4 + n * (4.0 + 8.0) + 8 + 8;       // count, edges_on_edge, weights, cells, 1/d_e
    const bool upd = e >= r.edge_upd.b && e < r.edge_upd.e;
    const bool acc = e >= r.edge_acc.b && e < r.edge_acc.e;
    if (upd) b += 2 * S;                     // u^n, the new u
    if (acc) b += 2 * S;
    if (wind) b += 3 * S;                    // wind components and C_W (per member)
    if (tang) {
      if (se.mark(e)) b += S;                // u of the edge
      for (int j = 0; j < n; ++j)
        if (se.mark(pm.e_eoe[(size_t)j * pm.es + e])) b += S;
    }
    if (drag || wind)
      for (int j = 0; j < 2; ++j)
        if (sc.mark(pm.e_cell[(size_t)j * pm.es + e])) b += S + (drag ? S : 0);   // h (+ C_D) of the cells
  }
  return b;
}

double compulsory_edge_fast_pass(const PermMesh& pm, const StageRanges& r, bool slow, int nm) {
  const double S = 8.0 * nm;
  double b = 0;
  for (int e = r.edge.b; e < r.edge.e; ++e) {
    b += 8 + 8;                              // cells, 1/d_e
    const bool upd = e >= r.edge_upd.b && e < r.edge_upd.e;
    const bool acc = e >= r.edge_acc.b && e < r.edge_acc.e;
    if (upd) b += 2 * S;
    if (acc) b += 2 * S;
    if (slow) b += S;                        // the frozen slow tendency (state of the split scheme)
  }
  return b;
}

}  // namespace fblts
