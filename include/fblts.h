/*
 * fblts.h - C ABI of the FB-LTS shallow-water library for AMD MI355X (gfx950).
 *
 * The library advances the TRiSK shallow-water equations on an unstructured
 * Voronoi C-grid (thickness h on cells, normal velocity u on edges) with the
 * forward-backward local time-stepping scheme FB-LTS of Lilly, Capodaglio,
 * Engwirda, Higdon and Petersen (arXiv 2405.10505), and with the global
 * schemes FB-RK(3,2) and RK4 it is compared against.  All arithmetic is FP64.
 *
 * Paper passages (section / equation labels of the paper):
 *   - semi-discrete system u_e' = Phi_e(u,h), h_i' = Psi_i(u,h): Section 2.2,
 *     eq. semi_discrete_sys;
 *   - Psi: eq. trisk_thickness; Phi: eq. nonlinear_swe in the vorticity-flux
 *     form of eq. trisk_vorticity, with quadratic bottom drag and wind stress
 *     of eq. hurricane_model;
 *   - FB-RK(3,2): Section 2.1, eq. fbrk32, FB weights (0.531, 0.531, 0.313);
 *   - FB-LTS: Section 2.2 (regions F, IF-1, IF-2, interior coarse; coarse
 *     advancement, interface prediction eq. preds, fine advancement eq.
 *     fine_fbrk32, interface correction eq. if_correction);
 *   - conserved quantities: Section 2.4, Theorems 1 and 2.
 *
 * Conventions shared by every call:
 *   - Every function returns an int status (FBLTS_OK = 0, negative on error);
 *     fblts_last_error() gives a message for the last failure on the calling
 *     thread.  No C++ exception crosses this boundary.
 *   - Host pointers passed in are borrowed for the duration of the call and
 *     deep-copied; the caller keeps ownership.  Device pointers (on_device=1)
 *     must be device memory of the solver's device, at least the stated size,
 *     and are only accessed in stream order on the solver's stream.
 *   - All state going in and out is in the caller's numbering.  The library
 *     reorders cells, edges and vertices internally so that every LTS region
 *     is a contiguous range; that permutation never leaks out.
 *   - Work is enqueued asynchronously on the HIP stream given at create time.
 *     fblts_get_state (host pointers), fblts_diagnostics and the ensemble /
 *     adjoint host-returning calls synchronise that stream.
 *   - A handle must not be used from several threads at once.
 */
#ifndef FBLTS_H
#define FBLTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FBLTS_OK = 0,
  FBLTS_EINVAL = -1,     /* bad argument, malformed mesh, size mismatch          */
  FBLTS_ENOMEM = -2,     /* host or device allocation failed                      */
  FBLTS_EDEVICE = -3,    /* a HIP runtime call failed                             */
  FBLTS_EREGION = -4,    /* region labels violate the stencil condition (Sec 2.2) */
  FBLTS_ESTATE = -5,     /* call out of order (e.g. step before set_state)        */
  FBLTS_ENONFINITE = -6  /* the state holds NaN/Inf or h <= 0                     */
};

enum { FBLTS_SCHEME_FBLTS = 0, FBLTS_SCHEME_FBRK32 = 1, FBLTS_SCHEME_RK4 = 2 };
/* Physics: LINEAR = TRiSK linearised about rest; NONLINEAR = eq. nonlinear_swe
 * with optional drag and wind stress (eq. hurricane_model); GRAVITY_WAVE = the
 * fast terms only (eq. fast_terms: Psi = -div(h u), Phi = -g grad(h + z_b)),
 * the external gravity-wave system of Section 2.3 (eq. grav_wave_model). */
enum { FBLTS_PHYS_LINEAR = 0, FBLTS_PHYS_NONLINEAR = 1, FBLTS_PHYS_GRAVITY_WAVE = 2 };
/* Operator splitting of the momentum equation (Section 3.2, eq. splitting):
 * NONE = unsplit; COARSE = slow terms (everything in Phi but the pressure
 * gradient: PV flux, -grad K, drag, wind) evaluated once at t^n and held for
 * the whole step, every stage uses the fast terms plus that frozen value;
 * FINE = as COARSE, but the fine advancement re-evaluates the slow terms
 * before each substep k from the substep's starting state (the variant
 * Section 4.2 proposes).  Needs FBLTS_PHYS_NONLINEAR; COARSE also applies to
 * global FB-RK(3,2). */
enum { FBLTS_SPLIT_NONE = 0, FBLTS_SPLIT_COARSE = 1, FBLTS_SPLIT_FINE = 2 };
enum { FBLTS_LABEL_F = 0, FBLTS_LABEL_IF1 = 1, FBLTS_LABEL_IF2 = 2, FBLTS_LABEL_INT = 3 };

/* Message of the last failing call on this thread ("" if none).  Valid until
 * the next library call on the same thread. */
const char* fblts_last_error(void);
int fblts_version(void);

/* ---------------------------------------------------------------- mesh --- */

/* MPAS-style Voronoi C-grid, caller numbering, 0-based, host pointers.
 *   cells_on_edge[2E]      (c0,c1) per edge; the normal n_e points c0 -> c1,
 *                          so n_{e,c0} = +1, n_{e,c1} = -1 (Sec 2.4).
 *   vertices_on_edge[2E]   (v0,v1); the tangent t_e = k x n_e points v0 -> v1.
 *   edges_on_cell (CSR)    counter-clockwise; vertices_on_cell (CSR, same
 *                          offsets): vertex j lies between edge j and j+1.
 *   edges_on_edge (CSR) + weights_on_edge: dimensionless TRiSK weights
 *                          w_{e,e'}, u_perp_e = (1/d_e) sum w l_e' u_e'.
 *   edges_on_vertex[3V]    edge j joins cells_on_vertex j and j+1.
 *   cells_on_vertex[3V], kite_areas_on_vertex[3V] (aligned).
 *   dc_edge (d_e, cell-centre distance), dv_edge (l_e, edge length),
 *   area_cell (A_i), area_triangle (A_v), f_vertex, f_edge (Coriolis),
 *   bottom_depth (resting depth H_i > 0; bottom z_b = -H).
 */
typedef struct {
  int32_t n_cells, n_edges, n_vertices;
  const int32_t* cells_on_edge;
  const int32_t* vertices_on_edge;
  const int32_t* edges_on_cell_off;
  const int32_t* edges_on_cell;
  const int32_t* vertices_on_cell_off;
  const int32_t* vertices_on_cell;
  const int32_t* edges_on_edge_off;
  const int32_t* edges_on_edge;
  const double* weights_on_edge;
  const int32_t* edges_on_vertex;
  const int32_t* cells_on_vertex;
  const double* kite_areas_on_vertex;
  const double* dc_edge;
  const double* dv_edge;
  const double* area_cell;
  const double* area_triangle;
  const double* f_vertex;
  const double* f_edge;
  const double* bottom_depth;
} fblts_mesh_desc;

typedef struct fblts_mesh fblts_mesh;

/* Validate the descriptor (host only, no device needed) and deep-copy it.
 * Errors: FBLTS_EINVAL with a message naming the first violated property
 * (index ranges, CSR monotonicity, edge/cell incidence, orientation
 * consistency between cells, edges and vertices, positive lengths/areas,
 * kite sums).  *out is set only on success; free with fblts_mesh_destroy. */
int fblts_mesh_create(const fblts_mesh_desc* desc, fblts_mesh** out);
/* Destroy after every solver created from the mesh is destroyed. */
void fblts_mesh_destroy(fblts_mesh* mesh);

/* Region layering (Sec 2.2, host only).  labels[n_cells] in caller numbering:
 * binary=1: 0 = fine, 1 = coarse; the coarse cells within r hops of the fine
 * set become interface one, the next r hops interface two, the rest interior.
 * binary=0: labels are already FBLTS_LABEL_*.  Writes the 4-level labels to
 * out_labels[n_cells] and the signed layer distance to out_layer[n_cells]
 * (fine: -hops to the coarse set, coarse: +hops to the fine set; may be NULL).
 * Errors: FBLTS_EINVAL (bad values), FBLTS_EREGION (adjacent cells more than
 * one region apart, the stencil condition of Sec 2.2). */
/* Region plan (Sec 2.2 and the library's pass ranges; host only, no device):
 * what fblts_set_regions builds for FB-LTS from these labels.  Cells are
 * renumbered region by region (fine, interface one, interface two,
 * interior), edges by their lower cell; every pass runs on an index range of
 * that numbering.  Per FB-RK(3,2) stage s = 0, 1, 2: the coarse advancement
 * updates cells [coarse_cell_begin[s], n_cells) and edges
 * [coarse_edge_begin[s], n_edges); a fine substep's passes cover cells
 * [0, fine_cell_end[s]) and edges [0, fine_edge_end[s]) (each range closed
 * under the stencils of the stages after it).  nonlinear selects the
 * nonlinear stencils, which are wider than the linear ones.
 * Errors as fblts_layer_regions. */
typedef struct fblts_plan_info {
  int32_t n_cells, n_edges;
  int32_t n_fine, n_if1, n_if2, n_int;          /* cells per region */
  int32_t n_fine_e, n_if1_e, n_if2_e, n_int_e;  /* edges per region */
  int32_t coarse_cell_begin[3], coarse_edge_begin[3];
  int32_t fine_cell_end[3], fine_edge_end[3];
} fblts_plan_info;
int fblts_plan(const fblts_mesh* mesh, const int8_t* labels, int32_t binary, int32_t r, int32_t nonlinear,
               fblts_plan_info* out);

int fblts_layer_regions(const fblts_mesh* mesh, const int8_t* labels, int32_t binary, int32_t r,
                        int8_t* out_labels, int32_t* out_layer);

/* ------------------------------------------------------------- solver --- */

typedef struct {
  double dt;              /* coarse step (s); FB-RK(3,2)/RK4: the global step */
  double g;               /* gravity (m/s^2) */
  double beta1, beta2, beta3;   /* FB weights (Sec 2.1: 0.531, 0.531, 0.313) */
  int32_t M;              /* fine substeps per coarse step (FB-LTS) */
  int32_t scheme;         /* FBLTS_SCHEME_* */
  int32_t physics;        /* FBLTS_PHYS_* */
  int32_t r_layers;       /* interface thickness in cell layers for binary labels (2) */
  double rho_air, rho_water;    /* wind-stress law densities (1.15, 1000) */
  int32_t split;          /* FBLTS_SPLIT_* (0) */
  int32_t reserved;       /* 0 */
} fblts_params;

typedef struct fblts_solver fblts_solver;

/* Create a solver on the current HIP device, ordered on hip_stream (a
 * hipStream_t owned by the caller; NULL: the solver creates, and destroys
 * with itself, a non-blocking stream of its own, at the default priority).
 * Errors: FBLTS_EINVAL, FBLTS_EDEVICE. */
int fblts_solver_create(const fblts_mesh* mesh, const fblts_params* params, void* hip_stream,
                        fblts_solver** out);
void fblts_solver_destroy(fblts_solver* s);

/* Install LTS regions (see fblts_layer_regions), reorder cells/edges/vertices
 * region-contiguously, derive every pass's index range from the stencil and
 * upload the reordered mesh.  Also required (all-coarse) for the global
 * schemes.  Invalidates any captured graph and the state.
 * Errors: FBLTS_EINVAL, FBLTS_EREGION, FBLTS_EDEVICE, FBLTS_ENOMEM. */
int fblts_set_regions(fblts_solver* s, const int8_t* labels, int32_t binary);

/* State in caller numbering: h[n_cells] thickness (m), u[n_edges] normal
 * velocity (m/s).  on_device selects device or host pointers.  set_state
 * starts a new trajectory: model time, step count and the storm clock of
 * fblts_set_cyclone restart at zero. */
int fblts_set_state(fblts_solver* s, const double* h, const double* u, int32_t on_device);
int fblts_get_state(fblts_solver* s, double* h, double* u, int32_t on_device);
/* Per-cell quadratic bottom drag coefficient C_D[n_cells] (nonlinear physics). */
int fblts_set_drag(fblts_solver* s, const double* cd, int32_t on_device);
/* Wind forcing at edge points, held fixed until the next call; enables the
 * wind-stress term C_W |u_W - u| (u_W - u) / h of eq. hurricane_model:
 *   wind_normal[n_edges], wind_tangential[n_edges]: the components of u_W
 *     (m/s) along n_e and t_e;
 *   wind_coef[n_edges]: the wind-stress coefficient C_W at each edge
 *     (dimensionless, kinematic: air stress over water density); the paper
 *     takes it from Garratt's drag law, which the caller applies.
 * Caller order, host or device (on_device).  Pass NULL arrays to disable. */
int fblts_set_wind(fblts_solver* s, const double* wind_normal, const double* wind_tangential,
                   const double* wind_coef, int32_t on_device);

/* Moving analytic cyclone as the wind of the wind-stress term of eq.
 * hurricane_model (the paper forces it with observed hurricane winds; this is
 * the analytic stand-in): a Holland (1980) gradient-wind vortex
 *   V(r) = sqrt((b/rho_air)(rm/r)^b dp exp(-(rm/r)^b) + (r f/2)^2) - r|f|/2,
 * f = 2 omega z, r the great-circle distance to the centre, turning
 * counter-clockwise about the centre where the centre's f > 0, plus a
 * translation part v_trans V(r)/V(rm, f_centre) along the track.  The centre
 * starts at `center` and moves about the unit `axis` at angular speed
 * v_trans/radius.  The wind of the k-th coarse step after this call (or
 * after the latest fblts_set_state, which starts a new trajectory at model
 * time zero) is evaluated on the device at t = t0 + k dt before that step's
 * first stage and
 * held for the whole step (coarse advancement and every fine substep); the
 * step counter lives on the device, so captured graphs replay correctly.
 * Components at edges: W.n_e and W.(x_e cross n_e) (the tangent convention of
 * the mesh, t_e = k x n_e).  With the wind the device also forms the
 * coefficient C_W = (rho_air / rho_water)(0.75 + 0.067 |W|) 1e-3 at each edge
 * (the kinematic form of Garratt's 10 m drag law; rho_air and rho_water from
 * the solver's parameters), part of the same forcing evaluation.
 *   x_edge[3*n_edges]: edge positions (any length; normalised), host, caller order;
 *   n_edge[3*n_edges]: unit edge normals n_e, host, caller order.
 * Both are copied.  c = NULL disables the wind (as does fblts_set_wind).
 * Errors: FBLTS_EINVAL (linear physics, NULL arrays, non-unit or non-tangent
 * normals, non-finite or non-positive parameters), FBLTS_ESTATE before
 * set_regions. */
typedef struct fblts_cyclone {
  double center[3];   /* initial centre (direction; normalised) */
  double axis[3];     /* track rotation axis (direction; normalised) */
  double v_trans;     /* translation speed (m/s) */
  double dp;          /* central pressure deficit (Pa) */
  double rm;          /* radius of maximum wind (m) */
  double b;           /* Holland shape parameter */
  double rho_air;     /* air density (kg/m^3) */
  double radius;      /* sphere radius (m) */
  double omega;       /* rotation rate in f = 2 omega z (1/s) */
  double t0;          /* time of the first step's wind (s) */
} fblts_cyclone;
int fblts_set_cyclone(fblts_solver* s, const fblts_cyclone* c, const double* x_edge, const double* n_edge);
/* Copy the wind forcing the last step used (or the first step will use,
 * right after fblts_set_cyclone) to host arrays in caller order: the two
 * components and C_W (wind_coef may be NULL).
 * Errors: FBLTS_ESTATE when no wind is set. */
int fblts_get_wind(fblts_solver* s, double* wind_normal, double* wind_tangential, double* wind_coef);

/* Advance n coarse steps (async).  Errors: FBLTS_ESTATE before set_state. */
int fblts_step(fblts_solver* s, int32_t n_coarse_steps);
/* Capture the step program in hipGraphs and replay them in fblts_step (1), or
 * launch kernels directly (0); see FBLTS_OPT_GRAPH_STEPS.  The graphs are
 * rebuilt after any call that changes the step program. */
int fblts_set_graph(fblts_solver* s, int32_t enable);

/* Tuning options (same results bit for bit, different launch structure);
 * each drops any captured graph.  FUSE_VERTEX, EDGE_CELLS and PIPELINE take
 * 0 (off) or 1 (on):
 *   FBLTS_OPT_FUSE_VERTEX: 1 (default) evaluates the vertex PV q_v inside the
 *     per-edge prep pass, one launch fewer per stage; 0 runs a vertex pass.
 *   FBLTS_OPT_BLOCK: threads per block of the stencil passes, 64/128/256
 *     (default 256).
 *   FBLTS_OPT_EDGE_CELLS: 1 forms the PV flux of the momentum pass (eq.
 *     trisk_vorticity) by walking the edge lists of the edge's two cells and
 *     building each TRiSK weight n_{e,i} n_{e',i} (1/2 - sum of the kite
 *     fractions R_{i,v} passed) on the fly, instead of reading the
 *     edges_on_edge list and its stored weights: about half the momentum
 *     pass's compulsory bytes.  Available (after set_regions) when the mesh's
 *     edges_on_edge lists and weights are those walks, in that order (each
 *     cell's edges counter-clockwise after e, the first cell's first); bit for
 *     bit identical when the stored weights equal the walk's FP64 arithmetic
 *     exactly, else within 1e-13 of them.  Default 0.
 *   FBLTS_OPT_GRAPH_STEPS: coarse steps captured per hipGraph (1..64, default
 *     8); fblts_step(n) replays the multi-step graph n / G times and a one-step
 *     graph for the remainder (each graph launch costs a fixed boundary).
 *   FBLTS_OPT_PERSISTENT: k > 0 runs each coarse step's consecutive stencil,
 *     prediction and assembly passes (Sec. 2.2 steps 1-4) in one cooperative
 *     launch (hipLaunchCooperativeKernel; k blocks of 256 threads per compute
 *     unit, at most as many as stay resident, whatever FBLTS_OPT_BLOCK says;
 *     a grid-wide barrier between passes); forcing and RK4-combination passes, and the
 *     EDGE_CELLS momentum pass, launch on their own between such runs; with
 *     graphs enabled the cooperative launches are captured and replayed like
 *     the per-pass ones.  A barrier that gives up waiting (only
 *     if the device cannot keep the grid resident, e.g. while another
 *     solver's persistent launch or other work occupies the GPU on another
 *     stream) makes the next state read or diagnostics fail with
 *     FBLTS_EDEVICE.  Default 0.
 *   FBLTS_OPT_PIPELINE: 1 (default) arranges an FB-LTS coarse step into fewer
 *     dependent launches (Sec. 2.2 steps 1-4, same arithmetic): the first fine
 *     substep, which needs each coarse stage only through its interface-one
 *     prediction, runs beside the coarse stages 2 and 3 on arrays of its own
 *     (segments of the same launches), and the prediction for the next
 *     substep, or the correction and assembly after the last one, is done by
 *     the substep's last momentum pass.  9M + 3 stencil launches per coarse
 *     step instead of 10M + 10 (q_v fused; a separate vertex pass adds 3M + 1).
 *     0 runs the steps one pass after another.  Ensembles take 0 only.
 * Errors: FBLTS_EINVAL for an unknown option or value, or EDGE_CELLS on a
 * mesh whose weights are not the kite-fraction walks. */
enum {
  FBLTS_OPT_FUSE_VERTEX = 1,
  FBLTS_OPT_BLOCK = 2,
  FBLTS_OPT_EDGE_CELLS = 3,
  FBLTS_OPT_GRAPH_STEPS = 4,
  FBLTS_OPT_PERSISTENT = 5,
  FBLTS_OPT_PIPELINE = 6
};
int fblts_set_option(fblts_solver* s, int32_t option, int32_t value);

typedef struct {
  double mass;              /* sum_i A_i h_i */
  double abs_vorticity;     /* sum_v A_v (zeta_v + f_v) */
  double abs_vorticity_scale; /* sum_v A_v |zeta_v + f_v| */
  double energy;            /* TRiSK energy (linear or nonlinear form) */
  double min_h;
  double time;
  int64_t n_nonfinite;      /* NaN/Inf entries of h and u */
  int64_t step;
} fblts_diag;

/* Deterministic device reductions of the current state; synchronises.
 * Returns FBLTS_ENONFINITE (and fills *out) if any h,u is non-finite or h <= 0. */
int fblts_diagnostics(fblts_solver* s, fblts_diag* out);

/* fblts_diagnostics without device allocation, for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, launch shape and results, bit for bit, but
 * the per-block partial sums and the results live in a fixed device array of
 * the library (8 quantities x 1024 blocks + 8 doubles, about 64 KiB, one per
 * GPU, taken when a solver is created, held until the process ends) instead
 * of buffers the solver allocates on first use.  Every
 * solver fits (its reduction uses at most 1024 blocks); a reduction that
 * would not fit is refused with FBLTS_EINVAL.  All calls on one GPU share
 * that array: calls that overlap on one GPU (other host threads, other
 * streams) race and must be serialised by the caller.  Copies 64 bytes to
 * the host and synchronises the solver's stream.  Errors: FBLTS_EINVAL,
 * FBLTS_ESTATE (no state), FBLTS_EDEVICE, FBLTS_ENONFINITE as
 * fblts_diagnostics. */
int fblts_diagnostics_noalloc(fblts_solver* s, fblts_diag* out);

typedef struct {
  int32_t n_cells, n_edges, n_vertices;
  int32_t n_fine, n_if1, n_if2, n_int;            /* cells per region */
  int32_t n_fine_e, n_if1_e, n_if2_e, n_int_e;    /* edges per region */
  int32_t max_edges, max_eoe;
  int64_t cell_substeps_per_step;   /* N_coarse + M N_fine (global schemes: N) */
  int64_t launches_per_step;
  /* Two byte models per coarse step, each counting every referenced array
   * element once per launch.  The per-pass model includes the intermediates
   * the passes exchange through memory (h*, B, q_v, the edge-prep records);
   * the compulsory model counts only mesh and state arrays (h, u and their
   * stage copies, accumulators, drag, wind), as any implementation must. */
  double model_bytes_per_step;      /* per-pass model, all launched passes */
  double model_bytes_edge_pass;     /* per-pass model, momentum (edge) passes */
  int64_t edge_pass_items_per_step; /* edges processed by momentum passes per step */
  double model_bytes_cell_pass;     /* per-pass model, thickness (cell) passes */
  double compulsory_bytes_per_step; /* compulsory model, all launched passes */
  double compulsory_bytes_edge_pass;/* compulsory model, momentum passes */
  double compulsory_bytes_cell_pass;/* compulsory model, thickness passes */
} fblts_info;
int fblts_get_info(fblts_solver* s, fblts_info* out);

/* Test export: evaluate one tendency on caller-numbered (h,u) over all
 * entities.  which = 0: Psi (out[n_cells]); 1: Phi (out[n_edges]); 2: the
 * slow part of Phi under the operator splitting (PV flux, -grad K, drag,
 * wind; nonlinear physics only).  Uses the solver's physics, drag and wind
 * (the unsplit Phi for which = 1 even when the solver splits).  Synchronises
 * when out is a host pointer. */
int fblts_debug_tendency(fblts_solver* s, int32_t which, const double* h, const double* u,
                         double* out, int32_t on_device);

/* Timing export: average duration (ms) per launch of the kernels of one
 * class launched during the last fblts_step: 0 = momentum (edge) passes,
 * 1 = thickness (cell) passes, 2 = vertex passes, 3 = edge-prep passes.
 * With timing enabled (fblts_set_timing(s,1)) steps launch directly (no
 * graph) and every pass of these classes records a pair of HIP events from
 * its own dispatch (kernel start and end timestamps, hipExtLaunchKernel), so
 * the figure is the kernels' execution time inside the step sequence.
 * Synchronises. */
int fblts_set_timing(fblts_solver* s, int32_t enable);
int fblts_kernel_time(fblts_solver* s, int32_t kernel_class, double* avg_ms, int64_t* launches);
/* Timing export: launch every pass of one class of the current step program
 * `repeats` times back to back between two events and return the mean
 * duration per launch (ms).  The passes overwrite state and scratch: use a
 * solver whose state is disposable.  Synchronises. */
int fblts_time_kernels(fblts_solver* s, int32_t kernel_class, int32_t repeats, double* avg_ms, int64_t* launches);

/* ------------------------------------------------------------ adjoint --- */

/* Reverse mode of the FB-LTS step (Sec. 2.2) for one-member nonlinear or
 * linear solvers without wind stress.
 *
 * fblts_adjoint_forward: advance n_steps coarse steps from the current state
 * (as fblts_step does), keeping a checkpoint of (h, u) every ckpt_every steps
 * on the device (n_steps/ckpt_every states).  Synchronises.
 *
 * fblts_adjoint_backward: given the cotangent of the final state (gh_final
 * [n_cells], gu_final [n_edges], caller numbering), return the gradient with
 * respect to the initial state (gh0, gu0) and to the per-cell drag
 * coefficient C_D (gcd [n_cells]); any output may be NULL.  Each segment of
 * ckpt_every steps is recomputed from its checkpoint in definition mode (the
 * coarse advancement over every cell and edge), taped, and swept backwards
 * with gather-only transposed kernels (deterministic, no atomics).  The
 * solver is left at the final state.  Device memory: about
 * ckpt_every * ((4+4M) n_cells + (4+3M) n_edges) doubles of tape.
 * One forward run serves any number of backward calls (several cotangents)
 * as long as nothing changes the trajectory in between: fblts_set_regions,
 * fblts_set_state, fblts_set_drag, fblts_set_wind, fblts_set_cyclone,
 * fblts_step, fblts_autotune (which steps) and another fblts_adjoint_forward
 * each invalidate the recording.
 * Errors: FBLTS_ESTATE without a preceding forward or after such a call (the
 * checkpoints, drag and final state would belong to another trajectory),
 * FBLTS_EINVAL for other schemes or when wind stress is set.  Synchronises. */
int fblts_adjoint_forward(fblts_solver* s, int32_t n_steps, int32_t ckpt_every);
/* The identity of the solver's current adjoint recording: *id > 0 names the
 * recording the last fblts_adjoint_forward made while it is still valid
 * (nothing above has invalidated it), *id = 0 when there is none.  A caller
 * that records several runs on one solver (a chain of applications) keeps
 * the id of each and records a run again when the id no longer matches.
 * Host only (no device work).  Errors: FBLTS_EINVAL (NULL argument). */
int fblts_adjoint_recording(fblts_solver* s, uint64_t* id);
int fblts_adjoint_backward(fblts_solver* s, const double* gh_final, const double* gu_final, double* gh0,
                           double* gu0, double* gcd, int32_t on_device);
/* Test export: transposed tendency at the point (h, u) (host arrays, caller
 * numbering).  which = 0: cot[n_cells] is a cotangent of Psi(u, h);
 * which = 1: cot[n_edges] of Phi(u, h) (h taken as the FB-averaged thickness).
 * Writes hbar[n_cells], ubar[n_edges] and, for Phi with drag, cdbar[n_cells]. */
int fblts_debug_vjp(fblts_solver* s, int32_t which, const double* h, const double* u, const double* cot,
                    double* hbar, double* ubar, double* cdbar);

/* ----------------------------------------------------------- ensemble --- */

/* A batch of independent FB-LTS members over one or more meshes, advanced by
 * the same kernels with the member index innermost (member-contiguous state),
 * one launch per pass covering every mesh.  n_meshes in 1..4;
 * members_per_mesh[k] a power of two in 1..64.  cell_labels[k] as in
 * fblts_set_regions.  hip_stream as in fblts_solver_create.  Errors as
 * solver_create / set_regions. */
typedef struct fblts_ensemble fblts_ensemble;
int fblts_ensemble_create(const fblts_mesh* const* meshes, const int8_t* const* cell_labels,
                          int32_t labels_are_binary, const int32_t* members_per_mesh,
                          int32_t n_meshes, const fblts_params* params, void* hip_stream,
                          fblts_ensemble** out);
void fblts_ensemble_destroy(fblts_ensemble* e);
/* State and per-cell drag of one member (caller numbering of that mesh). */
int fblts_ensemble_set_member(fblts_ensemble* e, int32_t mesh, int32_t member, const double* h,
                              const double* u, const double* cd, int32_t on_device);
int fblts_ensemble_get_member(fblts_ensemble* e, int32_t mesh, int32_t member, double* h,
                              double* u, int32_t on_device);
/* Per-member cyclone forcing (see fblts_set_cyclone): member `member` of mesh
 * `mesh` gets storm c, or calm air (zero wind, the wind-stress term then acts
 * on the water's own motion) when c is NULL.  The first call gives every
 * member of every mesh the atmosphere (calm air until given a storm) and
 * starts one step clock per mesh: every storm's wind at the k-th coarse step
 * after that first call is evaluated at t = t0 + k dt (stagger storms with
 * t0).  x_edge[3*n_edges] / n_edge[3*n_edges] (host, caller order of that
 * mesh) are required the first time a storm is given on a mesh and may be
 * NULL afterwards.  Drops any captured graph.  Errors: FBLTS_EINVAL (linear
 * physics, bad index or parameters, missing positions). */
int fblts_ensemble_set_cyclone(fblts_ensemble* e, int32_t mesh, int32_t member, const fblts_cyclone* c,
                               const double* x_edge, const double* n_edge);
int fblts_ensemble_step(fblts_ensemble* e, int32_t n_coarse_steps);
int fblts_ensemble_set_graph(fblts_ensemble* e, int32_t enable);
/* Tuning option of the ensemble's passes (see fblts_set_option). */
int fblts_ensemble_set_option(fblts_ensemble* e, int32_t option, int32_t value);
/* out[total members] in mesh-major, member-minor order; synchronises. */
int fblts_ensemble_diagnostics(fblts_ensemble* e, fblts_diag* out);
int fblts_ensemble_info(fblts_ensemble* e, int64_t* member_cells, int64_t* cell_substeps_per_step,
                        double* model_bytes_per_step);

/* -------------------------------------------------------- autotuning --- */

/* Launch-schedule search for a solver or an ensemble.  Times every candidate
 * schedule, in this order -- q_v fused into the prep pass or not
 * (FBLTS_OPT_FUSE_VERTEX) with blocks of 256, 128 or 64 threads
 * (FBLTS_OPT_BLOCK) on graph-replayed coarse steps; the persistent launch
 * (FBLTS_OPT_PERSISTENT) with q_v fused or not and 1 or 4 blocks per compute
 * unit, where the device supports cooperative launches; and, where every
 * mesh allows it, the momentum pass
 * through the cells' edge lists (FBLTS_OPT_EDGE_CELLS) with each fusion and
 * block size -- and leaves the fastest set.  Every candidate computes the
 * same bits, so tuning never
 * changes results.  Before the search the state, the model time and step
 * count, and with a moving storm its step clock and wind, are saved; they
 * are restored afterwards, as are the graph and timing settings.
 *   handle, handle_kind: a solver with a state (FBLTS_HANDLE_SOLVER) or an
 *     ensemble (FBLTS_HANDLE_ENSEMBLE);
 *   steps (1..10000), repeats (1..100): after two warm-up steps, each
 *     candidate runs `repeats` times `steps` coarse steps between two events
 *     on the handle's stream; its best run counts;
 *   cache_json_path: NULL, or a JSON file of earlier results with one
 *     workload per line, keyed by what sets the pass program and its sizes
 *     (mesh and region sizes, scheme, M, physics, splitting, drag, wind,
 *     steps per graph).  A hit sets the stored schedule without timing
 *     (from_cache = 1); a miss adds the result and rewrites the file through
 *     a temporary file and a rename.  A missing file counts as empty;
 *   out: the chosen schedule (may be NULL);
 *   tried[max_tried]: the timed candidates in search order (may be NULL when
 *     max_tried is 0); *n_tried (may be NULL) receives how many were timed,
 *     0 on a cache hit.
 * Synchronises the handle's stream and blocks until the search ends.  The
 * handle must not be used from another thread meanwhile.
 * Errors: FBLTS_EINVAL (NULL handle, unknown kind, counts out of range, a
 * cache file in another format, an unwritable cache), FBLTS_ESTATE (solver
 * without state), FBLTS_EDEVICE, FBLTS_ENOMEM. */
enum { FBLTS_HANDLE_SOLVER = 0, FBLTS_HANDLE_ENSEMBLE = 1 };
typedef struct fblts_schedule {
  int32_t fuse_vertex;   /* FBLTS_OPT_FUSE_VERTEX value */
  int32_t block;         /* FBLTS_OPT_BLOCK value */
  int32_t edge_cells;    /* FBLTS_OPT_EDGE_CELLS value */
  int32_t from_cache;    /* 1: read from the cache file, not timed */
  double ms_per_step;    /* best time per coarse step (ms), measured or cached */
  int32_t persistent;    /* FBLTS_OPT_PERSISTENT value */
} fblts_schedule;
int fblts_autotune(void* handle, int32_t handle_kind, int32_t steps, int32_t repeats, const char* cache_json_path,
                   fblts_schedule* out, fblts_schedule* tried, int32_t max_tried, int32_t* n_tried);

#ifdef __cplusplus
}
#endif

#endif /* FBLTS_H */
