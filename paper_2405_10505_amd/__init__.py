"""Python binding of libfblts (include/fblts.h): argument marshalling only.

Every step of the FB-LTS hot path runs in the library's HIP kernels; this
module converts arrays and handles.  It fails loudly when the library has not
been built -- there is no fallback.  PyTorch, when used, only provides device
memory and the HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfblts.so")

FBLTS_OK, FBLTS_EINVAL, FBLTS_ENOMEM, FBLTS_EDEVICE, FBLTS_EREGION, FBLTS_ESTATE, FBLTS_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
SCHEME_FBLTS, SCHEME_FBRK32, SCHEME_RK4 = 0, 1, 2
PHYS_LINEAR, PHYS_NONLINEAR, PHYS_GRAVITY_WAVE = 0, 1, 2
SPLIT_NONE, SPLIT_COARSE, SPLIT_FINE = 0, 1, 2
BETA = (0.531, 0.531, 0.313)
OPT_FUSE_VERTEX, OPT_BLOCK, OPT_EDGE_CELLS, OPT_GRAPH_STEPS, OPT_PERSISTENT, OPT_PIPELINE = 1, 2, 3, 4, 5, 6
HANDLE_SOLVER, HANDLE_ENSEMBLE = 0, 1

_P_i32 = C.POINTER(C.c_int32)
_P_f64 = C.POINTER(C.c_double)


class fblts_mesh_desc(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("n_edges", C.c_int32), ("n_vertices", C.c_int32),
                ("cells_on_edge", _P_i32), ("vertices_on_edge", _P_i32),
                ("edges_on_cell_off", _P_i32), ("edges_on_cell", _P_i32),
                ("vertices_on_cell_off", _P_i32), ("vertices_on_cell", _P_i32),
                ("edges_on_edge_off", _P_i32), ("edges_on_edge", _P_i32), ("weights_on_edge", _P_f64),
                ("edges_on_vertex", _P_i32), ("cells_on_vertex", _P_i32), ("kite_areas_on_vertex", _P_f64),
                ("dc_edge", _P_f64), ("dv_edge", _P_f64), ("area_cell", _P_f64), ("area_triangle", _P_f64),
                ("f_vertex", _P_f64), ("f_edge", _P_f64), ("bottom_depth", _P_f64)]


class fblts_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("g", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("beta3", C.c_double), ("M", C.c_int32), ("scheme", C.c_int32), ("physics", C.c_int32),
                ("r_layers", C.c_int32), ("rho_air", C.c_double), ("rho_water", C.c_double),
                ("split", C.c_int32), ("reserved", C.c_int32)]


class fblts_diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("abs_vorticity", C.c_double), ("abs_vorticity_scale", C.c_double),
                ("energy", C.c_double), ("min_h", C.c_double), ("time", C.c_double),
                ("n_nonfinite", C.c_int64), ("step", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fblts_plan_info(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n_cells", "n_edges", "n_fine", "n_if1", "n_if2", "n_int",
                                         "n_fine_e", "n_if1_e", "n_if2_e", "n_int_e")] + \
               [(n, C.c_int32 * 3) for n in ("coarse_cell_begin", "coarse_edge_begin", "fine_cell_end",
                                             "fine_edge_end")]

    def as_dict(self):
        return {k: (getattr(self, k) if t is C.c_int32 else list(getattr(self, k))) for k, t in self._fields_}


class fblts_schedule(C.Structure):
    _fields_ = [("fuse_vertex", C.c_int32), ("block", C.c_int32), ("edge_cells", C.c_int32),
                ("from_cache", C.c_int32), ("ms_per_step", C.c_double), ("persistent", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fblts_cyclone(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("axis", C.c_double * 3)] + [
        (k, C.c_double) for k in ("v_trans", "dp", "rm", "b", "rho_air", "radius", "omega", "t0")]


class fblts_info(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n_cells", "n_edges", "n_vertices", "n_fine", "n_if1", "n_if2", "n_int",
                                         "n_fine_e", "n_if1_e", "n_if2_e", "n_int_e", "max_edges", "max_eoe")] + \
               [("cell_substeps_per_step", C.c_int64), ("launches_per_step", C.c_int64),
                ("model_bytes_per_step", C.c_double), ("model_bytes_edge_pass", C.c_double),
                ("edge_pass_items_per_step", C.c_int64), ("model_bytes_cell_pass", C.c_double),
                ("compulsory_bytes_per_step", C.c_double), ("compulsory_bytes_edge_pass", C.c_double),
                ("compulsory_bytes_cell_pass", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol include/fblts.h declares, with its ctypes signature
_SIGS = {
    "fblts_last_error": (C.c_char_p, []),
    "fblts_version": (C.c_int, []),
    "fblts_mesh_create": (C.c_int, [C.POINTER(fblts_mesh_desc), C.POINTER(C.c_void_p)]),
    "fblts_mesh_destroy": (None, [C.c_void_p]),
    "fblts_layer_regions": (C.c_int, [C.c_void_p, C.POINTER(C.c_int8), C.c_int32, C.c_int32,
                                      C.POINTER(C.c_int8), _P_i32]),
    "fblts_plan": (C.c_int, [C.c_void_p, C.POINTER(C.c_int8), C.c_int32, C.c_int32, C.c_int32,
                             C.POINTER(fblts_plan_info)]),
    "fblts_solver_create": (C.c_int, [C.c_void_p, C.POINTER(fblts_params), C.c_void_p, C.POINTER(C.c_void_p)]),
    "fblts_solver_destroy": (None, [C.c_void_p]),
    "fblts_set_regions": (C.c_int, [C.c_void_p, C.POINTER(C.c_int8), C.c_int32]),
    "fblts_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "fblts_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "fblts_set_drag": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "fblts_set_wind": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "fblts_set_cyclone": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fblts_get_wind": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fblts_ensemble_set_cyclone": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fblts_step": (C.c_int, [C.c_void_p, C.c_int32]),
    "fblts_set_graph": (C.c_int, [C.c_void_p, C.c_int32]),
    "fblts_diagnostics": (C.c_int, [C.c_void_p, C.POINTER(fblts_diag)]),
    "fblts_diagnostics_noalloc": (C.c_int, [C.c_void_p, C.POINTER(fblts_diag)]),
    "fblts_get_info": (C.c_int, [C.c_void_p, C.POINTER(fblts_info)]),
    "fblts_debug_tendency": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "fblts_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "fblts_kernel_time": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "fblts_time_kernels": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int64)]),
    "fblts_adjoint_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "fblts_adjoint_recording": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "fblts_adjoint_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_int32]),
    "fblts_debug_vjp": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p]),
    "fblts_ensemble_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.POINTER(C.c_int8)), C.c_int32, _P_i32,
                                        C.c_int32, C.POINTER(fblts_params), C.c_void_p, C.POINTER(C.c_void_p)]),
    "fblts_ensemble_destroy": (None, [C.c_void_p]),
    "fblts_ensemble_set_member": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_int32]),
    "fblts_ensemble_get_member": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    "fblts_ensemble_step": (C.c_int, [C.c_void_p, C.c_int32]),
    "fblts_ensemble_set_graph": (C.c_int, [C.c_void_p, C.c_int32]),
    "fblts_ensemble_set_option": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "fblts_set_option": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "fblts_ensemble_diagnostics": (C.c_int, [C.c_void_p, C.POINTER(fblts_diag)]),
    "fblts_ensemble_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_double)]),
    "fblts_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_char_p, C.POINTER(fblts_schedule),
                                 C.POINTER(fblts_schedule), C.c_int32, _P_i32]),
}


class FBLTSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fblts error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """The loaded libfblts.so (raises ImportError if it has not been built).

    The environment variable FBLTS_LIB names another build of the library to
    load instead (same C ABI), e.g. to compare two builds on one machine."""
    global _lib
    if _lib is None:
        path = os.environ.get("FBLTS_LIB", LIB_PATH)
        if not os.path.exists(path):
            raise ImportError("libfblts.so is not built (%s); run paper_2405_10505_amd.build_lib.build()" % path)
        # Load PyTorch's HIP runtime first when PyTorch is present: libfblts
        # then binds to that same runtime (both carry SONAME libamdhip64.so.7),
        # so tensors, streams and the library share one device context.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != FBLTS_OK:
        raise FBLTSError(rc, lib().fblts_last_error().decode())
    return rc


# at most 2 x 2 x 3 candidate schedules (cells, fused q, block)
_MAX_CANDIDATES = 16


def _autotune(handle, kind, steps, repeats, cache_path):
    out = fblts_schedule()
    tried = (fblts_schedule * _MAX_CANDIDATES)()
    n = C.c_int32()
    path = os.fsencode(cache_path) if cache_path is not None else None
    _check(lib().fblts_autotune(handle, int(kind), int(steps), int(repeats), path, C.byref(out), tried,
                                _MAX_CANDIDATES, C.byref(n)))
    d = out.as_dict()
    d["candidates"] = [tried[k].as_dict() for k in range(n.value)]
    return d


def _ptr(a, dtype, n=None, what="array"):
    """(pointer, on_device, keepalive) for a numpy array or a torch tensor.

    n: the number of elements the library will read or write through the
    pointer; a different size raises ValueError (the C ABI cannot check)."""
    if a is None:
        return None, 0, None
    if hasattr(a, "data_ptr"):      # torch tensor
        import torch
        want = torch.float64 if dtype == np.float64 else torch.int32
        if a.dtype != want or not a.is_contiguous():
            raise TypeError("tensor must be contiguous %s" % want)
        if n is not None and a.numel() != n:
            raise ValueError("%s must have %d elements, got %d" % (what, n, a.numel()))
        return C.c_void_p(a.data_ptr()), (1 if a.is_cuda else 0), a
    arr = np.ascontiguousarray(a, dtype=dtype)
    if n is not None and arr.size != n:
        raise ValueError("%s must have %d elements, got %d" % (what, n, arr.size))
    return arr.ctypes.data_as(C.c_void_p), 0, arr


def _host(a, dtype, n, what):
    arr = np.ascontiguousarray(a, dtype=dtype)
    if arr.size != n:
        raise ValueError("%s must have %d elements, got %d" % (what, n, arr.size))
    return arr


class Mesh:
    """fblts_mesh: validated host copy of an MPAS-style mesh (no device needed)."""

    def __init__(self, mesh):
        arrs = mesh.desc_arrays()
        self._keep = arrs
        d = fblts_mesh_desc()
        d.n_cells, d.n_edges, d.n_vertices = mesh.n_cells, mesh.n_edges, mesh.n_vertices
        for k, v in arrs.items():
            setattr(d, k, v.ctypes.data_as(_P_i32 if v.dtype == np.int32 else _P_f64))
        h = C.c_void_p()
        _check(lib().fblts_mesh_create(C.byref(d), C.byref(h)))
        self.handle = h
        self.n_cells, self.n_edges, self.n_vertices = mesh.n_cells, mesh.n_edges, mesh.n_vertices

    def layer_regions(self, labels, binary=True, r=2):
        lab = _host(labels, np.int8, self.n_cells, "labels")
        out = np.zeros(self.n_cells, np.int8)
        layer = np.zeros(self.n_cells, np.int32)
        _check(lib().fblts_layer_regions(self.handle, lab.ctypes.data_as(C.POINTER(C.c_int8)), int(binary), int(r),
                                         out.ctypes.data_as(C.POINTER(C.c_int8)), layer.ctypes.data_as(_P_i32)))
        return out, layer

    def plan(self, labels, binary=True, r=2, nonlinear=True):
        """fblts_plan: region counts and pass ranges (host only)."""
        lab = _host(labels, np.int8, self.n_cells, "labels")
        out = fblts_plan_info()
        _check(lib().fblts_plan(self.handle, lab.ctypes.data_as(C.POINTER(C.c_int8)), int(binary), int(r),
                                int(nonlinear), C.byref(out)))
        return out.as_dict()

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fblts_mesh_destroy(self.handle)
            self.handle = None


def make_params(dt, M=1, scheme=SCHEME_FBLTS, linear=False, g=9.81, beta=BETA, r_layers=2,
                rho_air=1.15, rho_water=1000.0, physics=None, split=SPLIT_NONE):
    """physics overrides `linear` (PHYS_*); split selects the operator splitting (SPLIT_*)."""
    p = fblts_params()
    p.dt, p.g = float(dt), float(g)
    p.beta1, p.beta2, p.beta3 = beta
    if physics is None:
        physics = PHYS_LINEAR if linear else PHYS_NONLINEAR
    p.M, p.scheme, p.physics, p.r_layers = int(M), int(scheme), int(physics), int(r_layers)
    p.rho_air, p.rho_water = rho_air, rho_water
    p.split, p.reserved = int(split), 0
    return p


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _cyclone(center, axis, v_trans=5.0, dp=6000.0, rm=40e3, b=1.5, rho_air=1.15, radius=6.371229e6,
             omega=7.292e-5, t0=0.0):
    c = fblts_cyclone()
    for k in range(3):
        c.center[k] = float(center[k])
        c.axis[k] = float(axis[k])
    c.v_trans, c.dp, c.rm, c.b, c.rho_air = v_trans, dp, rm, b, rho_air
    c.radius, c.omega, c.t0 = radius, omega, t0
    return c


def _edge_vectors(mesh, x_edge, n_edge):
    if x_edge is None:
        return None, None, None
    x = np.ascontiguousarray(x_edge, dtype=np.float64).reshape(-1)
    n = np.ascontiguousarray(n_edge, dtype=np.float64).reshape(-1)
    if x.size != 3 * mesh.n_edges or n.size != 3 * mesh.n_edges:
        raise ValueError("x_edge and n_edge must hold 3 values per edge")
    return x, n, (x.ctypes.data, n.ctypes.data)


class Solver:
    """fblts_solver: one mesh, one member, one scheme."""

    def __init__(self, mesh: Mesh, dt, M=1, scheme=SCHEME_FBLTS, linear=False, stream=None, **kw):
        self.mesh = mesh
        self.params = make_params(dt, M, scheme, linear, **kw)
        h = C.c_void_p()
        _check(lib().fblts_solver_create(mesh.handle, C.byref(self.params), _stream_handle(stream), C.byref(h)))
        self.handle = h

    def set_regions(self, labels, binary=True):
        lab = _host(labels, np.int8, self.mesh.n_cells, "labels")
        _check(lib().fblts_set_regions(self.handle, lab.ctypes.data_as(C.POINTER(C.c_int8)), int(binary)))

    def set_state(self, h, u):
        ph, dh, kh = _ptr(h, np.float64, self.mesh.n_cells, "h")
        pu, du, ku = _ptr(u, np.float64, self.mesh.n_edges, "u")
        if dh != du:
            raise ValueError("h and u must both be host or both be device arrays")
        _check(lib().fblts_set_state(self.handle, ph, pu, dh))

    def get_state(self, h=None, u=None):
        """Into given arrays/tensors, or new numpy arrays when omitted."""
        if h is None and u is None:
            h = np.empty(self.mesh.n_cells)
            u = np.empty(self.mesh.n_edges)
        if h is not None and hasattr(h, "flags") and not h.flags.c_contiguous:
            raise ValueError("h must be C-contiguous")
        if u is not None and hasattr(u, "flags") and not u.flags.c_contiguous:
            raise ValueError("u must be C-contiguous")
        ph, dh, _ = _ptr(h, np.float64, self.mesh.n_cells, "h")
        pu, du, _ = _ptr(u, np.float64, self.mesh.n_edges, "u")
        _check(lib().fblts_get_state(self.handle, ph, pu, dh if h is not None else du))
        return h, u

    def set_drag(self, cd):
        p, d, k = _ptr(cd, np.float64, self.mesh.n_cells, "cd")
        _check(lib().fblts_set_drag(self.handle, p, d))

    def set_wind(self, wn, wt, cw):
        """Fixed wind forcing at edges: components (m/s) and the wind-stress coefficient C_W."""
        pn, dn, kn = _ptr(wn, np.float64, self.mesh.n_edges, "wind_normal")
        pt, dt, kt = _ptr(wt, np.float64, self.mesh.n_edges, "wind_tangential")
        pc, dc, kc = _ptr(cw, np.float64, self.mesh.n_edges, "wind_coef")
        if not (dn == dt == dc):
            raise ValueError("wind arrays must all be on the host or all on the device")
        _check(lib().fblts_set_wind(self.handle, pn, pt, pc, dn))

    def set_cyclone(self, x_edge, n_edge, **storm):
        """Moving Holland cyclone as the wind-stress forcing (device-evaluated per coarse step)."""
        c = _cyclone(**storm)
        x, n, (px, pn) = _edge_vectors(self.mesh, x_edge, n_edge)
        _check(lib().fblts_set_cyclone(self.handle, C.byref(c), px, pn))

    def clear_wind(self):
        _check(lib().fblts_set_cyclone(self.handle, None, None, None))

    def get_wind(self):
        """The wind forcing of the current step: (normal, tangential, C_W) at edges."""
        wn = np.empty(self.mesh.n_edges)
        wt = np.empty(self.mesh.n_edges)
        wc = np.empty(self.mesh.n_edges)
        _check(lib().fblts_get_wind(self.handle, wn.ctypes.data, wt.ctypes.data, wc.ctypes.data))
        return wn, wt, wc

    def step(self, n=1):
        _check(lib().fblts_step(self.handle, int(n)))

    def set_graph(self, on=True):
        _check(lib().fblts_set_graph(self.handle, int(on)))

    def set_option(self, option, value):
        _check(lib().fblts_set_option(self.handle, int(option), int(value)))

    def diagnostics(self, allow_nonfinite=False):
        d = fblts_diag()
        rc = lib().fblts_diagnostics(self.handle, C.byref(d))
        if rc == FBLTS_ENONFINITE and allow_nonfinite:
            return d.as_dict()
        _check(rc)
        return d.as_dict()

    def diagnostics_noalloc(self, allow_nonfinite=False):
        """fblts_diagnostics_noalloc: the same results without device allocation."""
        d = fblts_diag()
        rc = lib().fblts_diagnostics_noalloc(self.handle, C.byref(d))
        if rc == FBLTS_ENONFINITE and allow_nonfinite:
            return d.as_dict()
        _check(rc)
        return d.as_dict()

    def info(self):
        i = fblts_info()
        _check(lib().fblts_get_info(self.handle, C.byref(i)))
        return i.as_dict()

    def tendency(self, which, h, u):
        n = self.mesh.n_cells if which == 0 else self.mesh.n_edges
        out = np.empty(n)
        ph, dh, kh = _ptr(h, np.float64, self.mesh.n_cells, "h")
        pu, du, ku = _ptr(u, np.float64, self.mesh.n_edges, "u")
        if dh or du:
            raise ValueError("tendency takes host arrays")
        _check(lib().fblts_debug_tendency(self.handle, int(which), ph, pu, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def vjp(self, which, h, u, cot):
        """Transposed tendency at (h, u): returns (hbar, ubar, cdbar)."""
        hb = np.empty(self.mesh.n_cells)
        ub = np.empty(self.mesh.n_edges)
        cb = np.empty(self.mesh.n_cells)
        a = [_host(h, np.float64, self.mesh.n_cells, "h"), _host(u, np.float64, self.mesh.n_edges, "u"),
             _host(cot, np.float64, self.mesh.n_cells if which == 0 else self.mesh.n_edges, "cotangent")]
        _check(lib().fblts_debug_vjp(self.handle, int(which), *[x.ctypes.data_as(C.c_void_p) for x in a],
                                     hb.ctypes.data_as(C.c_void_p), ub.ctypes.data_as(C.c_void_p),
                                     cb.ctypes.data_as(C.c_void_p)))
        return hb, ub, cb

    def adjoint_forward(self, n_steps, ckpt_every):
        _check(lib().fblts_adjoint_forward(self.handle, int(n_steps), int(ckpt_every)))

    def adjoint_recording(self):
        """Identity of the current valid adjoint recording (0: none)."""
        v = C.c_uint64(0)
        _check(lib().fblts_adjoint_recording(self.handle, C.byref(v)))
        return v.value

    def adjoint_backward(self, gh_final, gu_final, out=None):
        """Gradients (gh0, gu0, gcd) from the final-state cotangent.

        Host (numpy) seeds give numpy results; CUDA tensors give tensors."""
        ph, dh, kh = _ptr(gh_final, np.float64, self.mesh.n_cells, "gh_final")
        pu, du, ku = _ptr(gu_final, np.float64, self.mesh.n_edges, "gu_final")
        if dh != du:
            raise ValueError("gh_final and gu_final must both be host or both be device arrays")
        if dh:
            import torch
            gh0 = torch.empty(self.mesh.n_cells, dtype=torch.float64, device=gh_final.device)
            gu0 = torch.empty(self.mesh.n_edges, dtype=torch.float64, device=gh_final.device)
            gcd = torch.empty(self.mesh.n_cells, dtype=torch.float64, device=gh_final.device)
            ptrs = [C.c_void_p(t.data_ptr()) for t in (gh0, gu0, gcd)]
        else:
            gh0, gu0, gcd = np.empty(self.mesh.n_cells), np.empty(self.mesh.n_edges), np.empty(self.mesh.n_cells)
            ptrs = [t.ctypes.data_as(C.c_void_p) for t in (gh0, gu0, gcd)]
        _check(lib().fblts_adjoint_backward(self.handle, ph, pu, *ptrs, dh))
        return gh0, gu0, gcd

    def set_timing(self, on=True):
        _check(lib().fblts_set_timing(self.handle, int(on)))

    def time_kernels(self, cls, repeats=20):
        """Mean duration (ms) per launch of one pass class replayed back to back (disposable state)."""
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().fblts_time_kernels(self.handle, int(cls), int(repeats), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def kernel_time(self, cls):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().fblts_kernel_time(self.handle, int(cls), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def autotune(self, steps=20, repeats=3, cache_path=None):
        """fblts_autotune: set the fastest launch schedule; returns it (dict)."""
        return _autotune(self.handle, HANDLE_SOLVER, steps, repeats, cache_path)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fblts_solver_destroy(self.handle)
            self.handle = None


class Ensemble:
    """fblts_ensemble: members of several meshes advanced by shared launches."""

    def __init__(self, meshes, labels, members, dt, M=1, scheme=SCHEME_FBLTS, linear=False, binary=True,
                 stream=None, **kw):
        self.meshes = list(meshes)
        self.members = [int(m) for m in members]
        self.params = make_params(dt, M, scheme, linear, **kw)
        n = len(self.meshes)
        mh = (C.c_void_p * n)(*[m.handle.value for m in self.meshes])
        if len(labels) != n or len(self.members) != n:
            raise ValueError("one label array and one member count per mesh")
        self._labs = [_host(l, np.int8, m.n_cells, "labels") for l, m in zip(labels, self.meshes)]
        lp = (C.POINTER(C.c_int8) * n)(*[l.ctypes.data_as(C.POINTER(C.c_int8)) for l in self._labs])
        mem = np.ascontiguousarray(self.members, dtype=np.int32)
        h = C.c_void_p()
        _check(lib().fblts_ensemble_create(mh, lp, int(binary), mem.ctypes.data_as(_P_i32), n,
                                           C.byref(self.params), _stream_handle(stream), C.byref(h)))
        self.handle = h

    def set_member(self, mesh, member, h, u, cd=None):
        m = self.meshes[mesh]
        ph, dh, kh = _ptr(h, np.float64, m.n_cells, "h")
        pu, du, ku = _ptr(u, np.float64, m.n_edges, "u")
        pc, dc, kc = _ptr(cd, np.float64, m.n_cells, "cd")
        if dh != du or (cd is not None and dc != dh):
            raise ValueError("h, u and cd must all be host or all be device arrays")
        _check(lib().fblts_ensemble_set_member(self.handle, int(mesh), int(member), ph, pu, pc, dh))

    def get_member(self, mesh, member):
        h = np.empty(self.meshes[mesh].n_cells)
        u = np.empty(self.meshes[mesh].n_edges)
        _check(lib().fblts_ensemble_get_member(self.handle, int(mesh), int(member), h.ctypes.data_as(C.c_void_p),
                                               u.ctypes.data_as(C.c_void_p), 0))
        return h, u

    def set_cyclone(self, mesh, member, x_edge=None, n_edge=None, storm=None):
        """Member `member` of mesh `mesh` gets the Holland storm `storm` (a dict of
        fblts_cyclone fields), or calm air when storm is None."""
        c = C.byref(_cyclone(**storm)) if storm is not None else None
        x, n, ptrs = _edge_vectors(self.meshes[mesh], x_edge, n_edge)
        px, pn = ptrs if ptrs else (None, None)
        _check(lib().fblts_ensemble_set_cyclone(self.handle, int(mesh), int(member), c, px, pn))

    def step(self, n=1):
        _check(lib().fblts_ensemble_step(self.handle, int(n)))

    def set_graph(self, on=True):
        _check(lib().fblts_ensemble_set_graph(self.handle, int(on)))

    def set_option(self, option, value):
        _check(lib().fblts_ensemble_set_option(self.handle, int(option), int(value)))

    def diagnostics(self):
        tot = sum(self.members)
        arr = (fblts_diag * tot)()
        _check(lib().fblts_ensemble_diagnostics(self.handle, arr))
        return [a.as_dict() for a in arr]

    def autotune(self, steps=10, repeats=2, cache_path=None):
        """fblts_autotune: set the fastest launch schedule; returns it (dict)."""
        return _autotune(self.handle, HANDLE_ENSEMBLE, steps, repeats, cache_path)

    def info(self):
        mc, cs, mb = C.c_int64(), C.c_int64(), C.c_double()
        _check(lib().fblts_ensemble_info(self.handle, C.byref(mc), C.byref(cs), C.byref(mb)))
        return dict(member_cells=mc.value, cell_substeps_per_step=cs.value, model_bytes_per_step=mb.value)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fblts_ensemble_destroy(self.handle)
            self.handle = None


def fblts_function():
    """torch.autograd.Function running n FB-LTS coarse steps on a Solver.

    forward(h0, u0, cd, solver, n_steps, ckpt_every) -> (h_N, u_N); backward
    returns the gradients with respect to h0, u0 and the per-cell drag cd
    through the library's hand-written adjoint (checkpoint every ckpt_every
    steps).  Tensors are float64 CUDA tensors in the caller's numbering.
    """
    import torch

    class FBLTSSteps(torch.autograd.Function):
        @staticmethod
        def forward(ctx, h0, u0, cd, solver, n_steps, ckpt_every):
            ins = (h0.detach().contiguous(), u0.detach().contiguous(), cd.detach().contiguous())
            solver.set_drag(ins[2])
            solver.set_state(ins[0], ins[1])
            solver.adjoint_forward(n_steps, ckpt_every)
            hN = torch.empty_like(h0)
            uN = torch.empty_like(u0)
            solver.get_state(hN, uN)
            ctx.solver = solver
            ctx.rec = solver.adjoint_recording()
            ctx.run = (n_steps, ckpt_every)
            # the inputs are kept (autograd checks that they are not modified
            # in place) to record this call again if a later use of the solver
            # replaced its recording
            ctx.save_for_backward(h0, u0, cd)
            ctx.shapes = (h0.shape, u0.shape, h0.device)
            return hN, uN

        @staticmethod
        def backward(ctx, ghN, guN):
            hs, us, dev = ctx.shapes
            if ghN is None:
                ghN = torch.zeros(hs, dtype=torch.float64, device=dev)
            if guN is None:
                guN = torch.zeros(us, dtype=torch.float64, device=dev)
            s = ctx.solver
            if s.adjoint_recording() != ctx.rec:
                # the solver recorded or ran something else since this call's
                # forward (a chain of applications on one solver): record this
                # call's run again
                h0, u0, cd = (t.detach().contiguous() for t in ctx.saved_tensors)
                s.set_drag(cd)
                s.set_state(h0, u0)
                s.adjoint_forward(*ctx.run)
            gh0, gu0, gcd = s.adjoint_backward(ghN.contiguous(), guN.contiguous())
            return gh0, gu0, gcd, None, None, None

    return FBLTSSteps
