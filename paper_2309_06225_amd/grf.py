"""Python binding of libgrf (argument marshalling only).

Every step of the hot path runs in libgrf's HIP kernels; this module converts
torch device tensors to pointers, the current torch stream to a hipStream_t,
and parameter dicts to the C structs of include/grf.h.  If the library is not
built, every entry point raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import inputs as _inputs

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GRF_LIBRARY", os.path.join(HERE, "libgrf.so"))

NF = 27
NG = 3
BC_FROZEN, BC_PERIODIC = 0, 1
STATUS = {0: "OK", 1: "EINVAL", 2: "ESHAPE", 3: "EHIP", 4: "ENONFINITE", 5: "EHYPERBOLIC", 6: "ENOMEM",
          7: "EUNSUPPORTED", 8: "ENONPOSITIVE"}


class GrfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libgrf {STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("lambda_gb", ctypes.c_double), ("lambda_kind", ctypes.c_int32), ("g2", ctypes.c_double),
                ("a_gauge", ctypes.c_double), ("b_gauge", ctypes.c_double),
                ("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double), ("kappa3", ctypes.c_double),
                ("lapse_coeff", ctypes.c_double), ("lapse_power", ctypes.c_double), ("lapse_advec", ctypes.c_double),
                ("shift_gamma_coeff", ctypes.c_double), ("shift_advec", ctypes.c_double), ("eta", ctypes.c_double),
                ("ko_sigma", ctypes.c_double), ("enforce", ctypes.c_int32), ("chi_min", ctypes.c_double),
                ("lapse_min", ctypes.c_double), ("decoupled", ctypes.c_int32), ("fd_order", ctypes.c_int32),
                ("lambda_lin", ctypes.c_double), ("beta", ctypes.c_double)]


class Box(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("ng", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
                ("field_stride", ctypes.c_int64), ("bc", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p


def lib():
    """Load libgrf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libgrf.so not found at {LIB_PATH}: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        P, B = ctypes.POINTER(Params), ctypes.POINTER(Box)
        L.grf_workspace_bytes.argtypes = [B]
        L.grf_workspace_bytes.restype = ctypes.c_size_t
        L.grf_vjp_workspace_bytes.argtypes = [B]
        L.grf_vjp_workspace_bytes.restype = ctypes.c_size_t
        L.grf_rhs_eval.argtypes = [P, B, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.grf_constraints.argtypes = [P, B, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.grf_constraints.restype = ctypes.c_int
        L.grf_energy_densities.argtypes = [P, B, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.grf_energy_densities.restype = ctypes.c_int
        L.grf_coupling_diagnostics.argtypes = [P, B, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.grf_coupling_diagnostics.restype = ctypes.c_int
        L.grf_rk4_stage.argtypes = [P, B, ctypes.c_int, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.grf_fill_periodic.argtypes = [B, _vp, _vp]
        L.grf_enforce.argtypes = [P, B, _vp, _vp]
        C = ctypes.POINTER(BC)
        L.grf_bc_ghost_cells.argtypes = [B]
        L.grf_bc_ghost_cells.restype = ctypes.c_int64
        L.grf_bc_fill.argtypes = [C, B, _vp, _vp]
        L.grf_bc_ghost_rhs.argtypes = [C, B, _vp, _vp, _vp]
        L.grf_rk4_stage_bc.argtypes = [P, B, C, ctypes.c_int, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, _vp,
                                       ctypes.c_size_t, _vp]
        L.grf_rhs_vjp.argtypes = [P, B, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.grf_rk4_step_vjp_workspace_bytes.argtypes = [B]
        L.grf_rk4_step_vjp_workspace_bytes.restype = ctypes.c_size_t
        L.grf_rk4_step_vjp.argtypes = [P, B, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                       _vp]
        L.grf_batch_scratch_bytes.argtypes = [B, ctypes.c_int]
        L.grf_batch_scratch_bytes.restype = ctypes.c_size_t
        L.grf_batch_create.argtypes = [P, B, ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_double), _vp,
                                       ctypes.c_size_t, ctypes.POINTER(_vp)]
        for name in ("grf_batch_step", "grf_batch_step_perbox", "grf_batch_autotune"):
            getattr(L, name).argtypes = [_vp, _vp]
        L.grf_batch_capture_step.argtypes = [_vp, _vp, ctypes.POINTER(_vp)]
        L.grf_batch_rk4_stage.argtypes = [_vp, ctypes.c_int, _vp]
        L.grf_batch_state.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(_vp)]
        L.grf_batch_tile_variant.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.grf_batch_set_tile_variant.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
        L.grf_batch_status_fetch.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_uint32)]
        L.grf_batch_destroy.argtypes = [_vp]
        L.grf_batch_destroy.restype = None
        L.grf_graph_launch.argtypes = [_vp, _vp]
        L.grf_graph_destroy.argtypes = [_vp]
        L.grf_status_fetch.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_uint32)]
        L.grf_status_clear.argtypes = [_vp, _vp]
        L.grf_flops_per_cell.argtypes = [ctypes.c_int]
        L.grf_flops_per_cell.restype = ctypes.c_int64
        L.grf_last_error.restype = ctypes.c_char_p
        L.grf_set_tile_variant.argtypes = [ctypes.c_int]
        L.grf_set_stage_path.argtypes = [ctypes.c_int]
        L.grf_set_slab_planes.argtypes = [ctypes.c_int]
        L.grf_rk4_stage_static.argtypes = [P, B, ctypes.c_int, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, _vp]
        L.grf_prof_begin.argtypes = [ctypes.c_int]
        L.grf_measure_peaks.argtypes = [_vp, ctypes.c_size_t, _vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]
        L.grf_measure_peaks.restype = ctypes.c_int
        L.grf_prof_end.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        for name in ("grf_rhs_eval", "grf_rk4_stage", "grf_fill_periodic", "grf_rhs_vjp", "grf_status_fetch",
                     "grf_status_clear", "grf_set_tile_variant", "grf_set_stage_path", "grf_set_slab_planes", "grf_rk4_stage_static",
                     "grf_prof_begin", "grf_prof_end",
                     "grf_rk4_step_vjp", "grf_enforce", "grf_batch_create", "grf_batch_step", "grf_batch_step_perbox",
                     "grf_batch_autotune", "grf_batch_capture_step", "grf_batch_rk4_stage", "grf_batch_state", "grf_batch_tile_variant",
                     "grf_batch_set_tile_variant",
                     "grf_batch_status_fetch", "grf_graph_launch", "grf_graph_destroy"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise GrfError(code, lib().grf_last_error().decode())


def make_params(p: dict | None = None, **over) -> Params:
    d = _inputs.default_params() if p is None else dict(p)
    d.update(over)
    return Params(lambda_gb=d["lambda_gb"], lambda_kind=0, g2=d["g2"], a_gauge=d["a_gauge"], b_gauge=d["b_gauge"],
                  kappa1=d["kappa1"], kappa2=d["kappa2"], kappa3=d["kappa3"], lapse_coeff=d["lapse_coeff"],
                  lapse_power=d["lapse_power"], lapse_advec=d["lapse_advec"],
                  shift_gamma_coeff=d["shift_gamma_coeff"], shift_advec=d["shift_advec"], eta=d["eta"],
                  ko_sigma=d["ko_sigma"], enforce=int(d.get("enforce", 0)), chi_min=d.get("chi_min", 0.0),
                  lapse_min=d.get("lapse_min", 0.0), decoupled=int(d.get("decoupled", 0)),
                  fd_order=int(d.get("fd_order", 4)), lambda_lin=float(d.get("lambda_lin", 0.0)),
                  beta=float(d.get("beta", 0.0)))


def make_box(dims, dx, bc=BC_FROZEN, origin=(0.0, 0.0, 0.0), ng=NG) -> Box:
    """ng: ghost layers, 3, or 4 for the sixth-order scheme with its
    eighth-difference dissipation."""
    nx, ny, nz = dims
    if not isinstance(dx, (tuple, list)):
        dx = (dx, dx, dx)
    e = 2 * ng
    return Box(nx=nx, ny=ny, nz=nz, ng=ng, dx=dx[0], dy=dx[1], dz=dx[2], x0=origin[0], y0=origin[1],
               z0=origin[2], field_stride=(nx + e) * (ny + e) * (nz + e), bc=bc)


def box_of(u: torch.Tensor, dx, bc=BC_FROZEN, origin=(0.0, 0.0, 0.0), ng=NG) -> Box:
    nz, ny, nx = (s - 2 * ng for s in u.shape[1:])
    return make_box((nx, ny, nz), dx, bc, origin, ng)


class BC(ctypes.Structure):
    """Per-face boundary rules (grf_bc): faces x-, x+, y-, y+, z-, z+."""
    _fields_ = [("rule", ctypes.c_int32 * 6), ("extrap_order", ctypes.c_int32), ("parity_phi", ctypes.c_int32),
                ("centre", ctypes.c_double * 3), ("speed", ctypes.c_double * NF),
                ("asymptote", ctypes.c_double * NF)]


FACE_RULES = {"frozen": 0, "periodic": 1, "reflective": 2, "extrapolating": 3, "sommerfeld": 4}


def make_bc(rules, extrap_order=1, parity_phi=1, centre=(0.0, 0.0, 0.0), speed=None, asymptote=None,
            origin=None) -> BC:
    """rules: six names of FACE_RULES (faces x-, x+, y-, y+, z-, z+); speed and
    asymptote per field (default 1 and 0).  The coordinates of the cells come
    from the box (make_box's origin); `origin` is accepted and ignored here."""
    speed = [1.0] * NF if speed is None else [float(x) for x in speed]
    asymptote = [0.0] * NF if asymptote is None else [float(x) for x in asymptote]
    return BC(rule=(ctypes.c_int32 * 6)(*[FACE_RULES[r] for r in rules]), extrap_order=int(extrap_order),
              parity_phi=int(parity_phi), centre=(ctypes.c_double * 3)(*[float(x) for x in centre]),
              speed=(ctypes.c_double * NF)(*speed), asymptote=(ctypes.c_double * NF)(*asymptote))


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def workspace_bytes(box: Box) -> int:
    return int(lib().grf_workspace_bytes(ctypes.byref(box)))


def vjp_workspace_bytes(box: Box) -> int:
    return int(lib().grf_vjp_workspace_bytes(ctypes.byref(box)))


def alloc_workspace(nbytes: int, device="cuda") -> torch.Tensor:
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device)
    status_clear(ws)
    return ws


def rhs_eval(params: Params, box: Box, u, rhs, ws, stream=None):
    _check(lib().grf_rhs_eval(ctypes.byref(params), ctypes.byref(box), _ptr(u), _ptr(rhs), _ptr(ws),
                              ws.numel() * 8, _stream(stream)))


def rk4_stage(params: Params, box: Box, stage, dt, u0, us, unext, acc, ws, stream=None):
    _check(lib().grf_rk4_stage(ctypes.byref(params), ctypes.byref(box), int(stage), float(dt), _ptr(u0), _ptr(us),
                               _ptr(unext), _ptr(acc), _ptr(ws), ws.numel() * 8, _stream(stream)))


def rk4_stage_static(params: Params, box: Box, stage, dt, u0, us, unext, acc, status, stream=None):
    """grf_rk4_stage without a workspace: the derivative records live in the
    library's own device scratch; ``status`` is a float64 device tensor whose
    first 4 bytes are the status word into which device conditions are OR-ed."""
    _check(lib().grf_rk4_stage_static(ctypes.byref(params), ctypes.byref(box), int(stage), float(dt), _ptr(u0),
                                      _ptr(us), _ptr(unext), _ptr(acc), _ptr(status), _stream(stream)))


def constraints(params: Params, box: Box, u, ws, stream=None):
    """-> (Hamiltonian (nz, ny, nx), momentum (3, nz, ny, nx)) on the interior."""
    out = torch.empty((4, box.nz, box.ny, box.nx), dtype=torch.float64, device=u.device)
    _check(lib().grf_constraints(ctypes.byref(params), ctypes.byref(box), _ptr(u), _ptr(out), _ptr(ws),
                                 ws.numel() * 8, _stream(stream)))
    return out[0], out[1:]


def energy_densities(params: Params, box: Box, u, ws, stream=None):
    """-> (3, nz, ny, nx): energy densities of the canonical, X^2 and
    Gauss-Bonnet terms on the interior."""
    out = torch.empty((3, box.nz, box.ny, box.nx), dtype=torch.float64, device=u.device)
    _check(lib().grf_energy_densities(ctypes.byref(params), ctypes.byref(box), _ptr(u), _ptr(out), _ptr(ws),
                                      ws.numel() * 8, _stream(stream)))
    return out


def bc_ghost_cells(box: Box) -> int:
    return int(lib().grf_bc_ghost_cells(ctypes.byref(box)))


def bc_fill(bc: BC, box: Box, u, stream=None):
    _check(lib().grf_bc_fill(ctypes.byref(bc), ctypes.byref(box), _ptr(u), _stream(stream)))


def bc_ghost_rhs(bc: BC, box: Box, u, stream=None):
    """-> state-layout tensor: the ghost right-hand side, interior cells 0."""
    out = torch.zeros_like(u)
    _check(lib().grf_bc_ghost_rhs(ctypes.byref(bc), ctypes.byref(box), _ptr(u), _ptr(out), _stream(stream)))
    return out


def rk4_stage_bc(params: Params, box: Box, bc: BC, stage, dt, u0, us, unext, acc, gacc, ws, stream=None):
    _check(lib().grf_rk4_stage_bc(ctypes.byref(params), ctypes.byref(box), ctypes.byref(bc), int(stage), float(dt),
                                  _ptr(u0), _ptr(us), _ptr(unext), _ptr(acc), _ptr(gacc), _ptr(ws), ws.numel() * 8,
                                  _stream(stream)))


def coupling_diagnostics(params: Params, box: Box, u, ws, stream=None):
    """-> (4, nz, ny, nx): the Gauss-Bonnet invariant, the weak-coupling
    indicators |lambda'(phi)| sqrt|L_GB| and |2 g2 X|, and the determinant of
    the per-cell system, on the interior."""
    out = torch.empty((4, box.nz, box.ny, box.nx), dtype=torch.float64, device=u.device)
    _check(lib().grf_coupling_diagnostics(ctypes.byref(params), ctypes.byref(box), _ptr(u), _ptr(out), _ptr(ws),
                                          ws.numel() * 8, _stream(stream)))
    return out


def enforce(params: Params, box: Box, u, stream=None):
    _check(lib().grf_enforce(ctypes.byref(params), ctypes.byref(box), _ptr(u), _stream(stream)))


def fill_periodic(box: Box, u, stream=None):
    _check(lib().grf_fill_periodic(ctypes.byref(box), _ptr(u), _stream(stream)))


def rhs_vjp(params: Params, box: Box, u, w, u_bar, theta_bar, ws, stream=None):
    _check(lib().grf_rhs_vjp(ctypes.byref(params), ctypes.byref(box), _ptr(u), _ptr(w), _ptr(u_bar),
                             _ptr(theta_bar), _ptr(ws), ws.numel() * 8, _stream(stream)))


def step_vjp_workspace_bytes(box: Box) -> int:
    return int(lib().grf_rk4_step_vjp_workspace_bytes(ctypes.byref(box)))


def rk4_step_vjp(params: Params, box: Box, dt, u, u2, u3, u4, ubar_new, ubar, theta_bar, ws, stream=None):
    _check(lib().grf_rk4_step_vjp(ctypes.byref(params), ctypes.byref(box), float(dt), _ptr(u), _ptr(u2), _ptr(u3),
                                  _ptr(u4), _ptr(ubar_new), _ptr(ubar), _ptr(theta_bar), _ptr(ws), ws.numel() * 8,
                                  _stream(stream)))


def status_fetch(ws, stream=None):
    bits = ctypes.c_uint32(0)
    code = lib().grf_status_fetch(_ptr(ws), _stream(stream), ctypes.byref(bits))
    return code, int(bits.value)


def status_clear(ws, stream=None):
    _check(lib().grf_status_clear(_ptr(ws), _stream(stream)))


def set_tile_variant(v: int):
    _check(lib().grf_set_tile_variant(int(v)))


def set_stage_path(path: int):
    """0: stencil kernel + plain pointwise kernel; 2 (default): stencil kernel
    + pointwise kernel with LDS-staged inputs."""
    _check(lib().grf_set_stage_path(int(path)))


def set_slab_planes(planes: int):
    """Interior z-planes per slab of the split stage paths (0: the whole box)."""
    _check(lib().grf_set_slab_planes(int(planes)))


def get_slab_planes() -> int:
    return int(lib().grf_get_slab_planes())


def get_stage_path() -> int:
    return int(lib().grf_get_stage_path())


def get_tile_variant() -> int:
    return int(lib().grf_get_tile_variant())


def measure_peaks(nbytes: int = 1 << 31, stream=None):
    """-> (FP64 TFLOP/s of an FMA-chain kernel, GB/s of a device copy)."""
    scratch = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    f, c = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().grf_measure_peaks(_ptr(scratch), scratch.numel() * 8, _stream(stream), ctypes.byref(f),
                                   ctypes.byref(c)))
    return f.value, c.value


def prof_begin(max_launches: int):
    _check(lib().grf_prof_begin(int(max_launches)))


def prof_end():
    """-> {'deriv': (ms, n), 'point': (ms, n), 'vjp': (ms, n), 'vjp_point': (ms, n)}
    from HIP events ('vjp': whole right-hand-side VJPs, 'vjp_point': their
    reverse pointwise kernel)."""
    ms = (ctypes.c_double * 4)()
    cnt = (ctypes.c_int * 4)()
    _check(lib().grf_prof_end(ms, cnt))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(("deriv", "point", "vjp", "vjp_point"))}


def flops_per_cell(which=0) -> int:
    return int(lib().grf_flops_per_cell(int(which)))


class Stepper:
    """Classic RK4 steps of one box, all buffers resident on the device.

    Buffers: u (current state), ua, ub (stage states), acc (compact
    accumulator), ws (workspace).  Frozen ghosts: ua and ub start as copies of
    u so that their ghosts hold the frozen values."""

    def __init__(self, params: Params, box: Box, u: torch.Tensor, dt: float):
        self.params, self.box, self.dt = params, box, float(dt)
        self.u = u.contiguous()
        self.ua = self.u.clone()
        self.ub = self.u.clone()
        n = box.nx * box.ny * box.nz
        self.acc = torch.zeros((NF, n), dtype=torch.float64, device=u.device)
        self.ws = alloc_workspace(workspace_bytes(box), u.device)

    def step(self, stream=None):
        p, b, dt = self.params, self.box, self.dt
        rk4_stage(p, b, 1, dt, self.u, self.u, self.ua, self.acc, self.ws, stream)
        rk4_stage(p, b, 2, dt, self.u, self.ua, self.ub, self.acc, self.ws, stream)
        rk4_stage(p, b, 3, dt, self.u, self.ub, self.ua, self.acc, self.ws, stream)
        rk4_stage(p, b, 4, dt, self.u, self.ua, self.ub, self.acc, self.ws, stream)
        self.u, self.ub = self.ub, self.u

    def status(self):
        return status_fetch(self.ws)


class StepperBC(Stepper):
    """Classic RK4 steps of one box with per-face boundary rules (BC).  The
    fill-rule ghosts of u are filled first; gacc accumulates the stages of the
    Sommerfeld ghosts."""

    def __init__(self, params: Params, box: Box, u: torch.Tensor, dt: float, bc: BC):
        u = u.contiguous()
        bc_fill(bc, box, u)
        super().__init__(params, box, u, dt)
        self.bc = bc
        self.gacc = torch.zeros((NF, bc_ghost_cells(box)), dtype=torch.float64, device=u.device)

    def step(self, stream=None):
        p, b, c, dt = self.params, self.box, self.bc, self.dt
        rk4_stage_bc(p, b, c, 1, dt, self.u, self.u, self.ua, self.acc, self.gacc, self.ws, stream)
        rk4_stage_bc(p, b, c, 2, dt, self.u, self.ua, self.ub, self.acc, self.gacc, self.ws, stream)
        rk4_stage_bc(p, b, c, 3, dt, self.u, self.ub, self.ua, self.acc, self.gacc, self.ws, stream)
        rk4_stage_bc(p, b, c, 4, dt, self.u, self.ua, self.ub, self.acc, self.gacc, self.ws, stream)
        self.u, self.ub = self.ub, self.u


class Batch:
    """Boxes of uneven sizes and levels advanced together (frozen ghosts).

    states: list of device tensors (state layout, one per box), advanced in
    place: after every step each box's new state is in its tensor (the stage
    states live in the batch's scratch); `state(b)` returns that tensor."""

    def __init__(self, params: Params, boxes, states, dts):
        self.params = params
        self.nb = len(boxes)
        self.boxes = (Box * self.nb)(*boxes)
        self.states = [s.contiguous() for s in states]
        self._ptrs = (_vp * self.nb)(*[s.data_ptr() for s in self.states])
        self._dts = (ctypes.c_double * self.nb)(*[float(d) for d in dts])
        nbytes = int(lib().grf_batch_scratch_bytes(self.boxes, self.nb))
        if nbytes == 0:
            raise ValueError("invalid boxes")
        self.scratch = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=self.states[0].device)
        h = _vp()
        _check(lib().grf_batch_create(ctypes.byref(params), self.boxes, self.nb, self._ptrs, self._dts,
                                      _ptr(self.scratch), nbytes, ctypes.byref(h)))
        self.h = h
        self.graphs = []

    def step(self, stream=None):
        _check(lib().grf_batch_step(self.h, _stream(stream)))

    def rk4_stage(self, stage, stream=None):
        """One RK4 stage (1..4) of every box; four in order make one step."""
        _check(lib().grf_batch_rk4_stage(self.h, int(stage), _stream(stream)))

    def step_perbox(self, stream=None):
        _check(lib().grf_batch_step_perbox(self.h, _stream(stream)))

    def autotune(self, stream=None):
        _check(lib().grf_batch_autotune(self.h, _stream(stream)))

    def tile_variant(self, b):
        v = ctypes.c_int(0)
        _check(lib().grf_batch_tile_variant(self.h, int(b), ctypes.byref(v)))
        return v.value

    def set_tile_variant(self, b, v):
        _check(lib().grf_batch_set_tile_variant(self.h, int(b), int(v)))

    def capture(self, stream):
        """Executable graph of one batched RK4 step (four stages), captured on
        `stream` (non-default); every replay advances the batch one step."""
        g = _vp()
        _check(lib().grf_batch_capture_step(self.h, _stream(stream), ctypes.byref(g)))
        self.graphs.append(g)
        return g

    def replay(self, graph, stream=None):
        _check(lib().grf_graph_launch(graph, _stream(stream)))

    def state(self, b):
        p = _vp()
        _check(lib().grf_batch_state(self.h, int(b), ctypes.byref(p)))
        assert p.value == self.states[b].data_ptr()
        return self.states[b]

    def status(self, stream=None):
        bits = ctypes.c_uint32(0)
        code = lib().grf_batch_status_fetch(self.h, _stream(stream), ctypes.byref(bits))
        return code, int(bits.value)

    def close(self):
        if getattr(self, "h", None):
            for g in self.graphs:
                lib().grf_graph_destroy(g)
            self.graphs = []
            lib().grf_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def __getattr__(name):
    """grf.Evolve / grf.Trajectory: the checkpointed trajectory adjoint of
    adjoint.py (imported on first use; that module builds on this one)."""
    if name in ("Evolve", "Trajectory", "shell_phi2"):
        from . import adjoint
        return getattr(adjoint, name)
    raise AttributeError(name)
