"""Python face of the solver: a Plan owning its device workspace, solve/adjoint
calls on torch tensors, and a torch.autograd.Function whose backward is the
hand-written adjoint solve.

Tensors are device-resident, C-contiguous, shaped (batch, nz, ny, nx) (or
(nz, ny, nx) for batch 1), float64 for 'f64' and 'f32_refined', float32 for
'f32'.  Every launch goes on torch's current HIP stream.
"""

import ctypes

import torch

from . import _lib

DTYPES = {"f64": (_lib.PP_F64, torch.float64), "f32": (_lib.PP_F32, torch.float32),
          "f32_refined": (_lib.PP_F32_REFINED, torch.float64)}
GAUGES = {"mean": _lib.PP_GAUGE_MEAN, "pin": _lib.PP_GAUGE_PIN, "pin_raw": _lib.PP_GAUGE_PIN_RAW}
ZSOLVERS = {"thomas": 0, "pcr": 1, "cr": 2}
ZSPLITS = {"auto": 0, "off": 1, "on": 2, "seg": 3}


class Plan:
    """A solve plan for grids of shape (nz, ny, nx) with boundary string bc
    (x-, x+, y-, y+, z-, z+ from 'P', 'D', 'N') and spacings h = (hx, hy, hz)."""

    def __init__(self, shape, bc, h, dtype="f64", batch=1, gauge="mean", device=None,
                 refine_tol=None, refine_max_iter=None, zsolver="thomas", zsplit="auto"):
        lib = _lib.load()
        nz, ny, nx = (int(v) for v in shape)
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {sorted(DTYPES)}")
        if gauge not in GAUGES:
            raise ValueError(f"gauge must be one of {sorted(GAUGES)}")
        if not isinstance(bc, str) or len(bc) != 6:
            raise ValueError("bc must be a 6-character string")
        self.shape = (nz, ny, nx)
        self.bc = bc
        self.h = tuple(float(v) for v in h)
        self.dtype = dtype
        self.batch = int(batch)
        self.gauge = gauge
        self.code, self.torch_dtype = DTYPES[dtype]
        hh = (ctypes.c_double * 3)(*self.h)
        handle = ctypes.c_void_p()
        _lib.check(lib.pp_plan_create(nx, ny, nz, bc.encode(), hh, self.code, self.batch, ctypes.byref(handle)),
                   "pp_plan_create")
        self._handle = handle
        _lib.check(lib.pp_plan_set_gauge(handle, GAUGES[gauge]), "pp_plan_set_gauge")
        if zsolver not in ZSOLVERS:
            raise ValueError(f"zsolver must be one of {sorted(ZSOLVERS)}")
        _lib.check(lib.pp_plan_set_zsolver(handle, ZSOLVERS[zsolver]), "pp_plan_set_zsolver")
        self.zsolver = zsolver
        if zsplit not in ZSPLITS:
            raise ValueError(f"zsplit must be one of {sorted(ZSPLITS)}")
        _lib.check(lib.pp_plan_set_zsplit(handle, ZSPLITS[zsplit]), "pp_plan_set_zsplit")
        self.zsplit = zsplit
        if refine_tol is not None or refine_max_iter is not None:
            _lib.check(lib.pp_plan_set_refinement(handle, 1e-13 if refine_tol is None else float(refine_tol),
                                                  8 if refine_max_iter is None else int(refine_max_iter)),
                       "pp_plan_set_refinement")
        self.workspace_bytes = int(lib.pp_plan_workspace_bytes(handle))
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.device = device
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def __del__(self):
        h = getattr(self, "_handle", None)
        if h is not None and h.value:
            try:
                _lib.load().pp_plan_destroy(h)
            except Exception:
                pass
            self._handle = None

    def _check_tensor(self, t, name):
        full = (self.batch,) + self.shape
        if tuple(t.shape) != full and not (self.batch == 1 and tuple(t.shape) == self.shape):
            raise ValueError(f"{name} must have shape {full}, got {tuple(t.shape)}")
        if t.dtype != self.torch_dtype:
            raise TypeError(f"{name} must be {self.torch_dtype}, got {t.dtype}")
        if t.device != self.workspace.device:
            raise ValueError(f"{name} must live on {self.workspace.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def _run(self, fn, src, out, what):
        self._check_tensor(src, "input")
        if out is None:
            out = torch.empty_like(src)
        self._check_tensor(out, "out")
        stream = torch.cuda.current_stream(self.workspace.device).cuda_stream
        status = fn(self._handle, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                    ctypes.c_void_p(self.workspace.data_ptr()), ctypes.c_void_p(stream))
        _lib.check(status, what)
        return out

    def face_shape(self, i):
        """Shape of the value array of face i (x-, x+, y-, y+, z-, z+)."""
        nz, ny, nx = self.shape
        dims = [(nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)][i]
        return (self.batch,) + dims

    def solve(self, f, out=None, faces=None):
        """u with L_h u = f (see include/ppsolve.h for the zero-mode gauge).

        faces: optional sequence of six tensors or None (x-, x+, y-, y+, z-, z+):
        Dirichlet face values or Neumann outward derivatives, each of shape
        face_shape(i) (the batch axis may be dropped for batch 1), in f's dtype,
        on f's device.  Periodic faces take None."""
        if faces is None:
            return self._run(_lib.load().pp_solve, f, out, "pp_solve")
        if len(faces) != 6:
            raise ValueError("faces must hold six entries (x-, x+, y-, y+, z-, z+)")
        ptrs = (ctypes.c_void_p * 6)()
        keep = []
        for i, g in enumerate(faces):
            if g is None:
                continue
            full = self.face_shape(i)
            if tuple(g.shape) != full and not (self.batch == 1 and tuple(g.shape) == full[1:]):
                raise ValueError(f"face {i} must have shape {full}, got {tuple(g.shape)}")
            if g.dtype != self.torch_dtype or g.device != self.workspace.device or not g.is_contiguous():
                raise ValueError(f"face {i} must be a contiguous {self.torch_dtype} tensor on {self.workspace.device}")
            ptrs[i] = g.data_ptr()
            keep.append(g)
        lib = _lib.load()

        def call(plan, src, dst, ws, stream):
            return lib.pp_solve_bc(plan, src, ptrs, dst, ws, stream)

        return self._run(call, f, out, "pp_solve_bc")

    def solve_noalloc(self, f, out=None):
        """solve() through pp_solve_noalloc: the library's fixed per-device
        workspace instead of this plan's (no device allocation in the call when
        out is given)."""
        lib = _lib.load()

        def call(plan, src, dst, ws, stream):
            return lib.pp_solve_noalloc(plan, src, dst, stream)

        return self._run(call, f, out, "pp_solve_noalloc")

    def adjoint(self, g, out=None):
        """G^T g for the map G: f -> u of solve()."""
        return self._run(_lib.load().pp_solve_adjoint, g, out, "pp_solve_adjoint")

    def last_info(self):
        """(refinement steps, removed source mean per batch entry, last relative correction)."""
        it = ctypes.c_int()
        rel = ctypes.c_double()
        means = (ctypes.c_double * self.batch)()
        _lib.check(_lib.load().pp_plan_last_info(self._handle, ctypes.byref(it), means, ctypes.byref(rel)),
                   "pp_plan_last_info")
        return it.value, list(means), rel.value


class PoissonSolve(torch.autograd.Function):
    """u = G f with dJ/df = G^T dJ/du computed by the adjoint solve."""

    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        return plan.solve(f.contiguous())

    @staticmethod
    def backward(ctx, grad_u):
        return ctx.plan.adjoint(grad_u.contiguous()), None


def poisson_solve(f, plan):
    return PoissonSolve.apply(f, plan)
