"""ctypes binding of libggem (the C-ABI in include/ggem.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the evaluation runs in the library's HIP kernels.  If
the shared library has not been built, importing works but creating a plan
raises, so no evaluation can silently fall back to anything else.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libggem.so")

INTERP_LAGRANGE = 0
INTERP_SPECTRAL = 1
FLOW_SHEAR = 0
FLOW_POISEUILLE = 1

FP64 = 0
MIXED = 1
MIXED_BF16 = 2
PRECISIONS = {"fp64": FP64, "mixed": MIXED, "mixed_bf16": MIXED_BF16}
PART_LOCAL = 1
PART_GLOBAL = 2
PART_ALL = 3

OK = 0
E_ARG = -1
E_DOMAIN = -2
E_CAPACITY = -3
E_NOMEM = -4
E_DEVICE = -5

EXPORTS = (
    "ggem_plan_create", "ggem_plan_destroy", "ggem_plan_set_stream", "ggem_plan_status",
    "ggem_single_layer", "ggem_double_layer", "ggem_spread_grid", "ggem_plan_time_stage",
    "ggem_plan_stage_time", "ggem_plan_work", "ggem_plan_count_work", "ggem_plan_set_interp",
    "ggem_solver_create",
    "ggem_solver_destroy",
    "ggem_fredholm_apply", "ggem_fredholm_solve", "ggem_surface_geometry", "ggem_drop_rhs",
    "ggem_surface_velocity", "ggem_advance", "ggem_fredholm_solve_guided", "ggem_mlp_create",
    "ggem_mlp_destroy", "ggem_mlp_set_params", "ggem_mlp_get_params", "ggem_mlp_features",
    "ggem_mlp_forward", "ggem_mlp_predict", "ggem_mlp_gradients", "ggem_mlp_train_step",
    "ggem_batch_create", "ggem_batch_destroy", "ggem_batch_single_layer",
    "ggem_batch_capture_single_layer", "ggem_batch_graph_launch", "ggem_batch_status",
    "ggem_batch_branch", "ggem_single_layer_noalloc", "ggem_rigid_create", "ggem_rigid_destroy",
    "ggem_bi_single_layer", "ggem_bi_double_layer", "ggem_rigid_solve", "ggem_poiseuille",
    "ggem_probe", "ggem_undisturbed_traction", "ggem_particle_stress", "ggem_traction_rhs",
    "ggem_membrane_create", "ggem_membrane_destroy", "ggem_membrane_traction",
    "ggem_capsule_volumes", "ggem_volume_correct", "ggem_capsule_separation",
    "ggem_overlap_correct", "ggem_bi_surface_velocity", "ggem_bi_fredholm_solve",
    "ggem_last_error",
)

MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 13, 128, 3, 35203

STAGES = ("bin", "near", "wall", "spread", "fft_fwd", "cheb_fwd", "tau", "cheb_inv",
          "fft_inv", "interp")


class GGEMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ggem error {code}: {msg}")
        self.code = code


class SolverParams(ctypes.Structure):
    _fields_ = [("max_nodes", ctypes.c_longlong), ("max_tri", ctypes.c_longlong),
                ("restart", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_double), ("Lz", ctypes.c_double), ("H", ctypes.c_double),
        ("alpha", ctypes.c_double), ("rc", ctypes.c_double),
        ("Nx", ctypes.c_int), ("Nz", ctypes.c_int), ("Ny", ctypes.c_int),
        ("precision", ctypes.c_int), ("sync_checks", ctypes.c_int),
        ("max_src", ctypes.c_longlong), ("max_tgt", ctypes.c_longlong),
        ("cell_scale", ctypes.c_double),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libggem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1109_6587_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp, ll, dp, ip = ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p, ctypes.c_int
    lib.ggem_plan_create.argtypes = [ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    lib.ggem_plan_destroy.argtypes = [vp]
    lib.ggem_plan_set_stream.argtypes = [vp, vp]
    lib.ggem_plan_status.argtypes = [vp]
    lib.ggem_single_layer.argtypes = [vp, ll, dp, dp, ll, dp, dp, ip]
    lib.ggem_double_layer.argtypes = [vp, ll, dp, dp, ll, dp, dp, dp, ip]
    lib.ggem_spread_grid.argtypes = [vp, ll, dp, dp, dp]
    lib.ggem_single_layer_noalloc.argtypes = [ctypes.POINTER(Params), vp, ll, dp, dp, ll, dp, dp]
    lib.ggem_plan_time_stage.argtypes = [vp, ip, ip]
    lib.ggem_plan_stage_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int)]
    lib.ggem_plan_work.argtypes = [vp, ctypes.POINTER(ctypes.c_ulonglong)]
    lib.ggem_plan_count_work.argtypes = [vp, ip]
    lib.ggem_plan_set_interp.argtypes = [vp, ip, ip]
    lib.ggem_solver_create.argtypes = [vp, ctypes.POINTER(SolverParams), ctypes.POINTER(vp)]
    lib.ggem_solver_destroy.argtypes = [vp]
    dd = ctypes.c_double
    lib.ggem_fredholm_apply.argtypes = [vp, ll, dp, dp, dp, dd, ll, dp, dp, dp]
    lib.ggem_fredholm_solve.argtypes = [vp, ll, dp, dp, dp, dd, ll, dp, dp, dp, dd, ip,
                                        ctypes.POINTER(ip), ctypes.POINTER(dd)]
    lib.ggem_surface_geometry.argtypes = [vp, ll, dp, ll, dp, dp, dp, dp, dp, dp]
    lib.ggem_drop_rhs.argtypes = [vp, ll, dp, dp, dd, dd, dd, dp]
    lib.ggem_surface_velocity.argtypes = [vp, ll, dp, ll, dp, dp, dd, dp]
    lib.ggem_advance.argtypes = [vp, ll, dp, dp, dd, dp]
    lib.ggem_traction_rhs.argtypes = [vp, ll, dp, dp, dd, dd, dp]
    lib.ggem_bi_surface_velocity.argtypes = [vp, ll, dp, ll, dp, dp, dp, dp, dd, dp]
    lib.ggem_bi_fredholm_solve.argtypes = [vp, ll, dp, ll, dp, dp, dp, dp, dd, dp, dp, dd, ip,
                                           ctypes.POINTER(ip), ctypes.POINTER(dd)]
    lib.ggem_membrane_create.argtypes = [vp, ll, ip, ip, dp, dp, dd, ctypes.POINTER(vp)]
    lib.ggem_membrane_destroy.argtypes = [vp]
    lib.ggem_membrane_traction.argtypes = [vp, dp, dp, dp, dp, ctypes.POINTER(dd)]
    lib.ggem_capsule_volumes.argtypes = [vp, dp, dp]
    lib.ggem_volume_correct.argtypes = [vp, dp, dp, dp, dp, dd, ctypes.POINTER(ip)]
    lib.ggem_capsule_separation.argtypes = [vp, dp, dd, dd, dd, ctypes.POINTER(dd),
                                            ctypes.POINTER(dd)]
    lib.ggem_overlap_correct.argtypes = [vp, dp, dd, dd, dd, dd, ip, ctypes.POINTER(ip)]
    lib.ggem_rigid_create.argtypes = [vp, ll, ll, ip, ctypes.POINTER(vp)]
    lib.ggem_rigid_destroy.argtypes = [vp]
    lib.ggem_bi_single_layer.argtypes = [vp, ll, dp, ll, dp, dp, dp, dp, dp]
    lib.ggem_bi_double_layer.argtypes = [vp, ll, dp, ll, dp, dp, dp, dp, dp, dp]
    lib.ggem_rigid_solve.argtypes = [vp, ll, dp, ll, dp, dp, dp, ctypes.POINTER(dd), dp, dp,
                                     ctypes.POINTER(dd), dd, ip, ctypes.POINTER(ip),
                                     ctypes.POINTER(dd)]
    lib.ggem_poiseuille.argtypes = [vp, dd, ll, dp, dp]
    lib.ggem_probe.argtypes = [vp, ll, dp, dp, ll, dp, dp, dp, dp]
    lib.ggem_undisturbed_traction.argtypes = [vp, ip, dd, ll, dp, dp, dp]
    lib.ggem_particle_stress.argtypes = [vp, ll, dp, ll, dp, dp, dp, dp, dp, dp, dd, dd,
                                         ctypes.POINTER(dd)]
    fp = ctypes.POINTER(ctypes.c_float)
    lib.ggem_fredholm_solve_guided.argtypes = [vp, ll, dp, dp, dp, dd, ll, dp, dp, dp, dp, dd, ip,
                                               ctypes.POINTER(ip), ctypes.POINTER(dd),
                                               ctypes.POINTER(dd)]
    lib.ggem_mlp_create.argtypes = [ip, vp, ctypes.POINTER(vp)]
    lib.ggem_mlp_destroy.argtypes = [vp]
    lib.ggem_mlp_set_params.argtypes = [vp, dp]
    lib.ggem_mlp_get_params.argtypes = [vp, dp]
    lib.ggem_mlp_features.argtypes = [vp, ll, dp, dp, dp, dp, dp, ip, fp, dp]
    lib.ggem_mlp_forward.argtypes = [vp, ll, dp, dp]
    lib.ggem_mlp_predict.argtypes = [vp, ll, dp, dd, dp]
    lib.ggem_mlp_gradients.argtypes = [vp, ll, dp, dp, dp, fp]
    lib.ggem_mlp_train_step.argtypes = [vp, ll, dp, dp, ctypes.c_float, fp]
    lp = ctypes.POINTER(ctypes.c_longlong)
    lib.ggem_batch_create.argtypes = [ip, ctypes.POINTER(Params), ip, ctypes.POINTER(vp)]
    lib.ggem_batch_destroy.argtypes = [vp]
    lib.ggem_batch_single_layer.argtypes = [vp, vp, lp, dp, dp, lp, dp, dp]
    lib.ggem_batch_capture_single_layer.argtypes = [vp, lp, dp, dp, lp, dp, dp]
    lib.ggem_batch_graph_launch.argtypes = [vp, vp]
    lib.ggem_batch_status.argtypes = [vp, vp]
    lib.ggem_batch_branch.argtypes = [vp, ip]
    lib.ggem_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "ggem_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code: int):
    if code != OK:
        msg = _lib.ggem_last_error()
        raise GGEMError(code, msg.decode() if msg else "")


def _dev_ptr(t, name, n=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.dim() != 2 or t.shape[1] != 3 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous (n, 3) tensor")
    if n is not None and t.shape[0] != n:
        raise ValueError(f"{name} must have {n} rows")
    return t.data_ptr()


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A GGEM plan: box, split parameter, grid, precision and capacities."""

    def __init__(self, Lx, Lz, H, alpha, Nx, Nz, Ny, rc=0.0, precision="fp64",
                 max_src=1, max_tgt=1, sync_checks=True, stream=None, cell_scale=0.0):
        lib = load_library()
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.params = Params(float(Lx), float(Lz), float(H), float(alpha), float(rc),
                             int(Nx), int(Nz), int(Ny), prec, 1 if sync_checks else 0,
                             int(max_src), int(max_tgt), float(cell_scale))
        self.Nx, self.Nz, self.Ny = int(Nx), int(Nz), int(Ny)
        self._h = ctypes.c_void_p()
        _check(lib.ggem_plan_create(ctypes.byref(self.params), _stream_handle(stream),
                                    ctypes.byref(self._h)))

    @classmethod
    def from_case(cls, c, precision="fp64", max_src=None, max_tgt=None, **kw):
        return cls(c.Lx, c.Lz, c.H, c.alpha, c.Nx, c.Nz, c.Ny, rc=c.rc, precision=precision,
                   max_src=max_src if max_src is not None else max(c.ns, 1),
                   max_tgt=max_tgt if max_tgt is not None else max(c.nt, 1), **kw)

    def close(self):
        if self._h:
            _check(_lib.ggem_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.ggem_plan_destroy(self._h)
        except Exception:
            pass

    def set_stream(self, stream):
        _check(_lib.ggem_plan_set_stream(self._h, _stream_handle(stream)))

    def status(self):
        _check(_lib.ggem_plan_status(self._h))

    def time_stage(self, stage, max_calls):
        """Record HIP events around one pipeline stage for the next calls."""
        sid = STAGES.index(stage) if isinstance(stage, str) else int(stage)
        _check(_lib.ggem_plan_time_stage(self._h, sid, int(max_calls)))

    def stage_time(self):
        """(total ms, number of evaluations) recorded for the timed stage."""
        ms = ctypes.c_double()
        n = ctypes.c_int()
        _check(_lib.ggem_plan_stage_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def count_work(self, on=True):
        """Have the kernels count their work units in the following calls."""
        _check(_lib.ggem_plan_count_work(self._h, 1 if on else 0))

    def set_interp(self, mode, msp=12):
        """Off-mesh evaluation of the global part: INTERP_LAGRANGE (4th-order
        stencil) or INTERP_SPECTRAL (the Fourier-Chebyshev series by NUFFT,
        msp oversampled nodes on each side)."""
        _check(_lib.ggem_plan_set_interp(self._h, int(mode), int(msp)))

    def work(self):
        """(local pairs, spread updates) counted by the kernels in the last call
        (zeros unless counting was on for it)."""
        c = (ctypes.c_ulonglong * 2)()
        _check(_lib.ggem_plan_work(self._h, c))
        return int(c[0]), int(c[1])

    def probe(self, xs, f, xt, out=None):
        """Velocity (nt, 3), pressure (nt,) and stress (nt, 6: xx, yy, zz, xy,
        xz, yz) of the point forces at the probes xt (ggem_probe); `out` may
        give the three arrays."""
        import torch
        ns, nt = xs.shape[0], xt.shape[0]
        if out is None:
            u = torch.empty((nt, 3), dtype=torch.float64, device=xt.device)
            p = torch.empty((nt,), dtype=torch.float64, device=xt.device)
            s = torch.empty((nt, 6), dtype=torch.float64, device=xt.device)
        else:
            u, p, s = out
            for t, shape in ((u, (nt, 3)), (p, (nt,)), (s, (nt, 6))):
                if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64
                        or t.shape != shape or not t.is_contiguous()):
                    raise TypeError(f"probe outputs must be contiguous float64 {shape} device tensors")
        _check(_lib.ggem_probe(self._h, ns, _dev_ptr(xs, "xs"), _dev_ptr(f, "f", ns), nt,
                               _dev_ptr(xt, "xt"), u.data_ptr(), p.data_ptr(), s.data_ptr()))
        return u, p, s

    def single_layer(self, xs, f, xt, parts=PART_ALL, out=None):
        import torch
        ns, nt = xs.shape[0], xt.shape[0]
        if out is None:
            out = torch.empty((nt, 3), dtype=torch.float64, device=xt.device)
        _check(_lib.ggem_single_layer(self._h, ns, _dev_ptr(xs, "xs"), _dev_ptr(f, "f", ns), nt,
                                      _dev_ptr(xt, "xt"), _dev_ptr(out, "out", nt), int(parts)))
        return out

    def double_layer(self, xs, q, xt, nrm, parts=PART_ALL, out=None):
        import torch
        ns, nt = xs.shape[0], xt.shape[0]
        if out is None:
            out = torch.empty((nt, 3), dtype=torch.float64, device=xt.device)
        _check(_lib.ggem_double_layer(self._h, ns, _dev_ptr(xs, "xs"), _dev_ptr(q, "q", ns), nt,
                                      _dev_ptr(xt, "xt"), _dev_ptr(nrm, "nrm", nt),
                                      _dev_ptr(out, "out", nt), int(parts)))
        return out

    def spread_grid(self, xs, f, out=None):
        import torch
        ns = xs.shape[0]
        if out is None:
            out = torch.empty((3, self.Ny, self.Nx, self.Nz), dtype=torch.float64, device=xs.device)
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
                and out.numel() == 3 * self.Ny * self.Nx * self.Nz):
            raise ValueError("out must be a contiguous float64 (3, Ny, Nx, Nz) device tensor")
        _check(_lib.ggem_spread_grid(self._h, ns, _dev_ptr(xs, "xs"), _dev_ptr(f, "f", ns),
                                     out.data_ptr()))
        return out


def single_layer_noalloc(Lx, Lz, H, alpha, Nx, Nz, Ny, xs, f, xt, rc=0.0, precision="fp64",
                         max_src=None, max_tgt=None, sync_checks=True, out=None, stream=None):
    """ggem_single_layer_noalloc: the single layer without a plan object, in
    the library's static per-GPU workspace (no device allocation inside the
    library).  Capacities default to the sizes of this call."""
    import torch
    lib = load_library()
    ns, nt = xs.shape[0], xt.shape[0]
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    prm = Params(float(Lx), float(Lz), float(H), float(alpha), float(rc), int(Nx), int(Nz),
                 int(Ny), prec, 1 if sync_checks else 0,
                 int(max_src if max_src is not None else max(ns, 1)),
                 int(max_tgt if max_tgt is not None else max(nt, 1)))
    if out is None:
        out = torch.empty((nt, 3), dtype=torch.float64, device=xt.device)
    _check(lib.ggem_single_layer_noalloc(ctypes.byref(prm), _stream_handle(stream), ns,
                                         _dev_ptr(xs, "xs"), _dev_ptr(f, "f", ns), nt,
                                         _dev_ptr(xt, "xt"), _dev_ptr(out, "out", nt)))
    return out


class Surface:
    """A triangulated surface on the device: nodes (n,3) f64, node normals
    (n,3) f64, triangles (m,3) int32, kappa per node (n,) f64 or a scalar."""

    def __init__(self, nodes, normals, tri, kappa):
        import torch
        self.nodes = nodes
        self.normals = normals
        if tri.dtype != torch.int32 or not tri.is_cuda or not tri.is_contiguous():
            raise TypeError("tri must be a contiguous int32 device tensor")
        self.tri = tri
        if isinstance(kappa, (int, float)):
            self.kappa, self.kappa0 = None, float(kappa)
        else:
            if (not isinstance(kappa, torch.Tensor) or not kappa.is_cuda
                    or kappa.dtype != torch.float64 or kappa.shape != (nodes.shape[0],)
                    or not kappa.is_contiguous()):
                raise TypeError("kappa must be a float or a contiguous (n,) float64 device tensor")
            self.kappa, self.kappa0 = kappa, 0.0

    def args(self):
        n = self.nodes.shape[0]
        kp = self.kappa.data_ptr() if self.kappa is not None else None
        return (n, _dev_ptr(self.nodes, "nodes"), _dev_ptr(self.normals, "normals", n), kp,
                self.kappa0, self.tri.shape[0], self.tri.data_ptr())


class FredholmSolver:
    """GMRES(m) for (I + kappa/4pi D) q = b on a plan (see include/ggem.h)."""

    def __init__(self, plan, max_nodes, max_tri, restart=30):
        self.plan = plan
        self._h = ctypes.c_void_p()
        prm = SolverParams(int(max_nodes), int(max_tri), int(restart))
        _check(_lib.ggem_solver_create(plan._h, ctypes.byref(prm), ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _check(_lib.ggem_solver_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.ggem_solver_destroy(self._h)
        except Exception:
            pass

    def apply(self, surf, x, out=None):
        import torch
        if out is None:
            out = torch.empty_like(x)
        _check(_lib.ggem_fredholm_apply(self._h, *surf.args(), _dev_ptr(x, "x"),
                                        _dev_ptr(out, "out")))
        return out

    def solve_guided(self, surf, b, q, dq, tol=1e-6, max_iter=200):
        """Solve from q + c dq (c chosen by the residual); returns (iters, rel_res, c)."""
        it = ctypes.c_int()
        rr = ctypes.c_double()
        st = ctypes.c_double()
        _check(_lib.ggem_fredholm_solve_guided(self._h, *surf.args(), _dev_ptr(b, "b"),
                                               _dev_ptr(q, "q"), _dev_ptr(dq, "dq"), float(tol),
                                               int(max_iter), ctypes.byref(it), ctypes.byref(rr),
                                               ctypes.byref(st)))
        return it.value, rr.value, st.value

    def solve(self, surf, b, q, tol=1e-6, max_iter=200):
        """Solve in place into q (initial guess on entry); returns (iters, rel_res)."""
        it = ctypes.c_int()
        rr = ctypes.c_double()
        _check(_lib.ggem_fredholm_solve(self._h, *surf.args(), _dev_ptr(b, "b"),
                                        _dev_ptr(q, "q"), float(tol), int(max_iter),
                                        ctypes.byref(it), ctypes.byref(rr)))
        return it.value, rr.value

    def geometry(self, nodes, tri, node_tri_off, node_tri):
        """Node normals, areas and Lap x of a triangulation (ggem_surface_geometry)."""
        import torch
        n = nodes.shape[0]
        _int_dev(tri, "tri", 2)
        _int_dev(node_tri_off, "node_tri_off", 1, n + 1)
        _int_dev(node_tri, "node_tri", 1)
        nrm = torch.empty_like(nodes)
        lap = torch.empty_like(nodes)
        area = torch.empty((n,), dtype=torch.float64, device=nodes.device)
        _check(_lib.ggem_surface_geometry(self._h, n, _dev_ptr(nodes, "nodes"), tri.shape[0],
                                          tri.data_ptr(), node_tri_off.data_ptr(),
                                          node_tri.data_ptr(), nrm.data_ptr(), area.data_ptr(),
                                          lap.data_ptr()))
        return nrm, area, lap

    def drop_rhs(self, normals, lap, lam, inv_ca, shear, out=None):
        import torch
        n = normals.shape[0]
        out = torch.empty_like(normals) if out is None else out
        _check(_lib.ggem_drop_rhs(self._h, n, _dev_ptr(normals, "normals"), _dev_ptr(lap, "lap", n),
                                  float(lam), float(inv_ca), float(shear), _dev_ptr(out, "out", n)))
        return out

    def traction_rhs(self, normals, df, lam, shear, out=None):
        """b of Eq. qa for a given traction jump (ggem_traction_rhs)."""
        import torch
        n = normals.shape[0]
        out = torch.empty_like(normals) if out is None else out
        _check(_lib.ggem_traction_rhs(self._h, n, _dev_ptr(normals, "normals"),
                                      _dev_ptr(df, "df", n), float(lam), float(shear),
                                      _dev_ptr(out, "out", n)))
        return out

    def velocity(self, nodes, tri, q, shear, out=None):
        import torch
        n = nodes.shape[0]
        _int_dev(tri, "tri", 2)
        out = torch.empty_like(nodes) if out is None else out
        _check(_lib.ggem_surface_velocity(self._h, n, _dev_ptr(nodes, "nodes"), tri.shape[0],
                                          tri.data_ptr(), _dev_ptr(q, "q", n), float(shear),
                                          _dev_ptr(out, "out", n)))
        return out

    def advance(self, x, u, dt, out=None):
        import torch
        n = x.shape[0]
        out = torch.empty_like(x) if out is None else out
        _check(_lib.ggem_advance(self._h, 3 * n, _dev_ptr(x, "x"), _dev_ptr(u, "u", n), float(dt),
                                 _dev_ptr(out, "out", n)))
        return out


class Membrane:
    """Neo-Hookean membranes of equal capsules on a Fredholm solver's stream
    (ggem_membrane_* in include/ggem.h)."""

    def __init__(self, solver, n_capsules, tri, ref_nodes, shear_modulus):
        n_tri, n_nodes = tri.shape[0], ref_nodes.shape[0]
        _int_dev(tri, "tri", 2)
        if n_tri % n_capsules or n_nodes % n_capsules:
            raise ValueError("nodes and triangles must split into equal capsules")
        self.solver = solver
        self.ncap = int(n_capsules)
        self.n_nodes = n_nodes
        self._h = ctypes.c_void_p()
        _check(_lib.ggem_membrane_create(solver._h, self.ncap, n_nodes // self.ncap,
                                         n_tri // self.ncap, tri.data_ptr(),
                                         _dev_ptr(ref_nodes, "ref_nodes"), float(shear_modulus),
                                         ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _check(_lib.ggem_membrane_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.ggem_membrane_destroy(self._h)
        except Exception:
            pass

    def traction(self, nodes, node_tri_off, node_tri, out=None, energy=False):
        """Traction jump (n, 3); with energy=True also the total energy."""
        import torch
        out = torch.empty_like(nodes) if out is None else out
        _int_dev(node_tri_off, "node_tri_off", 1, self.n_nodes + 1)
        _int_dev(node_tri, "node_tri", 1)
        e = ctypes.c_double()
        _check(_lib.ggem_membrane_traction(self._h, _dev_ptr(nodes, "nodes", self.n_nodes),
                                           node_tri_off.data_ptr(), node_tri.data_ptr(),
                                           _dev_ptr(out, "out", self.n_nodes),
                                           ctypes.byref(e) if energy else None))
        return (out, e.value) if energy else out

    def volumes(self, nodes, out=None):
        import torch
        out = torch.empty((self.ncap,), dtype=torch.float64, device=nodes.device) if out is None else out
        _check(_lib.ggem_capsule_volumes(self._h, _dev_ptr(nodes, "nodes", self.n_nodes),
                                         out.data_ptr()))
        return out

    def volume_correct(self, nodes, normals, area, v0, tol=1e-4):
        """Correct in place; returns the number of capsules moved."""
        import torch
        for t, name, n in ((area, "area", self.n_nodes), (v0, "v0", self.ncap)):
            if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64
                    or t.shape != (n,) or not t.is_contiguous()):
                raise TypeError(f"{name} must be a contiguous ({n},) float64 device tensor")
        k = ctypes.c_int()
        _check(_lib.ggem_volume_correct(self._h, _dev_ptr(nodes, "nodes", self.n_nodes),
                                        _dev_ptr(normals, "normals", self.n_nodes),
                                        area.data_ptr(), v0.data_ptr(), float(tol),
                                        ctypes.byref(k)))
        return k.value

    def separation(self, nodes, Lx, Lz, reach):
        """(shortest edge, smallest gap between capsules below reach or inf)."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(_lib.ggem_capsule_separation(self._h, _dev_ptr(nodes, "nodes", self.n_nodes),
                                            float(Lx), float(Lz), float(reach), ctypes.byref(a),
                                            ctypes.byref(b)))
        return a.value, b.value

    def overlap_correct(self, nodes, Lx, Lz, H, h_min, max_sweeps=100):
        """Correct in place; returns the number of sweeps that moved something."""
        k = ctypes.c_int()
        _check(_lib.ggem_overlap_correct(self._h, _dev_ptr(nodes, "nodes", self.n_nodes),
                                         float(Lx), float(Lz), float(H), float(h_min),
                                         int(max_sweeps), ctypes.byref(k)))
        return k.value


def _int_dev(t, name, dim, n=None):
    import torch
    if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32
            or t.dim() != dim or not t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {dim}-d int32 device tensor")
    if dim == 2 and t.shape[1] != 3:
        raise ValueError(f"{name} must have 3 columns")
    if n is not None and t.shape[0] != n:
        raise ValueError(f"{name} must have {n} entries")


def _f32_dev(t, name, cols):
    import torch
    if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32
            or t.dim() != 2 or t.shape[1] != cols or not t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous (n, {cols}) float32 device tensor")
    return t.data_ptr()


class MLP:
    """The warm-start network (ggem_mlp_*): 13 -> 128 -> 128 -> 128 -> 3."""

    def __init__(self, max_batch, params=None, stream=None):
        lib = load_library()
        self._h = ctypes.c_void_p()
        self.max_batch = int(max_batch)
        _check(lib.ggem_mlp_create(self.max_batch, _stream_handle(stream), ctypes.byref(self._h)))
        if params is not None:
            self.set_params(params)

    def close(self):
        if self._h:
            _check(_lib.ggem_mlp_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.ggem_mlp_destroy(self._h)
        except Exception:
            pass

    @staticmethod
    def _params_ptr(p):
        import torch
        if (not isinstance(p, torch.Tensor) or not p.is_cuda or p.dtype != torch.float32
                or p.shape != (MLP_PARAMS,) or not p.is_contiguous()):
            raise TypeError(f"params must be a contiguous ({MLP_PARAMS},) float32 device tensor")
        return p.data_ptr()

    def set_params(self, p):
        _check(_lib.ggem_mlp_set_params(self._h, self._params_ptr(p)))

    def get_params(self):
        import torch
        p = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        _check(_lib.ggem_mlp_get_params(self._h, p.data_ptr()))
        return p

    def features(self, nodes, normals, lap, q_prev, dq_prev, nodes_per_drop, scales, out=None):
        import torch
        n = nodes.shape[0]
        if out is None:
            out = torch.empty((n, MLP_IN), dtype=torch.float32, device=nodes.device)
        sc = (ctypes.c_float * MLP_IN)(*[float(v) for v in scales])
        _check(_lib.ggem_mlp_features(self._h, n, _dev_ptr(nodes, "nodes"),
                                      _dev_ptr(normals, "normals", n), _dev_ptr(lap, "lap", n),
                                      _dev_ptr(q_prev, "q_prev", n), _dev_ptr(dq_prev, "dq_prev", n),
                                      int(nodes_per_drop), sc,
                                      _f32_dev(out, "X", MLP_IN)))
        return out

    def forward(self, X):
        import torch
        Y = torch.empty((X.shape[0], MLP_OUT), dtype=torch.float32, device=X.device)
        _check(_lib.ggem_mlp_forward(self._h, X.shape[0], _f32_dev(X, "X", MLP_IN),
                                     Y.data_ptr()))
        return Y

    def predict(self, X, scale, out=None):
        import torch
        if out is None:
            out = torch.empty((X.shape[0], 3), dtype=torch.float64, device=X.device)
        _check(_lib.ggem_mlp_predict(self._h, X.shape[0], _f32_dev(X, "X", MLP_IN), float(scale),
                                     _dev_ptr(out, "dq", X.shape[0])))
        return out

    def gradients(self, X, T):
        import torch
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
        loss = ctypes.c_float()
        _check(_lib.ggem_mlp_gradients(self._h, X.shape[0], _f32_dev(X, "X", MLP_IN),
                                       _f32_dev(T, "T", MLP_OUT), g.data_ptr(), ctypes.byref(loss)))
        return float(loss.value), g

    def train_step(self, X, T, lr, want_loss=False):
        loss = ctypes.c_float()
        _check(_lib.ggem_mlp_train_step(self._h, X.shape[0], _f32_dev(X, "X", MLP_IN),
                                        _f32_dev(T, "T", MLP_OUT), float(lr),
                                        ctypes.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None


class Batch:
    """Independent slit problems evaluated together (ggem_batch_*).

    ``cases``: objects with Lx, Lz, H, alpha, rc, Nx, Nz, Ny and ns/nt (for
    the capacities), e.g. workloads.SlitCase."""

    def __init__(self, cases, precision="mixed", n_branches=4, cell_scales=None):
        """cell_scales: one ggem_params.cell_scale per instance (None: 0)."""
        lib = load_library()
        prec = PRECISIONS[precision]
        arr = (Params * len(cases))()
        if cell_scales is None:
            cell_scales = [0.0] * len(cases)
        if len(cell_scales) != len(cases):
            raise ValueError("cell_scales must have one entry per instance")
        for i, c in enumerate(cases):
            arr[i] = Params(float(c.Lx), float(c.Lz), float(c.H), float(c.alpha), float(c.rc),
                            int(c.Nx), int(c.Nz), int(c.Ny), prec, 0, max(int(c.ns), 1),
                            max(int(c.nt), 1), float(cell_scales[i]))
        self.n = len(cases)
        self._h = ctypes.c_void_p()
        _check(lib.ggem_batch_create(self.n, arr, int(n_branches), ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _check(_lib.ggem_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.ggem_batch_destroy(self._h)
        except Exception:
            pass

    def _offs(self, off):
        if len(off) != self.n + 1:
            raise ValueError(f"offsets must have {self.n + 1} entries")
        return (ctypes.c_longlong * (self.n + 1))(*[int(v) for v in off])

    def _arrays(self, src_off, xs, f, tgt_off, xt, u):
        ns, nt = int(src_off[-1]), int(tgt_off[-1])
        return (self._offs(src_off), _dev_ptr(xs, "xs", ns), _dev_ptr(f, "f", ns),
                self._offs(tgt_off), _dev_ptr(xt, "xt", nt), _dev_ptr(u, "u", nt))

    def single_layer(self, src_off, xs, f, tgt_off, xt, u, stream=None):
        so, a, b, to, c, d = self._arrays(src_off, xs, f, tgt_off, xt, u)
        _check(_lib.ggem_batch_single_layer(self._h, _stream_handle(stream), so, a, b, to, c, d))
        return u

    def capture(self, src_off, xs, f, tgt_off, xt, u):
        so, a, b, to, c, d = self._arrays(src_off, xs, f, tgt_off, xt, u)
        _check(_lib.ggem_batch_capture_single_layer(self._h, so, a, b, to, c, d))

    def replay(self, stream=None):
        _check(_lib.ggem_batch_graph_launch(self._h, _stream_handle(stream)))

    def status(self, stream=None):
        _check(_lib.ggem_batch_status(self._h, _stream_handle(stream)))

    def branch(self, i):
        r = _lib.ggem_batch_branch(self._h, int(i))
        if r < 0:
            _check(r)
        return r


class RigidParticle:
    """Boundary-integral single layer on a triangulated surface and the
    force- and torque-free rigid particle (see include/ggem.h)."""

    def __init__(self, plan, max_nodes, max_tri, restart=100):
        self.plan = plan
        self._h = ctypes.c_void_p()
        _check(_lib.ggem_rigid_create(plan._h, int(max_nodes), int(max_tri), int(restart),
                                      ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _check(_lib.ggem_rigid_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h and _lib is not None:
                _lib.ggem_rigid_destroy(self._h)
        except Exception:
            pass

    @staticmethod
    def _mesh(nodes, tri, inc_off, inc_tri):
        n = nodes.shape[0]
        _int_dev(tri, "tri", 2)
        _int_dev(inc_off, "inc_off", 1, n + 1)
        _int_dev(inc_tri, "inc_tri", 1)
        return (n, _dev_ptr(nodes, "nodes"), tri.shape[0], tri.data_ptr(), inc_off.data_ptr(),
                inc_tri.data_ptr())

    def single_layer(self, nodes, tri, inc_off, inc_tri, f, out=None):
        """(1/8pi) int f G dS at the nodes (ggem_bi_single_layer)."""
        import torch
        m = self._mesh(nodes, tri, inc_off, inc_tri)
        out = torch.empty_like(nodes) if out is None else out
        _check(_lib.ggem_bi_single_layer(self._h, *m, _dev_ptr(f, "f", m[0]),
                                         _dev_ptr(out, "out", m[0])))
        return out

    def double_layer(self, nodes, tri, inc_off, inc_tri, normals, q, out=None):
        """(1/8pi) n(z) . int q T dS at the nodes, n~ on the elements at z
        (ggem_bi_double_layer)."""
        import torch
        m = self._mesh(nodes, tri, inc_off, inc_tri)
        out = torch.empty_like(nodes) if out is None else out
        _check(_lib.ggem_bi_double_layer(self._h, *m, _dev_ptr(normals, "normals", m[0]),
                                         _dev_ptr(q, "q", m[0]), _dev_ptr(out, "out", m[0])))
        return out

    def surface_velocity(self, nodes, tri, inc_off, inc_tri, q, shear, out=None):
        """u = (shear y, 0, 0) + 8 pi w(q) at the nodes (ggem_bi_surface_velocity)."""
        import torch
        m = self._mesh(nodes, tri, inc_off, inc_tri)
        out = torch.empty_like(nodes) if out is None else out
        _check(_lib.ggem_bi_surface_velocity(self._h, *m, _dev_ptr(q, "q", m[0]), float(shear),
                                             _dev_ptr(out, "out", m[0])))
        return out

    def fredholm_solve(self, nodes, tri, inc_off, inc_tri, normals, kappa, b, q, tol=1e-6,
                       max_iter=200):
        """q + 2 kappa v(q) = b in place into q (guess on entry); returns
        (iters, rel_res) (ggem_bi_fredholm_solve)."""
        m = self._mesh(nodes, tri, inc_off, inc_tri)
        it = ctypes.c_int()
        rr = ctypes.c_double()
        _check(_lib.ggem_bi_fredholm_solve(self._h, *m, _dev_ptr(normals, "normals", m[0]),
                                           float(kappa), _dev_ptr(b, "b", m[0]),
                                           _dev_ptr(q, "q", m[0]), float(tol), int(max_iter),
                                           ctypes.byref(it), ctypes.byref(rr)))
        return it.value, rr.value

    def particle_stress(self, nodes, tri, inc_off, inc_tri, normals, df, u, lam, volume):
        """Sigma^p (3 x 3 nested list) of Sec. 7.1 (ggem_particle_stress)."""
        m = self._mesh(nodes, tri, inc_off, inc_tri)
        out = (ctypes.c_double * 9)()
        _check(_lib.ggem_particle_stress(self._h, *m, _dev_ptr(normals, "normals", m[0]),
                                         _dev_ptr(df, "df", m[0]), _dev_ptr(u, "u", m[0]),
                                         float(lam), float(volume), out))
        return [list(out[3 * i:3 * i + 3]) for i in range(3)]

    def solve(self, nodes, tri, inc_off, inc_tri, center, uinf, f, motion=None, tol=1e-10,
              max_iter=400):
        """Solve in place into f (initial guess on entry); returns
        (U, Omega, iters, rel_res)."""
        m = self._mesh(nodes, tri, inc_off, inc_tri)
        c = (ctypes.c_double * 3)(*[float(v) for v in center])
        mo = (ctypes.c_double * 6)(*([0.0] * 6 if motion is None else [float(v) for v in motion]))
        it = ctypes.c_int()
        rr = ctypes.c_double()
        _check(_lib.ggem_rigid_solve(self._h, *m, c, _dev_ptr(uinf, "uinf", m[0]),
                                     _dev_ptr(f, "f", m[0]), mo, float(tol), int(max_iter),
                                     ctypes.byref(it), ctypes.byref(rr)))
        return list(mo[:3]), list(mo[3:]), it.value, rr.value


def undisturbed_traction(plan, kind, rate, x, nrm, out=None):
    """sigma_inf . n of simple shear (FLOW_SHEAR) or Poiseuille flow
    (FLOW_POISEUILLE) at the points x (ggem_undisturbed_traction)."""
    import torch
    out = torch.empty_like(x) if out is None else out
    n = x.shape[0]
    _check(_lib.ggem_undisturbed_traction(plan._h, int(kind), float(rate), n, _dev_ptr(x, "x"),
                                          _dev_ptr(nrm, "nrm", n), _dev_ptr(out, "out", n)))
    return out


def poiseuille(plan, U0, x, out=None):
    """Undisturbed pressure-driven flow at the points x (ggem_poiseuille)."""
    import torch
    out = torch.empty_like(x) if out is None else out
    _check(_lib.ggem_poiseuille(plan._h, float(U0), x.shape[0], _dev_ptr(x, "x"),
                                _dev_ptr(out, "out", x.shape[0])))
    return out
