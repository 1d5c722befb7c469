"""Thin ctypes binding of libcm.so (include/cm.h): argument marshalling only.

Every computation runs in the HIP kernels of the library; torch supplies
device memory (tensors) and streams.  There is no CPU fallback: if the
library is missing, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# CM_LIB may point at another build of the same library (e.g. a variant being timed)
LIB_PATH = os.environ.get("CM_LIB", os.path.join(HERE, "libcm.so"))

CM_OK, CM_ERR_ARG, CM_ERR_HIP, CM_ERR_ALLOC, CM_ERR_UNSUPPORTED, CM_ERR_NONFINITE, CM_ERR_STATE = range(7)
CM_FP64, CM_FP32_BULK = 0, 1
CLOSURES = {"none": 0, "const": 1, "smag": 2, "mlp": 3, "vreman": 4}
FLUXES = {"rusanov": 0, "roe": 1, "hllc": 2}

EXPORTED = [
    "cm_grid_create", "cm_grid_destroy", "cm_grid_query", "cm_grid_copy_coords", "cm_grid_copy_wJ",
    "cm_grid_copy_metrics", "cm_model_create", "cm_model_destroy", "cm_model_set_mlp",
    "cm_model_mlp_fallbacks", "cm_dg_rhs", "cm_lsrk_step", "cm_lsrk144_step", "cm_exp_filter", "cm_diagnostics",
    "cm_hevi_workspace_bytes", "cm_hevi_step", "cm_hevi_operator", "cm_hevi_solve",
    "cm_diagnostics_noalloc", "cm_state_import", "cm_state_export",
    "cm_mlp_create",
    "cm_mlp_destroy", "cm_mlp_train_step", "cm_mlp_grads", "cm_mlp_infer", "cm_mlp_get_params",
    "cm_mlp_set_params", "cm_model_profile", "cm_model_profile_read", "cm_model_closure_inputs",
    "cm_last_error",
]


class CMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("cm status %d: %s" % (status, msg))
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("ne", C.c_int * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("periodic", C.c_int * 3), ("topo", C.c_int), ("topo_h", C.c_double),
                ("topo_a", C.c_double), ("topo_xc", C.c_double)]


class GridInfo(C.Structure):
    _fields_ = [("n_elem", C.c_int64), ("n_nodes", C.c_int64), ("N", C.c_int), ("warped", C.c_int),
                ("dmin_node", C.c_double), ("state_stride", C.c_int64)]


class ModelDesc(C.Structure):
    _fields_ = [("nvar", C.c_int), ("precision", C.c_int), ("closure", C.c_int), ("nu", C.c_double),
                ("Cs", C.c_double), ("Prt", C.c_double), ("richardson", C.c_int), ("g", C.c_double),
                ("f_cor", C.c_double), ("u_g", C.c_double), ("v_g", C.c_double), ("sponge", C.c_int),
                ("sp_zs", C.c_double), ("sp_ztop", C.c_double), ("sp_alpha", C.c_double),
                ("sp_gamma", C.c_double), ("sp_u", C.c_double * 3), ("sfc_flux", C.c_int),
                ("theta_flux", C.c_double), ("qt_flux", C.c_double), ("subsidence", C.c_int),
                ("sub_w0", C.c_double), ("sub_ztop", C.c_double), ("flux", C.c_int), ("ice", C.c_int)]


class Diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("energy", C.c_double), ("water", C.c_double), ("ke", C.c_double),
                ("max_abs_w", C.c_double), ("max_cfl", C.c_double), ("T_min", C.c_double),
                ("T_max", C.c_double), ("n_nonfinite", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MLPDesc(C.Structure):
    _fields_ = [("n_in", C.c_int), ("n_hidden", C.c_int), ("n_layers_hidden", C.c_int), ("n_out", C.c_int),
                ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


_lib = None
_VP = C.c_void_p


def load():
    """Load libcm.so (built in-tree by ``paper_2110_00853_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcm.so is not built (run __graft_entry__.build() or python -m "
                           "paper_2110_00853_amd.build); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    L.cm_last_error.restype = C.c_char_p
    L.cm_grid_create.argtypes = [C.POINTER(GridDesc), C.c_int, C.POINTER(_VP)]
    L.cm_grid_destroy.argtypes = [_VP]
    L.cm_grid_query.argtypes = [_VP, C.POINTER(GridInfo)]
    L.cm_grid_copy_coords.argtypes = [_VP, _VP]
    L.cm_grid_copy_wJ.argtypes = [_VP, _VP]
    L.cm_grid_copy_metrics.argtypes = [_VP, _VP, _VP]
    L.cm_model_create.argtypes = [_VP, C.POINTER(ModelDesc), _VP, C.POINTER(_VP)]
    L.cm_model_destroy.argtypes = [_VP]
    L.cm_model_set_mlp.argtypes = [_VP, _VP, _VP]
    L.cm_model_mlp_fallbacks.argtypes = [_VP, C.POINTER(C.c_int64), _VP]
    L.cm_dg_rhs.argtypes = [_VP, _VP, _VP, C.c_double, _VP]
    L.cm_lsrk_step.argtypes = [_VP, _VP, _VP, _VP, C.c_double, C.c_double, _VP]
    L.cm_lsrk144_step.argtypes = [_VP, _VP, _VP, _VP, C.c_double, C.c_double, _VP]
    L.cm_exp_filter.argtypes = [_VP, _VP, C.c_int, C.c_int, C.c_double, C.c_int, _VP]
    L.cm_state_import.argtypes = [_VP, _VP, _VP, _VP]
    L.cm_state_export.argtypes = [_VP, _VP, _VP, _VP]
    L.cm_hevi_workspace_bytes.argtypes = [_VP, C.POINTER(C.c_size_t)]
    L.cm_hevi_step.argtypes = [_VP, _VP, _VP, C.c_double, C.c_double, _VP]
    L.cm_hevi_operator.argtypes = [_VP, _VP, _VP, _VP]
    L.cm_hevi_solve.argtypes = [_VP, C.c_double, _VP, _VP, _VP, _VP]
    L.cm_diagnostics.argtypes = [_VP, _VP, C.c_double, C.POINTER(Diag), _VP]
    L.cm_diagnostics_noalloc.argtypes = [_VP, _VP, C.c_double, C.POINTER(Diag), _VP]
    L.cm_mlp_create.argtypes = [C.POINTER(MLPDesc), C.c_uint64, C.c_int, C.POINTER(_VP)]
    L.cm_mlp_destroy.argtypes = [_VP]
    L.cm_mlp_train_step.argtypes = [_VP, _VP, _VP, C.c_int, C.POINTER(C.c_float), _VP]
    L.cm_mlp_grads.argtypes = [_VP, _VP, _VP, C.c_int, _VP, _VP]
    L.cm_mlp_infer.argtypes = [_VP, _VP, _VP, C.c_int, _VP]
    L.cm_mlp_get_params.argtypes = [_VP, _VP]
    L.cm_mlp_set_params.argtypes = [_VP, _VP]
    L.cm_model_profile.argtypes = [_VP, C.c_int]
    L.cm_model_closure_inputs.argtypes = [_VP, _VP, _VP, _VP]
    L.cm_model_profile_read.argtypes = [_VP, _VP, _VP]
    for name in EXPORTED:
        if name != "cm_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status: int, allow=()):
    if status != CM_OK and status not in allow:
        raise CMError(status, load().cm_last_error().decode())
    return status


def _stream_ptr(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(_VP)


class Grid:
    """Hexahedral brick mesh with GLL nodes and metric terms (cm_grid_create)."""

    def __init__(self, desc: dict, device: int = 0):
        d = GridDesc()
        d.N = int(desc.get("N", 4))
        for a in range(3):
            d.ne[a] = int(desc["ne"][a])
            d.lo[a] = float(desc["lo"][a])
            d.hi[a] = float(desc["hi"][a])
            d.periodic[a] = int(bool(desc["periodic"][a]))
        d.topo = int(desc.get("topo", 0))
        d.topo_h = float(desc.get("topo_h", 0.0))
        d.topo_a = float(desc.get("topo_a", 1.0))
        d.topo_xc = float(desc.get("topo_xc", 0.0))
        self.desc = dict(desc)
        self.device = device
        h = _VP()
        _check(load().cm_grid_create(C.byref(d), device, C.byref(h)))
        self.h = h
        info = GridInfo()
        _check(load().cm_grid_query(self.h, C.byref(info)))
        self.n_elem, self.n_nodes, self.dmin = info.n_elem, info.n_nodes, info.dmin_node
        # state buffers: [nvar][state_stride], element runs of srun slots
        # (the element's 125 nodes, then padding)
        self.state_stride = info.state_stride
        self.srun = info.state_stride // info.n_elem

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.cm_grid_destroy(self.h)
            self.h = None

    def coords(self) -> np.ndarray:
        out = np.zeros((3, self.n_nodes))
        _check(load().cm_grid_copy_coords(self.h, _np_ptr(out)))
        return out

    def wJ(self) -> np.ndarray:
        out = np.zeros(self.n_nodes)
        _check(load().cm_grid_copy_wJ(self.h, _np_ptr(out)))
        return out

    def metrics(self):
        Ja = np.zeros((3, 3, self.n_nodes))
        J = np.zeros(self.n_nodes)
        _check(load().cm_grid_copy_metrics(self.h, _np_ptr(Ja), _np_ptr(J)))
        return Ja, J


def model_desc(m: dict, precision: str = "fp64") -> ModelDesc:
    d = ModelDesc()
    d.nvar = int(m.get("nvar", 5))
    d.precision = CM_FP64 if precision == "fp64" else CM_FP32_BULK
    d.closure = CLOSURES[m.get("closure", "none")]
    d.nu = float(m.get("nu", 0.0))
    d.Cs = float(m.get("Cs", 0.21))
    d.Prt = float(m.get("Prt", 1.0 / 3.0))
    d.richardson = int(bool(m.get("richardson", False)))
    d.g = float(m.get("g", 9.81))
    d.f_cor = float(m.get("f_cor", 0.0))
    d.u_g = float(m.get("u_g", 0.0))
    d.v_g = float(m.get("v_g", 0.0))
    sp = m.get("sponge")
    if sp:
        d.sponge = 1
        d.sp_zs, d.sp_ztop = float(sp["z_s"]), float(sp["z_top"])
        d.sp_alpha, d.sp_gamma = float(sp["alpha"]), float(sp["gamma"])
        for c in range(3):
            d.sp_u[c] = float(sp["u_relax"][c])
    sf = m.get("sfc_flux")
    if sf:
        d.sfc_flux = 1
        d.theta_flux, d.qt_flux = float(sf["theta_flux"]), float(sf["qt_flux"])
    sb = m.get("subsidence")
    if sb:
        d.subsidence = 1
        d.sub_w0, d.sub_ztop = float(sb["w0"]), float(sb["z_top"])
    d.flux = FLUXES[m.get("flux", "rusanov")]
    d.ice = int(bool(m.get("ice", False)))
    return d


class Model:
    """Model physics on a grid (cm_model_create) with the hot-path calls."""

    def __init__(self, grid: Grid, desc: dict, Yref: np.ndarray | None = None, precision: str = "fp64"):
        self.grid = grid
        self.nvar = int(desc.get("nvar", 5))
        self.precision = precision
        self._d = model_desc(desc, precision)
        yref = None
        if Yref is not None:
            yref = np.ascontiguousarray(Yref, dtype=np.float64)
            if yref.shape != (self.nvar, grid.n_nodes):
                raise ValueError("Yref must have shape [nvar, n_nodes]")
        h = _VP()
        _check(load().cm_model_create(grid.h, C.byref(self._d), _np_ptr(yref) if yref is not None else None,
                                      C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.cm_model_destroy(self.h)
            self.h = None

    @property
    def dtype(self):
        import torch

        return torch.float64 if self.precision == "fp64" else torch.float32

    def _chk(self, *ts):
        for t in ts:
            if not t.is_cuda:
                raise ValueError("state tensors must live on the GPU")
            if t.dtype != self.dtype or tuple(t.shape) != (self.nvar, self.grid.state_stride) or not t.is_contiguous():
                raise ValueError("state tensor must be contiguous %s of shape (%d, %d)"
                                 % (self.dtype, self.nvar, self.grid.state_stride))

    def new_state(self, Y: np.ndarray | None = None):
        """A device state buffer [nvar, state_stride] in the model's storage
        (FP32-bulk: deviations from the background); the model's storage of
        the node-ordered full state Y [nvar, n_nodes] if given (through
        cm_state_import), else zeros."""
        import torch

        g = self.grid
        dev = "cuda:%d" % g.device
        S = torch.zeros((self.nvar, g.state_stride), dtype=self.dtype, device=dev)
        if Y is None:
            return S
        Y = np.asarray(Y)
        if Y.shape != (self.nvar, g.n_nodes):
            raise ValueError("state must have shape [nvar, n_nodes] = (%d, %d)" % (self.nvar, g.n_nodes))
        P = np.zeros((self.nvar, g.n_elem, g.srun), dtype=np.float64)
        P[:, :, :125] = Y.reshape(self.nvar, g.n_elem, 125)
        Yd = torch.from_numpy(P.reshape(self.nvar, g.state_stride)).to(device=dev)
        _check(load().cm_state_import(self.h, Yd.data_ptr(), S.data_ptr(), _stream_ptr(None)))
        torch.cuda.current_stream().synchronize()
        return S

    def to_numpy(self, T) -> np.ndarray:
        """Node-ordered host copy [nvar, n_nodes] of the full state a device
        state buffer holds (through cm_state_export; padding slots dropped),
        in float64."""
        import torch

        g = self.grid
        self._chk(T)
        Yd = torch.empty((self.nvar, g.state_stride), dtype=torch.float64, device=T.device)
        _check(load().cm_state_export(self.h, T.data_ptr(), Yd.data_ptr(), _stream_ptr(None)))
        A = Yd.cpu().numpy().reshape(self.nvar, g.n_elem, g.srun)[:, :, :125]
        A = np.ascontiguousarray(A).reshape(self.nvar, g.n_nodes)
        return A

    def tendency_to_numpy(self, T) -> np.ndarray:
        """Node-ordered host copy [nvar, n_nodes] of a tendency buffer (dQ,
        dY/dt: full values in both precisions), in the buffer's precision."""
        g = self.grid
        self._chk(T)
        A = T.cpu().numpy().reshape(self.nvar, g.n_elem, g.srun)[:, :, :125]
        return np.ascontiguousarray(A).reshape(self.nvar, g.n_nodes)

    def rhs(self, Y, out, t: float = 0.0, stream=None):
        self._chk(Y, out)
        _check(load().cm_dg_rhs(self.h, Y.data_ptr(), out.data_ptr(), float(t), _stream_ptr(stream)))
        return out

    def lsrk_step(self, Y, Y_alt, dQ, t: float, dt: float, stream=None):
        """One LSRK54 step; the new state is in Y_alt on return."""
        self._chk(Y, Y_alt, dQ)
        _check(load().cm_lsrk_step(self.h, Y.data_ptr(), Y_alt.data_ptr(), dQ.data_ptr(), float(t), float(dt),
                                   _stream_ptr(stream)))
        return Y_alt

    def lsrk144_step(self, Y, Y_alt, dQ, t: float, dt: float, stream=None):
        """One LSRK144 step; the new state is in Y on return (Y_alt is scratch)."""
        self._chk(Y, Y_alt, dQ)
        _check(load().cm_lsrk144_step(self.h, Y.data_ptr(), Y_alt.data_ptr(), dQ.data_ptr(), float(t),
                                      float(dt), _stream_ptr(stream)))
        return Y

    def hevi_workspace(self):
        """A device workspace for the 1-D IMEX calls (uint8 tensor)."""
        import torch

        n = C.c_size_t()
        _check(load().cm_hevi_workspace_bytes(self.h, C.byref(n)))
        return torch.empty(int(n.value), dtype=torch.uint8, device="cuda:%d" % self.grid.device)

    def hevi_step(self, Y, work, t: float, dt: float, stream=None):
        """One 1-D IMEX (HEVI, ARK2) step; Y is advanced in place."""
        self._chk(Y)
        _check(load().cm_hevi_step(self.h, Y.data_ptr(), work.data_ptr(), float(t), float(dt), _stream_ptr(stream)))
        return Y

    def hevi_operator(self, Y, out, stream=None):
        self._chk(Y, out)
        _check(load().cm_hevi_operator(self.h, Y.data_ptr(), out.data_ptr(), _stream_ptr(stream)))
        return out

    def hevi_solve(self, tau: float, B, Y, work, stream=None):
        self._chk(B, Y)
        _check(load().cm_hevi_solve(self.h, float(tau), B.data_ptr(), Y.data_ptr(), work.data_ptr(),
                                    _stream_ptr(stream)))
        return Y

    def exp_filter(self, Y, mask: int, order: int = 64, alpha: float = 36.0, Nc: int = 0, stream=None):
        """Exponential modal filter in place on the variables in mask (bit v)."""
        self._chk(Y)
        _check(load().cm_exp_filter(self.h, Y.data_ptr(), int(mask), int(order), float(alpha), int(Nc),
                                    _stream_ptr(stream)))
        return Y

    def diagnostics(self, Y, dt: float = 0.0, stream=None, noalloc: bool = False) -> dict:
        """cm_diagnostics, or cm_diagnostics_noalloc (static workspace) with noalloc=True."""
        self._chk(Y)
        out = Diag()
        fn = load().cm_diagnostics_noalloc if noalloc else load().cm_diagnostics
        st = fn(self.h, Y.data_ptr(), float(dt), C.byref(out), _stream_ptr(stream))
        _check(st, allow=(CM_ERR_NONFINITE,))
        d = out.as_dict()
        d["status"] = st
        return d

    def set_mlp(self, params: np.ndarray, norm: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        nrm = np.ascontiguousarray(norm, dtype=np.float32)
        if p.size != 9282 or nrm.size != 48:
            raise ValueError("need 9282 parameters and 48 normalisation values")
        _check(load().cm_model_set_mlp(self.h, _np_ptr(p), _np_ptr(nrm)))

    def closure_inputs(self, Y, out=None, stream=None):
        """Raw closure inputs per node [n_nodes, 16] (see cm_model_closure_inputs)."""
        import torch

        self._chk(Y)
        if out is None:
            out = torch.empty((self.grid.n_nodes, 16), dtype=torch.float64, device=Y.device)
        _check(load().cm_model_closure_inputs(self.h, Y.data_ptr(), out.data_ptr(), _stream_ptr(stream)))
        return out

    def profile(self, enable: bool = True):
        """Bracket every kernel launch with hipEvents (see cm_model_profile)."""
        _check(load().cm_model_profile(self.h, int(enable)))

    def profile_read(self):
        """Summed kernel durations [ms] and launch counts: {'grad': (ms, n), 'tend': (ms, n)}."""
        ms = np.zeros(2)
        cnt = np.zeros(2, dtype=np.int64)
        _check(load().cm_model_profile_read(self.h, _np_ptr(ms), _np_ptr(cnt)))
        return {"grad": (float(ms[0]), int(cnt[0])), "tend": (float(ms[1]), int(cnt[1]))}

    def mlp_fallbacks(self, stream=None) -> int:
        c = C.c_int64()
        _check(load().cm_model_mlp_fallbacks(self.h, C.byref(c), _stream_ptr(stream)))
        return c.value


class MLP:
    """Learned-closure network (cm_mlp_*): 12-64-64-64-2 SiLU, BF16 MFMA
    forward/backward with FP32 accumulation, FP32 master weights, Adam."""

    NPARAM = 9282

    def __init__(self, seed: int = 0, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, device: int = 0):
        d = MLPDesc()
        d.n_in, d.n_hidden, d.n_layers_hidden, d.n_out = 12, 64, 3, 2
        d.lr, d.beta1, d.beta2, d.eps = lr, beta1, beta2, eps
        h = _VP()
        _check(load().cm_mlp_create(C.byref(d), int(seed), device, C.byref(h)))
        self.h = h
        self.device = device

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.cm_mlp_destroy(self.h)
            self.h = None

    @staticmethod
    def _chk(t, cols):
        if not t.is_cuda or t.dtype.itemsize != 4 or t.dim() != 2 or t.shape[1] != cols or not t.is_contiguous():
            raise ValueError("expected a contiguous float32 CUDA tensor [batch, %d]" % cols)

    def params(self) -> np.ndarray:
        out = np.zeros(self.NPARAM, dtype=np.float32)
        _check(load().cm_mlp_get_params(self.h, _np_ptr(out)))
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.NPARAM:
            raise ValueError("need 9282 parameters")
        _check(load().cm_mlp_set_params(self.h, _np_ptr(p)))

    def infer(self, X, out=None, stream=None):
        import torch

        self._chk(X, 12)
        if out is None:
            out = torch.empty((X.shape[0], 2), dtype=torch.float32, device=X.device)
        self._chk(out, 2)
        _check(load().cm_mlp_infer(self.h, X.data_ptr(), out.data_ptr(), X.shape[0], _stream_ptr(stream)))
        return out

    def grads(self, X, T, stream=None) -> np.ndarray:
        self._chk(X, 12)
        self._chk(T, 2)
        g = np.zeros(self.NPARAM, dtype=np.float32)
        _check(load().cm_mlp_grads(self.h, X.data_ptr(), T.data_ptr(), X.shape[0], _np_ptr(g), _stream_ptr(stream)))
        return g

    def train_step(self, X, T, want_loss: bool = True, stream=None):
        self._chk(X, 12)
        self._chk(T, 2)
        loss = C.c_float(0.0)
        _check(load().cm_mlp_train_step(self.h, X.data_ptr(), T.data_ptr(), X.shape[0],
                                         C.byref(loss) if want_loss else None, _stream_ptr(stream)))
        return float(loss.value) if want_loss else None
