"""FP64 CPU oracle for the DG LES right-hand side and LSRK54 step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_2110_00853_amd``) and never imports it; both are
fed the same seeded inputs by ``paper_2110_00853_amd.workloads``.

The C sources (``cmref.c``, ``cmref_mlp.c``) are compiled with gcc, ``-O2
-ffp-contract=off`` and no fast-math, into ``liboracle.so`` next to them.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_FMA_PATH = os.path.join(_HERE, "liboracle_fma.so")
_SOURCES = ["cmref.c", "cmref_mlp.c"]
_lib = None
_lib_fma = None


def build(force: bool = True, contract: bool = False) -> str:
    """Compile the oracle shared library (gcc, OpenMP, no FMA contraction).
    contract=True builds the same sources with fused multiply-adds allowed
    (``-ffp-contract=fast -mfma``) into ``liboracle_fma.so``: a second
    correct FP64 evaluation of the same operator that differs only in
    rounding, whose distance from the plain build measures how closely two
    such implementations can agree."""
    path = _FMA_PATH if contract else _LIB_PATH
    if not force and os.path.exists(path):
        return path
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = path + ".tmp%d" % os.getpid()
    fp = ["-ffp-contract=fast", "-mfma"] if contract else ["-ffp-contract=off"]
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp"] + fp + [
        "-fno-fast-math", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, path)
    return path


class GridDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("ne", C.c_int * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("periodic", C.c_int * 3), ("topo", C.c_int),
                ("topo_h", C.c_double), ("topo_a", C.c_double), ("topo_xc", C.c_double)]


class ModelDesc(C.Structure):
    _fields_ = [("nvar", C.c_int), ("closure", C.c_int), ("nu", C.c_double),
                ("Cs", C.c_double), ("Prt", C.c_double), ("richardson", C.c_int),
                ("g", C.c_double), ("f_cor", C.c_double), ("u_g", C.c_double),
                ("v_g", C.c_double), ("sponge", C.c_int), ("sp_zs", C.c_double),
                ("sp_ztop", C.c_double), ("sp_alpha", C.c_double), ("sp_gamma", C.c_double),
                ("sp_u", C.c_double * 3), ("sfc_flux", C.c_int), ("theta_flux", C.c_double),
                ("qt_flux", C.c_double), ("subsidence", C.c_int), ("sub_w0", C.c_double),
                ("sub_ztop", C.c_double), ("flux", C.c_int), ("ice", C.c_int)]


FLUXES = {"rusanov": 0, "roe": 1, "hllc": 2}

_P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib(contract: bool = False):
    """The oracle library; contract=True the FMA-contracted build of the
    same sources (see build)."""
    global _lib, _lib_fma
    if contract:
        if _lib_fma is None:
            if not os.path.exists(_FMA_PATH):
                build(contract=True)
            _lib_fma = _declare(C.CDLL(_FMA_PATH))
        return _lib_fma
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _declare(C.CDLL(_LIB_PATH))
    return _lib


def _declare(L):
    """Argument and result types of the library's exports."""
    L.cmref_gll.argtypes = [C.c_int, _P, _P, _P]
    L.cmref_grid_create.argtypes = [C.POINTER(GridDesc), C.c_int]
    L.cmref_grid_create.restype = C.c_void_p
    L.cmref_grid_destroy.argtypes = [C.c_void_p]
    L.cmref_grid_nnodes.argtypes = [C.c_void_p]
    L.cmref_grid_nnodes.restype = C.c_long
    L.cmref_grid_coords.argtypes = [C.c_void_p, _P]
    L.cmref_grid_metrics.argtypes = [C.c_void_p, _P, _P]
    L.cmref_grid_wJ.argtypes = [C.c_void_p, _P]
    L.cmref_grid_metric_identity.argtypes = [C.c_void_p, _P]
    L.cmref_pvsat.argtypes = [C.c_double]
    L.cmref_pvsat.restype = C.c_double
    L.cmref_saturation_adjust.argtypes = [C.c_double, C.c_double, C.c_double,
                                          C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.cmref_thermo_nodes.argtypes = [C.c_int, C.c_int, C.c_long, _P, _P, C.c_double, _P, _P, _P, _P]
    L.cmref_pvsat_ice.argtypes = [C.c_double]
    L.cmref_pvsat_ice.restype = C.c_double
    L.cmref_liquid_fraction.argtypes = [C.c_double]
    L.cmref_liquid_fraction.restype = C.c_double
    L.cmref_saturation_adjust_phase.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.POINTER(C.c_double),
                                                C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.cmref_numflux_point.argtypes = [C.c_int, C.c_int, _P, _P, C.c_double, C.c_double, C.c_double, _P, _P]
    L.cmref_ark2_coeffs.argtypes = [_P, _P, _P]
    L.cmref_hevi_steps.argtypes = [C.c_void_p, _P, C.c_double, C.c_double, C.c_int]
    L.cmref_hevi_steps.restype = C.c_int
    L.cmref_hevi_operator.argtypes = [C.c_void_p, _P, _P]
    L.cmref_hevi_solve.argtypes = [C.c_void_p, C.c_double, _P, _P]
    L.cmref_hevi_solve_lines.argtypes = [C.c_void_p, C.c_double, _P, _P,
                                         np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS"), C.c_int]
    L.cmref_exp_filter.argtypes = [C.c_void_p, _P, C.c_int, C.c_int, C.c_double, C.c_int]
    L.cmref_rusanov_point.argtypes = [C.c_int, _P, _P, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, _P, _P]
    L.cmref_smagorinsky_point.argtypes = [_P, C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.c_int, C.POINTER(C.c_double)]
    L.cmref_vreman_point.argtypes = [_P, C.c_double, C.c_double, _P, C.c_double, C.c_int,
                                     C.POINTER(C.c_double)]
    L.cmref_model_create.argtypes = [C.c_void_p, C.POINTER(ModelDesc), C.c_void_p]
    L.cmref_model_create.restype = C.c_void_p
    L.cmref_model_destroy.argtypes = [C.c_void_p]
    L.cmref_model_reference.argtypes = [C.c_void_p, _P, _P]
    L.cmref_model_set_mlp.argtypes = [C.c_void_p, _P, C.c_int, _P, _P, C.c_int, C.c_int]
    L.cmref_mlp_nparams.restype = C.c_int
    L.cmref_mlp_forward.argtypes = [_P, _P, C.c_int, _P]
    L.cmref_mlp_forward_bf16.argtypes = [_P, _P, C.c_int, _P]
    L.cmref_mlp_grad.argtypes = [_P, _P, _P, C.c_int, _P]
    L.cmref_mlp_grad.restype = C.c_double
    L.cmref_mlp_grad_bf16.argtypes = [_P, _P, _P, C.c_int, _P, _P]
    L.cmref_mlp_grad_bf16.restype = C.c_double
    L.cmref_adam_step.argtypes = [_P, _P, _P, _P, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
    L.cmref_bf16.argtypes = [C.c_double]
    L.cmref_bf16.restype = C.c_double
    L.cmref_model_mlp_fallbacks.argtypes = [C.c_void_p]
    L.cmref_model_mlp_fallbacks.restype = C.c_long
    L.cmref_rhs.argtypes = [C.c_void_p, _P, _P, C.c_double]
    L.cmref_gradients.argtypes = [C.c_void_p, _P, _P, _P]
    L.cmref_gradients.restype = C.c_int
    L.cmref_lsrk54_coeffs.argtypes = [_P, _P, _P]
    L.cmref_lsrk_steps.argtypes = [C.c_void_p, _P, _P, C.c_double, C.c_double, C.c_int]
    L.cmref_lsrk144_coeffs.argtypes = [_P, _P, _P]
    L.cmref_lsrk144_steps.argtypes = [C.c_void_p, _P, _P, C.c_double, C.c_double, C.c_int]
    L.cmref_integrals.argtypes = [C.c_void_p, _P, _P]
    L.cmref_num_threads.restype = C.c_int
    L.cmref_set_num_threads.argtypes = [C.c_int]
    L.cmref_set_mutation.argtypes = [C.c_int]
    L.cmref_mlp_closure.argtypes = [_P, C.c_void_p, _P, _P, C.c_int, _P, C.c_double, C.c_double,
                                    C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.cmref_mlp_closure.restype = C.c_int
    return L


def gll(N: int):
    """GLL nodes, weights and differentiation matrix D[i, j] = l_j'(x_i)."""
    Q = N + 1
    xi = np.zeros(Q)
    w = np.zeros(Q)
    D = np.zeros(Q * Q)
    if lib().cmref_gll(N, xi, w, D):
        raise ValueError("unsupported N")
    return xi, w, D.reshape(Q, Q)


def _grid_desc(g: dict) -> GridDesc:
    d = GridDesc()
    d.N = int(g.get("N", 4))
    for a in range(3):
        d.ne[a] = int(g["ne"][a])
        d.lo[a] = float(g["lo"][a])
        d.hi[a] = float(g["hi"][a])
        d.periodic[a] = int(bool(g["periodic"][a]))
    d.topo = int(g.get("topo", 0))
    d.topo_h = float(g.get("topo_h", 0.0))
    d.topo_a = float(g.get("topo_a", 1.0))
    d.topo_xc = float(g.get("topo_xc", 0.0))
    return d


def _model_desc(m: dict) -> ModelDesc:
    d = ModelDesc()
    d.nvar = int(m.get("nvar", 5))
    d.closure = {"none": 0, "const": 1, "smag": 2, "mlp": 3, "vreman": 4}[m.get("closure", "none")]
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
        d.theta_flux = float(sf["theta_flux"])
        d.qt_flux = float(sf["qt_flux"])
    sb = m.get("subsidence")
    if sb:
        d.subsidence = 1
        d.sub_w0 = float(sb["w0"])
        d.sub_ztop = float(sb["z_top"])
    d.flux = FLUXES[m.get("flux", "rusanov")]
    d.ice = int(bool(m.get("ice", False)))
    return d


class Grid:
    def __init__(self, desc: dict, dense: bool = False, contract: bool = False):
        self._L = lib(contract)
        self._d = _grid_desc(desc)
        self.h = self._L.cmref_grid_create(C.byref(self._d), int(dense))
        if not self.h:
            raise RuntimeError("oracle grid creation failed")
        self.nnodes = self._L.cmref_grid_nnodes(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            self._L.cmref_grid_destroy(self.h)
            self.h = None

    def coords(self):
        out = np.zeros(3 * self.nnodes)
        self._L.cmref_grid_coords(self.h, out)
        return out.reshape(3, self.nnodes)

    def metrics(self):
        Ja = np.zeros(9 * self.nnodes)
        J = np.zeros(self.nnodes)
        self._L.cmref_grid_metrics(self.h, Ja, J)
        return Ja.reshape(3, 3, self.nnodes), J

    def wJ(self):
        out = np.zeros(self.nnodes)
        self._L.cmref_grid_wJ(self.h, out)
        return out

    def metric_identity(self):
        out = np.zeros(3 * self.nnodes)
        self._L.cmref_grid_metric_identity(self.h, out)
        return out.reshape(3, self.nnodes)


class Model:
    def __init__(self, grid: Grid, desc: dict, Yref: np.ndarray | None = None):
        self.grid = grid
        self._L = grid._L  # the grid's build of the oracle library
        self._d = _model_desc(desc)
        self.nvar = self._d.nvar
        yref = None
        if Yref is not None:
            yref = np.ascontiguousarray(Yref, dtype=np.float64)
            assert yref.shape == (self.nvar, grid.nnodes)
        self._yref = yref
        ptr = yref.ctypes.data_as(C.c_void_p) if yref is not None else None
        self.h = self._L.cmref_model_create(grid.h, C.byref(self._d), ptr)
        if not self.h:
            raise ValueError("oracle model creation failed (Roe and HLLC fluxes are for dry models only)")

    def __del__(self):
        if getattr(self, "h", None):
            self._L.cmref_model_destroy(self.h)
            self.h = None

    def _chk(self, Y):
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        assert Y.shape == (self.nvar, self.grid.nnodes)
        return Y

    def rhs(self, Y, t: float = 0.0):
        Y = self._chk(Y)
        R = np.zeros_like(Y)
        self._L.cmref_rhs(self.h, Y, R, float(t))
        return R

    def gradients(self, Y):
        Y = self._chk(Y)
        nn = self.grid.nnodes
        grad = np.zeros(8 * 3 * nn)
        F2 = np.zeros(self.nvar * 3 * nn)
        nG = self._L.cmref_gradients(self.h, Y, grad, F2)
        return grad[: nG * 3 * nn].reshape(nG, 3, nn), F2.reshape(self.nvar, 3, nn)

    def reference(self):
        nn = self.grid.nnodes
        pr = np.zeros(nn)
        rr = np.zeros(nn)
        self._L.cmref_model_reference(self.h, pr, rr)
        return pr, rr

    def steps(self, Y, dt: float, nsteps: int, t: float = 0.0, dQ=None, scheme: str = "lsrk54"):
        """Advance a copy of Y by nsteps steps of LSRK54 (or scheme="lsrk144");
        returns (Y, dQ)."""
        Y = self._chk(Y).copy()
        dQ = np.zeros_like(Y) if dQ is None else np.ascontiguousarray(dQ, dtype=np.float64).copy()
        fn = {"lsrk54": self._L.cmref_lsrk_steps, "lsrk144": self._L.cmref_lsrk144_steps}[scheme]
        fn(self.h, Y, dQ, float(t), float(dt), int(nsteps))
        return Y, dQ

    def hevi_steps(self, Y, dt: float, nsteps: int, t: float = 0.0):
        """Advance a copy of Y by nsteps ARK2 HEVI steps (dry, flat mesh)."""
        Y = self._chk(Y).copy()
        if self._L.cmref_hevi_steps(self.h, Y, float(t), float(dt), int(nsteps)):
            raise ValueError("the HEVI step is for dry models")
        return Y

    def hevi_operator(self, Y):
        """L (Y - Y_ref): the linear vertical operator (rho, rho w, rho e_tot rows)."""
        Y = self._chk(Y)
        out = np.zeros_like(Y)
        self._L.cmref_hevi_operator(self.h, Y, out)
        return out

    def hevi_solve(self, tau: float, B):
        """Y_ref + x with (I - tau L) x = B - Y_ref on every vertical line."""
        B = self._chk(B)
        out = np.zeros_like(B)
        self._L.cmref_hevi_solve(self.h, float(tau), B, out)
        return out

    def hevi_solve_lines(self, tau: float, B, lines):
        """hevi_solve on the listed vertical lines only (line = (ex + ne0 ey)
        25 + i + 5 j); the other lines of the result hold B."""
        B = self._chk(B)
        out = B.copy()
        ln = np.ascontiguousarray(np.asarray(lines, dtype=np.int64))
        n_lines = self.grid._d.ne[0] * self.grid._d.ne[1] * 25
        assert len(np.unique(ln)) == len(ln) and np.all((ln >= 0) & (ln < n_lines)), "bad line list"
        self._L.cmref_hevi_solve_lines(self.h, float(tau), B, out, ln, int(len(ln)))
        return out

    def exp_filter(self, Y, mask: int, order: int = 64, alpha: float = 36.0, Nc: int = 0):
        """A filtered copy of Y (exponential modal filter on the deviation of
        the variables in mask from the background)."""
        Y = self._chk(Y).copy()
        self._L.cmref_exp_filter(self.h, Y, int(mask), int(order), float(alpha), int(Nc))
        return Y

    def integrals(self, Y):
        """Domain integrals of each variable (w J weighted) and kinetic energy."""
        Y = self._chk(Y)
        out = np.zeros(self.nvar + 1)
        self._L.cmref_integrals(self.h, Y, out)
        return out

    def set_mlp(self, params: np.ndarray, mean: np.ndarray, std: np.ndarray, lo: np.ndarray,
                hi: np.ndarray, use_fallback=True, bf16=False):
        """Learned closure: network parameters, input mean/std and the
        standardised training range; bf16 emulates the GPU's operand rounding."""
        p = np.ascontiguousarray(np.concatenate([np.asarray(params, np.float64), np.asarray(mean, np.float64),
                                                 np.asarray(std, np.float64)]))
        self._L.cmref_model_set_mlp(self.h, p, p.size, np.ascontiguousarray(lo, dtype=np.float64),
                                  np.ascontiguousarray(hi, dtype=np.float64), int(use_fallback), int(bf16))
        self._mlp = p

    def mlp_fallbacks(self) -> int:
        return self._L.cmref_model_mlp_fallbacks(self.h)


def pvsat(T: float) -> float:
    return lib().cmref_pvsat(float(T))


def saturation_adjust(rho: float, qt: float, I: float):
    T = C.c_double()
    ql = C.c_double()
    lib().cmref_saturation_adjust(float(rho), float(qt), float(I), C.byref(T), C.byref(ql))
    return T.value, ql.value


def pvsat_ice(T: float) -> float:
    return lib().cmref_pvsat_ice(float(T))


def liquid_fraction(T: float) -> float:
    return lib().cmref_liquid_fraction(float(T))


def saturation_adjust_phase(rho: float, qt: float, I: float, ice: bool = True):
    """(T, q_l, q_i) of the equilibrium state, with or without the ice phase."""
    T, ql, qi = C.c_double(), C.c_double(), C.c_double()
    lib().cmref_saturation_adjust_phase(float(rho), float(qt), float(I), int(ice), C.byref(T), C.byref(ql),
                                        C.byref(qi))
    return T.value, ql.value, qi.value


def thermo_nodes(Y: np.ndarray, z: np.ndarray, g: float, ice: bool = False):
    """T, p, total condensate q_l + q_i, theta_v at every node of a state [nvar, n]."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    nvar, n = Y.shape
    z = np.ascontiguousarray(z, dtype=np.float64)
    T, p, ql, thv = (np.zeros(n) for _ in range(4))
    lib().cmref_thermo_nodes(nvar, int(ice), n, Y, z, float(g), T, p, ql, thv)
    return T, p, ql, thv


def rusanov(Ym, Yp, n, zm=0.0, zp=0.0, g=0.0, prm=0.0, prp=0.0):
    Ym = np.ascontiguousarray(Ym, dtype=np.float64)
    Yp = np.ascontiguousarray(Yp, dtype=np.float64)
    out = np.zeros(Ym.size)
    lib().cmref_rusanov_point(Ym.size, Ym, Yp, zm, zp, g, prm, prp,
                              np.ascontiguousarray(n, dtype=np.float64), out)
    return out


def numflux(kind, Ym, Yp, n, z=0.0, g=0.0, pr=0.0):
    """Numerical flux n.F1* ("rusanov", "roe", "hllc") between two states at
    a face node at height z with reference pressure pr."""
    Ym = np.ascontiguousarray(Ym, dtype=np.float64)
    out = np.zeros(Ym.size)
    lib().cmref_numflux_point(FLUXES[kind], Ym.size, Ym, np.ascontiguousarray(Yp, dtype=np.float64), float(z),
                              float(g), float(pr), np.ascontiguousarray(n, dtype=np.float64), out)
    return out


def smagorinsky(gu: np.ndarray, N2: float, Cs: float, Delta: float, Prt: float, richardson: bool):
    nu = C.c_double()
    lib().cmref_smagorinsky_point(np.ascontiguousarray(gu, dtype=np.float64).ravel(), N2, Cs,
                                  Delta, Prt, int(richardson), C.byref(nu))
    return nu.value


def vreman(gu, N2, Cs, Dm, Prt=1.0 / 3.0, richardson=False):
    """Vreman eddy viscosity at one node (eq. vreman-sgs); gu[i][j] = du_i/dx_j,
    Dm the mixing length per direction."""
    nu = C.c_double()
    lib().cmref_vreman_point(np.ascontiguousarray(gu, dtype=np.float64).ravel(), float(N2), float(Cs),
                             np.ascontiguousarray(Dm, dtype=np.float64), float(Prt), int(richardson), C.byref(nu))
    return nu.value


def lsrk54_coeffs():
    A, B, Cc = np.zeros(5), np.zeros(5), np.zeros(5)
    lib().cmref_lsrk54_coeffs(A, B, Cc)
    return A, B, Cc


NPARAM = 9282


def ark2_coeffs():
    """Explicit and implicit tableaus [3][3] and weights of the ARK2 IMEX scheme."""
    AE, AI, b = np.zeros(9), np.zeros(9), np.zeros(3)
    lib().cmref_ark2_coeffs(AE, AI, b)
    return AE.reshape(3, 3), AI.reshape(3, 3), b


def lsrk144_coeffs():
    """A, B, C of the 14-stage LSRK (Niegemann, Diehl & Busch 2012)."""
    A, B, Cc = np.zeros(14), np.zeros(14), np.zeros(14)
    lib().cmref_lsrk144_coeffs(A, B, Cc)
    return A, B, Cc


def mlp_forward(params, X, bf16=False):
    """Raw outputs [n, 2] of the 12-64-64-64-2 SiLU network for standardised
    inputs X [n, 12] (FP64, or with bfloat16 matrix operands)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    out = np.zeros((X.shape[0], 2))
    (lib().cmref_mlp_forward_bf16 if bf16 else lib().cmref_mlp_forward)(p, X.ravel(), X.shape[0], out.ravel())
    return out


def mlp_grad(params, X, T):
    """Mean squared error of the raw outputs and its gradient (FP64)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    g = np.zeros(NPARAM)
    loss = lib().cmref_mlp_grad(p, X.ravel(), T.ravel(), X.shape[0], g)
    return loss, g


def mlp_grad_bf16(params, X, T):
    """(loss, gradient, magnitude) with the GPU's rounding points: bfloat16
    matrix operands, FP32 sums, FP32 bias / SiLU / derivative arithmetic;
    magnitude[q] = sum of |terms| of gradient q."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    g = np.zeros(p.size)
    mag = np.zeros(p.size)
    loss = lib().cmref_mlp_grad_bf16(p, X.ravel(), T.ravel(), X.shape[0], g, mag)
    return loss, g, mag


def adam_step(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place on float64 arrays."""
    lib().cmref_adam_step(params, np.ascontiguousarray(grad, dtype=np.float64), m, v, int(step), lr, b1, b2, eps)


def mlp_closure(params, mean, std, lo, hi, gu, N2, Delta, nu_sl, use_fallback=True):
    """The learned closure at one node: (fell_back, nu_t, Pr_t) for the
    velocity gradient gu[3][3], N^2, filter width and Smagorinsky viscosity
    (FP64 network)."""
    p = np.ascontiguousarray(np.concatenate([np.asarray(params, np.float64), np.asarray(mean, np.float64),
                                             np.asarray(std, np.float64)]))
    nu, pr = C.c_double(), C.c_double()
    fb = lib().cmref_mlp_closure(p, None, np.ascontiguousarray(lo, dtype=np.float64),
                                 np.ascontiguousarray(hi, dtype=np.float64), int(use_fallback),
                                 np.ascontiguousarray(gu, dtype=np.float64).ravel(), float(N2), float(Delta),
                                 float(nu_sl), C.byref(nu), C.byref(pr))
    return bool(fb), nu.value, pr.value


def bf16(x: float) -> float:
    return lib().cmref_bf16(float(x))


def set_mutation(code: int) -> None:
    """Plant a known mistake in the operator (tests of the pins only; 0 = none)."""
    lib().cmref_set_mutation(int(code))


def num_threads() -> int:
    return lib().cmref_num_threads()


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's parallel loops from now on."""
    lib().cmref_set_num_threads(int(n))
