"""Parity metrics shared by the GPU tests (GPU path vs FP64 oracle).

Tendency: per variable v, max-norm error divided by
max(||R_ref_v||, 1e-3 N_v), N_v = the natural tendency scale (|rho| c/h for
mass, |rho| c^2/h for momentum, |Y_v| c/h for energy and water).  Two
independent FP64 evaluations of a tendency built from fluxes of size ~N_v h
cannot agree better than about eps ||D|| N_v ~ 2e-15 N_v (pressure alone is
1e5 Pa); so a 1e-11 relative target is meaningful only where ||R_ref_v|| is
above ~1e-3 N_v.  Below that (a variable at or near rest) the bound becomes
1e-11 * 1e-3 N_v, still tighter than an absolute 1e-11 N_v.
State: per variable, max-norm error relative to max(||Y_ref_v||, 1e-3 S_v),
S_v = |rho| c for the momenta (which start at or near rest) and ||Y_ref_v||
for the others.
"""
import numpy as np

C_SOUND = 350.0


def natural_scales(Y, h):
    rho_c = np.abs(Y[0]).max() * C_SOUND
    nat = [rho_c / h] + [rho_c * C_SOUND / h] * 3 + [np.abs(Y[4]).max() * C_SOUND / h]
    if Y.shape[0] > 5:
        nat.append(np.abs(Y[5]).max() * C_SOUND / h)
    return np.array(nat)


def rhs_errors(Rg, Rref, Y, h):
    nat = natural_scales(Y, h)
    out = []
    for v in range(Y.shape[0]):
        ref = np.abs(Rref[v]).max()
        scale = max(ref, 1e-3 * nat[v])
        out.append(np.abs(Rg[v] - Rref[v]).max() / scale)
    return np.array(out)


def literal_rhs_errors(Rg, Rref):
    """The plain relative max-norm error per variable,
    ||R_gpu - R_ref||_inf / ||R_ref||_inf, without the floor of rhs_errors
    (printed next to it; where ||R_ref|| is small against the natural scale
    it is dominated by the rounding of the fluxes, not by the method)."""
    return np.array([np.abs(Rg[v] - Rref[v]).max() / max(np.abs(Rref[v]).max(), 1e-300)
                     for v in range(Rref.shape[0])])


def state_errors(Yg, Yref):
    out = []
    rho_c = np.abs(Yref[0]).max() * C_SOUND
    for v in range(Yg.shape[0]):
        ref = np.abs(Yref[v]).max()
        floor = 1e-3 * rho_c if 1 <= v <= 3 else 0.0
        out.append(np.abs(Yg[v] - Yref[v]).max() / max(ref, floor))
    return np.array(out)


def hmin(grid):
    return float(min((np.array(grid["hi"], float) - np.array(grid["lo"], float)) / np.array(grid["ne"], float)))


def rounding_floor(rhs, Y, h, draws=2, seed=1):
    """How far the oracle's own tendency moves, in the rhs_errors metric,
    when every input word is perturbed by at most one unit in the last place
    (random sign, a third left unchanged).  Two FP64 implementations that
    differ only in rounding cannot be expected to agree much closer than
    this; where it exceeds the 1e-11 target (moist states, whose pressure
    and temperature come out of the saturation adjustment), the tolerance is
    a small multiple of it."""
    R0 = rhs(Y)
    rng = np.random.default_rng(seed)
    fl = np.zeros(Y.shape[0])
    for _ in range(draws):
        Yp = Y * (1.0 + 2.2e-16 * rng.choice([-1.0, 0.0, 1.0], size=Y.shape))
        fl = np.maximum(fl, rhs_errors(rhs(Yp), R0, Y, h))
    return R0, fl


def contraction_floor(grid, model, Yref, Y, R0, h):
    """How far the same oracle sources, compiled with fused multiply-adds
    allowed, land from the plain build's tendency R0 (rhs_errors norm): the
    distance between two correct FP64 evaluations of the operator that
    differ only in rounding (the GPU contracts to FMA as well)."""
    import oracle

    R1 = oracle.Model(oracle.Grid(grid, contract=True), model, Yref).rhs(Y)
    return rhs_errors(R1, R0, Y, h)
