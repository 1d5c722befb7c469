"""Learned SGS closure: training data from a resolved run, training on the
GPU, and the a-posteriori comparison against Smagorinsky-Lilly.

Pipeline (all GPU work through the C ABI):
  1. run the bubble at 2x resolution (FP64) and take snapshots;
  2. coarse-grain each snapshot onto the 2x coarser mesh by the exact L2
     projection of each fine element polynomial onto its parent element
     (8 children -> 1 parent, tensor product of 1-D projections);
  3. SGS targets from the filtered fields: Favre stress tau = bar(rho u u) -
     bar(rho u) bar(rho u)/bar(rho), nu* = max(0, -tau_dev : S / (2 rho S:S)),
     heat flux q = bar(rho theta u) - bar(rho theta) bar(rho u)/bar(rho),
     D* = max(0, -q . grad theta / (rho |grad theta|^2)), Pr* = clip(nu*/D*,
     0.1, 10); inputs (velocity gradient, N^2, Delta, TKE estimate) exactly as
     the gradient pass computes them (cm_model_closure_inputs);
  4. train the network (cm_mlp_train_step, BF16 MFMA, Adam) on targets mapped
     into the raw-output space: o1 = softplus^-1(nu* / (Delta^2 |S|)),
     o2 = softplus^-1(Pr* - 0.1);
  5. run the coarse mesh with Smagorinsky and with the network from the
     filtered initial state and compare theta and w with the filtered
     resolved run at a later time.
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np

from . import binding as B
from . import workloads as W

_RD, _CVD, _T0, _P0 = 287.0, 717.5, 273.16, 1.0e5
_KAPPA = _RD / (_CVD + _RD)


# ---------------------------------------------------------------------------
# exact L2 projection of two child elements onto their parent (1-D)
# ---------------------------------------------------------------------------
def _lagrange(nodes, x):
    """Values of the Lagrange basis on `nodes` at points x: [len(x), len(nodes)]."""
    V = np.ones((x.size, nodes.size))
    for j in range(nodes.size):
        for m in range(nodes.size):
            if m != j:
                V[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return V


def projection_matrix(N: int = 4) -> np.ndarray:
    """P [N+1, 2(N+1)]: parent nodal values of the L2 projection of the
    piecewise polynomial given by the nodal values on the left child
    [-1, 0] (first N+1 columns) and the right child [0, 1]."""
    xi = W.gll_points(N)
    xg, wg = np.polynomial.legendre.leggauss(2 * N + 2)
    M = np.zeros((N + 1, N + 1))
    Bm = np.zeros((N + 1, 2 * (N + 1)))
    Lp = _lagrange(xi, xg)                                   # parent basis on [-1, 1]
    M = (Lp * wg[:, None]).T @ Lp
    for c, (a, b) in enumerate(((-1.0, 0.0), (0.0, 1.0))):
        xs = 0.5 * (b - a) * xg + 0.5 * (a + b)              # points in the child
        ws = 0.5 * (b - a) * wg
        Lpar = _lagrange(xi, xs)
        Lch = _lagrange(xi, 2.0 * (xs - a) / (b - a) - 1.0)  # child basis
        Bm[:, c * (N + 1):(c + 1) * (N + 1)] = (Lpar * ws[:, None]).T @ Lch
    return np.linalg.solve(M, Bm)


def coarse_grain(f: np.ndarray, ne_fine, P=None) -> np.ndarray:
    """Project a fine nodal field [n_fine] (element-major, i fastest) onto the
    2x coarser mesh; returns [n_coarse] in the same layout."""
    P = projection_matrix() if P is None else P
    fx, fy, fz = ne_fine
    cx, cy, cz = fx // 2, fy // 2, fz // 2
    a = f.reshape(cz, 2, cy, 2, cx, 2, 5, 5, 5)               # [cz oz cy oy cx ox k j i]
    a = a.transpose(0, 2, 4, 1, 6, 3, 7, 5, 8).reshape(cz, cy, cx, 10, 10, 10)  # (oz k)(oy j)(ox i)
    a = np.tensordot(a, P, axes=([5], [1]))                   # i
    a = np.tensordot(a, P, axes=([4], [1]))                   # j  -> [..., 10(k), 5(i), 5(j)]
    a = np.tensordot(a, P, axes=([3], [1]))                   # k  -> [cz cy cx i j k]
    return a.transpose(0, 1, 2, 5, 4, 3).reshape(-1)


def _theta(Y, z, g=9.81):
    rho = Y[0]
    e = Y[4] / rho
    ke = 0.5 * (Y[1] ** 2 + Y[2] ** 2 + Y[3] ** 2) / rho ** 2
    T = _T0 + (e - ke - g * z) / _CVD
    p = rho * _RD * T
    return T * (_P0 / p) ** _KAPPA


def filtered(Yf: np.ndarray, zf: np.ndarray, ne_fine, g=9.81):
    """Filtered state (projected conserved variables) and the products
    needed for the SGS targets, on the coarse mesh."""
    P = projection_matrix()
    cg = lambda a: coarse_grain(a, ne_fine, P)
    Yc = np.stack([cg(Yf[v]) for v in range(Yf.shape[0])])
    rho = Yf[0]
    u = Yf[1:4] / rho
    th = _theta(Yf, zf, g)
    ruu = np.stack([cg(Yf[1 + a] * u[b]) for a, b in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))])
    rth = cg(rho * th)
    rthu = np.stack([cg(rho * th * u[b]) for b in range(3)])
    return Yc, ruu, rth, rthu


def sgs_targets(Yc, ruu, rth, rthu, feat, Delta, nu_min_ratio=1e-4):
    """Targets in the raw-output space and a mask of usable nodes."""
    rho = Yc[0]
    m = Yc[1:4]
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    tau = np.zeros((3, 3, rho.size))
    for q, (a, b) in enumerate(pairs):
        tau[a, b] = ruu[q] - m[a] * m[b] / rho
        tau[b, a] = tau[a, b]
    tr = (tau[0, 0] + tau[1, 1] + tau[2, 2]) / 3.0
    for a in range(3):
        tau[a, a] -= tr
    gu = feat[:, :9].T.reshape(3, 3, -1)
    S = 0.5 * (gu + gu.transpose(1, 0, 2))
    SS = np.sum(S * S, axis=(0, 1))
    nu_s = np.maximum(0.0, -np.sum(tau * S, axis=(0, 1)) / (2.0 * rho * np.maximum(SS, 1e-30)))
    q = rthu - rth[None] * m / rho[None]
    gth = feat[:, 12:15].T
    gg = np.sum(gth * gth, axis=0)
    D_s = np.maximum(0.0, -np.sum(q * gth, axis=0) / (rho * np.maximum(gg, 1e-30)))
    Pr_s = np.clip(nu_s / np.maximum(D_s, 1e-30), 0.1, 10.0)
    Smag = np.sqrt(2.0 * SS)
    z1 = nu_s / (Delta * Delta * np.maximum(Smag, 1e-30))
    t1 = np.log(np.expm1(np.clip(z1, nu_min_ratio, 10.0)))
    t2 = np.log(np.expm1(np.clip(Pr_s - 0.1, 1e-3, 9.9)))
    mask = (Smag > 1e-3) & np.isfinite(t1) & np.isfinite(t2)
    return np.stack([t1, t2], axis=1), mask


def run_pipeline(fine_ne=64, t_train=(60.0, 90.0, 120.0, 150.0, 180.0), t_eval=240.0, train_steps=3000,
                 batch=8192, seed=0, out_json=None, out_npz=None, n_holdout=10000, log=print):
    """The whole pipeline at one resolution; returns a dict of results."""
    import torch

    t_start = time.time()
    coarse_ne = fine_ne // 2
    cf = W.case("bubble_32", ne=(fine_ne,) * 3)
    cc = W.case("bubble_32", ne=(coarse_ne,) * 3)
    L = cc["grid"]["hi"][0]
    Yf0, Yref_f, dt_f = W.initial_state(cf)
    xyz_f = W.node_coords(cf["grid"])
    gf = B.Grid(cf["grid"])
    mf = B.Model(gf, cf["model"], Yref_f)
    gc = B.Grid(cc["grid"])
    Yref_c = coarse_grain_state(Yref_f, cf["grid"]["ne"])
    Delta = float(np.cbrt(np.prod((np.array(cc["grid"]["hi"]) / np.array(cc["grid"]["ne"])) / 4.0)))
    feat_model = B.Model(gc, dict(cc["model"], closure="smag", richardson=True), Yref_c)

    snaps = {}
    want = sorted(set(list(t_train) + [0.0, t_eval]))
    Ya, Yb, dQ = mf.new_state(Yf0), mf.new_state(), mf.new_state()
    t = 0.0
    nsteps = 0
    for tw in want:
        n = int(round((tw - t) / dt_f))
        for s in range(n):
            mf.lsrk_step(Ya, Yb, dQ, t, dt_f)
            Ya, Yb = Yb, Ya
            t += dt_f
            nsteps += 1
            if nsteps % 2000 == 0:
                torch.cuda.synchronize()
                log("fine run: step %d  t = %.1f s  (%.0f s elapsed)" % (nsteps, t, time.time() - t_start))
        Yh = mf.to_numpy(Ya)
        snaps[tw] = filtered(Yh, xyz_f[2], cf["grid"]["ne"])
        d = mf.diagnostics(Ya, dt_f)
        log("snapshot t = %.1f s  max|w| %.3f  (%.0f s elapsed)" % (t, d["max_abs_w"], time.time() - t_start))
    del Ya, Yb, dQ, mf

    # training set
    Xs, Ts = [], []
    for tw in t_train:
        Yc, ruu, rth, rthu = snaps[tw]
        feat = feat_model.closure_inputs(feat_model.new_state(Yc)).cpu().numpy()
        T, mask = sgs_targets(Yc, ruu, rth, rthu, feat, Delta)
        Xs.append(feat[mask, :12])
        Ts.append(T[mask])
    X = np.concatenate(Xs)
    T = np.concatenate(Ts)
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std == 0] = 1.0
    Xn = (X - mean) / std
    lo, hi = Xn.min(axis=0), Xn.max(axis=0)
    log("training samples: %d" % X.shape[0])
    rng = np.random.default_rng(seed + 1)
    net = B.MLP(seed=seed, lr=1e-3)
    Xd = torch.from_numpy(Xn.astype(np.float32)).cuda()
    Td = torch.from_numpy(T.astype(np.float32)).cuda()
    losses = []
    for it in range(train_steps):
        idx = torch.from_numpy(rng.integers(0, X.shape[0], batch)).cuda()
        l = net.train_step(Xd[idx].contiguous(), Td[idx].contiguous(), want_loss=(it % 500 == 0 or it == train_steps - 1))
        if l is not None:
            losses.append((it, l))
            log("train step %d loss %.4f" % (it, l))
    params = net.params()
    norm = np.concatenate([mean, std, lo, hi]).astype(np.float32)

    # held-out samples: the evaluation snapshot (not trained on), raw inputs
    # and targets, for the a-priori comparison with Smagorinsky-Lilly
    Yc, ruu, rth, rthu = snaps[t_eval]
    feat = feat_model.closure_inputs(feat_model.new_state(Yc)).cpu().numpy()
    Th, mask = sgs_targets(Yc, ruu, rth, rthu, feat, Delta)
    sel = np.flatnonzero(mask)
    sel = rng.choice(sel, size=min(n_holdout, sel.size), replace=False)
    X_hold, T_hold = feat[sel, :12], Th[sel]

    # a-posteriori: coarse runs from the filtered initial state
    Yc0 = snaps[0.0][0]
    Yc_eval = snaps[t_eval][0]
    xyz_c = W.node_coords(cc["grid"])
    th_ref = snaps[t_eval][2] / Yc_eval[0]
    w_ref = Yc_eval[3] / Yc_eval[0]
    th_bg = _theta(Yref_c, xyz_c[2])
    dt_c = W.cfl_dt(cc["grid"], 360.0)
    n_c = int(round(t_eval / dt_c))
    dt_c = t_eval / n_c
    results = {"fine_ne": fine_ne, "coarse_ne": coarse_ne, "t_eval": t_eval, "t_train": list(t_train),
               "train_samples": int(X.shape[0]), "train_steps": train_steps, "losses": losses,
               "dt_fine": dt_f, "dt_coarse": dt_c}
    for name, closure in (("smagorinsky", "smag"), ("learned", "mlp"), ("learned_no_fallback", "mlp")):
        m = B.Model(gc, dict(cc["model"], closure=closure), Yref_c)
        if closure == "mlp":
            nrm = norm.copy()
            if name == "learned_no_fallback":
                nrm[24:36] = -1e30
                nrm[36:48] = 1e30
            m.set_mlp(params, nrm)
        Ya, Yb, dQ = m.new_state(Yc0), m.new_state(), m.new_state()
        tt = 0.0
        t0 = time.time()
        for s in range(n_c):
            m.lsrk_step(Ya, Yb, dQ, tt, dt_c)
            Ya, Yb = Yb, Ya
            tt += dt_c
        torch.cuda.synchronize()
        el = time.time() - t0
        Y = m.to_numpy(Ya)
        th = _theta(Y, xyz_c[2])
        w = Y[3] / Y[0]
        e_th = float(np.linalg.norm(th - th_ref) / np.linalg.norm(th_ref - th_bg))
        e_w = float(np.linalg.norm(w - w_ref) / np.linalg.norm(w_ref))
        r = {"theta_rel_l2": e_th, "w_rel_l2": e_w, "steps": n_c, "seconds": el,
             "dof_updates_per_s": gc.n_nodes * 5 * 5 * n_c / el}
        if closure == "mlp":
            r["fallback_fraction"] = m.mlp_fallbacks() / float(gc.n_nodes * 5 * n_c)
        results[name] = r
        log("%s: theta err %.4f  w err %.4f  (%.1f s)" % (name, e_th, e_w, el))
    results["seconds_total"] = time.time() - t_start
    results["params"] = params.tolist()
    results["norm"] = norm.tolist()
    if out_json:
        with open(out_json, "w") as f:
            json.dump(results, f)
    if out_npz:
        np.savez_compressed(out_npz, params=params, norm=norm, X_holdout=X_hold.astype(np.float32),
                            T_holdout=T_hold.astype(np.float32), Delta=np.float64(Delta),
                            Prt=np.float64(cc["model"]["Prt"]), Cs=np.float64(cc["model"]["Cs"]))
    return results


def coarse_grain_state(Yf, ne_fine):
    P = projection_matrix()
    return np.stack([coarse_grain(Yf[v], ne_fine, P) for v in range(Yf.shape[0])])


if __name__ == "__main__":
    fine = int(sys.argv[1]) if len(sys.argv) > 1 else 64
    out = sys.argv[2] if len(sys.argv) > 2 else None
    npz = sys.argv[3] if len(sys.argv) > 3 else None
    run_pipeline(fine_ne=fine, out_json=out, out_npz=npz, log=lambda s: print(s, flush=True))
