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

Schedule (`train`): the 64^3 FP64 resolved run to 650 s, training snapshots
every 50 s over 100-600 s, the a-posteriori comparison at 600 s for
Smagorinsky, the network with the Smagorinsky fallback (three training seeds)
and without it; held out: the t = 650 s snapshot and (`heldout`) a +3 K
bubble, for which the trained network is run a posteriori as well.  Each
held-out set is stored as a box of the filtered state and the SGS fluxes, so
that the closure inputs can be recomputed independently of the GPU.
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


def sgs_fluxes(Yc, ruu, rth, rthu):
    """Deviatoric Favre SGS stress [3, 3, n] and SGS potential-temperature
    flux [3, n] from the filtered state and filtered products."""
    rho = Yc[0]
    m = Yc[1:4]
    tau = np.zeros((3, 3, rho.size))
    for q, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        tau[a, b] = ruu[q] - m[a] * m[b] / rho
        tau[b, a] = tau[a, b]
    tr = (tau[0, 0] + tau[1, 1] + tau[2, 2]) / 3.0
    for a in range(3):
        tau[a, a] -= tr
    return tau, rthu - rth[None] * m / rho[None]


def targets_from_fluxes(rho, tau, q, gu, gth, Delta, nu_min_ratio=1e-4):
    """Targets in the raw-output space and a mask of usable nodes from the
    SGS fluxes and the filtered gradients gu [3, 3, n] (d u_i / d x_j) and
    gth [3, n]: nu* = max(0, -tau : S / (2 rho S:S)), D* = max(0, -q . grad
    theta / (rho |grad theta|^2)), Pr* = clip(nu*/D*, 0.1, 10),
    o1 = softplus^-1(nu* / (Delta^2 |S|)), o2 = softplus^-1(Pr* - 0.1)."""
    S = 0.5 * (gu + gu.transpose(1, 0, 2))
    SS = np.sum(S * S, axis=(0, 1))
    nu_s = np.maximum(0.0, -np.sum(tau * S, axis=(0, 1)) / (2.0 * rho * np.maximum(SS, 1e-30)))
    gg = np.sum(gth * gth, axis=0)
    D_s = np.maximum(0.0, -np.sum(q * gth, axis=0) / (rho * np.maximum(gg, 1e-30)))
    Pr_s = np.clip(nu_s / np.maximum(D_s, 1e-30), 0.1, 10.0)
    Smag = np.sqrt(2.0 * SS)
    z1 = nu_s / (Delta * Delta * np.maximum(Smag, 1e-30))
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.log(np.expm1(np.clip(z1, nu_min_ratio, 10.0)))
        t2 = np.log(np.expm1(np.clip(Pr_s - 0.1, 1e-3, 9.9)))
    mask = (Smag > 1e-3) & np.isfinite(t1) & np.isfinite(t2)
    return np.stack([t1, t2], axis=1), mask


def sgs_targets(Yc, ruu, rth, rthu, feat, Delta, nu_min_ratio=1e-4):
    """Targets and mask from the filtered fields and the gradient-pass
    features feat [n, 16] (grad u in columns 0-8, grad theta_v in 12-14)."""
    tau, q = sgs_fluxes(Yc, ruu, rth, rthu)
    return targets_from_fluxes(Yc[0], tau, q, feat[:, :9].T.reshape(3, 3, -1), feat[:, 12:15].T, Delta,
                               nu_min_ratio)


# the configured schedule: training snapshots every 50 s over 100-600 s,
# a-posteriori errors at 600 s, held out: t = 650 s and a +3 K bubble
C5_TRAIN = tuple(100.0 + 50.0 * k for k in range(11))
C5_EVAL = 600.0
C5_HOLDOUT = 650.0
HELDOUT_DTHETA = 1.5          # cosine bell dtheta (1 + cos): a 3 K peak
HELDOUT_T = 500.0


class _Filterer:
    """Coarse-grains snapshots on a host thread while the GPU keeps stepping."""

    def __init__(self, zf, ne_fine):
        import queue
        import threading

        self.zf, self.ne = zf, ne_fine
        self.q = queue.Queue(maxsize=2)
        self.out, self.err = {}, None
        self.th = threading.Thread(target=self._run, daemon=True)
        self.th.start()

    def _run(self):
        while True:
            item = self.q.get()
            if item is None:
                return
            key, Y = item
            try:
                self.out[key] = filtered(Y, self.zf, self.ne)
            except BaseException as e:  # re-raised by finish()
                self.err = e

    def submit(self, key, Y):
        self.q.put((key, Y))

    def finish(self):
        self.q.put(None)
        self.th.join()
        if self.err is not None:
            raise self.err
        return self.out


def resolved_run(cf, times, log, t_start):
    """The resolved (fine) run with LSRK54 from the case's initial state;
    returns the filtered snapshots at `times` (keyed by the requested time),
    the fine background and the fine step."""
    import torch

    Yf0, Yref_f, dt_f = W.initial_state(cf)
    zf = W.node_coords(cf["grid"])[2]
    mf = B.Model(B.Grid(cf["grid"]), cf["model"], Yref_f)
    flt = _Filterer(zf, cf["grid"]["ne"])
    Ya, Yb, dQ = mf.new_state(Yf0), mf.new_state(), mf.new_state()
    del Yf0
    t, nsteps = 0.0, 0
    for tw in sorted(set(times)):
        for _ in range(int(round((tw - t) / dt_f))):
            mf.lsrk_step(Ya, Yb, dQ, t, dt_f)
            Ya, Yb = Yb, Ya
            t += dt_f
            nsteps += 1
            if nsteps % 2000 == 0:
                torch.cuda.synchronize()
                log("resolved run: step %d  t = %.1f s  (%.0f s elapsed)" % (nsteps, t, time.time() - t_start))
        flt.submit(tw, mf.to_numpy(Ya))
        d = mf.diagnostics(Ya, dt_f)
        log("snapshot t = %.1f s  max|w| %.3f  (%.0f s elapsed)" % (t, d["max_abs_w"], time.time() - t_start))
    del Ya, Yb, dQ, mf
    return flt.finish(), Yref_f, dt_f


def _features(feat_model, snap, Delta):
    Yc, ruu, rth, rthu = snap
    feat = feat_model.closure_inputs(feat_model.new_state(Yc)).cpu().numpy()
    T, mask = sgs_targets(Yc, ruu, rth, rthu, feat, Delta)
    return feat, T, mask


def train(X, T, seed, train_steps, batch, log):
    """Standardise the raw inputs and train the network on the GPU (init
    seed `seed`, minibatch seed `seed` + 1); returns params, norm, losses."""
    import torch

    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std == 0] = 1.0
    Xn = (X - mean) / std
    lo, hi = Xn.min(axis=0), Xn.max(axis=0)
    rng = np.random.default_rng(seed + 1)
    net = B.MLP(seed=seed, lr=1e-3)
    Xd = torch.from_numpy(Xn.astype(np.float32)).cuda()
    Td = torch.from_numpy(T.astype(np.float32)).cuda()
    losses = []
    for it in range(train_steps):
        idx = torch.from_numpy(rng.integers(0, X.shape[0], batch)).cuda()
        want = it % 500 == 0 or it == train_steps - 1
        l = net.train_step(Xd[idx].contiguous(), Td[idx].contiguous(), want_loss=want)
        if l is not None:
            losses.append((it, l))
            log("seed %d train step %d loss %.4f" % (seed, it, l))
    return net.params(), np.concatenate([mean, std, lo, hi]).astype(np.float32), losses


def no_fallback(norm):
    n = norm.copy()
    n[24:36] = -1e30
    n[36:48] = 1e30
    return n


def _errors(Y, zc, th_bg, snap):
    """theta and w errors of a coarse state against a filtered snapshot:
    relative L2 (theta of its deviation from the background) and RMS."""
    Yr = snap[0]
    th_ref = snap[2] / Yr[0]
    w_ref = Yr[3] / Yr[0]
    th = _theta(Y, zc)
    w = Y[3] / Y[0]
    n = float(th.size)
    return {"theta_rel_l2": float(np.linalg.norm(th - th_ref) / np.linalg.norm(th_ref - th_bg)),
            "w_rel_l2": float(np.linalg.norm(w - w_ref) / np.linalg.norm(w_ref)),
            "theta_rms_K": float(np.linalg.norm(th - th_ref) / np.sqrt(n)),
            "theta_dev_rms_K": float(np.linalg.norm(th_ref - th_bg) / np.sqrt(n)),
            "w_rms": float(np.linalg.norm(w - w_ref) / np.sqrt(n)),
            "w_ref_rms": float(np.linalg.norm(w_ref) / np.sqrt(n))}


def posteriori(cc, Yref_c, Yc0, snaps, t_eval, nets, log, on_result=None):
    """Coarse runs from the filtered initial state to t_eval, one per
    (name, closure, params, norm), against the filtered resolved run at
    t_eval (and, as a history, at every other snapshot time after 0): theta
    (its deviation from the background) and w errors."""
    import torch

    gc = B.Grid(cc["grid"])
    zc = W.node_coords(cc["grid"])[2]
    th_bg = _theta(Yref_c, zc)
    dt_c = W.cfl_dt(cc["grid"], 360.0)
    n_c = int(round(t_eval / dt_c))
    dt_c = t_eval / n_c
    checks = {int(round(tc / dt_c)): tc for tc in snaps if 0.0 < tc < t_eval}
    out = {"dt_coarse": dt_c, "steps": n_c}
    for name, closure, params, norm in nets:
        m = B.Model(gc, dict(cc["model"], closure=closure), Yref_c)
        if closure == "mlp":
            m.set_mlp(params, norm)
        Ya, Yb, dQ = m.new_state(Yc0), m.new_state(), m.new_state()
        tt = 0.0
        hist = {}
        el = 0.0
        t0 = time.time()
        for s in range(1, n_c + 1):
            m.lsrk_step(Ya, Yb, dQ, tt, dt_c)
            Ya, Yb = Yb, Ya
            tt += dt_c
            if s in checks:
                torch.cuda.synchronize()
                el += time.time() - t0
                e = _errors(m.to_numpy(Ya), zc, th_bg, snaps[checks[s]])
                hist["%g" % checks[s]] = [e["theta_rel_l2"], e["w_rel_l2"]]
                t0 = time.time()
        torch.cuda.synchronize()
        el += time.time() - t0
        r = _errors(m.to_numpy(Ya), zc, th_bg, snaps[t_eval])
        r.update({"seconds": el, "dof_updates_per_s": gc.n_nodes * 5 * 5 * n_c / el, "history": hist})
        if closure == "mlp":
            r["fallback_fraction"] = m.mlp_fallbacks() / float(gc.n_nodes * 5 * n_c)
        out[name] = r
        log("%s: theta err %.4f  w err %.4f  (%.1f s)  history %s"
            % (name, r["theta_rel_l2"], r["w_rel_l2"], el, hist))
        if on_result is not None:
            on_result(out)
        del Ya, Yb, dQ, m
    return out


def heldout_box(snap, mask, grid_c, nb=6):
    """A box of nb^3 coarse elements around the element with the most
    usable nodes: the filtered state (float32) on the box and the SGS fluxes
    (float32) on its interior elements, whose face neighbours are all in the
    box, so closure inputs can be recomputed from the box alone."""
    ne = grid_c["ne"]
    Yc = snap[0]
    tau, q = sgs_fluxes(*snap)
    cnt = mask.reshape(-1, 125).sum(axis=1)
    e = int(cnt.argmax())
    ec = (e % ne[0], (e // ne[0]) % ne[1], e // (ne[0] * ne[1]))
    st = [int(min(max(ec[d] - nb // 2, 0), ne[d] - nb)) for d in range(3)]
    ez, ey, ex = np.meshgrid(*[np.arange(st[d], st[d] + nb) for d in (2, 1, 0)], indexing="ij")
    elems = ((ez * ne[1] + ey) * ne[0] + ex).ravel()                    # box order, x fastest
    nodes = (elems[:, None] * 125 + np.arange(125)[None]).ravel()
    inner = np.zeros((nb, nb, nb), bool)
    inner[1:-1, 1:-1, 1:-1] = True
    inner_nodes = np.repeat(inner.ravel(), 125)
    sel = nodes[inner_nodes]
    h = (np.array(grid_c["hi"]) - np.array(grid_c["lo"])) / np.array(ne)
    lo = np.array(grid_c["lo"]) + np.array(st) * h
    return {"Y": Yc[:, nodes].astype(np.float32), "tau": tau[:, :, sel].astype(np.float32),
            "q": q[:, sel].astype(np.float32), "inner": inner_nodes, "lo": lo, "hi": lo + nb * h,
            "ne": np.array([nb] * 3), "start": np.array(st)}


def run_pipeline(fine_ne=64, t_train=C5_TRAIN, t_eval=C5_EVAL, t_holdout=C5_HOLDOUT, train_steps=3000,
                 batch=8192, seeds=(0, 1, 2), out_json=None, out_npz=None, log=print):
    """Resolved run, coarse-graining, training (one network per seed; the
    first is the deployed one) and the a-posteriori comparison at t_eval;
    the t_holdout snapshot (not trained on) gives the held-out box."""
    t_start = time.time()
    coarse_ne = fine_ne // 2
    cf = W.case("bubble_32", ne=(fine_ne,) * 3)
    cc = W.case("bubble_32", ne=(coarse_ne,) * 3)
    times = [0.0] + list(t_train) + [t_eval] + ([t_holdout] if t_holdout else [])
    snaps, Yref_f, dt_f = resolved_run(cf, times, log, t_start)
    gc = B.Grid(cc["grid"])
    Yref_c = coarse_grain_state(Yref_f, cf["grid"]["ne"])
    Delta = float(np.cbrt(np.prod((np.array(cc["grid"]["hi"]) / np.array(cc["grid"]["ne"])) / 4.0)))
    feat_model = B.Model(gc, dict(cc["model"], closure="smag", richardson=True), Yref_c)
    Xs, Ts = [], []
    for tw in t_train:
        feat, T, mask = _features(feat_model, snaps[tw], Delta)
        Xs.append(feat[mask, :12])
        Ts.append(T[mask])
    X = np.concatenate(Xs)
    T = np.concatenate(Ts)
    del Xs, Ts
    log("training samples: %d" % X.shape[0])
    trained = [train(X, T, s, train_steps, batch, log) for s in seeds]
    params, norm, losses = trained[0]
    results = {"fine_ne": fine_ne, "coarse_ne": coarse_ne, "t_eval": t_eval, "t_train": list(t_train),
               "t_holdout": t_holdout, "train_samples": int(X.shape[0]), "train_steps": train_steps,
               "batch": batch, "seeds": list(seeds), "losses": losses, "dt_fine": dt_f}
    box = None
    if t_holdout:
        _, _, mask = _features(feat_model, snaps[t_holdout], Delta)
        box = heldout_box(snaps[t_holdout], mask, cc["grid"])
    del feat_model
    nets = [("smagorinsky", "smag", None, None), ("learned", "mlp", params, norm),
            ("learned_no_fallback", "mlp", params, no_fallback(norm))]
    nets += [("learned_seed%d" % s, "mlp", p, nm) for s, (p, nm, _) in zip(seeds[1:], trained[1:])]
    results["params"] = params.tolist()
    results["norm"] = norm.tolist()

    def save(partial):
        results.update(partial)
        results["seconds_total"] = time.time() - t_start
        if out_json:
            with open(out_json, "w") as f:
                json.dump(results, f)

    if out_npz:
        extra = {} if box is None else {"box_%s" % k: v for k, v in box.items()}
        np.savez_compressed(out_npz, params=params, norm=norm, Delta=np.float64(Delta),
                            Prt=np.float64(cc["model"]["Prt"]), Cs=np.float64(cc["model"]["Cs"]),
                            t_box=np.float64(t_holdout or 0.0), **extra)
    save(posteriori(cc, Yref_c, snaps[0.0][0], snaps, t_eval, nets, log, on_result=save))
    return results


def run_heldout(weights_npz, fine_ne=64, dtheta=HELDOUT_DTHETA, t_eval=HELDOUT_T, out_json=None, out_npz=None,
                log=print):
    """The held-out +3 K bubble: resolved run to t_eval, the a-posteriori
    comparison of the trained network (never shown this bubble) with
    Smagorinsky, and a held-out box of the filtered t_eval state."""
    t_start = time.time()
    z = np.load(weights_npz)
    params, norm = z["params"].astype(np.float32), z["norm"].astype(np.float32)
    coarse_ne = fine_ne // 2
    cf = W.case("bubble_32", ne=(fine_ne,) * 3)
    cc = W.case("bubble_32", ne=(coarse_ne,) * 3)
    cf["ic"]["dtheta"] = cc["ic"]["dtheta"] = dtheta
    snaps, Yref_f, dt_f = resolved_run(cf, [0.0] + [t_eval * k / 5.0 for k in range(1, 6)], log, t_start)
    gc = B.Grid(cc["grid"])
    Yref_c = coarse_grain_state(Yref_f, cf["grid"]["ne"])
    Delta = float(np.cbrt(np.prod((np.array(cc["grid"]["hi"]) / np.array(cc["grid"]["ne"])) / 4.0)))
    feat_model = B.Model(gc, dict(cc["model"], closure="smag", richardson=True), Yref_c)
    _, _, mask = _features(feat_model, snaps[t_eval], Delta)
    box = heldout_box(snaps[t_eval], mask, cc["grid"])
    del feat_model
    nets = [("smagorinsky", "smag", None, None), ("learned", "mlp", params, norm),
            ("learned_no_fallback", "mlp", params, no_fallback(norm))]
    results = {"fine_ne": fine_ne, "coarse_ne": coarse_ne, "dtheta": dtheta, "t_eval": t_eval, "dt_fine": dt_f}
    if out_npz:
        np.savez_compressed(out_npz, Delta=np.float64(Delta), dtheta=np.float64(dtheta), t_box=np.float64(t_eval),
                            **{"box_%s" % k: v for k, v in box.items()})

    def save(partial):
        results.update(partial)
        results["seconds_total"] = time.time() - t_start
        if out_json:
            with open(out_json, "w") as f:
                json.dump(results, f)

    save(posteriori(cc, Yref_c, snaps[0.0][0], snaps, t_eval, nets, log, on_result=save))
    return results


def coarse_grain_state(Yf, ne_fine):
    P = projection_matrix()
    return np.stack([coarse_grain(Yf[v], ne_fine, P) for v in range(Yf.shape[0])])


if __name__ == "__main__":
    # python -m paper_2110_00853_amd.learned train OUT.json OUT.npz [fine_ne]
    # python -m paper_2110_00853_amd.learned heldout WEIGHTS.npz OUT.json OUT.npz [fine_ne]
    say = lambda s: print(s, flush=True)
    if sys.argv[1] == "train":
        fine = int(sys.argv[4]) if len(sys.argv) > 4 else 64
        run_pipeline(fine_ne=fine, out_json=sys.argv[2], out_npz=sys.argv[3], log=say)
    elif sys.argv[1] == "heldout":
        fine = int(sys.argv[5]) if len(sys.argv) > 5 else 64
        run_heldout(sys.argv[2], fine_ne=fine, out_json=sys.argv[3], out_npz=sys.argv[4], log=say)
    else:
        raise SystemExit("usage: learned.py train OUT.json OUT.npz | heldout WEIGHTS.npz OUT.json OUT.npz")
