"""Throughput of the DG right-hand side + LSRK54 step on one MI355X.

A step is one LSRK54 time step: five stages, each one gradient/closure pass
and one tendency pass with the fused stage update, over the whole mesh
(1000 timed steps by default, as the workload is defined).
Default workload: the dry rising bubble on 32 x 32 x 32 elements, N = 4
(4,096,000 nodes, 5 variables), Smagorinsky-Lilly with the Richardson
correction, FP64.  Inputs are synthetic and resident in HBM before timing.

Prints ONE JSON line: DOF-updates/s = nodes x vars x 5 stages x steps / t,
the roofline of the dominant kernel (tendency pass) from hipEvents around
every launch in the timed region, the FP32-bulk variant, the learned-closure
variant (fused BF16 network in the gradient pass), the moist shallow-convection
(64x64x30) and warped Agnesi-mountain (96x16x50) setups in FP64 and FP32-bulk,
and the FP64 CPU oracle timed on this host on whole steps of the main workload.  The HBM traffic of
the tendency pass comes from the rocprofv3 counter summary under profiles/
when that summary was taken on the current kernel source (same SHA-256),
else it is null.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
KERNEL_SRC = os.path.join(ROOT, "paper_2110_00853_amd", "csrc", "dg_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_tend_bubble32_fp64.json")
MLP_WEIGHTS = os.path.join(ROOT, "paper_2110_00853_amd", "data", "mlp_bubble64_to_32.npz")


def measured_traffic(case: str, ne=None):
    """Counter-derived HBM bytes per tendency launch, if the summary was
    taken on this workload (the 32^3 bubble at its own element counts) and on
    the kernel source being timed; else None."""
    if case != "bubble_32" or ne is not None or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(KERNEL_SRC, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != sha:
        return None
    return t["hbm_bytes_per_launch"]


def alg_bytes(nvar: int, nf: int, s: int):
    """Algorithmic HBM bytes per node: gradient pass reads Y, writes F2;
    tendency pass reads Y, F2, dQ and writes dQ, Y_new (the first stage does
    not read dQ).  Neighbour face re-reads are counted as cache hits."""
    grad = (nvar + nf) * s
    tend_first = (3 * nvar + nf) * s
    tend_other = (4 * nvar + nf) * s
    return grad, tend_first, tend_other


def run(args):
    import numpy as np
    import torch

    from paper_2110_00853_amd import binding as B
    from paper_2110_00853_amd import workloads as W

    c = W.case(args.case)
    if args.ne:
        ne = [int(a) for a in args.ne.split(",")]
        scale = [ne[a] / c["grid"]["ne"][a] for a in range(3)]
        c["grid"]["hi"] = [c["grid"]["hi"][a] * scale[a] for a in range(3)]
        c["grid"]["ne"] = ne
    Y0, Yref, dt = W.initial_state(c)
    grid = B.Grid(c["grid"], device=0)
    nn, nvar = grid.n_nodes, c["model"]["nvar"]

    def timed(precision: str, steps: int, warmup: int, model=None, mlp=None):
        m = B.Model(grid, model or c["model"], Yref, precision=precision)
        if mlp is not None:
            m.set_mlp(*mlp)
        Ya, Yb, dQ = m.new_state(Y0), m.new_state(), m.new_state()
        stream = torch.cuda.current_stream()
        t = 0.0
        for _ in range(warmup):
            m.lsrk_step(Ya, Yb, dQ, t, dt, stream)
            Ya, Yb = Yb, Ya
            t += dt
        torch.cuda.synchronize()
        # the timed K steps (the throughput), then K more with an event pair
        # around every kernel launch (the per-kernel averages of the roofline;
        # the events add a few microseconds between launches, so they stay out
        # of the throughput run)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            m.lsrk_step(Ya, Yb, dQ, t, dt, stream)
            Ya, Yb = Yb, Ya
            t += dt
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ms = e0.elapsed_time(e1)
        m.profile(True)
        for _ in range(steps):
            m.lsrk_step(Ya, Yb, dQ, t, dt, stream)
            Ya, Yb = Yb, Ya
            t += dt
        torch.cuda.synchronize()
        prof = m.profile_read()
        m.profile(False)
        diag = m.diagnostics(Ya, dt)
        return m, Ya, ms, wall, prof, diag

    m64, Y64, ms, wall, prof, diag = timed("fp64", args.steps, args.warmup)
    ms_step = ms / args.steps
    value = nn * nvar * 5 * args.steps / (ms * 1e-3)
    nf = {5: 9, 6: 12}[nvar] + (0 if not c["model"].get("subsidence") else (1 if nvar == 5 else 2))
    g_b, tf_b, to_b = alg_bytes(nvar, nf, 8)
    tend_ms, tend_n = prof["tend"]
    grad_ms, grad_n = prof["grad"]
    tend_bytes = nn * (tf_b + 4 * to_b) / 5.0          # average launch (1 first + 4 other stages)
    tend_avg_s = tend_ms * 1e-3 / tend_n
    grad_avg_s = grad_ms * 1e-3 / max(grad_n, 1)
    achieved = tend_bytes / tend_avg_s / 1e9
    step_bytes = nn * (5 * g_b + tf_b + 4 * to_b)
    out = {
        "metric": "DOF-updates/s (nodes x vars x RK stages) for DG RHS+LSRK",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "%s: dry rising bubble, %dx%dx%d elements N=4 (%d nodes, %d vars), "
                        "Smagorinsky-Lilly Cs=0.21 + Richardson, LSRK54" % (
                            args.case, *c["grid"]["ne"], nn, nvar),
            "n_nodes": nn, "nvar": nvar, "dt": dt, "wall_s": wall,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_tend (tendency pass + fused LSRK54 stage update)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(args.case, args.ne),
            "avg_launch_us": tend_avg_s * 1e6,
            "alg_bytes_per_launch": tend_bytes,
            "grad_kernel": {"avg_launch_us": grad_avg_s * 1e6,
                            "achieved": nn * g_b / grad_avg_s / 1e9},
            "whole_step_alg_GBs": step_bytes / (ms_step * 1e-3) / 1e9,
            "whole_step_frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
        "diagnostics_after": {k: diag[k] for k in ("max_abs_w", "max_cfl", "T_min", "T_max", "n_nonfinite")},
    }
    if not args.no_fp32:
        m32, Y32, ms32, _, prof32, _ = timed("fp32", args.steps, args.warmup)
        v32 = nn * nvar * 5 * args.steps / (ms32 * 1e-3)
        a = m64.to_numpy(Y64)
        b = m32.to_numpy(Y32).astype(np.float64)
        err = [float(np.abs(a[v] - b[v]).max() / np.abs(a[v]).max()) for v in range(nvar)]
        g32, tf32, to32 = alg_bytes(nvar, nf, 4)
        t32_ms, t32_n = prof32["tend"]
        out["fp32_bulk"] = {
            "value": v32, "ms_per_step": ms32 / args.steps, "speedup_vs_fp64": v32 / value,
            "tend_achieved_GBs": nn * (tf32 + 4 * to32) / 5.0 / (t32_ms * 1e-3 / t32_n) / 1e9,
            "state_rel_err_vs_fp64_after_steps": err,
            "note": "warmup + 2 x steps LSRK54 steps from the same initial state (the timed steps, then the "
                    "profiled ones); max-norm error per variable",
        }
        del m32, Y32
    if not args.no_learned and c["model"].get("closure") == "smag":
        params, norm, origin = mlp_weights(B, grid, c, Yref, Y0)
        mdl = dict(c["model"], closure="mlp")
        mL, YL, msL, _, profL, _ = timed("fp64", args.steps, args.warmup, model=mdl, mlp=(params, norm))
        vL = nn * nvar * 5 * args.steps / (msL * 1e-3)
        fb = mL.mlp_fallbacks() / float(nn * 5 * (2 * args.steps + args.warmup))
        gL_ms, gL_n = profL["grad"]
        out["learned_closure"] = {
            "value": vL, "ms_per_step": msL / args.steps, "speedup_vs_fp64_smagorinsky": vL / value,
            "grad_kernel_avg_launch_us": gL_ms * 1e3 / gL_n,
            "fallback_fraction": fb, "weights": origin,
            "note": "FP64 state and fluxes; 12-64-64-64-2 SiLU network in BF16 MFMA (FP32 accumulate) "
                    "fused into the gradient pass, Smagorinsky-Lilly fallback",
        }
        del mL, YL
    out["hbm_copy_GBs"] = copy_bandwidth()
    out["roofline"]["achieved_vs_copy"] = achieved / out["hbm_copy_GBs"]
    if not args.no_setups:
        out["other_setups"] = {name: other_setup(name, args.setup_steps, 2) for name in ("moist_64", "agnesi_96")}
    if not args.no_next:
        out["next_rows"] = next_rows(max(args.setup_steps, 10), 2)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, Y0, Yref, nn, nvar, dt)
    return out


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 5):
    """Plain device-to-device copy on the same GPU: (read + write bytes) / time,
    the practical HBM ceiling next to the 8 TB/s vendor figure."""
    import torch

    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def other_setup(name: str, steps: int, warmup: int):
    """FP64 and FP32-bulk throughput of another named setup (same step, same
    timing as the main line, fewer steps)."""
    import numpy as np
    import torch

    from paper_2110_00853_amd import binding as B
    from paper_2110_00853_amd import workloads as W

    c = W.case(name)
    t0 = time.perf_counter()
    Y0, Yref, dt = W.initial_state(c)
    t_ic = time.perf_counter() - t0
    grid = B.Grid(c["grid"], device=0)
    nn, nvar = grid.n_nodes, c["model"]["nvar"]
    res = {"n_nodes": nn, "nvar": nvar, "elements": c["grid"]["ne"], "steps": steps, "ic_seconds": t_ic}
    # algorithmic words per node and stage: 5 nv state words, the stored
    # diffusive flux written once and read once, and on warped meshes the
    # per-node metric terms (10) and face metrics (about 4.8) read in both
    # passes
    nf_words = {5: 9, 6: 12}[nvar]
    metric_words = 2 * (10 + 4.8) if c["grid"].get("topo") == 1 else 0
    R0 = {}
    for prec in ("fp64", "fp32"):
        m = B.Model(grid, c["model"], Yref, precision=prec)
        Ya, Yb, dQ = m.new_state(Y0), m.new_state(), m.new_state()
        stream = torch.cuda.current_stream()
        # right-hand side at t = 0, for the FP32-bulk error against FP64
        m.rhs(Ya, dQ, 0.0, stream)
        R0[prec] = m.tendency_to_numpy(dQ).astype(np.float64)
        t = 0.0
        for _ in range(warmup):
            m.lsrk_step(Ya, Yb, dQ, t, dt, stream)
            Ya, Yb = Yb, Ya
            t += dt
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            m.lsrk_step(Ya, Yb, dQ, t, dt, stream)
            Ya, Yb = Yb, Ya
            t += dt
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        m.profile(True)           # per-kernel averages from a second, profiled run
        for _ in range(steps):
            m.lsrk_step(Ya, Yb, dQ, t, dt, stream)
            Ya, Yb = Yb, Ya
            t += dt
        torch.cuda.synchronize()
        prof = m.profile_read()
        m.profile(False)
        d = m.diagnostics(Ya, dt)
        sb = 8 if prec == "fp64" else 4
        b_alg = (5 * nvar + 2 * nf_words + metric_words) * sb  # bytes per node and stage
        res[prec] = {"value": nn * nvar * 5 * steps / (ms * 1e-3), "ms_per_step": ms / steps,
                     "alg_bytes_per_node_stage": b_alg,
                     "roofline_frac": nn * 5 * steps * b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "tend_avg_us": prof["tend"][0] * 1e3 / prof["tend"][1],
                     "grad_avg_us": prof["grad"][0] * 1e3 / max(prof["grad"][1], 1),
                     "n_nonfinite": d["n_nonfinite"]}
        del m, Ya, Yb, dQ
    # max-norm error per variable, relative to the largest tendency of its
    # equation (the three momentum components share one scale: at t = 0 a
    # component can have an almost vanishing tendency)
    a, b = R0["fp64"], R0["fp32"]
    scale = [np.abs(a[v]).max() for v in range(nvar)]
    mom = max(scale[1:4])
    res["fp32"]["rhs_rel_err_vs_fp64_t0"] = [float(np.abs(b[v] - a[v]).max() / (mom if 1 <= v <= 3 else scale[v]))
                                             for v in range(nvar)]
    return res


def lsrk_throughput(B, grid, c, Y0, Yref, dt, steps, warmup, scheme="lsrk54", precision="fp64"):
    """Throughput of one model with LSRK54 or LSRK144 (timed steps without
    per-kernel events, then as many profiled ones for the kernel averages)
    and the tendency pass's fraction of the HBM roofline on the algorithmic
    bytes of the headline formula."""
    import torch

    m = B.Model(grid, c["model"], Yref, precision=precision)
    Ya, Yb, dQ = m.new_state(Y0), m.new_state(), m.new_state()
    stream = torch.cuda.current_stream()
    nst = 5 if scheme == "lsrk54" else 14
    state = {"Ya": Ya, "Yb": Yb, "t": 0.0}

    def advance():
        if scheme == "lsrk54":
            m.lsrk_step(state["Ya"], state["Yb"], dQ, state["t"], dt, stream)
            state["Ya"], state["Yb"] = state["Yb"], state["Ya"]
        else:
            m.lsrk144_step(state["Ya"], state["Yb"], dQ, state["t"], dt, stream)
        state["t"] += dt

    for _ in range(warmup):
        advance()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        advance()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    m.profile(True)
    for _ in range(steps):
        advance()
    torch.cuda.synchronize()
    prof = m.profile_read()
    m.profile(False)
    d = m.diagnostics(state["Ya"], dt)
    nn, nvar = grid.n_nodes, c["model"]["nvar"]
    nf = 0
    if c["model"].get("closure", "none") != "none":
        nf = {5: 9, 6: 12}[nvar] + ((1 if nvar == 5 else 2) if c["model"].get("subsidence") else 0)
    sb = 8 if precision == "fp64" else 4
    _, tf_b, to_b = alg_bytes(nvar, nf, sb)
    tend_avg = prof["tend"][0] * 1e-3 / prof["tend"][1]
    tend_bytes = nn * (tf_b + (nst - 1) * to_b) / nst
    return {"value": nn * nvar * nst * steps / (ms * 1e-3), "ms_per_step": ms / steps, "stages": nst,
            "tend_avg_us": tend_avg * 1e6, "grad_avg_us": prof["grad"][0] * 1e3 / max(prof["grad"][1], 1),
            "tend_roofline_frac": tend_bytes / tend_avg / 1e9 / HBM_PEAK_GBS, "n_nonfinite": d["n_nonfinite"]}


def next_rows(steps: int, warmup: int):
    """The widened rows on their own workloads, FP64: LSRK144, the Vreman
    closure and the Roe and HLLC fluxes on the 32^3 bubble; the ice phase on
    the moist set-up; the density current; the exponential filter (one
    in-place pass over all five variables of the 32^3 bubble) and the 1-D
    IMEX step on a strongly anisotropic mesh, against LSRK54 at its own
    stable step there."""
    import torch

    from paper_2110_00853_amd import binding as B
    from paper_2110_00853_amd import workloads as W

    res = {}
    c = W.case("bubble_32")
    Y0, Yref, dt = W.initial_state(c)
    grid = B.Grid(c["grid"], device=0)
    res["lsrk144_bubble_32"] = lsrk_throughput(B, grid, c, Y0, Yref, dt, steps, warmup, scheme="lsrk144")
    for name, over in (("vreman_bubble_32", {"closure": "vreman"}), ("roe_bubble_32", {"flux": "roe"}),
                       ("hllc_bubble_32", {"flux": "hllc"})):
        cv = dict(c, model=dict(c["model"], **over))
        res[name] = lsrk_throughput(B, grid, cv, Y0, Yref, dt, steps, warmup)
    # exponential filter: read and write of every variable, in place
    m = B.Model(grid, c["model"], Yref)
    Yd = m.new_state(Y0)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        m.exp_filter(Yd, 0b11111, 64, 36.0, 0, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    nrep = 50
    for _ in range(nrep):
        m.exp_filter(Yd, 0b11111, 64, 36.0, 0, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / nrep
    fbytes = 2.0 * 5 * 8 * grid.n_nodes
    res["exp_filter_bubble_32"] = {"us_per_call": us, "alg_bytes": fbytes, "achieved_GBs": fbytes / us / 1e3,
                                   "roofline_frac": fbytes / us / 1e3 / HBM_PEAK_GBS}
    del m, Yd, grid
    cd = W.case("density_current")
    Yc, Yrc, dtc = W.initial_state(cd)
    res["density_current"] = lsrk_throughput(B, B.Grid(cd["grid"], device=0), cd, Yc, Yrc, dtc, steps, warmup)
    cm = W.case("moist_64")
    cm["model"]["ice"] = 1
    Ym, Yrm, dtm = W.initial_state(cm)
    res["ice_moist_64"] = lsrk_throughput(B, B.Grid(cm["grid"], device=0), cm, Ym, Yrm, dtm, max(steps // 10, 5), 2)
    # 1-D IMEX on 5 m-tall, 200 m-wide elements (32 x 32 x 32), constant
    # nu = 1: twelve times the explicit vertical limit (a horizontal Courant
    # number of 0.12), against LSRK54 at that limit
    ch = W.case("bubble_32", hi=(6400.0, 6400.0, 160.0))
    ch["model"] = dict(ch["model"], closure="const", nu=1.0)
    ch["ic"] = dict(ch["ic"], center=(3200.0, 3200.0, 80.0))
    Yh, Yrh, dth = W.initial_state(ch)
    gh = B.Grid(ch["grid"], device=0)
    mh = B.Model(gh, ch["model"], Yrh)
    Ya = mh.new_state(Yh)
    work = mh.hevi_workspace()
    dt_hevi = 12.0 * dth
    nh = max(steps // 10, 10)
    # the first step also forms the line factor (once per step size: every
    # line shares one matrix on this mesh); timed on its own
    torch.cuda.synchronize()
    e0.record(stream)
    mh.hevi_step(Ya, work, 0.0, dt_hevi, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_first = e0.elapsed_time(e1)
    for _ in range(2):
        mh.hevi_step(Ya, work, 0.0, dt_hevi, stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(nh):
        mh.hevi_step(Ya, work, 0.0, dt_hevi, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_h = e0.elapsed_time(e1) / nh
    dh = mh.diagnostics(Ya, dt_hevi)
    del mh, Ya, work
    ex = lsrk_throughput(B, gh, ch, Yh, Yrh, dth, nh, 3)
    res["hevi_anisotropic_32"] = {
        "ms_per_step": ms_h, "first_step_ms_with_line_factor": ms_first, "dt": dt_hevi,
        "lsrk54_ms_per_step": ex["ms_per_step"], "lsrk54_dt": dth,
        "simulated_time_speedup_vs_lsrk54": (dt_hevi / ms_h) / (dth / ex["ms_per_step"]),
        "n_nonfinite": dh["n_nonfinite"],
        "note": "ARK2 (explicit horizontal, implicit vertical acoustics), 32x32x32 elements of 200 x 200 x 5 m, "
                "const nu = 1, dt = 12 x the explicit vertical limit; LSRK54 at that limit on the same mesh; "
                "the timed steps reuse the line factor the first step formed (same dt)"}
    return res


def mlp_weights(B, grid, c, Yref, Y0):
    """Trained weights of the learned closure if the package holds them,
    else a seeded random initialisation standardised on this state's inputs
    (the cost of the fused network does not depend on its weights)."""
    import numpy as np
    import torch

    if os.path.exists(MLP_WEIGHTS):
        z = np.load(MLP_WEIGHTS)
        return z["params"], z["norm"], "trained: 2x coarse-grained 64^3 bubble run"
    m = B.Model(grid, dict(c["model"], closure="smag", richardson=True), Yref)
    f = m.closure_inputs(m.new_state(Y0))[:, :12]
    mean, std = f.mean(0), f.std(0)
    std = torch.where(std > 0, std, torch.ones_like(std))
    xn = (f - mean) / std
    norm = torch.cat([mean, std, xn.min(0).values, xn.max(0).values]).cpu().numpy()
    del m, f, xn
    return B.MLP(seed=0).params(), norm, "seeded random initialisation"


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(c, Y0, Yref, nn, nvar, dt, budget_s=15.0, max_steps=40, one_thread_s=5.0):
    """The FP64 oracle on this host, as it stands: whole LSRK54 steps of the
    same workload, repeated until about budget_s seconds of CPU work, with
    all the host threads it gets; then right-hand-side evaluations on one
    thread for about one_thread_s seconds (a fifth of a step each)."""
    import oracle

    og = oracle.Grid(c["grid"])
    om = oracle.Model(og, c["model"], Yref)
    Y, dQ = Y0, None
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps:
        Y, dQ = om.steps(Y, dt, 1, dQ=dQ)
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    t = time.perf_counter() - t0
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    n1 = 0
    t1 = time.perf_counter()
    while True:
        om.rhs(Y0)
        n1 += 1
        if time.perf_counter() - t1 >= one_thread_s:
            break
    t1 = time.perf_counter() - t1
    oracle.set_num_threads(threads)
    return {
        "value": nn * nvar * 5 * steps / t,
        "unit": "DOF-updates/s",
        "cores": threads,
        "kind": "oracle",
        "cpu": cpu_model(),
        "sample": "%d LSRK54 step(s) of the same workload (%d nodes x %d vars x 5 stages), %.1f s"
                  % (steps, nn, nvar, t),
        "one_thread": {"value": nn * nvar * n1 / t1, "unit": "DOF-updates/s",
                       "sample": "%d right-hand-side evaluation(s), %.1f s" % (n1, t1)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--case", default="bubble_32")
    ap.add_argument("--ne", default=None, help="override element counts, e.g. 16,16,16")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-setups", action="store_true", help="skip the moist and mountain setups")
    ap.add_argument("--no-next", action="store_true",
                    help="skip LSRK144, Vreman, Roe, HLLC, ice, density current, filter and 1-D IMEX")
    ap.add_argument("--setup-steps", type=int, default=100)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    out = run(args)
    if args.calibrate_copy:
        import torch

        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 8
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
