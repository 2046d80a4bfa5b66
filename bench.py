"""Benchmark: RK4 LLG steps (each = 4 h_eff evaluations: demag by pruned FFT
convolution with the Newell tensor + exchange, fused with the stage updates)
on one MI355X, through the HIP C ABI.

Default workload: 1024 x 1024 x 128 cells (134,217,728), cell 2.5 x 2.5 x 3 nm,
zero-padded 2048 x 2048 x 256, Ms 8e5 A/m, A 1.3e-11 J/m, alpha 0.02, dt 1e-13 s,
m = 3D Voronoi grains of 20 nm mean spacing with a random unit vector each,
FP32, FP64 tensor setup timed separately; the same workload in FP64 is timed
too.  Prints one JSON line.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12   # MI355X HBM3E, bytes/s
METRIC = "Mcell-updates/s of h_eff+LLG step, FP32 vs FP64 at stated error; % HBM roofline"

WORKLOADS = {
    "large": dict(grid=(1024, 1024, 128), cell=(2.5e-9, 2.5e-9, 3e-9), m="voronoi", seed=3,
                  name="single grid 1024x1024x128 (134M cells, padded 2048x2048x256), Voronoi grains 20 nm, "
                       "h_eff + RK4 LLG step, FP64 tensor setup timed separately"),
    "film": dict(grid=(512, 512, 16), cell=(2.5e-9, 2.5e-9, 3e-9), m="smooth", seed=2,
                 name="thin film 512x512x16 (padded 1024x1024x32), smooth texture + 1% noise, RK4 LLG steps"),
    "small": dict(grid=(32, 32, 4), cell=(2e-9, 2e-9, 2e-9), m="random", seed=1,
                  name="32x32x4 (padded 64x64x8), random unit m"),
    "sweep": dict(grid=None, cell=(2.5e-9, 2.5e-9, 3e-9), m="random", seed=4,
                  name="batched sweep: 64 uneven geometries (nx, ny in 48..384, nz in 1..8, Ms in 4e5..1.2e6), "
                       "h_eff + RK4 LLG step of all in one graph replay"),
    "rkf45": dict(grid=(1024, 1024, 128), cell=(2.5e-9, 2.5e-9, 3e-9), m="voronoi", seed=3,
                  name="single grid 1024x1024x128, Voronoi grains 20 nm, adaptive RKF45 LLG steps "
                       "(tolerance 1e-3 on the max-norm error, six h_eff evaluations per attempt)"),
    "sp4": dict(grid=(100, 25, 1), cell=(5e-9, 5e-9, 3e-9), m="sp4", seed=0,
                name="standard problem 4 as in the paper's script: 100x25x1 cells of 5x5x3 nm, relaxation with "
                     "the Barzilai-Borwein minimiser, then 1 ns of RKF45 LLG in (-24.6, 4.3, 0) mT, "
                     "output every 10 ps"),
    "fields": dict(grid=None, cell=(2e-9, 2e-9, 2e-9), m="random", seed=7,
                   name="each field term alone on a %sx%sx%s cube of random m (demag, exchange, Slonczewski "
                        "spin-transfer torque), FP64 as the paper times them"),
    "grad": dict(grid=(256, 256, 8), cell=(2.5e-9, 2.5e-9, 3e-9), m="smooth", seed=5,
                 name="differentiable 256x256x8: 200 RK4 steps, checkpoint every 20, gradient of mean m_z "
                      "w.r.t. per-cell Ms through the adjoint"),
}
MS, A, ALPHA, GAMMA, DT = 8e5, 1.3e-11, 0.02, 2.211e5, 1e-13
PASS_NAMES = ["z_fwd", "x_fwd", "y_fused", "x_inv", "z_inv_stage", "z_inv_heff"]
# kernel-name patterns of each pass (specialised first, runtime-planned second)
KERNEL_PATTERNS = {
    "z_fwd": [r"k_zfwd_ct<float", r"k_zfwd<float"],
    "x_fwd": [r"k_line_(ct|hx)<float, \d+, -1,", r"k_line_pass<float, -1, false>"],
    "y_fused": [r"k_fused_y_(ct|cr|hx|pf|pt|h2)<float", r"k_fused_y<float"],
    "x_inv": [r"k_line_(ct|hx)<float, \d+, 1,", r"k_line_pass<float, 1, false>"],
    "z_inv_stage": [r"k_zinv_ct<float, \d+, 1,", r"k_zinv<float, 1>"],
    "z_inv_heff": [r"k_zinv_ct<float, \d+, 0,", r"k_zinv<float, 0>"],
}
KERNEL_SYMBOL = {"z_fwd": "k_zfwd_ct", "x_fwd": "k_line_ct", "y_fused": "k_fused_y_ct", "x_inv": "k_line_ct",
                 "z_inv_stage": "k_zinv_ct", "z_inv_heff": "k_zinv_ct"}
# y pass variant (mm_plan_info tiles[2]) -> kernel; negative: runtime-planned
Y_SYMBOL = {0: "k_fused_y_ct", 1: "k_fused_y_hx", 2: "k_fused_y_cr", 3: "k_fused_y_pf", 4: "k_fused_y_pf",
            5: "k_fused_y_pt", 6: "k_fused_y_h2"}


def pass_bytes(grid, L, r):
    """Algorithmic HBM bytes per launch of each pass: every array the pass must
    read or write, once (no padding is ever materialised)."""
    nx, ny, nz = grid
    Lx, Ly, Lz = L
    c = 2 * r
    hx, hy, hz = Lx // 2 + 1, Ly // 2 + 1, Lz // 2 + 1
    N3 = 3 * nx * ny * nz
    S1 = 3 * nx * ny * hz
    S2 = 3 * Lx * ny * hz      # [kz][kx][y][c]: every kx < Lx, the ny rows that exist
    T6 = 6 * hx * hy * hz
    b = {
        "z_fwd": r * N3 + c * S1,
        "x_fwd": c * (S1 + S2),
        "y_fused": 2 * c * S2 + r * T6,
        "x_inv": c * (S2 + S1),
        # stage 1/2 of RK4: read S1, m_s, m_n, acc; write m_s', acc, S1 (next stage z spectrum)
        "z_inv_stage": c * S1 + 3 * r * N3 + 2 * r * N3 + c * S1,
        "z_inv_heff": c * S1 + r * N3 + r * N3,
    }
    stage = [c * S1 + r * N3 + 2 * r * N3 + c * S1,          # stage 0: m_s = m_n, writes acc, m_s'
             b["z_inv_stage"], b["z_inv_stage"],
             c * S1 + 3 * r * N3 + r * N3]                   # stage 3: writes m_n
    step = b["z_fwd"] + 4 * (b["x_fwd"] + b["y_fused"] + b["x_inv"]) + sum(stage)
    return b, step


def make_m(w):
    import numpy as np
    import synth
    if w["m"] == "voronoi":
        # the grain assignment of 134M cells takes a minute; keep one copy per
        # host in the temp directory for repeated runs
        import tempfile
        key = "mmx_voronoi_%s_%s_%d.npy" % ("x".join(map(str, w["grid"])), "_".join("%g" % c for c in w["cell"]), w["seed"])
        path = os.path.join(tempfile.gettempdir(), key)
        if os.path.exists(path):
            return np.load(path, mmap_mode="r")
        m = synth.voronoi_grains(w["grid"], w["cell"], w["seed"])
        try:
            np.save(path + ".tmp.npy", m)
            os.replace(path + ".tmp.npy", path)
        except OSError:
            pass
        return m
    if w["m"] == "smooth":
        return synth.smooth_film(w["grid"], w["cell"], w["seed"])
    return synth.random_unit(w["grid"], w["seed"])


def src_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_01114_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(pname, workload, prec, symbol=None):
    """HBM bytes per launch of pass `pname` from committed rocprofv3 counter
    runs, if they were taken on the current kernel sources and (given the
    running kernel's `symbol`) on that kernel; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(p) as f:
            t = json.load(f)
        e = t.get("%s/%s/%s" % (workload, prec, pname))
        if not e or e.get("src_hash") != src_hash():
            return None
        if symbol is None or (symbol + "<") in e["kernel"]:
            return e["bytes_per_launch"]
        # another variant of the pass: its own counters (the tuner's trial
        # launches), the most dispatched one of that kernel
        cand = [(v["dispatches"], v["bytes_per_launch"]) for k, v in e.get("variants", {}).items()
                if (symbol + "<") in k]
        return max(cand)[1] if cand else None
    except (OSError, ValueError, KeyError):
        pass
    return None


def run_gpu(wname, prec, steps, warmup, m_host):
    import torch
    from paper_2606_01114_amd import DemagPlan, _lib
    w = WORKLOADS[wname]
    dt = torch.float32 if prec == "f32" else torch.float64
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = DemagPlan(w["grid"], w["cell"], prec, autotune=True)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = plan.info()
    L = info["L"]
    m = torch.tensor(m_host, dtype=dt).to("cuda")
    for _ in range(warmup):
        plan.llg_step(m, MS, A, ALPHA, GAMMA, DT, n_steps=1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    plan.llg_step(m, MS, A, ALPHA, GAMMA, DT, n_steps=steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    # h_eff alone
    h = torch.empty_like(m)
    plan.h_eff(m, MS, A, out=h)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(max(3, steps)):
        plan.h_eff(m, MS, A, out=h)
    e1.record()
    torch.cuda.synchronize()
    heff_ms = e0.elapsed_time(e1) / max(3, steps)
    # per-pass durations, HIP events on the plan stream
    ms = (ctypes.c_double * 6)()
    _lib.check(_lib.lib().mm_plan_time_passes(plan._h, 5, ms))
    passes = dict(zip(PASS_NAMES, list(ms)))
    finite = bool(torch.isfinite(m).all().item())
    plan.close()
    del m, h
    torch.cuda.empty_cache()
    return dict(setup_s=setup_s, wall_s=wall, ev_ms=ev_ms, heff_ms=heff_ms, passes=passes, L=L, finite=finite,
                tiles=info["tiles"])


def run_sweep(steps, warmup, prec="f32", padding="ct"):
    """Aggregate cell-updates/s of the batched sweep (all geometries per graph
    replay) with the autotuned launch groups, the same with the default
    schedule, the groups the tuner chose, and the sweep's algorithmic bytes
    against the HBM roofline."""
    import numpy as np
    import torch
    import synth
    from paper_2606_01114_amd import Batch
    geo = synth.batch_geometries(4)
    grids = [g for g, _ in geo]
    Ms = [ms for _, ms in geo]
    dt = torch.float32 if prec == "f32" else torch.float64
    cells = int(sum(np.prod(g) for g in grids))
    # algorithmic bytes: the single-grid pass model of every geometry at its
    # padded lengths (the power of two >= 2n-1, or the shortest compile-time
    # length: powers of two and q*2^k with one odd radix q)
    r = 4 if prec == "f32" else 8
    padlen = _pow2_len if padding == "pow2" else _ct_len
    step_bytes = sum(pass_bytes(g, tuple(padlen(v, a) for a, v in enumerate(g)), r)[1] for g in grids)
    out = {"cells": cells, "geometries": len(grids), "prec": prec, "padding": padding,
           "step_algorithmic_bytes": step_bytes}
    for mode in ("off", "search"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = Batch(grids, [WORKLOADS["sweep"]["cell"]] * len(grids), prec, autotune=mode, padding=padding)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        ms = [torch.tensor(synth.random_unit(g, 100 + k), dtype=dt, device="cuda") for k, g in enumerate(grids)]
        for _ in range(warmup):
            b.llg_step(ms, Ms, A, ALPHA, GAMMA, DT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.llg_step(ms, Ms, A, ALPHA, GAMMA, DT, n_steps=steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms_step = wall * 1e3 / steps
        r_ = {"ms_per_step": ms_step, "Mcell_updates_per_s": cells * steps / wall / 1e6, "setup_s": setup}
        if mode == "search":
            out.update(r_)
            out["schedule"] = [{k: g[k] for k in ("pass", "L", "specialised", "variant", "W", "geometries")}
                               for g in b.schedule()["groups"]]
            ach = step_bytes / (ms_step * 1e-3)
            out["roofline"] = {"bound": "hbm", "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                               "frac": ach / HBM_PEAK, "bytes": "per step, all geometries, pass model"}
            out["step_hbm_frac"] = ach / HBM_PEAK
        else:
            out["default_schedule"] = r_
        b.close()
        del ms
    return out


def _pow2_len(n, axis=0):
    """Smallest power of two >= 2n-1 (1 for one cell): a batch's padding."""
    if n == 1:
        return 1
    L = 1
    while L < 2 * n - 1:
        L *= 2
    return L


# lengths with one odd radix that have compile-time kernels (x and y; z up
# to 896)
CT_ODD_XY = (96, 160, 192, 224, 320, 384, 448, 640, 768, 896, 1280, 1536, 1792)
CT_ODD_Z = tuple(L for L in CT_ODD_XY if L <= 896)


def _ct_len(n, axis=0):
    """Shortest length >= 2n-1 with compile-time FP32 kernels (powers of two
    and CT_ODD_XY on x and y, CT_ODD_Z on z), as the library's padding mode 3."""
    if n == 1:
        return 1
    odd = CT_ODD_XY if axis < 2 else CT_ODD_Z
    lim = 2048 if axis == 2 else 4096
    c = [L for L in [1 << k for k in range(13)] if L <= lim] + list(odd)
    ok = [L for L in c if L >= 2 * n - 1]
    return min(ok) if ok else _pow2_len(n)


def run_grad(prec="f32", steps=200, every=20):
    """Forward + backward time of the checkpointed LLG run and its gradient."""
    import torch
    import synth
    from paper_2606_01114_amd import DemagPlan, llg_run_checkpointed
    w = WORKLOADS["grad"]
    dt = torch.float32 if prec == "f32" else torch.float64
    plan = DemagPlan(w["grid"], w["cell"], prec, autotune=True)
    m0 = torch.tensor(synth.smooth_film(w["grid"], w["cell"], 5), dtype=dt, device="cuda")
    Ms = torch.tensor(synth.ms_field(w["grid"], 5), dtype=dt, device="cuda")
    out = {}
    for rep in range(2):
        Mst = Ms.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mT = llg_run_checkpointed(plan, m0, Mst, A, ALPHA, GAMMA, DT, steps, every=every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mT[..., 2].mean().backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out = {"forward_s": t1 - t0, "backward_s": t2 - t1, "steps": steps, "checkpoint_every": every,
               "cells": int(m0.numel() // 3), "prec": prec,
               "grad_finite": bool(torch.isfinite(Mst.grad).all().item())}
    plan.close()
    return out


# the paper's own per-field timings (FP64, N x N x N cube): context, another machine
PAPER_FIELD_MS = {
    350: {"demag": {"ms": 164.9, "hardware": "1x H100 HBM3"}},
    400: {"demag": {"ms": 31.2, "hardware": "8x H100 HBM3 (one node)"},
          "exchange": {"ms": 1.4, "hardware": "8x H100 HBM3 (one node)"},
          "stt": {"ms": 0.4, "hardware": "8x H100 HBM3 (one node)"}},
}


def run_fields(prec, N, steps, warmup, paddings=("smooth", "pow2", "auto")):
    """Per-field evaluation time on an N x N x N cube as the paper times its
    field terms (each term alone, FP64 by default): demag, exchange and the
    Slonczewski spin-transfer torque, for the 7-smooth padding 2N (runtime
    planned), the power-of-two padding and the default padding (the
    shortest compile-time length, odd-radix lengths included), or the given paddings."""
    import numpy as np
    import torch
    import synth
    from paper_2606_01114_amd import DemagPlan, MM_DEMAG, MM_EXCHANGE
    dt = torch.float32 if prec == "f32" else torch.float64
    r = 4 if prec == "f32" else 8
    grid, cell = (N, N, N), (2e-9, 2e-9, 2e-9)
    print("# generating inputs: random unit m on %d^3" % N, file=sys.stderr, flush=True)
    m = torch.tensor(synth.random_unit(grid, 7), dtype=dt, device="cuda")
    h = torch.empty_like(m)
    out = {"grid": list(grid), "cells": N ** 3, "prec": prec, "paddings": {}}
    names = {"smooth": "7-smooth", "pow2": "pow2", "auto": "auto"}
    for name, pad in ((names[p], p) for p in paddings):
        print("# timing %s padding" % name, file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = DemagPlan(grid, cell, prec, autotune=True, padding=pad)
        torch.cuda.synchronize()
        res = {"L": list(plan.info()["L"]), "setup_s": time.perf_counter() - t0}

        def timed(terms):
            for _ in range(warmup):
                plan.h_eff(m, MS, A, out=h, terms=terms)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(steps):
                plan.h_eff(m, MS, A, out=h, terms=terms)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / steps

        res["demag_ms"] = timed(MM_DEMAG)
        res["exchange_ms"] = timed(MM_EXCHANGE)
        plan.set_stt(1e11, P=0.4, Lambda=2.0, eps_prime=0.1, d_layer=1e-9, p=(0.0, 0.0, 1.0))
        res["stt_ms"] = timed(0)
        plan.set_stt(0.0)
        # the stencil and local terms read m (neighbours from cache) and write h
        res["exchange_GBps"] = 6 * r * N ** 3 / (res["exchange_ms"] * 1e-3) / 1e9
        res["stt_GBps"] = 6 * r * N ** 3 / (res["stt_ms"] * 1e-3) / 1e9
        res["demag_Mcell_per_s"] = N ** 3 / (res["demag_ms"] * 1e-3) / 1e6
        out["paddings"][name] = res
        plan.close()
        del plan
        torch.cuda.empty_cache()
    best = min(out["paddings"].values(), key=lambda v: v["demag_ms"])
    out["best"] = {k: best[k] for k in ("L", "demag_ms", "exchange_ms", "stt_ms")}
    out["paper"] = PAPER_FIELD_MS.get(N)
    return out


def run_rkf45(steps, warmup, prec, m_host, tol=1e-3):
    """Adaptive RKF45 on the large grid: attempted steps per second and
    accepted cell-updates per second (each attempt synchronises to read the
    max-norm error)."""
    import numpy as np
    import torch
    from paper_2606_01114_amd import DemagPlan
    w = WORKLOADS["rkf45"]
    dt_ = torch.float32 if prec == "f32" else torch.float64
    plan = DemagPlan(w["grid"], w["cell"], prec, autotune=True)
    m = torch.tensor(m_host, dtype=dt_, device="cuda")
    dt = DT
    for _ in range(warmup):
        _, _, dt = plan.rkf45_step(m, MS, A, ALPHA, GAMMA, dt, tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc, errs, dts = 0, [], []
    for _ in range(steps):
        ok, err, dt_next = plan.rkf45_step(m, MS, A, ALPHA, GAMMA, dt, tol)
        acc += int(ok)
        errs.append(err)
        dts.append(dt)
        dt = dt_next
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cells = int(np.prod(w["grid"]))
    plan.close()
    return {"attempts": steps, "accepted": acc, "ms_per_attempt": wall * 1e3 / steps,
            "Mcell_updates_per_s": cells * acc / wall / 1e6, "max_err": max(errs), "dt_first": dts[0],
            "dt_last": dts[-1], "tol": tol, "prec": prec,
            "finite": bool(torch.isfinite(m).all().item())}


def run_sp4(prec="f64", t_end=1e-9, out_dt=1e-11, tol=1e-5, min_tol=None):
    """Wall time of the standard-problem-4 script: relaxation and the field-1
    run, with the mean magnetisation every out_dt.  The minimiser stops at a
    max torque of 0.1 A/m in FP64 and 1 A/m in FP32 (whose rounding floor on
    fields of about 1e6 A/m is near 0.1 A/m)."""
    if min_tol is None:
        min_tol = 0.1 if prec == "f64" else 1.0
    import numpy as np
    import torch
    from paper_2606_01114_amd import DemagPlan
    w = WORKLOADS["sp4"]
    n = w["grid"]
    dt_ = torch.float32 if prec == "f32" else torch.float64
    mu0 = 4e-7 * np.pi
    H1 = (-24.6e-3 / mu0, 4.3e-3 / mu0, 0.0)
    m0 = np.zeros(n + (3,))
    m0[1:-1, :, :, 0] = 1.0
    m0[0, :, :, 1] = 1.0
    m0[-1, :, :, 1] = 1.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = DemagPlan(n, w["cell"], prec)
    m = torch.tensor(m0, dtype=dt_, device="cuda")
    it, tq = plan.minimize(m, MS, A, tol=min_tol, max_iter=20000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    relaxed = m.reshape(-1, 3).mean(0).tolist()
    series, t, dt, att, acc = [], 0.0, 1e-13, 0, 0
    for k in range(1, int(round(t_end / out_dt)) + 1):
        t_next = k * out_dt
        while t < t_next * (1 - 1e-12):
            h = min(dt, t_next - t)
            ok, _, dt = plan.rkf45_step(m, MS, A, ALPHA, GAMMA, h, tol, h_ext=H1)
            att += 1
            if ok:
                t += h
                acc += 1
        series.append(m.reshape(-1, 3).mean(0).tolist())
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    plan.close()
    return {"relax_s": t1 - t0, "relax_iterations": it, "relax_torque": tq, "relaxed_mean_m": relaxed,
            "llg_s": t2 - t1, "attempts": att, "accepted": acc, "final_mean_m": series[-1],
            "mean_m_every_100ps": series[9::10], "prec": prec}


def run_film_compare(steps=100):
    """The thin film in FP32 and FP64: RK4 throughput of each, the FP32 field
    error against the FP64 mode at step 0 over every cell, and the FP32
    trajectory against FP64 after `steps` steps (the increment m_n - m_0,
    relative L2)."""
    import numpy as np
    import torch
    from paper_2606_01114_amd import DemagPlan
    w = WORKLOADS["film"]
    m_host = make_m(w)
    m32h = torch.tensor(m_host, dtype=torch.float32)
    p = {prec: DemagPlan(w["grid"], w["cell"], prec, autotune=True) for prec in ("f32", "f64")}
    m0 = {"f32": m32h.to("cuda"), "f64": m32h.double().to("cuda")}

    def dev_rel(x, ref):
        return float(torch.linalg.vector_norm(x.double() - ref) / torch.linalg.vector_norm(ref))
    h32 = p["f32"].h_eff(m0["f32"], MS, A)
    h64 = p["f64"].h_eff(m0["f64"], MS, A)
    out = {"grid": list(w["grid"]), "heff_fp32_vs_fp64_rel_l2": dev_rel(h32, h64)}
    del h32, h64
    for prec in ("f32", "f64"):
        m = m0[prec].clone()
        p[prec].llg_step(m, MS, A, ALPHA, GAMMA, DT, n_steps=2)
        torch.cuda.synchronize()
        m = m0[prec].clone()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        p[prec].llg_step(m, MS, A, ALPHA, GAMMA, DT, n_steps=steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[prec] = {"ms_per_step": ms, "Mcell_updates_per_s": int(np.prod(w["grid"])) / (ms * 1e-3) / 1e6}
        out["m_" + prec] = m
    d32 = out.pop("m_f32").double() - m0["f64"]
    d64 = out.pop("m_f64") - m0["f64"]
    out["steps"] = steps
    out["increment_fp32_vs_fp64_rel_l2_after_steps"] = dev_rel(d32, d64)
    out["fp32_over_fp64"] = out["f32"]["Mcell_updates_per_s"] / out["f64"]["Mcell_updates_per_s"]
    for q in p.values():
        q.close()
    return out


def tensor_setup_time(w, prec):
    """Wall time of plan creation without the autotuner: the FP64 Newell
    tensor, its transforms and rounding, plus the plan's tables."""
    import torch
    from paper_2606_01114_amd import DemagPlan
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = DemagPlan(w["grid"], w["cell"], prec, autotune=False)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    plan.close()
    torch.cuda.empty_cache()
    return t


def copy_bandwidth():
    import torch
    from paper_2606_01114_amd import _lib
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(3):
        _lib.check(_lib.lib().mm_device_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), n, s))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        _lib.check(_lib.lib().mm_device_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), n, s))
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * n * 10 / (e0.elapsed_time(e1) * 1e-3)


def _cpu_worker(args):
    """One process of the CPU baseline: RK4 steps of the FP64 oracle on its
    own sub-grid of the workload's recipe until the time budget is spent."""
    w, sub, seed, budget_s = args
    import numpy as np
    import oracle
    import synth
    from threadpoolctl import threadpool_limits
    if w["m"] == "voronoi":
        m0 = synth.voronoi_grains(sub, w["cell"], seed)
    elif w["m"] == "smooth":
        m0 = synth.smooth_film(sub, w["cell"], seed)
    else:
        m0 = synth.random_unit(sub, seed)
    oct_ = oracle.tensor_octant(sub, w["cell"])
    L = tuple(oracle.default_L(v) for v in sub)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        steps, m = 0, m0
        while True:
            m = oracle.rk4_step(m, MS, A, w["cell"], oct_, L, ALPHA, GAMMA, DT)
            steps += 1
            if time.perf_counter() - t0 > budget_s or steps >= 200:
                break
        el = time.perf_counter() - t0
    return int(np.prod(sub)) * steps, steps, el


def _cpu_config_worker(name):
    """The oracle's h_eff and one RK4 step on a whole small workload (one
    process, one thread)."""
    import numpy as np
    import oracle
    import synth
    from threadpoolctl import threadpool_limits
    w = WORKLOADS[name]
    m0 = make_m(w)
    with threadpool_limits(limits=1):
        oct_ = oracle.tensor_octant(w["grid"], w["cell"])
        L = tuple(oracle.default_L(v) for v in w["grid"])
        t0 = time.perf_counter()
        oracle.h_eff(m0, MS, A, w["cell"], oct_, L)
        t1 = time.perf_counter()
        oracle.rk4_step(m0, MS, A, w["cell"], oct_, L, ALPHA, GAMMA, DT)
        t2 = time.perf_counter()
    cells = int(np.prod(w["grid"]))
    return {"workload": name, "grid": list(w["grid"]), "heff_s": t1 - t0, "rk4_step_s": t2 - t1,
            "Mcell_updates_per_s": cells / (t2 - t1) / 1e6}


def cpu_baseline(w, budget_s=15.0, configs=("small", "grad")):
    """The oracle as it stands (FP64, numpy FFT, one thread per process) on
    every host core the box gives this job (at most 16): each process steps
    its own 64x64x32 sub-grid of the workload's recipe (a bounded sample:
    the whole grid would take hours), and the rate is their sum.  Beside it,
    the oracle's h_eff and RK4 step on the whole 32x32x4 and 256x256x8
    workloads, one process each."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    nx, ny, nz = w["grid"]
    sub = (min(nx, 64), min(ny, 64), min(nz, 32))
    cores = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ProcessPoolExecutor(max_workers=cores, mp_context=ctx) as ex:
        res = list(ex.map(_cpu_worker, [(w, sub, w["seed"] + 1000 * k, budget_s) for k in range(cores)]))
    wall = time.perf_counter() - t0
    upd = sum(r[0] for r in res)
    steps = sum(r[1] for r in res)
    busy = max(r[2] for r in res)
    out = {"value": upd / busy / 1e6, "unit": "Mcell-updates/s", "cores": cores, "kind": "oracle",
           "sample": "%d processes (one thread each), each RK4-stepping its own %dx%dx%d sub-grid of the same "
                     "recipe with the FP64 oracle (numpy FFT) for %.0f s: %d steps in all (%.1f s wall with "
                     "start-up)" % (cores, sub[0], sub[1], sub[2], budget_s, steps, wall),
           "host_cpus": os.cpu_count()}
    if configs:
        with ProcessPoolExecutor(max_workers=len(configs), mp_context=ctx) as ex:
            out["per_workload"] = list(ex.map(_cpu_config_worker, configs))
    return out


def _pmc_means(path, counter):
    """Mean per-dispatch value of `counter` for every kernel name in a
    rocprofv3 counter-collection CSV."""
    import csv
    vals = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in vals.items()}


def traffic_from(fetch_csv, write_csv, workload, prec):
    """HBM bytes per launch of each pass from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by what the same
    counter reads for the 1 GiB plain copy kernel; written to profiles/traffic.json."""
    import re
    f = _pmc_means(fetch_csv, "FETCH_SIZE")
    w = _pmc_means(write_csv, "WRITE_SIZE")
    copy_f = [v[0] for k, v in f.items() if "k_copy16" in k]
    copy_w = [v[0] for k, v in w.items() if "k_copy16" in k]
    if not copy_f or not copy_w:
        raise SystemExit("no copy kernel in the counter runs")
    kf = copy_f[0] * 1024.0 / float(1 << 30)
    kw = copy_w[0] * 1024.0 / float(1 << 30)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            out = json.load(fh)
    except (OSError, ValueError):
        out = {}
    h = src_hash()
    for pname, pats in KERNEL_PATTERNS.items():
        for pat in pats:
            # the most-dispatched matching kernel (autotuner trials dispatch others a few times)
            fk = sorted((k for k in f if re.search(pat, k)), key=lambda k: -f[k][1])
            wk = sorted((k for k in w if re.search(pat, k)), key=lambda k: -w[k][1])
            if fk and wk:
                by = f[fk[0]][0] * 1024.0 / kf + w[wk[0]][0] * 1024.0 / kw
                variants = {k: {"bytes_per_launch": f[k][0] * 1024.0 / kf + w[k][0] * 1024.0 / kw,
                                "dispatches": min(f[k][1], w[k][1])} for k in fk if k in w}
                out["%s/%s/%s" % (workload, prec, pname)] = {
                    "bytes_per_launch": by, "kernel": fk[0], "fetch_KiB": f[fk[0]][0], "write_KiB": w[wk[0]][0],
                    "copy_scale_fetch": kf, "copy_scale_write": kw, "src_hash": h, "variants": variants}
                break
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1, sort_keys=True))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--traffic-from":
        traffic_from(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else "large",
                     sys.argv[5] if len(sys.argv) > 5 else "f32")
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 runs (the FP64 step and the per-field FP64 timings)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the film, sweep, gradient and small-grid runs of the default workload")
    ap.add_argument("--fields-n", default="350", help="cube edge of the fields workload (a comma list sweeps sizes)")
    ap.add_argument("--fields-f32", action="store_true", help="fields workload in FP32 (default FP64)")
    ap.add_argument("--padding", default="ct", choices=["pow2", "ct"],
                    help="sweep padding: the shortest compile-time lengths (powers of two and q*2^k, q = 3, 5, 7), or powers "
                         "of two only")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X (no GPU visible)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "sweep":
        r = run_sweep(args.steps, args.warmup, args.prec, args.padding)
        print(json.dumps({"metric": METRIC, "value": r["Mcell_updates_per_s"], "unit": "Mcell-updates/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
                          "data": "synthetic", "config": {"workload": WORKLOADS["sweep"]["name"]}, "extra": r}))
        return
    if args.workload == "fields":
        prec = "f64" if args.prec == "f32" and not args.fields_f32 else args.prec
        ns = [int(v) for v in str(args.fields_n).split(",")]
        if len(ns) > 1:
            # a sweep over cube sizes with the default padding, as the paper's
            # per-field curves over N
            rows = []
            for n in ns:
                r = run_fields(prec, n, args.steps, args.warmup, paddings=("auto",))
                rows.append(dict(N=n, cells=n ** 3, **r["best"]))
                print("# N=%d: %s" % (n, json.dumps(rows[-1])), file=sys.stderr, flush=True)
            print(json.dumps({"metric": "ms per field evaluation over cube sizes (each field term timed alone)",
                              "value": rows[-1]["demag_ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
                              "warmup": args.warmup, "ms_per_step": rows[-1]["demag_ms"], "higher_is_better": False,
                              "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
                              "config": {"workload": WORKLOADS["fields"]["name"] % ("N", "N", "N")
                                         + ", N in " + ",".join(map(str, ns))},
                              "extra": {"sweep": rows}}))
            return
        args.fields_n = ns[0]
        r = run_fields(prec, args.fields_n, args.steps, args.warmup)
        print(json.dumps({"metric": "ms per demag field evaluation (each field term timed alone)",
                          "value": r["best"]["demag_ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": r["best"]["demag_ms"], "higher_is_better": False,
                          "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
                          "config": {"workload": WORKLOADS["fields"]["name"] % (args.fields_n, args.fields_n,
                                                                               args.fields_n)},
                          "extra": r}))
        return
    if args.workload == "rkf45":
        print("# generating inputs: %s" % WORKLOADS["rkf45"]["name"], file=sys.stderr, flush=True)
        r = run_rkf45(args.steps, args.warmup, args.prec, make_m(WORKLOADS["rkf45"]))
        print(json.dumps({"metric": METRIC, "value": r["Mcell_updates_per_s"], "unit": "Mcell-updates/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_attempt"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
                          "data": "synthetic", "config": {"workload": WORKLOADS["rkf45"]["name"]}, "extra": r}))
        return
    if args.workload == "sp4":
        r = run_sp4(args.prec)
        print(json.dumps({"metric": "seconds for the standard-problem-4 script (relaxation + 1 ns)",
                          "value": r["relax_s"] + r["llg_s"], "unit": "s", "n_gpus": 1, "steps": r["attempts"],
                          "warmup": 0, "ms_per_step": r["llg_s"] * 1e3 / max(1, r["attempts"]),
                          "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
                          "data": "synthetic", "config": {"workload": WORKLOADS["sp4"]["name"]}, "extra": r}))
        return
    if args.workload == "grad":
        r = run_grad(args.prec)
        print(json.dumps({"metric": "forward+backward seconds of the differentiable run", "value":
                          r["forward_s"] + r["backward_s"], "unit": "s", "n_gpus": 1, "steps": r["steps"],
                          "warmup": 1, "ms_per_step": (r["forward_s"] + r["backward_s"]) * 1e3 / r["steps"],
                          "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
                          "data": "synthetic", "config": {"workload": WORKLOADS["grad"]["name"]}, "extra": r}))
        return
    w = WORKLOADS[args.workload]
    print("# generating inputs: %s" % w["name"], file=sys.stderr, flush=True)
    m_host = make_m(w)
    ncell = int(np.prod(w["grid"]))
    print("# timing %s" % args.prec, file=sys.stderr, flush=True)
    res = run_gpu(args.workload, args.prec, args.steps, args.warmup, m_host)
    r = 4 if args.prec == "f32" else 8
    pb, step_bytes = pass_bytes(w["grid"], res["L"], r)
    ms_step = res["ev_ms"] / args.steps
    value = ncell * args.steps / (res["wall_s"]) / 1e6
    launches = {"z_fwd": 1, "x_fwd": 4, "y_fused": 4, "x_inv": 4, "z_inv_stage": 4, "z_inv_heff": 0}
    share = {k: res["passes"][k] * launches[k] for k in launches}
    dom = max(share, key=share.get)
    ach = pb[dom] / (res["passes"][dom] * 1e-3)
    sym = dict(KERNEL_SYMBOL)
    sym["y_fused"] = Y_SYMBOL.get(res["tiles"][2], "k_fused_y")
    for pname, v in (("x_fwd", res["tiles"][3]), ("x_inv", res["tiles"][4])):
        if v >= 2:
            sym[pname] = "k_line_hx"
    roof = {"bound": "hbm", "kernel": sym[dom] + " (" + dom + ")", "achieved": ach / 1e9,
            "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": ach / HBM_PEAK,
            "traffic": load_traffic(dom, args.workload, args.prec, sym[dom]),
            "algorithmic_bytes_per_launch": pb[dom], "launch_ms": res["passes"][dom]}
    extra = {
        "ms_per_step_events": ms_step,
        "step_algorithmic_bytes": step_bytes,
        "step_hbm_frac": step_bytes / (ms_step * 1e-3) / HBM_PEAK,
        "heff_ms": res["heff_ms"], "heff_Mcell_per_s": ncell / (res["heff_ms"] * 1e-3) / 1e6,
        "plan_setup_s": res["setup_s"],
        "pass_ms": res["passes"],
        "pass_GBps": {k: pb[k] / (res["passes"][k] * 1e-3) / 1e9 for k in pb},
        "padded_L": list(res["L"]),
        "tiles": {"z_cols": res["tiles"][0], "x_cols": res["tiles"][1], "y_variant": res["tiles"][2],
                  "y_kernel": sym["y_fused"],
                  "x_variant_fwd": res["tiles"][3], "x_variant_inv": res["tiles"][4]},
        "finite": res["finite"],
    }
    try:
        extra["copy_GBps"] = copy_bandwidth() / 1e9
    except Exception as ex:  # measurement aid only
        extra["copy_GBps"] = None
        print("# copy bandwidth failed: %s" % ex, file=sys.stderr)
    if not args.no_fp64 and args.prec == "f32":
        print("# timing f64", file=sys.stderr, flush=True)
        s64 = max(2, args.steps // 2)
        r64 = run_gpu(args.workload, "f64", s64, 1, m_host)
        v64 = ncell * s64 / r64["wall_s"] / 1e6
        pb64, sb64 = pass_bytes(w["grid"], r64["L"], 8)
        extra["fp64"] = {"value": v64, "ms_per_step": r64["ev_ms"] / s64, "heff_ms": r64["heff_ms"],
                         "step_hbm_frac": sb64 / (r64["ev_ms"] / s64 * 1e-3) / HBM_PEAK,
                         "plan_setup_s": r64["setup_s"], "pass_ms": r64["passes"]}
        extra["fp32_over_fp64"] = value / v64
    if not args.no_fp64 and args.workload == "large":
        # the paper's own per-field measurement (FP64, each term alone, 350^3
        # cube), default padding; the paper's figure is another machine's
        print("# timing the per-field FP64 evaluations on a 350^3 cube", file=sys.stderr, flush=True)
        rf = run_fields("f64", 350, 10, 2, paddings=("auto",))
        extra["paper_fields_350_fp64"] = dict(rf["best"], paper=rf["paper"])
    if args.workload == "large":
        # the FP64 tensor setup alone (a plan without the autotuner's trials)
        for prec in ("f32", "f64"):
            extra.setdefault("tensor_setup_s", {})[prec] = tensor_setup_time(w, prec)
    if args.workload == "large" and not args.no_others:
        print("# the other workloads: thin film, sweep, gradient, small grid", file=sys.stderr, flush=True)
        extra["film"] = run_film_compare(100)
        extra["sweep"] = run_sweep(10, 3)
        extra["grad"] = run_grad("f32")
        rs = run_gpu("small", "f32", 200, 20, make_m(WORKLOADS["small"]))
        extra["small"] = {"ms_per_step": rs["ev_ms"] / 200, "Mcell_updates_per_s": 32 * 32 * 4 * 200 / rs["wall_s"] / 1e6}
    out = {
        "metric": METRIC, "value": value, "unit": "Mcell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["wall_s"] * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": w["name"], "grid": list(w["grid"]), "cell_m": list(w["cell"]), "cells": ncell,
                   "Ms": MS, "A": A, "alpha": ALPHA, "gamma": GAMMA, "dt": DT},
        "roofline": roof,
        "extra": extra,
    }
    if not args.no_cpu:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
