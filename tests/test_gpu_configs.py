"""GPU parity at the workload sizes: the thin film (512x512x16), the large
grid (1024x1024x128, 134M cells, in the launch configuration the benchmark
times), the batched sweep of uneven geometries, and the differentiable run
(256x256x8, 200 steps).  At full size the oracle is evaluated one sampled cell
at a time (direct sum + local exchange) and FP32 is also compared with the
GPU's FP64 mode over every cell."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rel_l2, rounded, to_dev

pytestmark = pytest.mark.gpu

MS, A, ALPHA, GAMMA, DT = 8e5, 1.3e-11, 0.02, 2.211e5, 1e-13
D = (2.5e-9, 2.5e-9, 3e-9)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sampled_ref(m, Ms, oct_, cells):
    hd = oracle.demag_direct_at(m, Ms, oct_, cells)
    hx = oracle.exchange_at(m, Ms, A, D, cells)
    return hd, hx


def test_film_step0_sampled_and_fp32_vs_fp64():
    import torch
    from paper_2606_01114_amd import DemagPlan
    n = (512, 512, 16)
    _say("film: oracle tensor")
    oct_ = oracle.tensor_octant(n, D)
    m0 = synth.smooth_film(n, D, 2)
    cells = synth.sample_cells(n, 2, 16)
    p64 = DemagPlan(n, D, "f64")
    p64.tensor_set(oct_)
    h64 = p64.h_eff(to_dev(m0, torch.float64), MS, A).cpu().numpy()[cells[:, 0], cells[:, 1], cells[:, 2]]
    hd64 = p64.h_eff(to_dev(m0, torch.float64), MS, A, terms=1).cpu().numpy()[cells[:, 0], cells[:, 1], cells[:, 2]]
    _say("film: direct sums")
    rd, rx = _sampled_ref(m0, MS, oct_, cells)
    assert rel_l2(hd64, rd) <= 1e-12
    assert rel_l2(h64, rd + rx) <= 1e-12
    p32 = DemagPlan(n, D, "f32")
    m32 = rounded(m0, torch.float32)
    rd32, rx32 = _sampled_ref(m32, MS, oct_, cells)
    full32 = p32.h_eff(to_dev(m32, torch.float32), MS, A)
    h32 = full32.cpu().numpy()[cells[:, 0], cells[:, 1], cells[:, 2]]
    hd32 = p32.h_eff(to_dev(m32, torch.float32), MS, A, terms=1).cpu().numpy()[cells[:, 0], cells[:, 1], cells[:, 2]]
    assert rel_l2(hd32, rd32) <= 1e-5
    assert rel_l2(h32, rd32 + rx32) <= 1e-5
    # every cell: FP32 against the GPU's FP64 mode on the same rounded input
    full64 = p64.h_eff(to_dev(m32, torch.float64), MS, A).cpu().numpy()
    assert rel_l2(full32.cpu().numpy(), full64) <= 1e-5
    # one RK4 step: the increment in FP32 against FP64
    a = to_dev(m32, torch.float32)
    b = to_dev(m32, torch.float64)
    p32.llg_step(a, MS, A, ALPHA, GAMMA, DT)
    p64.llg_step(b, MS, A, ALPHA, GAMMA, DT)
    e1 = rel_l2(a.double().cpu().numpy() - m32, b.cpu().numpy() - m32)
    assert e1 <= 1e-5
    # 100 steps (the workload's run): the FP32 trajectory against FP64,
    # reported (not a parity bar: the FP32 rounding of every step accumulates)
    p32.llg_step(a, MS, A, ALPHA, GAMMA, DT, n_steps=99)
    p64.llg_step(b, MS, A, ALPHA, GAMMA, DT, n_steps=99)
    e100 = rel_l2(a.double().cpu().numpy() - m32, b.cpu().numpy() - m32)
    _say("film: FP32 vs FP64 increment rel-L2 after 1 step %.3e, after 100 steps %.3e" % (e1, e100))
    assert e100 <= 1e-3


def test_large_grid_fp32_vs_fp64_and_sampled():
    """1024x1024x128 (Voronoi grains) in the benchmark's launch configuration
    (autotuned tiles): FP32 h_eff and demag field against the oracle's
    compensated direct sum plus local exchange at 16 seeded cells (1e-5);
    the FP64 mode with the oracle's tensor held equal against the same sums
    (1e-12); FP32 against the FP64 mode over every cell; the FP32 RK4 step
    increment against the FP64 one over every cell."""
    import torch
    from paper_2606_01114_amd import DemagPlan
    n = (1024, 1024, 128)
    _say("large: inputs and oracle tensor")
    m0 = rounded(synth.voronoi_grains(n, D, 3), torch.float32)
    oct_ = oracle.tensor_octant(n, D)
    cells = synth.sample_cells(n, 3, 16)
    ci = (cells[:, 0], cells[:, 1], cells[:, 2])
    _say("large: direct sums at", len(cells), "cells")
    rd = oracle.demag_direct_at(m0, MS, oct_, cells)
    rx = oracle.exchange_at(m0, MS, A, D, cells)
    p32 = DemagPlan(n, D, "f32", autotune=True)
    _say("large: fp32 tiles", p32.info()["tiles"])
    m = to_dev(m0, torch.float32)
    h32 = p32.h_eff(m, MS, A)
    hd32 = p32.h_eff(m, MS, A, terms=1)
    s32 = h32[ci].double().cpu().numpy()
    sd32 = hd32[ci].double().cpu().numpy()
    e_h32, e_d32 = rel_l2(s32, rd + rx), rel_l2(sd32, rd)
    _say("large: fp32 sampled rel-L2 h_eff %.3e demag %.3e" % (e_h32, e_d32))
    assert e_h32 <= 1e-5 and e_d32 <= 1e-5
    p32.llg_step(m, MS, A, ALPHA, GAMMA, DT)
    dm32 = (m.double() - to_dev(m0, torch.float64)).cpu()
    del m
    _say("large: fp64 plan, oracle tensor held")
    p64 = DemagPlan(n, D, "f64", autotune=True)
    p64.tensor_set(oct_)
    del oct_
    m = to_dev(m0, torch.float64)

    def dev_rel(x, ref):       # relative L2 on the device, FP64 accumulation
        return float(torch.linalg.vector_norm(x.double() - ref) / torch.linalg.vector_norm(ref))
    h64 = p64.h_eff(m, MS, A)
    e_h64 = rel_l2(h64[ci].cpu().numpy(), rd + rx)
    e_32_64 = dev_rel(h32, h64)
    del h64
    hd64 = p64.h_eff(m, MS, A, terms=1)
    e_d64 = rel_l2(hd64[ci].cpu().numpy(), rd)
    e_d32_64 = dev_rel(hd32, hd64)
    del hd64, h32, hd32
    _say("large: fp64 sampled rel-L2 h_eff %.3e demag %.3e; fp32 vs fp64 every cell %.3e / %.3e"
         % (e_h64, e_d64, e_32_64, e_d32_64))
    assert e_h64 <= 1e-12 and e_d64 <= 1e-12
    assert e_32_64 <= 1e-5 and e_d32_64 <= 1e-5
    # one RK4 step: the FP32 increment against the FP64 one
    p64.llg_step(m, MS, A, ALPHA, GAMMA, DT)
    dm64 = m - to_dev(m0, torch.float64)
    e_step = float(torch.linalg.vector_norm(dm32.to(dm64.device) - dm64) / torch.linalg.vector_norm(dm64))
    _say("large: step increment rel-L2", e_step)
    assert e_step <= 1e-5
    del m, dm64, dm32
    p64.close()
    p32.close()
    torch.cuda.empty_cache()


GEOMS = [((53, 20, 3), 6e5), ((48, 61, 1), 1.1e6), ((7, 9, 5), 4e5), ((32, 16, 8), 9e5), ((1, 24, 2), 7e5)]


def _pow2_L(n):
    """Smallest power of two >= 2n-1 (1 for a single cell)."""
    if n == 1:
        return 1
    L = 1
    while L < 2 * n - 1:
        L *= 2
    return L


@pytest.mark.parametrize("prec,pow2", [("f32", True), ("f64", True), ("f32", False), ("f64", False)])
def test_batch_against_oracle_and_plans(prec, pow2):
    """Five uneven geometries (power-of-two and 7-smooth padding): h_eff and
    one RK4 step (graph and direct launches) of each against the oracle --
    FP64 with every geometry's tensor held equal (1e-12), FP32 with the
    GPU's own tensors (1e-5) -- and against single plans of the same
    geometry."""
    import torch
    from paper_2606_01114_amd import Batch, DemagPlan
    dt = torch.float32 if prec == "f32" else torch.float64
    tol = 1e-12 if prec == "f64" else 1e-5
    grids = [g for g, _ in GEOMS]
    Ms = [ms for _, ms in GEOMS]
    octs = [oracle.tensor_octant(g, D) for g in grids]
    b = Batch(grids, [D] * len(grids), prec, pow2_padding=pow2)
    if prec == "f64":
        for k in range(len(grids)):
            b.tensor_set(k, octs[k])
    m0 = [rounded(synth.random_unit(g, 40 + k), dt) for k, g in enumerate(grids)]
    ms = [to_dev(x, dt) for x in m0]
    hs = b.h_eff(ms, Ms, A)
    for k, g in enumerate(grids):
        L = tuple((_pow2_L if pow2 else oracle.default_L)(v) for v in g)
        ref = oracle.h_eff(m0[k], Ms[k], A, D, octs[k], L)
        e = rel_l2(hs[k].cpu().numpy(), ref)
        _say("batch", prec, pow2, g, "h_eff rel-L2", e)
        assert e <= tol, (g, e)
        pl = DemagPlan(g, D, prec, L=L)
        if prec == "f64":
            pl.tensor_set(octs[k])
        single = pl.h_eff(ms[k], Ms[k], A)
        assert rel_l2(hs[k].cpu().numpy(), single.cpu().numpy()) <= (1e-14 if prec == "f64" else 1e-6)
    # one RK4 step, graph and direct, against the oracle
    b.llg_step(ms, Ms, A, ALPHA, GAMMA, DT, n_steps=1)
    ms2 = [to_dev(x, dt) for x in m0]
    b.llg_step(ms2, Ms, A, ALPHA, GAMMA, DT, n_steps=1, graph=False)
    for k, g in enumerate(grids):
        assert torch.equal(ms[k], ms2[k])
        L = tuple((_pow2_L if pow2 else oracle.default_L)(v) for v in g)
        ref = oracle.rk4_step(m0[k], Ms[k], A, D, octs[k], L, ALPHA, GAMMA, DT)
        e = rel_l2(ms[k].cpu().numpy() - m0[k], ref - m0[k])
        _say("batch", prec, pow2, g, "step rel-L2", e)
        assert e <= tol, (g, e)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_odd_radix_lengths_against_oracle(prec):
    """A batch padded to the compile-time lengths (padding="ct") whose axes
    take lengths with an odd radix on x, y and z (96, 160, 224, 320 and
    powers of two): the grouped x, fused y and z kernels at those lengths,
    h_eff and one RK4 step of every geometry against the oracle (FP64 with
    the tensors held equal, 1e-12; FP32 1e-5)."""
    import torch
    from paper_2606_01114_amd import Batch
    grids = [(45, 6, 48), (6, 70, 80), (100, 5, 10), (5, 110, 112), (150, 3, 4)]
    want = [(96, 16, 96), (16, 160, 160), (224, 16, 32), (16, 224, 224), (320, 8, 8)]
    Ms = [4e5 + 1.5e5 * k for k in range(len(grids))]
    dt = torch.float32 if prec == "f32" else torch.float64
    tol = 1e-12 if prec == "f64" else 1e-5
    octs = [oracle.tensor_octant(g, D) for g in grids]
    b = Batch(grids, [D] * len(grids), prec, padding="ct")
    lens = sorted({(g["pass"], g["L"]) for g in b.schedule()["groups"]})
    _say("batch odd lengths", prec, lens)
    for axis, key in ((0, "x_fwd"), (1, "y_fused"), (2, "z")):
        for w in want:
            if w[axis] & (w[axis] - 1):
                assert (key, w[axis]) in lens, (key, w[axis], lens)
    if prec == "f64":
        for k in range(len(grids)):
            b.tensor_set(k, octs[k])
    m0 = [rounded(synth.random_unit(g, 60 + k), dt) for k, g in enumerate(grids)]
    ms = [to_dev(x, dt) for x in m0]
    hs = b.h_eff(ms, Ms, A)
    for k, g in enumerate(grids):
        L = tuple(oracle.default_L(v) for v in g)
        ref = oracle.h_eff(m0[k], Ms[k], A, D, octs[k], L)
        e = rel_l2(hs[k].cpu().numpy(), ref)
        _say("batch odd", prec, g, "h_eff rel-L2", e)
        assert e <= tol, (g, e)
    b.llg_step(ms, Ms, A, ALPHA, GAMMA, DT, n_steps=1)
    for k, g in enumerate(grids):
        L = tuple(oracle.default_L(v) for v in g)
        ref = oracle.rk4_step(m0[k], Ms[k], A, D, octs[k], L, ALPHA, GAMMA, DT)
        e = rel_l2(ms[k].cpu().numpy() - m0[k], ref - m0[k])
        _say("batch odd", prec, g, "step rel-L2", e)
        assert e <= tol, (g, e)
    b.close()


def test_batch_groups_side_by_side_match_serial():
    """The launch groups of a pass run side by side on the batch's internal
    streams (parallel branches of the step's graph); the same batch with the
    groups one after the other (MMX_NO_FANOUT at creation) gives bit-identical
    fields and steps, through the graph and through direct launches, on 16
    uneven geometries of the sweep recipe (several groups per pass)."""
    import os
    import torch
    from paper_2606_01114_amd import Batch
    geo = synth.batch_geometries(4)[:16]
    grids = [g for g, _ in geo]
    Ms = [ms for _, ms in geo]
    m0 = [to_dev(rounded(synth.random_unit(g, 300 + k), torch.float32), torch.float32) for k, g in enumerate(grids)]
    outs = []
    old = os.environ.get("MMX_NO_FANOUT")
    try:
        for serial in (False, True):
            if serial:
                os.environ["MMX_NO_FANOUT"] = "1"
            else:
                os.environ.pop("MMX_NO_FANOUT", None)
            b = Batch(grids, [D] * len(grids), "f32", padding="ct")
            groups = b.schedule()["groups"]
            assert sum(g["pass"] == "x_fwd" for g in groups) >= 3, groups
            hs = [h.clone() for h in b.h_eff(m0, Ms, A)]
            ms = [x.clone() for x in m0]
            b.llg_step(ms, Ms, A, ALPHA, GAMMA, DT, n_steps=2)
            md = [x.clone() for x in m0]
            b.llg_step(md, Ms, A, ALPHA, GAMMA, DT, n_steps=2, graph=False)
            torch.cuda.synchronize()
            outs.append((hs, ms, md))
            b.close()
    finally:
        if old is None:
            os.environ.pop("MMX_NO_FANOUT", None)
        else:
            os.environ["MMX_NO_FANOUT"] = old
    for k in range(len(grids)):
        for part in range(3):
            assert torch.equal(outs[0][part][k], outs[1][part][k]), (k, part)
    _say("batch side by side: %d geometries bit-identical to the serial order" % len(grids))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_wide_x_tiles_against_oracle(prec):
    """A batch whose x lines are 2048 and 1024 points long runs the grouped
    half-LDS x kernel on wide tiles (and 64 points the full-LDS one): h_eff
    and one RK4 step of every geometry against the oracle."""
    import torch
    from paper_2606_01114_amd import Batch
    dt = torch.float32 if prec == "f32" else torch.float64
    geo = [((600, 4, 2), 8e5), ((300, 5, 3), 6e5), ((20, 6, 2), 1e6)]
    grids = [g for g, _ in geo]
    Ms = [ms for _, ms in geo]
    b = Batch(grids, [D] * len(grids), prec)
    octs = [oracle.tensor_octant(g, D) for g in grids]
    if prec == "f64":
        for k in range(len(grids)):
            b.tensor_set(k, octs[k])
    m0 = [rounded(synth.random_unit(g, 60 + k), dt) for k, g in enumerate(grids)]
    ms = [to_dev(x, dt) for x in m0]
    hs = b.h_eff(ms, Ms, A)
    b.llg_step(ms, Ms, A, ALPHA, GAMMA, DT, n_steps=1)
    tol = 1e-12 if prec == "f64" else 1e-5
    for k, g in enumerate(grids):
        oct_ = octs[k]
        L = tuple(_pow2_L(v) for v in g)
        e = rel_l2(hs[k].cpu().numpy(), oracle.h_eff(m0[k], Ms[k], A, D, oct_, L))
        ref = oracle.rk4_step(m0[k], Ms[k], A, D, oct_, L, ALPHA, GAMMA, DT)
        es = rel_l2(ms[k].cpu().numpy() - m0[k], ref - m0[k])
        _say("batch wide", prec, g, L, e, es)
        assert e <= tol and es <= tol, (g, e, es)


def test_batch_sweep_64_geometries():
    """The 64-geometry sweep (FP32, autotuned grouped launches, one graph per step):
    every geometry's h_eff against the oracle (1e-5), and one RK4 step of
    eight geometries spanning the size range against the oracle's step
    (increment, 1e-5)."""
    import torch
    from paper_2606_01114_amd import Batch
    from tests.gpu_util import oracle_field_and_step, oracle_pool_map
    geo = synth.batch_geometries(4)
    grids = [g for g, _ in geo]
    Ms = [ms for _, ms in geo]
    _say("sweep: plans (autotuned launch groups)")
    b = Batch(grids, [D] * len(grids), "f32", autotune="search")
    _say("sweep: schedule", [(g["pass"], g["L"], g["variant"]) for g in b.schedule()["groups"]])
    m0 = [rounded(synth.random_unit(g, 100 + k), torch.float32) for k, g in enumerate(grids)]
    hs = [h.cpu().numpy() for h in b.h_eff([to_dev(x, torch.float32) for x in m0], Ms, A)]
    ms = [to_dev(x, torch.float32) for x in m0]
    b.llg_step(ms, Ms, A, ALPHA, GAMMA, DT, n_steps=1)
    steps = [x.cpu().numpy() for x in ms]
    size_order = list(np.argsort([np.prod(g) for g in grids]))
    stepped = set(size_order[:: (len(size_order) - 1) // 7][:8]) | {size_order[-1]}
    _say("sweep: oracle over", len(grids), "geometries, steps of", sorted(int(k) for k in stepped))
    jobs = [(grids[k], D, m0[k], Ms[k], A, k in stepped, ALPHA, GAMMA, DT) for k in size_order[::-1]]
    refs = dict(zip(size_order[::-1], oracle_pool_map(oracle_field_and_step, jobs)))
    worst_h = worst_s = 0.0
    for k, g in enumerate(grids):
        rh, rs = refs[k]
        e = rel_l2(hs[k], rh)
        worst_h = max(worst_h, e)
        assert e <= 1e-5, (k, g, e)
        if rs is not None:
            es = rel_l2(steps[k] - m0[k], rs - m0[k])
            worst_s = max(worst_s, es)
            assert es <= 1e-5, (k, g, es)
    _say("sweep: worst h_eff rel-L2 %.3e, worst step rel-L2 %.3e (%d steps)" % (worst_h, worst_s, len(stepped)))
    assert len(stepped) >= 8


def test_gradient_small_against_oracle_adjoint():
    import torch
    from paper_2606_01114_amd import DemagPlan, llg_run_checkpointed
    n = (32, 32, 4)
    oct_ = oracle.tensor_octant(n, D)
    L = tuple(oracle.default_L(v) for v in n)
    plan = DemagPlan(n, D, "f64")
    plan.tensor_set(oct_)
    m0 = synth.smooth_film(n, D, 5)
    Ms = synth.ms_field(n, 5)
    steps = 20
    Mst = to_dev(Ms, torch.float64).requires_grad_(True)
    mT = llg_run_checkpointed(plan, to_dev(m0, torch.float64), Mst, A, ALPHA, GAMMA, DT, steps, every=6)
    loss = mT[..., 2].mean()
    loss.backward()
    gfin = np.zeros(n + (3,))
    gfin[..., 2] = 1.0 / np.prod(n)
    _, gref, mref = oracle.rk4_run_grad_Ms(m0, Ms, A, D, oct_, L, ALPHA, GAMMA, DT, steps, gfin)
    em = rel_l2(mT.detach().cpu().numpy() - m0, mref - m0)
    eg = rel_l2(Mst.grad.cpu().numpy(), gref)
    _say("20-step run rel-L2 %.3e, gradient rel-L2 %.3e" % (em, eg))
    assert em <= 1e-12 and eg <= 1e-12


def test_gradient_c5_against_fd():
    import torch
    from paper_2606_01114_amd import DemagPlan, llg_run_checkpointed
    n = (256, 256, 8)
    steps, every = 200, 20
    m0 = synth.smooth_film(n, D, 5)
    Ms = synth.ms_field(n, 5)
    cells = synth.sample_cells(n, 5, 16)
    p64 = DemagPlan(n, D, "f64")

    def loss64(Msx):
        m = to_dev(m0, torch.float64)
        p64.llg_step(m, to_dev(Msx, torch.float64), A, ALPHA, GAMMA, DT, n_steps=steps)
        return float(m[..., 2].mean())

    _say("c5: fd")
    fd = []
    for (i, j, k) in cells:
        e = 1e-3 * Ms[i, j, k]
        Mp, Mm = Ms.copy(), Ms.copy()
        Mp[i, j, k] += e
        Mm[i, j, k] -= e
        fd.append((loss64(Mp) - loss64(Mm)) / (2 * e))
    fd = np.array(fd)
    scale = np.abs(fd).max()
    for prec, tol in (("f64", 1e-5), ("f32", 1e-2)):
        _say("c5: adjoint", prec)
        dt = torch.float32 if prec == "f32" else torch.float64
        plan = p64 if prec == "f64" else DemagPlan(n, D, prec)
        Mst = to_dev(Ms, dt).requires_grad_(True)
        mT = llg_run_checkpointed(plan, to_dev(m0, dt), Mst, A, ALPHA, GAMMA, DT, steps, every=every)
        mT[..., 2].mean().backward()
        g = Mst.grad.double().cpu().numpy()[cells[:, 0], cells[:, 1], cells[:, 2]]
        err = np.abs(g - fd).max() / scale
        _say("c5", prec, "max err / max|g| = %.3e" % err)
        assert err <= tol, (prec, err)


def test_x_pass_variants_against_oracle():
    """Every variant of the specialised x pass, selected with MMX_XVAR at plan
    creation: two tile widths (0, 1), the half-LDS kernel (2) and the
    half-LDS kernel on tiles twice as wide (3, lines of 1024 and 2048
    points), with ragged last tiles, and both tile widths of the 640-point
    line with a radix-5 stage and the 768-point line with a radix-3 stage,
    FP32 (1e-5) and FP64 with the oracle's tensor held (1e-12), against the
    oracle's h_eff."""
    import os
    import torch
    from paper_2606_01114_amd import DemagPlan
    cases = [((64, 500, 16), (("f32", 0, 1e-5), ("f32", 1, 1e-5), ("f32", 2, 1e-5), ("f64", 2, 1e-12))),
             ((300, 40, 3), (("f32", 0, 1e-5), ("f32", 1, 1e-5), ("f64", 0, 1e-12), ("f64", 1, 1e-12))),
             ((350, 40, 3), (("f32", 0, 1e-5), ("f32", 1, 1e-5), ("f64", 1, 1e-12))),
             ((480, 40, 3), (("f32", 3, 1e-5), ("f64", 3, 1e-12), ("f32", 2, 1e-5))),
             ((1024, 8, 2), (("f32", 3, 1e-5), ("f64", 3, 1e-12)))]
    old = os.environ.get("MMX_XVAR")
    try:
        for n, runs in cases:
            oct_ = oracle.tensor_octant(n, D)
            m0 = synth.random_unit(n, 17)
            ref = None
            for prec, var, tol in runs:
                os.environ["MMX_XVAR"] = str(var)
                dt = torch.float32 if prec == "f32" else torch.float64
                plan = DemagPlan(n, D, prec)
                if prec == "f64":
                    plan.tensor_set(oct_)
                info = plan.info()
                L = tuple(info["L"])
                if ref is None:
                    _say("x variants: oracle h_eff", n, L)
                    ref = oracle.h_eff(m0, MS, A, D, oct_, L)
                assert info["tiles"][3] == var and info["tiles"][4] == var, info["tiles"]
                h = plan.h_eff(to_dev(rounded(m0, dt), dt), MS, A)
                e = rel_l2(h.cpu().numpy(), ref)
                _say("x variant", n, prec, var, "W", info["tiles"][1], "rel-L2", e)
                assert e <= tol, (n, prec, var, e)
                plan.close()
    finally:
        if old is None:
            os.environ.pop("MMX_XVAR", None)
        else:
            os.environ["MMX_XVAR"] = old


@pytest.mark.parametrize("n,Lset", [((2048, 6, 2), None), ((6, 2048, 2), None), ((3, 4, 1024), None),
                                    ((1000, 5, 3), None), ((700, 5, 3), (1536, 16, 8)), ((6, 350, 2), (16, 768, 4)),
                                    ((4, 3, 350), (8, 8, 768)), ((150, 180, 3), (384, 384, 8)),
                                    ((150, 180, 3), (320, 448, 8)), ((300, 420, 2), (640, 896, 4)),
                                    ((600, 5, 3), (1280, 16, 8)), ((6, 800, 2), (16, 1792, 4)),
                                    ((800, 6, 2), (1792, 16, 4)), ((45, 70, 3), (96, 160, 8)),
                                    ((90, 100, 3), (192, 224, 8)), ((5, 4, 45), (16, 8, 96)),
                                    ((6, 3, 80), (16, 8, 160)), ((4, 4, 95), (8, 8, 192)),
                                    ((4, 3, 100), (8, 8, 224)), ((4, 5, 160), (8, 16, 320)),
                                    ((4, 4, 220), (8, 8, 448)), ((4, 4, 300), (8, 8, 640)),
                                    ((3, 4, 400), (8, 8, 896))])
def test_longest_specialised_lengths(n, Lset):
    """The longest compile-time transforms (x and y length 4096, z length
    2048: x tiles of one or two columns, the 768-thread fused y pencil, the
    1024-point folded z line), the compile-time lengths with one odd radix
    (radix 3: x 1536, y 768, z 768 folded to 384, x and y 384, 96, 192;
    radix 5: 160, 320, 640, 1280; radix 7: 224, 448, 896, 1792 on x and y;
    z 96 ... 896, folded to half that length)
    and a long non-power-of-two x line (runtime planned), FP32 (1e-5) and
    FP64 with the oracle's tensor held (1e-12), h_eff and one RK4 step
    against the oracle."""
    import torch
    from paper_2606_01114_amd import DemagPlan
    oct_ = oracle.tensor_octant(n, D)
    L = tuple(Lset) if Lset else tuple(oracle.default_L(v) for v in n)
    m0 = synth.random_unit(n, 23)
    Ms = synth.ms_field(n, 24)
    _say("long lengths", n, L)
    ref_h = oracle.h_eff(m0, Ms, A, D, oct_, L)
    ref_s = oracle.rk4_step(m0, Ms, A, D, oct_, L, ALPHA, GAMMA, DT)
    for prec, tol in (("f32", 1e-5), ("f64", 1e-12)):
        dt = torch.float32 if prec == "f32" else torch.float64
        plan = DemagPlan(n, D, prec, padding="smooth", L=Lset)
        if prec == "f64":
            plan.tensor_set(oct_)
        assert tuple(plan.info()["L"]) == L
        if prec == "f64" and L[1] == 4096:
            # a 4096-long FP64 pencil of three components exceeds the LDS:
            # it runs as two half-spectra of 2048 points (y variant 6), and a
            # batch, whose grouped kernels hold the whole pencil, refuses it
            assert plan.info()["tiles"][2] == 6
            from paper_2606_01114_amd import Batch
            from paper_2606_01114_amd._lib import MM_ENOTSUP, MMError
            with pytest.raises(MMError) as ei:
                Batch([n], [D], prec)
            assert ei.value.code == MM_ENOTSUP
        if Lset:
            # the lengths with an odd radix run the compile-time kernels
            sch = plan.schedule()
            for key, Lv in (("x_fwd", L[0]), ("y_fused", L[1]), ("z", L[2])):
                if Lv & (Lv - 1):
                    assert sch[key]["specialised"], (key, sch)
        mr = rounded(m0, dt)
        Msr = to_dev(rounded(Ms, dt), dt)
        h = plan.h_eff(to_dev(mr, dt), Msr, A)
        e = rel_l2(h.cpu().numpy(), ref_h)
        _say("  ", prec, "h_eff rel-L2", e)
        assert e <= tol, (prec, e)
        m = to_dev(mr, dt)
        plan.llg_step(m, Msr, A, ALPHA, GAMMA, DT)
        e = rel_l2(m.cpu().numpy() - m0, ref_s - m0)
        _say("  ", prec, "step rel-L2", e)
        assert e <= tol, (prec, e)
        plan.close()


@pytest.mark.parametrize("n", [(6, 128, 3), (5, 256, 2), (4, 512, 2), (3, 1024, 2), (40, 600, 6), (200, 512, 8),
                               (2, 2048, 2)])
def test_y_pass_variants_against_oracle(n):
    """Every specialised y pass, selected with MMX_YVAR at plan creation: the
    LDS-resident pencil (0), the register-resident one with half-line
    exchanges (1), the LDS-resident pencil with rotated waves (2), the
    persistent kernel with the next pencil's loads in flight (3; 4: held to
    three waves per SIMD; 5: with its twiddles from a root table in LDS) and
    the pencil split into its even and odd half-spectra (6), for every
    length each has (a variant a length lacks leaves the default in place),
    FP32 (1e-5) and FP64 with the oracle's tensor held (1e-12), against the
    oracle's h_eff; the persistent kernel's grid walks more pencils than it
    has workgroups."""
    import os
    import torch
    from paper_2606_01114_amd import DemagPlan
    oct_ = oracle.tensor_octant(n, D)
    L = tuple(oracle.default_L(v) for v in n)
    m0 = synth.random_unit(n, 29)
    ref = oracle.h_eff(m0, MS, A, D, oct_, L)
    old = os.environ.get("MMX_YVAR")
    try:
        for var in (0, 1, 2, 3, 4, 5, 6):
            os.environ["MMX_YVAR"] = str(var)
            for prec, tol in (("f32", 1e-5), ("f64", 1e-12)):
                dt = torch.float32 if prec == "f32" else torch.float64
                plan = DemagPlan(n, D, prec)
                if prec == "f64":
                    plan.tensor_set(oct_)
                Ly = plan.info()["L"][1]
                has = {0: Ly & (Ly - 1) == 0, 1: Ly in (256, 512, 1024, 2048), 2: Ly in (512, 1024, 2048, 4096),
                       3: Ly in (1024, 2048), 4: Ly == 2048, 5: Ly in (1024, 2048), 6: Ly in (1024, 2048, 4096)}[var]
                # a whole 4096-point FP64 pencil exceeds the LDS: only the
                # half-spectrum kernel runs it
                full = not (prec == "f64" and Ly == 4096)
                has = has and (full or var == 6)
                yv = plan.info()["tiles"][2]
                assert yv == (var if has else (0 if full else 6)), (var, Ly, yv)
                h = plan.h_eff(to_dev(rounded(m0, dt), dt), MS, A)
                e = rel_l2(h.cpu().numpy(), ref)
                _say("y variant", var, prec, n, e)
                assert e <= tol, (var, prec, e)
                plan.close()
    finally:
        if old is None:
            os.environ.pop("MMX_YVAR", None)
        else:
            os.environ["MMX_YVAR"] = old


def _factors(L):
    """The library's default radix list of a 7-smooth length: radix-16 stages
    with an 8/4/2 tail for the power of two, then 3s, 5s and 7s."""
    r, p2 = [], 0
    while L % 2 == 0:
        L //= 2
        p2 += 1
    if p2 == 1:
        r.append(2)
    elif p2 > 1:
        a, rem = divmod(p2, 4)
        if rem == 1 and a >= 1:
            r += [16] * (a - 1) + [8, 4]
        else:
            r += [16] * a + {3: [8], 2: [4], 1: [2], 0: []}[rem]
    for q in (3, 5, 7):
        while L % q == 0:
            L //= q
            r.append(q)
    return r


def test_radix_orders_against_oracle():
    """Runtime-planned transforms in every radix order (MMX_ORDER): all 12
    orders of the 90-point y line (2,3,3,5) and both orders of the 14-point x
    and 10-point z lines, FP32 (1e-5) and FP64 with the oracle's tensor held
    (1e-12), h_eff against the oracle; then a plan
    that searches the orders itself (autotune "search") reports permutations
    of each length's radices and matches the oracle too."""
    import itertools
    import os
    import torch
    from paper_2606_01114_amd import DemagPlan
    n = (7, 45, 5)
    oct_ = oracle.tensor_octant(n, D)
    m0 = synth.random_unit(n, 31)
    ref = None
    old = os.environ.get("MMX_ORDER")
    try:
        orders = sorted(set(itertools.permutations(_factors(90))))
        assert len(orders) == 12
        runs = [("y", o) for o in orders] + [("x", (7, 2)), ("z", (5, 2))]
        for ax, o in runs:
            os.environ["MMX_ORDER"] = "%s:%s" % (ax, ",".join(map(str, o)))
            for prec, tol in (("f32", 1e-5), ("f64", 1e-12)):
                dt = torch.float32 if prec == "f32" else torch.float64
                plan = DemagPlan(n, D, prec, padding="smooth")
                if prec == "f64":
                    plan.tensor_set(oct_)
                L = plan.info()["L"]
                if ref is None:
                    assert L == (14, 90, 10), L
                    ref = oracle.h_eff(m0, MS, A, D, oct_, L)
                got = plan.schedule()["radix_order"][ax]
                assert got == ",".join(map(str, o)), (got, o)
                e = rel_l2(plan.h_eff(to_dev(rounded(m0, dt), dt), MS, A).cpu().numpy(), ref)
                _say("radix order", ax, o, prec, e)
                assert e <= tol, (ax, o, prec, e)
                plan.close()
    finally:
        if old is None:
            os.environ.pop("MMX_ORDER", None)
        else:
            os.environ["MMX_ORDER"] = old
    for prec, tol in (("f32", 1e-5), ("f64", 1e-12)):
        dt = torch.float32 if prec == "f32" else torch.float64
        plan = DemagPlan(n, D, prec, padding="smooth", autotune="search")
        if prec == "f64":
            plan.tensor_set(oct_)
        sch = plan.schedule()
        for ax, Lv in zip("xyz", (14, 90, 10)):
            assert sorted(int(v) for v in sch["radix_order"][ax].split(",")) == sorted(_factors(Lv)), sch
        e = rel_l2(plan.h_eff(to_dev(rounded(m0, dt), dt), MS, A).cpu().numpy(), ref)
        _say("searched radix orders", prec, sch["radix_order"], e)
        assert e <= tol
        plan.close()


@pytest.mark.parametrize("xv,yv", [(0, 0), (1, 1), (2, 2), (3, 0)])
def test_batch_kernel_variants_against_oracle(xv, yv):
    """Every grouped kernel variant (MMX_XVAR / MMX_YVAR at batch creation:
    both x tile widths, the half-LDS and wide half-LDS x kernels; the
    LDS-resident, register-resident and wave-rotated fused y kernels) over
    geometries with x lines of 2048, 1024 and 256 points and y lines of 128
    to 1024 points, FP32 (1e-5) and FP64 with the oracle's tensors held
    (1e-12), h_eff against the oracle."""
    import os
    import torch
    from paper_2606_01114_amd import Batch
    geo = [((600, 4, 2), 8e5), ((300, 5, 3), 6e5), ((100, 40, 3), 1e6), ((20, 300, 2), 7e5)]
    grids = [g for g, _ in geo]
    Ms = [ms for _, ms in geo]
    octs = [oracle.tensor_octant(g, D) for g in grids]
    m0 = [synth.random_unit(g, 80 + k) for k, g in enumerate(grids)]
    refs = [oracle.h_eff(m0[k], Ms[k], A, D, octs[k], tuple(_pow2_L(v) for v in g)) for k, g in enumerate(grids)]
    saved = {k: os.environ.get(k) for k in ("MMX_XVAR", "MMX_YVAR")}
    try:
        os.environ["MMX_XVAR"], os.environ["MMX_YVAR"] = str(xv), str(yv)
        for prec, tol in (("f32", 1e-5), ("f64", 1e-12)):
            dt = torch.float32 if prec == "f32" else torch.float64
            b = Batch(grids, [D] * len(grids), prec)
            if prec == "f64":
                for k in range(len(grids)):
                    b.tensor_set(k, octs[k])
            sch = b.schedule()["groups"]
            xs = {g["variant"] for g in sch if g["pass"] in ("x_fwd", "x_inv") and g["specialised"]}
            _say("batch variants", xv, yv, prec, [(g["pass"], g["L"], g["variant"], g["W"]) for g in sch])
            hs = b.h_eff([to_dev(rounded(x, dt), dt) for x in m0], Ms, A)
            for k, g in enumerate(grids):
                e = rel_l2(hs[k].cpu().numpy(), refs[k])
                assert e <= tol, (xv, yv, prec, g, e)
            assert xv in xs or xv == 3, xs
            b.close()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_batch_autotune_cache_roundtrip(tmp_path):
    """A batch created with autotune "search" records a winner per launch
    group in the schedule cache file; a second batch in "cached" mode reads
    the same schedule back (no timing), and both match the oracle."""
    import os
    import torch
    from paper_2606_01114_amd import Batch
    geo = [((300, 5, 3), 6e5), ((100, 40, 3), 1e6), ((20, 300, 2), 7e5)]
    grids = [g for g, _ in geo]
    Ms = [ms for _, ms in geo]
    octs = [oracle.tensor_octant(g, D) for g in grids]
    m0 = [synth.random_unit(g, 90 + k) for k, g in enumerate(grids)]
    cache = tmp_path / "schedules.tsv"
    old = os.environ.get("MMX_AUTOTUNE_CACHE")
    os.environ["MMX_AUTOTUNE_CACHE"] = str(cache)
    try:
        b1 = Batch(grids, [D] * len(grids), "f32", autotune="search")
        s1 = b1.schedule()
        b2 = Batch(grids, [D] * len(grids), "f32", autotune="cached")
        s2 = b2.schedule()
    finally:
        if old is None:
            os.environ.pop("MMX_AUTOTUNE_CACHE", None)
        else:
            os.environ["MMX_AUTOTUNE_CACHE"] = old
    _say("tuned schedule", s1)
    assert s1 == s2
    lines = cache.read_text().splitlines()
    assert any("batch_x_fwd" in ln for ln in lines) and any("batch_y_fused" in ln for ln in lines), lines
    for b in (b1, b2):
        hs = b.h_eff([to_dev(rounded(x, torch.float32), torch.float32) for x in m0], Ms, A)
        for k, g in enumerate(grids):
            ref = oracle.h_eff(m0[k], Ms[k], A, D, octs[k], tuple(_pow2_L(v) for v in g))
            assert rel_l2(hs[k].cpu().numpy(), ref) <= 1e-5
        b.close()
