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
    hd = oracle.demag_direct(m, Ms, oct_, cells=cells)
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
    assert rel_l2(a.double().cpu().numpy() - m32, b.cpu().numpy() - m32) <= 1e-5


def test_large_grid_fp32_vs_fp64_and_sampled():
    import torch
    from paper_2606_01114_amd import DemagPlan
    n = (1024, 1024, 128)
    _say("large: inputs")
    m0 = rounded(synth.voronoi_grains(n, D, 3), torch.float32)
    # the benchmark's launch configuration: tile variants chosen by the autotuner
    p32 = DemagPlan(n, D, "f32", autotune=True)
    _say("large: fp32 tiles", p32.info()["tiles"])
    m = to_dev(m0, torch.float32)
    h32 = p32.h_eff(m, MS, A)
    hd32 = p32.h_eff(m, MS, A, terms=1)
    cells = synth.sample_cells(n, 3, 2)
    s32 = h32[cells[:, 0], cells[:, 1], cells[:, 2]].double().cpu().numpy()
    sd32 = hd32[cells[:, 0], cells[:, 1], cells[:, 2]].double().cpu().numpy()
    p32.llg_step(m, MS, A, ALPHA, GAMMA, DT)
    dm32 = (m.double() - to_dev(m0, torch.float64)).cpu()
    del m
    _say("large: fp64 plan")
    p64 = DemagPlan(n, D, "f64", autotune=True)
    m = to_dev(m0, torch.float64)
    def dev_rel(x, ref):       # relative L2 on the device, FP64 accumulation
        return float(torch.linalg.vector_norm(x.double() - ref) / torch.linalg.vector_norm(ref))
    h64 = p64.h_eff(m, MS, A)
    assert dev_rel(h32, h64) <= 1e-5
    del h64
    hd64 = p64.h_eff(m, MS, A, terms=1)
    assert dev_rel(hd32, hd64) <= 1e-5
    del hd64, h32, hd32
    # one RK4 step: the FP32 increment against the FP64 one
    p64.llg_step(m, MS, A, ALPHA, GAMMA, DT)
    dm64 = m - to_dev(m0, torch.float64)
    e_step = float(torch.linalg.vector_norm(dm32.to(dm64.device) - dm64) / torch.linalg.vector_norm(dm64))
    _say("large: step increment rel-L2", e_step)
    assert e_step <= 1e-5
    del m, dm64, dm32
    p64.close()
    torch.cuda.empty_cache()
    _say("large: oracle tensor and direct sums")
    oct_ = oracle.tensor_octant(n, D)
    rd, rx = _sampled_ref(m0, MS, oct_, cells)
    assert rel_l2(sd32, rd) <= 1e-5
    assert rel_l2(s32, rd + rx) <= 1e-5


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
    import torch
    from paper_2606_01114_amd import Batch, DemagPlan
    dt = torch.float32 if prec == "f32" else torch.float64
    grids = [g for g, _ in GEOMS]
    Ms = [ms for _, ms in GEOMS]
    b = Batch(grids, [D] * len(grids), prec, pow2_padding=pow2)
    m0 = [rounded(synth.random_unit(g, 40 + k), dt) for k, g in enumerate(grids)]
    ms = [to_dev(x, dt) for x in m0]
    hs = b.h_eff(ms, Ms, A)
    for k, g in enumerate(grids):
        oct_ = oracle.tensor_octant(g, D)
        L = tuple((_pow2_L if pow2 else oracle.default_L)(v) for v in g)
        ref = oracle.h_eff(m0[k], Ms[k], A, D, oct_, L)
        e = rel_l2(hs[k].cpu().numpy(), ref)
        assert e <= (1e-9 if prec == "f64" else 1e-5), (g, e)
        pl = DemagPlan(g, D, prec, L=L)
        single = pl.h_eff(ms[k], Ms[k], A)
        assert rel_l2(hs[k].cpu().numpy(), single.cpu().numpy()) <= (1e-14 if prec == "f64" else 1e-6)
    # one and two RK4 steps, graph and direct, against the oracle
    b.llg_step(ms, Ms, A, ALPHA, GAMMA, DT, n_steps=1)
    ms2 = [to_dev(x, dt) for x in m0]
    b.llg_step(ms2, Ms, A, ALPHA, GAMMA, DT, n_steps=1, graph=False)
    for k, g in enumerate(grids):
        assert torch.equal(ms[k], ms2[k])
        oct_ = oracle.tensor_octant(g, D)
        L = tuple((_pow2_L if pow2 else oracle.default_L)(v) for v in g)
        ref = oracle.rk4_step(m0[k], Ms[k], A, D, oct_, L, ALPHA, GAMMA, DT)
        e = rel_l2(ms[k].cpu().numpy() - m0[k], ref - m0[k])
        assert e <= (1e-9 if prec == "f64" else 1e-5), (g, e)


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
    m0 = [rounded(synth.random_unit(g, 60 + k), dt) for k, g in enumerate(grids)]
    ms = [to_dev(x, dt) for x in m0]
    hs = b.h_eff(ms, Ms, A)
    b.llg_step(ms, Ms, A, ALPHA, GAMMA, DT, n_steps=1)
    tol = 1e-9 if prec == "f64" else 1e-5
    for k, g in enumerate(grids):
        oct_ = oracle.tensor_octant(g, D)
        L = tuple(_pow2_L(v) for v in g)
        e = rel_l2(hs[k].cpu().numpy(), oracle.h_eff(m0[k], Ms[k], A, D, oct_, L))
        ref = oracle.rk4_step(m0[k], Ms[k], A, D, oct_, L, ALPHA, GAMMA, DT)
        es = rel_l2(ms[k].cpu().numpy() - m0[k], ref - m0[k])
        _say("batch wide", prec, g, L, e, es)
        assert e <= tol and es <= tol, (g, e, es)


def test_batch_sweep_64_geometries():
    import torch
    from paper_2606_01114_amd import Batch, DemagPlan
    geo = synth.batch_geometries(4)
    grids = [g for g, _ in geo]
    Ms = [ms for _, ms in geo]
    _say("sweep: plans")
    b = Batch(grids, [D] * len(grids), "f32")
    m0 = [rounded(synth.random_unit(g, 100 + k), torch.float32) for k, g in enumerate(grids)]
    ms = [to_dev(x, torch.float32) for x in m0]
    b.llg_step(ms, Ms, A, ALPHA, GAMMA, DT, n_steps=1)
    for k in (0, 17, 41, 63):
        pl = DemagPlan(grids[k], D, "f32")
        x = to_dev(m0[k], torch.float32)
        pl.llg_step(x, Ms[k], A, ALPHA, GAMMA, DT)
        assert rel_l2(ms[k].cpu().numpy() - m0[k], x.cpu().numpy() - m0[k]) <= 1e-5, k
    # the oracle on the smallest geometries of the sweep
    order = np.argsort([np.prod(g) for g in grids])[:3]
    hs = b.h_eff([to_dev(x, torch.float32) for x in m0], Ms, A)
    for k in order:
        g = grids[k]
        oct_ = oracle.tensor_octant(g, D)
        L = tuple(oracle.default_L(v) for v in g)
        ref = oracle.h_eff(m0[k], Ms[k], A, D, oct_, L)
        assert rel_l2(hs[k].cpu().numpy(), ref) <= 1e-5, g


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
    assert rel_l2(mT.detach().cpu().numpy() - m0, mref - m0) <= 1e-10
    assert rel_l2(Mst.grad.cpu().numpy(), gref) <= 1e-9


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
    points), with ragged last tiles, FP32 and FP64, against the oracle's
    h_eff."""
    import os
    import torch
    from paper_2606_01114_amd import DemagPlan
    cases = [((64, 500, 16), (("f32", 0, 1e-5), ("f32", 1, 1e-5), ("f32", 2, 1e-5), ("f64", 2, 1e-9))),
             ((400, 40, 3), (("f32", 3, 1e-5), ("f64", 3, 1e-9), ("f32", 2, 1e-5))),
             ((1024, 8, 2), (("f32", 3, 1e-5), ("f64", 3, 1e-9)))]
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


@pytest.mark.parametrize("n", [(2048, 6, 2), (6, 2048, 2), (3, 4, 1024), (1000, 5, 3)])
def test_longest_specialised_lengths(n):
    """The longest compile-time transforms (x and y length 4096, z length
    2048: x tiles of one or two columns, the 768-thread fused y pencil, the
    1024-point folded z line) and a long non-power-of-two x line (runtime
    planned), FP32 and FP64, h_eff and one RK4 step against the oracle."""
    import torch
    from paper_2606_01114_amd import DemagPlan
    oct_ = oracle.tensor_octant(n, D)
    L = tuple(oracle.default_L(v) for v in n)
    m0 = synth.random_unit(n, 23)
    Ms = synth.ms_field(n, 24)
    _say("long lengths", n, L)
    ref_h = oracle.h_eff(m0, Ms, A, D, oct_, L)
    ref_s = oracle.rk4_step(m0, Ms, A, D, oct_, L, ALPHA, GAMMA, DT)
    for prec, tol in (("f32", 1e-5), ("f64", 1e-9)):
        dt = torch.float32 if prec == "f32" else torch.float64
        if prec == "f64" and L[1] == 4096:
            # a 4096-long FP64 pencil of three components exceeds the LDS
            from paper_2606_01114_amd._lib import MM_ENOTSUP, MMError
            with pytest.raises(MMError) as ei:
                DemagPlan(n, D, prec, padding="smooth")
            assert ei.value.code == MM_ENOTSUP
            continue
        plan = DemagPlan(n, D, prec, padding="smooth")
        assert tuple(plan.info()["L"]) == L
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


@pytest.mark.parametrize("n", [(6, 128, 3), (5, 256, 2), (4, 512, 2), (3, 1024, 2)])
def test_y_pass_variants_against_oracle(n):
    """Both specialised y passes (the LDS-resident pencil and the
    register-resident one with half-line exchanges, selected with MMX_YVAR at
    plan creation) for every length the register-resident kernel has, FP32 and
    FP64, against the oracle's h_eff."""
    import os
    import torch
    from paper_2606_01114_amd import DemagPlan
    oct_ = oracle.tensor_octant(n, D)
    L = tuple(oracle.default_L(v) for v in n)
    m0 = synth.random_unit(n, 29)
    ref = oracle.h_eff(m0, MS, A, D, oct_, L)
    old = os.environ.get("MMX_YVAR")
    try:
        for var in (0, 1):
            os.environ["MMX_YVAR"] = str(var)
            for prec, tol in (("f32", 1e-5), ("f64", 1e-9)):
                dt = torch.float32 if prec == "f32" else torch.float64
                plan = DemagPlan(n, D, prec)
                assert (plan.info()["tiles"][2] < 0) == (var == 1)
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
