"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars: FP64 within 1e-12 relative L2 with the demag tensor held equal (the
oracle's real-space octant is loaded with mm_demag_tensor_set and transformed
by the GPU); FP32 within 1e-5 relative L2 against the FP64 oracle with the
GPU's own tensor, for the full field and for the demag part alone.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rel_l2, rounded, to_dev

pytestmark = pytest.mark.gpu

MS, A = 8e5, 1.3e-11
GAMMA, ALPHA = 2.211e5, 0.02


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _plan(n, d, prec, L=None, hold=None, P=16.0):
    import torch
    from paper_2606_01114_amd import DemagPlan
    plan = DemagPlan(n, d, prec, L=L, far_radius=P)
    if hold is not None:
        plan.tensor_set(hold)
    dt = torch.float32 if prec == "f32" else torch.float64
    return plan, dt


CASES = [  # (grid, cell, L override)
    ((4, 4, 2), (2e-9, 2e-9, 2e-9), None),
    ((32, 32, 4), (2e-9, 2e-9, 2e-9), None),
    ((7, 5, 3), (2.5e-9, 2e-9, 3e-9), (14, 9, 5)),
    ((9, 6, 1), (2.5e-9, 2.5e-9, 3e-9), (18, 12, 1)),
    ((1, 6, 5), (2e-9, 2e-9, 1e-9), None),
    ((5, 1, 4), (2e-9, 2e-9, 1e-9), (9, 1, 7)),
    ((53, 20, 3), (2.5e-9, 2.5e-9, 3e-9), None),
    ((1, 1, 1), (2e-9, 2e-9, 2e-9), None),
]


@pytest.mark.parametrize("grid,cell,L", CASES)
def test_h_eff_fp64_tensor_held_equal(grid, cell, L):
    _say("case", grid, cell, L)
    oct_ = oracle.tensor_octant(grid, cell)
    plan, dt = _plan(grid, cell, "f64", L=L, hold=oct_)
    Lp = plan.info()["L"]
    m0 = synth.random_unit(grid, 1)
    Msv = synth.ms_field(grid, 2)
    for Ms in (MS, Msv):
        m = to_dev(m0, dt)
        Msd = to_dev(Ms, dt) if isinstance(Ms, np.ndarray) else Ms
        for terms, dm, ex in ((3, True, True), (1, True, False), (2, False, True)):
            h = plan.h_eff(m, Msd, A, terms=terms).cpu().numpy()
            ref = oracle.h_eff(m0, Ms, A, cell, oct_, Lp, demag=dm, exchange=ex)
            if np.linalg.norm(ref) == 0:
                assert np.abs(h).max() == 0
                continue
            e = rel_l2(h, ref)
            assert e <= 1e-12, (terms, e)


@pytest.mark.parametrize("grid,cell,L", CASES[:4] + CASES[6:7])
def test_h_eff_fp32_against_oracle(grid, cell, L):
    _say("case", grid, cell, L)
    oct_ = oracle.tensor_octant(grid, cell)
    plan, dt = _plan(grid, cell, "f32", L=L)
    Lp = plan.info()["L"]
    m0 = rounded(synth.random_unit(grid, 1), dt)
    m = to_dev(m0, dt)
    h = plan.h_eff(m, MS, A).cpu().numpy()
    assert rel_l2(h, oracle.h_eff(m0, MS, A, cell, oct_, Lp)) <= 1e-5
    hd = plan.h_eff(m, MS, A, terms=1).cpu().numpy()
    assert rel_l2(hd, oracle.demag_fft(m0, MS, oct_, Lp)) <= 1e-5


def test_direct_sum_brute_force_4x4x2():
    grid, cell = (4, 4, 2), (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant(grid, cell)
    m0 = synth.random_unit(grid, 11)
    ref = oracle.demag_direct(m0, MS, oct_)
    plan, dt = _plan(grid, cell, "f64", hold=oct_)
    h = plan.h_eff(to_dev(m0, dt), MS, A, terms=1).cpu().numpy()
    assert rel_l2(h, ref) <= 1e-12
    plan32, dt32 = _plan(grid, cell, "f32")
    m32 = rounded(m0, dt32)
    h32 = plan32.h_eff(to_dev(m32, dt32), MS, A, terms=1).cpu().numpy()
    assert rel_l2(h32, oracle.demag_direct(m32, MS, oct_)) <= 1e-5


@pytest.mark.parametrize("grid,cell", [((32, 32, 4), (2e-9, 2e-9, 2e-9)), ((20, 12, 6), (2.5e-9, 2.5e-9, 3e-9)),
                                       ((40, 3, 2), (1e-9, 3e-9, 0.5e-9))])
def test_gpu_tensor_octant_and_spectrum(grid, cell):
    oct_ = oracle.tensor_octant(grid, cell)
    plan, _ = _plan(grid, cell, "f64")
    g = plan.tensor_get()
    # near field: FP64 Newell loses digits to cancellation; bound each entry by
    # the cancellation scale sum|w f|/(4 pi V) of its stencil
    dmax = max(cell)
    for idx in np.ndindex(*grid):
        r = np.sqrt(sum((idx[a] * cell[a]) ** 2 for a in range(3)))
        if r <= 16 * dmax:
            sc = oracle.newell_scale_at(*idx, cell)
            assert np.all(np.abs(g[idx] - oct_[idx]) <= 64 * 2.2e-16 * sc + 1e-300), idx
    far = np.array([np.sqrt(sum((i[a] * cell[a]) ** 2 for a in range(3))) > 16 * dmax for i in np.ndindex(*grid)]).reshape(grid)
    if far.any():
        d = np.abs(g[far] - oct_[far]).max() / np.abs(oct_[far]).max()
        assert d <= 1e-14
    # spectrum of the held tensor vs the oracle's DFT of the wrapped octant
    plan.tensor_set(oct_)
    L = plan.info()["L"]
    S = plan.spectrum_get()
    ref = oracle.tensor_spectrum(oct_, L).real
    h = [v // 2 + 1 for v in L]
    ref = ref[:, :h[0], :h[1], :h[2]]
    ref = np.moveaxis(ref, 0, -1) * (-1.0 / np.prod(L))
    assert np.abs(S - ref).max() <= 1e-14 * np.abs(ref).max()


def test_energies():
    grid, cell = (20, 12, 6), (2.5e-9, 2.5e-9, 3e-9)
    oct_ = oracle.tensor_octant(grid, cell)
    plan, dt = _plan(grid, cell, "f64", hold=oct_)
    L = plan.info()["L"]
    m0 = synth.random_unit(grid, 3)
    Ms = synth.ms_field(grid, 4)
    _, (ed, ex) = plan.h_eff(to_dev(m0, dt), to_dev(Ms, dt), A, energy=True)
    hd = oracle.demag_fft(m0, Ms, oct_, L)
    hx = oracle.exchange_field(m0, Ms, A, cell)
    red, rex = oracle.energies(m0, Ms, hd, hx, cell)
    assert abs(ed - red) <= 1e-12 * abs(red) and abs(ex - rex) <= 1e-12 * abs(rex)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_llg_step_increment(prec):
    grid, cell = (32, 32, 4), (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant(grid, cell)
    plan, dt = _plan(grid, cell, prec, hold=oct_ if prec == "f64" else None)
    L = plan.info()["L"]
    m0 = rounded(synth.random_unit(grid, 1), dt)
    Msv = rounded(synth.ms_field(grid, 2), dt)
    for Ms, hext in ((MS, None), (Msv, (1e4, -2e4, 3e4))):
        m = to_dev(m0, dt)
        Msd = to_dev(Ms, dt) if isinstance(Ms, np.ndarray) else Ms
        plan.llg_step(m, Msd, A, ALPHA, GAMMA, 1e-13, n_steps=2, h_ext=hext)
        ref = oracle.rk4_run(m0, 2, Ms, A, cell, oct_, L, ALPHA, GAMMA, 1e-13, h_ext=hext)
        e = rel_l2(m.cpu().numpy() - m0, ref - m0)
        _say("llg step", prec, "rel-L2", e)
        assert e <= (1e-12 if prec == "f64" else 1e-5), e


def test_llg_no_renorm_and_graph_equivalence():
    import torch
    grid, cell = (16, 10, 3), (2.5e-9, 2.5e-9, 3e-9)
    oct_ = oracle.tensor_octant(grid, cell)
    plan, dt = _plan(grid, cell, "f64", hold=oct_)
    L = plan.info()["L"]
    m0 = synth.random_unit(grid, 5)
    a = to_dev(m0, dt)
    b = to_dev(m0, dt)
    plan.llg_step(a, MS, A, ALPHA, GAMMA, 1e-13, n_steps=3, renorm=False)
    plan.llg_step(b, MS, A, ALPHA, GAMMA, 1e-13, n_steps=3, renorm=False, graph=False)
    assert torch.equal(a, b)
    ref = oracle.rk4_run(m0, 3, MS, A, cell, oct_, L, ALPHA, GAMMA, 1e-13, renorm=False)
    e = rel_l2(a.cpu().numpy() - m0, ref - m0)
    _say("no-renorm rel-L2", e)
    assert e <= 1e-12


def test_macrospin_closed_form():
    grid, cell = (1, 1, 1), (2e-9, 2e-9, 2e-9)
    plan, dt = _plan(grid, cell, "f64")
    th0, ph0, H, alpha = 1.0, 0.3, 2e5, 0.1
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)]).reshape(1, 1, 1, 3)
    m = to_dev(m0, dt)
    plan.llg_step(m, MS, A, alpha, GAMMA, 1e-13, n_steps=400, h_ext=(0, 0, H))
    ref = oracle.macrospin_closed_form(th0, ph0, H, alpha, GAMMA, 400e-13)
    assert np.abs(m.cpu().numpy().reshape(3) - ref).max() < 1e-10


def test_determinism():
    import torch
    grid, cell = (32, 32, 4), (2e-9, 2e-9, 2e-9)
    plan, dt = _plan(grid, cell, "f32")
    m0 = synth.random_unit(grid, 1)
    m = to_dev(m0, dt)
    h1 = plan.h_eff(m, MS, A)
    h2 = plan.h_eff(m, MS, A)
    assert torch.equal(h1, h2)
    a, b = to_dev(m0, dt), to_dev(m0, dt)
    plan.llg_step(a, MS, A, ALPHA, GAMMA, 1e-13, n_steps=2)
    plan.llg_step(b, MS, A, ALPHA, GAMMA, 1e-13, n_steps=2)
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec,vacuum", [("f64", False), ("f32", False), ("f64", True), ("f32", True)])
def test_h_eff_adjoint(prec, vacuum):
    """VJP of h_eff against the oracle's, with per-cell Ms and (vacuum=True)
    every seventh cell empty: vacuum neighbours carry no exchange weight and a
    vacuum cell's Ms cotangent has the demag part only."""
    grid, cell = (12, 10, 3), (2.5e-9, 2.5e-9, 3e-9)
    oct_ = oracle.tensor_octant(grid, cell)
    plan, dt = _plan(grid, cell, prec, hold=oct_ if prec == "f64" else None)
    L = plan.info()["L"]
    m0 = rounded(synth.random_unit(grid, 1), dt)
    Ms = synth.ms_field(grid, 5)
    if vacuum:
        Ms.reshape(-1)[::7] = 0.0
    Ms = rounded(Ms, dt)
    g = rounded(synth.random_unit(grid, 3), dt)
    gm, gMs = plan.h_eff_adjoint(to_dev(m0, dt), to_dev(Ms, dt), A, to_dev(g, dt))
    rm, rMs = oracle.h_eff_vjp(m0, Ms, A, cell, oct_, L, g)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert rel_l2(gm.cpu().numpy(), rm) <= tol
    assert rel_l2(gMs.cpu().numpy(), rMs) <= tol


def test_llg_step_adjoint_fp64():
    grid, cell = (12, 10, 3), (2.5e-9, 2.5e-9, 3e-9)
    oct_ = oracle.tensor_octant(grid, cell)
    plan, dt = _plan(grid, cell, "f64", hold=oct_)
    L = plan.info()["L"]
    m0 = synth.smooth_film(grid, cell, 5)
    Ms = synth.ms_field(grid, 5)
    g0 = synth.random_unit(grid, 7)
    g = to_dev(g0, dt)
    import torch
    gMs = torch.zeros(grid, dtype=dt, device="cuda")
    plan.llg_step_adjoint(to_dev(m0, dt), to_dev(Ms, dt), A, ALPHA, GAMMA, 1e-13, g, gMs)
    rm, rMs = oracle.rk4_step_vjp(m0, Ms, A, cell, oct_, L, ALPHA, GAMMA, 1e-13, g0)
    em, eMs = rel_l2(g.cpu().numpy(), rm), rel_l2(gMs.cpu().numpy(), rMs)
    _say("llg_step_adjoint rel-L2 g_m %.3e g_Ms %.3e" % (em, eMs))
    assert em <= 1e-12 and eMs <= 1e-12


def test_attached_memory_same_results():
    """After mm_plan_attach_memory and mm_plan_attach_scratch the plan runs on
    torch-owned buffers of the sizes mm_plan_bytes and mm_plan_scratch_bytes
    report and gives bit-identical h_eff, RK4 steps, RKF45 step, minimiser
    iterates and adjoints; the plan's own device memory drops to zero and
    stays there; a second attach is refused; an attached plan without
    scratch refuses the calls that need it (no hidden allocation);
    non-finite input energies report MM_ENONFINITE."""
    import torch
    from paper_2606_01114_amd import DemagPlan, plan_bytes, plan_scratch_bytes
    from paper_2606_01114_amd._lib import MM_ENONFINITE, MM_ESTATE, MMError
    n, d = (48, 40, 6), (2.5e-9, 2.5e-9, 3e-9)
    hz = (2e3, -1e3, 5e2)

    def run_all(plan, m0, dt):
        h = plan.h_eff(m0, MS, A)
        s = m0.clone()
        plan.llg_step(s, MS, A, ALPHA, GAMMA, 1e-13, n_steps=2)
        r = m0.clone()
        ok, err, _ = plan.rkf45_step(r, MS, A, ALPHA, GAMMA, 2e-14, 1e-2)
        b = m0.clone()
        plan.minimize(b, MS, A, tol=0.0, max_iter=3, h_ext=hz)
        gm, gMs = plan.h_eff_adjoint(m0, to_dev(np.full(n, MS), dt), A, h)
        g = h.clone()
        gMs2 = torch.zeros(n, dtype=dt, device="cuda")
        plan.llg_step_adjoint(m0, to_dev(np.full(n, MS), dt), A, ALPHA, GAMMA, 1e-13, g, gMs2)
        return [h, s, r, b, gm, gMs, g, gMs2], (ok, err)

    for prec in ("f32", "f64"):
        dt = torch.float32 if prec == "f32" else torch.float64
        plan = DemagPlan(n, d, prec, autotune=True)
        m0 = to_dev(synth.random_unit(n, 31), dt)
        ref, rinfo = run_all(plan, m0, dt)
        before = plan.info()
        assert before["device_bytes"] > 0
        t, w, sc = plan.attach_memory()
        tb, wb = plan_bytes(n, prec)
        need = plan_scratch_bytes(n, prec)
        assert t.numel() == tb and w.numel() == wb and sc.numel() == max(need)
        after = plan.info()
        assert after["device_bytes"] == 0 and after["tiles"] == before["tiles"], (before, after)
        got, ginfo = run_all(plan, m0, dt)
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
        assert rinfo == ginfo
        assert plan.info()["device_bytes"] == 0
        with pytest.raises(MMError) as ei:
            plan.attach_memory()
        assert ei.value.code == MM_ESTATE
        # attached forward memory, no scratch: the scratch calls are refused
        p2 = DemagPlan(n, d, prec)
        p2.attach_memory(scratch=())
        x = m0.clone()
        with pytest.raises(MMError) as ei:
            p2.rkf45_step(x, MS, A, ALPHA, GAMMA, 2e-14, 1e-2)
        assert ei.value.code == MM_ESTATE and torch.equal(x, m0)
        g = ref[0].clone()
        with pytest.raises(MMError) as ei:
            p2.llg_step_adjoint(m0, MS, A, ALPHA, GAMMA, 1e-13, g)
        assert ei.value.code == MM_ESTATE and torch.equal(g, ref[0])
        with pytest.raises(MMError) as ei:
            p2.minimize(x, MS, A, tol=0.0, max_iter=2)
        assert ei.value.code == MM_ESTATE and torch.equal(x, m0)
        # h_eff and its adjoint need no scratch
        assert torch.equal(p2.h_eff(m0, MS, A), ref[0])
        assert p2.info()["device_bytes"] == 0
        p2.close()
        bad = m0.clone()
        bad[0, 0, 0, 0] = float("nan")
        with pytest.raises(MMError) as ei:
            plan.h_eff(bad, MS, A, energy=True)
        assert ei.value.code == MM_ENONFINITE
        plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_rkf45_step_against_oracle(prec):
    """One attempted RKF45 step on 32x32x4 (random m, per-cell Ms): the accepted
    result, the error estimate and the next step against the oracle (FP64 with
    the tensor held equal); a rejected attempt leaves m untouched."""
    import torch
    n, d = (32, 32, 4), (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant(n, d)
    L = tuple(oracle.default_L(v) for v in n)
    plan, dt_ = _plan(n, d, prec, hold=oct_ if prec == "f64" else None)
    m0 = rounded(synth.random_unit(n, 41), dt_)
    Ms = rounded(synth.ms_field(n, 42), dt_)
    dt, tol = 2e-14, 1e-2
    ref, err_ref, ok_ref, dtn_ref = oracle.rkf45_step(m0, Ms, A, d, oct_, L, ALPHA, GAMMA, dt, tol)
    assert ok_ref
    m = to_dev(m0, dt_)
    ok, err, dtn = plan.rkf45_step(m, to_dev(Ms, dt_), A, ALPHA, GAMMA, dt, tol)
    _say(prec, "err", err, err_ref, "dt_next", dtn, dtn_ref)
    assert ok
    e = rel_l2(m.cpu().numpy() - m0, ref - m0)
    assert e <= (1e-12 if prec == "f64" else 1e-5), e
    # err is a small difference of stage derivatives: in FP32 its absolute
    # error scales with dt max|k|, not with err itself
    k1 = oracle.llg_rhs(m0, oracle.h_eff(m0, Ms, A, d, oct_, L), ALPHA, GAMMA)
    scale = dt * np.abs(k1).max()
    if prec == "f64":
        assert abs(err / err_ref - 1) <= 1e-8
    else:
        assert abs(err - err_ref) <= 1e-5 * scale, (err, err_ref, scale)
    assert abs(dtn / dtn_ref - 1) <= (1e-8 if prec == "f64" else 1e-2)
    # a tolerance below the error: rejected, m bitwise unchanged, dt shrinks
    m = to_dev(m0, dt_)
    before = m.clone()
    ok, err2, dtn2 = plan.rkf45_step(m, to_dev(Ms, dt_), A, ALPHA, GAMMA, dt, err_ref / 10)
    assert not ok and torch.equal(m, before)
    _, _, ok_ref2, dtn_ref2 = oracle.rkf45_step(m0, Ms, A, d, oct_, L, ALPHA, GAMMA, dt, err_ref / 10)
    assert not ok_ref2 and abs(dtn2 / dtn_ref2 - 1) <= (1e-8 if prec == "f64" else 1e-2)


def test_rkf45_macrospin_adaptive_run():
    """Adaptive RKF45 on the 1x1x1 cubic cell in a field along z (FP64): the
    same accepted/rejected sequence as the oracle and the closed form within
    the tolerance scale."""
    import torch
    n, d = (1, 1, 1), (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant(n, d)
    plan, dt_ = _plan(n, d, "f64", hold=oct_)
    th0, ph0, H = 1.0, 0.3, 2e5
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)]).reshape(1, 1, 1, 3)
    T, tol = 2e-10, 1e-8
    m = to_dev(m0, dt_)
    acc, rej, _ = plan.rkf45_run(m, MS, A, 0.1, GAMMA, T, 5e-11, tol, h_ext=(0, 0, H))
    mr, acc_r, rej_r = oracle.rkf45_run(m0, T, 5e-11, tol, MS, A, d, oct_, n, 0.1, GAMMA, h_ext=(0, 0, H))
    ref = oracle.macrospin_closed_form(th0, ph0, H, 0.1, GAMMA, T)
    _say("rkf45 macrospin", acc, rej, acc_r, rej_r)
    assert (acc, rej) == (acc_r, rej_r) and rej >= 1
    got = m.cpu().numpy().reshape(3)
    assert np.abs(got - mr.reshape(3)).max() < 1e-12
    assert np.abs(got - ref).max() < 50 * tol


def test_minimize_bb_against_oracle():
    """Barzilai-Borwein minimisation of a 20x5x1 platelet (5x5x3 nm cells)
    from the uniform (1,1,1) state: FP64 iterates against the oracle's
    after 1, 2, 5 and 12 updates (tensor held equal), and the converged
    state in FP64 and FP32."""
    import torch
    n, d = (20, 5, 1), (5e-9, 5e-9, 3e-9)
    oct_ = oracle.tensor_octant(n, d)
    L = tuple(oracle.default_L(v) for v in n)
    m0 = np.ones(n + (3,)) / np.sqrt(3.0)
    hz = (1e3, -2e3, 0.0)
    plan, dt_ = _plan(n, d, "f64", hold=oct_)
    for k in (1, 2, 5, 12):
        m = to_dev(m0, dt_)
        it, tq = plan.minimize(m, MS, A, tol=0.0, max_iter=k, h_ext=hz)
        ref, kr, tqr = oracle.bb_minimize(m0, MS, A, d, oct_, L, h_ext=hz, tol=0.0, max_iter=k)
        assert it == kr == k
        e = np.abs(m.cpu().numpy() - ref).max()
        _say("bb iterate", k, e, tq, tqr)
        assert e <= 1e-10 and abs(tq / tqr - 1) <= 1e-8
    ref, kr, tqr = oracle.bb_minimize(m0, MS, A, d, oct_, L, h_ext=hz, tol=1e-2)
    Eref = oracle.total_energy(ref, MS, A, d, oct_, L, h_ext=hz)
    for prec, tol, mtol, etol in (("f64", 1e-2, 1e-6, 1e-8), ("f32", 1.0, 2e-4, 1e-6)):
        plan, dt_ = _plan(n, d, prec, hold=oct_ if prec == "f64" else None)
        m = to_dev(rounded(m0, dt_), dt_)
        it, tq = plan.minimize(m, MS, A, tol=tol, max_iter=5000, h_ext=hz)
        got = m.cpu().numpy()
        E = oracle.total_energy(got, MS, A, d, oct_, L, h_ext=hz)
        _say("bb converged", prec, it, kr, tq, np.abs(got - ref).max(), E / Eref - 1)
        assert tq <= tol
        assert np.abs(got - ref).max() <= mtol
        assert abs(E / Eref - 1) <= etol


@pytest.mark.parametrize("kind,D", [("interfacial", 3e-3), ("bulk", -2e-3)])
def test_dmi_against_oracle(kind, D):
    """h_eff and one RK4 step with the DMI field of eq. (3) on a 24x20x3 grid
    with per-cell Ms and a few vacuum cells, FP64 (tensor held equal) and
    FP32; removing the term restores the plain field; the adjoint refuses."""
    import torch
    from paper_2606_01114_amd._lib import MM_ENOTSUP, MMError
    n, d = (24, 20, 3), (2e-9, 2.5e-9, 1.5e-9)
    oct_ = oracle.tensor_octant(n, d)
    L = tuple(oracle.default_L(v) for v in n)
    m0 = synth.random_unit(n, 51)
    Ms = synth.ms_field(n, 52)
    Ms[3, 4, 1] = Ms[10, 0, 2] = Ms[23, 19, 0] = 0.0
    ref_h = oracle.h_eff(m0, Ms, A, d, oct_, L, dmi=(kind, D))
    heff = lambda s: oracle.h_eff(s, Ms, A, d, oct_, L, dmi=(kind, D))
    dt = 2e-14
    ref_s = oracle.rk4_step(m0, Ms, A, d, oct_, L, ALPHA, GAMMA, dt, heff=heff)
    for prec, tol in (("f64", 1e-12), ("f32", 1e-5)):
        plan, dt_ = _plan(n, d, prec, hold=oct_ if prec == "f64" else None)
        mr, Msr = rounded(m0, dt_), rounded(Ms, dt_)
        plan.set_dmi(kind, D)
        h = plan.h_eff(to_dev(mr, dt_), to_dev(Msr, dt_), A)
        e = rel_l2(h.cpu().numpy(), ref_h)
        m = to_dev(mr, dt_)
        plan.llg_step(m, to_dev(Msr, dt_), A, ALPHA, GAMMA, dt)
        es = rel_l2(m.cpu().numpy() - m0, ref_s - m0)
        _say("dmi", kind, prec, e, es)
        assert e <= tol and es <= tol
        with pytest.raises(MMError) as ei:
            plan.h_eff_adjoint(to_dev(mr, dt_), to_dev(Msr, dt_), A, h)
        assert ei.value.code == MM_ENOTSUP
        plan.set_dmi(None, 0.0)
        h0 = plan.h_eff(to_dev(mr, dt_), to_dev(Msr, dt_), A)
        assert rel_l2(h0.cpu().numpy(), oracle.h_eff(m0, Ms, A, d, oct_, L)) <= tol
        plan.close()


def test_anisotropy_with_dmi_against_oracle():
    """Uniaxial anisotropy (tilted axis) together with interfacial DMI: h_eff
    and one RK4 step against the oracle, FP64 (tensor held equal) and FP32;
    the minimiser reproduces the Stoner-Wohlfarth reversal of a single cell."""
    import torch
    n, d = (16, 12, 2), (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant(n, d)
    L = tuple(oracle.default_L(v) for v in n)
    m0 = synth.random_unit(n, 61)
    Ms = synth.ms_field(n, 62)
    Ku, u = 4e5, (0.3, -0.4, 0.866)
    heff = lambda s: oracle.h_eff(s, Ms, A, d, oct_, L, dmi=("interfacial", 2e-3), aniso=(Ku, u))
    ref_h = heff(m0)
    dt = 2e-14
    ref_s = oracle.rk4_step(m0, Ms, A, d, oct_, L, ALPHA, GAMMA, dt, heff=heff)
    for prec, tol in (("f64", 1e-12), ("f32", 1e-5)):
        plan, dt_ = _plan(n, d, prec, hold=oct_ if prec == "f64" else None)
        mr, Msr = rounded(m0, dt_), rounded(Ms, dt_)
        plan.set_dmi("interfacial", 2e-3)
        plan.set_anisotropy(Ku, u)
        h = plan.h_eff(to_dev(mr, dt_), to_dev(Msr, dt_), A)
        m = to_dev(mr, dt_)
        plan.llg_step(m, to_dev(Msr, dt_), A, ALPHA, GAMMA, dt)
        e, es = rel_l2(h.cpu().numpy(), ref_h), rel_l2(m.cpu().numpy() - m0, ref_s - m0)
        _say("aniso", prec, e, es)
        assert e <= tol and es <= tol
        plan.close()
    # single cell: reverses above H_k = 2 Ku/(mu0 Ms), stays below
    d1 = (2e-9, 2e-9, 2e-9)
    Hk = 2 * 2e5 / (oracle.MU0 * MS)
    uu = np.array([0.0, 0.6, 0.8])
    t = np.cross(uu, [1.0, 0.0, 0.0])
    m1 = (uu + 0.05 * t / np.linalg.norm(t)).reshape(1, 1, 1, 3)
    m1 = m1 / np.linalg.norm(m1)
    plan, dt_ = _plan((1, 1, 1), d1, "f64")
    plan.set_anisotropy(2e5, uu)
    for f, sign in ((0.97, 1.0), (1.03, -1.0)):
        m = to_dev(m1, dt_)
        it, tq = plan.minimize(m, MS, A, tol=1e-6, max_iter=100000, h_ext=tuple(-f * Hk * uu))
        assert tq <= 1e-6 and np.dot(m.cpu().numpy().reshape(3), uu) * sign > 0.99, (f, it)


def test_stt_against_oracle():
    """Slonczewski spin-transfer torque (lambda != 1, field-like part, tilted
    polarisation) with anisotropy, per-cell Ms with vacuum cells: h_eff, the
    term alone (terms = 0) and one RK4 step against the oracle, FP64 (tensor
    held equal) and FP32, through the compile-time z kernel (nz = 2) and the
    runtime-planned one (nz = 3, Lz = 6); removing it restores the plain
    field; the adjoint refuses it."""
    import torch
    from paper_2606_01114_amd import MMError
    stt = (6e11, 0.45, 1.7, 0.15, 2e-9, (0.2, -0.5, 0.8))
    for n, d in (((16, 12, 2), (2e-9, 2e-9, 2e-9)), ((10, 6, 3), (2.5e-9, 2e-9, 3e-9))):
        oct_ = oracle.tensor_octant(n, d)
        L = tuple(oracle.default_L(v) for v in n)
        m0 = synth.random_unit(n, 71)
        Ms = synth.ms_field(n, 72)
        Ms.reshape(-1)[::7] = 0.0
        heff = lambda s: oracle.h_eff(s, Ms, A, d, oct_, L, aniso=(3e5, (0, 1, 1)), stt=stt)
        ref_h = heff(m0)
        ref_loc = oracle.stt_field(m0, Ms, *stt) + oracle.anisotropy_field(m0, Ms, 3e5, (0, 1, 1))
        ref_plain = oracle.h_eff(m0, Ms, A, d, oct_, L)
        dt = 2e-14
        ref_s = oracle.rk4_step(m0, Ms, A, d, oct_, L, ALPHA, GAMMA, dt, heff=heff)
        for prec, tol in (("f64", 1e-12), ("f32", 1e-5)):
            plan, dt_ = _plan(n, d, prec, hold=oct_ if prec == "f64" else None)
            mr, Msr = rounded(m0, dt_), rounded(Ms, dt_)
            plan.set_anisotropy(3e5, (0, 1, 1))
            plan.set_stt(stt[0], P=stt[1], Lambda=stt[2], eps_prime=stt[3], d_layer=stt[4], p=stt[5])
            h = plan.h_eff(to_dev(mr, dt_), to_dev(Msr, dt_), A)
            hl = plan.h_eff(to_dev(mr, dt_), to_dev(Msr, dt_), A, terms=0)
            m = to_dev(mr, dt_)
            plan.llg_step(m, to_dev(Msr, dt_), A, ALPHA, GAMMA, dt)
            e, el = rel_l2(h.cpu().numpy(), ref_h), rel_l2(hl.cpu().numpy(), ref_loc)
            es = rel_l2(m.cpu().numpy() - m0, ref_s - m0)
            _say("stt", n, prec, e, el, es)
            assert e <= tol and el <= tol and es <= tol
            with pytest.raises(MMError):
                plan.h_eff_adjoint(to_dev(mr, dt_), to_dev(Msr, dt_), A, torch.zeros_like(h))
            plan.set_stt(0.0)
            plan.set_anisotropy(0.0)
            h0 = plan.h_eff(to_dev(mr, dt_), to_dev(Msr, dt_), A)
            assert rel_l2(h0.cpu().numpy(), ref_plain) <= tol
            with pytest.raises(MMError):
                plan.h_eff(to_dev(mr, dt_), to_dev(Msr, dt_), A, terms=0)
            plan.close()


def test_stt_macrospin_closed_form_on_gpu():
    """One cubic cell, lambda = 1 (constant eps), p and an applied field along
    z: the GPU's RK4 run follows the closed-form precession and relaxation
    with rates g (H' - alpha b) and g (b + alpha H') (FP64)."""
    j, d_layer, P, epsp, alpha, H = 5e11, 2e-9, 0.4, 0.1, 0.05, 1e5
    d = (2e-9, 2e-9, 2e-9)
    th0, ph0 = 1.1, -0.4
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)]).reshape(1, 1, 1, 3)
    beta = oracle.HBAR * j / (oracle.MU0 * oracle.E_CHARGE * MS * d_layer)
    b, Hp = beta * P / 2, H + beta * epsp
    g = GAMMA / (1 + alpha * alpha)
    T = 4e-11
    ph = ph0 + g * (Hp - alpha * b) * T
    th = 2 * np.arctan(np.tan(th0 / 2) * np.exp(-g * (b + alpha * Hp) * T))
    ref = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    plan, dt_ = _plan((1, 1, 1), d, "f64")
    plan.set_stt(j, P=P, Lambda=1.0, eps_prime=epsp, d_layer=d_layer, p=(0, 0, 3))
    m = to_dev(m0, dt_)
    plan.llg_step(m, MS, A, alpha, GAMMA, 1e-13, n_steps=400, h_ext=(0, 0, H))
    err = np.abs(m.cpu().numpy().reshape(3) - ref).max()
    _say("stt macrospin", err)
    assert err < 1e-9
    plan.close()


STENCIL_GRIDS = [(5, 7, 3), (3, 40, 33), (70, 9, 17), (1, 1, 1), (2, 600, 2), (4, 3, 512), (40, 2, 1), (3, 2, 600)]


@pytest.mark.parametrize("n", STENCIL_GRIDS)
def test_h_eff_without_demag_against_oracle(n):
    """h_eff without the demag term runs the streaming stencil kernel (for
    nz <= 512; nz = 600 takes the z pass): exchange alone with per-cell Ms and
    vacuum cells, its energy, and the local terms (DMI, anisotropy,
    spin-transfer torque) alone and with exchange, FP64 to 1e-12 and FP32 to
    1e-5 against the oracle; ragged plane blocks, x chunks, nz = 1 and the
    largest nz."""
    from paper_2606_01114_amd import MM_EXCHANGE
    d = (2e-9, 2.5e-9, 3e-9)
    m0 = synth.random_unit(n, 81)
    Ms = synth.ms_field(n, 82)
    Ms.reshape(-1)[::5] = 0.0
    stt = (4e11, 0.35, 1.6, 0.2, 2e-9, (0.3, 0.4, -0.5))
    ref_ex = oracle.exchange_field(m0, Ms, A, d)
    ref_loc = (oracle.dmi_field(m0, Ms, 1.5e-3, d, "bulk") + oracle.anisotropy_field(m0, Ms, 2e5, (1, 0, 1))
               + oracle.stt_field(m0, Ms, *stt))
    ref_e = oracle.energies(m0, Ms, np.zeros_like(ref_ex), ref_ex, d)[1]

    def rel(x, ref):       # a field that is exactly zero (a single cell) must come out zero
        return rel_l2(x, ref) if np.any(ref) else float(np.abs(x).max())

    for prec, tol in (("f64", 1e-12), ("f32", 1e-5)):
        plan, dt_ = _plan(n, d, prec)
        mr, Msr = to_dev(rounded(m0, dt_), dt_), to_dev(rounded(Ms, dt_), dt_)
        h, (e_d, e_x) = plan.h_eff(mr, Msr, A, terms=MM_EXCHANGE, energy=True)
        e1 = rel(h.cpu().numpy(), ref_ex)
        ee = abs(e_x - ref_e) / abs(ref_e) if ref_e != 0.0 else abs(e_x)
        plan.set_dmi("bulk", 1.5e-3)
        plan.set_anisotropy(2e5, (1, 0, 1))
        plan.set_stt(stt[0], P=stt[1], Lambda=stt[2], eps_prime=stt[3], d_layer=stt[4], p=stt[5])
        hl = plan.h_eff(mr, Msr, A, terms=0)
        hx = plan.h_eff(mr, Msr, A, terms=MM_EXCHANGE)
        e2 = rel(hl.cpu().numpy(), ref_loc)
        e3 = rel(hx.cpu().numpy(), ref_ex + ref_loc)
        # scalar Ms (no vacuum): exchange with the local terms
        hs = plan.h_eff(mr, MS, A, terms=MM_EXCHANGE)
        plan.set_stt(0.0)
        plan.set_anisotropy(0.0)
        plan.set_dmi(None, 0.0)
        hs0 = plan.h_eff(mr, MS, A, terms=MM_EXCHANGE)
        ref_s0 = oracle.exchange_field(m0, MS, A, d)
        ref_s = (ref_s0 + oracle.dmi_field(m0, MS, 1.5e-3, d, "bulk") + oracle.anisotropy_field(m0, MS, 2e5, (1, 0, 1))
                 + oracle.stt_field(m0, MS, *stt))
        e4, e5 = rel(hs.cpu().numpy(), ref_s), rel(hs0.cpu().numpy(), ref_s0)
        _say("no-demag", n, prec, e1, ee, e2, e3, e4, e5, e_d)
        assert e1 <= tol and ee <= tol and e2 <= tol and e3 <= tol and e4 <= tol and e5 <= tol and e_d == 0.0
        plan.close()


@pytest.mark.parametrize("padding", ["auto", "smooth"])
def test_rkf45_with_local_terms_against_oracle(padding):
    """One RKF45 step with DMI, anisotropy and the spin-transfer torque set
    (the tableau epilogue's local-term instantiation), through the
    compile-time z kernels (automatic padding) and the runtime-planned ones
    (7-smooth padding, Lz = 6), FP64 with the tensor held equal and FP32,
    against the oracle."""
    from paper_2606_01114_amd import DemagPlan
    import torch
    n, d = (20, 12, 3), (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant(n, d)
    m0 = synth.random_unit(n, 91)
    Ms = synth.ms_field(n, 92)
    stt = (3e11, 0.4, 1.8, 0.1, 2e-9, (0.0, 0.6, 0.8))
    dt, tol = 2e-14, 1e-2
    for prec, tolp in (("f64", 1e-12), ("f32", 1e-5)):
        plan = DemagPlan(n, d, prec, padding=padding)
        dt_ = torch.float64 if prec == "f64" else torch.float32
        if prec == "f64":
            plan.tensor_set(oct_)
        L = tuple(plan.info()["L"])
        if padding == "smooth":
            assert L[2] == 6
        mr, Msr = rounded(m0, dt_), rounded(Ms, dt_)
        heff = lambda s: oracle.h_eff(s, Msr, A, d, oct_, L, dmi=("interfacial", 1e-3), aniso=(2e5, (1, 1, 0)),
                                      stt=stt)
        ref, err_ref, ok_ref, _ = oracle.rkf45_step(mr, Msr, A, d, oct_, L, ALPHA, GAMMA, dt, tol, heff=heff)
        assert ok_ref
        plan.set_dmi("interfacial", 1e-3)
        plan.set_anisotropy(2e5, (1, 1, 0))
        plan.set_stt(stt[0], P=stt[1], Lambda=stt[2], eps_prime=stt[3], d_layer=stt[4], p=stt[5])
        m = to_dev(mr, dt_)
        ok, err, _ = plan.rkf45_step(m, to_dev(Msr, dt_), A, ALPHA, GAMMA, dt, tol)
        e = rel_l2(m.cpu().numpy() - mr, ref - mr)
        _say("rkf45 local", padding, prec, L, e, err, err_ref)
        assert ok and e <= tolp
        plan.close()


def test_minimize_stoner_wohlfarth_angle_on_gpu():
    """The GPU minimiser on one cubic cell with a z easy axis and a field at
    50 degrees lands on the Stoner-Wohlfarth equilibrium angle, the root of
    Ku sin(2 theta) = mu0 Ms H sin(psi - theta) (FP64)."""
    from scipy.optimize import brentq
    Ku, H, psi = 3e5, 2e5, np.deg2rad(50.0)
    d = (2e-9, 2e-9, 2e-9)
    theta = brentq(lambda t: Ku * np.sin(2 * t) - oracle.MU0 * MS * H * np.sin(psi - t), 0.0, psi, xtol=1e-15)
    plan, dt_ = _plan((1, 1, 1), d, "f64")
    plan.set_anisotropy(Ku, (0, 0, 1))
    m0 = np.array([0.1, 0.0, 1.0]).reshape(1, 1, 1, 3)
    m = to_dev(m0 / np.linalg.norm(m0), dt_)
    it, tq = plan.minimize(m, MS, A, tol=1e-8, max_iter=100000, h_ext=(H * np.sin(psi), 0.0, H * np.cos(psi)))
    mm = m.cpu().numpy().reshape(3)
    _say("SW angle", it, tq, np.arctan2(mm[0], mm[2]), theta)
    assert tq <= 1e-8 and abs(np.arctan2(mm[0], mm[2]) - theta) < 1e-10
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_heff_autograd_function(prec):
    """HEff (the torch.autograd.Function over h_eff and its hand-written
    adjoint): the gradient of a scalar loss through it against the oracle's
    VJP (FP64 with the tensor held equal: 1e-12; FP32: 1e-5), with a
    non-contiguous m; in FP64 a central finite difference of the loss along
    a random direction of m and of Ms matches the directional derivative."""
    import torch
    from paper_2606_01114_amd import HEff
    grid, cell = (10, 8, 3), (2.5e-9, 2.5e-9, 3e-9)
    oct_ = oracle.tensor_octant(grid, cell)
    plan, dt = _plan(grid, cell, prec, hold=oct_ if prec == "f64" else None)
    L = plan.info()["L"]
    m0 = rounded(synth.random_unit(grid, 13), dt)
    Ms = rounded(synth.ms_field(grid, 14), dt)
    w = rounded(synth.random_unit(grid, 15), dt)
    # a non-contiguous view with the same values
    big = torch.zeros(grid + (6,), dtype=dt, device="cuda")
    big[..., ::2] = to_dev(m0, dt)
    m = big[..., ::2].requires_grad_(False)
    assert not m.is_contiguous()
    m = m.detach().requires_grad_(True)
    Mst = to_dev(Ms, dt).requires_grad_(True)
    wt = to_dev(w, dt)
    h = HEff.apply(m, Mst, plan, A)
    loss = (h * wt).sum()
    loss.backward()
    rm, rMs = oracle.h_eff_vjp(m0, Ms, A, cell, oct_, L, w)
    tol = 1e-12 if prec == "f64" else 1e-5
    em, eMs = rel_l2(m.grad.cpu().numpy(), rm), rel_l2(Mst.grad.cpu().numpy(), rMs)
    _say("HEff", prec, "rel-L2 grad m %.3e Ms %.3e" % (em, eMs))
    assert em <= tol and eMs <= tol
    if prec == "f64":
        rng = np.random.default_rng(16)
        vm, vMs = rng.standard_normal(m0.shape), rng.standard_normal(Ms.shape) * 1e3

        def L_of(mm, MM):
            return float((plan.h_eff(to_dev(mm, dt), to_dev(MM, dt), A) * wt).sum())
        eps = 1e-3
        fd_m = (L_of(m0 + eps * vm, Ms) - L_of(m0 - eps * vm, Ms)) / (2 * eps)
        fd_M = (L_of(m0, Ms + eps * vMs) - L_of(m0, Ms - eps * vMs)) / (2 * eps)
        dm = float(np.sum(m.grad.cpu().numpy() * vm))
        dM = float(np.sum(Mst.grad.cpu().numpy() * vMs))
        _say("HEff FD", fd_m, dm, fd_M, dM)
        # h_eff is linear in m and affine in 1/Ms: central differences are exact
        # in m up to rounding and second order in Ms
        assert abs(fd_m - dm) <= 1e-9 * abs(dm)
        assert abs(fd_M - dM) <= 1e-6 * abs(dM)
    plan.close()


def test_allocation_failure_reports_enomem():
    """With MMX_TEST_FAIL_ALLOC set, plan creation fails with MM_ENOMEM (no
    plan, no device memory left behind); unset, it succeeds again."""
    import os
    from paper_2606_01114_amd import DemagPlan
    from paper_2606_01114_amd._lib import MM_ENOMEM, MMError
    os.environ["MMX_TEST_FAIL_ALLOC"] = "1"
    try:
        with pytest.raises(MMError) as ei:
            DemagPlan((8, 6, 2), (2e-9, 2e-9, 2e-9), "f32")
        assert ei.value.code == MM_ENOMEM
    finally:
        os.environ.pop("MMX_TEST_FAIL_ALLOC", None)
    plan = DemagPlan((8, 6, 2), (2e-9, 2e-9, 2e-9), "f32")
    assert plan.info()["device_bytes"] > 0
    plan.close()


def test_stream_switch_orders_work():
    """An asynchronous RK4 run queued on one torch stream, then h_eff of an
    unrelated field on another stream with no torch-level dependency between
    them: both share the plan's workspace, and mm_plan_set_stream orders the
    second stream after the first, so the results are bit-identical to the
    same calls on one stream."""
    import torch
    grid, cell = (64, 48, 8), (2.5e-9, 2.5e-9, 3e-9)
    plan, dt = _plan(grid, cell, "f32")
    m0 = to_dev(synth.random_unit(grid, 17), dt)
    c = to_dev(synth.random_unit(grid, 18), dt)
    a = m0.clone()
    plan.llg_step(a, MS, A, ALPHA, GAMMA, 1e-13, n_steps=20)
    hc = plan.h_eff(c, MS, A)
    b = m0.clone()
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        plan.llg_step(b, MS, A, ALPHA, GAMMA, 1e-13, n_steps=20)
    with torch.cuda.stream(s2):
        hc2 = plan.h_eff(c, MS, A)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(hc, hc2)
    plan.close()


def test_z_index_widths_agree():
    """The compile-time RK4-stage z-inverse kernels in 32-bit and 64-bit cell
    indexing (MMX_NO_I32 at plan creation) give bit-identical RK4 steps
    (graph replay) and steps with local terms, FP32 and FP64, on a grid with
    ragged z tiles (h_eff, 64-bit in both, as a control)."""
    import os
    import torch
    from paper_2606_01114_amd import DemagPlan
    n, d = (37, 29, 6), (2.5e-9, 2e-9, 3e-9)
    m0 = synth.random_unit(n, 71)
    Ms = synth.ms_field(n, 72)
    out = {}
    old = os.environ.get("MMX_NO_I32")
    try:
        for key in ("i32", "i64"):
            if key == "i64":
                os.environ["MMX_NO_I32"] = "1"
            else:
                os.environ.pop("MMX_NO_I32", None)
            for prec in ("f32", "f64"):
                dt = torch.float32 if prec == "f32" else torch.float64
                plan = DemagPlan(n, d, prec)
                Msd = to_dev(Ms, dt)
                h = plan.h_eff(to_dev(m0, dt), Msd, A)
                m = to_dev(m0, dt)
                plan.llg_step(m, Msd, A, ALPHA, GAMMA, 2e-14, n_steps=3)
                plan.set_anisotropy(4e5, (0.0, 0.6, 0.8))
                m2 = to_dev(m0, dt)
                plan.llg_step(m2, Msd, A, ALPHA, GAMMA, 2e-14, n_steps=2, graph=False)
                out[key, prec] = (h.cpu(), m.cpu(), m2.cpu())
                plan.close()
    finally:
        if old is None:
            os.environ.pop("MMX_NO_I32", None)
        else:
            os.environ["MMX_NO_I32"] = old
    for prec in ("f32", "f64"):
        for a, b in zip(out["i32", prec], out["i64", prec]):
            assert torch.equal(a, b), prec
