"""Pins of the oracle's LLG right-hand side and RK4 step."""
import numpy as np

import oracle
import synth

MS = 8e5
A = 1.3e-11
GAMMA = 2.211e5


def _macrospin(alpha, dt, steps, renorm=True):
    d = (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant((1, 1, 1), d)
    th0, ph0 = 1.0, 0.3
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)]).reshape(1, 1, 1, 3)
    H = 2e5
    m = oracle.rk4_run(m0, steps, MS, A, d, oct_, (1, 1, 1), alpha, GAMMA, dt, h_ext=(0, 0, H), renorm=renorm)
    ref = oracle.macrospin_closed_form(th0, ph0, H, alpha, GAMMA, dt * steps)
    return m.reshape(3), ref


def test_macrospin_closed_form_through_full_field():
    # a cubic single cell: H_d = -Ms m / 3 is parallel to m, exchange is 0,
    # so only the applied field along z acts
    m, ref = _macrospin(0.1, 1e-13, 400)
    assert np.abs(m - ref).max() < 1e-10


def test_rk4_fourth_order():
    e1 = np.abs(np.subtract(*_macrospin(0.1, 4e-13, 100))).max()
    e2 = np.abs(np.subtract(*_macrospin(0.1, 2e-13, 200))).max()
    assert 12 < e1 / e2 < 20


def test_norm_drift_without_renormalisation():
    m, _ = _macrospin(0.05, 2e-13, 50, renorm=False)
    m2, _ = _macrospin(0.05, 1e-13, 100, renorm=False)
    dr1, dr2 = abs(np.linalg.norm(m) - 1), abs(np.linalg.norm(m2) - 1)
    assert dr1 < 1e-6 and dr2 < dr1 / 8


def test_rhs_orthogonal_to_m():
    m = synth.random_unit((4, 3, 2), 5)
    h = synth.random_unit((4, 3, 2), 6) * 1e5
    f = oracle.llg_rhs(m, h, 0.02, GAMMA)
    assert np.abs(np.sum(f * m, -1)).max() <= 1e-12 * np.abs(f).max()


def test_energy_decays_with_damping():
    n = (6, 5, 2)
    d = (2.5e-9, 2.5e-9, 3e-9)
    oct_ = oracle.tensor_octant(n, d)
    L = tuple(oracle.default_L(v) for v in n)
    m = synth.random_unit(n, 12)

    def E(m):
        hd = oracle.demag_fft(m, MS, oct_, L)
        hx = oracle.exchange_field(m, MS, A, d)
        return sum(oracle.energies(m, MS, hd, hx, d))

    es = [E(m)]
    for _ in range(8):
        m = oracle.rk4_step(m, MS, A, d, oct_, L, 0.5, GAMMA, 2e-14)
        es.append(E(m))
    assert all(b < a for a, b in zip(es, es[1:]))
