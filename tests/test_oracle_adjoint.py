"""Pins of the oracle's vector-Jacobian products: exact dot-product identities
for the linear part and central finite differences for the rest."""
import numpy as np

import oracle
import synth

MS = 8e5
A = 1.3e-11
GAMMA = 2.211e5
D = (2.5e-9, 2.5e-9, 3e-9)


def _setup(n=(4, 3, 2)):
    oct_ = oracle.tensor_octant(n, D)
    L = tuple(oracle.default_L(v) for v in n)
    Ms = synth.ms_field(n, 5)
    return oct_, L, Ms


def test_h_eff_vjp_m_is_exact_transpose():
    n = (4, 3, 2)
    oct_, L, Ms = _setup(n)
    m = synth.random_unit(n, 1)
    v = synth.random_unit(n, 2)
    g = synth.random_unit(n, 3)
    g_m, _ = oracle.h_eff_vjp(m, Ms, A, D, oct_, L, g)
    Jv = oracle.h_eff(v, Ms, A, D, oct_, L)          # h_eff is linear in m
    lhs, rhs = np.sum(g * Jv), np.sum(g_m * v)
    assert abs(lhs - rhs) <= 1e-12 * np.abs(g * Jv).sum()


def test_h_eff_vjp_Ms_fd():
    n = (4, 3, 2)
    oct_, L, Ms = _setup(n)
    m = synth.random_unit(n, 1)
    g = synth.random_unit(n, 3)
    _, g_Ms = oracle.h_eff_vjp(m, Ms, A, D, oct_, L, g)
    w = np.random.default_rng(4).standard_normal(n)
    eps = 1e-4 * MS

    def F(Msx):
        return np.sum(g * oracle.h_eff(m, Msx, A, D, oct_, L))
    fd = (F(Ms + eps * w) - F(Ms - eps * w)) / (2 * eps)
    assert abs(fd - np.sum(g_Ms * w)) <= 1e-7 * abs(fd)


def test_rk4_step_vjp_fd():
    n = (4, 3, 2)
    oct_, L, Ms = _setup(n)
    m = synth.random_unit(n, 1)
    g = synth.random_unit(n, 3)
    dt, alpha = 1e-13, 0.02
    g_m, g_Ms = oracle.rk4_step_vjp(m, Ms, A, D, oct_, L, alpha, GAMMA, dt, g)

    def F(mx, Msx):
        return np.sum(g * oracle.rk4_step(mx, Msx, A, D, oct_, L, alpha, GAMMA, dt))
    v = synth.random_unit(n, 8)
    eps = 1e-6
    fd = (F(m + eps * v, Ms) - F(m - eps * v, Ms)) / (2 * eps)
    assert abs(fd - np.sum(g_m * v)) <= 1e-7 * abs(fd)
    w = np.random.default_rng(9).standard_normal(n)
    e2 = 1e-3 * MS
    fd2 = (F(m, Ms + e2 * w) - F(m, Ms - e2 * w)) / (2 * e2)
    assert abs(fd2 - np.sum(g_Ms * w)) <= 1e-5 * abs(fd2)


def test_run_gradient_wrt_Ms_fd():
    n = (4, 3, 2)
    oct_, L, Ms = _setup(n)
    m0 = synth.smooth_film(n, D, 5)
    dt, alpha, steps = 1e-13, 0.02, 6
    gfin = np.zeros(n + (3,))
    gfin[..., 2] = 1.0 / np.prod(n)                      # loss = mean m_z
    _, gMs, _ = oracle.rk4_run_grad_Ms(m0, Ms, A, D, oct_, L, alpha, GAMMA, dt, steps, gfin)

    def loss(Msx):
        return oracle.rk4_run(m0, steps, Msx, A, D, oct_, L, alpha, GAMMA, dt)[..., 2].mean()
    for idx in [(0, 0, 0), (2, 1, 1), (3, 2, 0)]:
        e = 1e-3 * Ms[idx]
        Mp, Mm = Ms.copy(), Ms.copy()
        Mp[idx] += e
        Mm[idx] -= e
        fd = (loss(Mp) - loss(Mm)) / (2 * e)
        assert abs(fd - gMs[idx]) <= 1e-5 * np.abs(gMs).max()
