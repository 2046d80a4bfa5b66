"""Pins of the oracle's Barzilai-Borwein energy minimiser."""
import numpy as np

import oracle

MS, A = 8e5, 1.3e-11


def test_single_cell_aligns_with_field():
    # a cubic cell: the demag self field -Ms m/3 is parallel to m, so the
    # minimum is m parallel to the applied field
    d = (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant((1, 1, 1), d)
    m0 = np.array([0.6, -0.48, 0.64]).reshape(1, 1, 1, 3)
    hz = np.array([1e4, 2e4, -2e4])
    m, k, tq = oracle.bb_minimize(m0, MS, A, d, oct_, (1, 1, 1), h_ext=hz, tol=1e-6)
    assert tq <= 1e-6 and k < 200
    assert np.abs(m.reshape(3) - hz / np.linalg.norm(hz)).max() < 1e-9


def test_platelet_same_minimum_as_damped_llg():
    """From the uniform (1,1,1) state of a 20x5x1 platelet of 5x5x3 nm cells,
    the minimiser and a strongly damped LLG run (RK4, alpha = 1) end in the
    same state: same energy, fixed point of the torque."""
    d = (5e-9, 5e-9, 3e-9)
    n = (20, 5, 1)
    oct_ = oracle.tensor_octant(n, d)
    L = tuple(oracle.default_L(v) for v in n)
    m0 = np.ones(n + (3,)) / np.sqrt(3.0)
    E0 = oracle.total_energy(m0, MS, A, d, oct_, L)
    m, k, tq = oracle.bb_minimize(m0, MS, A, d, oct_, L, tol=1e-2)
    E = oracle.total_energy(m, MS, A, d, oct_, L)
    assert tq <= 1e-2 and E < E0
    # damped LLG to rest
    ml = m0.copy()
    for _ in range(60):
        ml = oracle.rk4_run(ml, 50, MS, A, d, oct_, L, 1.0, 2.211e5, 4e-13)
        h = oracle.h_eff(ml, MS, A, d, oct_, L)
        if np.max(np.linalg.norm(np.cross(ml, h), axis=-1)) < 1e-2:
            break
    El = oracle.total_energy(ml, MS, A, d, oct_, L)
    assert abs(E - El) <= 1e-7 * abs(El)
    assert np.abs(m - ml).max() < 1e-4


def test_thin_film_relaxes_in_plane():
    d = (3e-9, 3e-9, 1e-9)
    n = (12, 12, 1)
    oct_ = oracle.tensor_octant(n, d)
    L = tuple(oracle.default_L(v) for v in n)
    rng = np.random.default_rng(3)
    m0 = np.array([1.0, 0.2, 0.6]) + 0.05 * rng.standard_normal(n + (3,))
    m0 /= np.linalg.norm(m0, axis=-1, keepdims=True)
    m, k, tq = oracle.bb_minimize(m0, MS, A, d, oct_, L, tol=1e-1)
    assert tq <= 1e-1
    assert np.abs(m[..., 2]).max() < 0.05
    assert oracle.total_energy(m, MS, A, d, oct_, L) < oracle.total_energy(m0, MS, A, d, oct_, L)


def test_stoner_wohlfarth_equilibrium_angle():
    """One cubic cell (no demag torque, no exchange) with a uniaxial easy axis
    along z and a field at 50 degrees to it in the x-z plane: the minimum of
    E(theta) = Ku sin^2(theta) - mu0 Ms H cos(theta - psi) solves
    Ku sin(2 theta) = mu0 Ms H sin(psi - theta), found here by bracketing; the
    minimiser must land on that angle."""
    from scipy.optimize import brentq
    Ku, H, psi = 3e5, 2e5, np.deg2rad(50.0)
    d = (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant((1, 1, 1), d)
    heff = lambda s: oracle.h_eff(s, MS, A, d, oct_, (1, 1, 1), aniso=(Ku, (0, 0, 1))) + \
        np.array([H * np.sin(psi), 0.0, H * np.cos(psi)])
    f = lambda t: Ku * np.sin(2 * t) - oracle.MU0 * MS * H * np.sin(psi - t)
    theta = brentq(f, 0.0, psi, xtol=1e-15)
    m0 = np.array([0.1, 0.0, 1.0]).reshape(1, 1, 1, 3)
    m0 = m0 / np.linalg.norm(m0)
    m, k, tq = oracle.bb_minimize(m0, MS, A, d, oct_, (1, 1, 1), tol=1e-8, max_iter=100000, heff=heff)
    mm = m.reshape(3)
    assert tq <= 1e-8 and abs(mm[1]) < 1e-12
    assert abs(np.arctan2(mm[0], mm[2]) - theta) < 1e-10, (np.arctan2(mm[0], mm[2]), theta)
