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


# ---- RKF45 pins ---------------------------------------------------------------
def _trees(order):
    """Rooted trees with `order` nodes, each as a sorted tuple of subtrees."""
    if order == 1:
        return [()]
    out = set()

    def parts(n, maxfirst):
        # multisets of subtree sizes summing to n (non-increasing)
        if n == 0:
            yield []
            return
        for k in range(min(n, maxfirst), 0, -1):
            for rest in parts(n - k, k):
                yield [k] + rest

    for sizes in parts(order - 1, order - 1):
        combos = [[]]
        for k in sizes:
            combos = [c + [t] for c in combos for t in _trees(k)]
        for c in combos:
            out.add(tuple(sorted(c)))
    return sorted(out)


def _phi(tree, A, s):
    """Elementary weight of stage s for a tree (sum over the stage matrix)."""
    from fractions import Fraction
    v = Fraction(1)
    for sub in tree:
        v *= sum((A[s][j] * _phi(sub, A, j) for j in range(len(A[s]))), Fraction(0))
    return v


def _density(tree):
    n = 1 + sum(_size(t) for t in tree)
    d = n
    for t in tree:
        d *= _density(t)
    return d


def _size(tree):
    return 1 + sum(_size(t) for t in tree)


def _satisfies(b, order):
    from fractions import Fraction
    A = oracle.RKF45_A
    return all(sum(b[s] * _phi(t, A, s) for s in range(6)) == Fraction(1, _density(t))
               for t in _trees(order))


def test_rkf45_tableau_order_conditions_exact():
    from fractions import Fraction
    assert [len(_trees(k)) for k in range(1, 6)] == [1, 1, 2, 4, 9]
    A, C = oracle.RKF45_A, oracle.RKF45_C
    for s in range(6):
        assert sum(A[s], Fraction(0)) == C[s]
    for k in range(1, 6):
        assert _satisfies(oracle.RKF45_B5, k), k
    for k in range(1, 5):
        assert _satisfies(oracle.RKF45_B4, k), k
    assert not _satisfies(oracle.RKF45_B4, 5)


def _ms_setup():
    d = (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant((1, 1, 1), d)
    th0, ph0, H = 1.0, 0.3, 2e5
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)]).reshape(1, 1, 1, 3)
    return d, oct_, th0, ph0, H, m0


def test_rkf45_local_orders_and_error_estimate():
    """One step of the macrospin: y4's local error falls as dt^5, y5's as dt^6,
    and err = |y5 - y4| matches y4's true local error."""
    d, oct_, th0, ph0, H, m0 = _ms_setup()
    heff = lambda s: oracle.h_eff(s, MS, A, d, oct_, (1, 1, 1), h_ext=(0, 0, H))
    e4, e5, est = [], [], []
    for dt in (3.2e-12, 1.6e-12, 8e-13):      # above the rounding floor of y5
        ks = oracle.rkf45_stages(m0, heff, 0.1, GAMMA, dt)
        y4 = m0 + dt * sum(float(b) * k for b, k in zip(oracle.RKF45_B4, ks))
        y5 = m0 + dt * sum(float(b) * k for b, k in zip(oracle.RKF45_B5, ks))
        ref = oracle.macrospin_closed_form(th0, ph0, H, 0.1, GAMMA, dt)
        e4.append(np.abs(y4.reshape(3) - ref).max())
        e5.append(np.abs(y5.reshape(3) - ref).max())
        est.append(np.abs(y5 - y4).max())
    for a, b in zip(e4, e4[1:]):
        assert 24 < a / b < 40          # 2^5
    for a, b in zip(e5, e5[1:]):
        assert 48 < a / b < 80          # 2^6
    for e, s in zip(e4, est):
        assert 0.8 < s / e < 1.25


def test_rkf45_adaptive_run_within_tolerance():
    d, oct_, th0, ph0, H, m0 = _ms_setup()
    T = 2e-10
    for tol in (1e-6, 1e-8):
        m, acc, rej = oracle.rkf45_run(m0, T, 1e-12, tol, MS, A, d, oct_, (1, 1, 1), 0.1, GAMMA,
                                       h_ext=(0, 0, H))
        ref = oracle.macrospin_closed_form(th0, ph0, H, 0.1, GAMMA, T)
        assert np.abs(m.reshape(3) - ref).max() < 50 * tol
        assert acc > 3
    # a step far too long is rejected, leaves m unchanged and shrinks dt
    m2, err, ok, dt2 = oracle.rkf45_step(m0, MS, A, d, oct_, (1, 1, 1), 0.1, GAMMA, 5e-11, 1e-8, h_ext=(0, 0, H))
    assert not ok and np.array_equal(m2, m0) and dt2 == 0.2 * 5e-11 and err > 1e-8


# ---- uniaxial anisotropy ---------------------------------------------------------
def _aniso_cell(Ku, u, theta0, phi0):
    d = (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant((1, 1, 1), d)
    m0 = np.array([np.sin(theta0) * np.cos(phi0), np.sin(theta0) * np.sin(phi0), np.cos(theta0)]).reshape(1, 1, 1, 3)
    heff = lambda s: oracle.h_eff(s, MS, A, d, oct_, (1, 1, 1), aniso=(Ku, u))
    return d, oct_, m0, heff


def test_anisotropy_undamped_precession_closed_form():
    """One cubic cell with a z easy axis and alpha = 0: the demag self field is
    parallel to m, so m precesses about z at fixed theta with angular rate
    gamma H_k cos(theta), H_k = 2 Ku/(mu0 Ms)."""
    Ku, th0, ph0 = 5e5, 0.7, 0.2
    d, oct_, m0, heff = _aniso_cell(Ku, (0, 0, 1), th0, ph0)
    Hk = 2 * Ku / (oracle.MU0 * MS)
    ref = oracle.macrospin_closed_form(th0, ph0, Hk * np.cos(th0), 0.0, GAMMA, 3e-11)
    errs = []
    for dt, n in ((1e-13, 300), (5e-14, 600)):
        m = oracle.rk4_run(m0, n, MS, A, d, oct_, (1, 1, 1), 0.0, GAMMA, dt, heff=heff)
        errs.append(np.abs(m.reshape(3) - ref).max())
    # RK4's own error, fourth order, on the exact precession
    assert errs[1] < 2e-10 and 12 < errs[0] / errs[1] < 20


def test_anisotropy_stoner_wohlfarth_switching_field():
    """Field antiparallel to the easy axis: a single cell stays near +u below
    H_k = 2 Ku/(mu0 Ms) and reverses above it (the minimiser from a slightly
    tilted start)."""
    Ku = 2e5
    Hk = 2 * Ku / (oracle.MU0 * MS)
    u = np.array([0.0, 0.6, 0.8])
    d = (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant((1, 1, 1), d)
    t = np.cross(u, [1.0, 0.0, 0.0])
    m0 = (u + 0.05 * t / np.linalg.norm(t)).reshape(1, 1, 1, 3)
    m0 = m0 / np.linalg.norm(m0)
    for f, sign in ((0.97, 1.0), (1.03, -1.0)):
        heff = lambda s, f=f: oracle.h_eff(s, MS, A, d, oct_, (1, 1, 1), aniso=(Ku, u)) - f * Hk * u
        m, k, tq = oracle.bb_minimize(m0, MS, A, d, oct_, (1, 1, 1), tol=1e-6, max_iter=100000, heff=heff)
        assert tq <= 1e-6
        assert np.dot(m.reshape(3), u) * sign > 0.99, (f, m)


# ---- Slonczewski spin-transfer torque ------------------------------------------
def _stt_beta(j, d_layer):
    return oracle.HBAR * j / (oracle.MU0 * oracle.E_CHARGE * MS * d_layer)


def test_stt_macrospin_closed_form_constant_eps():
    """Lam = 1 makes eps = P/2 constant.  One cubic cell (no demag torque, no
    exchange) with p and an applied field H along z: the field is
    H' z + b (m x z) with H' = H + beta eps', b = beta eps, and the motion is
    phi = phi0 + g (H' - alpha b) t, tan(theta/2) = tan(theta0/2) exp(-g (b + alpha H') t)."""
    j, d_layer, P, epsp, alpha, H = 5e11, 2e-9, 0.4, 0.1, 0.05, 1e5
    d = (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant((1, 1, 1), d)
    th0, ph0 = 1.1, -0.4
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)]).reshape(1, 1, 1, 3)
    stt = (j, P, 1.0, epsp, d_layer, (0.0, 0.0, 2.0))
    heff = lambda s: oracle.h_eff(s, MS, A, d, oct_, (1, 1, 1), h_ext=(0, 0, H), stt=stt)
    beta = _stt_beta(j, d_layer)
    b, Hp = beta * P / 2, H + beta * epsp
    g = GAMMA / (1 + alpha * alpha)
    T = 4e-11
    ph = ph0 + g * (Hp - alpha * b) * T
    th = 2 * np.arctan(np.tan(th0 / 2) * np.exp(-g * (b + alpha * Hp) * T))
    ref = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    errs = []
    for dt, n in ((2e-13, 200), (1e-13, 400)):
        m = oracle.rk4_run(m0, n, MS, A, d, oct_, (1, 1, 1), alpha, GAMMA, dt, heff=heff)
        errs.append(np.abs(m.reshape(3) - ref).max())
    assert errs[1] < 1e-9 and 12 < errs[0] / errs[1] < 20, errs


def test_stt_polar_travel_time_and_azimuth():
    """Lam = 2 (eps depends on m . p), no applied field, eps' = 0, negative
    current: theta obeys dtheta/dt = -g beta eps(cos theta) sin theta, so the
    time from theta0 to theta1 is a quadrature, and dphi/dtheta = alpha/sin theta
    gives phi1 - phi0 = alpha ln(tan(theta1/2)/tan(theta0/2)) whatever eps is."""
    from scipy.integrate import quad
    j, d_layer, P, Lam, alpha = -8e11, 2e-9, 0.5, 2.0, 0.02
    d = (2e-9, 2e-9, 2e-9)
    oct_ = oracle.tensor_octant((1, 1, 1), d)
    th0, th1, ph0 = 0.3, 2.0, 0.25
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)]).reshape(1, 1, 1, 3)
    stt = (j, P, Lam, 0.0, d_layer, (0.0, 0.0, 1.0))
    heff = lambda s: oracle.h_eff(s, MS, A, d, oct_, (1, 1, 1), stt=stt)
    beta = _stt_beta(j, d_layer)
    g = GAMMA / (1 + alpha * alpha)
    L2 = Lam * Lam
    eps = lambda th: P * L2 / ((L2 + 1) + (L2 - 1) * np.cos(th))
    t1, qerr = quad(lambda th: 1.0 / (-g * beta * eps(th) * np.sin(th)), th0, th1, epsabs=0, epsrel=1e-13, limit=200)
    assert qerr < 1e-12 * t1
    n = 1500
    m = oracle.rk4_run(m0, n, MS, A, d, oct_, (1, 1, 1), alpha, GAMMA, t1 / n, heff=heff).reshape(3)
    assert abs(np.arccos(m[2]) - th1) < 1e-8
    dphi = np.arctan2(m[1], m[0]) - ph0
    assert abs(dphi - alpha * np.log(np.tan(th1 / 2) / np.tan(th0 / 2))) < 1e-8


def test_stt_field_vanishes_without_current_and_in_vacuum():
    m = synth.random_unit((3, 2, 2), 4)
    Ms = np.full((3, 2, 2), MS)
    Ms[1, 0, 1] = 0.0
    h0 = oracle.stt_field(m, Ms, 0.0, 0.4, 1.5, 0.1, 2e-9, (1, 0, 0))
    assert np.all(h0 == 0.0)
    h = oracle.stt_field(m, Ms, 1e12, 0.4, 1.5, 0.1, 2e-9, (1, 0, 0))
    assert np.all(h[1, 0, 1] == 0.0) and np.all(np.abs(h[0, 0, 0]) > 0)
