"""Oracle: LLG right-hand side and the classic RK4 step (test infrastructure only).

* RHS (paper eq. (1), read for the unit vector m with M = Ms m):
  dm/dt = -gamma/(1+alpha^2) [ m x h + alpha m x (m x h) ].
* Classic fixed-step RK4 (the paper's own integrator is RKF45; the fixed-step
  RK4 is the reading used here): stage inputs are not normalised; the step ends
  with m <- m~/|m~| unless ``renorm`` is False.

* RKF45 (the paper's own integrator, section "Implementation": the
  Runge-Kutta-Fehlberg method, with the step size set from the maximum error
  over the whole grid).  One attempted step evaluates Fehlberg's six stages,
  forms the fourth- and fifth-order solutions y4, y5 and the error
  err = max over cells and components of |y5 - y4|.  Readings (the paper
  gives no tolerance or controller): the step is accepted when err <= tol;
  the fourth-order solution is advanced (Fehlberg's original pairing) and
  renormalised like the RK4 step; the next step size is
  dt * min(5, max(0.2, 0.9 (tol/err)^(1/5))) (5 dt when err = 0), both after
  an accepted and after a rejected attempt.

Pins (tests/test_oracle_llg.py): the 1x1x1 cubic macrospin under a field along
z against its closed form; fourth-order convergence when dt halves; |m|
drift bound without renormalisation; energy decay for alpha > 0.  RKF45: the
tableau satisfies every order condition up to order 5 (fifth-order weights)
and 4 (fourth-order weights) exactly in rational arithmetic, the fourth-order
weights fail an order-5 condition; local errors of y4 and y5 fall as dt^5 and
dt^6 on the macrospin; the error estimate tracks the true local error of y4;
an adaptive run stays within its tolerance of the closed form.
"""
from fractions import Fraction as _F

import numpy as np

from .field import h_eff as _h_eff


def llg_rhs(m, h, alpha, gamma):
    g = gamma / (1.0 + alpha * alpha)
    mxh = np.cross(m, h)
    return -g * (mxh + alpha * np.cross(m, mxh))


def rk4_step(m, Ms, A, d, octant, L, alpha, gamma, dt, h_ext=None, renorm=True,
             demag=True, exchange=True, heff=None):
    """One classic RK4 step; ``heff(m)`` overrides the field evaluation."""
    if heff is None:
        def heff(s):
            return _h_eff(s, Ms, A, d, octant, L, demag=demag, exchange=exchange, h_ext=h_ext)
    m = np.asarray(m, dtype=np.float64)
    k1 = llg_rhs(m, heff(m), alpha, gamma)
    k2 = llg_rhs(m + 0.5 * dt * k1, heff(m + 0.5 * dt * k1), alpha, gamma)
    k3 = llg_rhs(m + 0.5 * dt * k2, heff(m + 0.5 * dt * k2), alpha, gamma)
    k4 = llg_rhs(m + dt * k3, heff(m + dt * k3), alpha, gamma)
    u = m + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    if renorm:
        u = u / np.linalg.norm(u, axis=-1, keepdims=True)
    return u


def rk4_run(m, n_steps, *args, **kw):
    for _ in range(int(n_steps)):
        m = rk4_step(m, *args, **kw)
    return m


def macrospin_closed_form(theta0, phi0, H, alpha, gamma, t):
    """Exact motion of one moment in a static field H along +z:
    phi = phi0 + g H t, tan(theta/2) = tan(theta0/2) exp(-alpha g H t),
    g = gamma/(1+alpha^2).  Returns m(t) (3,)."""
    g = gamma / (1.0 + alpha * alpha)
    phi = phi0 + g * H * t
    theta = 2.0 * np.arctan(np.tan(theta0 / 2.0) * np.exp(-alpha * g * H * t))
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])


# ---- RKF45 ------------------------------------------------------------------
# Fehlberg's 4(5) pair: nodes c, stage matrix a (rows 2..6), weights of the
# fourth-order (b4) and fifth-order (b5) solutions, as exact rationals.
RKF45_C = [_F(0), _F(1, 4), _F(3, 8), _F(12, 13), _F(1), _F(1, 2)]
RKF45_A = [
    [],
    [_F(1, 4)],
    [_F(3, 32), _F(9, 32)],
    [_F(1932, 2197), _F(-7200, 2197), _F(7296, 2197)],
    [_F(439, 216), _F(-8), _F(3680, 513), _F(-845, 4104)],
    [_F(-8, 27), _F(2), _F(-3544, 2565), _F(1859, 4104), _F(-11, 40)],
]
RKF45_B4 = [_F(25, 216), _F(0), _F(1408, 2565), _F(2197, 4104), _F(-1, 5), _F(0)]
RKF45_B5 = [_F(16, 135), _F(0), _F(6656, 12825), _F(28561, 56430), _F(-9, 50), _F(2, 55)]


def rkf45_stages(m, heff, alpha, gamma, dt):
    """The six stage derivatives k_s = f(m + dt sum_j a_sj k_j)."""
    ks = []
    for s in range(6):
        x = m.copy()
        for j, a in enumerate(RKF45_A[s]):
            x = x + dt * float(a) * ks[j]
        ks.append(llg_rhs(x, heff(x), alpha, gamma))
    return ks


def rkf45_step(m, Ms, A, d, octant, L, alpha, gamma, dt, tol, h_ext=None, renorm=True,
               demag=True, exchange=True, heff=None):
    """One attempted RKF45 step.  Returns (m_next, err, accepted, dt_next):
    m_next is the renormalised fourth-order solution when accepted, else m."""
    if heff is None:
        def heff(s):
            return _h_eff(s, Ms, A, d, octant, L, demag=demag, exchange=exchange, h_ext=h_ext)
    m = np.asarray(m, dtype=np.float64)
    ks = rkf45_stages(m, heff, alpha, gamma, dt)
    y4 = m + dt * sum(float(b) * k for b, k in zip(RKF45_B4, ks))
    y5 = m + dt * sum(float(b) * k for b, k in zip(RKF45_B5, ks))
    err = float(np.max(np.abs(y5 - y4)))
    accepted = err <= tol
    fac = 5.0 if err == 0.0 else min(5.0, max(0.2, 0.9 * (tol / err) ** 0.2))
    if accepted:
        out = y4 / np.linalg.norm(y4, axis=-1, keepdims=True) if renorm else y4
    else:
        out = m.copy()
    return out, err, accepted, dt * fac


def rkf45_run(m, t_end, dt0, tol, *args, max_steps=100000, **kw):
    """Adaptive integration to t_end (the last step is shortened to land on it).
    Returns (m, accepted steps, rejected attempts)."""
    t, dt, acc, rej = 0.0, float(dt0), 0, 0
    for _ in range(max_steps):
        if t >= t_end:
            break
        h = min(dt, t_end - t)
        m2, err, ok, dt = rkf45_step(m, *args, h, tol, **kw)
        if ok:
            m, t, acc = m2, t + h, acc + 1
        else:
            rej += 1
    return m, acc, rej
