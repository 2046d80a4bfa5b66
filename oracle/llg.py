"""Oracle: LLG right-hand side and the classic RK4 step (test infrastructure only).

* RHS (paper eq. (1), read for the unit vector m with M = Ms m):
  dm/dt = -gamma/(1+alpha^2) [ m x h + alpha m x (m x h) ].
* Classic fixed-step RK4 (the paper's own integrator is RKF45; the fixed-step
  RK4 is the reading used here): stage inputs are not normalised; the step ends
  with m <- m~/|m~| unless ``renorm`` is False.

Pins (tests/test_oracle_llg.py): the 1x1x1 cubic macrospin under a field along
z against its closed form; fourth-order convergence when dt halves; |m|
drift bound without renormalisation; energy decay for alpha > 0.
"""
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
