"""Oracle: vector-Jacobian products (test infrastructure only).

The paper relies on automatic differentiation for inverse problems (paper,
Introduction); these are the hand-derived reverse-mode products of the same
operators, in FP64:

* h_eff = H_d(Ms m) + H_ex(m; Ms).  The demag operator M -> -N (*) M is
  self-adjoint (N(r) = N(-r) and N is a symmetric 3x3 tensor), so for a
  cotangent g on h:  g_m = Ms H_d(g) + Lap(c g),  g_Ms = m . H_d(g) - g . h_ex / Ms,
  with c_i = 2A/(mu0 Ms_i) and Lap the Neumann graph Laplacian (vacuum cells
  excluded) with 1/d_a^2 weights.
* RHS f = -g' [m x h + alpha m x (m x h)]: with a = m x h and cotangent y,
  y_m = -g' [h x y + alpha (a x y + h x (y x m))],
  y_h = -g' [y x m + alpha (y x m) x m].
* one RK4 step including the final normalisation u -> u/|u|:
  u_bar = (I - u^ u^T) g / |u|, then the four stages in reverse.

Pins (tests/test_oracle_adjoint.py): dot-product identities against the
forward operators and central finite differences on small grids.
"""
import numpy as np

from .field import MU0, demag_fft, exchange_field, _ms_array
from .llg import llg_rhs
from .field import h_eff as _h_eff


def _neumann_lap(v, mag, d):
    lap = np.zeros_like(v)
    for ax in range(3):
        for s in (+1, -1):
            nb = np.zeros_like(v)
            nbmask = np.zeros(mag.shape, dtype=bool)
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if s == +1:
                src[ax], dst[ax] = slice(1, None), slice(0, -1)
            else:
                src[ax], dst[ax] = slice(0, -1), slice(1, None)
            nb[tuple(dst)] = v[tuple(src)]
            nbmask[tuple(dst)] = mag[tuple(src)]
            lap += np.where((nbmask & mag)[..., None], nb - v, 0.0) / d[ax] ** 2
    return lap


def h_eff_vjp(m, Ms, A, d, octant, L, g_h, demag=True, exchange=True):
    """(g_m, g_Ms) for the cotangent g_h of h_eff(m, Ms)."""
    m = np.asarray(m, dtype=np.float64)
    g_h = np.asarray(g_h, dtype=np.float64)
    Msa = _ms_array(Ms, m.shape[:3])
    mag = Msa > 0
    g_m = np.zeros_like(m)
    g_Ms = np.zeros(m.shape[:3])
    if demag:
        hg = demag_fft(g_h, 1.0, octant, L)          # -N (*) g
        g_m += Msa[..., None] * hg
        g_Ms += np.sum(m * hg, axis=-1)
    if exchange:
        c = np.where(mag, 2.0 * A / (MU0 * np.where(mag, Msa, 1.0)), 0.0)
        g_m += _neumann_lap(c[..., None] * g_h, mag, d)
        hex_ = exchange_field(m, Msa, A, d)
        g_Ms += np.where(mag, -np.sum(g_h * hex_, axis=-1) / np.where(mag, Msa, 1.0), 0.0)
    return g_m, g_Ms


def llg_rhs_vjp(m, h, alpha, gamma, y):
    g = gamma / (1.0 + alpha * alpha)
    a = np.cross(m, h)
    yxm = np.cross(y, m)
    y_m = -g * (np.cross(h, y) + alpha * (np.cross(a, y) + np.cross(h, yxm)))
    y_h = -g * (yxm + alpha * np.cross(yxm, m))
    return y_m, y_h


def rk4_step_vjp(m, Ms, A, d, octant, L, alpha, gamma, dt, g_next, h_ext=None,
                 renorm=True, demag=True, exchange=True):
    """Reverse of one RK4 step: returns (g_m, g_Ms)."""
    m = np.asarray(m, dtype=np.float64)

    def H(s):
        return _h_eff(s, Ms, A, d, octant, L, demag=demag, exchange=exchange, h_ext=h_ext)

    s1 = m
    h1 = H(s1); k1 = llg_rhs(s1, h1, alpha, gamma)
    s2 = m + 0.5 * dt * k1
    h2 = H(s2); k2 = llg_rhs(s2, h2, alpha, gamma)
    s3 = m + 0.5 * dt * k2
    h3 = H(s3); k3 = llg_rhs(s3, h3, alpha, gamma)
    s4 = m + dt * k3
    h4 = H(s4); k4 = llg_rhs(s4, h4, alpha, gamma)
    u = m + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    g_next = np.asarray(g_next, dtype=np.float64)
    if renorm:
        nu = np.linalg.norm(u, axis=-1, keepdims=True)
        uh = u / nu
        ub = (g_next - uh * np.sum(uh * g_next, axis=-1, keepdims=True)) / nu
    else:
        ub = g_next
    g_m = ub.copy()
    g_Ms = np.zeros(m.shape[:3])
    kb = [dt / 6.0 * ub, dt / 3.0 * ub, dt / 3.0 * ub, dt / 6.0 * ub]
    stages = [(s1, h1), (s2, h2), (s3, h3), (s4, h4)]
    coef = [None, 0.5 * dt, 0.5 * dt, dt]   # s_{q} = m + coef[q] k_{q-1}
    for q in (3, 2, 1, 0):
        s, h = stages[q]
        ym, yh = llg_rhs_vjp(s, h, alpha, gamma, kb[q])
        gm_h, gMs_h = h_eff_vjp(s, Ms, A, d, octant, L, yh, demag=demag, exchange=exchange)
        sb = ym + gm_h
        g_Ms += gMs_h
        g_m += sb
        if q > 0:
            kb[q - 1] = kb[q - 1] + coef[q] * sb
    return g_m, g_Ms


def rk4_run_grad_Ms(m0, Ms, A, d, octant, L, alpha, gamma, dt, n_steps, g_final, **kw):
    """Gradient w.r.t. Ms (and m0) of <g_final, m_T> after n_steps RK4 steps,
    by storing every m_n and reversing."""
    from .llg import rk4_step
    ms = [np.asarray(m0, dtype=np.float64)]
    for _ in range(int(n_steps)):
        ms.append(rk4_step(ms[-1], Ms, A, d, octant, L, alpha, gamma, dt, **kw))
    g = np.asarray(g_final, dtype=np.float64)
    gMs = np.zeros(ms[0].shape[:3])
    for n in range(int(n_steps) - 1, -1, -1):
        g, gm = rk4_step_vjp(ms[n], Ms, A, d, octant, L, alpha, gamma, dt, g, **kw)
        gMs += gm
    return g, gMs, ms[-1]
