"""Oracle: energy minimisation with Barzilai-Borwein step sizes (test
infrastructure only).

The paper (section "Implementation") minimises the system energy with the
Barzilai-Borwein algorithm and reduces its convergence criterion over the
whole grid so that all ranks stop together; it gives no formulas.  Readings
(a projected-gradient descent on the unit sphere per cell, in the form of
Exl et al. that the original magnum.np follows):

* h = h_eff (demag + exchange + applied field); the energy gradient with
  respect to m_i is -mu0 Ms_i V h_i, whose tangential part gives the descent
  direction -g_i with g_i = m_i x (m_i x h_i) = (m_i . h_i) m_i - h_i.
* update m <- normalise(m - tau g) for every cell.
* tau: the first iteration takes tau = 0.01 / max_i |m_i x h_i| (equal to
  max_i |g_i| for unit m_i: the most tilted moment turns by about 0.01 rad); iteration k >= 1 takes the Barzilai-
  Borwein lengths alternately, tau = (s.s)/(s.y) for odd k and
  (s.y)/(y.y) for even k, with s = m_k - m_{k-1}, y = g_k - g_{k-1} summed
  over all cells and components (FP64); a non-positive or non-finite value
  falls back to 0.01 / max_i |m_i x h_i|.
* stop at the first iterate with max_i |m_i x h_i| <= tol (that reduction
  is the global criterion), or after max_iter updates.

Pins (tests/test_oracle_minimize.py): a single cubic cell in an applied field
ends parallel to it; a uniformly magnetised platelet relaxes to the same
energy as a long damped LLG relaxation from the same start; the final state
is a fixed point (torque below tol) with lower energy than the start; a thin
film's moments end in plane.
"""
import numpy as np

from .field import demag_fft as _demag, exchange_field as _exch, energies as _energies, MU0


def torque_dir(m, h):
    """g = m x (m x h) per cell."""
    return np.cross(m, np.cross(m, h))


def bb_minimize(m, Ms, A, d, octant, L, h_ext=None, tol=1.0, max_iter=10000, heff=None):
    """Returns (m, iterations, final max torque |m x h|)."""
    if heff is None:
        def heff(s):
            h = _demag(s, Ms, octant, L) + _exch(s, Ms, A, d)
            if h_ext is not None:
                h = h + np.asarray(h_ext, dtype=np.float64)
            return h
    m = np.asarray(m, dtype=np.float64).copy()
    m_prev = g_prev = None
    k = 0
    while True:
        h = heff(m)
        g = torque_dir(m, h)
        torque = float(np.max(np.linalg.norm(np.cross(m, h), axis=-1)))
        if torque <= tol or k >= max_iter:
            return m, k, torque
        tau = 0.0
        if k >= 1:
            s = m - m_prev
            y = g - g_prev
            ss, sy, yy = float(np.sum(s * s)), float(np.sum(s * y)), float(np.sum(y * y))
            tau = ss / sy if k % 2 == 1 else sy / yy
        if not (np.isfinite(tau) and tau > 0.0):
            tau = 0.01 / torque   # |g_i| = |m_i x h_i| for unit m_i
        m_prev, g_prev = m, g
        u = m - tau * g
        m = u / np.linalg.norm(u, axis=-1, keepdims=True)
        k += 1


def total_energy(m, Ms, A, d, octant, L, h_ext=None):
    """E_demag + E_exchange + E_zeeman (J); E_zeeman = -mu0 V sum Ms m . h_ext."""
    hd = _demag(m, Ms, octant, L)
    hx = _exch(m, Ms, A, d)
    ed, ex = _energies(m, Ms, hd, hx, d)
    ez = 0.0
    if h_ext is not None:
        Msa = np.broadcast_to(np.asarray(Ms, dtype=np.float64), np.asarray(m).shape[:3])
        V = float(d[0]) * float(d[1]) * float(d[2])
        ez = -MU0 * V * float(np.sum(Msa[..., None] * m * np.asarray(h_ext, dtype=np.float64)))
    return ed + ex + ez
