"""Oracle: demag field, exchange field, energies (test infrastructure only).

* demag (paper eq. (4), with the sign made explicit): H_d,i = -sum_j N(r_i-r_j) M_j,
  M_j = Ms_j m_j.  ``demag_fft`` is the zero-padded FFT convolution (pad to L,
  full complex DFT with numpy as the library step, pointwise 3x3 product,
  inverse DFT, truncate); ``demag_direct`` is the O(N^2) sum over all pairs.
* exchange (paper eq. (2) with uniform A): h_ex,i = 2A/(mu0 Ms_i) *
  sum over the 6 neighbours j inside the grid of (m_j - m_i)/d_a^2 (a missing
  neighbour contributes nothing).  A cell with Ms = 0 is vacuum: it is no
  neighbour of anything and its own exchange field is 0.
* DMI (paper eq. (3)): h_dmi,i = 2D/(mu0 Ms_i) sum_k e_k^DMI x dm/dk with
  e^DMI = (e_y, -e_x, 0) for interfacial and (e_x, e_y, e_z) for bulk DMI;
  dm/dk by central differences (m_{i+1} - m_{i-1}) / (2 d_k).  The paper is
  silent on the boundary; reading: a neighbour outside the grid or in vacuum
  is replaced by the cell itself (as for exchange), so its difference is 0.
* uniaxial anisotropy (one of the local fields of section "Implementation"):
  h_ani,i = 2 Ku/(mu0 Ms_i) (m_i . u) u with the unit easy axis u; 0 in vacuum.
* Slonczewski spin-transfer torque (the other local field named in section
  "Implementation"; the paper takes its model from the cited literature and
  prints no formula).  Reading: the torque of Slonczewski's model written as an
  effective field that enters the LLG equation like every other field,
  h_stt,i = beta_i [eps(m_i . p) (m_i x p) + eps' p],
  beta_i = hbar j / (mu0 e Ms_i d), eps(x) = P Lam^2 / ((Lam^2 + 1) + (Lam^2 - 1) x),
  with current density j, free-layer thickness d, spin polarisation P, the
  asymmetry parameter Lam, the field-like ratio eps' and the unit
  polarisation vector p; 0 in vacuum.  No energy (the torque is not
  conservative).
* energies: E = -(mu0/2) V sum_i Ms_i m_i . h_i for each term, in FP64.

Pins (tests/test_oracle_field.py): direct sum == FFT convolution; naive DFT ==
numpy.fft; a uniformly magnetised cube/prism block gives the block's Newell
self term (Aharoni); exchange of a uniform m is 0; the discrete helix closed
form; the exchange energy pair-sum identity; the discrete cycloid (interfacial)
and helix (bulk) closed forms of the DMI field; DMI of a uniform m is 0.
Spin-transfer torque (tests/test_oracle_llg.py): the macrospin closed form
with Lam = 1 (constant eps, field-like part and an applied field along p), and
for Lam != 1 the polar-angle travel time from a quadrature of the exact
angular equation together with the closed-form azimuth phi(theta).
"""
import numpy as np

from .tensor import wrap_full, PARITY

MU0 = 4e-7 * np.pi
HBAR = 1.054571817e-34      # J s (CODATA 2018)
E_CHARGE = 1.602176634e-19  # C (exact in the SI since 2019)


def _ms_array(Ms, shape):
    Ms = np.asarray(Ms, dtype=np.float64)
    if Ms.ndim == 0:
        return np.full(shape, float(Ms))
    assert Ms.shape == tuple(shape)
    return Ms


def naive_dft(x, axis=-1, inverse=False):
    """X_k = sum_n x_n exp(-+2 pi i (k n mod L) / L), no normalisation; the
    angle index is reduced in integers before the FP64 cos/sin."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    L = x.shape[-1]
    kn = (np.arange(L)[:, None] * np.arange(L)[None, :]) % L
    sgn = 1.0 if inverse else -1.0
    Wm = np.cos(2 * np.pi * kn / L) + 1j * sgn * np.sin(2 * np.pi * kn / L)
    return np.moveaxis(x @ Wm.T, -1, axis)


def demag_fft(m, Ms, octant, L, fft=np.fft):
    """Zero-padded FFT convolution: H = -N (*) (Ms m) on the first n cells."""
    m = np.asarray(m, dtype=np.float64)
    nx, ny, nz, _ = m.shape
    Lx, Ly, Lz = (int(v) for v in L)
    M = m * _ms_array(Ms, (nx, ny, nz))[..., None]
    Mp = np.zeros((3, Lx, Ly, Lz))
    for a in range(3):
        Mp[a, :nx, :ny, :nz] = M[..., a]
    Mh = fft.fftn(Mp, axes=(1, 2, 3))
    Nh = fft.fftn(wrap_full(octant, L), axes=(1, 2, 3))
    idx = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (0, 2): 4, (2, 0): 4, (1, 2): 5, (2, 1): 5}
    H = np.zeros((nx, ny, nz, 3))
    for a in range(3):
        Ha = sum(Nh[idx[(a, b)]] * Mh[b] for b in range(3))
        H[..., a] = -fft.ifftn(Ha, axes=(0, 1, 2)).real[:nx, :ny, :nz]
    return H


def full_tensor_at_offsets(octant, di, dj, dk):
    """N at signed offsets (arrays) from the octant using each parity."""
    out = np.empty(np.broadcast(di, dj, dk).shape + (6,))
    base = octant[np.abs(di), np.abs(dj), np.abs(dk)]
    for q in range(6):
        px, py, pz = PARITY[q]
        s = np.ones(base.shape[:-1])
        if px:
            s = s * np.where(di < 0, -1.0, 1.0)
        if py:
            s = s * np.where(dj < 0, -1.0, 1.0)
        if pz:
            s = s * np.where(dk < 0, -1.0, 1.0)
        out[..., q] = base[..., q] * s
    return out


def demag_direct(m, Ms, octant, cells=None, chunk=1 << 22):
    """O(N^2) direct sum H_i = -sum_j N(r_i - r_j) M_j, optionally only at the
    listed target cells (K,3) -> (K,3); else at every cell -> (nx,ny,nz,3).
    Sources are visited in chunks of ``chunk`` cells to bound memory."""
    m = np.asarray(m, dtype=np.float64)
    nx, ny, nz, _ = m.shape
    M = (m * _ms_array(Ms, (nx, ny, nz))[..., None]).reshape(-1, 3)
    ntot = nx * ny * nz
    if cells is None:
        I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        targets = np.stack([I.ravel(), J.ravel(), K.ravel()], 1)
    else:
        targets = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    H = np.zeros((targets.shape[0], 3))
    for s0 in range(0, ntot, chunk):
        idx = np.arange(s0, min(ntot, s0 + chunk))
        I, r = np.divmod(idx, ny * nz)
        J, K = np.divmod(r, nz)
        Mc = M[idx]
        for t, (i, j, k) in enumerate(targets):
            Nt = full_tensor_at_offsets(octant, i - I, j - J, k - K)   # (chunk,6)
            H[t, 0] -= (Nt[:, 0] * Mc[:, 0] + Nt[:, 3] * Mc[:, 1] + Nt[:, 4] * Mc[:, 2]).sum()
            H[t, 1] -= (Nt[:, 3] * Mc[:, 0] + Nt[:, 1] * Mc[:, 1] + Nt[:, 5] * Mc[:, 2]).sum()
            H[t, 2] -= (Nt[:, 4] * Mc[:, 0] + Nt[:, 5] * Mc[:, 1] + Nt[:, 2] * Mc[:, 2]).sum()
    return H if cells is not None else H.reshape(nx, ny, nz, 3)


def demag_direct_at(m, Ms, octant, cells):
    """The same direct sum as ``demag_direct`` at the listed target cells
    (K,3) -> (K,3), looped in plain C over every source cell with
    compensated summation (direct_sum.c), for grids where the numpy sum
    is too slow (10^8 cells and more)."""
    import ctypes
    from . import _native
    m = np.ascontiguousarray(m, dtype=np.float64)
    nx, ny, nz, _ = m.shape
    oc = np.ascontiguousarray(octant, dtype=np.float64)
    assert oc.shape == (nx, ny, nz, 6)
    Msa = np.asarray(Ms, dtype=np.float64)
    Msp = None
    if Msa.ndim != 0:
        Msa = np.ascontiguousarray(Msa)
        assert Msa.shape == (nx, ny, nz)
    tg = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).reshape(-1, 3))
    out = np.zeros((tg.shape[0], 3))
    pd = ctypes.POINTER(ctypes.c_double)
    if Msa.ndim != 0:
        Msp = Msa.ctypes.data_as(pd)
    _native.lib().oracle_demag_direct_at(nx, ny, nz, oc.ctypes.data_as(pd), m.ctypes.data_as(pd), Msp,
                                         float(Msa) if Msa.ndim == 0 else 0.0, tg.shape[0],
                                         tg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), out.ctypes.data_as(pd))
    return out


def exchange_at(m, Ms, A, d, cells):
    """Exchange field at the listed cells only (K,3) -> (K,3), same rule as
    ``exchange_field``."""
    m = np.asarray(m, dtype=np.float64)
    nx, ny, nz, _ = m.shape
    Msa = _ms_array(Ms, (nx, ny, nz))
    out = np.zeros((len(cells), 3))
    for t, (i, j, k) in enumerate(np.asarray(cells, dtype=np.int64)):
        if not Msa[i, j, k] > 0:
            continue
        lap = np.zeros(3)
        for ax, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            for s in (1, -1):
                a, b, c = i + s * di, j + s * dj, k + s * dk
                if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz and Msa[a, b, c] > 0:
                    lap += (m[a, b, c] - m[i, j, k]) / d[ax] ** 2
        out[t] = 2.0 * A / (MU0 * Msa[i, j, k]) * lap
    return out


def exchange_field(m, Ms, A, d):
    """6-point exchange field with free (Neumann) boundaries and vacuum cells."""
    m = np.asarray(m, dtype=np.float64)
    nx, ny, nz, _ = m.shape
    Msa = _ms_array(Ms, (nx, ny, nz))
    mag = Msa > 0
    lap = np.zeros_like(m)
    for ax in range(3):
        for s in (+1, -1):
            nb = np.zeros_like(m)
            nbmask = np.zeros(mag.shape, dtype=bool)
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if s == +1:
                src[ax], dst[ax] = slice(1, None), slice(0, -1)
            else:
                src[ax], dst[ax] = slice(0, -1), slice(1, None)
            nb[tuple(dst)] = m[tuple(src)]
            nbmask[tuple(dst)] = mag[tuple(src)]
            lap += np.where(nbmask[..., None], nb - m, 0.0) / d[ax] ** 2
    pref = np.where(mag, 2.0 * A / (MU0 * np.where(mag, Msa, 1.0)), 0.0)
    return pref[..., None] * lap


def dmi_field(m, Ms, D, d, kind):
    """DMI field of eq. (3); kind "interfacial" or "bulk"."""
    m = np.asarray(m, dtype=np.float64)
    nx, ny, nz, _ = m.shape
    Msa = _ms_array(Ms, (nx, ny, nz))
    mag = Msa > 0
    # central difference along each axis, missing / vacuum neighbour -> the cell
    dm = []
    for ax in range(3):
        diff = np.zeros_like(m)
        for s in (+1, -1):
            nb = m.copy()
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if s == +1:
                src[ax], dst[ax] = slice(1, None), slice(0, -1)
            else:
                src[ax], dst[ax] = slice(0, -1), slice(1, None)
            okm = np.zeros(mag.shape, dtype=bool)
            okm[tuple(dst)] = mag[tuple(src)]
            nb[tuple(dst)] = m[tuple(src)]
            nb = np.where(okm[..., None], nb, m)
            diff += s * (nb - m)
        dm.append(diff / (2.0 * d[ax]))
    ex, ey, ez = np.eye(3)
    if kind == "interfacial":
        evec = (ey, -ex, np.zeros(3))
    elif kind == "bulk":
        evec = (ex, ey, ez)
    else:
        raise ValueError("kind must be interfacial or bulk")
    h = np.zeros_like(m)
    for k in range(3):
        h += np.cross(np.broadcast_to(evec[k], m.shape), dm[k])
    pref = np.where(mag, 2.0 * D / (MU0 * np.where(mag, Msa, 1.0)), 0.0)
    return pref[..., None] * h


def anisotropy_field(m, Ms, Ku, u):
    """Uniaxial anisotropy field 2 Ku/(mu0 Ms) (m . u) u, u normalised here."""
    m = np.asarray(m, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    u = u / np.linalg.norm(u)
    Msa = _ms_array(Ms, m.shape[:3])
    mag = Msa > 0
    pref = np.where(mag, 2.0 * Ku / (MU0 * np.where(mag, Msa, 1.0)), 0.0)
    return (pref * (m @ u))[..., None] * u


def stt_field(m, Ms, j, P, Lam, eps_prime, d_layer, p):
    """Slonczewski torque as an effective field (reading in the module
    docstring); p is normalised here."""
    m = np.asarray(m, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    p = p / np.linalg.norm(p)
    Msa = _ms_array(Ms, m.shape[:3])
    mag = Msa > 0
    beta = np.where(mag, HBAR * j / (MU0 * E_CHARGE * np.where(mag, Msa, 1.0) * d_layer), 0.0)
    L2 = Lam * Lam
    eps = P * L2 / ((L2 + 1.0) + (L2 - 1.0) * (m @ p))
    return beta[..., None] * (eps[..., None] * np.cross(m, p) + eps_prime * p)


def h_eff(m, Ms, A, d, octant, L, demag=True, exchange=True, h_ext=None, dmi=None, aniso=None, stt=None):
    """dmi: None or (kind, D); aniso: None or (Ku, u); stt: None or
    (j, P, Lam, eps_prime, d_layer, p)."""
    h = np.zeros(np.asarray(m).shape)
    if stt is not None:
        h = h + stt_field(m, Ms, *stt)
    if aniso is not None:
        h = h + anisotropy_field(m, Ms, aniso[0], aniso[1])
    if demag:
        h = h + demag_fft(m, Ms, octant, L)
    if exchange:
        h = h + exchange_field(m, Ms, A, d)
    if dmi is not None:
        h = h + dmi_field(m, Ms, dmi[1], d, dmi[0])
    if h_ext is not None:
        h = h + np.asarray(h_ext, dtype=np.float64)
    return h


def energies(m, Ms, h_d, h_ex, d):
    """(E_demag, E_exchange) = -(mu0/2) V sum Ms_i m_i . h_i."""
    m = np.asarray(m, dtype=np.float64)
    V = float(d[0]) * float(d[1]) * float(d[2])
    Msa = _ms_array(Ms, m.shape[:3])
    e_d = -0.5 * MU0 * V * float(np.sum(Msa[..., None] * m * h_d))
    e_x = -0.5 * MU0 * V * float(np.sum(Msa[..., None] * m * h_ex))
    return e_d, e_x
