"""Oracle: the demag tensor and its spectrum (test infrastructure only).

Definition (paper, Implementation section, eq. (4): the demag field is the
convolution of M with a kernel N obtained from Newell's formulas):

* N(r) for a lattice offset r = (i dx, j dy, k dz) is the cell-averaged
  interaction of two equal cells.  Inside the switch radius
  ``|r|_2 <= P * max(d)`` it is Newell's closed form (binary128, in
  newell_q.c); outside, a 27-node dipole quadrature matching the 2nd and 4th
  moments of the cell-pair displacement.  P <= 0 means Newell everywhere.
* Component order is xx, yy, zz, xy, xz, yz.  The diagonal components are even
  in every axis; xy is odd in x and y, xz odd in x and z, yz odd in y and z.
* The convolution is zero-padded: per axis a length L >= 2n-1 and
  T[i mod L] = N(i) for |i| < n, every other slot zero.

Pins (tests/test_oracle_tensor.py): the cube self term 1/3; the trace
N_xx+N_yy+N_zz = delta(r); parity; the self term of any prism against
Aharoni's independent closed form; the block-superposition identity; the
point-dipole asymptote; the far rule against binary128 Newell with its
(d/r)^6 error law; real spectra.
"""
import numpy as np

from . import _native

PARITY = {  # per component: (odd in x, odd in y, odd in z)
    0: (0, 0, 0), 1: (0, 0, 0), 2: (0, 0, 0),
    3: (1, 1, 0), 4: (1, 0, 1), 5: (0, 1, 1),
}


def _dptr(a):
    import ctypes
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def newell_at(i, j, k, d):
    """Newell tensor (binary128, rounded to binary64) at one offset -> (6,)."""
    out = np.zeros(6)
    _native.lib().oracle_newell(int(i), int(j), int(k), float(d[0]), float(d[1]), float(d[2]), _dptr(out), None)
    return out


def newell_scale_at(i, j, k, d):
    """Cancellation scale sum_e |w(e) f(...)| / (4 pi V) per component -> (6,)."""
    out = np.zeros(6)
    sc = np.zeros(6)
    _native.lib().oracle_newell(int(i), int(j), int(k), float(d[0]), float(d[1]), float(d[2]), _dptr(out), _dptr(sc))
    return sc


def far_at(i, j, k, d):
    """The moment-matched dipole quadrature at one offset -> (6,)."""
    out = np.zeros(6)
    _native.lib().oracle_far(int(i), int(j), int(k), float(d[0]), float(d[1]), float(d[2]), _dptr(out))
    return out


def tensor_at(offsets, d, P=16.0):
    """The tensor definition at many offsets: offsets (K,3) int -> (K,6)."""
    import ctypes
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64).reshape(-1, 3))
    out = np.zeros((off.shape[0], 6))
    _native.lib().oracle_tensor_many(off.shape[0], off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     float(d[0]), float(d[1]), float(d[2]), float(P), _dptr(out))
    return out


def tensor_octant(n, d, P=16.0):
    """Real-space octant N(i,j,k), 0 <= i,j,k < n, as (nx,ny,nz,6) float64."""
    nx, ny, nz = (int(v) for v in n)
    out = np.zeros((nx, ny, nz, 6))
    _native.lib().oracle_tensor_octant(nx, ny, nz, float(d[0]), float(d[1]), float(d[2]), float(P), _dptr(out))
    return out


def is_7smooth(v):
    v = int(v)
    if v < 1:
        return False
    for p in (2, 3, 5, 7):
        while v % p == 0:
            v //= p
    return v == 1


def default_L(n):
    """Padded length per axis: 1 for n == 1, 2n when n is 7-smooth, else the
    smallest 7-smooth length >= 2n-1 (any L >= 2n-1 gives the same linear
    convolution)."""
    n = int(n)
    if n == 1:
        return 1
    if is_7smooth(n):
        return 2 * n
    L = 2 * n - 1
    while not is_7smooth(L):
        L += 1
    return L


def wrap_full(octant, L):
    """Periodic wrap of the octant into (6, Lx, Ly, Lz): T[i mod L] = N(i)
    for |i| < n (using each component's parity), zero elsewhere."""
    nx, ny, nz, _ = octant.shape
    Lx, Ly, Lz = (int(v) for v in L)
    assert Lx >= 2 * nx - 1 and Ly >= 2 * ny - 1 and Lz >= 2 * nz - 1
    T = np.zeros((6, Lx, Ly, Lz))
    ii = np.arange(-nx + 1, nx)
    jj = np.arange(-ny + 1, ny)
    kk = np.arange(-nz + 1, nz)
    for q in range(6):
        px, py, pz = PARITY[q]
        full = octant[np.abs(ii)][:, np.abs(jj)][:, :, np.abs(kk)][..., q].copy()
        full *= np.where(ii < 0, -1.0, 1.0)[:, None, None] ** px
        full *= np.where(jj < 0, -1.0, 1.0)[None, :, None] ** py
        full *= np.where(kk < 0, -1.0, 1.0)[None, None, :] ** pz
        T[q][np.ix_(ii % Lx, jj % Ly, kk % Lz)] = full
    return T


def tensor_spectrum(octant, L):
    """Full complex DFT (numpy) of the wrapped components, (6, Lx, Ly, Lz).
    By the parities the result is real; the imaginary part is returned too so
    a test can check that."""
    T = wrap_full(octant, L)
    return np.fft.fftn(T, axes=(1, 2, 3))
