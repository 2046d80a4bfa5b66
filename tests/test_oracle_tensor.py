"""Pins of the oracle's demag tensor against facts that do not come from it.

The paper gives N only by reference to Newell's formulas (Implementation
section, eq. (4)); everything checked here is fixed by the mathematics of the
cell-averaged dipolar kernel, by an independent textbook closed form (Aharoni's
rectangular-prism demagnetising factors, J. Appl. Phys. 83, 3432 (1998)), or
by the dipole limit.
"""
import mpmath as mp
import numpy as np
import pytest

import oracle

D1 = (2.5e-9, 2.5e-9, 3e-9)


def aharoni_zz(a, b, c):
    """Aharoni's closed form for the zz factor of a prism of sides 2a, 2b, 2c
    (an independent derivation; evaluated at 40 digits)."""
    mp.mp.dps = 40
    a, b, c = mp.mpf(a), mp.mpf(b), mp.mpf(c)
    abc = a * b * c
    r = mp.sqrt(a * a + b * b + c * c)
    ab, bc, ac = mp.sqrt(a * a + b * b), mp.sqrt(b * b + c * c), mp.sqrt(a * a + c * c)
    t = ((b * b - c * c) / (2 * b * c) * mp.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * mp.log((r - b) / (r + b))
         + b / (2 * c) * mp.log((ab + a) / (ab - a)) + a / (2 * c) * mp.log((ab + b) / (ab - b))
         + c / (2 * a) * mp.log((bc - b) / (bc + b)) + c / (2 * b) * mp.log((ac - a) / (ac + a))
         + 2 * mp.atan(a * b / (c * r)) + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * abc)
         + (a * a + b * b - 2 * c * c) / (3 * abc) * r + c / (a * b) * (ac + bc)
         - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * abc))
    return float(t / mp.pi)


def test_cube_self_term_is_one_third():
    v = oracle.newell_at(0, 0, 0, (1e-9, 1e-9, 1e-9))
    assert np.allclose(v[:3], 1.0 / 3.0, rtol=0, atol=2e-16)
    assert np.all(np.abs(v[3:]) < 1e-30)


@pytest.mark.parametrize("cell", [(1.0, 1.0, 1.0), (2.0, 3.0, 0.5), (1.0, 1.0, 0.1),
                                  (1.0, 1.0, 0.01), (1.0, 1.0, 0.001), (4.0, 4.0, 0.7)])
def test_self_term_matches_aharoni(cell):
    d = tuple(c * 1e-9 for c in cell)
    v = oracle.newell_at(0, 0, 0, d)
    zz = aharoni_zz(cell[0] / 2, cell[1] / 2, cell[2] / 2)
    xx = aharoni_zz(cell[1] / 2, cell[2] / 2, cell[0] / 2)   # permute axes: x plays z
    yy = aharoni_zz(cell[2] / 2, cell[0] / 2, cell[1] / 2)
    assert abs(v[2] - zz) <= 4e-16
    assert abs(v[0] - xx) <= 4e-16
    assert abs(v[1] - yy) <= 4e-16


def test_thin_film_nzz_tends_to_one():
    vals = [oracle.newell_at(0, 0, 0, (1e-9, 1e-9, t * 1e-9))[2] for t in (1e-1, 1e-2, 1e-3)]
    assert vals[0] < vals[1] < vals[2] < 1.0
    assert 1.0 - vals[2] < 5e-3
    # a one-layer film lattice sum of Nzz approaches 1 as the film widens
    sums = []
    for half in (5, 20):
        I, J = np.meshgrid(np.arange(-half, half + 1), np.arange(-half, half + 1), indexing="ij")
        offs = np.stack([I.ravel(), J.ravel(), np.zeros(I.size, dtype=int)], 1)
        sums.append(oracle.tensor_at(offs, (1e-9, 1e-9, 0.5e-9), P=0)[:, 2].sum())
    assert sums[0] < sums[1] < 1.0 and sums[1] > 0.98


@pytest.mark.parametrize("off", [(0, 0, 0), (1, 0, 0), (0, 1, 1), (3, 2, 1), (7, -5, 2), (12, 3, -4), (40, 9, 2)])
def test_trace_is_delta(off):
    for d in (D1, (1e-9, 2e-9, 0.5e-9)):
        v = oracle.newell_at(*off, d)
        tr = v[:3].sum()
        target = 1.0 if off == (0, 0, 0) else 0.0
        assert abs(tr - target) <= 4e-16 * max(1.0 if target else 0.0, np.abs(v[:3]).max())


def test_parity():
    base = oracle.newell_at(3, 2, 1, D1)
    for sx, sy, sz in [(-1, 1, 1), (1, -1, 1), (1, 1, -1), (-1, -1, -1)]:
        v = oracle.newell_at(3 * sx, 2 * sy, 1 * sz, D1)
        expect = base * np.array([1, 1, 1, sx * sy, sx * sz, sy * sz])
        assert np.allclose(v, expect, rtol=1e-15, atol=0)


def test_block_superposition():
    """Cell-averaged interactions are additive: the interaction of two a x b x c
    blocks of cells equals Newell's kernel for the merged cells (both blocks
    uniformly magnetised), at zero and non-zero block offsets."""
    a, b, c = 2, 3, 2
    d = D1
    big = (a * d[0], b * d[1], c * d[2])
    cells = np.array([(i, j, k) for i in range(a) for j in range(b) for k in range(c)])
    for I, J, K in [(0, 0, 0), (1, 0, 0), (1, 2, 0), (2, -1, 1), (-3, 2, 2)]:
        shift = np.array([I * a, J * b, K * c])
        offs = (cells[:, None, :] + shift) - cells[None, :, :]
        vals = oracle.tensor_at(offs.reshape(-1, 3), d, P=0).reshape(len(cells), len(cells), 6)
        lhs = vals.sum(axis=(0, 1)) / len(cells)
        rhs = oracle.newell_at(I, J, K, big)
        scale = np.abs(vals).sum(axis=(0, 1)).max() / len(cells)
        assert np.all(np.abs(lhs - rhs) <= 1e-14 * scale), (I, J, K, lhs - rhs)


def test_dipole_limit():
    d = D1
    V = d[0] * d[1] * d[2]
    errs = []
    for r in (10, 20, 40):
        i, j, k = r, r // 2, r // 3
        v = oracle.newell_at(i, j, k, d)
        x, y, z = i * d[0], j * d[1], k * d[2]
        R2 = x * x + y * y + z * z
        dip = V / (4 * np.pi) * np.array([R2 - 3 * x * x, R2 - 3 * y * y, R2 - 3 * z * z,
                                          -3 * x * y, -3 * x * z, -3 * y * z]) / R2 ** 2.5
        errs.append(np.abs(v - dip).max() / np.abs(dip).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3
    assert 2.5 < errs[0] / errs[1] < 6 and 2.5 < errs[1] / errs[2] < 6   # O((d/r)^2)


def test_far_rule_vs_newell():
    d = D1
    errs = {}
    for r in (16, 24, 32):
        far = oracle.far_at(r, 2, 1, d)
        ex = oracle.newell_at(r, 2, 1, d)
        errs[r] = np.abs(far - ex).max() / np.abs(ex).max()
    assert errs[16] < 1e-8 and errs[24] < 1e-9 and errs[32] < 2e-10
    ratio = errs[16] / errs[32]
    assert 20 < ratio < 150          # ~ 2^6
    tr = oracle.far_at(30, 7, 3, d)[:3].sum()
    assert abs(tr) <= 1e-15 * np.abs(oracle.far_at(30, 7, 3, d)).max()


def test_switch_radius():
    d = D1
    P = 16.0
    lim = P * max(d)
    near = (int(lim / d[0]) - 1, 0, 0)
    far = (int(lim / d[0]) + 1, 0, 0)
    assert np.array_equal(oracle.tensor_at([near], d, P)[0], oracle.newell_at(*near, d))
    assert np.array_equal(oracle.tensor_at([far], d, P)[0], oracle.far_at(*far, d))


def test_octant_and_real_spectrum():
    n = (6, 5, 3)
    oct_ = oracle.tensor_octant(n, D1)
    for (i, j, k) in [(0, 0, 0), (5, 4, 2), (2, 3, 1)]:
        assert np.array_equal(oct_[i, j, k], oracle.tensor_at([(i, j, k)], D1)[0])
    for L in [(12, 10, 6), (11, 9, 5), (16, 15, 7)]:
        S = oracle.tensor_spectrum(oct_, L)
        assert np.abs(S.imag).max() <= 1e-13 * np.abs(S.real).max()
        T = oracle.wrap_full(oct_, L)
        # inverse: the wrapped arrays come back, and each has its parity
        assert np.allclose(np.fft.ifftn(S, axes=(1, 2, 3)).real, T, atol=1e-15)
        for q in range(6):
            px, py, pz = oracle.tensor.PARITY[q]
            R = T[q][(-np.arange(L[0])) % L[0]][:, (-np.arange(L[1])) % L[1]][:, :, (-np.arange(L[2])) % L[2]]
            assert np.array_equal(R, T[q] * (-1) ** (px + py + pz))


def test_default_L():
    assert oracle.default_L(1) == 1
    assert oracle.default_L(32) == 64 and oracle.default_L(1024) == 2048 and oracle.default_L(128) == 256
    assert oracle.default_L(53) == 105   # 106 = 2 * 53 is not 7-smooth
    for n in range(2, 400):
        L = oracle.default_L(n)
        assert L >= 2 * n - 1 and oracle.is_7smooth(L)
