"""Pins of the oracle's DFT, demag convolution, exchange field and energies."""
import numpy as np
import pytest

import oracle
import synth

D2 = (2e-9, 2e-9, 2e-9)
MS = 8e5
A = 1.3e-11


@pytest.mark.parametrize("L", [1, 2, 7, 8, 15, 63, 64, 105])
def test_naive_dft_matches_numpy(L):
    rng = np.random.default_rng(L)
    x = rng.standard_normal((3, L)) + 1j * rng.standard_normal((3, L))
    ref = np.fft.fft(x, axis=-1)
    assert np.abs(oracle.naive_dft(x) - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    inv = oracle.naive_dft(x, inverse=True)
    assert np.abs(inv - np.fft.ifft(x, axis=-1) * L).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    # impulse and constant closed forms
    e = np.zeros(L); e[0] = 1
    assert np.allclose(oracle.naive_dft(e), np.ones(L), atol=1e-15)
    assert np.allclose(oracle.naive_dft(np.ones(L)), np.eye(1, L, 0)[0] * L, atol=1e-12)


def test_direct_sum_equals_fft_convolution_small():
    n = (4, 4, 2)
    m = synth.random_unit(n, 11)
    oct_ = oracle.tensor_octant(n, D2)
    L = tuple(oracle.default_L(v) for v in n)
    h1 = oracle.demag_fft(m, MS, oct_, L)
    h2 = oracle.demag_direct(m, MS, oct_)
    assert np.abs(h1 - h2).max() <= 1e-14 * np.abs(h2).max()
    # an odd (non 2n) padding gives the same linear convolution
    h3 = oracle.demag_fft(m, MS, oct_, (7, 9, 3))
    assert np.abs(h3 - h2).max() <= 1e-14 * np.abs(h2).max()
    # the naive DFT as the transform gives the same field
    class NaiveFFT:
        @staticmethod
        def fftn(x, axes):
            for ax in axes:
                x = oracle.naive_dft(x, axis=ax)
            return x

        @staticmethod
        def ifftn(x, axes):
            for ax in axes:
                x = oracle.naive_dft(x, axis=ax, inverse=True) / x.shape[ax]
            return x
    h4 = oracle.demag_fft(m, MS, oct_, L, fft=NaiveFFT)
    assert np.abs(h4 - h2).max() <= 1e-13 * np.abs(h2).max()


def test_direct_sum_equals_fft_convolution_c1_sampled():
    n = (32, 32, 4)
    m = synth.random_unit(n, 1)
    oct_ = oracle.tensor_octant(n, D2)
    L = (64, 64, 8)
    h = oracle.demag_fft(m, MS, oct_, L)
    cells = synth.sample_cells(n, 1, 48)
    hd = oracle.demag_direct(m, MS, oct_, cells=cells)
    got = h[cells[:, 0], cells[:, 1], cells[:, 2]]
    assert np.abs(got - hd).max() <= 1e-13 * np.abs(h).max()


def test_compiled_direct_sum_against_numpy_sum_and_fft():
    """The C direct sum (compensated, every source cell) agrees with the
    numpy direct sum and with the FFT convolution at every target, for a
    scalar and for a per-cell Ms with vacuum cells, at corner, edge and
    interior targets of a grid whose sizes are all different."""
    n, d = (9, 7, 5), (2.5e-9, 2e-9, 3e-9)
    m = synth.random_unit(n, 21)
    oct_ = oracle.tensor_octant(n, d)
    Ms = synth.ms_field(n, 22)
    Ms.reshape(-1)[::4] = 0.0
    cells = np.array([[0, 0, 0], [8, 6, 4], [4, 3, 2], [0, 6, 1], [8, 0, 4], [3, 0, 0]])
    L = tuple(oracle.default_L(v) for v in n)
    for ms in (MS, Ms):
        c = oracle.demag_direct_at(m, ms, oct_, cells)
        ref = oracle.demag_direct(m, ms, oct_, cells=cells)
        full = oracle.demag_fft(m, ms, oct_, L)[cells[:, 0], cells[:, 1], cells[:, 2]]
        assert np.abs(c - ref).max() <= 1e-14 * np.abs(ref).max()
        assert np.abs(c - full).max() <= 1e-13 * np.abs(ref).max()


def test_compiled_direct_sum_uniform_block():
    """Uniformly magnetised 4x3x2 block: the C direct sum averaged over every
    cell is -Ms N_block m with Newell's self term of the merged cell."""
    blk, d = (4, 3, 2), (2.5e-9, 2.5e-9, 3e-9)
    oct_ = oracle.tensor_octant(blk, d, P=0)
    mdir = np.array([-0.2, 0.7, 0.5]); mdir /= np.linalg.norm(mdir)
    m = np.broadcast_to(mdir, blk + (3,)).copy()
    cells = np.array(list(np.ndindex(*blk)))
    h = oracle.demag_direct_at(m, MS, oct_, cells).mean(0)
    Nb = oracle.newell_at(0, 0, 0, (blk[0] * d[0], blk[1] * d[1], blk[2] * d[2]))
    Nm = np.array([[Nb[0], Nb[3], Nb[4]], [Nb[3], Nb[1], Nb[5]], [Nb[4], Nb[5], Nb[2]]])
    assert np.allclose(h, -MS * Nm @ mdir, rtol=0, atol=1e-13 * MS)


@pytest.mark.parametrize("blk", [(1, 1, 1), (3, 4, 2), (5, 2, 1)])
def test_uniform_block_mean_field(blk):
    """A uniformly magnetised block made of cells: the mean demag field is
    -Ms N_block m with N_block Newell's self term of one merged cell."""
    d = (2.5e-9, 2.5e-9, 3e-9)
    oct_ = oracle.tensor_octant(blk, d, P=0)
    L = tuple(oracle.default_L(v) for v in blk)
    mdir = np.array([0.3, -0.5, 0.81]); mdir /= np.linalg.norm(mdir)
    m = np.broadcast_to(mdir, tuple(blk) + (3,))
    h = oracle.demag_fft(m, MS, oct_, L).reshape(-1, 3).mean(0)
    Nb = oracle.newell_at(0, 0, 0, (blk[0] * d[0], blk[1] * d[1], blk[2] * d[2]))
    Nm = np.array([[Nb[0], Nb[3], Nb[4]], [Nb[3], Nb[1], Nb[5]], [Nb[4], Nb[5], Nb[2]]])
    assert np.allclose(h, -MS * Nm @ mdir, rtol=0, atol=1e-13 * MS)
    if blk == (1, 1, 1) and d[0] == d[2]:
        assert np.allclose(h, -MS * mdir / 3)


def test_demag_self_adjoint_and_positive():
    n = (6, 5, 3)
    oct_ = oracle.tensor_octant(n, D2)
    L = tuple(oracle.default_L(v) for v in n)
    a = synth.random_unit(n, 3)
    b = synth.random_unit(n, 4)
    ha = oracle.demag_fft(a, 1.0, oct_, L)
    hb = oracle.demag_fft(b, 1.0, oct_, L)
    assert abs(np.sum(a * hb) - np.sum(b * ha)) <= 1e-13 * np.abs(a * hb).sum()
    assert -np.sum(a * ha) > 0     # the self-energy of any M is positive


def test_exchange_uniform_is_zero():
    n = (5, 4, 3)
    m = np.broadcast_to(np.array([0.6, 0.0, 0.8]), n + (3,)).copy()
    assert np.all(oracle.exchange_field(m, MS, A, D2) == 0.0)


@pytest.mark.parametrize("ax", [0, 1, 2])
def test_exchange_helix_closed_form(ax):
    d = (2.5e-9, 2e-9, 3e-9)
    n = [3, 3, 3]
    n[ax] = 12
    k = 2 * np.pi / (7.3 * d[ax])
    pos = np.arange(n[ax]) * d[ax]
    shape = [1, 1, 1]
    shape[ax] = n[ax]
    ph = (k * pos).reshape(shape)
    m = np.stack(np.broadcast_arrays(np.cos(ph), np.sin(ph), np.zeros_like(ph)), -1)
    m = np.broadcast_to(m, tuple(n) + (3,)).copy()
    h = oracle.exchange_field(m, MS, A, d)
    c = 2 * A / (oracle.MU0 * MS)
    sl = [slice(None)] * 3
    sl[ax] = slice(1, -1)
    interior = h[tuple(sl)]
    expect = -c * (2 - 2 * np.cos(k * d[ax])) / d[ax] ** 2 * m[tuple(sl)]
    assert np.allclose(interior, expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())
    # the first cell sees one neighbour only
    sl0 = [0, 0, 0]
    sl0[ax] = 0
    sl1 = list(sl0)
    sl1[ax] = 1
    e0 = c * (m[tuple(sl1)] - m[tuple(sl0)]) / d[ax] ** 2
    e0c = c * np.array([np.cos(k * d[ax]) - 1, np.sin(k * d[ax]), 0]) / d[ax] ** 2
    assert np.allclose(h[tuple(sl0)], e0, rtol=1e-13) and np.allclose(e0, e0c, rtol=1e-9, atol=1e-6 * np.abs(e0c).max())


def test_exchange_energy_pair_identity():
    n = (5, 4, 3)
    d = (2.5e-9, 2e-9, 3e-9)
    m = synth.random_unit(n, 7)
    h = oracle.exchange_field(m, MS, A, d)
    _, ex = oracle.energies(m, MS, np.zeros_like(h), h, d)
    V = d[0] * d[1] * d[2]
    s = 0.0
    for ax in range(3):
        diff = np.diff(m, axis=ax)
        s += np.sum(diff ** 2) / d[ax] ** 2
    assert np.isclose(ex, A * V * s, rtol=1e-12)


def test_vacuum_cells():
    """Ms = 0 cells carry no moment, feel no exchange and are no neighbours."""
    n = (4, 3, 2)
    m = synth.random_unit(n, 9)
    Ms = np.full(n, MS)
    Ms[1, 1, 0] = 0.0
    h = oracle.exchange_field(m, Ms, A, D2)
    assert np.all(h[1, 1, 0] == 0)
    # the neighbour (0,1,0) sees only its in-grid magnetic neighbours
    c = 2 * A / (oracle.MU0 * MS)
    e = c * ((m[0, 0, 0] - m[0, 1, 0]) + (m[0, 2, 0] - m[0, 1, 0]) + (m[0, 1, 1] - m[0, 1, 0])) / D2[0] ** 2
    assert np.allclose(h[0, 1, 0], e, rtol=1e-13)


def test_exchange_at_matches_field():
    n = (6, 5, 3)
    d = (2.5e-9, 2e-9, 3e-9)
    m = synth.random_unit(n, 1)
    Ms = synth.ms_field(n, 2)
    Ms[1, 1, 1] = 0.0
    cells = synth.sample_cells(n, 3, 12)
    full = oracle.exchange_field(m, Ms, A, d)
    assert np.array_equal(oracle.exchange_at(m, Ms, A, d, cells), full[cells[:, 0], cells[:, 1], cells[:, 2]])


# ---- DMI (eq. (3)) -----------------------------------------------------------
def test_dmi_uniform_is_zero():
    m = np.zeros((5, 4, 3, 3))
    m[..., 0] = 0.6
    m[..., 2] = 0.8
    d = (2e-9, 3e-9, 1e-9)
    for kind in ("interfacial", "bulk"):
        assert np.abs(oracle.dmi_field(m, 8e5, 3e-3, d, kind)).max() == 0.0


def _pref(D, Ms):
    return 2.0 * D / (oracle.MU0 * Ms)


def test_dmi_interfacial_cycloid_closed_form():
    """m = (sin kx, 0, cos kx): in the interior the central differences give
    dm/dx = sin(kd)/d (cos kx, 0, -sin kx), so eq. (3) with
    e^DMI = (e_y, -e_x, 0) gives h = -(2D/mu0 Ms) sin(kd)/d m."""
    nx, d, D, Ms, k = 24, (2e-9, 2e-9, 1e-9), 3e-3, 8e5, 2 * np.pi / 17e-9
    x = (np.arange(nx) + 0.5) * d[0]
    m = np.zeros((nx, 3, 1, 3))
    m[..., 0] = np.sin(k * x)[:, None, None]
    m[..., 2] = np.cos(k * x)[:, None, None]
    h = oracle.dmi_field(m, Ms, D, d, "interfacial")
    ref = -_pref(D, Ms) * np.sin(k * d[0]) / d[0] * m
    assert np.abs(h[1:-1] - ref[1:-1]).max() <= 1e-12 * np.abs(ref).max()
    # the same texture along z feels no interfacial DMI (e_z^DMI = 0)
    mz = np.transpose(m, (2, 1, 0, 3))
    assert np.abs(oracle.dmi_field(mz, Ms, D, d, "interfacial")).max() == 0.0


def test_dmi_bulk_helix_closed_form():
    """m = (cos kz, sin kz, 0) along z and m = (0, cos kx, sin kx) along x:
    bulk DMI (e^DMI = e_k) gives h = -(2D/mu0 Ms) sin(kd)/d m in the interior."""
    n, d, D, Ms, k = 20, (1.5e-9, 2e-9, 2.5e-9), 2e-3, 6e5, 2 * np.pi / 23e-9
    z = (np.arange(n) + 0.5) * d[2]
    m = np.zeros((2, 2, n, 3))
    m[..., 0] = np.cos(k * z)
    m[..., 1] = np.sin(k * z)
    h = oracle.dmi_field(m, Ms, D, d, "bulk")
    ref = -_pref(D, Ms) * np.sin(k * d[2]) / d[2] * m
    assert np.abs(h[:, :, 1:-1] - ref[:, :, 1:-1]).max() <= 1e-12 * np.abs(ref).max()
    x = (np.arange(n) + 0.5) * d[0]
    m = np.zeros((n, 2, 2, 3))
    m[..., 1] = np.cos(k * x)[:, None, None]
    m[..., 2] = np.sin(k * x)[:, None, None]
    h = oracle.dmi_field(m, Ms, D, d, "bulk")
    ref = -_pref(D, Ms) * np.sin(k * d[0]) / d[0] * m
    assert np.abs(h[1:-1] - ref[1:-1]).max() <= 1e-12 * np.abs(ref).max()
