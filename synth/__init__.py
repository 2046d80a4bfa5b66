"""Seeded synthetic inputs shaped like the paper's workloads.

This module generates inputs only (random unit vectors, smooth textures,
grain structures, geometry lists, per-cell Ms); it holds none of the method's
arithmetic and is the one piece of code shared by the oracle-side tests and the
GPU-side tests and benchmark.  All generators use numpy's PCG64
``default_rng(seed)`` and return float64 arrays in the (nx, ny, nz, 3) layout.
"""
import numpy as np


def _normalise(v, rng):
    n = np.linalg.norm(v, axis=-1, keepdims=True)
    bad = n[..., 0] < 1e-12
    while np.any(bad):
        v[bad] = rng.standard_normal((int(bad.sum()), 3))
        n = np.linalg.norm(v, axis=-1, keepdims=True)
        bad = n[..., 0] < 1e-12
    return v / n


def random_unit(n, seed):
    """i.i.d. uniform directions on the sphere: normalised N(0, I) triples."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(tuple(int(x) for x in n) + (3,))
    return _normalise(v, rng)


def smooth_film(n, d, seed, noise=0.01, waves=6):
    """Smoothly varying in-plane texture plus noise:
    theta = pi/2 + 0.4 S1, phi = pi S2, with S1, S2 sums of ``waves`` seeded
    in-plane plane waves (wavelength U[40,200] nm, phase U[0,2pi), random
    direction), scaled so max|S| <= 1; then m = normalise(m0 + noise * xi),
    xi ~ N(0, I)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in n)
    x = (np.arange(nx) + 0.5) * d[0]
    y = (np.arange(ny) + 0.5) * d[1]
    X, Y = np.meshgrid(x, y, indexing="ij")
    S = []
    for _ in range(2):
        s = np.zeros((nx, ny))
        for _w in range(waves):
            lam = rng.uniform(40e-9, 200e-9)
            ang = rng.uniform(0, 2 * np.pi)
            ph = rng.uniform(0, 2 * np.pi)
            s += np.cos(2 * np.pi / lam * (np.cos(ang) * X + np.sin(ang) * Y) + ph)
        s /= max(np.abs(s).max(), 1e-300)
        S.append(s)
    theta = np.pi / 2 + 0.4 * S[0]
    phi = np.pi * S[1]
    m0 = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], -1)
    m0 = np.broadcast_to(m0[:, :, None, :], (nx, ny, nz, 3))
    v = m0 + noise * rng.standard_normal((nx, ny, nz, 3))
    return _normalise(v, rng)


def voronoi_grains(n, d, seed, spacing=20e-9, chunk=1 << 22, workers=-1):
    """3D non-periodic Voronoi grains: round(volume/spacing^3) seeds uniform in
    the box, every cell takes the grain of the seed nearest to its centre (ties
    to the lower seed index), each grain a uniform random unit vector."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in n)
    box = np.array([nx * d[0], ny * d[1], nz * d[2]])
    count = max(1, int(round(np.prod(box) / spacing ** 3)))
    seeds = rng.uniform(0, 1, (count, 3)) * box
    dirs = _normalise(rng.standard_normal((count, 3)), rng)
    tree = cKDTree(seeds)
    out = np.empty((nx, ny, nz, 3))
    flat = out.reshape(-1, 3)
    total = nx * ny * nz
    for s in range(0, total, chunk):
        idx = np.arange(s, min(total, s + chunk))
        i, r = np.divmod(idx, ny * nz)
        j, k = np.divmod(r, nz)
        pts = np.stack([(i + 0.5) * d[0], (j + 0.5) * d[1], (k + 0.5) * d[2]], 1)
        _, g = tree.query(pts, k=1, workers=workers)
        flat[s:s + len(idx)] = dirs[g]
    return out


def batch_geometries(seed, count=64, nxy=(48, 384), nz=(1, 8), ms=(4e5, 1.2e6)):
    """Parameter-sweep geometries: in-plane sizes U{48..384}, thickness
    U{1..8} cells, Ms U[4e5, 1.2e6] A/m.  Returns a list of (grid, Ms)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        g = (int(rng.integers(nxy[0], nxy[1] + 1)), int(rng.integers(nxy[0], nxy[1] + 1)),
             int(rng.integers(nz[0], nz[1] + 1)))
        out.append((g, float(rng.uniform(ms[0], ms[1]))))
    return out


def ms_field(n, seed, ms0=8e5, spread=0.05):
    """Per-cell Ms = ms0 (1 + spread xi), xi ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    return ms0 * (1.0 + spread * rng.uniform(-1.0, 1.0, tuple(int(v) for v in n)))


def sample_cells(n, seed, count=16):
    """``count`` distinct cell indices (K,3) drawn without replacement."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in n)
    flat = rng.choice(nx * ny * nz, size=count, replace=False)
    i, r = np.divmod(flat, ny * nz)
    j, k = np.divmod(r, nz)
    return np.stack([i, j, k], 1)
