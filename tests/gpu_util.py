"""Helpers for the GPU parity tests (no method arithmetic here)."""
import numpy as np


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def to_dev(a, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rounded(a, dtype):
    """The values a GPU run of this dtype actually receives, as float64."""
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype).double().numpy()


def oracle_field_and_step(args):
    """Oracle h_eff (and, if asked, one RK4 step) of one geometry with its
    own tensor and 7-smooth padding (any L >= 2n-1 gives the same linear
    convolution); a process-pool worker, so it imports the oracle itself."""
    import oracle
    g, d, m0, Ms, A, step = args[:6]
    oct_ = oracle.tensor_octant(g, d)
    L = tuple(oracle.default_L(v) for v in g)
    h = oracle.h_eff(m0, Ms, A, d, oct_, L)
    s = None
    if step:
        alpha, gamma, dt = args[6:9]
        s = oracle.rk4_step(m0, Ms, A, d, oct_, L, alpha, gamma, dt)
    return h, s


def oracle_pool_map(fn, jobs, workers=8):
    """Map over a pool of fresh interpreters (spawned: the children never
    touch the GPU), largest jobs first."""
    import multiprocessing as mp
    import os
    from concurrent.futures import ProcessPoolExecutor
    n = max(1, min(workers, os.cpu_count() or 1, len(jobs)))
    with ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(fn, jobs))
