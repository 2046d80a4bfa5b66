"""Plans, batches and autograd wrappers over the C ABI (marshalling only)."""
import ctypes

import torch

from . import _lib
from ._lib import MM_DEMAG, MM_EXCHANGE, MM_F32, MM_F64, MM_NO_GRAPH, MM_NO_RENORM, PlanOpts, check

_DT = {MM_F32: torch.float32, MM_F64: torch.float64}


def _prec(precision):
    if precision in (MM_F32, "f32", "float32", torch.float32):
        return MM_F32
    if precision in (MM_F64, "f64", "float64", torch.float64):
        return MM_F64
    raise ValueError("precision must be f32 or f64")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


_PADDING = {"auto": 2, "smooth": 0, "pow2": 1, "ct": 3}


def _opts(far_radius=16.0, L=None, autotune=False, padding="auto"):
    opts = PlanOpts()
    check(_lib.lib().mm_plan_opts_default(ctypes.byref(opts)))
    opts.far_radius = float(far_radius)
    opts.pow2_padding = _PADDING[padding]
    if L is not None:
        for a in range(3):
            opts.L[a] = int(L[a])
    opts.autotune = _tune_mode(autotune)
    return opts


_TUNE = {"off": 0, "cached": 1, "search": 2}


def _tune_mode(autotune):
    """False/"off" -> 0, True/"cached" -> 1 (recorded winners, time on a
    miss), "search" -> 2 (always time)."""
    if isinstance(autotune, str):
        return _TUNE[autotune]
    return 1 if autotune else 0


def _schedule(fn, h):
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    check(fn(h, buf, len(buf)))
    return json.loads(buf.value.decode())


RK4_IMAG_LIMIT = 2.0 * 2.0 ** 0.5   # classic RK4 is stable on the imaginary axis up to 2 sqrt(2)
_warned = set()


def llg_stability(cell, Ms_min, A, gamma, dt):
    """omega_max * dt of the exchange term on a grid of this cell size
    (mm_llg_stability, host only); above RK4_IMAG_LIMIT the step diverges."""
    c = (ctypes.c_double * 3)(*[float(v) for v in cell])
    out = ctypes.c_double()
    check(_lib.lib().mm_llg_stability(c, float(Ms_min), float(A), float(gamma), float(dt), ctypes.byref(out)))
    return out.value


def _stability_warning(cell, Ms, A, gamma, dt):
    key = (tuple(cell), float(Ms), float(A), float(gamma), float(dt))
    if key in _warned:
        return
    _warned.add(key)
    w = llg_stability(cell, Ms, A, gamma, dt)
    if w > RK4_IMAG_LIMIT:
        import warnings
        warnings.warn("llg_step: omega_max*dt = %.3g exceeds RK4's stability limit %.3f (cell %s, Ms %g, dt %g): "
                      "the step will diverge; reduce dt" % (w, RK4_IMAG_LIMIT, tuple(cell), Ms, dt), RuntimeWarning,
                      stacklevel=3)


def plan_bytes(grid, precision="f32", far_radius=16.0, L=None, padding="auto"):
    """(tensor_bytes, workspace_bytes) of a plan for this grid (no GPU call)."""
    opts = _opts(far_radius, L, padding=padding)
    g = (ctypes.c_int64 * 3)(*[int(v) for v in grid])
    t, w = ctypes.c_size_t(), ctypes.c_size_t()
    check(_lib.lib().mm_plan_bytes(g, _prec(precision), ctypes.byref(opts), ctypes.byref(t), ctypes.byref(w)))
    return t.value, w.value


def plan_scratch_bytes(grid, precision="f32", far_radius=16.0, L=None, padding="auto"):
    """Scratch bytes per call of (the adjoint entry points, the RKF45 step,
    the minimiser) for this grid (no GPU call)."""
    opts = _opts(far_radius, L, padding=padding)
    g = (ctypes.c_int64 * 3)(*[int(v) for v in grid])
    out = (ctypes.c_size_t * 3)()
    check(_lib.lib().mm_plan_scratch_bytes(g, _prec(precision), ctypes.byref(opts), out))
    return tuple(out)


class DemagPlan:
    """One geometry: grid (nx,ny,nz), cell (dx,dy,dz) in metres, FP32 or FP64.
    Creating it computes the Newell tensor spectrum on the GPU (FP64)."""

    def __init__(self, grid, cell, precision="f32", far_radius=16.0, L=None, autotune=False, padding="auto"):
        self.grid = tuple(int(v) for v in grid)
        self.cell = tuple(float(v) for v in cell)
        self.prec = _prec(precision)
        self.dtype = _DT[self.prec]
        self._far, self._L, self._pad = float(far_radius), L, padding
        self._attached = None
        opts = _opts(far_radius, L, autotune, padding)
        g = (ctypes.c_int64 * 3)(*self.grid)
        c = (ctypes.c_double * 3)(*self.cell)
        self._h = ctypes.c_void_p()
        self.device = torch.device("cuda", torch.cuda.current_device())
        check(_lib.lib().demag_tensor_init(ctypes.byref(self._h), g, c, self.prec, _stream(), ctypes.byref(opts)))

    # -- helpers --------------------------------------------------------------
    def _vec(self, t, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != self.dtype:
            raise TypeError("%s must be a CUDA %s tensor" % (name, self.dtype))
        if tuple(t.shape) != self.grid + (3,) or not t.is_contiguous():
            raise ValueError("%s must be contiguous with shape %s" % (name, self.grid + (3,)))
        return t

    def _ms(self, Ms):
        if isinstance(Ms, torch.Tensor):
            if Ms.device.type != "cuda" or Ms.dtype != self.dtype or tuple(Ms.shape) != self.grid or not Ms.is_contiguous():
                raise ValueError("per-cell Ms must be a contiguous CUDA %s tensor of shape %s" % (self.dtype, self.grid))
            return Ms, 0.0
        return None, float(Ms)

    def _sync_stream(self):
        check(_lib.lib().mm_plan_set_stream(self._h, _stream()))

    # -- API ------------------------------------------------------------------
    def set_dmi(self, kind, D):
        """Add the DMI field of eq. (3) to every later field evaluation:
        kind "interfacial" or "bulk" (or None / D = 0 to remove it), D in J/m^2."""
        k = {None: 0, "none": 0, "interfacial": 1, "bulk": 2}[kind]
        self._sync_stream()
        check(_lib.lib().mm_plan_set_dmi(self._h, k, float(D)))

    def set_anisotropy(self, Ku, axis=(0.0, 0.0, 1.0)):
        """Add the uniaxial anisotropy field 2 Ku/(mu0 Ms) (m.u) u to every
        later field evaluation (Ku = 0 removes it)."""
        self._sync_stream()
        ax = (ctypes.c_double * 3)(*[float(v) for v in axis])
        check(_lib.lib().mm_plan_set_anisotropy(self._h, float(Ku), ax))

    def set_stt(self, j, P=0.4, Lambda=1.0, eps_prime=0.0, d_layer=1e-9, p=(0.0, 0.0, 1.0)):
        """Add the Slonczewski spin-transfer torque as an effective field,
        beta (eps(m.p) (m x p) + eps_prime p), beta = hbar j/(mu0 e Ms d_layer),
        eps(x) = P Lambda^2/((Lambda^2+1) + (Lambda^2-1) x), to every later
        field evaluation (j = 0 removes it)."""
        self._sync_stream()
        pv = (ctypes.c_double * 3)(*[float(v) for v in p])
        check(_lib.lib().mm_plan_set_stt(self._h, float(j), float(P), float(Lambda), float(eps_prime),
                                         float(d_layer), pv))

    def attach_memory(self, scratch=("adjoint", "rkf45", "minimize")):
        """Move the plan's tensor spectrum and workspace into torch-owned
        device buffers, and give it a torch-owned scratch region large enough
        for the listed entry points ("adjoint": llg_step_adjoint, "rkf45",
        "minimize"; empty: none, and those calls then fail): torch's caching
        allocator then
        holds all of the plan's device memory.  Returns the uint8 tensors
        (tensor, workspace, scratch or None), which the plan keeps alive
        until close()."""
        tb, wb = plan_bytes(self.grid, self.prec, self._far, self._L, self._pad)
        need = plan_scratch_bytes(self.grid, self.prec, self._far, self._L, self._pad)
        which = {"adjoint": 0, "rkf45": 1, "minimize": 2}
        sb = max([need[which[k]] for k in scratch], default=0)
        # 256-byte alignment: torch's CUDA allocator returns 512-byte aligned blocks
        t = torch.empty(max(tb, 1), dtype=torch.uint8, device=self.device)
        w = torch.empty(max(wb, 1), dtype=torch.uint8, device=self.device)
        sc = torch.empty(sb, dtype=torch.uint8, device=self.device) if sb else None
        self._sync_stream()
        torch.cuda.current_stream().synchronize()
        check(_lib.lib().mm_plan_attach_memory(self._h, _ptr(t), _ptr(w)))
        if sc is not None:
            check(_lib.lib().mm_plan_attach_scratch(self._h, _ptr(sc), sb))
        self._attached = (t, w, sc)
        return t, w, sc

    def info(self):
        L = (ctypes.c_int64 * 3)()
        b = ctypes.c_size_t()
        t = (ctypes.c_int * 5)()
        check(_lib.lib().mm_plan_info(self._h, L, ctypes.byref(b), t))
        return {"L": tuple(L), "device_bytes": b.value, "tiles": tuple(t)}

    def schedule(self):
        """The launch schedule the plan runs (mm_plan_schedule), as a dict."""
        return _schedule(_lib.lib().mm_plan_schedule, self._h)

    def h_eff(self, m, Ms, A, out=None, terms=MM_DEMAG | MM_EXCHANGE, energy=False):
        self._vec(m, "m")
        Mst, Mss = self._ms(Ms)
        if out is None:
            out = torch.empty_like(m)
        self._vec(out, "out")
        self._sync_stream()
        E = (ctypes.c_double * 2)() if energy else None
        check(_lib.lib().h_eff(self._h, _ptr(m), _ptr(Mst), Mss, float(A), _ptr(out), int(terms), E))
        return (out, (E[0], E[1])) if energy else out

    def llg_step(self, m, Ms, A, alpha, gamma, dt, n_steps=1, h_ext=None, renorm=True, graph=True):
        self._vec(m, "m")
        Mst, Mss = self._ms(Ms)
        if Mst is None and Mss > 0:
            _stability_warning(self.cell, Mss, A, gamma, dt)
        self._sync_stream()
        he = (ctypes.c_double * 3)(*[float(v) for v in h_ext]) if h_ext is not None else None
        flags = (0 if renorm else MM_NO_RENORM) | (0 if graph else MM_NO_GRAPH)
        check(_lib.lib().llg_step(self._h, _ptr(m), _ptr(Mst), Mss, float(A), float(alpha), float(gamma), float(dt),
                                  int(n_steps), he, flags))
        return m

    def rkf45_step(self, m, Ms, A, alpha, gamma, dt, tol, h_ext=None, renorm=True):
        """One attempted RKF45 step (in place on acceptance).  Returns
        (accepted, err, dt_next)."""
        self._vec(m, "m")
        Mst, Mss = self._ms(Ms)
        self._sync_stream()
        he = (ctypes.c_double * 3)(*[float(v) for v in h_ext]) if h_ext is not None else None
        d = ctypes.c_double(float(dt))
        err = ctypes.c_double()
        ok = ctypes.c_int()
        check(_lib.lib().llg_rkf45_step(self._h, _ptr(m), _ptr(Mst), Mss, float(A), float(alpha), float(gamma),
                                        ctypes.byref(d), float(tol), he, 0 if renorm else MM_NO_RENORM,
                                        ctypes.byref(err), ctypes.byref(ok)))
        return bool(ok.value), err.value, d.value

    def rkf45_run(self, m, Ms, A, alpha, gamma, t_end, dt0, tol, h_ext=None, renorm=True, max_attempts=100000):
        """Adaptive integration to t_end (the last step lands on it).
        Returns (accepted steps, rejected attempts, last dt)."""
        t, dt, acc, rej = 0.0, float(dt0), 0, 0
        for _ in range(max_attempts):
            if t >= t_end:
                break
            h = min(dt, t_end - t)
            ok, _, dt = self.rkf45_step(m, Ms, A, alpha, gamma, h, tol, h_ext, renorm)
            if ok:
                t, acc = t + h, acc + 1
            else:
                rej += 1
        return acc, rej, dt

    def minimize(self, m, Ms, A, tol=1.0, max_iter=10000, h_ext=None):
        """Barzilai-Borwein energy minimisation in place.  Returns
        (iterations, final max torque |m x h| in A/m)."""
        self._vec(m, "m")
        Mst, Mss = self._ms(Ms)
        self._sync_stream()
        he = (ctypes.c_double * 3)(*[float(v) for v in h_ext]) if h_ext is not None else None
        it = ctypes.c_int()
        tq = ctypes.c_double()
        check(_lib.lib().mm_minimize_bb(self._h, _ptr(m), _ptr(Mst), Mss, float(A), he, float(tol), int(max_iter),
                                        ctypes.byref(it), ctypes.byref(tq)))
        return it.value, tq.value

    def h_eff_adjoint(self, m, Ms, A, g_h, terms=MM_DEMAG | MM_EXCHANGE, want_Ms=True):
        self._vec(m, "m")
        self._vec(g_h, "g_h")
        Mst, Mss = self._ms(Ms)
        g_m = torch.empty_like(m)
        g_Ms = torch.empty(self.grid, dtype=self.dtype, device=m.device) if want_Ms else None
        self._sync_stream()
        check(_lib.lib().h_eff_adjoint(self._h, _ptr(m), _ptr(Mst), Mss, float(A), _ptr(g_h), _ptr(g_m), _ptr(g_Ms),
                                       int(terms)))
        return g_m, g_Ms

    def llg_step_adjoint(self, m, Ms, A, alpha, gamma, dt, g, g_Ms=None, h_ext=None, renorm=True):
        """In place: g <- cotangent of m(t) from that of m(t+dt); g_Ms += ..."""
        self._vec(m, "m")
        self._vec(g, "g")
        Mst, Mss = self._ms(Ms)
        self._sync_stream()
        he = (ctypes.c_double * 3)(*[float(v) for v in h_ext]) if h_ext is not None else None
        flags = 0 if renorm else MM_NO_RENORM
        check(_lib.lib().llg_step_adjoint(self._h, _ptr(m), _ptr(Mst), Mss, float(A), float(alpha), float(gamma),
                                          float(dt), he, flags, _ptr(g), _ptr(g_Ms)))
        return g

    def llg_step_adjoint_noalloc(self, m, Ms, A, alpha, gamma, dt, g, g_Ms=None, h_ext=None, renorm=True):
        """llg_step_adjoint with its recorded fields in the library's fixed
        per-GPU array: no device allocation (calls overlapping on one GPU race)."""
        self._vec(m, "m")
        self._vec(g, "g")
        Mst, Mss = self._ms(Ms)
        self._sync_stream()
        he = (ctypes.c_double * 3)(*[float(v) for v in h_ext]) if h_ext is not None else None
        flags = 0 if renorm else MM_NO_RENORM
        check(_lib.lib().llg_step_adjoint_noalloc(self._h, _ptr(m), _ptr(Mst), Mss, float(A), float(alpha),
                                                  float(gamma), float(dt), he, flags, _ptr(g), _ptr(g_Ms)))
        return g

    def tensor_get(self):
        import numpy as np
        out = np.zeros(self.grid + (6,))
        check(_lib.lib().mm_demag_tensor_get(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def tensor_set(self, octant):
        import numpy as np
        a = np.ascontiguousarray(octant, dtype=np.float64)
        if a.shape != self.grid + (6,):
            raise ValueError("octant must have shape %s" % (self.grid + (6,),))
        check(_lib.lib().mm_demag_tensor_set(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def spectrum_get(self):
        import numpy as np
        L = self.info()["L"]
        out = np.zeros((L[0] // 2 + 1, L[1] // 2 + 1, L[2] // 2 + 1, 6))
        check(_lib.lib().mm_demag_spectrum_get(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lib().mm_plan_destroy(self._h)   # synchronises the plan's stream
            self._h = ctypes.c_void_p()
        self._attached = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent geometries advanced by grouped launches (one HIP graph
    per step of all of them)."""

    def __init__(self, grids, cells, precision="f32", far_radius=16.0, pow2_padding=True, autotune=False,
                 padding=None):
        """padding: "pow2" (the default, as pow2_padding=True), "smooth" (as
        pow2_padding=False), "ct" (shortest length with compile-time
        kernels: powers of two and q*2^k with q = 3, 5, 7) or "auto"."""
        self.grids = [tuple(int(v) for v in g) for g in grids]
        self.cells = [tuple(float(v) for v in c) for c in cells]
        self.prec = _prec(precision)
        self.dtype = _DT[self.prec]
        n = len(self.grids)
        G = (ctypes.c_int64 * (3 * n))(*[v for g in self.grids for v in g])
        C = (ctypes.c_double * (3 * n))(*[v for c in self.cells for v in c])
        opts = PlanOpts()
        check(_lib.lib().mm_plan_opts_default(ctypes.byref(opts)))
        opts.far_radius = float(far_radius)
        opts.pow2_padding = _PADDING[padding] if padding is not None else (1 if pow2_padding else 0)
        opts.autotune = _tune_mode(autotune)
        self._h = ctypes.c_void_p()
        check(_lib.lib().mm_batch_create(ctypes.byref(self._h), n, G, C, self.prec, _stream(), ctypes.byref(opts)))

    def _ptrs(self, ts):
        for t, g in zip(ts, self.grids):
            if t.dtype != self.dtype or tuple(t.shape) != g + (3,) or not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError("batch tensors must be contiguous CUDA %s of shape (nx,ny,nz,3)" % self.dtype)
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def info(self):
        n = ctypes.c_int64()
        b = ctypes.c_size_t()
        check(_lib.lib().mm_batch_info(self._h, ctypes.byref(n), ctypes.byref(b)))
        return {"total_cells": n.value, "device_bytes": b.value}

    def schedule(self):
        """The launch groups the batch runs (mm_batch_schedule), as a dict."""
        return _schedule(_lib.lib().mm_batch_schedule, self._h)

    def h_eff(self, ms, Ms, A, outs=None, terms=MM_DEMAG | MM_EXCHANGE):
        if outs is None:
            outs = [torch.empty_like(m) for m in ms]
        M = (ctypes.c_double * len(ms))(*[float(v) for v in Ms])
        check(_lib.lib().mm_batch_h_eff(self._h, self._ptrs(ms), M, float(A), self._ptrs(outs), int(terms)))
        return outs

    def llg_step(self, ms, Ms, A, alpha, gamma, dt, n_steps=1, renorm=True, graph=True):
        M = (ctypes.c_double * len(ms))(*[float(v) for v in Ms])
        flags = (0 if renorm else MM_NO_RENORM) | (0 if graph else MM_NO_GRAPH)
        check(_lib.lib().mm_batch_llg_step(self._h, self._ptrs(ms), M, float(A), float(alpha), float(gamma), float(dt),
                                           int(n_steps), flags))
        return ms

    def tensor_set(self, k, octant):
        """Replace geometry k's tensor by the transform of a real-space FP64
        octant (nx,ny,nz,6) of that geometry (the parity tests' hook)."""
        import numpy as np
        a = np.ascontiguousarray(octant, dtype=np.float64)
        if a.shape != self.grids[k] + (6,):
            raise ValueError("octant must have shape %s" % (self.grids[k] + (6,),))
        check(_lib.lib().mm_batch_tensor_set(self._h, int(k), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.lib().mm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HEff(torch.autograd.Function):
    """h = h_eff(m, Ms) with its backward through the hand-written adjoint."""

    @staticmethod
    def forward(ctx, m, Ms, plan, A, terms=MM_DEMAG | MM_EXCHANGE):
        mc = m.contiguous()
        Msc = Ms.contiguous() if isinstance(Ms, torch.Tensor) else None
        h = plan.h_eff(mc, Msc if Msc is not None else Ms, A, terms=terms)
        ctx.save_for_backward(mc, Msc)
        ctx.plan, ctx.A, ctx.terms, ctx.Ms_scalar = plan, A, terms, None if Msc is not None else Ms
        return h

    @staticmethod
    def backward(ctx, g):
        m, Ms = ctx.saved_tensors
        Msv = Ms if Ms is not None else ctx.Ms_scalar
        g_m, g_Ms = ctx.plan.h_eff_adjoint(m, Msv, ctx.A, g.contiguous(), terms=ctx.terms, want_Ms=Ms is not None)
        return g_m, g_Ms, None, None, None


class _LLGRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m0, Ms, plan, A, alpha, gamma, dt, n_steps, every):
        m = m0.detach().clone()
        ckpts = []
        done = 0
        while done < n_steps:
            k = min(every, n_steps - done)
            ckpts.append((done, m.clone()))
            plan.llg_step(m, Ms, A, alpha, gamma, dt, n_steps=k)
            done += k
        ctx.save_for_backward(Ms)
        ctx.ckpts, ctx.args = ckpts, (plan, A, alpha, gamma, dt, n_steps)
        return m

    @staticmethod
    def backward(ctx, g_out):
        (Ms,) = ctx.saved_tensors
        plan, A, alpha, gamma, dt, n_steps = ctx.args
        g = g_out.detach().contiguous().clone()
        gMs = torch.zeros_like(Ms)
        starts = [s for s, _ in ctx.ckpts] + [n_steps]
        # the recompute steps all run on one work buffer, so the step's graph
        # (keyed by the m pointer) is captured once for the whole backward
        work = torch.empty_like(g)
        states = None
        for seg in range(len(ctx.ckpts) - 1, -1, -1):
            start, ck = ctx.ckpts[seg]
            end = starts[seg + 1]
            # states m_start .. m_{end-1} of this segment, recomputed from its checkpoint
            if states is None or states.shape[0] < end - start:
                states = torch.empty((end - start,) + tuple(g.shape), dtype=g.dtype, device=g.device)
            states[0].copy_(ck)
            work.copy_(ck)
            for i in range(1, end - start):
                plan.llg_step(work, Ms, A, alpha, gamma, dt, n_steps=1)
                states[i].copy_(work)
            for i in range(end - start - 1, -1, -1):
                plan.llg_step_adjoint(states[i], Ms, A, alpha, gamma, dt, g, gMs)
        return g, gMs, None, None, None, None, None, None, None


def llg_run_checkpointed(plan, m0, Ms, A, alpha, gamma, dt, n_steps, every=20):
    """m after n_steps RK4 steps, differentiable w.r.t. m0 and per-cell Ms;
    the backward pass recomputes each segment of `every` steps from its
    checkpoint and reverses it with llg_step_adjoint."""
    return _LLGRun.apply(m0, Ms, plan, A, alpha, gamma, dt, int(n_steps), int(every))
