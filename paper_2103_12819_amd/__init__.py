"""MI355X coupled Maxwell-LLG time stepper: Python binding of libmm.so.

The binding only marshals arguments to the C ABI of include/mm.h; every
step of the computation runs in the HIP kernels of the library.  PyTorch
supplies the device memory (through its caching allocator) and the stream.
If the library has not been built, constructing a Sim raises: there is no
CPU fallback.

Scheme: Yao, Jambunathan, Zeng & Nonaka, "A Massively Parallel Time-Domain
Coupled Electrodynamics-Micromagnetics Solver", Sec. 3.2.2.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np

from . import _native as N

FIELD_NAMES = ["Ex", "Ey", "Ez", "Hx", "Hy", "Hz",
               "Mxx", "Mxy", "Mxz", "Myx", "Myy", "Myz", "Mzx", "Mzy", "Mzz",
               "Bx", "By", "Bz"]
FIELD_ID = {n: i for i, n in enumerate(FIELD_NAMES)}


class MMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{N.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c64(a):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=np.float64)


class _TorchAlloc:
    """Device memory from torch's caching allocator on a given stream."""

    def __init__(self, stream_ptr):
        import torch
        self.torch = torch
        self.stream = int(stream_ptr or 0)
        self.alloc_fn = N.ALLOC_FN(self._alloc)
        self.free_fn = N.FREE_FN(self._free)

    def _alloc(self, size, ctx):
        try:
            return int(self.torch.cuda.caching_allocator_alloc(int(size), stream=self.stream))
        except Exception:  # allocation failure is reported by the library
            return None

    def _free(self, ptr, ctx):
        if not ptr:
            return
        cuda = getattr(self.torch, "cuda", None)
        fn = getattr(cuda, "caching_allocator_delete", None)
        if fn is not None:   # None only while the interpreter tears torch down
            fn(int(ptr))


class Sim:
    """One simulation context (mm_init ... mm_destroy).

    Arguments follow mm_init: grid cells `n`, spacings `d`, time step `dt`,
    cell maps in host layout (x fastest: numpy shape (nz, ny, nx)), bias
    `H0`, optional source (comp, profile, f0, Tp, t0), periodic flags,
    precision 'fp64' or 'fp32', tol, max_iter, fixed_iter, `scheme` 2
    (second-order, iterative) or 1 (first-order), and `pml`: None or
    (cells, R0, order), cells = layer thicknesses (x_lo, x_hi, y_lo, y_hi,
    z_lo, z_hi) (see mm_pml), `fused` 0 / 1 / -1 (automatic, on, off: see
    mm_options.fused).  `stream` is a raw hipStream_t (int) or None for
    torch's current stream.
    """

    def __init__(self, n, d, dt, eps_r=None, sigma=None, mu_r=None, Ms=None, alpha=None,
                 gamma=None, m0_dir=None, H0=(0.0, 0.0, 0.0), source=None,
                 periodic=(False, False, False), precision="fp64", tol=1e-10, max_iter=100,
                 fixed_iter=0, stream=None, torch_alloc=True, scheme=2, pml=None, fused=0):
        self._lib = N.load()
        self._ctx = C.c_void_p()
        g = N.mm_grid(int(n[0]), int(n[1]), int(n[2]),
                      (C.c_int32 * 3)(*[N.MM_BC_PERIODIC if p else N.MM_BC_PEC for p in periodic]),
                      float(d[0]), float(d[1]), float(d[2]))
        self.n = tuple(int(v) for v in n)
        self.d = tuple(float(v) for v in d)
        self.dt = float(dt)
        self.periodic = tuple(bool(p) for p in periodic)
        self._keep = [_c64(a) for a in (eps_r, sigma, mu_r, Ms, alpha, gamma, m0_dir)]
        mat = N.mm_materials(*[_dp(a) for a in self._keep])
        bias = N.mm_bias((C.c_double * 3)(*[float(v) for v in H0]))
        src_p = None
        if source is not None:
            comp, prof, f0, Tp, t0 = source
            self._prof = _c64(prof)
            src_p = C.byref(N.mm_source(int(comp), _dp(self._prof), float(f0), float(Tp), float(t0)))
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
        self.stream = int(stream or 0)
        opt = N.mm_options()
        opt.prec = N.MM_FP32 if precision == "fp32" else N.MM_FP64
        opt.tol = float(tol)
        opt.max_iter = int(max_iter)
        opt.fixed_iter = int(fixed_iter)
        opt.scheme = int(scheme)
        opt.fused = int(fused)
        if pml is not None:
            cells, R0, order = pml
            self._pml = N.mm_pml((C.c_int32 * 6)(*[int(v) for v in cells]), float(R0), float(order))
            opt.pml = C.pointer(self._pml)
        opt.hip_stream = self.stream or None
        self._alloc = None
        if torch_alloc:
            self._alloc = _TorchAlloc(self.stream)
            opt.dev_alloc = self._alloc.alloc_fn
            opt.dev_free = self._alloc.free_fn
        self.precision = precision
        st = self._lib.mm_init(C.byref(self._ctx), C.byref(g), float(dt), C.byref(mat), C.byref(bias),
                               src_p, C.byref(opt))
        if st != 0:
            raise MMError(st, "mm_init rejected the arguments")
        _LIVE.add(self)
        self._keep = None
        self._prof = None

    # -- helpers -------------------------------------------------------------
    def _check(self, st):
        if st != 0:
            msg = self._lib.mm_last_error(self._ctx)
            raise MMError(st, msg.decode() if msg else "")

    def nodes(self, ax):
        return self.n[ax] if self.periodic[ax] else self.n[ax] + 1

    def extent(self, field):
        """Host-layout shape (nz', ny', nx') of a field id or name."""
        fid = FIELD_ID[field] if isinstance(field, str) else int(field)
        if fid < 3:
            ext = [self.n[a] if a == fid else self.nodes(a) for a in range(3)]
        else:
            f = fid - 3 if fid < 6 else ((fid - 6) // 3 if fid < 15 else fid - 15)
            ext = [self.nodes(a) if a == f else self.n[a] for a in range(3)]
        return (ext[2], ext[1], ext[0])

    # -- API -------------------------------------------------------------------
    def add_probe(self, kind, field=0, i=0, j=0, k=0):
        pid = C.c_int32()
        self._check(self._lib.mm_add_probe(self._ctx, C.byref(N.mm_probe_desc(kind, field, i, j, k)),
                                           C.byref(pid)))
        return pid.value

    def add_hard_source(self, field, profile, f0, Tp, t0):
        """Hard source on field id 0-5 (Ex..Hz): see mm_add_hard_source."""
        fid = FIELD_ID[field] if isinstance(field, str) else int(field)
        prof = np.ascontiguousarray(profile, dtype=np.float64)
        if prof.shape != self.extent(fid):
            raise ValueError(f"profile shape {prof.shape} != {self.extent(fid)}")
        self._check(self._lib.mm_add_hard_source(self._ctx, C.byref(N.mm_hard_source(fid, _dp(prof), f0, Tp, t0))))

    def add_surface_current(self, axis, side, comp, profile, f0, Tp, t0):
        """Surface current J_s along `comp` on the PEC wall normal to `axis`
        (side 0: low end, 1: high end): see mm_add_surface_current."""
        prof = np.ascontiguousarray(profile, dtype=np.float64)
        if prof.shape != self.extent(int(comp)):
            raise ValueError(f"profile shape {prof.shape} != {self.extent(int(comp))}")
        self._check(self._lib.mm_add_surface_current(
            self._ctx, C.byref(N.mm_surface_current(axis, side, comp, _dp(prof), f0, Tp, t0))))

    def step(self, n=1):
        self._check(self._lib.mm_step(self._ctx, int(n)))

    def probe(self, pid):
        """(series, time integral) of a probe; synchronises."""
        cnt = C.c_size_t()
        self._check(self._lib.mm_probe(self._ctx, int(pid), None, 0, C.byref(cnt), None))
        out = np.zeros(cnt.value)
        s = C.c_double()
        self._check(self._lib.mm_probe(self._ctx, int(pid), _dp(out), out.size, C.byref(cnt), C.byref(s)))
        return out, s.value

    def field(self, name):
        fid = FIELD_ID[name] if isinstance(name, str) else int(name)
        out = np.zeros(self.extent(fid))
        self._check(self._lib.mm_get_field(self._ctx, fid, _dp(out)))
        return out

    def set_field(self, name, arr):
        fid = FIELD_ID[name] if isinstance(name, str) else int(name)
        a = np.ascontiguousarray(arr, dtype=np.float64)
        if a.shape != self.extent(fid):
            raise ValueError(f"{name}: expected shape {self.extent(fid)}, got {a.shape}")
        self._check(self._lib.mm_set_field(self._ctx, fid, _dp(a)))

    def field_tensor(self, name):
        """E or H component as a torch tensor on the device (storage precision,
        host-layout shape), filled on the context's stream without a host copy."""
        import torch
        fid = FIELD_ID[name] if isinstance(name, str) else int(name)
        if fid > 5:
            raise ValueError("device access covers E and H components only")
        dt = torch.float32 if self.precision == "fp32" else torch.float64
        with torch.cuda.stream(torch.cuda.ExternalStream(self.stream)) if self.stream else _nullctx():
            out = torch.empty(self.extent(fid), dtype=dt, device="cuda")
        self._check(self._lib.mm_get_field_device(self._ctx, fid, C.c_void_p(out.data_ptr())))
        return out

    def set_field_tensor(self, name, t):
        """Overwrite an E or H component from a contiguous device tensor of the
        storage precision and host-layout shape (PEC-pinned entries -> 0)."""
        import torch
        fid = FIELD_ID[name] if isinstance(name, str) else int(name)
        dt = torch.float32 if self.precision == "fp32" else torch.float64
        if t.dtype != dt or tuple(t.shape) != self.extent(fid) or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"expected a contiguous {dt} device tensor of shape {self.extent(fid)}")
        self._check(self._lib.mm_set_field_device(self._ctx, fid, C.c_void_p(t.data_ptr())))

    def set_fields(self, E=None, H=None):
        if E is not None:
            for c in range(3):
                self.set_field(c, E[c])
        if H is not None:
            for c in range(3):
                self.set_field(3 + c, H[c])

    def stats(self):
        """Iteration counts of every sub-step so far (raises on a sticky device condition)."""
        cnt = C.c_size_t()
        self._check(self._lib.mm_stats(self._ctx, None, 0, C.byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.int32)
        self._check(self._lib.mm_stats(self._ctx, out.ctypes.data_as(C.POINTER(C.c_int32)), out.size,
                                       C.byref(cnt)))
        return out

    def sync(self):
        self._check(self._lib.mm_sync(self._ctx))

    def info(self):
        out = (C.c_int64 * 8)()
        self._check(self._lib.mm_info(self._ctx, out))
        keys = ["n_mag", "n_wall_mag", "n_src", "px", "py", "pz", "elem_bytes", "device_bytes"]
        return dict(zip(keys, list(out)))

    def tiles(self):
        """Bulk tiling, its near/far split and the material-id mode (see mm_layout)."""
        out = (C.c_int64 * 8)()
        self._check(self._lib.mm_layout(self._ctx, out))
        keys = ["tiles", "near_tiles", "far_tiles", "near_cells", "far_cells", "planes_per_tile",
                "materials", "pml_tiles"]
        return dict(zip(keys, list(out)))

    def enable_adjoint(self, checkpoint_every=100, inner_every=0):
        """Save checkpoints while stepping so that adjoint() can run (before the
        first step); inner_every > 0 makes the adjoint two-level (see
        mm_adjoint_enable)."""
        self._check(self._lib.mm_adjoint_enable(self._ctx, int(checkpoint_every), int(inner_every)))

    def adjoint(self, probe_id):
        """Gradients (d L/d eps_r, d L/d Ms) as host-layout cell maps, where L is
        the time integral of flux probe `probe_id` over all steps taken."""
        shp = (self.n[2], self.n[1], self.n[0])
        ge = np.zeros(shp)
        gm = np.zeros(shp)
        self._check(self._lib.mm_adjoint(self._ctx, int(probe_id), _dp(ge), _dp(gm)))
        return ge, gm

    KERNEL_CLASSES = ["e_update", "h_bulk", "hm_pre", "hm_step", "hm_finish", "probes", "hm_commit", "h_far"]

    def profile(self, enable=True):
        """Bracket every later kernel launch with HIP events (see mm_profile)."""
        self._check(self._lib.mm_profile(self._ctx, 1 if enable else 0))

    def profile_read(self):
        """{class: (total ms, launches)} since the last read; synchronises."""
        ms = (C.c_double * 8)()
        cnt = (C.c_int64 * 8)()
        self._check(self._lib.mm_profile_read(self._ctx, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNEL_CLASSES)}

    def close(self):
        if self._ctx:
            self._lib.mm_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _close_all():
    """Close the contexts still open at exit, while torch is intact."""
    for sim in list(_LIVE):
        sim.close()


_LIVE = weakref.WeakSet()
atexit.register(_close_all)


def from_config(cfg, precision="fp64", fixed_iter=0, with_probes=True, **kw):
    """Build a Sim from a workloads.Config (same inputs the oracle takes)."""
    src = None
    if cfg.source is not None:
        s = cfg.source
        src = (s.comp, s.profile, s.f0, s.Tp, s.t0)
    sim = Sim(cfg.n, cfg.d, cfg.dt, eps_r=cfg.eps_r, sigma=cfg.sigma, mu_r=cfg.mu_r, Ms=cfg.Ms,
              alpha=cfg.alpha, gamma=cfg.gamma, m0_dir=cfg.m0_dir, H0=cfg.H0, source=src,
              periodic=cfg.periodic, precision=precision, tol=cfg.tol, max_iter=cfg.max_iter,
              fixed_iter=fixed_iter, **({"pml": cfg.pml} if cfg.pml is not None else {}), **kw)
    for h in cfg.hard_sources:
        sim.add_hard_source(h.field, h.profile, h.f0, h.Tp, h.t0)
    for sc in cfg.surface_currents:
        sim.add_surface_current(sc.axis, sc.side, sc.comp, sc.profile, sc.f0, sc.Tp, sc.t0)
    if cfg.E_init is not None or cfg.H_init is not None:
        sim.set_fields(cfg.E_init, cfg.H_init)
    if with_probes:
        for p in cfg.probes:
            sim.add_probe(p.kind, p.field, p.i, p.j, p.k)
    return sim


class FluxLoss:
    """torch.autograd.Function for L(eps_r, Ms) = time-integrated Poynting flux
    through a probe plane after `steps` steps of a workload.

        L = FluxLoss.apply(eps_r, Ms, cfg, steps, probe_id, precision, checkpoint_every)

    eps_r and Ms are host-layout (nz, ny, nx) float64 tensors (any device);
    every other input of `cfg` (a workloads.Config) is held fixed.  The forward
    runs the HIP path; backward calls mm_adjoint (reverse sweep with
    checkpoint-and-recompute) and scales the gradients by dL.
    """

    _fn = None

    @classmethod
    def apply(cls, *args):
        if cls._fn is None:
            cls._fn = _make_flux_loss()
        return cls._fn.apply(*args)


def _make_flux_loss():
    import torch

    class _FluxLossFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, eps_r, Ms, cfg, steps, probe_id, precision="fp64", checkpoint_every=100):
            import copy
            c2 = copy.copy(cfg)
            c2.eps_r = eps_r.detach().to("cpu", torch.float64).numpy()
            c2.Ms = Ms.detach().to("cpu", torch.float64).numpy()
            sim = from_config(c2, precision=precision)
            sim.enable_adjoint(checkpoint_every)
            sim.step(int(steps))
            _, L = sim.probe(int(probe_id))
            ctx.sim = sim
            ctx.probe_id = int(probe_id)
            ctx.devices = (eps_r.device, Ms.device)
            return torch.tensor(L, dtype=torch.float64, device=eps_r.device)

        @staticmethod
        def backward(ctx, dL):
            ge, gm = ctx.sim.adjoint(ctx.probe_id)
            ctx.sim.close()
            s = float(dL)
            g_eps = torch.from_numpy(ge * s).to(ctx.devices[0])
            g_ms = torch.from_numpy(gm * s).to(ctx.devices[1])
            return g_eps, g_ms, None, None, None, None, None

    return _FluxLossFn
