"""ctypes binding of libmm.so (the C ABI in include/mm.h).

Argument marshalling only: every step of the scheme runs in the library's HIP
kernels.  There is no fallback: if libmm.so is missing or fails to load, the
import of this module raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmm.so")

MM_OK, MM_EINVAL, MM_ENOMEM, MM_EDEVICE, MM_ENONPHYS, MM_ESTATE = range(6)
BC = {"extrap": 0, "periodic": 1, "wall": 2, "inflow": 3}
TAU = {"rho": 0, "p": 1, "hs1d": 2, "const": 3}
PROJ = {"discrete": 0, "paper": 1}
CFL = {"min": 0, "sum": 1}
PRECISION = {"fp64": 0, "mixed": 1, "closure": 2}
SOURCE = {"none": 0, "mms": 1}

# every entry point declared in include/mm.h
EXPORTS = ("mm_init", "mm_step", "mm_step_async", "mm_sync", "mm_moments", "mm_get_g", "mm_set_state",
           "mm_free", "mm_dt", "mm_failed_step", "mm_strerror", "mm_timing", "mm_timing_get", "mm_device_ptrs",
           "mm_get_g_cells", "mm_mlp_create", "mm_mlp_free", "mm_mlp_fit_norm", "mm_mlp_get", "mm_mlp_set",
           "mm_mlp_forward", "mm_mlp_grad", "mm_mlp_train", "mm_closure_attach", "mm_closure_cells",
           "mm_closure_snapshot", "mm_closure_features", "mm_closure_rebuild", "mm_step2d_noalloc",
           "mm_set_source")

MLP_NPARAM = 6599
MLP_NNORM = 74
N_FEAT, N_OUT = 30, 7


class MMError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {_lib.mm_strerror(code).decode()} (status {code})")
        self.code = code


class NonPhysical(MMError):
    pass


class mm_bc(C.Structure):
    _fields_ = [("kind", C.c_int), ("T_wall", C.c_double), ("u_wall", C.c_double),
                ("rho", C.c_double), ("u1", C.c_double), ("u2", C.c_double), ("T", C.c_double)]


class mm_config(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nv1", C.c_int), ("nv2", C.c_int),
                ("x_lo", C.c_double), ("x_hi", C.c_double), ("y_lo", C.c_double), ("y_hi", C.c_double),
                ("v1_lo", C.c_double), ("v1_hi", C.c_double), ("v2_lo", C.c_double), ("v2_hi", C.c_double),
                ("eps", C.c_double), ("cfl", C.c_double), ("cfl_rule", C.c_int), ("nu", C.c_double),
                ("tau_model", C.c_int), ("tau_coef", C.c_double), ("bc", mm_bc * 4),
                ("proj_mode", C.c_int), ("wall_es_term", C.c_int), ("dt", C.c_double),
                ("precision", C.c_int), ("device", C.c_int), ("stream", C.c_void_p),
                ("dev_buffers", C.c_void_p * 3)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    # torch ships its own HIP runtime: load it first, so that this library binds to
    # the runtime that owns the device tensors it is handed (loaded the other way
    # round, the process holds two runtimes and mm_init fails)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    cp = C.POINTER(mm_config)
    L.mm_init.argtypes = [cp, dp, dp, C.POINTER(vp)]
    L.mm_step.argtypes = [vp, C.c_int]
    L.mm_step_async.argtypes = [vp, C.c_int]
    L.mm_sync.argtypes = [vp]
    L.mm_moments.argtypes = [vp, dp, dp, dp]
    L.mm_get_g.argtypes = [vp, dp]
    L.mm_get_g_cells.argtypes = [vp, C.POINTER(C.c_int), C.c_int, dp]
    L.mm_set_state.argtypes = [vp, dp, dp]
    L.mm_free.argtypes = [vp]
    L.mm_free.restype = None
    L.mm_dt.argtypes = [cp, C.c_double, C.POINTER(C.c_int)]
    L.mm_dt.restype = C.c_double
    L.mm_failed_step.argtypes = [vp]
    L.mm_strerror.argtypes = [C.c_int]
    L.mm_strerror.restype = C.c_char_p
    L.mm_timing.argtypes = [vp, C.c_int]
    L.mm_timing_get.argtypes = [vp, C.c_int, C.POINTER(C.c_int), dp]
    L.mm_device_ptrs.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int)]
    fp = C.POINTER(C.c_float)
    bp = C.POINTER(C.c_ubyte)
    L.mm_mlp_create.argtypes = [C.c_int, vp, C.c_ulonglong, C.POINTER(vp)]
    L.mm_mlp_free.argtypes = [vp]
    L.mm_mlp_free.restype = None
    L.mm_mlp_fit_norm.argtypes = [vp, vp, vp, C.c_int]
    L.mm_mlp_get.argtypes = [vp, fp, fp]
    L.mm_mlp_set.argtypes = [vp, fp, fp]
    L.mm_mlp_forward.argtypes = [vp, vp, C.c_int, vp]
    L.mm_mlp_grad.argtypes = [vp, vp, vp, C.c_int, fp, dp]
    L.mm_mlp_train.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_ulonglong, dp]
    L.mm_closure_attach.argtypes = [vp, vp, C.c_double, C.c_int]
    L.mm_closure_cells.argtypes = [vp, C.POINTER(C.c_longlong), bp]
    L.mm_closure_snapshot.argtypes = [vp, C.c_double, C.c_int, vp, vp, C.c_int, C.POINTER(C.c_int)]
    L.mm_closure_features.argtypes = [vp, fp, fp, bp]
    L.mm_closure_rebuild.argtypes = [vp, fp, bp]
    L.mm_step2d_noalloc.argtypes = [cp, vp, vp, vp, vp, C.c_int, C.POINTER(C.c_int)]
    L.mm_set_source.argtypes = [vp, C.c_int, C.c_double]
    for name in EXPORTS:
        getattr(L, name)
    return L


_lib = _load()


def lib():
    return _lib


def config(p, stream=None, device=0, dev_buffers=None):
    """mm_config from a problem dictionary (see mm_workloads); dev_buffers: None or the
    device addresses (G0, G1, Q) of caller-owned buffers."""
    c = mm_config()
    c.dim = p["dim"]
    c.nx, c.ny = p["nx"], p.get("ny", 1)
    c.nv1, c.nv2 = p["nv1"], p.get("nv2", 1)
    c.x_lo, c.x_hi = p["x"]
    c.y_lo, c.y_hi = p.get("y", (0.0, 1.0))
    c.v1_lo, c.v1_hi = p["v1"]
    c.v2_lo, c.v2_hi = p.get("v2", (0.0, 1.0))
    c.eps, c.cfl = p["eps"], p["cfl"]
    c.cfl_rule = CFL[p.get("cfl_rule", "min")]
    c.nu = p.get("nu", 0.0)
    c.tau_model = TAU[p["tau_model"]]
    c.tau_coef = p["tau_coef"]
    for s, b in enumerate(p["bc"]):
        c.bc[s].kind = BC[b["kind"]]
        c.bc[s].T_wall = b.get("T_wall", 1.0)
        c.bc[s].u_wall = b.get("u_wall", 0.0)
        c.bc[s].rho = b.get("rho", 1.0)
        c.bc[s].u1 = b.get("u1", 0.0)
        c.bc[s].u2 = b.get("u2", 0.0)
        c.bc[s].T = b.get("T", 1.0)
    c.proj_mode = PROJ[p.get("proj_mode", "discrete")]
    c.wall_es_term = 1 if p.get("wall_es_term", True) else 0
    c.dt = p.get("dt", 0.0)
    c.precision = PRECISION[p.get("precision", "fp64")]
    c.device = device
    c.stream = stream
    if dev_buffers is not None:
        for k in range(3):
            c.dev_buffers[k] = dev_buffers[k]
    return c


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else None


def _bp(a):
    return a.ctypes.data_as(C.POINTER(C.c_ubyte)) if a is not None else None


def _dev(t, cols):
    """Device address of a contiguous float32 GPU tensor with `cols` columns."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError("expected a contiguous float32 tensor on the GPU")
    if t.dim() != 2 or t.shape[1] != cols:
        raise ValueError(f"expected shape [n, {cols}], got {tuple(t.shape)}")
    return t.data_ptr()


def _check(rc, what):
    if rc == MM_ENONPHYS:
        raise NonPhysical(rc, what)
    if rc != MM_OK:
        raise MMError(rc, what)


def dt(p, t_final=0.0):
    n = C.c_int(0)
    d = _lib.mm_dt(C.byref(config(p)), float(t_final), C.byref(n))
    if d < 0:
        raise MMError(MM_EINVAL, "mm_dt")
    return d, n.value


NOALLOC_MAX_CELLS = 65536


def step2d_noalloc(p, q, g0, g1, nsteps, h=None, stream=None, device=0, wait=True):
    """mm_step2d_noalloc on caller-owned device tensors: q float64 [ny, nx, 6] (in/out),
    g0 / g1 the two G buffers (float64 for fp64, float32 for mixed; g0 holds G^n, the
    result is in g0 after an even and in g1 after an odd nsteps), h float64 [ny, nx, 4]
    or None.  wait=False only enqueues; otherwise returns -1 or raises NonPhysical."""
    import torch
    gdt = torch.float64 if p.get("precision", "fp64") == "fp64" else torch.float32
    ncell, nv = p["nx"] * p["ny"], p["nv1"] * p["nv2"]
    for t, dtp, n in ((q, torch.float64, 6 * ncell), (g0, gdt, nv * ncell), (g1, gdt, nv * ncell),
                      (h, torch.float64, 4 * ncell)):
        if t is None:
            continue
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtp and t.is_contiguous() and t.numel() == n):
            raise TypeError("expected contiguous GPU tensors of the configuration's sizes and precisions")
    fs = C.c_int(-1)
    rc = _lib.mm_step2d_noalloc(C.byref(config(p, stream, device)), q.data_ptr(), g0.data_ptr(), g1.data_ptr(),
                                h.data_ptr() if h is not None else None, int(nsteps),
                                C.byref(fs) if wait else None)
    _check(rc, "mm_step2d_noalloc")
    return fs.value


class Solver:
    """One mm_ctx: Q, G and H live in device memory owned by the library."""

    def __init__(self, p, Q0, G0=None, stream=None, device=0, dev_buffers=None):
        """dev_buffers: None, or caller-owned GPU tensors (G0, G1, Q) that hold the state
        (zero-copy; see mm_config.dev_buffers).  With dev_buffers, Q0 = None takes the
        state already in them."""
        self.p = dict(p)
        self.ncell = p["nx"] * p.get("ny", 1)
        self.nv = p["nv1"] * p.get("nv2", 1)
        self.ncomp = 6 if p["dim"] == 2 else 3
        addrs = None
        if dev_buffers is not None:
            import torch
            gdt = torch.float64 if p.get("precision", "fp64") == "fp64" else torch.float32
            sizes = (self.ncell * self.nv, self.ncell * self.nv, self.ncell * self.ncomp)
            for t, n, dtp in zip(dev_buffers, sizes, (gdt, gdt, torch.float64)):
                if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtp and t.is_contiguous()
                        and t.numel() == n):
                    raise TypeError("dev_buffers: contiguous GPU tensors (G0, G1, Q) of the state's sizes")
            addrs = [t.data_ptr() for t in dev_buffers]
            self._keep = tuple(dev_buffers)       # the buffers must outlive the context
        if Q0 is None:
            q = None
            if addrs is None:
                raise ValueError("Q0 is required without dev_buffers")
        else:
            q = np.ascontiguousarray(Q0, dtype=np.float64).reshape(-1)
            if q.size != self.ncell * self.ncomp:
                raise ValueError("Q0 has the wrong size")
        g = None
        if G0 is not None:
            g = np.ascontiguousarray(G0, dtype=np.float64).reshape(-1)
            if g.size != self.ncell * self.nv:
                raise ValueError("G0 has the wrong size")
        self._cfg = config(p, stream, device, addrs)
        self._ctx = C.c_void_p()
        _check(_lib.mm_init(C.byref(self._cfg), _dp(q), _dp(g), C.byref(self._ctx)), "mm_init")

    def close(self):
        if self._ctx:
            _lib.mm_free(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def dt(self):
        return _lib.mm_dt(C.byref(self._cfg), 0.0, None)

    def step(self, n=1):
        _check(_lib.mm_step(self._ctx, int(n)), "mm_step")

    def step_async(self, n=1):
        _check(_lib.mm_step_async(self._ctx, int(n)), "mm_step_async")

    def sync(self):
        _check(_lib.mm_sync(self._ctx), "mm_sync")

    def failed_step(self):
        return _lib.mm_failed_step(self._ctx)

    def set_source(self, kind, t0=0.0):
        """kind: "none" or "mms" (the manufactured solution of the convergence study)."""
        _check(_lib.mm_set_source(self._ctx, SOURCE[kind], float(t0)), "mm_set_source")

    def moments(self, with_h=False, with_gmom=False):
        Q = np.empty(self.ncell * self.ncomp)
        H = np.empty(self.ncell * (4 if self.ncomp == 6 else 1)) if with_h else None
        M = np.empty(self.ncell * 7) if with_gmom else None
        _check(_lib.mm_moments(self._ctx, _dp(Q), _dp(H), _dp(M)), "mm_moments")
        out = [Q]
        if with_h:
            out.append(H)
        if with_gmom:
            out.append(M)
        return out[0] if len(out) == 1 else tuple(out)

    def get_g(self):
        G = np.empty(self.ncell * self.nv)
        _check(_lib.mm_get_g(self._ctx, _dp(G)), "mm_get_g")
        return G

    def get_g_cells(self, cells):
        """g of the given cells (cell index j * nx + i) as FP64, shape [len(cells), nv]."""
        idx = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1)
        G = np.empty((idx.size, self.nv))
        _check(_lib.mm_get_g_cells(self._ctx, idx.ctypes.data_as(C.POINTER(C.c_int)), int(idx.size), _dp(G)),
               "mm_get_g_cells")
        return G

    def set_state(self, Q, G=None):
        q = np.ascontiguousarray(Q, dtype=np.float64).reshape(-1)
        g = None if G is None else np.ascontiguousarray(G, dtype=np.float64).reshape(-1)
        _check(_lib.mm_set_state(self._ctx, _dp(q), _dp(g)), "mm_set_state")

    def timing(self, enable=True):
        _check(_lib.mm_timing(self._ctx, 1 if enable else 0), "mm_timing")

    def timing_get(self, which=0):
        n = C.c_int(0)
        ms = C.c_double(0.0)
        _check(_lib.mm_timing_get(self._ctx, int(which), C.byref(n), C.byref(ms)), "mm_timing_get")
        return n.value, ms.value

    def device_ptrs(self):
        q, g, h = C.c_void_p(), C.c_void_p(), C.c_void_p()
        gb = C.c_int(0)
        _check(_lib.mm_device_ptrs(self._ctx, C.byref(q), C.byref(g), C.byref(h), C.byref(gb)), "mm_device_ptrs")
        return q.value, g.value, h.value, gb.value

    # ---- closure form
    def closure_attach(self, net, kn_max, residual=0):
        """net: an Mlp, or None for the Navier-Stokes-Fourier closure; residual: 0 the network
        predicts (q, S, t) / eps, 1 its correction to the NSF values, 2 that correction / eps."""
        self._net = net       # the context keeps the network by pointer
        _check(_lib.mm_closure_attach(self._ctx, net._h if net is not None else None, float(kn_max),
                                      int(residual)), "mm_closure_attach")

    def closure_cells(self):
        """(closure cells summed over the steps since the last call, classes of the last step [ncell])."""
        n = C.c_longlong(0)
        cls = np.empty(self.ncell, dtype=np.uint8)
        _check(_lib.mm_closure_cells(self._ctx, C.byref(n), _bp(cls)), "mm_closure_cells")
        return n.value, cls

    def closure_snapshot(self, kn_max, X, Y, count, residual=0):
        """Append training rows to the device tensors X [cap, 30], Y [cap, 7]; returns the new count."""
        cap = X.shape[0]
        if Y.shape[0] != cap:
            raise ValueError("X and Y capacities differ")
        c = C.c_int(int(count))
        _check(_lib.mm_closure_snapshot(self._ctx, float(kn_max), int(residual), _dev(X, N_FEAT),
                                        _dev(Y, N_OUT), int(cap), C.byref(c)), "mm_closure_snapshot")
        return c.value

    def closure_features(self):
        F = np.empty((self.ncell, N_FEAT), dtype=np.float32)
        kn = np.empty(self.ncell, dtype=np.float32)
        edge = np.empty(self.ncell, dtype=np.uint8)
        _check(_lib.mm_closure_features(self._ctx, _fp(F), _fp(kn), _bp(edge)), "mm_closure_features")
        return F, kn, edge.astype(bool)

    def closure_rebuild(self, out, mask):
        o = np.ascontiguousarray(out, dtype=np.float32).reshape(-1)
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        if o.size != self.ncell * N_OUT or m.size != self.ncell:
            raise ValueError("wrong sizes")
        _check(_lib.mm_closure_rebuild(self._ctx, _fp(o), _bp(m)), "mm_closure_rebuild")


class Mlp:
    """The closure network (mm_mlp): FP32 master weights on the device, bf16 matrix-core kernels."""

    def __init__(self, seed=0, device=0, stream=None):
        self._h = C.c_void_p()
        _check(_lib.mm_mlp_create(int(device), stream, int(seed), C.byref(self._h)), "mm_mlp_create")

    def close(self):
        if self._h:
            _lib.mm_mlp_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fit_norm(self, X, Y):
        _check(_lib.mm_mlp_fit_norm(self._h, _dev(X, N_FEAT), _dev(Y, N_OUT), int(X.shape[0])), "mm_mlp_fit_norm")

    def get(self):
        P = np.empty(MLP_NPARAM, dtype=np.float32)
        N = np.empty(MLP_NNORM, dtype=np.float32)
        _check(_lib.mm_mlp_get(self._h, _fp(P), _fp(N)), "mm_mlp_get")
        return P, N

    def set(self, params=None, norm=None):
        P = None if params is None else np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        N = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32).reshape(-1)
        if (P is not None and P.size != MLP_NPARAM) or (N is not None and N.size != MLP_NNORM):
            raise ValueError("wrong sizes")
        _check(_lib.mm_mlp_set(self._h, _fp(P), _fp(N)), "mm_mlp_set")

    def forward(self, X, Y=None):
        import torch
        n = X.shape[0]
        if Y is None:
            Y = torch.empty((n, N_OUT), dtype=torch.float32, device=X.device)
        _check(_lib.mm_mlp_forward(self._h, _dev(X, N_FEAT), int(n), _dev(Y, N_OUT)), "mm_mlp_forward")
        return Y

    def grad(self, X, Y):
        g = np.empty(MLP_NPARAM, dtype=np.float32)
        loss = C.c_double(0.0)
        _check(_lib.mm_mlp_grad(self._h, _dev(X, N_FEAT), _dev(Y, N_OUT), int(X.shape[0]), _fp(g), C.byref(loss)),
               "mm_mlp_grad")
        return g, loss.value

    def train(self, X, Y, epochs=10, batch=1024, lr=2e-3, seed=0):
        """Adam epochs over (X, Y) on the GPU; returns the mean batch loss per epoch."""
        L = np.empty(int(epochs))
        _check(_lib.mm_mlp_train(self._h, _dev(X, N_FEAT), _dev(Y, N_OUT), int(X.shape[0]), int(epochs), int(batch),
                                 float(lr), int(seed), _dp(L)), "mm_mlp_train")
        return L
