"""FP64 CPU oracle for the micro-macro KFVS scheme (arXiv:2509.21832).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.

The arithmetic lives in ``mm_oracle.c`` (plain C, FP64, compensated velocity
sums) and, for the learned-closure form, ``mm_closure_oracle.c``.  This module only builds it, marshals arguments through ctypes and
turns problem dictionaries (see ``mm_workloads``) into the oracle's own
configuration struct.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mm_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "mm_closure_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

BC = {"extrap": 0, "periodic": 1, "wall": 2, "inflow": 3}
TAU = {"rho": 0, "p": 1, "hs1d": 2, "const": 3}
PROJ = {"discrete": 0, "paper": 1}
CFL = {"min": 0, "sum": 1}


def build(verbose=False):
    """Compile the oracle (gcc, -O2, no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-o", _LIB + ".tmp"] + _SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Bc(C.Structure):
    _fields_ = [("kind", C.c_int), ("T_wall", C.c_double), ("u_wall", C.c_double),
                ("rho", C.c_double), ("u1", C.c_double), ("u2", C.c_double), ("T", C.c_double)]


class _Cfg(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nv1", C.c_int), ("nv2", C.c_int),
                ("x_lo", C.c_double), ("x_hi", C.c_double), ("y_lo", C.c_double), ("y_hi", C.c_double),
                ("v1_lo", C.c_double), ("v1_hi", C.c_double), ("v2_lo", C.c_double), ("v2_hi", C.c_double),
                ("eps", C.c_double), ("cfl", C.c_double), ("cfl_rule", C.c_int), ("nu", C.c_double),
                ("tau_model", C.c_int), ("tau_coef", C.c_double), ("bc", _Bc * 4),
                ("proj_mode", C.c_int), ("wall_es_term", C.c_int), ("dt", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        cp = C.POINTER(_Cfg)
        ip = C.POINTER(C.c_int)
        L.o_dt.argtypes = [cp, C.c_double, ip]
        L.o_dt.restype = C.c_double
        L.o_run2d.argtypes = [cp, dp, dp, C.c_int, dp, ip]
        L.o_run1d.argtypes = [cp, dp, dp, C.c_int, dp, ip]
        L.o_mms1d.argtypes = [cp, C.c_double, dp]
        L.o_mms2d.argtypes = [cp, C.c_double, dp]
        L.o_mms1d_run.argtypes = [cp, C.c_double, C.c_int, dp, dp, dp]
        L.o_mms2d_run.argtypes = [cp, C.c_double, C.c_int, dp, dp, dp]
        L.o_mms1d_exact.argtypes = [cp, C.c_double, dp, dp]
        L.o_mms2d_exact.argtypes = [cp, C.c_double, dp, dp]
        L.o_micro2d.argtypes = [cp, dp, dp, dp]
        L.o_macro2d.argtypes = [cp, dp, dp]
        L.o_ghat2d.argtypes = [cp, dp, dp]
        L.o_project2d.argtypes = [cp, dp, dp, dp]
        L.o_gaussians2d.argtypes = [cp, dp, dp, dp]
        L.o_kfvs_half2d.argtypes = [dp, C.c_int, C.c_int, dp]
        L.o_kfvs_half2d.restype = None
        L.o_kfvs_half1d.argtypes = [dp, C.c_int, dp]
        L.o_kfvs_half1d.restype = None
        L.o_trbdf2_W.argtypes = [C.c_double] * 4
        L.o_trbdf2_W.restype = C.c_double
        L.o_wall_R.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
        L.o_wall_R.restype = C.c_double
        L.o_set_threads.argtypes = [C.c_int]
        L.o_set_threads.restype = None
        L.o_get_threads.restype = C.c_int
        L.o_features2d.argtypes = [cp, dp, dp, dp, ip]
        L.o_mlp_nparam.restype = C.c_int
        L.o_mlp_forward.argtypes = [dp, dp, dp, C.c_int, C.c_int, dp]
        L.o_mlp_grad.argtypes = [dp, dp, dp, dp, C.c_int, C.c_int, dp, dp]
        L.o_gelu.argtypes = [C.c_double]
        L.o_gelu.restype = C.c_double
        L.o_gelu_d.argtypes = [C.c_double]
        L.o_gelu_d.restype = C.c_double
        L.o_bf16.argtypes = [C.c_double]
        L.o_bf16.restype = C.c_double
        L.o_closure_H.argtypes = [dp, dp, dp]
        L.o_closure_H.restype = None
        L.o_closure_grec.argtypes = [cp, dp, dp, dp, dp, dp]
        L.o_nsf_closure.argtypes = [cp, dp, dp, dp, dp]
        L.o_nsf_closure.restype = None
        _lib = L
    return _lib


def cfg(p):
    """Oracle struct from a problem dictionary."""
    c = _Cfg()
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
    return c


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def dt(p, t_final=0.0):
    """Time step of the CFL rule; with t_final > 0 the reset rule, returns (dt, nsteps)."""
    n = C.c_int(0)
    d = lib().o_dt(C.byref(cfg(p)), float(t_final), C.byref(n))
    return d, n.value


def set_threads(n):
    lib().o_set_threads(int(n))


def threads():
    return lib().o_get_threads()


class NonPhysical(RuntimeError):
    pass


def run(p, Q, G, nsteps):
    """Advance (Q, G) by nsteps; returns (Q, G, H) as new arrays."""
    Q = _f64(Q).copy()
    G = _f64(G).copy()
    ncell = p["nx"] * p.get("ny", 1)
    H = np.zeros(ncell * (4 if p["dim"] == 2 else 1))
    fs = C.c_int(-1)
    fn = lib().o_run2d if p["dim"] == 2 else lib().o_run1d
    rc = fn(C.byref(cfg(p)), _dp(Q), _dp(G), int(nsteps), _dp(H), C.byref(fs))
    if rc == 4:
        raise NonPhysical(f"non-physical state at step {fs.value}")
    if rc:
        raise ValueError(f"oracle returned {rc}")
    return Q, G, H


def mms1d(p, t_final):
    """The 1D manufactured-solution run of the convergence study (Sec. 3.4, tab5-2)
    on the grid of p (periodic in x): (macro, micro) relative L2 errors at t_final."""
    e = np.zeros(2)
    rc = lib().o_mms1d(C.byref(cfg(p)), float(t_final), _dp(e))
    if rc:
        raise RuntimeError(f"o_mms1d failed ({rc})")
    return float(e[0]), float(e[1])


def mms2d(p, t_final):
    """The 2D manufactured-solution run of the convergence study (Sec. 6.2, tab5-4)
    on the grid of p (periodic in x and y): (macro, micro) relative L2 errors at t_final."""
    e = np.zeros(2)
    rc = lib().o_mms2d(C.byref(cfg(p)), float(t_final), _dp(e))
    if rc:
        raise RuntimeError(f"o_mms2d failed ({rc})")
    return float(e[0]), float(e[1])


def mms_exact(p, t):
    """(Q, G): the invented solution of the convergence study (1D: Sec. 3.4, 2D: Sec. 6.2)
    at time t, point values at the cell centres, in the solver's layouts."""
    ncell = p["nx"] * p.get("ny", 1)
    nv = p["nv1"] * p.get("nv2", 1)
    Q = np.zeros(ncell * (6 if p["dim"] == 2 else 3))
    G = np.zeros(ncell * nv)
    fn = lib().o_mms2d_exact if p["dim"] == 2 else lib().o_mms1d_exact
    if fn(C.byref(cfg(p)), float(t), _dp(Q), _dp(G)):
        raise ValueError("mms_exact")
    return Q, G


def mms_run(p, t_final, max_steps=-1):
    """The convergence-study run of p (from the exact point values at t = 0, the Delta t reset
    to land on t_final, the source terms), stopped after max_steps steps (< 0: all):
    returns (Q, G, errs) with errs = (macro, micro) relative L2 errors, or None if stopped
    early."""
    ncell = p["nx"] * p.get("ny", 1)
    nv = p["nv1"] * p.get("nv2", 1)
    Q = np.zeros(ncell * (6 if p["dim"] == 2 else 3))
    G = np.zeros(ncell * nv)
    e = np.full(2, np.nan)
    fn = lib().o_mms2d_run if p["dim"] == 2 else lib().o_mms1d_run
    rc = fn(C.byref(cfg(p)), float(t_final), int(max_steps), _dp(Q), _dp(G), _dp(e))
    if rc:
        raise RuntimeError(f"mms run failed ({rc})")
    return Q, G, (None if np.isnan(e[0]) else (float(e[0]), float(e[1])))


def micro2d(p, Q, G):
    """One micro step: returns (G^{n+1}, H^{n+1})."""
    Q = _f64(Q)
    G = _f64(G).copy()
    H = np.zeros(p["nx"] * p["ny"] * 4)
    rc = lib().o_micro2d(C.byref(cfg(p)), _dp(Q), _dp(G), _dp(H))
    if rc:
        raise ValueError(rc)
    return G, H


def macro2d(p, Q, H):
    Q = _f64(Q).copy()
    rc = lib().o_macro2d(C.byref(cfg(p)), _dp(Q), _dp(_f64(H)))
    if rc == 4:
        raise NonPhysical("non-physical macro state")
    return Q


def ghat2d(p, Q):
    Gh = np.zeros(p["nx"] * p["ny"] * p["nv1"] * p["nv2"])
    lib().o_ghat2d(C.byref(cfg(p)), _dp(_f64(Q)), _dp(Gh))
    return Gh


def project2d(p, q, F):
    F = _f64(F)
    out = np.zeros_like(F)
    lib().o_project2d(C.byref(cfg(p)), _dp(_f64(q)), _dp(F), _dp(out))
    return out


def gaussians2d(p, q):
    n = p["nv1"] * p["nv2"]
    M = np.zeros(n)
    Gs = np.zeros(n)
    lib().o_gaussians2d(C.byref(cfg(p)), _dp(_f64(q)), _dp(M), _dp(Gs))
    return M, Gs


def kfvs_half2d(q, direction, sign):
    out = np.zeros(6)
    lib().o_kfvs_half2d(_dp(_f64(q)), int(direction), int(sign), _dp(out))
    return out


def kfvs_half1d(q, sign):
    out = np.zeros(3)
    lib().o_kfvs_half1d(_dp(_f64(q)), int(sign), _dp(out))
    return out


def trbdf2_W(eps, tau, nu, dt_):
    return lib().o_trbdf2_W(eps, tau, nu, dt_)


def wall_R(u, Taa, T_wall, sign):
    return lib().o_wall_R(u, Taa, T_wall, int(sign))


# ---------------------------------------------------------------- closure form

N_FEAT, N_HID, N_OUT = 30, 64, 7


def mlp_nparam():
    return lib().o_mlp_nparam()


def features2d(p, Q):
    """Per-cell features [ncell, 30], local Knudsen indicator [ncell] and the
    always-micro mask of cells next to non-periodic sides [ncell]."""
    n = p["nx"] * p["ny"]
    F = np.zeros(n * N_FEAT)
    kn = np.zeros(n)
    edge = np.zeros(n, dtype=np.int32)
    rc = lib().o_features2d(C.byref(cfg(p)), _dp(_f64(Q)), _dp(F), _dp(kn), edge.ctypes.data_as(C.POINTER(C.c_int)))
    if rc:
        raise ValueError(rc)
    return F.reshape(n, N_FEAT), kn, edge.astype(bool)


def _norm(norm):
    return _f64(np.concatenate([np.ravel(norm[k]) for k in ("in_mean", "in_std", "out_mean", "out_std")]))


def mlp_forward(params, norm, X, bf16=False):
    """Raw outputs [n, 7] of the closure network for raw features X [n, 30]:
    (q1, q2, S11, S12, S22, t1, t2) / eps; norm: dict of in_mean, in_std (30),
    out_mean, out_std (7)."""
    X = _f64(X).reshape(-1, N_FEAT)
    Y = np.zeros((X.shape[0], N_OUT))
    lib().o_mlp_forward(_dp(_f64(params)), _dp(_norm(norm)), _dp(X), X.shape[0], int(bf16), _dp(Y))
    return Y


def mlp_grad(params, norm, X, Y, bf16=False):
    """(gradient of the normalised mean-square loss w.r.t. every parameter, loss)."""
    X = _f64(X).reshape(-1, N_FEAT)
    Y = _f64(Y).reshape(-1, N_OUT)
    g = np.zeros(mlp_nparam())
    loss = C.c_double(0.0)
    lib().o_mlp_grad(_dp(_f64(params)), _dp(_norm(norm)), _dp(X), _dp(Y), X.shape[0], int(bf16), _dp(g),
                     C.byref(loss))
    return g, loss.value


def gelu(x):
    return lib().o_gelu(float(x))


def gelu_d(x):
    return lib().o_gelu_d(float(x))


def bf16(x):
    return lib().o_bf16(float(x))


def closure_H(q, t=None):
    """(H111, H112, H122, H222) from the heat flux q and the traceless part t
    (t = 0: the isotropic form)."""
    H = np.zeros(4)
    lib().o_closure_H(_dp(_f64(q)), None if t is None else _dp(_f64(t)), _dp(H))
    return H


def closure_grec(p, q, qt, St, tt=None):
    g = np.zeros(p["nv1"] * p["nv2"])
    rc = lib().o_closure_grec(C.byref(cfg(p)), _dp(_f64(q)), _dp(_f64(qt)), _dp(_f64(St)),
                              None if tt is None else _dp(_f64(tt)), _dp(g))
    if rc:
        raise ValueError(rc)
    return g


def nsf_closure(p, f):
    """Navier-Stokes-Fourier (qt, St, tt) of one cell from its features."""
    qt = np.zeros(2)
    St = np.zeros(3)
    tt = np.zeros(2)
    lib().o_nsf_closure(C.byref(cfg(p)), _dp(_f64(f)), _dp(qt), _dp(St), _dp(tt))
    return qt, St, tt
