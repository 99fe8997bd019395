"""ctypes binding of the FP64 oracle (oracle.c).  TEST INFRASTRUCTURE ONLY.

Every routine here hands numpy float64 arrays to the C oracle; none of the
method's arithmetic is done in Python.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")

NRED = 10
MLP_NPARAM = 6212
_lib = None


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("two_phase", C.c_int),
        ("tau", C.c_double), ("rho_l", C.c_double), ("rho_g", C.c_double),
        ("sigma", C.c_double), ("mobility", C.c_double), ("width", C.c_double),
        ("p0", C.c_double), ("n_modes", C.c_int), ("modes", C.POINTER(C.c_double)),
        ("curv_mode", C.c_int), ("k_lo", C.c_double), ("k_hi", C.c_double),
        ("mlp", C.POINTER(C.c_double)),
        ("gravity", C.c_double * 3), ("tau_g", C.c_double), ("ac_rk3", C.c_int),
    ]


def lib():
    """The oracle library (built on first use)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from .build import build
            build()
        _lib = load(LIBPATH)
    return _lib


def load(path):
    """Load and bind a build of oracle.c.  Tests that plant a mistake in a
    copy of the oracle (to show that a pin catches it) pass that build to
    `Oracle(..., library=load(path))`."""
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [C.POINTER(_Params), dp, dp, dp]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_step.argtypes = [C.c_void_p, C.c_long]
    L.orc_moments.argtypes = [C.c_void_p, dp, dp, dp, dp]
    L.orc_reduce.argtypes = [C.c_void_p, dp]
    L.orc_get_f.argtypes = [C.c_void_p, dp]
    L.orc_set_f.argtypes = [C.c_void_p, dp]
    L.orc_get_uprev.argtypes = [C.c_void_p, dp]
    L.orc_set_aext.argtypes = [C.c_void_p, dp]
    L.orc_forcing_window.argtypes = [dp] + [C.c_int] * 10 + [dp]
    L.orc_steps_done.argtypes = [C.c_void_p]
    L.orc_steps_done.restype = C.c_long
    L.orc_lattice.argtypes = [C.POINTER(C.c_int), dp]
    L.orc_feq.argtypes = [C.c_double, dp, dp]
    L.orc_guo.argtypes = [dp, dp, dp]
    L.orc_collide.argtypes = [dp, dp, dp, C.c_double, dp, dp]
    for name in ("orc_gradient", "orc_hessian", "orc_laplacian"):
        getattr(L, name).argtypes = [C.c_int, C.c_int, C.c_int, dp, dp]
    L.orc_curvature.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp]
    L.orc_weno5.restype = C.c_double
    L.orc_weno5.argtypes = [C.c_double] * 5
    L.orc_ac_update.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_double, C.c_double, dp]
    L.orc_threads.restype = C.c_int
    L.orc_to_half.restype = C.c_double
    L.orc_to_half.argtypes = [C.c_double]
    L.orc_mlp_set_fp16.argtypes = [C.c_int]
    L.orc_mlp_forward.argtypes = [dp, dp, C.c_long, dp]
    L.orc_mlp_loss_grad.restype = C.c_double
    L.orc_mlp_loss_grad.argtypes = [dp, dp, dp, C.c_long, dp]
    L.orc_adam.argtypes = [dp, dp, dp, dp, C.c_long, C.c_long, C.c_double, C.c_double, C.c_double,
                           C.c_double, dp]
    L.orc_harvest.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, C.c_int, dp, dp, C.c_long,
                              C.POINTER(C.c_long)]
    return L


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def lattice():
    c = np.zeros((27, 3), dtype=np.int32)
    w = np.zeros(27)
    lib().orc_lattice(c.ctypes.data_as(C.POINTER(C.c_int)), _p(w))
    return c, w


def feq(pstar, u):
    u = _f64(u)
    out = np.zeros(27)
    lib().orc_feq(float(pstar), _p(u), _p(out))
    return out


def guo(u, acc):
    u, acc = _f64(u), _f64(acc)
    out = np.zeros(27)
    lib().orc_guo(_p(u), _p(acc), _p(out))
    return out


def collide(f, u, acc, tau):
    f, u, acc = _f64(f), _f64(u), _f64(acc)
    fp = np.zeros(27)
    a2 = np.zeros(6)
    lib().orc_collide(_p(f), _p(u), _p(acc), float(tau), _p(fp), _p(a2))
    return fp, a2


def _field_op(name, psi, ncomp):
    psi = _f64(psi)
    nz, ny, nx = psi.shape
    out = np.zeros((ncomp,) + psi.shape) if ncomp > 1 else np.zeros(psi.shape)
    getattr(lib(), name)(nx, ny, nz, _p(psi), _p(out))
    return out


def gradient(psi):
    return _field_op("orc_gradient", psi, 3)


def hessian(psi):
    """Returns [6, nz, ny, nx] in the order xx, yy, zz, xy, xz, yz."""
    return _field_op("orc_hessian", psi, 6)


def laplacian(psi):
    return _field_op("orc_laplacian", psi, 1)


def curvature(phi):
    phi = _f64(phi)
    nz, ny, nx = phi.shape
    K = np.zeros(phi.shape)
    n = np.zeros((3,) + phi.shape)
    lib().orc_curvature(nx, ny, nz, _p(phi), _p(K), _p(n))
    return K, n


def weno5(vm2, vm1, v0, vp1, vp2):
    return lib().orc_weno5(float(vm2), float(vm1), float(v0), float(vp1), float(vp2))


def ac_update(phi, u, D, width):
    phi, u = _f64(phi), _f64(u)
    nz, ny, nx = phi.shape
    out = np.zeros(phi.shape)
    lib().orc_ac_update(nx, ny, nz, _p(phi), _p(u), float(D), float(width), _p(out))
    return out


def forcing_window(modes, box, origin, window):
    """Body acceleration [3, wz, wy, wx] of the mode table on a box of shape `box`
    (nz, ny, nx), on the window of shape `window` starting at `origin` (z, y, x)."""
    modes = _f64(modes)
    nz, ny, nx = box
    oz, oy, ox = origin
    wz, wy, wx = window
    out = np.zeros((3, wz, wy, wx))
    lib().orc_forcing_window(_p(modes), len(modes), nx, ny, nz, ox, oy, oz, wx, wy, wz, _p(out))
    return out


def threads():
    return lib().orc_threads()


def to_half(v):
    return lib().orc_to_half(float(v))


def mlp_set_fp16(on):
    lib().orc_mlp_set_fp16(int(bool(on)))


def mlp_forward(w, x):
    w, x = _f64(w), _f64(x)
    B = x.shape[0]
    y = np.zeros((B, 4))
    lib().orc_mlp_forward(_p(w), _p(x), B, _p(y))
    return y


def mlp_loss_grad(w, x, yt):
    w, x, yt = _f64(w), _f64(x), _f64(yt)
    g = np.zeros(MLP_NPARAM)
    loss = lib().orc_mlp_loss_grad(_p(w), _p(x), _p(yt), x.shape[0], _p(g))
    return loss, g


def adam(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays; returns the fp16-rounded weights."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    w16 = np.zeros_like(w)
    lib().orc_adam(_p(w), _p(m), _p(v), _p(g), len(w), int(t), lr, b1, b2, eps, _p(w16))
    return w16


def harvest(phi, centers, radii, cap=1 << 20):
    phi = _f64(phi)
    nz, ny, nx = phi.shape
    centers, radii = _f64(centers), _f64(radii)
    X = np.zeros((cap, 27))
    Y = np.zeros((cap, 4))
    n = C.c_long(0)
    lib().orc_harvest(nx, ny, nz, _p(phi), _p(centers), _p(radii), len(radii), _p(X), _p(Y), cap, C.byref(n))
    m = min(n.value, cap)
    return X[:m].copy(), Y[:m].copy(), n.value


class Oracle:
    """FP64 solver state.  Arguments mirror the GPU library's configuration."""

    def __init__(self, shape, tau, phi0=None, u0=None, pstar0=None, two_phase=None, rho_l=1.0, rho_g=1.0,
                 sigma=0.0, mobility=0.0, width=4.0, p0=1.0, modes=None, curv_mode=0, k_lo=0.4, k_hi=0.6,
                 mlp=None, gravity=(0.0, 0.0, 0.0), tau_g=0.0, ac_rk3=False, library=None):
        self._L = library if library is not None else lib()
        nz, ny, nx = shape
        self.shape = tuple(shape)
        self.N = nx * ny * nz
        if two_phase is None:
            two_phase = phi0 is not None
        self._modes = _f64(modes) if modes is not None else None
        self._mlp = _f64(mlp) if mlp is not None else None
        prm = _Params(nx, ny, nz, int(two_phase), tau, rho_l, rho_g, sigma, mobility, width, p0,
                      0 if modes is None else len(self._modes), _p(self._modes), int(curv_mode), k_lo, k_hi,
                      _p(self._mlp), (C.c_double * 3)(*[float(v) for v in gravity]), float(tau_g), int(ac_rk3))
        self._phi0 = _f64(phi0)
        self._u0 = _f64(u0)
        self._ps0 = _f64(pstar0)
        h = self._L.orc_create(C.byref(prm), _p(self._phi0), _p(self._u0), _p(self._ps0))
        if not h:
            raise ValueError("oracle: invalid parameters")
        self._h = C.c_void_p(h)
        self.two_phase = bool(two_phase)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_destroy(h)
            self._h = None

    def step(self, n=1):
        self._L.orc_step(self._h, int(n))

    @property
    def steps(self):
        return self._L.orc_steps_done(self._h)

    def moments(self):
        rho = np.zeros(self.shape)
        p = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        phi = np.zeros(self.shape)
        self._L.orc_moments(self._h, _p(rho), _p(p), _p(u), _p(phi))
        return {"rho": rho, "p": p, "u": u, "phi": phi}

    def reduce(self):
        out = np.zeros(NRED)
        self._L.orc_reduce(self._h, _p(out))
        return out

    def get_f(self):
        f = np.zeros((27,) + self.shape)
        self._L.orc_get_f(self._h, _p(f))
        return f

    def set_f(self, f):
        f = _f64(f)
        self._L.orc_set_f(self._h, _p(f))

    def set_accel(self, a):
        """Replace the body acceleration field ([3, nz, ny, nx])."""
        self._aext = _f64(a)
        assert self._aext.size == 3 * self.N
        self._L.orc_set_aext(self._h, _p(self._aext))

    def get_uprev(self):
        u = np.zeros((3,) + self.shape)
        self._L.orc_get_uprev(self._h, _p(u))
        return u
