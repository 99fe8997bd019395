"""ctypes binding of liblbm.so (include/lbm.h): argument marshalling only.

Every step of the lattice update runs in the library's HIP kernels; PyTorch
supplies device memory (the workspace and the field buffers) and the stream.
There is no fallback: a missing library or a missing GPU raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(PKG, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOSPACE, LBM_EHIP, LBM_ESTATE, LBM_ERANGE = 0, -1, -2, -3, -4, -5
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
CURV = {"fd": 0, "mlp": 1}
PHI_STORAGE = {"f64": 0, "fix32": 1}
NRED = 10
MAX_MODES = 64
MLP_NPARAM = 6212
MLP_STATIC_MAX_BATCH = 16384  # lbm_mlp_backward_static
REDUCE_NAMES = ("sum_phi", "sum_rho", "sum_pstar", "sum_rho_ux", "sum_rho_uy", "sum_rho_uz", "kinetic",
                "max_u", "phi_overshoot", "nonfinite")


class LbmError(RuntimeError):
    pass


class lbm_config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("storage", C.c_int32), ("two_phase", C.c_int32), ("curv_mode", C.c_int32),
        ("tau", C.c_double), ("rho_l", C.c_double), ("rho_g", C.c_double),
        ("sigma", C.c_double), ("mobility", C.c_double), ("width", C.c_double), ("p0", C.c_double),
        ("n_modes", C.c_int32), ("zchunk", C.c_int32), ("modes", C.POINTER(C.c_double)),
        ("mlp_k_lo", C.c_double), ("mlp_k_hi", C.c_double),
        ("phi_storage", C.c_int32), ("reserved", C.c_int32),
        ("gravity", C.c_double * 3), ("tau_g", C.c_double),
        ("ac_rk3", C.c_int32), ("reserved2", C.c_int32),
    ]


_lib = None

SYMBOLS = {
    "lbm_abi_version": (C.c_int, []),
    "lbm_workspace_bytes": (C.c_size_t, [C.POINTER(lbm_config)]),
    "lbm_init": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(lbm_config), C.c_void_p, C.c_size_t, C.c_void_p,
                           C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_moments": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lbm_reduce": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "lbm_steps_done": (C.c_int64, [C.c_void_p]),
    "lbm_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_destroy": (C.c_int, [C.c_void_p]),
    "lbm_strerror": (C.c_char_p, [C.c_int]),
    "lbm_last_error": (C.c_char_p, [C.c_void_p]),
    "lbm_mlp_work_bytes": (C.c_size_t, [C.c_int64]),
    "lbm_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "lbm_mlp_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_size_t, C.c_void_p]),
    "lbm_mlp_backward_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                          C.c_void_p]),
    "lbm_mlp_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float,
                               C.c_float, C.c_float, C.c_float, C.c_void_p]),
    "lbm_set_mlp": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_harvest": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int, C.c_void_p,
                              C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    "lbm_batch_bytes": (C.c_size_t, [C.c_int]),
    "lbm_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int, C.c_void_p, C.c_size_t]),
    "lbm_batch_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_batch_tune": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "lbm_batch_set_tiling": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "lbm_batch_destroy": (C.c_int, [C.c_void_p]),
    "lbm_batch_last_error": (C.c_char_p, [C.c_void_p]),
}
BATCH_MAX = 4096
MLP_IN = 32


def load_library(path=LIBPATH):
    """Load liblbm.so and declare every exported symbol (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LbmError(f"{path} is missing: build it with `python -m paper_2505_01126_amd.build` "
                       "(or __graft_entry__.build())")
    L = C.CDLL(path)
    for name, (res, args) in SYMBOLS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc, handle=None, what=""):
    if rc != LBM_OK:
        L = load_library()
        msg = L.lbm_last_error(handle).decode() if handle is not None else L.lbm_last_error(None).decode()
        raise LbmError(f"{what}: {L.lbm_strerror(rc).decode()} ({rc}): {msg}")


def make_config(shape, tau, two_phase=False, storage="f32", rho_l=1.0, rho_g=1.0, sigma=0.0, mobility=0.0,
                width=4.0, p0=1.0, modes=None, zchunk=0, curv_mode="fd", mlp_k_lo=0.0, mlp_k_hi=0.0,
                phi_storage="f64", gravity=(0.0, 0.0, 0.0), tau_g=0.0, ac_rk3=False):
    """Build an lbm_config; returns (config, keepalive) where keepalive owns the mode table."""
    nz, ny, nx = shape
    tab = None if modes is None or len(modes) == 0 else np.ascontiguousarray(modes, dtype=np.float64)
    cfg = lbm_config(nx, ny, nz, STORAGE[storage], int(bool(two_phase)), CURV[curv_mode], float(tau),
                     float(rho_l), float(rho_g), float(sigma), float(mobility), float(width), float(p0),
                     0 if tab is None else len(tab), int(zchunk),
                     None if tab is None else tab.ctypes.data_as(C.POINTER(C.c_double)),
                     float(mlp_k_lo), float(mlp_k_hi), PHI_STORAGE.get(phi_storage, phi_storage), 0,
                     (C.c_double * 3)(*[float(v) for v in gravity]), float(tau_g), int(ac_rk3), 0)
    return cfg, tab


def lbm_abi_version():
    return load_library().lbm_abi_version()


def lbm_workspace_bytes(cfg):
    return load_library().lbm_workspace_bytes(C.byref(cfg))


def lbm_init(cfg, d_ws, ws_bytes, d_phi0, d_u0, d_pstar0, stream):
    h = C.c_void_p()
    rc = load_library().lbm_init(C.byref(h), C.byref(cfg), d_ws, ws_bytes, d_phi0, d_u0, d_pstar0, stream)
    _check(rc, None, "lbm_init")
    return h


def lbm_step(h, nsteps):
    _check(load_library().lbm_step(h, int(nsteps)), h, "lbm_step")


def lbm_moments(h, d_rho, d_p, d_u, d_phi):
    _check(load_library().lbm_moments(h, d_rho, d_p, d_u, d_phi), h, "lbm_moments")


def lbm_reduce(h, out, out_is_host):
    _check(load_library().lbm_reduce(h, out, int(out_is_host)), h, "lbm_reduce")


def lbm_steps_done(h):
    return load_library().lbm_steps_done(h)


def lbm_set_stream(h, stream):
    _check(load_library().lbm_set_stream(h, stream), h, "lbm_set_stream")


def lbm_destroy(h):
    load_library().lbm_destroy(h)


def lbm_mlp_work_bytes(batch):
    return load_library().lbm_mlp_work_bytes(int(batch))


def lbm_mlp_forward(d_w, d_x, batch, d_y, stream):
    _check(load_library().lbm_mlp_forward(d_w, d_x, int(batch), d_y, stream), None, "lbm_mlp_forward")


def lbm_mlp_backward(d_w, d_x, d_t, batch, d_grad, d_loss, d_work, work_bytes, stream):
    _check(load_library().lbm_mlp_backward(d_w, d_x, d_t, int(batch), d_grad, d_loss, d_work, work_bytes, stream),
           None, "lbm_mlp_backward")


def lbm_mlp_backward_static(d_w, d_x, d_t, batch, d_grad, d_loss, stream):
    _check(load_library().lbm_mlp_backward_static(d_w, d_x, d_t, int(batch), d_grad, d_loss, stream), None,
           "lbm_mlp_backward_static")


def lbm_mlp_adam(d_master, d_m, d_v, d_grad, d_w16, step, lr, beta1, beta2, eps, stream):
    _check(load_library().lbm_mlp_adam(d_master, d_m, d_v, d_grad, d_w16, int(step), lr, beta1, beta2, eps, stream),
           None, "lbm_mlp_adam")


def lbm_set_mlp(h, d_w):
    _check(load_library().lbm_set_mlp(h, d_w), h, "lbm_set_mlp")


def lbm_harvest(h, centers, radii, d_x, d_y, cap):
    """centers [nb,3], radii [nb] host float64; returns the total count."""
    c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    n = C.c_int64(0)
    dp = C.POINTER(C.c_double)
    _check(load_library().lbm_harvest(h, c.ctypes.data_as(dp), r.ctypes.data_as(dp), len(r), d_x, d_y, int(cap),
                                      C.byref(n)), h, "lbm_harvest")
    return n.value


def _check_batch(rc, b, what):
    if rc != LBM_OK:
        L = load_library()
        raise LbmError(f"{what}: {L.lbm_strerror(rc).decode()} ({rc}): {L.lbm_batch_last_error(b).decode()}")


def lbm_batch_bytes(n):
    return load_library().lbm_batch_bytes(int(n))


def lbm_batch_create(members, d_table, table_bytes):
    """members: sequence of handles (c_void_p); returns the batch handle."""
    arr = (C.c_void_p * len(members))(*[m.value if isinstance(m, C.c_void_p) else m for m in members])
    b = C.c_void_p()
    rc = load_library().lbm_batch_create(C.byref(b), arr, len(members), d_table, table_bytes)
    _check_batch(rc, None, "lbm_batch_create")
    return b


def lbm_batch_step(b, nsteps):
    _check_batch(load_library().lbm_batch_step(b, int(nsteps)), b, "lbm_batch_step")


def lbm_batch_tune(b, steps_per_candidate):
    """Returns (tile width, z-chunk length)."""
    tile = C.c_int(0)
    zc = C.c_int(0)
    _check_batch(load_library().lbm_batch_tune(b, int(steps_per_candidate), C.byref(tile), C.byref(zc)), b,
                 "lbm_batch_tune")
    return tile.value, zc.value


def lbm_batch_set_tiling(b, tile, zchunk):
    _check_batch(load_library().lbm_batch_set_tiling(b, int(tile), int(zchunk)), b, "lbm_batch_set_tiling")


def lbm_batch_destroy(b):
    load_library().lbm_batch_destroy(b)


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise LbmError("no GPU visible: the lattice library runs only on the MI355X")
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Lattice:
    """One simulation: owns the workspace tensor and the library handle.

    shape = (nz, ny, nx).  phi0 [nz,ny,nx], u0 [3,nz,ny,nx], pstar0 [nz,ny,nx]
    are numpy or torch arrays (float64 on the device after conversion).
    """

    def __init__(self, shape, tau, phi0=None, u0=None, pstar0=None, two_phase=None, storage="f32", rho_l=1.0,
                 rho_g=1.0, sigma=0.0, mobility=0.0, width=4.0, p0=1.0, modes=None, zchunk=0, curv_mode="fd",
                 mlp_k_lo=0.0, mlp_k_hi=0.0, phi_storage="f64", gravity=(0.0, 0.0, 0.0), tau_g=0.0,
                 ac_rk3=False, device="cuda:0"):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.shape = tuple(int(s) for s in shape)
        nz, ny, nx = self.shape
        self.N = nx * ny * nz
        if two_phase is None:
            two_phase = phi0 is not None
        self.two_phase = bool(two_phase)
        self.cfg, self._tab = make_config(self.shape, tau, self.two_phase, storage, rho_l, rho_g, sigma, mobility,
                                          width, p0, modes, zchunk, curv_mode, mlp_k_lo, mlp_k_hi, phi_storage,
                                          gravity, tau_g, ac_rk3)
        nbytes = lbm_workspace_bytes(self.cfg)
        if nbytes == 0:
            raise LbmError("invalid configuration")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)

        def dev(a, n):
            if a is None:
                return None
            t = torch.as_tensor(np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a)
            t = t.to(device=self.device, dtype=torch.float64).contiguous()
            if t.numel() != n:
                raise LbmError(f"input has {t.numel()} values, expected {n}")
            return t

        phi = dev(phi0, self.N) if self.two_phase else None
        u = dev(u0, 3 * self.N)
        ps = dev(pstar0, self.N)
        self.stream = torch.cuda.current_stream(self.device)
        self.h = lbm_init(self.cfg, C.c_void_p(self.ws.data_ptr()), nbytes, _ptr(phi), _ptr(u), _ptr(ps),
                          C.c_void_p(self.stream.cuda_stream))
        self.stream.synchronize()  # the inputs may be released after this
        self.ws_bytes = nbytes

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        lbm_step(self.h, n)

    @property
    def steps(self):
        return lbm_steps_done(self.h)

    def moments(self):
        """Fields at the current time as device tensors: rho, p (fp32), u [3,...] (fp32), phi (fp64)."""
        torch = self.torch
        rho = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        p = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=torch.float32, device=self.device)
        phi = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        lbm_moments(self.h, _ptr(rho), _ptr(p), _ptr(u), _ptr(phi))
        return {"rho": rho, "p": p, "u": u, "phi": phi}

    def reduce(self):
        """The ten FP64 global statistics at the current time (host numpy array)."""
        out = np.zeros(NRED)
        lbm_reduce(self.h, out.ctypes.data_as(C.c_void_p), 1)
        return out

    def synchronize(self):
        self.stream.synchronize()

    def set_mlp(self, w16):
        """Install fp16 network weights (torch.int16/uint16-compatible device tensor of 6212 values)."""
        self._mlp_w = w16.contiguous()
        lbm_set_mlp(self.h, _ptr(self._mlp_w))

    def harvest(self, centers, radii, cap):
        """Training rows from the current phi: (X [n,32] fp16 bits as int16, Y [n,4] fp32, total count)."""
        torch = self.torch
        X = torch.zeros((max(cap, 1), MLP_IN), dtype=torch.int16, device=self.device)
        Y = torch.zeros((max(cap, 1), 4), dtype=torch.float32, device=self.device)
        n = lbm_harvest(self.h, centers, radii, _ptr(X), _ptr(Y), cap)
        m = min(n, cap)
        return X[:m], Y[:m], n


class Mlp:
    """Device-side network parameters plus Adam state; every computation runs in
    the library's MFMA kernels."""

    def __init__(self, w_init, device="cuda:0"):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        w = np.asarray(w_init, dtype=np.float64).reshape(-1)
        if w.size != MLP_NPARAM:
            raise LbmError(f"expected {MLP_NPARAM} parameters")
        self.master = torch.tensor(w.astype(np.float32), device=self.device)
        self.w16 = torch.tensor(w.astype(np.float16).view(np.int16), device=self.device)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.t = 0
        self._work = None

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def forward(self, X):
        y = self.torch.empty((X.shape[0], 4), dtype=self.torch.float32, device=self.device)
        lbm_mlp_forward(_ptr(self.w16), _ptr(X), X.shape[0], _ptr(y), self.stream())
        return y

    def backward(self, X, T):
        B = X.shape[0]
        need = lbm_mlp_work_bytes(B)
        if self._work is None or self._work.numel() < need:
            self._work = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        lbm_mlp_backward(_ptr(self.w16), _ptr(X), _ptr(T), B, _ptr(self.grad), _ptr(self.loss), _ptr(self._work),
                         self._work.numel(), self.stream())
        return self.grad, self.loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        lbm_mlp_adam(_ptr(self.master), _ptr(self.m), _ptr(self.v), _ptr(self.grad), _ptr(self.w16), self.t, lr,
                     beta1, beta2, eps, self.stream())

    def weights_fp16(self):
        return self.w16.cpu().numpy().view(np.float16).astype(np.float64)


class Batch:
    """Independent Lattice objects advanced together by one persistent launch
    per step (see lbm_batch_* in include/lbm.h).  The lattices must outlive it."""

    def __init__(self, lattices):
        torch = _torch()
        self.lattices = list(lattices)
        n = len(self.lattices)
        nbytes = lbm_batch_bytes(n)
        if nbytes == 0:
            raise LbmError(f"a batch holds 1 .. {BATCH_MAX} lattices")
        self.table = torch.empty(nbytes, dtype=torch.uint8, device=self.lattices[0].device)
        self.b = lbm_batch_create([g.h for g in self.lattices], C.c_void_p(self.table.data_ptr()), nbytes)

    def step(self, n=1):
        lbm_batch_step(self.b, n)

    def tune(self, steps_per_candidate=4):
        """Pick the tile width and z-chunk length by timing; returns (tile, zchunk)
        (the timed steps advance the lattices)."""
        return lbm_batch_tune(self.b, steps_per_candidate)

    def set_tiling(self, tile, zchunk):
        """Work decomposition by hand: tile width 64 or 32, z-chunk length."""
        lbm_batch_set_tiling(self.b, tile, zchunk)

    def close(self):
        if getattr(self, "b", None) is not None:
            lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
