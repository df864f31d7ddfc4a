"""Thin ctypes binding of libtmq.so (include/tmq.h).

Only argument marshalling happens here: every step of the operator and the
solver runs in the HIP library.  Device buffers are torch tensors on the
lattice's GPU (complex128, canonical layout); host buffers are numpy arrays.
If libtmq.so is missing this module raises ImportError: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtmq.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_0905_3331_amd.build` "
        "(hipcc, gfx950); there is no CPU fallback"
    )

_lib = ctypes.CDLL(LIB_PATH)

FP64, FP32, FP16, BF16 = 0, 1, 2, 3
MAX_RHS = 64
NOALLOC_SCRATCH_BYTES = 64 << 20  # TMQ_NOALLOC_SCRATCH_BYTES
PREC = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16}

TMQ_OK, TMQ_EINVAL, TMQ_ENOMEM, TMQ_ENOCONV, TMQ_EDEVICE, TMQ_ENAN, TMQ_ESTATE = 0, -1, -2, -3, -4, -5, -6
TMQ_PENDING = 1
STATUS = {0: "TMQ_OK", -1: "TMQ_EINVAL", -2: "TMQ_ENOMEM", -3: "TMQ_ENOCONV", -4: "TMQ_EDEVICE",
          -5: "TMQ_ENAN", -6: "TMQ_ESTATE", 1: "TMQ_PENDING"}


class tmq_params(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("mu_tilde", ctypes.c_double), ("theta", ctypes.c_double * 4)]


class tmq_nd_params(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("mubar_tilde", ctypes.c_double), ("epsbar_tilde", ctypes.c_double),
                ("theta", ctypes.c_double * 4)]


class tmq_solver_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("relative", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("sloppy", ctypes.c_int), ("sloppy_link", ctypes.c_int), ("delta", ctypes.c_double),
                ("mode", ctypes.c_int)]


class tmq_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("true_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


class tmq_server_config(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_batch", ctypes.c_int)]


class tmq_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_long), ("completed", ctypes.c_long), ("failed", ctypes.c_long),
                ("rejected", ctypes.c_long), ("queued", ctypes.c_long), ("running", ctypes.c_long),
                ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double), ("mean_s", ctypes.c_double),
                ("mean_wait_s", ctypes.c_double), ("solves_per_s", ctypes.c_double),
                ("elapsed_s", ctypes.c_double), ("budget_bytes", ctypes.c_size_t),
                ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t), ("engines", ctypes.c_int),
                ("peak_running", ctypes.c_int), ("steps", ctypes.c_long)]


_vp = ctypes.c_void_p
_ip = ctypes.c_int
_P = ctypes.POINTER

_SIGS = {
    "tmq_lattice_create": (_ip, [_P(ctypes.c_int), _ip, _P(_vp)]),
    "tmq_lattice_destroy": (None, [_vp]),
    "tmq_load_gauge": (_ip, [_vp, _vp]),
    "tmq_load_gauge_dev": (_ip, [_vp, _vp, _vp]),
    "tmq_gauge_is_su3": (_ip, [_vp]),
    "tmq_apply_Qhat": (_ip, [_vp, _P(tmq_params), _ip, _ip, _vp, _vp]),
    "tmq_apply_Qhat_dev": (_ip, [_vp, _P(tmq_params), _ip, _ip, _vp, _vp, _vp]),
    "tmq_apply_Qhat_noalloc_dev": (_ip, [_vp, _P(tmq_params), _ip, _ip, _vp, _vp, _vp]),
    "tmq_apply_QhatQhat_dev": (_ip, [_vp, _P(tmq_params), _vp, _vp, _vp]),
    "tmq_apply_Q_full": (_ip, [_vp, _P(tmq_params), _ip, _vp, _vp]),
    "tmq_apply_Q_full_dev": (_ip, [_vp, _P(tmq_params), _ip, _vp, _vp, _vp]),
    "tmq_solve": (_ip, [_vp, _P(tmq_params), _P(tmq_solver_opts), _vp, _vp, _P(tmq_solve_info)]),
    "tmq_solve_dev": (_ip, [_vp, _P(tmq_params), _P(tmq_solver_opts), _vp, _vp, _vp, _P(tmq_solve_info)]),
    "tmq_solve_batch": (_ip, [_vp, _ip, _P(tmq_params), _P(tmq_solver_opts), _P(_vp), _P(_vp),
                              _P(tmq_solve_info)]),
    "tmq_solve_batch_dev": (_ip, [_vp, _ip, _P(tmq_params), _P(tmq_solver_opts), _P(_vp), _P(_vp), _vp,
                                  _P(tmq_solve_info)]),
    "tmq_solve_full_dev": (_ip, [_vp, _P(tmq_params), _P(tmq_solver_opts), _vp, _vp, _vp, _P(tmq_solve_info)]),
    "tmq_solve_M": (_ip, [_vp, _P(tmq_params), _ip, _P(tmq_solver_opts), _vp, _vp, _P(tmq_solve_info)]),
    "tmq_solve_M_dev": (_ip, [_vp, _P(tmq_params), _ip, _P(tmq_solver_opts), _vp, _vp, _vp, _P(tmq_solve_info)]),
    "tmq_apply_Qhat_nd": (_ip, [_vp, _P(tmq_nd_params), _ip, _ip, _vp, _vp]),
    "tmq_apply_Qhat_nd_dev": (_ip, [_vp, _P(tmq_nd_params), _ip, _ip, _vp, _vp, _vp]),
    "tmq_solve_nd": (_ip, [_vp, _P(tmq_nd_params), _P(tmq_solver_opts), _vp, _vp, _P(tmq_solve_info)]),
    "tmq_solve_nd_dev": (_ip, [_vp, _P(tmq_nd_params), _P(tmq_solver_opts), _vp, _vp, _vp, _P(tmq_solve_info)]),
    "tmq_solve_nd_batch_dev": (_ip, [_vp, _ip, _P(tmq_nd_params), _P(tmq_solver_opts), _P(_vp), _P(_vp), _vp,
                                     _P(tmq_solve_info)]),
    "tmq_solve_Qhat": (_ip, [_vp, _P(tmq_params), _ip, _P(tmq_solver_opts), _vp, _vp, _P(tmq_solve_info)]),
    "tmq_solve_Qhat_dev": (_ip, [_vp, _P(tmq_params), _ip, _P(tmq_solver_opts), _vp, _vp, _vp,
                                 _P(tmq_solve_info)]),
    "tmq_solve_force_dev": (_ip, [_vp, _P(tmq_params), _P(tmq_solver_opts), _vp, _vp, _vp,
                                  _P(ctypes.c_double), _vp, _P(tmq_solve_info)]),
    "tmq_timeslice_bilinear_dev": (_ip, [_vp, _vp, _vp, _ip, _vp, _vp]),
    "tmq_pion_correlator_dev": (_ip, [_vp, _P(tmq_params), _P(tmq_solver_opts), _vp, _ip, _vp, _vp, _vp,
                                      _P(tmq_solve_info)]),
    "tmq_split_eo": (_ip, [_vp, _vp, _vp, _vp]),
    "tmq_merge_eo": (_ip, [_vp, _vp, _vp, _vp]),
    "tmq_split_eo_dev": (_ip, [_vp, _vp, _vp, _vp, _vp]),
    "tmq_merge_eo_dev": (_ip, [_vp, _vp, _vp, _vp, _vp]),
    "tmq_solve_M_batch_dev": (_ip, [_vp, _P(tmq_params), _ip, _P(tmq_solver_opts), _ip, _P(_vp), _P(_vp), _vp,
                                    _P(tmq_solve_info)]),
    "tmq_set_kernel_timing": (_ip, [_vp, _ip]),
    "tmq_kernel_stats": (_ip, [_vp, ctypes.c_char_p, _P(ctypes.c_int), _P(ctypes.c_double),
                               _P(ctypes.c_double), _P(ctypes.c_double)]),
    "tmq_stream_copy": (_ip, [_ip, ctypes.c_size_t, _ip, _P(ctypes.c_double)]),
    "tmq_tuning_report": (_ip, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "tmq_encode_dev": (_ip, [_vp, _ip, ctypes.c_long, _vp, _vp, _vp, _vp]),
    "tmq_footprint_bytes": (_ip, [_P(ctypes.c_int), _P(tmq_solver_opts), _ip, _P(ctypes.c_size_t)]),
    "tmq_server_create": (_ip, [_ip, _P(tmq_server_config), _P(_vp)]),
    "tmq_server_add_lattice": (_ip, [_vp, _P(ctypes.c_int), _vp, _P(ctypes.c_int)]),
    "tmq_server_submit": (_ip, [_vp, _ip, _P(tmq_params), _P(tmq_solver_opts), _vp, _vp,
                                _P(ctypes.c_uint64)]),
    "tmq_server_poll": (_ip, [_vp, ctypes.c_uint64, _P(tmq_solve_info)]),
    "tmq_server_wait": (_ip, [_vp, ctypes.c_uint64, ctypes.c_double, _P(tmq_solve_info)]),
    "tmq_server_get_stats": (_ip, [_vp, _P(tmq_server_stats)]),
    "tmq_server_reset_stats": (_ip, [_vp]),
    "tmq_server_destroy": (None, [_vp]),
    "tmq_last_error": (ctypes.c_char_p, []),
    "tmq_version": (ctypes.c_char_p, []),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class TmqError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.tmq_last_error().decode()
        super().__init__(f"{where}: {STATUS.get(code, code)}: {msg}")
        self.code = code


def _check(code: int, where: str, ok=(TMQ_OK,)):
    if code not in ok:
        raise TmqError(code, where)
    return code


def version() -> str:
    return _lib.tmq_version().decode()


def params(kappa: float, mu_tilde: float, theta=(1.0, 0.0, 0.0, 0.0)) -> tmq_params:
    p = tmq_params()
    p.kappa = float(kappa)
    p.mu_tilde = float(mu_tilde)
    for i in range(4):
        p.theta[i] = float(theta[i])
    return p


def nd_params(kappa: float, mubar_tilde: float, epsbar_tilde: float, theta=(1.0, 0.0, 0.0, 0.0)) -> tmq_nd_params:
    """Parameters of the flavour doublet of eq. (Dh): 2 kappa mubar and 2 kappa epsbar."""
    p = tmq_nd_params()
    p.kappa = float(kappa)
    p.mubar_tilde = float(mubar_tilde)
    p.epsbar_tilde = float(epsbar_tilde)
    for i in range(4):
        p.theta[i] = float(theta[i])
    return p


MODE_RELIABLE, MODE_SWITCH, MODE_BICGSTAB = 0, 1, 2


def solver_opts(tol=1e-10, relative=True, max_iter=10000, sloppy="fp64", sloppy_link="fp16",
                delta=0.0, mode="reliable") -> tmq_solver_opts:
    o = tmq_solver_opts()
    o.tol = float(tol)
    o.relative = 1 if relative else 0
    o.max_iter = int(max_iter)
    o.sloppy = PREC[sloppy] if isinstance(sloppy, str) else int(sloppy)
    o.sloppy_link = PREC[sloppy_link] if isinstance(sloppy_link, str) else int(sloppy_link)
    o.delta = float(delta)
    o.mode = ({"reliable": MODE_RELIABLE, "switch": MODE_SWITCH, "bicgstab": MODE_BICGSTAB}[mode]
              if isinstance(mode, str) else int(mode))
    return o


def stream_copy_gbps(nbytes: int = 1 << 30, reps: int = 10, device: int = 0) -> float:
    """Read + write bandwidth of a plain device-to-device copy kernel (calibration)."""
    g = ctypes.c_double(0)
    _check(_lib.tmq_stream_copy(device, nbytes, reps, ctypes.byref(g)), "tmq_stream_copy")
    return g.value


def footprint_bytes(dims, opts=None, nrhs=1) -> int:
    d = (ctypes.c_int * 4)(*dims)
    out = ctypes.c_size_t(0)
    _check(_lib.tmq_footprint_bytes(d, ctypes.byref(opts) if opts is not None else None, nrhs,
                                    ctypes.byref(out)), "tmq_footprint_bytes")
    return int(out.value)


def _stream(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, n_complex: int, what: str):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what}: expected a CUDA/HIP torch tensor")
    if t.dtype != torch.complex128 or not t.is_contiguous() or t.numel() != n_complex:
        raise ValueError(f"{what}: expected a contiguous complex128 tensor of {n_complex} elements, "
                         f"got {t.dtype} {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a: np.ndarray, n_complex: int, what: str):
    if not isinstance(a, np.ndarray) or a.dtype != np.complex128 or not a.flags.c_contiguous or a.size != n_complex:
        raise ValueError(f"{what}: expected a C-contiguous complex128 array of {n_complex} elements")
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class SolveInfo:
    status: int
    iters: int
    reliable_updates: int
    true_rel_residual: float
    seconds: float
    name: str = field(default="")


def _info(i: tmq_solve_info) -> SolveInfo:
    return SolveInfo(i.status, i.iters, i.reliable_updates, i.true_rel_residual, i.seconds,
                     STATUS.get(i.status, str(i.status)))


class Lattice:
    """A lattice of extents (T, LZ, LY, LX) on one GPU, owning its gauge copies."""

    def __init__(self, dims, device: int = 0):
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.device = device
        h = ctypes.c_void_p()
        _check(_lib.tmq_lattice_create((ctypes.c_int * 4)(*self.dims), device, ctypes.byref(h)),
               "tmq_lattice_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.tmq_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---------------------------------------------------------------- gauge
    def load_gauge(self, U, stream=None):
        """U: numpy (host) or torch (device) complex128, canonical (T,LZ,LY,LX,4,3,3)."""
        n = self.V * 36
        if isinstance(U, np.ndarray):
            _check(_lib.tmq_load_gauge(self._h, _hptr(U, n, "U")), "tmq_load_gauge")
        else:
            _check(_lib.tmq_load_gauge_dev(self._h, _dptr(U, n, "U"), _stream(stream)), "tmq_load_gauge_dev")

    @property
    def su3(self) -> bool:
        return bool(_lib.tmq_gauge_is_su3(self._h))

    # ------------------------------------------------------------ operators
    def apply_Qhat(self, p: tmq_params, sign: int, src, out=None, prec="fp64", stream=None):
        """Qhat^{sign} on an odd-site field (V/2, 4, 3); device tensors or host arrays."""
        pr = PREC[prec] if isinstance(prec, str) else int(prec)
        n = self.V // 2 * 12
        if isinstance(src, np.ndarray):
            out = np.empty_like(src) if out is None else out
            _check(_lib.tmq_apply_Qhat(self._h, ctypes.byref(p), sign, pr, _hptr(src, n, "in"),
                                       _hptr(out, n, "out")), "tmq_apply_Qhat")
            return out
        import torch

        out = torch.empty_like(src) if out is None else out
        _check(_lib.tmq_apply_Qhat_dev(self._h, ctypes.byref(p), sign, pr, _dptr(src, n, "in"),
                                       _dptr(out, n, "out"), _stream(stream)), "tmq_apply_Qhat_dev")
        return out

    def apply_Qhat_noalloc(self, p: tmq_params, sign: int, src, out, prec="fp64", stream=None):
        """Qhat^{sign} through tmq_apply_Qhat_noalloc_dev: device tensors only, the
        output tensor given (the call allocates nothing; its work fields are the
        library's fixed device array)."""
        pr = PREC[prec] if isinstance(prec, str) else int(prec)
        n = self.V // 2 * 12
        _check(_lib.tmq_apply_Qhat_noalloc_dev(self._h, ctypes.byref(p), sign, pr, _dptr(src, n, "in"),
                                               _dptr(out, n, "out"), _stream(stream)), "tmq_apply_Qhat_noalloc_dev")
        return out

    def apply_QhatQhat(self, p: tmq_params, src, out=None, stream=None):
        import torch

        n = self.V // 2 * 12
        out = torch.empty_like(src) if out is None else out
        _check(_lib.tmq_apply_QhatQhat_dev(self._h, ctypes.byref(p), _dptr(src, n, "in"), _dptr(out, n, "out"),
                                           _stream(stream)), "tmq_apply_QhatQhat_dev")
        return out

    def apply_Q_full(self, p: tmq_params, sign: int, src, out=None, stream=None):
        n = self.V * 12
        if isinstance(src, np.ndarray):
            out = np.empty_like(src) if out is None else out
            _check(_lib.tmq_apply_Q_full(self._h, ctypes.byref(p), sign, _hptr(src, n, "in"),
                                         _hptr(out, n, "out")), "tmq_apply_Q_full")
            return out
        import torch

        out = torch.empty_like(src) if out is None else out
        _check(_lib.tmq_apply_Q_full_dev(self._h, ctypes.byref(p), sign, _dptr(src, n, "in"),
                                         _dptr(out, n, "out"), _stream(stream)), "tmq_apply_Q_full_dev")
        return out

    # --------------------------------------------------------------- solves
    def solve(self, p: tmq_params, b, opts: tmq_solver_opts, x=None, stream=None, check=True):
        """Solve Qhat^+ Qhat^- x = b on the odd sites; returns (x, SolveInfo)."""
        n = self.V // 2 * 12
        info = tmq_solve_info()
        if isinstance(b, np.ndarray):
            x = np.empty_like(b) if x is None else x
            code = _lib.tmq_solve(self._h, ctypes.byref(p), ctypes.byref(opts), _hptr(b, n, "b"),
                                  _hptr(x, n, "x"), ctypes.byref(info))
        else:
            import torch

            x = torch.empty_like(b) if x is None else x
            code = _lib.tmq_solve_dev(self._h, ctypes.byref(p), ctypes.byref(opts), _dptr(b, n, "b"),
                                      _dptr(x, n, "x"), _stream(stream), ctypes.byref(info))
        if check:
            _check(code, "tmq_solve")
        return x, _info(info)

    def solve_batch(self, ps, bs, opts: tmq_solver_opts, xs=None, stream=None, check=True):
        """Solve Qhat^+ Qhat^- x_r = b_r for a batch (list of params, list of sources,
        device tensors or host arrays); returns (list of x, list of SolveInfo)."""
        n = len(bs)
        if len(ps) != n or not 1 <= n <= MAX_RHS:
            raise ValueError(f"need 1..{MAX_RHS} sources and one params per source")
        nc = self.V // 2 * 12
        parr = (tmq_params * n)(*ps)
        infos = (tmq_solve_info * n)()
        host = isinstance(bs[0], np.ndarray)
        if xs is None:
            if host:
                xs = [np.empty_like(b) for b in bs]
            else:
                import torch

                xs = [torch.empty_like(b) for b in bs]
        conv = _hptr if host else _dptr
        bp = (ctypes.c_void_p * n)(*[conv(b, nc, "b").value for b in bs])
        xp = (ctypes.c_void_p * n)(*[conv(x, nc, "x").value for x in xs])
        if host:
            code = _lib.tmq_solve_batch(self._h, n, parr, ctypes.byref(opts), bp, xp, infos)
        else:
            code = _lib.tmq_solve_batch_dev(self._h, n, parr, ctypes.byref(opts), bp, xp, _stream(stream), infos)
        if check:
            _check(code, "tmq_solve_batch")
        return xs, [_info(i) for i in infos]

    def solve_Qhat(self, p: tmq_params, sign: int, b, opts: tmq_solver_opts, x=None, stream=None, check=True):
        """Solve Qhat^{sign} x = b by BiCGstab (FP64); device tensor or host array (V/2, 4, 3)."""
        n = self.V // 2 * 12
        info = tmq_solve_info()
        if isinstance(b, np.ndarray):
            x = np.empty_like(b) if x is None else x
            code = _lib.tmq_solve_Qhat(self._h, ctypes.byref(p), sign, ctypes.byref(opts), _hptr(b, n, "b"),
                                       _hptr(x, n, "x"), ctypes.byref(info))
        else:
            import torch

            x = torch.empty_like(b) if x is None else x
            code = _lib.tmq_solve_Qhat_dev(self._h, ctypes.byref(p), sign, ctypes.byref(opts), _dptr(b, n, "b"),
                                           _dptr(x, n, "x"), _stream(stream), ctypes.byref(info))
        if check:
            _check(code, "tmq_solve_Qhat")
        return x, _info(info)

    # ------------------------------------------------- consumers of the solver
    def solve_force(self, p: tmq_params, phi, opts: tmq_solver_opts, stream=None, check=True, with_y=True):
        """X = (Qhat^+ Qhat^-)^-1 phi, Y = Qhat^- X (eq. (eo6)) and S_PF = Re phi^+ X;
        device tensors (V/2, 4, 3); returns (X, Y or None, S_PF, SolveInfo)."""
        import torch

        n = self.V // 2 * 12
        X = torch.empty_like(phi)
        Y = torch.empty_like(phi) if with_y else None
        act = ctypes.c_double(0.0)
        info = tmq_solve_info()
        code = _lib.tmq_solve_force_dev(self._h, ctypes.byref(p), ctypes.byref(opts), _dptr(phi, n, "phi"),
                                        _dptr(X, n, "X"), _dptr(Y, n, "Y") if with_y else None,
                                        ctypes.byref(act), _stream(stream), ctypes.byref(info))
        if check:
            _check(code, "tmq_solve_force")
        return X, Y, act.value, _info(info)

    def timeslice_bilinear(self, gamma, psi, t0=0, stream=None):
        """Per time slice sum of psi^+ Gamma psi (Gamma 4x4 complex) of a full field; returns complex (T,)."""
        n = self.V * 12
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.complex128).reshape(4, 4))
        out = np.zeros(self.dims[0], dtype=np.complex128)
        _check(_lib.tmq_timeslice_bilinear_dev(self._h, g.ctypes.data, _dptr(psi, n, "psi"), int(t0),
                                               out.ctypes.data, _stream(stream)), "tmq_timeslice_bilinear")
        return out

    def pion_correlator(self, p: tmq_params, xi, opts: tmq_solver_opts, t0=0, stream=None, check=True):
        """One-end-trick pseudoscalar correlator of one noise sample xi (full field, device);
        returns (C (T,), phi, SolveInfo)."""
        import torch

        n = self.V * 12
        phi = torch.empty_like(xi)
        corr = np.zeros(self.dims[0], dtype=np.float64)
        info = tmq_solve_info()
        code = _lib.tmq_pion_correlator_dev(self._h, ctypes.byref(p), ctypes.byref(opts), _dptr(xi, n, "xi"),
                                            int(t0), corr.ctypes.data, _dptr(phi, n, "phi"), _stream(stream),
                                            ctypes.byref(info))
        if check:
            _check(code, "tmq_pion_correlator")
        return corr, phi, _info(info)

    # ------------------------------------------------------ flavour doublet
    def apply_Qhat_nd(self, p: tmq_nd_params, sign: int, src, out=None, prec="fp64", stream=None):
        """Qhat_h^{sign} on a doublet of odd-site fields (2, V/2, 4, 3); device tensor or host array."""
        pr = PREC[prec] if isinstance(prec, str) else int(prec)
        n = self.V * 12
        if isinstance(src, np.ndarray):
            out = np.empty_like(src) if out is None else out
            _check(_lib.tmq_apply_Qhat_nd(self._h, ctypes.byref(p), sign, pr, _hptr(src, n, "in"),
                                          _hptr(out, n, "out")), "tmq_apply_Qhat_nd")
            return out
        import torch

        out = torch.empty_like(src) if out is None else out
        _check(_lib.tmq_apply_Qhat_nd_dev(self._h, ctypes.byref(p), sign, pr, _dptr(src, n, "in"),
                                          _dptr(out, n, "out"), _stream(stream)), "tmq_apply_Qhat_nd_dev")
        return out

    def solve_nd(self, p: tmq_nd_params, b, opts: tmq_solver_opts, x=None, stream=None, check=True):
        """Solve Qhat_h^+ Qhat_h^- x = b for a doublet (2, V/2, 4, 3); returns (x, SolveInfo)."""
        n = self.V * 12
        info = tmq_solve_info()
        if isinstance(b, np.ndarray):
            x = np.empty_like(b) if x is None else x
            code = _lib.tmq_solve_nd(self._h, ctypes.byref(p), ctypes.byref(opts), _hptr(b, n, "b"),
                                     _hptr(x, n, "x"), ctypes.byref(info))
        else:
            import torch

            x = torch.empty_like(b) if x is None else x
            code = _lib.tmq_solve_nd_dev(self._h, ctypes.byref(p), ctypes.byref(opts), _dptr(b, n, "b"),
                                         _dptr(x, n, "x"), _stream(stream), ctypes.byref(info))
        if check:
            _check(code, "tmq_solve_nd")
        return x, _info(info)

    def solve_nd_batch(self, ps, bs, opts: tmq_solver_opts, xs=None, stream=None, check=True):
        """Solve a batch of doublets (device tensors (2, V/2, 4, 3)); returns (list of x, list of SolveInfo)."""
        import torch

        n = len(bs)
        if len(ps) != n or not 1 <= n <= MAX_RHS // 2:
            raise ValueError(f"need 1..{MAX_RHS // 2} doublets and one params per doublet")
        nc = self.V * 12
        parr = (tmq_nd_params * n)(*ps)
        infos = (tmq_solve_info * n)()
        xs = [torch.empty_like(b) for b in bs] if xs is None else xs
        bp = (ctypes.c_void_p * n)(*[_dptr(b, nc, "b").value for b in bs])
        xp = (ctypes.c_void_p * n)(*[_dptr(x, nc, "x").value for x in xs])
        code = _lib.tmq_solve_nd_batch_dev(self._h, n, parr, ctypes.byref(opts), bp, xp, _stream(stream), infos)
        if check:
            _check(code, "tmq_solve_nd_batch")
        return xs, [_info(i) for i in infos]

    def solve_full(self, p: tmq_params, b, opts: tmq_solver_opts, x=None, stream=None, check=True):
        """Solve Q^+ Q^- x = b on the full lattice (FP64 CG); device tensors (V, 4, 3)."""
        import torch

        n = self.V * 12
        info = tmq_solve_info()
        x = torch.empty_like(b) if x is None else x
        code = _lib.tmq_solve_full_dev(self._h, ctypes.byref(p), ctypes.byref(opts), _dptr(b, n, "b"),
                                       _dptr(x, n, "x"), _stream(stream), ctypes.byref(info))
        if check:
            _check(code, "tmq_solve_full")
        return x, _info(info)

    def solve_M(self, p: tmq_params, sign: int, phi, opts: tmq_solver_opts, psi=None, stream=None, check=True):
        """Solve M^{sign} psi = phi on the full lattice through the even/odd
        factorisation; phi: (V, 4, 3) device tensor or host array; returns (psi, SolveInfo)."""
        n = self.V * 12
        info = tmq_solve_info()
        if isinstance(phi, np.ndarray):
            psi = np.empty_like(phi) if psi is None else psi
            code = _lib.tmq_solve_M(self._h, ctypes.byref(p), sign, ctypes.byref(opts), _hptr(phi, n, "phi"),
                                    _hptr(psi, n, "psi"), ctypes.byref(info))
        else:
            import torch

            psi = torch.empty_like(phi) if psi is None else psi
            code = _lib.tmq_solve_M_dev(self._h, ctypes.byref(p), sign, ctypes.byref(opts), _dptr(phi, n, "phi"),
                                        _dptr(psi, n, "psi"), _stream(stream), ctypes.byref(info))
        if check:
            _check(code, "tmq_solve_M")
        return psi, _info(info)

    def split_eo(self, full, stream=None):
        """Split a full (V, 4, 3) complex128 field (device tensor or host array)
        into its (even, odd) parts, each (V/2, 4, 3)."""
        n, nh = self.V * 12, self.V // 2 * 12
        if isinstance(full, np.ndarray):
            ev = np.empty((self.V // 2, 4, 3), np.complex128)
            od = np.empty_like(ev)
            _check(_lib.tmq_split_eo(self._h, _hptr(full, n, "full"), _hptr(ev, nh, "even"), _hptr(od, nh, "odd")),
                   "tmq_split_eo")
        else:
            import torch

            ev = torch.empty((self.V // 2, 4, 3), dtype=torch.complex128, device=full.device)
            od = torch.empty_like(ev)
            _check(_lib.tmq_split_eo_dev(self._h, _dptr(full, n, "full"), _dptr(ev, nh, "even"), _dptr(od, nh, "odd"),
                                         _stream(stream)), "tmq_split_eo")
        return ev, od

    def merge_eo(self, even, odd, stream=None):
        """Merge (even, odd) parts (either may be None: zero) into a full (V, 4, 3) field."""
        n, nh = self.V * 12, self.V // 2 * 12
        ref = even if even is not None else odd
        if isinstance(ref, np.ndarray):
            full = np.empty((self.V, 4, 3), np.complex128)
            e = _hptr(even, nh, "even") if even is not None else None
            o = _hptr(odd, nh, "odd") if odd is not None else None
            _check(_lib.tmq_merge_eo(self._h, e, o, _hptr(full, n, "full")), "tmq_merge_eo")
        else:
            import torch

            full = torch.empty((self.V, 4, 3), dtype=torch.complex128, device=ref.device)
            e = _dptr(even, nh, "even") if even is not None else None
            o = _dptr(odd, nh, "odd") if odd is not None else None
            _check(_lib.tmq_merge_eo_dev(self._h, e, o, _dptr(full, n, "full"), _stream(stream)), "tmq_merge_eo")
        return full

    def solve_M_batch(self, p: tmq_params, sign: int, phis, opts: tmq_solver_opts, psis=None, stream=None,
                      check=True):
        """M^{sign} psi_r = phi_r for a batch of full-lattice sources (device tensors (V, 4, 3)) with common
        parameters; returns (list of psi, list of SolveInfo)."""
        import torch

        n = len(phis)
        if not 1 <= n <= MAX_RHS:
            raise ValueError(f"need 1..{MAX_RHS} sources")
        nc = self.V * 12
        psis = [torch.empty_like(f) for f in phis] if psis is None else psis
        infos = (tmq_solve_info * n)()
        pp = (ctypes.c_void_p * n)(*[_dptr(f, nc, "phi").value for f in phis])
        qp = (ctypes.c_void_p * n)(*[_dptr(f, nc, "psi").value for f in psis])
        code = _lib.tmq_solve_M_batch_dev(self._h, ctypes.byref(p), sign, ctypes.byref(opts), n, pp, qp,
                                          _stream(stream), infos)
        if check:
            _check(code, "tmq_solve_M_batch")
        return psis, [_info(i) for i in infos]

    # ---------------------------------------------------------- diagnostics
    def set_kernel_timing(self, on: bool):
        _check(_lib.tmq_set_kernel_timing(self._h, 1 if on else 0), "tmq_set_kernel_timing")

    def kernel_stats(self, family="hop"):
        n = ctypes.c_int(0)
        ms = ctypes.c_double(0)
        by = ctypes.c_double(0)
        fl = ctypes.c_double(0)
        _check(_lib.tmq_kernel_stats(self._h, family.encode(), ctypes.byref(n), ctypes.byref(ms),
                                     ctypes.byref(by), ctypes.byref(fl)), "tmq_kernel_stats")
        return {"launches": n.value, "ms": ms.value, "bytes": by.value, "flops": fl.value}

    def tuning_report(self) -> dict:
        import json

        buf = ctypes.create_string_buffer(1 << 14)
        _check(_lib.tmq_tuning_report(self._h, buf, len(buf)), "tmq_tuning_report")
        return json.loads(buf.value.decode())

    def encode(self, src, prec="fp16", stream=None):
        """Encode (n,4,3) complex128 device sites to 16-bit codes: returns (codes int16 (n,24), scale f32 (n,))."""
        import torch

        n_sites = src.numel() // 12
        codes = torch.empty((n_sites, 24), dtype=torch.int16, device=src.device)
        scale = torch.empty((n_sites,), dtype=torch.float32, device=src.device)
        _check(_lib.tmq_encode_dev(self._h, PREC[prec], n_sites, _dptr(src, n_sites * 12, "in"),
                                   ctypes.c_void_p(codes.data_ptr()), ctypes.c_void_p(scale.data_ptr()),
                                   _stream(stream)), "tmq_encode_dev")
        return codes, scale


class Server:
    """A solve server on one GPU (tmq_server_*): registered lattices stay
    resident; submitted solves are batched continuously per lattice and inner
    precision, admitted within a device-memory budget, and finish
    independently.  Sources and solutions are device tensors (V/2, 4, 3)
    complex128; the server keeps references to them until the request has
    been collected with poll() or wait()."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, max_batch: int = 0):
        cfg = tmq_server_config()
        cfg.budget_bytes = int(budget_bytes)
        cfg.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        _check(_lib.tmq_server_create(device, ctypes.byref(cfg), ctypes.byref(h)), "tmq_server_create")
        self._h = h
        self.device = device
        self._vh = {}
        self._live = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.tmq_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def add_lattice(self, dims, U) -> int:
        """Register a lattice (T, LZ, LY, LX) with its gauge field U (device tensor)."""
        dims = tuple(int(d) for d in dims)
        V = int(np.prod(dims))
        lid = ctypes.c_int(-1)
        _check(_lib.tmq_server_add_lattice(self._h, (ctypes.c_int * 4)(*dims), _dptr(U, V * 36, "U"),
                                           ctypes.byref(lid)), "tmq_server_add_lattice")
        self._vh[lid.value] = V // 2
        return lid.value

    def submit(self, lattice_id: int, p: tmq_params, b, opts: tmq_solver_opts, x=None, sync=True) -> int:
        """Queue a solve; sync: first wait for the current stream (the server's
        streams do not order themselves after the caller's work on b)."""
        import torch

        if sync:
            torch.cuda.current_stream().synchronize()
        if lattice_id not in self._vh:
            raise ValueError(f"unknown lattice id {lattice_id}")
        n = self._vh[lattice_id] * 12
        x = torch.empty_like(b) if x is None else x
        t = ctypes.c_uint64(0)
        _check(_lib.tmq_server_submit(self._h, lattice_id, ctypes.byref(p), ctypes.byref(opts), _dptr(b, n, "b"),
                                      _dptr(x, n, "x"), ctypes.byref(t)), "tmq_server_submit")
        self._live[t.value] = (b, x)
        return t.value

    def _finish(self, ticket: int, code: int, info: tmq_solve_info, where: str):
        # a finished request returns its solve status; EINVAL only for an unknown ticket
        if code == TMQ_EINVAL:
            _check(code, where)
        _b, x = self._live.pop(ticket, (None, None))
        return x, _info(info)

    def poll(self, ticket: int):
        """None while pending, else (x, SolveInfo) (the ticket is then retired)."""
        info = tmq_solve_info()
        code = _lib.tmq_server_poll(self._h, ticket, ctypes.byref(info))
        if code == TMQ_PENDING:
            return None
        return self._finish(ticket, code, info, "tmq_server_poll")

    def wait(self, ticket: int, timeout: float | None = None):
        """(x, SolveInfo) once finished; TimeoutError after `timeout` seconds."""
        info = tmq_solve_info()
        code = _lib.tmq_server_wait(self._h, ticket, -1.0 if timeout is None else float(timeout),
                                    ctypes.byref(info))
        if code == TMQ_PENDING:
            raise TimeoutError(f"request {ticket} still pending after {timeout} s")
        return self._finish(ticket, code, info, "tmq_server_wait")

    def stats(self) -> dict:
        st = tmq_server_stats()
        _check(_lib.tmq_server_get_stats(self._h, ctypes.byref(st)), "tmq_server_get_stats")
        return {f: getattr(st, f) for f, _ in tmq_server_stats._fields_}

    def reset_stats(self):
        _check(_lib.tmq_server_reset_stats(self._h), "tmq_server_reset_stats")
