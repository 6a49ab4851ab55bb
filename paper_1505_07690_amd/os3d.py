"""Python binding of libos3d (the C ABI declared in include/os3d.h).

Argument marshalling only: every step of the transform runs in the HIP
library.  PyTorch provides device memory and the current stream.  There is
no CPU fallback: if libos3d.so is missing the import of this module fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libos3d.so")

OS3D_C64, OS3D_BF16X2, OS3D_F16X2 = 0, 1, 2
DTYPES = {"c64": OS3D_C64, "bf16": OS3D_BF16X2, "fp16": OS3D_F16X2}
VARIANTS = {"cake": 0, "plate": 1}
COEFFS = {"lsq": 0, "quadrature": 1}


class OS3DError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"os3d status {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("s_theta", ctypes.c_double), ("k", ctypes.c_int32),
                ("taylor_N", ctypes.c_int32), ("gamma", ctypes.c_double), ("eps", ctypes.c_double),
                ("variant", ctypes.c_int32), ("coeffs", ctypes.c_int32)]


class BankInfo(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int64 * 3), ("n_orients", ctypes.c_int32), ("n_unique", ctypes.c_int32),
                ("paired", ctypes.c_int32), ("kappa", ctypes.c_double), ("approx_norm", ctypes.c_double),
                ("M_dev", ctypes.c_void_p)]


_lib = None

_SIGS = {
    "os3d_wavelet_coeffs": [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p],
    "os3d_steering_matrix": [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p],
    "os3d_bank_bytes": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Params),
                        ctypes.POINTER(ctypes.c_size_t)],
    "os3d_build_bank": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_void_p,
                        ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "os3d_free_bank": [ctypes.c_void_p],
    "os3d_get_bank_info": [ctypes.c_void_p, ctypes.POINTER(BankInfo)],
    "os3d_bank_psi": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p],
    "os3d_bank_M": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "os3d_workspace_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "os3d_forward": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "os3d_adjoint": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "os3d_reconstruct": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "os3d_reconstruct_noalloc": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                 ctypes.c_void_p, ctypes.c_void_p],
    "os3d_reconstruct_approx": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                ctypes.c_void_p, ctypes.c_void_p],
    "os3d_process": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "os3d_stream_probe": [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "os3d_profile_enable": [ctypes.c_int32],
    "os3d_profile_count": [ctypes.POINTER(ctypes.c_int32)],
    "os3d_profile_get": [ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_int64),
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_double)],
}


def lib():
    """The loaded libos3d (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1505_07690_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.os3d_last_error.restype = ctypes.c_char_p
        L.os3d_last_error.argtypes = []
        L.os3d_version.restype = ctypes.c_char_p
        L.os3d_version.argtypes = []
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise OS3DError(rc, lib().os3d_last_error().decode())


def make_params(L=16, s_theta=0.7, k=2, taylor_N=20, gamma=0.8, eps=1e-3, variant="cake", coeffs="lsq"):
    return Params(int(L), float(s_theta), int(k), int(taylor_N), float(gamma), float(eps),
                  VARIANTS[variant] if isinstance(variant, str) else int(variant),
                  COEFFS[coeffs] if isinstance(coeffs, str) else int(coeffs))


def _as_params(p):
    if isinstance(p, Params):
        return p
    if isinstance(p, dict):
        return make_params(**p)
    # any object with the attributes (e.g. the oracle's WaveletParams)
    return make_params(p.L, p.s_theta, p.k, p.taylor_N, p.gamma, p.eps, getattr(p, "variant", "cake"),
                       getattr(p, "coeffs", "lsq"))


def _orients(o):
    o = np.ascontiguousarray(np.asarray(o, dtype=np.float64).reshape(-1, 3))
    return o


def wavelet_coeffs(params):
    """Host FP64 coefficients (c_l, a_l) of the window and the wavelet profile."""
    p = _as_params(params)
    c = np.zeros(p.L + 1)
    a = np.zeros(p.L + 1)
    _check(lib().os3d_wavelet_coeffs(ctypes.byref(p), c.ctypes.data, a.ctypes.data))
    return c, a


def steering_matrix(params, orients):
    """Host FP64 steering matrix [(L+1)^2][N_o] in the standard (l*l+l+m) order."""
    p = _as_params(params)
    o = _orients(orients)
    S = np.zeros(((p.L + 1) ** 2, o.shape[0]))
    _check(lib().os3d_steering_matrix(ctypes.byref(p), o.ctypes.data, o.shape[0], S.ctypes.data))
    return S


def bank_bytes(shape, orients, params):
    p = _as_params(params)
    o = _orients(orients)
    dims = (ctypes.c_int64 * 3)(*[int(s) for s in shape])
    n = ctypes.c_size_t()
    _check(lib().os3d_bank_bytes(dims, o.ctypes.data, o.shape[0], ctypes.byref(p), ctypes.byref(n)))
    return n.value


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Bank:
    """A wavelet bank resident on the GPU (device buffer owned by torch)."""

    def __init__(self, shape, orients, params, device="cuda", stream=None):
        import torch
        self.shape = tuple(int(s) for s in shape)
        self.orients = _orients(orients)
        self.params = _as_params(params)
        self.n_orients = self.orients.shape[0]
        if torch.device(device).type != "cuda":
            raise ValueError(f"a bank lives on a GPU, not on {device}")
        nbytes = bank_bytes(self.shape, self.orients, self.params)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.device = self.buf.device
        dims = (ctypes.c_int64 * 3)(*self.shape)
        h = ctypes.c_void_p()
        _check(lib().os3d_build_bank(dims, self.orients.ctypes.data, self.n_orients, ctypes.byref(self.params),
                                     ctypes.c_void_p(self.buf.data_ptr()), nbytes, _stream_ptr(stream),
                                     ctypes.byref(h)))
        self.handle = h
        info = BankInfo()
        _check(lib().os3d_get_bank_info(self.handle, ctypes.byref(info)))
        self.kappa = info.kappa
        self.approx_norm = info.approx_norm
        self.n_unique = info.n_unique
        self.paired = bool(info.paired)
        n = ctypes.c_size_t()
        _check(lib().os3d_workspace_bytes(self.handle, ctypes.byref(n)))
        self.ws_bytes = n.value
        self._ws = None

    @property
    def V(self):
        return self.shape[0] * self.shape[1] * self.shape[2]

    def workspace(self):
        """The bank's own workspace (the default of the compute calls).  Calls
        that run concurrently on different streams must pass workspaces of
        their own (`ws=`); the bank itself may be shared."""
        import torch
        if self._ws is None:
            self._ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def psi(self, i, stream=None):
        """psi_hat_i as a float32 [Nz, Ny, Nx] device tensor (natural DFT order)."""
        import torch
        out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        _check(lib().os3d_bank_psi(self.handle, int(i), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def M(self, stream=None):
        import torch
        out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        _check(lib().os3d_bank_M(self.handle, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.os3d_free_bank(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _same_device(t, device):
    return t.device.type == device.type and (t.device.index or 0) == (device.index or 0)


def _need(t, name, shape, dtypes, device):
    """Every tensor handed to the library is checked here, before any call:
    a pointer of the wrong device, size or type would reach the kernels."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor, got {type(t).__name__}")
    if not _same_device(t, device):
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} must be {' or '.join(str(d) for d in dtypes)}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _workspace(ws, bank):
    """(pointer, bytes) of the workspace; the library checks the size."""
    ws = bank.workspace() if ws is None else ws
    if not _same_device(ws, bank.device) or not ws.is_contiguous():
        raise ValueError(f"the workspace must be a contiguous tensor on {bank.device}")
    return ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()


def _batched(f, bank):
    import torch
    if f.dim() == 3:
        _need(f, "f", bank.shape, (torch.float32,), bank.device)
        return f.unsqueeze(0), True
    if f.dim() == 4:
        _need(f, "f", (f.shape[0],) + bank.shape, (torch.float32,), bank.device)
        if f.shape[0] < 1:
            raise ValueError("the batch of f is empty")
        return f, False
    raise ValueError(f"expected f of shape [B, {bank.shape}] or {bank.shape}, got {tuple(f.shape)}")


def _scores(U, bank, dtype):
    """U as [B, N_o, Nz, Ny, Nx] of the storage type of `dtype`."""
    import torch
    code = DTYPES[dtype]
    Ub = U if U.dim() == 5 else U.unsqueeze(0)
    _need(Ub, "U", (Ub.shape[0], bank.n_orients) + bank.shape,
          (torch.complex64,) if code == OS3D_C64 else (torch.int32,), bank.device)
    if Ub.shape[0] < 1:
        raise ValueError("the batch of U is empty")
    return Ub, code


def _scales_arg(scales, B, bank, code):
    import torch
    if code == OS3D_C64:
        return None
    if scales is None:
        raise ValueError("16-bit scores need their scales")
    sc = scales if scales.dim() == 2 else scales.unsqueeze(0)
    return _need(sc, "scales", (B, bank.n_orients), (torch.float32,), bank.device)


def forward(f, bank, dtype="c64", ws=None, out=None, scales=None, stream=None):
    """U = W f (Eq. 7) for a float32 device volume f [B, Nz, Ny, Nx] (or [Nz, Ny, Nx]).
    Returns (U, scales): U is complex64 [B, N_o, Nz, Ny, Nx] for "c64", else an
    int32 tensor of packed 16-bit (re, im) pairs with float32 scales [B, N_o]."""
    import torch
    fb, single = _batched(f, bank)
    B = fb.shape[0]
    code = DTYPES[dtype]
    udt = torch.complex64 if code == OS3D_C64 else torch.int32
    if out is None:
        out = torch.empty((B, bank.n_orients) + bank.shape, dtype=udt, device=bank.device)
    else:
        _need(out if out.dim() == 5 else out.unsqueeze(0), "out", (B, bank.n_orients) + bank.shape, (udt,),
              bank.device)
    if code != OS3D_C64:
        if scales is None:
            scales = torch.empty((B, bank.n_orients), dtype=torch.float32, device=bank.device)
        _scales_arg(scales, B, bank, code)
    wp, wb = _workspace(ws, bank)
    _check(lib().os3d_forward(bank.handle, ctypes.c_void_p(fb.data_ptr()), B, ctypes.c_void_p(out.data_ptr()), code,
                              ctypes.c_void_p(scales.data_ptr() if code != OS3D_C64 else 0),
                              wp, wb, _stream_ptr(stream)))
    if single and out.dim() == 5:
        out = out[0]
        scales = scales[0] if scales is not None and scales.dim() == 2 else scales
    return out, (scales if code != OS3D_C64 else None)


def _volume_out(out, B, bank):
    import torch
    if out is None:
        return torch.empty((B,) + bank.shape, dtype=torch.float32, device=bank.device)
    _need(out if out.dim() == 4 else out.unsqueeze(0), "out", (B,) + bank.shape, (torch.float32,), bank.device)
    return out


def _reduce(fn, U, bank, scales, dtype, ws, out, stream):
    Ub, code = _scores(U, bank, dtype)
    B = Ub.shape[0]
    out = _volume_out(out, B, bank)
    sc = _scales_arg(scales, B, bank, code)
    wp, wb = _workspace(ws, bank)
    _check(fn(bank.handle, ctypes.c_void_p(Ub.data_ptr()), code, ctypes.c_void_p(sc.data_ptr() if sc is not None else 0),
              B, ctypes.c_void_p(out.data_ptr()), wp, wb, _stream_ptr(stream)))
    return out if U.dim() == 5 or out.dim() == 3 else out[0]


def adjoint(U, bank, scales=None, dtype="c64", ws=None, out=None, stream=None):
    """W* U = Re IDFT(sum_i psi_hat_i DFT(U_i))."""
    return _reduce(lib().os3d_adjoint, U, bank, scales, dtype, ws, out, stream)


def reconstruct(U, bank, scales=None, dtype="c64", ws=None, out=None, stream=None):
    """Stabilised exact reconstruction, Eq. (8) with max(M, eps)."""
    return _reduce(lib().os3d_reconstruct, U, bank, scales, dtype, ws, out, stream)


def reconstruct_noalloc(U, bank, scales=None, dtype="c64", out=None, stream=None):
    """os3d_reconstruct with the library's static device scratch instead of a
    workspace (no device allocation inside the call; volumes up to 2^22
    voxels; calls that overlap on one device race)."""
    Ub, code = _scores(U, bank, dtype)
    B = Ub.shape[0]
    out = _volume_out(out, B, bank)
    sc = _scales_arg(scales, B, bank, code)
    _check(lib().os3d_reconstruct_noalloc(bank.handle, ctypes.c_void_p(Ub.data_ptr()), code,
                                          ctypes.c_void_p(sc.data_ptr() if sc is not None else 0), B,
                                          ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out if U.dim() == 5 or out.dim() == 3 else out[0]


def reconstruct_approx(U, bank, scales=None, dtype="c64", out=None, stream=None):
    """Approximate reconstruction of Eq. (6): Re(sum_i U_i) / S."""
    Ub, code = _scores(U, bank, dtype)
    B = Ub.shape[0]
    out = _volume_out(out, B, bank)
    sc = _scales_arg(scales, B, bank, code)
    _check(lib().os3d_reconstruct_approx(bank.handle, ctypes.c_void_p(Ub.data_ptr()), code,
                                         ctypes.c_void_p(sc.data_ptr() if sc is not None else 0), B,
                                         ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out if U.dim() == 5 or out.dim() == 3 else out[0]


PHIS = {"identity": 0, "soft_threshold": 1}


def process(f, bank, phi="soft_threshold", power=1.5, ws=None, out=None, stream=None):
    """Processing via scores, Eq. (23): Re W^+ Phi(W f) with a pointwise Phi
    ("identity" or "soft_threshold": |U|^power sgn(U))."""
    fb, single = _batched(f, bank)
    B = fb.shape[0]
    out = _volume_out(out, B, bank)
    if phi not in PHIS:
        raise ValueError(f"phi must be one of {sorted(PHIS)}")
    wp, wb = _workspace(ws, bank)
    _check(lib().os3d_process(bank.handle, ctypes.c_void_p(fb.data_ptr()), B, PHIS[phi], float(power),
                              ctypes.c_void_p(out.data_ptr()), wp, wb, _stream_ptr(stream)))
    return out[0] if single and out.dim() == 4 else out


def unpack16(Uq, scales, dtype):
    """Packed 16-bit score pairs -> complex64 (a test/inspection helper on the
    device; the library itself dequantises inside its kernels)."""
    import torch
    q = Uq.contiguous().view(torch.int16).reshape(Uq.shape + (2,))
    t = torch.float16 if dtype == "fp16" else torch.bfloat16
    v = q.view(t).to(torch.float32)
    s = scales.reshape(scales.shape + (1,) * (Uq.dim() - scales.dim())).to(torch.float32)
    return torch.complex(v[..., 0] * s, v[..., 1] * s)


STREAM_KINDS = {"copy": 0, "read": 1, "write": 2, "read_nt": 3}


def stream_probe(kind, src, dst, stream=None):
    """One pass of the library's plain copy / read / write kernel over the
    device tensors (measurement support)."""
    nbytes = (dst if kind == "write" else src).numel() * (dst if kind == "write" else src).element_size()
    _check(lib().os3d_stream_probe(STREAM_KINDS[kind], ctypes.c_void_p(src.data_ptr() if src is not None else 0),
                                   ctypes.c_void_p(dst.data_ptr()), nbytes, _stream_ptr(stream)))


def profile_enable(on=True, kernel=None):
    """Per-kernel HIP-event timing inside the library (clears old records):
    every launch, or with kernel=<slot name> only that kernel's launches."""
    if not on:
        mode = 0
    elif kernel is None:
        mode = 1
    else:
        mode = 2 + profile_slots().index(kernel)
    _check(lib().os3d_profile_enable(mode))


def profile_slots():
    """Names of the library's kernel timing slots, in slot order."""
    n = ctypes.c_int32()
    _check(lib().os3d_profile_count(ctypes.byref(n)))
    names = []
    for i in range(n.value):
        name = ctypes.c_char_p()
        launches, ms, by, fl = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        lib().os3d_profile_get(i, ctypes.byref(name), ctypes.byref(launches), ctypes.byref(ms), ctypes.byref(by),
                               ctypes.byref(fl))
        names.append(name.value.decode())
    return names


def profile_read():
    """{kernel name: (launches, total ms, algorithmic bytes, algorithmic flops)}
    of the records since profile_enable (waits for the recorded events)."""
    n = ctypes.c_int32()
    _check(lib().os3d_profile_count(ctypes.byref(n)))
    out = {}
    for i in range(n.value):
        name = ctypes.c_char_p()
        cnt = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        fl = ctypes.c_double()
        _check(lib().os3d_profile_get(i, ctypes.byref(name), ctypes.byref(cnt), ctypes.byref(ms), ctypes.byref(by),
                                      ctypes.byref(fl)))
        if cnt.value:
            out[name.value.decode()] = (cnt.value, ms.value, by.value, fl.value)
    return out
