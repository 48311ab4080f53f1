"""ctypes binding of libircur (the C ABI declared in include/ircur.h).

Argument marshalling only: every step of IRCUR runs in the library's HIP
kernels.  torch tensors supply device memory and the stream.  The library is
loaded on first use; a missing library raises instead of falling back.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("IRCUR_LIBRARY") or os.path.join(_PKG, "libircur.so")

OK, NOT_CONVERGED, WARN_RANK_DEFICIENT, WARN_SVD_INEXACT = 0, 1, 2, 3
ERR_ARG, ERR_ALLOC, ERR_DEVICE, ERR_SVD, ERR_NONFINITE, ERR_STATE, ERR_UNSUPPORTED = -1, -2, -3, -4, -5, -6, -7
F64, F32, BF16 = 0, 1, 2
MAX_RANK = 32


class Params(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int64), ("n2", ctypes.c_int64), ("ldD", ctypes.c_int64),
        ("r", ctypes.c_int32), ("sI", ctypes.c_int32), ("sJ", ctypes.c_int32),
        ("dtype", ctypes.c_int32), ("resample", ctypes.c_int32), ("err_mode", ctypes.c_int32),
        ("zeta0", ctypes.c_double), ("gamma", ctypes.c_double), ("eps", ctypes.c_double),
        ("max_iter", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("svd_tol", ctypes.c_double), ("svd_max_it", ctypes.c_int32), ("svd_block", ctypes.c_int32),
        ("zeta_sched", ctypes.POINTER(ctypes.c_double)),
    ]


class IrcurError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class Instance(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int64), ("n2", ctypes.c_int64), ("ldD", ctypes.c_int64),
        ("sI", ctypes.c_int32), ("sJ", ctypes.c_int32),
        ("D", ctypes.c_void_p), ("Dt", ctypes.c_void_p), ("ldDt", ctypes.c_int64),
        ("Wstar", ctypes.c_void_p), ("Vstar", ctypes.c_void_p), ("seed", ctypes.c_uint64),
    ]


_lib = None
_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_DP = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "ircur_params_default": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "ircur_init": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(Params), _P, _P, ctypes.c_int64, _P]),
    "ircur_step": (ctypes.c_int, [_P, _I32P, _I32P, _DP]),
    "ircur_enqueue": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ircur_sync": (ctypes.c_int, [_P, _I32P, _DP]),
    "ircur_solve": (ctypes.c_int, [_P, _I32P, _DP]),
    "ircur_reset": (ctypes.c_int, [_P]),
    "ircur_get_factors": (ctypes.c_int, [_P, _P, _P]),
    "ircur_set_factors": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "ircur_get_history": (ctypes.c_int, [_P, _DP, ctypes.c_int32, _I32P]),
    "ircur_get_sets": (ctypes.c_int, [_P, _I32P, _I32P]),
    "ircur_get_core": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "ircur_get_cur": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "ircur_to_svd": (ctypes.c_int, [_P, _P, _P, _P]),
    "ircur_to_svd_noalloc": (ctypes.c_int, [_P, _P, _P, _P]),
    "ircur_sparse_full": (ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "ircur_get_state": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_size_t)]),
    "ircur_set_state": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "ircur_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ircur_get_timing": (ctypes.c_int, [_P, _DP, ctypes.POINTER(ctypes.c_int64)]),
    "ircur_time_pass": (ctypes.c_int, [_P, ctypes.c_int32, _DP]),
    "ircur_time_sparse": (ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.c_int64, ctypes.c_int32, _DP]),
    "ircur_get_info": (ctypes.c_int, [_P, _I32P, _DP, _DP, _I32P]),
    "ircur_get_svd_history": (ctypes.c_int, [_P, _I32P, _DP, _I32P, ctypes.c_int32, _I32P]),
    "ircur_sample": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_int32, ctypes.c_int32, _I32P, _I32P]),
    "ircur_get_phase_profile": (ctypes.c_int, [_P, _DP]),
    "ircur_get_phase_profile2": (ctypes.c_int, [_P, _DP]),
    "ircur_unrolled_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(Instance), ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _P]),
    "ircur_unrolled_forward": (ctypes.c_int, [_P, _P, _P]),
    "ircur_backward": (ctypes.c_int, [_P, _P, _P]),
    "ircur_unrolled_get_factors": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "ircur_unrolled_get_sets": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _I32P, _I32P]),
    "ircur_unrolled_status": (ctypes.c_int, [_P, _I32P]),
    "ircur_unrolled_destroy": (None, [_P]),
    "ircur_unrolled_last_error": (ctypes.c_char_p, [_P]),
    "ircur_destroy": (None, [_P]),
    "ircur_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ircur_last_error": (ctypes.c_char_p, [_P]),
}


def lib():
    """Load libircur.so (raises FileNotFoundError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} is missing: build it with "
                                    "`python -m paper_2010_07422_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().ircur_strerror(code).decode()


def sample(seed: int, t: int, n1: int, n2: int, sI: int, sJ: int):
    """The library's index sampler (host): sorted I (sI of n1), J (sJ of n2)."""
    I = np.zeros(sI, np.int32)
    J = np.zeros(sJ, np.int32)
    rc = lib().ircur_sample(seed, t, n1, n2, sI, sJ, I.ctypes.data_as(_I32P), J.ctypes.data_as(_I32P))
    if rc != OK:
        raise IrcurError(rc, strerror(rc))
    return I, J


def _dtype_code(t):
    import torch
    return {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[t]


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _i32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(_I32P)


@dataclass
class Info:
    svd_iters: int
    svd_resid: float
    gap: float
    kept: int


class IRCUR:
    """One IRCUR context over a device matrix D (torch tensor, float64 /
    float32 / bfloat16, row-major with unit column stride)."""

    def __init__(self, D, r, sI, sJ, zeta0, gamma=0.7, eps=1e-5, max_iter=100, seed=0,
                 resample=True, err_mode=0, Dt=None, svd_tol=0.0, svd_max_it=0,
                 svd_block=0, stream=None, zeta_sched=None):
        import torch
        if not (isinstance(D, torch.Tensor) and D.is_cuda and D.dim() == 2 and D.stride(1) == 1):
            raise ValueError("D must be a 2-D CUDA tensor with unit column stride")
        self.D = D
        self.Dt = Dt
        self.dtype = _dtype_code(D.dtype)
        self.fdtype = torch.float64 if self.dtype == F64 else torch.float32
        p = Params()
        lib().ircur_params_default(ctypes.byref(p))
        p.n1, p.n2 = D.shape
        p.ldD = D.stride(0)
        p.r, p.sI, p.sJ = r, sI, sJ
        p.dtype = self.dtype
        p.resample = 1 if resample else 0
        p.err_mode = err_mode
        p.zeta0, p.gamma, p.eps = float(zeta0), float(gamma), float(eps)
        p.max_iter = max_iter
        p.seed = seed
        p.svd_tol, p.svd_max_it, p.svd_block = float(svd_tol), svd_max_it, svd_block
        sched = None
        if zeta_sched is not None:
            z = [float(v) for v in zeta_sched]
            if len(z) < max_iter:
                raise ValueError("zeta_sched needs max_iter entries")
            sched = (ctypes.c_double * max_iter)(*z[:max_iter])
            p.zeta_sched = ctypes.cast(sched, ctypes.POINTER(ctypes.c_double))
        self.p = p
        self.stream = stream
        h = ctypes.c_void_p()
        ldDt = 0 if Dt is None else Dt.stride(0)
        rc = lib().ircur_init(ctypes.byref(h), ctypes.byref(p), ctypes.c_void_p(D.data_ptr()),
                              None if Dt is None else ctypes.c_void_p(Dt.data_ptr()),
                              ldDt, _stream_handle(stream))
        if rc != OK:
            raise IrcurError(rc, "ircur_init: " + strerror(rc))
        self.h = h

    # ------------------------------------------------------------ control
    def _check(self, rc, what):
        if rc < 0:
            msg = lib().ircur_last_error(self.h).decode()
            raise IrcurError(rc, f"{what}: {strerror(rc)}: {msg}")
        return rc

    def step(self, I=None, J=None):
        e = ctypes.c_double()
        if I is None:
            rc = lib().ircur_step(self.h, None, None, ctypes.byref(e))
        else:
            Ia, Ip = _i32(I)
            Ja, Jp = _i32(J)
            rc = lib().ircur_step(self.h, Ip, Jp, ctypes.byref(e))
        self._check(rc, "ircur_step")
        return e.value

    def solve(self):
        it = ctypes.c_int32()
        e = ctypes.c_double()
        rc = self._check(lib().ircur_solve(self.h, ctypes.byref(it), ctypes.byref(e)), "ircur_solve")
        return it.value, e.value, rc

    def enqueue(self, n):
        self._check(lib().ircur_enqueue(self.h, n), "ircur_enqueue")

    def sync(self):
        k = ctypes.c_int32()
        e = ctypes.c_double()
        self._check(lib().ircur_sync(self.h, ctypes.byref(k), ctypes.byref(e)), "ircur_sync")
        return k.value, e.value

    def reset(self):
        self._check(lib().ircur_reset(self.h), "ircur_reset")

    # ------------------------------------------------------------ outputs
    def factors(self):
        """(A^T, B): r x n1 and r x n2 tensors, L_k = A B."""
        import torch
        n1, n2, r = self.p.n1, self.p.n2, self.p.r
        At = torch.empty((r, n1), dtype=self.fdtype, device=self.D.device)
        B = torch.empty((r, n2), dtype=self.fdtype, device=self.D.device)
        self._check(lib().ircur_get_factors(self.h, ctypes.c_void_p(At.data_ptr()),
                                            ctypes.c_void_p(B.data_ptr())), "ircur_get_factors")
        self._sync_stream()
        return At, B

    def set_factors(self, At, B, k):
        At = At.to(self.fdtype).contiguous()
        B = B.to(self.fdtype).contiguous()
        self._check(lib().ircur_set_factors(self.h, ctypes.c_void_p(At.data_ptr()),
                                            ctypes.c_void_p(B.data_ptr()), k), "ircur_set_factors")

    def history(self):
        cap = self.p.max_iter
        buf = np.zeros(cap, np.float64)
        n = ctypes.c_int32()
        self._check(lib().ircur_get_history(self.h, buf.ctypes.data_as(_DP), cap, ctypes.byref(n)),
                    "ircur_get_history")
        return buf[: n.value].tolist()

    def sets(self):
        I = np.zeros(self.p.sI, np.int32)
        J = np.zeros(self.p.sJ, np.int32)
        self._check(lib().ircur_get_sets(self.h, I.ctypes.data_as(_I32P), J.ctypes.data_as(_I32P)),
                    "ircur_get_sets")
        return I, J

    def core(self):
        """(M, Wt, Kc, Q) of the last iteration, float64 tensors, with
        H_r(M) = Wt @ Kc @ Q.T (Wt, Q orthonormal)."""
        import torch
        sI, sJ, r = self.p.sI, self.p.sJ, self.p.r
        dev = self.D.device
        M = torch.empty((sI, sJ), dtype=torch.float64, device=dev)
        W = torch.empty((sI, r), dtype=torch.float64, device=dev)
        K = torch.empty((r, r), dtype=torch.float64, device=dev)
        V = torch.empty((sJ, r), dtype=torch.float64, device=dev)
        self._check(lib().ircur_get_core(self.h, *(ctypes.c_void_p(t.data_ptr()) for t in (M, W, K, V))),
                    "ircur_get_core")
        self._sync_stream()
        return M, W, K, V

    def cur(self):
        """Output of Algorithm 1 for the last completed iteration: dict with
        C (n1 x sJ), Upinv (sJ x sI), R (sI x n2), S_I (sI x n2), S_J (n1 x sJ),
        in the factor dtype, plus the index sets I, J."""
        import torch
        n1, n2, sI, sJ = self.p.n1, self.p.n2, self.p.sI, self.p.sJ
        dev = self.D.device
        out = {"C": torch.empty((n1, sJ), dtype=self.fdtype, device=dev),
               "Upinv": torch.empty((sJ, sI), dtype=self.fdtype, device=dev),
               "R": torch.empty((sI, n2), dtype=self.fdtype, device=dev),
               "S_I": torch.empty((sI, n2), dtype=self.fdtype, device=dev),
               "S_J": torch.empty((n1, sJ), dtype=self.fdtype, device=dev)}
        self._check(lib().ircur_get_cur(self.h, *(ctypes.c_void_p(out[k].data_ptr())
                                                  for k in ("C", "Upinv", "R", "S_I", "S_J"))),
                    "ircur_get_cur")
        out["I"], out["J"] = self.sets()
        return out

    def to_svd(self, out=None, noalloc=False):
        """Algorithm 2 on the current factors: (W n1 x r, sigma r, V n2 x r),
        float64, L_k = W diag(sigma) V^T.  out: optional (W, sigma, V)
        tensors to fill; noalloc selects ircur_to_svd_noalloc."""
        import torch
        n1, n2, r = self.p.n1, self.p.n2, self.p.r
        dev = self.D.device
        if out is None:
            out = (torch.empty((n1, r), dtype=torch.float64, device=dev),
                   torch.empty((r,), dtype=torch.float64, device=dev),
                   torch.empty((n2, r), dtype=torch.float64, device=dev))
        for t, shape in zip(out, ((n1, r), (r,), (n2, r))):
            if t.dtype != torch.float64 or tuple(t.shape) != shape or not t.is_contiguous() or t.device != dev:
                raise ValueError("out must hold contiguous float64 tensors of shapes (n1, r), (r,), (n2, r)")
        name = "ircur_to_svd_noalloc" if noalloc else "ircur_to_svd"
        self._check(getattr(lib(), name)(self.h, *(ctypes.c_void_p(t.data_ptr()) for t in out)), name)
        return out

    def sparse_full(self, zeta=-1.0, out=None):
        """T_zeta(D - A_k B_k) over all of D in the dtype of D; zeta < 0 picks
        gamma^k zeta_0.  Returns (S, nnz)."""
        import torch
        n1, n2 = self.p.n1, self.p.n2
        S = torch.empty((n1, n2), dtype=self.D.dtype, device=self.D.device) if out is None else out
        if S.dim() != 2 or S.shape != (n1, n2) or S.stride(1) != 1 or S.dtype != self.D.dtype:
            raise ValueError("out must be an n1 x n2 tensor of D's dtype with unit column stride")
        nnz = ctypes.c_int64()
        self._check(lib().ircur_sparse_full(self.h, float(zeta), ctypes.c_void_p(S.data_ptr()), S.stride(0),
                                            ctypes.byref(nnz)), "ircur_sparse_full")
        return S, nnz.value

    def info(self):
        it = ctypes.c_int32()
        res = ctypes.c_double()
        gap = ctypes.c_double()
        kept = ctypes.c_int32()
        self._check(lib().ircur_get_info(self.h, ctypes.byref(it), ctypes.byref(res), ctypes.byref(gap),
                                         ctypes.byref(kept)), "ircur_get_info")
        return Info(it.value, res.value, gap.value, kept.value)

    def svd_history(self):
        """Per completed iteration: (subspace iterations, Ritz gap estimate
        sigma_{r+1}/sigma_r or -1, kept components), as three lists."""
        cap = self.p.max_iter
        it = np.zeros(cap, np.int32)
        gap = np.zeros(cap, np.float64)
        kept = np.zeros(cap, np.int32)
        n = ctypes.c_int32()
        self._check(lib().ircur_get_svd_history(self.h, it.ctypes.data_as(_I32P), gap.ctypes.data_as(_DP),
                                                kept.ctypes.data_as(_I32P), cap, ctypes.byref(n)),
                    "ircur_get_svd_history")
        m = n.value
        return it[:m].tolist(), gap[:m].tolist(), kept[:m].tolist()

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        self._check(lib().ircur_get_state(self.h, None, ctypes.byref(n)), "ircur_get_state")
        buf = ctypes.create_string_buffer(n.value)
        self._check(lib().ircur_get_state(self.h, buf, ctypes.byref(n)), "ircur_get_state")
        return buf.raw[: n.value]

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(lib().ircur_set_state(self.h, buf, len(blob)), "ircur_set_state")

    def set_timing(self, on: bool):
        self._check(lib().ircur_set_timing(self.h, 1 if on else 0), "ircur_set_timing")

    def timing(self):
        ms = (ctypes.c_double * 4)()
        cnt = ctypes.c_int64()
        self._check(lib().ircur_get_timing(self.h, ms, ctypes.byref(cnt)), "ircur_get_timing")
        return list(ms), cnt.value

    def time_pass(self, reps=200):
        """Mean duration in microseconds of the last iteration's pass kernel,
        launched `reps` times back to back between two HIP events."""
        us = ctypes.c_double()
        self._check(lib().ircur_time_pass(self.h, int(reps), ctypes.byref(us)), "ircur_time_pass")
        return us.value

    def time_sparse(self, S, zeta=-1.0, reps=10):
        """Mean duration in microseconds of the full sparse-part extraction
        into S (an n1 x n2 tensor of D's dtype), launched `reps` times back to
        back between two HIP events."""
        n1, n2 = self.p.n1, self.p.n2
        if S.dim() != 2 or S.shape != (n1, n2) or S.stride(1) != 1 or S.dtype != self.D.dtype:
            raise ValueError("S must be an n1 x n2 tensor of D's dtype with unit column stride")
        us = ctypes.c_double()
        self._check(lib().ircur_time_sparse(self.h, float(zeta), ctypes.c_void_p(S.data_ptr()), S.stride(0),
                                            int(reps), ctypes.byref(us)), "ircur_time_sparse")
        return us.value

    def phase_profile(self, second=False):
        buf = (ctypes.c_double * 16)()
        name = "ircur_get_phase_profile2" if second else "ircur_get_phase_profile"
        self._check(getattr(lib(), name)(self.h, buf), name)
        return list(buf)

    def _sync_stream(self):
        import torch
        (torch.cuda.current_stream() if self.stream is None else self.stream).synchronize()

    def close(self):
        if getattr(self, "h", None):
            lib().ircur_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ unrolled

class IRCURUnrolled:
    """A batch of independent instances for the unrolled, differentiable mode.

    instances: list of (D, W*, V*, sI, sJ, seed) with D a CUDA tensor (float64
    or float32, all the same dtype) and W*, V* its target factors (n1 x r,
    n2 x r, same dtype).  K steps, rank r, gate width tau_rel.
    """

    def __init__(self, instances, r, K, tau_rel=0.05, stream=None):
        import torch
        if not instances:
            raise ValueError("empty batch")
        dt = instances[0][0].dtype
        if dt not in (torch.float64, torch.float32):
            raise ValueError("the unrolled mode takes float64 or float32 data")
        self.dtype = F64 if dt == torch.float64 else F32
        self.tdtype = dt
        self.r, self.K, self.nb = r, K, len(instances)
        self.stream = stream
        self._keep = []
        arr = (Instance * self.nb)()
        self.shapes = []
        for b, (D, Ws, Vs, sI, sJ, seed) in enumerate(instances):
            if not (D.is_cuda and D.dim() == 2 and D.stride(1) == 1 and D.dtype == dt):
                raise ValueError("every D must be a 2-D CUDA tensor of the batch dtype with unit column stride")
            Ws = Ws.to(dt).contiguous()
            Vs = Vs.to(dt).contiguous()
            if Ws.shape != (D.shape[0], r) or Vs.shape != (D.shape[1], r):
                raise ValueError("W* must be n1 x r and V* n2 x r")
            self._keep += [D, Ws, Vs]
            it = arr[b]
            it.n1, it.n2 = D.shape
            it.ldD = D.stride(0)
            it.sI, it.sJ = sI, sJ
            it.D = D.data_ptr()
            it.Dt = None
            it.ldDt = 0
            it.Wstar, it.Vstar = Ws.data_ptr(), Vs.data_ptr()
            it.seed = seed
            self.shapes.append((D.shape[0], D.shape[1], sI, sJ))
        h = ctypes.c_void_p()
        rc = lib().ircur_unrolled_create(ctypes.byref(h), arr, self.nb, r, K, self.dtype, float(tau_rel),
                                         _stream_handle(stream))
        if rc != OK:
            raise IrcurError(rc, "ircur_unrolled_create: " + strerror(rc))
        self.h = h
        self.device = instances[0][0].device

    def _check(self, rc, what):
        if rc < 0:
            raise IrcurError(rc, f"{what}: {strerror(rc)}: {lib().ircur_unrolled_last_error(self.h).decode()}")
        return rc

    def forward(self, zeta):
        """Losses (nb,) float64 for thresholds zeta (K,)."""
        import torch
        z = zeta.detach().to(device=self.device, dtype=torch.float64).contiguous()
        if z.shape != (self.K,):
            raise ValueError(f"zeta must have shape ({self.K},)")
        self._z = z
        loss = torch.empty(self.nb, dtype=torch.float64, device=self.device)
        self._check(lib().ircur_unrolled_forward(self.h, ctypes.c_void_p(z.data_ptr()),
                                                 ctypes.c_void_p(loss.data_ptr())), "ircur_unrolled_forward")
        return loss

    def backward(self, dloss=None):
        """d(sum_b dloss_b loss_b)/d zeta (K,) float64 for the last forward."""
        import torch
        dz = torch.empty(self.K, dtype=torch.float64, device=self.device)
        w = None
        if dloss is not None:
            w = dloss.detach().to(device=self.device, dtype=torch.float64).contiguous()
            self._w = w
        self._check(lib().ircur_backward(self.h, None if w is None else ctypes.c_void_p(w.data_ptr()),
                                         ctypes.c_void_p(dz.data_ptr())), "ircur_backward")
        return dz

    def factors(self, b, k):
        import torch
        n1, n2, _, _ = self.shapes[b]
        At = torch.empty((self.r, n1), dtype=self.tdtype, device=self.device)
        B = torch.empty((self.r, n2), dtype=self.tdtype, device=self.device)
        self._check(lib().ircur_unrolled_get_factors(self.h, b, k, ctypes.c_void_p(At.data_ptr()),
                                                     ctypes.c_void_p(B.data_ptr())), "ircur_unrolled_get_factors")
        (torch.cuda.current_stream() if self.stream is None else self.stream).synchronize()
        return At, B

    def sets(self, b, k):
        _, _, sI, sJ = self.shapes[b]
        I = np.zeros(sI, np.int32)
        J = np.zeros(sJ, np.int32)
        self._check(lib().ircur_unrolled_get_sets(self.h, b, k, I.ctypes.data_as(_I32P), J.ctypes.data_as(_I32P)),
                    "ircur_unrolled_get_sets")
        return I, J

    def status(self):
        f = np.zeros(self.nb, np.int32)
        self._check(lib().ircur_unrolled_status(self.h, f.ctypes.data_as(_I32P)), "ircur_unrolled_status")
        return f

    def close(self):
        if getattr(self, "h", None):
            lib().ircur_unrolled_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_function():
    import torch

    class UnrolledLoss(torch.autograd.Function):
        """loss = sum_b loss_b(zeta) of an IRCURUnrolled batch; backward is the
        library's adjoint (ircur_backward)."""

        @staticmethod
        def forward(ctx, zeta, batch):
            losses = batch.forward(zeta)
            ctx.batch = batch
            ctx.zdtype = zeta.dtype
            ctx.zdev = zeta.device
            return losses.sum().to(device=zeta.device, dtype=zeta.dtype)

        @staticmethod
        def backward(ctx, g):
            dz = ctx.batch.backward(None).to(device=ctx.zdev)
            return (dz * g.to(torch.float64)).to(ctx.zdtype), None

    return UnrolledLoss


def unrolled_loss(zeta, batch):
    """Differentiable total loss of the batch as a function of zeta (K,)."""
    return _autograd_function().apply(zeta, batch)
