"""ctypes binding of include/altgdmin.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

MASK_LINES, MASK_INDEX = 0, 1
FP32, MIXED = 0, 1
TIMED_KERNELS = {"fwd_transform": 1, "gram_rhs": 2, "solve": 3, "fold": 4, "adj_transform": 5,
                 "qr_gram": 6, "qr_small": 7, "apply_qr": 8}

_STATUS = {0: "ok", 1: "invalid argument", 2: "call out of order", 3: "HIP runtime error",
           4: "Gram matrix not positive definite", 5: "non-finite value", 6: "unsupported configuration",
           7: "problem too large for the built-in scratch"}


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nc", ctypes.c_int32),
                ("q", ctypes.c_int32), ("r", ctypes.c_int32), ("m_max", ctypes.c_int32),
                ("mask_kind", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("trunc_c", ctypes.c_double), ("eta_c", ctypes.c_double),
                ("eta_cap_c", ctypes.c_double), ("eps_exit", ctypes.c_double),
                ("t_max", ctypes.c_int32), ("exit_consec", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int32), ("exited", ctypes.c_int32), ("f", ctypes.c_double),
                ("sd", ctypes.c_double), ("grad_norm", ctypes.c_double), ("eta", ctypes.c_double),
                ("gamma", ctypes.c_double), ("n_trunc", ctypes.c_int32)]


class AltGDminError(RuntimeError):
    def __init__(self, status: int, where: str, frame: Optional[int] = None):
        self.status = status
        self.frame = frame
        msg = f"{where}: {_STATUS.get(status, 'unknown')} (status {status})"
        if frame is not None and frame >= 0:
            msg += f", frame {frame}"
        super().__init__(msg)


_LIB = None


def lib_path() -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "libaltgdmin.so")


def load_library():
    """Load libaltgdmin.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2212_09664_amd.build")
    L = ctypes.CDLL(path)
    vp, i32, pi32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_double
    sig = {
        "altgdmin_create": ([ctypes.POINTER(Params), ctypes.POINTER(vp)], i32),
        "altgdmin_workspace_bytes": ([vp, ctypes.POINTER(ctypes.c_size_t)], i32),
        "altgdmin_set_problem": ([vp, vp, vp, vp, vp, vp, vp], i32),
        "altgdmin_init": ([vp, vp], i32),
        "altgdmin_init_from": ([vp, vp, vp], i32),
        "altgdmin_iterate": ([vp, i32, vp, vp, vp, pi32], i32),
        "altgdmin_get_eta": ([vp, ctypes.POINTER(dbl)], i32),
        "altgdmin_set_eta": ([vp, dbl], i32),
        "altgdmin_cost": ([vp, vp, vp], i32),
        "altgdmin_gradient": ([vp, vp, vp, vp], i32),
        "altgdmin_apply_A": ([vp, vp, vp], i32),
        "altgdmin_apply_AH": ([vp, vp, vp], i32),
        "altgdmin_get_stats": ([vp, ctypes.POINTER(Stats)], i32),
        "altgdmin_last_error": ([vp, pi32], i32),
        "altgdmin_set_timing": ([vp, i32], i32),
        "altgdmin_kernel_time": ([vp, ctypes.POINTER(ctypes.c_char_p), pi32, ctypes.POINTER(dbl)], i32),
        "altgdmin_status_string": ([i32], ctypes.c_char_p),
        "altgdmin_destroy": ([vp], None),
        "altgdmin_cnn_input": ([vp, vp], i32),
        "altgdmin_aux_bytes": ([vp, ctypes.POINTER(ctypes.c_size_t)], i32),
        "altgdmin_mean": ([vp, dbl, i32, vp, vp, pi32], i32),
        "altgdmin_mean_noalloc": ([vp, dbl, i32, vp, pi32], i32),
        "altgdmin_residual": ([vp, vp, vp, vp, vp], i32),
        "altgdmin_mec_cgls": ([vp, vp, i32, dbl, vp, vp], i32),
        "altgdmin_mec_ista": ([vp, vp, i32, dbl, dbl, vp, vp, pi32], i32),
        "altgdmin_rank_energy": ([vp, i32, ctypes.POINTER(dbl), vp], i32),
        "altgdmin_expand": ([vp, vp, vp, vp, vp, vp], i32),
        "altgdmin_auto_rank": ([vp, dbl, pi32, pi32, vp], i32),
        "altgdmin_init_warm": ([vp, vp, vp, vp], i32),
        "altgdmin_init_warm_from": ([vp, vp, vp, vp, vp], i32),
        "wsinit_create": ([i32, i32, i32, i32, i32, i32, i32, vp, ctypes.POINTER(vp)], i32),
        "wsinit_param_count": ([vp, ctypes.POINTER(ctypes.c_int64)], i32),
        "wsinit_workspace_bytes": ([vp, ctypes.POINTER(ctypes.c_size_t)], i32),
        "wsinit_forward": ([vp, vp, vp, i32, vp, vp], i32),
        "wsinit_loss_backward": ([vp, vp, vp, vp, i32, vp, vp, vp], i32),
        "wsinit_adam_step": ([vp, vp, vp, vp, vp, ctypes.c_float, i32], i32),
        "wsinit_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = L
    return L


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class AltGDmin:
    """One reconstruction context (one problem shape, one bound problem)."""

    def __init__(self, nx, ny, nc, q, r, m_max, mask_kind=MASK_LINES, precision=FP32, trunc_c=36.0,
                 eta_c=0.14, eta_cap_c=0.0, eps_exit=0.0, t_max=70, exit_consec=1):
        self._L = load_library()
        self.p = Params(nx, ny, nc, q, r, m_max, mask_kind, precision, trunc_c, eta_c, eta_cap_c,
                        eps_exit, t_max, exit_consec)
        self.n = nx * ny
        h = ctypes.c_void_p()
        self._check(self._L.altgdmin_create(ctypes.byref(self.p), ctypes.byref(h)), "create")
        self._h = h
        nb = ctypes.c_size_t()
        self._check(self._L.altgdmin_workspace_bytes(self._h, ctypes.byref(nb)), "workspace_bytes")
        self.workspace_bytes = nb.value
        self._keep = []
        self.ws = None
        self.device = None

    def _check(self, st, where):
        if st != 0:
            frame = None
            if st == 4 and getattr(self, "_h", None):
                f = ctypes.c_int32(-1)
                self._L.altgdmin_last_error(self._h, ctypes.byref(f))
                frame = f.value
            raise AltGDminError(st, where, frame)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and self._L is not None:
            self._L.altgdmin_destroy(h)
            self._h = None

    # --- binding -------------------------------------------------------------
    def set_problem(self, coils, mask, m_k, y=None, workspace=None, stream=None):
        dev = coils.device
        if dev.type != "cuda":
            raise ValueError("inputs must be on the GPU")
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        base = workspace.data_ptr()
        off = (-base) % 256
        ws = workspace[off: off + self.workspace_bytes]
        coils = coils.contiguous()
        mask = mask.to(torch.int32).contiguous()
        m_k = m_k.to(torch.int32).contiguous()
        y = None if y is None else y.contiguous()
        self._keep = [coils, mask, m_k, y, workspace]
        self.ws = ws
        self.device = dev
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        self.stream = s
        self._check(self._L.altgdmin_set_problem(self._h, _ptr(coils), _ptr(mask), _ptr(m_k), _ptr(y),
                                                 ctypes.c_void_p(ws.data_ptr()),
                                                 ctypes.c_void_p(s.cuda_stream)), "set_problem")

    def _new(self, *shape, dtype=torch.complex64):
        return torch.empty(*shape, dtype=dtype, device=self.device)

    # --- algorithm -----------------------------------------------------------
    def init(self, U=None):
        U = self._new(self.p.r, self.n) if U is None else U
        self._check(self._L.altgdmin_init(self._h, _ptr(U)), "init")
        return U

    def init_from(self, U0, U=None):
        U = U0 if U is None else U
        self._check(self._L.altgdmin_init_from(self._h, _ptr(U0), _ptr(U)), "init_from")
        return U

    def cnn_input(self, out=None):
        """The learned initialiser's input: (2q, ny, nx) float32 planes."""
        out = torch.empty(2 * self.p.q, self.p.ny, self.p.nx, dtype=torch.float32, device=self.device) \
            if out is None else out
        self._check(self._L.altgdmin_cnn_input(self._h, _ptr(out)), "cnn_input")
        return out

    def init_warm(self, M, U=None, choice=None):
        """Spectral U_0 vs QR(M), the lower-cost one into U; choice (device
        int32, optional) receives 1 if M's basis was kept."""
        U = self._new(self.p.r, self.n) if U is None else U
        self._check(self._L.altgdmin_init_warm(self._h, _ptr(M), _ptr(U), _ptr(choice)), "init_warm")
        return U

    def init_warm_from(self, M, U_fb, U=None, choice=None):
        """init_warm with the fallback basis U_fb given (e.g. from init on this
        context) instead of computed; U may be U_fb."""
        U = self._new(self.p.r, self.n) if U is None else U
        self._check(self._L.altgdmin_init_warm_from(self._h, _ptr(M), _ptr(U_fb), _ptr(U), _ptr(choice)),
                    "init_warm_from")
        return U

    def iterate(self, n_iter, U, B=None, U_prev=None, sync=False):
        B = self._new(self.p.q, self.p.r) if B is None else B
        done = ctypes.c_int32(0)
        self._check(self._L.altgdmin_iterate(self._h, int(n_iter), _ptr(U), _ptr(B), _ptr(U_prev),
                                             ctypes.byref(done) if sync else None), "iterate")
        return (B, done.value) if sync else B

    def get_eta(self):
        v = ctypes.c_double()
        self._check(self._L.altgdmin_get_eta(self._h, ctypes.byref(v)), "get_eta")
        return v.value

    def set_eta(self, eta):
        self._check(self._L.altgdmin_set_eta(self._h, float(eta)), "set_eta")

    def cost(self, U):
        f = torch.zeros(1, dtype=torch.float64, device=self.device)
        self._check(self._L.altgdmin_cost(self._h, _ptr(U), _ptr(f)), "cost")
        return f

    def gradient(self, U):
        """(B, G) at U: B (q, r) the LS coefficients, G (r, n) the gradient."""
        B = self._new(self.p.q, self.p.r)
        G = self._new(self.p.r, self.n)
        self._check(self._L.altgdmin_gradient(self._h, _ptr(U), _ptr(B), _ptr(G)), "gradient")
        return B, G

    def ls(self, U, B=None):
        """B (q, r): the LS coefficients b_k = (A_k U)^dagger y_k at U."""
        B = self._new(self.p.q, self.p.r) if B is None else B
        self._check(self._L.altgdmin_gradient(self._h, _ptr(U), _ptr(B), None), "ls")
        return B

    # --- the steps around the loop (altGDmin-MRI) ----------------------------
    def aux(self):
        """The auxiliary workspace of the steps around the loop (allocated
        once per context, 256-byte aligned)."""
        if getattr(self, "_aux", None) is None:
            nb = ctypes.c_size_t()
            self._check(self._L.altgdmin_aux_bytes(self._h, ctypes.byref(nb)), "aux_bytes")
            buf = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
            off = (-buf.data_ptr()) % 256
            self._aux = (buf, buf[off: off + nb.value])
        return self._aux[1]

    def mean(self, tol=1e-3, maxit=10, zbar=None, sync=False):
        """The mean image zbar (n,) by CG on the normal equations."""
        zbar = self._new(self.n) if zbar is None else zbar
        it = ctypes.c_int32(-1)
        self._check(self._L.altgdmin_mean(self._h, float(tol), int(maxit), _ptr(zbar), _ptr(self.aux()),
                                          ctypes.byref(it) if sync else None), "mean")
        return (zbar, it.value) if sync else zbar

    def mean_noalloc(self, zbar, tol=1e-3, maxit=10, sync=False):
        """The mean image into the caller's zbar (n,), with the library's
        built-in scratch instead of an auxiliary workspace (allocates nothing)."""
        it = ctypes.c_int32(-1)
        self._check(self._L.altgdmin_mean_noalloc(self._h, float(tol), int(maxit), _ptr(zbar),
                                                  ctypes.byref(it) if sync else None), "mean_noalloc")
        return it.value if sync else None

    def residual(self, zbar=None, X=None, out=None):
        """y - A(zbar 1^T + X) in the padded layout (q, nc, m_max); X is (q, n)."""
        out = self._new(self.p.q, self.p.nc, self.p.m_max) if out is None else out
        self._check(self._L.altgdmin_residual(self._h, _ptr(zbar), _ptr(X), _ptr(out), _ptr(self.aux())),
                    "residual")
        return out

    def mec_cgls(self, yres, iters=3, tol=1e-36, E=None):
        """MEC model 1: E (q, n), per-frame CGLS from zero."""
        E = self._new(self.p.q, self.n) if E is None else E
        self._check(self._L.altgdmin_mec_cgls(self._h, _ptr(yres), int(iters), float(tol), _ptr(E),
                                              _ptr(self.aux())), "mec_cgls")
        return E

    def mec_ista(self, yres, max_iter=10, omega_frac=1e-3, tol=0.0025, E=None, sync=False):
        """MEC model 2: E (q, n) by ISTA on the temporal DFT."""
        E = self._new(self.p.q, self.n) if E is None else E
        it = ctypes.c_int32(-1)
        self._check(self._L.altgdmin_mec_ista(self._h, _ptr(yres), int(max_iter), float(omega_frac), float(tol),
                                              _ptr(E), _ptr(self.aux()), ctypes.byref(it) if sync else None),
                    "mec_ista")
        return (E, it.value) if sync else E

    def expand(self, U=None, B=None, zbar=None, E=None, Z=None):
        """Z (q, n): zbar + U b_k + e_k per frame (U (r, n), B (q, r), E (q, n))."""
        Z = self._new(self.p.q, self.n) if Z is None else Z
        self._check(self._L.altgdmin_expand(self._h, _ptr(U), _ptr(B), _ptr(zbar), _ptr(E), _ptr(Z)), "expand")
        return Z

    def rank_energy(self, r_cap):
        out = (ctypes.c_double * int(r_cap))()
        self._check(self._L.altgdmin_rank_energy(self._h, int(r_cap), out, _ptr(self.aux())), "rank_energy")
        return list(out)

    def auto_rank(self, b_percent=85.0):
        """(r_hat, r_cap) by Algorithm 2's energy rule."""
        r, cap = ctypes.c_int32(), ctypes.c_int32()
        self._check(self._L.altgdmin_auto_rank(self._h, float(b_percent), ctypes.byref(r), ctypes.byref(cap),
                                               _ptr(self.aux())), "auto_rank")
        return r.value, cap.value

    def apply_A(self, X, Y=None):
        Y = self._new(self.p.q, self.p.nc, self.p.m_max) if Y is None else Y
        self._check(self._L.altgdmin_apply_A(self._h, _ptr(X.contiguous()), _ptr(Y)), "apply_A")
        return Y

    def apply_AH(self, Y, X=None):
        X = self._new(self.p.q, self.n) if X is None else X
        self._check(self._L.altgdmin_apply_AH(self._h, _ptr(Y.contiguous()), _ptr(X)), "apply_AH")
        return X

    def stats(self) -> dict:
        s = Stats()
        self._check(self._L.altgdmin_get_stats(self._h, ctypes.byref(s)), "get_stats")
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def last_error(self):
        f = ctypes.c_int32(-1)
        st = self._L.altgdmin_last_error(self._h, ctypes.byref(f))
        return st, f.value

    def set_timing(self, kernel: str):
        self._check(self._L.altgdmin_set_timing(self._h, TIMED_KERNELS.get(kernel, 0)), "set_timing")

    def kernel_time(self):
        name = ctypes.c_char_p()
        cnt = ctypes.c_int32()
        ms = ctypes.c_double()
        self._check(self._L.altgdmin_kernel_time(self._h, ctypes.byref(name), ctypes.byref(cnt),
                                                 ctypes.byref(ms)), "kernel_time")
        return name.value.decode(), cnt.value, ms.value


class WsInit:
    """The warm-start CNN (include/wsinit.h): forward, loss + backward, Adam.
    Parameters, gradients and moments are flat float32 tensors."""

    def __init__(self, nx, ny, q, r, width=32, layers=4, batch=16, stream=None):
        self._L = load_library()
        self.nx, self.ny, self.q, self.r, self.width, self.batch = nx, ny, q, r, width, batch
        self.n = nx * ny
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        st = self._L.wsinit_create(nx, ny, q, r, width, layers, batch, ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h))
        if st != 0:
            raise AltGDminError(st, "wsinit_create", None)
        self._h = h
        c = ctypes.c_int64()
        self._L.wsinit_param_count(self._h, ctypes.byref(c))
        self.param_count = c.value
        nb = ctypes.c_size_t()
        self._L.wsinit_workspace_bytes(self._h, ctypes.byref(nb))
        self.workspace_bytes = nb.value
        buf = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        off = (-buf.data_ptr()) % 256
        self._buf = buf
        self.ws = buf[off: off + nb.value]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.wsinit_destroy(h)
            self._h = None

    def _check(self, st, where):
        if st != 0:
            raise AltGDminError(st, where, None)

    def forward(self, params, x, M=None):
        """x (B, 2q, ny, nx) -> M (B, r, n) complex64."""
        b = x.shape[0]
        M = torch.empty(b, self.r, self.n, dtype=torch.complex64, device=x.device) if M is None else M
        self._check(self._L.wsinit_forward(self._h, _ptr(params), _ptr(x), b, _ptr(M),
                                           ctypes.c_void_p(self.ws.data_ptr())), "wsinit_forward")
        return M

    def loss_backward(self, params, x, Ut, grads=None, loss=None):
        """Mean loss (device float64 scalar) and mean gradient over the batch."""
        b = x.shape[0]
        grads = torch.empty_like(params) if grads is None else grads
        loss = torch.empty(1, dtype=torch.float64, device=x.device) if loss is None else loss
        self._check(self._L.wsinit_loss_backward(self._h, _ptr(params), _ptr(x), _ptr(Ut), b, _ptr(grads),
                                                 _ptr(loss), ctypes.c_void_p(self.ws.data_ptr())),
                    "wsinit_loss_backward")
        return loss, grads

    def adam_step(self, params, grads, m, v, lr, step):
        self._check(self._L.wsinit_adam_step(self._h, _ptr(params), _ptr(grads), _ptr(m), _ptr(v),
                                             ctypes.c_float(lr), int(step)), "wsinit_adam_step")
