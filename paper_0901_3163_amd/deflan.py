"""Thin ctypes binding of libdeflan.so (include/deflan.h).

Every function here only marshals arguments: it converts numpy arrays (host
memory, ``DL_HOST``) or torch complex128 device tensors (``DL_DEVICE``) to
pointers, calls the C entry point of the same name and turns a negative status
into an exception.  All arithmetic runs in the library's HIP kernels; there is
no fallback path.  If the shared library is missing, importing this module
raises.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdeflan.so")

DL_OK, DL_NOT_CONVERGED = 0, 1
DL_E_INVALID, DL_E_HIP, DL_E_NOMEM, DL_E_BREAKDOWN, DL_E_NONFINITE, DL_E_MISMATCH = -1, -2, -3, -4, -5, -6
DL_MDAGM, DL_G5M = 0, 1
DL_EVEN_ODD = 16
DL_FP64, DL_FP32, DL_BF16 = 0, 1, 2
DL_HOST, DL_DEVICE = 0, 1
DL_METHOD_DEFAULT, DL_METHOD_CG = 0, 1
DL_APPLY_M, DL_APPLY_MDAG, DL_APPLY_G5M, DL_APPLY_MDAGM = 0, 1, 2, 3
DL_REORTH_FULL, DL_REORTH_KEPT = 0, 1
DL_TSK_DOTS64, DL_TSK_DOTS32, DL_TSK_DOTS16, DL_TSK_UPD64, DL_TSK_UPD32, DL_TSK_COMBINE = range(6)
STOP_RULES = {0: "linear", 1: "eigen", 2: "mvp_factor", 3: "max_mvp", 4: "breakdown", -1: "none"}


class DeflanError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"deflan error {code}: {msg}")
        self.code = code


class dl_first_opts(C.Structure):
    _fields_ = [("eig_tol", C.c_double), ("past_conv_factor", C.c_double), ("max_mvp", C.c_long),
                ("reorth", C.c_int), ("reorth_period", C.c_int)]


class dl_next_opts(C.Structure):
    _fields_ = [("storage", C.c_int), ("reliable_every", C.c_int), ("batched", C.c_int),
                ("x0_given", C.c_int), ("max_mvp", C.c_long), ("net", C.c_void_p), ("graph", C.c_int),
                ("inner_drop", C.c_double), ("eig_storage", C.c_int), ("net_prec", C.c_int), ("method", C.c_int),
                ("minres_window", C.c_int)]


class dl_batch_item(C.Structure):
    _fields_ = [("op", C.c_void_p), ("eig", C.c_void_p), ("nrhs", C.c_int), ("B", C.c_void_p), ("X", C.c_void_p),
                ("tol", C.c_double)]


class dl_stats(C.Structure):
    _fields_ = [("status", C.c_int), ("stop_rule", C.c_int), ("cycles", C.c_int), ("guess", C.c_int),
                ("mvp", C.c_long), ("mvp_lin", C.c_long), ("iters", C.c_long),
                ("relres", C.c_double), ("time_s", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int), ("history_len", C.c_int)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("history", "history_cap", "history_len")}
        d["stop_rule"] = STOP_RULES.get(self.stop_rule, str(self.stop_rule))
        return d


def _stats(n, history):
    """n dl_stats entries; history > 0: each gets a caller buffer of that many (mvp, relres) pairs."""
    st = (dl_stats * max(n, 1))()
    bufs = []
    if history:
        for i in range(n):
            b = np.zeros((int(history), 2))
            bufs.append(b)
            st[i].history = b.ctypes.data_as(C.POINTER(C.c_double))
            st[i].history_cap = int(history)
    return st, bufs


def _stats_dicts(st, bufs, n):
    out = []
    for i in range(n):
        d = st[i].as_dict()
        if bufs:
            d["history"] = bufs[i][: st[i].history_len].copy()
        out.append(d)
    return out


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_0901_3163_amd/build.py`")
    lib = C.CDLL(LIB_PATH)
    P, I, L, D = C.c_void_p, C.c_int, C.c_long, C.c_double
    sig = {
        "dl_last_error": (C.c_char_p, []),
        "dl_version": (I, []),
        "dl_ctx_create": (I, [I, P, C.POINTER(P)]),
        "dl_ctx_destroy": (None, [P]),
        "dl_ctx_sync": (I, [P]),
        "dl_timing": (I, [P, I]),
        "dl_kernel_time": (I, [P, C.c_char_p, C.POINTER(L), C.POINTER(D), C.POINTER(D)]),
        "dl_op_create": (I, [P, C.POINTER(I), P, I, D, I, C.POINTER(P)]),
        "dl_op_destroy": (None, [P]),
        "dl_op_size": (L, [P]),
        "dl_op_fingerprint": (I, [P, C.POINTER(C.c_ulonglong)]),
        "dl_eo_prepare": (I, [P, P, P, I]),
        "dl_eo_reconstruct": (I, [P, P, P, P, I]),
        "dl_eig_save": (I, [P, C.c_char_p]),
        "dl_eig_load": (I, [P, C.c_char_p, C.POINTER(P)]),
        "dl_apply": (I, [P, I, P, P, I]),
        "dl_solve_first": (I, [P, P, P, I, I, I, D, C.POINTER(dl_first_opts), C.POINTER(P), C.POINTER(dl_stats)]),
        "dl_solve_next": (I, [P, P, I, P, P, I, D, C.POINTER(dl_next_opts), C.POINTER(dl_stats)]),
        "dl_eig_create": (I, [P, I, P, I, C.POINTER(P)]),
        "dl_bench_wilson": (I, [P, I, I, I, I, C.POINTER(D), C.POINTER(D)]),
        "dl_bench_copy": (I, [P, L, I, C.POINTER(D)]),
        "dl_apply_batched": (I, [P, I, I, I, P, P, I]),
        "dl_solve_next_multi": (I, [P, I, C.POINTER(dl_batch_item), I, C.POINTER(dl_next_opts),
                                    C.POINTER(dl_stats)]),
        "dl_tune_wilson": (I, [P, I, I, I, C.POINTER(I), C.POINTER(I), C.POINTER(D)]),
        "dl_tune_tsk": (I, [P, I, L, I, I, I, C.POINTER(I), C.POINTER(I), C.POINTER(D)]),
        "dl_eig_info": (I, [P, C.POINTER(I), P, P]),
        "dl_eig_vectors": (I, [P, P, I]),
        "dl_eig_destroy": (None, [P]),
        "dl_tsk_project": (I, [P, L, I, P, P, P, I, I]),
        "dl_tsk_project_noalloc": (I, [P, L, I, P, P, P, I]),
        "dl_tsk_combine": (I, [P, L, I, P, P, I, P, I]),
        "dl_tsk_project_multi": (I, [P, L, I, P, I, P, P, P, I]),
        "dl_tsk_project_lowp": (I, [P, I, L, I, P, I, P, P, P, I]),
        "dl_eig_lower": (I, [P, P, I, C.POINTER(L)]),
        "dl_small_eigh": (I, [P, I, P, P, P]),
        "dl_net_num_weights": (I, []),
        "dl_net_create": (I, [P, P, C.POINTER(P)]),
        "dl_net_get_weights": (I, [P, P]),
        "dl_net_set_weights": (I, [P, P]),
        "dl_net_destroy": (None, [P]),
        "dl_net_apply": (I, [P, P, I, P, P, I]),
        "dl_net_apply_prec": (I, [P, P, I, I, P, P, I]),
        "dl_net_loss_grad": (I, [P, P, I, P, P, I, C.POINTER(D), P]),
        "dl_net_train": (I, [P, P, I, P, P, I, I, I, D, P]),
        "dl_net_set_projection": (I, [P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()
EXPORTED = ("dl_last_error", "dl_version", "dl_ctx_create", "dl_ctx_destroy", "dl_ctx_sync", "dl_timing",
            "dl_kernel_time", "dl_op_create", "dl_op_destroy", "dl_op_size", "dl_apply", "dl_solve_first",
            "dl_solve_next", "dl_eig_create", "dl_eig_info", "dl_eig_vectors", "dl_eig_destroy",
            "dl_tsk_project", "dl_tsk_combine", "dl_small_eigh", "dl_bench_wilson", "dl_tune_wilson", "dl_tune_tsk",
            "dl_net_num_weights", "dl_net_create", "dl_net_get_weights", "dl_net_set_weights", "dl_net_destroy",
            "dl_net_apply", "dl_net_loss_grad", "dl_net_train", "dl_apply_batched",
            "dl_solve_next_multi", "dl_tsk_project_multi", "dl_tsk_project_lowp", "dl_eig_lower",
            "dl_net_apply_prec", "dl_op_fingerprint", "dl_eig_save", "dl_eig_load", "dl_tsk_project_noalloc", "dl_net_set_projection", "dl_bench_copy", "dl_eo_prepare",
            "dl_eo_reconstruct")


def _check(rc):
    if rc < 0:
        raise DeflanError(rc, lib.dl_last_error().decode())
    return rc


def _ptr(a):
    """(pointer, mem) of a numpy array (host) or a torch tensor (device if on GPU)."""
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data_as(C.c_void_p), DL_HOST
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if a.is_cuda:
            # the library works on its own stream: torch's pending work on the tensor (a fill, a
            # copy) must be done before the library reads or writes it
            torch.cuda.current_stream(a.device).synchronize()
        return C.c_void_p(a.data_ptr()), (DL_DEVICE if a.is_cuda else DL_HOST)
    raise TypeError(f"unsupported array type {type(a)}")


def _c128(a):
    if isinstance(a, np.ndarray):
        return np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _empty_like(a, shape=None):
    shape = a.shape if shape is None else shape
    if isinstance(a, np.ndarray):
        return np.zeros(shape, dtype=np.complex128)
    import torch
    return torch.zeros(shape, dtype=torch.complex128, device=a.device)


# ---------------------------------------------------------------------------
class Context:
    """dl_ctx: one HIP device and stream (hip_stream: an int handle or None)."""

    def __init__(self, device: int = 0, hip_stream=None):
        h = C.c_void_p()
        _check(lib.dl_ctx_create(device, C.c_void_p(hip_stream) if hip_stream else None, C.byref(h)))
        self.h = h
        self._children = weakref.WeakSet()  # operators and handles that must be freed first

    def sync(self):
        _check(lib.dl_ctx_sync(self.h))

    def timing(self, enable: bool = True):
        _check(lib.dl_timing(self.h, 1 if enable else 0))

    def kernel_time(self, name: str):
        """(launches, total ms, algorithmic bytes) of a kernel family since timing was enabled."""
        n, ms, by = C.c_long(), C.c_double(), C.c_double()
        _check(lib.dl_kernel_time(self.h, name.encode(), C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def bench_copy(self, nbytes: int, reps: int = 20):
        """Milliseconds per launch of the library's copy kernel over nbytes (read once, written once)."""
        ms = C.c_double()
        _check(lib.dl_bench_copy(self.h, int(nbytes), int(reps), C.byref(ms)))
        return ms.value

    def tune_tsk(self, kind: int, n: int, nv: int, nw: int, reps: int = 5):
        """(grid, tile, microseconds) of the fastest launch shape of a contraction kind."""
        g, t, us = C.c_int(), C.c_int(), C.c_double()
        _check(lib.dl_tune_tsk(self.h, int(kind), int(n), int(nv), int(nw), int(reps), C.byref(g), C.byref(t),
                               C.byref(us)))
        return g.value, t.value, us.value

    def close(self):
        if getattr(self, "h", None):
            kids = list(self._children)
            for ch in kids:  # eigenvector handles and networks before operators
                if isinstance(ch, (Eig, Net)):
                    ch.close()
            for ch in kids:
                ch.close()
            lib.dl_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Eig:
    """dl_eig: eigenvectors kept from the first right-hand side."""

    def __init__(self, h, op):
        self.h = h
        self.op = op
        op.ctx._children.add(self)

    def info(self):
        k = C.c_int()
        _check(lib.dl_eig_info(self.h, C.byref(k), None, None))
        ev = np.zeros(k.value)
        rs = np.zeros(k.value)
        _check(lib.dl_eig_info(self.h, C.byref(k), ev.ctypes.data_as(C.c_void_p), rs.ctypes.data_as(C.c_void_p)))
        return ev, rs

    @property
    def k(self):
        k = C.c_int()
        _check(lib.dl_eig_info(self.h, C.byref(k), None, None))
        return k.value

    def lower(self, prec):
        """Lowered copies for the batched projection (DL_FP32 or DL_BF16; DL_FP64 drops them).
        Returns the MVPs used (k for the FP32 basis's Gram matrix, 0 if already built)."""
        used = C.c_long()
        _check(lib.dl_eig_lower(self.op.h, self.h, int(prec), C.byref(used)))
        return used.value

    def save(self, path):
        """Write the handle to a file (dl_eig_save)."""
        _check(lib.dl_eig_save(self.h, os.fspath(path).encode()))

    def vectors(self):
        V = np.zeros((self.k, self.op.V, 4, 3), dtype=np.complex128)
        if self.k:
            p, mem = _ptr(V)
            _check(lib.dl_eig_vectors(self.h, p, mem))
        return V

    def close(self):
        if getattr(self, "h", None):
            lib.dl_eig_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """dl_op: the Wilson matrix with links U, hopping parameter kappa, Hermitian form kind."""

    def __init__(self, ctx: Context, dims, links, kappa: float, kind: int):
        self.ctx = ctx
        self.dims = tuple(int(d) for d in dims)
        self.eo = bool(int(kind) & DL_EVEN_ODD)
        self.V_full = int(np.prod(self.dims))
        self.V = self.V_full // 2 if self.eo else self.V_full  # sites of the fields it acts on
        links = _c128(links)
        p, mem = _ptr(links)
        d = (C.c_int * 4)(*self.dims)
        h = C.c_void_p()
        _check(lib.dl_op_create(ctx.h, d, p, mem, float(kappa), int(kind), C.byref(h)))
        self.h = h
        ctx._children.add(self)
        self.kind = int(kind) & ~DL_EVEN_ODD
        self.kappa = kappa

    def apply(self, which: int, psi):
        psi = _c128(psi)
        out = _empty_like(psi)
        pi, mem = _ptr(psi)
        po, _ = _ptr(out)
        _check(lib.dl_apply(self.h, int(which), pi, po, mem))
        return out

    def apply_batched(self, which: int, prec: int, Psi):
        """op(psi_j) for each field of Psi ([n][V][4][3]) by the multi-rhs stencil (FP64 or FP32)."""
        Psi = _c128(Psi)
        out = _empty_like(Psi)
        pi, mem = _ptr(Psi)
        po, _ = _ptr(out)
        _check(lib.dl_apply_batched(self.h, int(which), int(prec), int(Psi.shape[0]), pi, po, mem))
        return out

    def eo_prepare(self, b):
        """bhat = b_e + kappa D_eo b_o (even half field) for a whole-lattice b (DL_EVEN_ODD operators)."""
        b = _c128(b)
        bh = _empty_like(b, (self.V,) + tuple(b.shape[1:]))
        pb, mem = _ptr(b)
        ph, _ = _ptr(bh)
        _check(lib.dl_eo_prepare(self.h, pb, ph, mem))
        return bh

    def eo_reconstruct(self, b, xe):
        """The whole-lattice solution from the even-site one (DL_EVEN_ODD operators)."""
        b, xe = _c128(b), _c128(xe)
        x = _empty_like(b)
        pb, mem = _ptr(b)
        pxe, _ = _ptr(xe)
        px, _ = _ptr(x)
        _check(lib.dl_eo_reconstruct(self.h, pb, pxe, px, mem))
        return x

    def fingerprint(self):
        f = C.c_ulonglong()
        _check(lib.dl_op_fingerprint(self.h, C.byref(f)))
        return f.value

    def eig_load(self, path):
        """An eigenvector handle read from a file written by Eig.save (dl_eig_load)."""
        h = C.c_void_p()
        _check(lib.dl_eig_load(self.h, os.fspath(path).encode(), C.byref(h)))
        return Eig(h, self)

    def solve_first(self, b, m: int, k: int, tol: float, eig_tol=None, past_conv_factor=None, max_mvp=None,
                    want_eig=True, reorth=DL_REORTH_FULL, reorth_period=0, history=0):
        """history > 0: the stats dict also holds 'history', an array of (mvp, relres) rows."""
        b = _c128(b)
        x = _empty_like(b)
        o = dl_first_opts(eig_tol or 0.0, past_conv_factor or 0.0, int(max_mvp or 0), int(reorth),
                          int(reorth_period))
        st, bufs = _stats(1, history)
        eh = C.c_void_p()
        pb, mem = _ptr(b)
        px, _ = _ptr(x)
        rc = _check(lib.dl_solve_first(self.h, pb, px, mem, int(m), int(k), float(tol), C.byref(o),
                                       C.byref(eh) if want_eig else None, st))
        eig = Eig(eh, self) if want_eig else None
        return x, eig, dict(_stats_dicts(st, bufs, 1)[0], rc=rc)

    def solve_next(self, B, eig, tol: float, storage=DL_FP64, batched=0, x0=None, max_mvp=None,
                   reliable_every=None, net=None, graph=False, inner_drop=None, eig_storage=DL_FP64,
                   net_prec=DL_FP32, method=0, minres_window=0, history=0):
        B = _c128(B)
        nrhs = B.shape[0]
        X = _empty_like(B) if x0 is None else _c128(x0).copy()
        o = dl_next_opts(int(storage), int(reliable_every or 0), int(batched), 1 if x0 is not None else 0,
                         int(max_mvp or 0), net.h if net is not None else None, 1 if graph else 0,
                         float(inner_drop or 0.0), int(eig_storage), int(net_prec), int(method),
                         int(minres_window))
        st, bufs = _stats(nrhs, history)
        pB, mem = _ptr(B)
        pX, _ = _ptr(X)
        rc = _check(lib.dl_solve_next(self.h, eig.h if eig is not None else None, nrhs, pB, pX, mem, float(tol),
                                      C.byref(o), st))
        return X, _stats_dicts(st, bufs, nrhs), rc

    def eig_create(self, Vecs):
        Vecs = _c128(Vecs)
        p, mem = _ptr(Vecs)
        h = C.c_void_p()
        _check(lib.dl_eig_create(self.h, int(Vecs.shape[0]), p, mem, C.byref(h)))
        return Eig(h, self)

    def bench_wilson(self, which: int, prec: int, nrhs: int = 1, reps: int = 20):
        """(ms per launch, algorithmic bytes per launch) of the Wilson stencil on device fields."""
        ms, by = C.c_double(), C.c_double()
        _check(lib.dl_bench_wilson(self.h, int(which), int(prec), int(nrhs), int(reps), C.byref(ms), C.byref(by)))
        return ms.value, by.value

    def tune_wilson(self, prec: int, nrhs: int = 1, reps: int = 10):
        """Run the stencil autotuner; returns (variant, order, best microseconds)."""
        v, o, us = C.c_int(), C.c_int(), C.c_double()
        _check(lib.dl_tune_wilson(self.h, int(prec), int(nrhs), int(reps), C.byref(v), C.byref(o), C.byref(us)))
        return v.value, o.value, us.value

    @property
    def n(self):
        return int(lib.dl_op_size(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib.dl_op_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """dl_net: the gauge-covariant network of the learned initial guess (weights complex128 [n])."""

    def __init__(self, ctx: Context, weights):
        self.ctx = ctx
        w = np.ascontiguousarray(weights, dtype=np.complex128)
        if w.shape != (num_weights(),):
            raise ValueError(f"expected {num_weights()} complex weights, got shape {w.shape}")
        h = C.c_void_p()
        _check(lib.dl_net_create(ctx.h, w.ctypes.data_as(C.c_void_p), C.byref(h)))
        self.h = h
        ctx._children.add(self)

    def weights(self):
        w = np.zeros(num_weights(), dtype=np.complex128)
        _check(lib.dl_net_get_weights(self.h, w.ctypes.data_as(C.c_void_p)))
        return w

    def set_weights(self, weights):
        w = np.ascontiguousarray(weights, dtype=np.complex128)
        if w.shape != (num_weights(),):
            raise ValueError(f"expected {num_weights()} complex weights, got shape {w.shape}")
        _check(lib.dl_net_set_weights(self.h, w.ctypes.data_as(C.c_void_p)))

    def apply(self, op: "Operator", B, prec=None):
        """net(b) for each field of B ([n][V][4][3]); prec DL_BF16: BF16 matrix-core inference."""
        B = _c128(B)
        Y = _empty_like(B)
        pB, mem = _ptr(B)
        pY, _ = _ptr(Y)
        if prec is None:
            _check(lib.dl_net_apply(self.h, op.h, int(B.shape[0]), pB, pY, mem))
        else:
            _check(lib.dl_net_apply_prec(self.h, op.h, int(prec), int(B.shape[0]), pB, pY, mem))
        return Y

    def loss_grad(self, op: "Operator", B, X, grad: bool = True):
        B, X = _c128(B), _c128(X)
        pB, mem = _ptr(B)
        pX, _ = _ptr(X)
        L = C.c_double()
        g = np.zeros(num_weights(), dtype=np.complex128) if grad else None
        _check(lib.dl_net_loss_grad(self.h, op.h, int(B.shape[0]), pB, pX, mem, C.byref(L),
                                    g.ctypes.data_as(C.c_void_p) if grad else None))
        return L.value, g

    def set_projection(self, eig):
        """Train on the error left after the Galerkin projection over eig (None: the raw error)."""
        _check(lib.dl_net_set_projection(self.h, eig.h if eig is not None else None))

    def train(self, op: "Operator", B, X, batch: int, steps: int, lr: float):
        """Adam steps on the pairs (B, X); returns the per-step minibatch losses."""
        B, X = _c128(B), _c128(X)
        pB, mem = _ptr(B)
        pX, _ = _ptr(X)
        losses = np.zeros(max(int(steps), 1))
        _check(lib.dl_net_train(self.h, op.h, int(B.shape[0]), pB, pX, mem, int(batch), int(steps), float(lr),
                                losses.ctypes.data_as(C.c_void_p)))
        return losses[:int(steps)]

    def close(self):
        if getattr(self, "h", None):
            lib.dl_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def num_weights() -> int:
    return int(lib.dl_net_num_weights())


def solve_next_multi(ctx: Context, items, reliable_every=None, max_mvp=None, x0s=None, graph=False,
                     storage=DL_FP32, inner_drop=None, eig_storage=DL_FP64, minres_window=0, history=0):
    """Later right-hand sides of several operators in one batched solve.

    items: sequence of (op, eig or None, B [nrhs][V][4][3], tol); all B numpy (host) or all
    torch device tensors.  Returns (list of X, list of per-rhs stats dicts per item, rc)."""
    its = (dl_batch_item * max(len(items), 1))()
    keep, Xs, mem = [], [], None
    for i, (op, eig, B, tol) in enumerate(items):
        B = _c128(B)
        X = _empty_like(B) if x0s is None else _c128(x0s[i]).copy()
        pB, m = _ptr(B)
        pX, _ = _ptr(X)
        if mem is None:
            mem = m
        elif m != mem:
            raise ValueError("all right-hand sides must live in the same memory (host or device)")
        its[i] = dl_batch_item(op.h, eig.h if eig is not None else None, int(B.shape[0]), pB, pX, float(tol))
        keep.append(B)
        Xs.append(X)
    o = dl_next_opts(int(storage), int(reliable_every or 0), 1, 1 if x0s is not None else 0, int(max_mvp or 0), None,
                     1 if graph else 0, float(inner_drop or 0.0), int(eig_storage), DL_FP32, 0,
                     int(minres_window))
    ntot = sum(int(B.shape[0]) for B in keep)
    st, bufs = _stats(ntot, history)
    rc = _check(lib.dl_solve_next_multi(ctx.h, len(items), its, mem if mem is not None else DL_HOST, C.byref(o), st))
    flat = _stats_dicts(st, bufs, ntot)
    out, r = [], 0
    for B in keep:
        out.append(flat[r:r + int(B.shape[0])])
        r += int(B.shape[0])
    return Xs, out, rc


# ---- kernel-level entry points ------------------------------------------------
def dl_tsk_project(ctx: Context, V, w, subtract: bool = False):
    """c = V^H w (and w <- w - V c if subtract); V: [nv][n] complex, w: [n]."""
    V = _c128(V)
    w = _c128(w).copy() if isinstance(w, np.ndarray) else w.clone()
    c = _empty_like(w, (V.shape[0],))
    pV, mem = _ptr(V)
    pw, _ = _ptr(w)
    pc, _ = _ptr(c)
    _check(lib.dl_tsk_project(ctx.h, int(V.shape[1]), int(V.shape[0]), pV, pw, pc, 1 if subtract else 0, mem))
    return c, w


def dl_tsk_project_noalloc(ctx: Context, V, w, c, subtract: bool = False):
    """dl_tsk_project with no device allocation: V [nv][n], w [n] and c [nv] are complex128
    device tensors owned by the caller; c receives V^H w and, if subtract, w <- w - V c in place."""
    ptrs = []
    for a in (V, w, c):
        p, mem = _ptr(a)
        if mem != DL_DEVICE:
            raise ValueError("dl_tsk_project_noalloc takes device tensors only")
        ptrs.append(p)
    if V.dim() != 2 or w.shape != (V.shape[1],) or c.shape != (V.shape[0],):
        raise ValueError("shapes must be V [nv][n], w [n], c [nv]")
    _check(lib.dl_tsk_project_noalloc(ctx.h, int(V.shape[1]), int(V.shape[0]), ptrs[0], ptrs[1], ptrs[2],
                                      1 if subtract else 0))
    return c, w


def dl_tsk_project_multi(ctx: Context, V, W, X=None):
    """C = V^H W per column ([nw][nv]) and, if X is given, X + V C^T per column."""
    V, W = _c128(V), _c128(W)
    C = _empty_like(W, (W.shape[0], V.shape[0]))
    Xo = None if X is None else (_c128(X).copy() if isinstance(X, np.ndarray) else X.clone())
    pV, mem = _ptr(V)
    pW, _ = _ptr(W)
    pC, _ = _ptr(C)
    pX = _ptr(Xo)[0] if Xo is not None else None
    _check(lib.dl_tsk_project_multi(ctx.h, int(V.shape[1]), int(V.shape[0]), pV, int(W.shape[0]), pW, pC, pX, mem))
    return C, Xo


def dl_tsk_project_lowp(ctx: Context, prec, V, W, X=None):
    """C = q(V)^H q(W) per column ([nw][nv]) on the matrix cores, q = rounding to prec (DL_FP32 or
    DL_BF16); if X is given, X + fp32(V) C^T per column in FP64."""
    V, W = _c128(V), _c128(W)
    C = _empty_like(W, (W.shape[0], V.shape[0]))
    Xo = None if X is None else (_c128(X).copy() if isinstance(X, np.ndarray) else X.clone())
    pV, mem = _ptr(V)
    pW, _ = _ptr(W)
    pC, _ = _ptr(C)
    pX = _ptr(Xo)[0] if Xo is not None else None
    _check(lib.dl_tsk_project_lowp(ctx.h, int(prec), int(V.shape[1]), int(V.shape[0]), pV, int(W.shape[0]), pW, pC,
                                   pX, mem))
    return C, Xo


def dl_tsk_combine(ctx: Context, V, G):
    """Y = V G for V [nv][n] complex and real G [nv][ny]; Y: [ny][n]."""
    V = _c128(V)
    if isinstance(G, np.ndarray):
        G = np.ascontiguousarray(G, dtype=np.float64)
    Y = _empty_like(V, (G.shape[1], V.shape[1]))
    pV, mem = _ptr(V)
    pG, _ = _ptr(G)
    pY, _ = _ptr(Y)
    _check(lib.dl_tsk_combine(ctx.h, int(V.shape[1]), int(V.shape[0]), pV, pG, int(G.shape[1]), pY, mem))
    return Y


def dl_small_eigh(ctx: Context, A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    ev = np.zeros(n)
    Z = np.zeros((n, n))
    _check(lib.dl_small_eigh(ctx.h, n, A.ctypes.data_as(C.c_void_p), ev.ctypes.data_as(C.c_void_p),
                             Z.ctypes.data_as(C.c_void_p)))
    return ev, Z
