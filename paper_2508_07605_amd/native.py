"""Thin Python binding of libopen (include/open.h).

Argument marshalling only: torch tensors supply device memory and the stream, every step
of the computation runs in the library's HIP kernels.  The functions carry the C names.
There is no fallback: if the library is missing or fails to load, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load torch's HIP runtime before the library binds to it)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libopen.so")

OPEN_OK, OPEN_E_INVALID, OPEN_E_NOMEM, OPEN_E_DEVICE, OPEN_E_UNSUPPORTED = 0, -1, -2, -3, -4
ROW_OK, ROW_EMPTY, ROW_NONPOS_PIVOT, ROW_NONFINITE, ROW_NONPOS_BASE, ROW_BADINDEX = 0, 1, 2, 3, 4, 5

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_F32 = ctypes.c_float
_F64 = ctypes.c_double

# name -> (restype, argtypes); mirrors include/open.h
SIGNATURES = {
    "open_create": (_I32, [ctypes.POINTER(_P), _I32, _P]),
    "open_destroy": (_I32, [_P]),
    "open_set_stream": (_I32, [_P, _P]),
    "open_last_error": (ctypes.c_char_p, [_P]),
    "open_sync": (_I32, [_P]),
    "open_profile": (_I32, [_P, _I32]),
    "open_profile_read": (_I32, [_P, _P, _P, _P, _I32, _I32]),
    "open_foldin": (_I32, [_P, _P, _I32, _I32, _I64, _P, _P, _P, _F32, _I32, _P, _P]),
    "open_foldin_graph": (_I32, [_P, _P, _I32, _I32, _I64, _P, _P, _P, _F32, _I32, _P, _P]),
    "open_foldin_noalloc": (_I32, [_P, _P, _I32, _I32, _I64, _P, _P, _P, _F32, _I32, _P, _P]),
    "open_foldin_noalloc_max_rows": (_I64, []),
    "open_phase_detect": (_I32, [_P, _P, _I64, _I64, _I64, _F32, _I32, _P]),
    "open_perf_predict": (_I32, [_P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "open_ncf_foldin": (_I32, [_P, _P, _I32, _I32, _P, _P, _P, _P, _P, _P, _I64, _P, _P, _P, _I32, _F32, _F32, _P,
                               _P, _P]),
    "open_ncf_num_params": (_I64, [_I64, _I32]),
    "open_ncf_train": (_I32, [_P, _I64, _I32, _I32, _P, _P, _I32, _F32, _I32, ctypes.c_uint64, _P]),
    "open_ncf_loss_grad": (_I32, [_P, _I64, _I32, _I32, _P, _P, _P, _I32, _P, _P]),
    "open_refit": (_I32, [_P, _I64, _I64, _I32, _I32, _P, _P, _P, _F32, _I32, _I32, _P, _P, _P]),
    "open_tune_info": (_I32, [_I32, _P, _P, _I32]),
    "open_tune_get": (_I32, [_P, _I32, _P, _I32]),
    "open_tune_set": (_I32, [_P, _I32, _P, _I32]),
    "open_autotune": (_I32, [_P, _P, _I32, _I32, _I64, _P, _P, _P, _F32, _I32, _P, _P, _I32, _P]),
    "open_csr_to_csc": (_I32, [_P, _I64, _I32, _P, _P, _P, _P, _P, _P]),
    "open_fit": (_I32, [_P, _I64, _I32, _I32, _P, _P, _P, _F32, _I32, _I32, _P, _P, _P]),
    "open_objective": (_I32, [_P, _I64, _I32, _I32, _P, _P, _P, _P, _P, _F32, _I32, _P]),
    "open_residual": (_I32, [_P, _I64, _I32, _I32, _P, _P, _P, _P, _P, _P]),
    "open_predict": (_I32, [_P, _P, _I64, _P, _I32, _I32, _P, _P, _P, _I32, _F32, _P, _P, _P]),
    "open_mlp_create": (_I32, [_P, ctypes.POINTER(_P), _I32, _I32, _I32, _P, ctypes.c_uint64]),
    "open_mlp_destroy": (_I32, [_P]),
    "open_mlp_num_params": (_I64, [_I32, _I32, _I32]),
    "open_mlp_get_weights": (_I32, [_P, _P]),
    "open_mlp_set_weights": (_I32, [_P, _P]),
    "open_mlp_forward": (_I32, [_P, _I64, _P, _P, _P, _P]),
    "open_mlp_loss_grad": (_I32, [_P, _I64, _P, _P, _P, _P, _P, _P]),
    "open_mlp_train_step": (_I32, [_P, _I64, _P, _P, _P, _P, _P, _I32, _F32, _P]),
    "open_mlp_train": (_I32, [_P, _I64, _P, _P, _P, _P, _I32, _F32, _I32, ctypes.c_uint64, _P]),
    "open_mlp_foldin": (_I32, [_P, _P, _I64, _P, _P, _P, _F32, _F32, _I32, _P, _P, _P, _P]),
}

_lib = None


class OpenError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libopen status %d: %s" % (status, msg))
        self.status = status


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OpenError(OPEN_E_DEVICE, "libopen.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, name, numel=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), numel))
    return _ptr(t)


class Context:
    """open_ctx bound to a device and to torch's current stream on it."""

    def __init__(self, device: int = 0, stream=None):
        L = lib()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = ctypes.c_void_p()
        st = L.open_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != OPEN_OK:
            raise OpenError(st, "open_create failed")
        self.handle = h

    def check(self, st):
        if st != OPEN_OK:
            raise OpenError(st, lib().open_last_error(self.handle).decode())

    def set_stream(self, stream):
        self._stream = stream
        self.check(lib().open_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)))

    def sync(self):
        self.check(lib().open_sync(self.handle))

    def profile(self, enable=True):
        self.check(lib().open_profile(self.handle, int(bool(enable))))

    def profile_read(self, reset=True):
        """{kernel name: (total ms, launches)} since the last reset."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        tot = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int64 * cap)()
        n = lib().open_profile_read(self.handle, names, tot, cnt, cap, int(bool(reset)))
        if n < 0:
            raise OpenError(OPEN_E_DEVICE, "open_profile_read failed")
        return {names[i].decode(): (tot[i], cnt[i]) for i in range(min(n, cap))}

    def tune_get(self, k):
        """Chosen kernel variant per class group of rank k."""
        ng = len(open_tune_info(k))
        buf = (ctypes.c_int8 * ng)()
        self.check(lib().open_tune_get(self.handle, k, buf, ng))
        return list(buf)

    def tune_set(self, k, choice):
        buf = (ctypes.c_int8 * len(choice))(*choice)
        self.check(lib().open_tune_set(self.handle, k, buf, len(choice)))

    def close(self):
        if getattr(self, "handle", None):
            lib().open_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def open_foldin(ctx, F, row_ptr, col, val, lam, weighted=True, U_out=None, row_status=None):
    n, k = F.shape
    m = row_ptr.numel() - 1
    if U_out is None:
        U_out = torch.empty((m, k), dtype=torch.float32, device=F.device)
    ctx.check(lib().open_foldin(ctx.handle, _dev(F, torch.float32, "F"), n, k, m,
                                _dev(row_ptr, torch.int64, "row_ptr", m + 1), _dev(col, torch.int32, "col"),
                                _dev(val, torch.float32, "val"), float(lam), int(bool(weighted)),
                                _dev(U_out, torch.float32, "U_out", m * k),
                                _dev(row_status, torch.int32, "row_status", m)))
    return U_out


def open_foldin_graph(ctx, F, row_ptr, col, val, lam, weighted=True, U_out=None, row_status=None):
    """open_foldin recorded once into a HIP graph and replayed while the arguments repeat."""
    n, k = F.shape
    m = row_ptr.numel() - 1
    if U_out is None:
        U_out = torch.empty((m, k), dtype=torch.float32, device=F.device)
    ctx.check(lib().open_foldin_graph(ctx.handle, _dev(F, torch.float32, "F"), n, k, m,
                                      _dev(row_ptr, torch.int64, "row_ptr", m + 1), _dev(col, torch.int32, "col"),
                                      _dev(val, torch.float32, "val"), float(lam), int(bool(weighted)),
                                      _dev(U_out, torch.float32, "U_out", m * k),
                                      _dev(row_status, torch.int32, "row_status", m)))
    return U_out


def open_foldin_noalloc(ctx, F, row_ptr, col, val, lam, weighted, U_out, row_status=None):
    """open_foldin with the library's static scratch array instead of context workspaces (the
    caller provides the output; nothing is allocated)."""
    n, k = F.shape
    m = row_ptr.numel() - 1
    ctx.check(lib().open_foldin_noalloc(ctx.handle, _dev(F, torch.float32, "F"), n, k, m,
                                        _dev(row_ptr, torch.int64, "row_ptr", m + 1), _dev(col, torch.int32, "col"),
                                        _dev(val, torch.float32, "val"), float(lam), int(bool(weighted)),
                                        _dev(U_out, torch.float32, "U_out", m * k),
                                        _dev(row_status, torch.int32, "row_status", m)))
    return U_out


def open_phase_detect(ctx, power, threshold=60.0, n_window=25, first_index=None):
    """Algorithm 1 over the rows of a 2-D device tensor of power readings."""
    T, L = power.shape
    if first_index is None:
        first_index = torch.empty(T, dtype=torch.int64, device=power.device)
    ctx.check(lib().open_phase_detect(ctx.handle, _dev(power, torch.float32, "power", T * L), T, L,
                                      power.stride(0) if T > 0 else L, float(threshold), int(n_window),
                                      _dev(first_index, torch.int64, "first_index", T)))
    return first_index


def open_perf_predict(ctx, X, params, y=None):
    """Offline predictor over the rows of X (device float32 [runs, 7]); params holds device
    float32 tensors mu[7], rs[7], W1[64, 7], b1[64], W2[64, 64], b2[64], w3[64], b3[1]."""
    n = X.shape[0]
    if X.dim() != 2 or X.shape[1] != 7:
        raise ValueError("X must be [runs, 7]")
    if y is None:
        y = torch.empty(n, dtype=torch.float32, device=X.device)
    sizes = {"mu": 7, "rs": 7, "W1": 448, "b1": 64, "W2": 4096, "b2": 64, "w3": 64, "b3": 1}
    ptrs = [_dev(params[name], torch.float32, name, cnt) for name, cnt in sizes.items()]
    ctx.check(lib().open_perf_predict(ctx.handle, _dev(X, torch.float32, "X", n * 7), n, *ptrs,
                                      _dev(y, torch.float32, "y", n)))
    return y


def open_ncf_foldin(ctx, S, params, row_ptr, col, val, steps, eta, mu, E_out=None, loss_out=None,
                    row_status=None):
    """NCF fold-in of the CSR rows against setting embeddings S (device float32 [n, 32]);
    params holds device float32 W1[64, 64], b1[64], W2[64, 64], b2[64], w3[64], b3[1]."""
    n, d = S.shape
    m = row_ptr.numel() - 1
    if E_out is None:
        E_out = torch.empty((m, d), dtype=torch.float32, device=S.device)
    sizes = {"W1": 64 * 2 * d, "b1": 64, "W2": 4096, "b2": 64, "w3": 64, "b3": 1}
    ptrs = [_dev(params[name], torch.float32, name, cnt) for name, cnt in sizes.items()]
    ctx.check(lib().open_ncf_foldin(ctx.handle, _dev(S, torch.float32, "S", n * d), n, d, *ptrs, m,
                                    _dev(row_ptr, torch.int64, "row_ptr", m + 1), _dev(col, torch.int32, "col"),
                                    _dev(val, torch.float32, "val"), int(steps), float(eta), float(mu),
                                    _dev(E_out, torch.float32, "E_out", m * d),
                                    _dev(loss_out, torch.float32, "loss_out", m),
                                    _dev(row_status, torch.int32, "row_status", m)))
    return E_out


def open_tune_info(k):
    """[(group kernel name, variants compiled)] of rank k."""
    cap = 32
    names = (ctypes.c_char_p * cap)()
    nvar = (ctypes.c_int32 * cap)()
    n = lib().open_tune_info(k, names, nvar, cap)
    if n < 0:
        raise OpenError(OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64")
    return [(names[i].decode(), nvar[i]) for i in range(min(n, cap))]


def open_autotune(ctx, F, row_ptr, col, val, lam, weighted=True, reps=5, U_out=None, row_status=None):
    """Time every kernel variant on this batch, keep the fastest per class group in ctx.
    Returns (U_out, {group name: [ms per launch of each variant, None if untimed]})."""
    n, k = F.shape
    m = row_ptr.numel() - 1
    groups = open_tune_info(k)
    if U_out is None:
        U_out = torch.empty((m, k), dtype=torch.float32, device=F.device)
    ms = (ctypes.c_double * (4 * len(groups)))()
    ctx.check(lib().open_autotune(ctx.handle, _dev(F, torch.float32, "F"), n, k, m,
                                  _dev(row_ptr, torch.int64, "row_ptr", m + 1), _dev(col, torch.int32, "col"),
                                  _dev(val, torch.float32, "val"), float(lam), int(bool(weighted)),
                                  _dev(U_out, torch.float32, "U_out", m * k),
                                  _dev(row_status, torch.int32, "row_status", m), int(reps), ms))
    table = {}
    for g, (name, nv) in enumerate(groups):
        table[name] = [ms[4 * g + v] if ms[4 * g + v] >= 0 else None for v in range(nv)]
    return U_out, table


def open_csr_to_csc(ctx, row_ptr, col, val, n):
    m = row_ptr.numel() - 1
    nnz = col.numel()
    dev = row_ptr.device
    col_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    row_idx = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    cval = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)
    ctx.check(lib().open_csr_to_csc(ctx.handle, m, n, _dev(row_ptr, torch.int64, "row_ptr", m + 1),
                                    _dev(col, torch.int32, "col"), _dev(val, torch.float32, "val"),
                                    _ptr(col_ptr), _ptr(row_idx), _ptr(cval)))
    return col_ptr, row_idx[:nnz], cval[:nnz]


def open_fit(ctx, row_ptr, col, val, U, V, lam, sweeps, weighted=True, want_obj=False):
    import numpy as np
    m, k = U.shape
    n = V.shape[0]
    obj = np.zeros(2 * sweeps) if want_obj else None
    ctx.check(lib().open_fit(ctx.handle, m, n, k, _dev(row_ptr, torch.int64, "row_ptr", m + 1),
                             _dev(col, torch.int32, "col"), _dev(val, torch.float32, "val"), float(lam),
                             int(bool(weighted)), int(sweeps), _dev(U, torch.float32, "U", m * k),
                             _dev(V, torch.float32, "V", n * k),
                             obj.ctypes.data_as(ctypes.c_void_p) if obj is not None else None))
    return obj


def open_refit(ctx, m_old, row_ptr, col, val, U, V, lam, sweeps, weighted=True, want_obj=False):
    """Fold the rows after the first m_old into U against V, then `sweeps` ALS sweeps on all."""
    import numpy as np
    m, k = U.shape
    n = V.shape[0]
    obj = np.zeros(2 * max(sweeps, 0)) if want_obj else None
    ctx.check(lib().open_refit(ctx.handle, int(m_old), m - int(m_old), n, k,
                               _dev(row_ptr, torch.int64, "row_ptr", m + 1), _dev(col, torch.int32, "col"),
                               _dev(val, torch.float32, "val"), float(lam), int(bool(weighted)), int(sweeps),
                               _dev(U, torch.float32, "U", m * k), _dev(V, torch.float32, "V", n * k),
                               obj.ctypes.data_as(ctypes.c_void_p) if obj is not None else None))
    return obj


def open_objective(ctx, row_ptr, col, val, U, V, lam, weighted=True):
    m, k = U.shape
    n = V.shape[0]
    out = ctypes.c_double()
    ctx.check(lib().open_objective(ctx.handle, m, n, k, _dev(row_ptr, torch.int64, "row_ptr", m + 1),
                                   _dev(col, torch.int32, "col"), _dev(val, torch.float32, "val"),
                                   _dev(U, torch.float32, "U", m * k), _dev(V, torch.float32, "V", n * k),
                                   float(lam), int(bool(weighted)), ctypes.byref(out)))
    return out.value


def open_residual(ctx, row_ptr, col, val, U, V, rho=None):
    m, k = U.shape
    n = V.shape[0]
    if rho is None:
        rho = torch.empty(m, dtype=torch.float32, device=U.device)
    ctx.check(lib().open_residual(ctx.handle, m, n, k, _dev(row_ptr, torch.int64, "row_ptr", m + 1),
                                  _dev(col, torch.int32, "col"), _dev(val, torch.float32, "val"),
                                  _dev(U, torch.float32, "U", m * k), _dev(V, torch.float32, "V", n * k),
                                  _dev(rho, torch.float32, "rho", m)))
    return rho


def open_predict(ctx, U, V, cap_cpu, cap_gpu, base, gamma, P=None, best_idx=None, best_saving=None,
                 row_status=None):
    m, k = U.shape
    n = V.shape[0]
    dev = U.device
    if best_idx is None:
        best_idx = torch.empty(m, dtype=torch.int32, device=dev)
    if best_saving is None:
        best_saving = torch.empty(m, dtype=torch.float32, device=dev)
    ctx.check(lib().open_predict(ctx.handle, _dev(U, torch.float32, "U", m * k), m, _dev(V, torch.float32, "V", n * k),
                                 n, k, _dev(P, torch.float32, "P", m * n), _dev(cap_cpu, torch.float32, "cap_cpu", n),
                                 _dev(cap_gpu, torch.float32, "cap_gpu", n), int(base), float(gamma),
                                 _dev(best_idx, torch.int32, "best_idx", m),
                                 _dev(best_saving, torch.float32, "best_saving", m),
                                 _dev(row_status, torch.int32, "row_status", m)))
    return best_idx, best_saving


def open_mlp_num_params(n, k, hidden=256):
    return int(lib().open_mlp_num_params(n, k, hidden))


class Surrogate:
    """open_mlp handle: the fold-in surrogate network."""

    def __init__(self, ctx, n, k, hidden=256, init=None, seed=0):
        import numpy as np
        self.ctx, self.n, self.k, self.hidden = ctx, n, k, hidden
        self.num_params = open_mlp_num_params(n, k, hidden)
        buf = None
        if init is not None:
            buf = np.ascontiguousarray(init, dtype=np.float32)
            if buf.size != self.num_params:
                raise ValueError("init holds %d values, needs %d" % (buf.size, self.num_params))
        h = ctypes.c_void_p()
        ctx.check(lib().open_mlp_create(ctx.handle, ctypes.byref(h), n, k, hidden,
                                        buf.ctypes.data_as(ctypes.c_void_p) if buf is not None else None,
                                        int(seed)))
        self.handle = h

    def get_weights(self):
        import numpy as np
        out = np.empty(self.num_params, dtype=np.float32)
        self.ctx.check(lib().open_mlp_get_weights(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_weights(self, w):
        import numpy as np
        buf = np.ascontiguousarray(w, dtype=np.float32)
        if buf.size != self.num_params:
            raise ValueError("weights hold %d values, needs %d" % (buf.size, self.num_params))
        self.ctx.check(lib().open_mlp_set_weights(self.handle, buf.ctypes.data_as(ctypes.c_void_p)))

    def forward(self, row_ptr, col, val, out=None):
        m = row_ptr.numel() - 1
        if out is None:
            out = torch.empty((m, self.k), dtype=torch.float32, device=row_ptr.device)
        self.ctx.check(lib().open_mlp_forward(self.handle, m, _dev(row_ptr, torch.int64, "row_ptr", m + 1),
                                              _dev(col, torch.int32, "col"), _dev(val, torch.float32, "val"),
                                              _dev(out, torch.float32, "out", m * self.k)))
        return out

    def loss_grad(self, row_ptr, col, val, target):
        import numpy as np
        m = row_ptr.numel() - 1
        grads = np.empty(self.num_params, dtype=np.float32)
        loss = ctypes.c_double()
        self.ctx.check(lib().open_mlp_loss_grad(self.handle, m, _dev(row_ptr, torch.int64, "row_ptr", m + 1),
                                                _dev(col, torch.int32, "col"), _dev(val, torch.float32, "val"),
                                                _dev(target, torch.float32, "target", m * self.k),
                                                ctypes.byref(loss), grads.ctypes.data_as(ctypes.c_void_p)))
        return loss.value, grads

    def train_step(self, row_ptr, col, val, target, rows, lr, loss_out=None):
        m = row_ptr.numel() - 1
        batch = rows.numel() if rows is not None else m
        self.ctx.check(lib().open_mlp_train_step(self.handle, m, _dev(row_ptr, torch.int64, "row_ptr", m + 1),
                                                 _dev(col, torch.int32, "col"), _dev(val, torch.float32, "val"),
                                                 _dev(target, torch.float32, "target", m * self.k),
                                                 _dev(rows, torch.int64, "rows"), int(batch), float(lr),
                                                 _dev(loss_out, torch.float32, "loss_out", 1)))

    def train(self, row_ptr, col, val, target, batch, lr, epochs, seed=0):
        """open_mlp_train: epochs of seeded on-device shuffles, one Adam step per full batch;
        returns the mean batch loss of each epoch (numpy float32)."""
        import numpy as np
        m = row_ptr.numel() - 1
        hist = np.zeros(max(int(epochs), 1), dtype=np.float32)
        self.ctx.check(lib().open_mlp_train(self.handle, m, _dev(row_ptr, torch.int64, "row_ptr", m + 1),
                                            _dev(col, torch.int32, "col"), _dev(val, torch.float32, "val"),
                                            _dev(target, torch.float32, "target", m * self.k), int(batch),
                                            float(lr), int(epochs), int(seed),
                                            hist.ctypes.data_as(ctypes.c_void_p)))
        return hist[:int(epochs)]

    def foldin(self, F, row_ptr, col, val, tau, lam, weighted=True, U_out=None, used_fallback=None, rho=None,
               count=True):
        m = row_ptr.numel() - 1
        if U_out is None:
            U_out = torch.empty((m, self.k), dtype=torch.float32, device=F.device)
        nf = ctypes.c_int64(-1)
        self.ctx.check(lib().open_mlp_foldin(self.handle, _dev(F, torch.float32, "F"), m,
                                             _dev(row_ptr, torch.int64, "row_ptr", m + 1),
                                             _dev(col, torch.int32, "col"), _dev(val, torch.float32, "val"),
                                             float(tau), float(lam), int(bool(weighted)),
                                             _dev(U_out, torch.float32, "U_out", m * self.k),
                                             _dev(used_fallback, torch.uint8, "used_fallback", m),
                                             _dev(rho, torch.float32, "rho", m),
                                             ctypes.byref(nf) if count else None))
        return U_out, (nf.value if count else None)

    def close(self):
        if getattr(self, "handle", None):
            lib().open_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NCF_D, NCF_H = 32, 64


def ncf_pack(E, S, net):
    """Flat NCF parameter vector (E, S, W1, b1, W2, b2, w3, b3) as float32 numpy."""
    import numpy as np
    parts = [E, S, net["W1"], net["b1"], net["W2"], net["b2"], net["w3"], net["b3"]]
    return np.concatenate([np.asarray(x, np.float32).reshape(-1) for x in parts])


def ncf_unpack(flat, m_off, n):
    """Views (E, S, {W1, b1, W2, b2, w3, b3}) into a flat NCF parameter vector (numpy or torch)."""
    d, H = NCF_D, NCF_H
    shapes = [("E", (m_off, d)), ("S", (n, d)), ("W1", (H, 2 * d)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
              ("w3", (H,)), ("b3", (1,))]
    out, o = {}, 0
    for name, shp in shapes:
        c = 1
        for x in shp:
            c *= x
        out[name] = flat[o:o + c].reshape(shp)
        o += c
    E, S = out.pop("E"), out.pop("S")
    return E, S, out


def open_ncf_train(ctx, R, params, apps_per_batch, lr, epochs, seed=0):
    """Train the NCF model (flat device parameter vector, updated in place) on the dense offline
    matrix R (device float32, m_off x n); returns the mean batch loss of each epoch."""
    import numpy as np
    m_off, n = R.shape
    hist = np.zeros(max(int(epochs), 1), dtype=np.float32)
    ctx.check(lib().open_ncf_train(ctx.handle, m_off, n, NCF_D, _dev(R, torch.float32, "R", m_off * n),
                                   _dev(params, torch.float32, "params", lib().open_ncf_num_params(m_off, n)),
                                   int(apps_per_batch), float(lr), int(epochs), int(seed),
                                   hist.ctypes.data_as(ctypes.c_void_p)))
    return hist[:int(epochs)]


def open_ncf_loss_grad(ctx, R, params, apps):
    """Loss and gradient (numpy float32, the flat packing) of the batch of applications `apps`."""
    import numpy as np
    m_off, n = R.shape
    npar = lib().open_ncf_num_params(m_off, n)
    g = np.empty(npar, dtype=np.float32)
    loss = ctypes.c_double()
    ctx.check(lib().open_ncf_loss_grad(ctx.handle, m_off, n, NCF_D, _dev(R, torch.float32, "R", m_off * n),
                                       _dev(params, torch.float32, "params", npar), _dev(apps, torch.int64, "apps"),
                                       int(apps.numel()), ctypes.byref(loss), g.ctypes.data_as(ctypes.c_void_p)))
    return loss.value, g
