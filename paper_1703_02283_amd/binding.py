"""ctypes binding of include/ipr.h: argument marshalling only.

Tensors passed in must be CUDA (HIP) tensors of the documented dtype and
shape, contiguous, on the current device. Work is queued on torch's current
stream unless a stream is given.
"""
from __future__ import annotations

import ctypes as ct
import os

import torch

IPR_OK, IPR_EARG, IPR_EMAXITER, IPR_EFLOOR, IPR_EDIVERGED, IPR_EHIP, IPR_EGUARD = range(7)
IPR_INIT_IDENTITY, IPR_INIT_PAPER_EQ3, IPR_INIT_POLY, IPR_INIT_LEARNED, IPR_INIT_USER = range(5)
IPR_EVAL_COUPLED, IPR_EVAL_LITERAL, IPR_EVAL_NEWTON_SCHULZ = range(3)
IPR_FP64, IPR_BF16, IPR_FP16, IPR_FP8_E4M3, IPR_FP64_INT8_EMUL = range(5)
IPR_STORE_NONE, IPR_STORE_FLOAT, IPR_STORE_FIXED = range(3)
IPR_MLP_NPARAM = 64 * 16 + 64 + 64 * 64 + 64 + 3 * 64 + 3
STATUS_NAMES = {0: "OK", 1: "EARG", 2: "EMAXITER", 3: "EFLOOR", 4: "EDIVERGED", 5: "EHIP",
                6: "EGUARD"}


class IprSchedule(ct.Structure):
    _fields_ = [("init", ct.c_int), ("bulk_dtype", ct.c_int), ("max_iter", ct.c_int),
                ("triangle", ct.c_int), ("guard_fallback", ct.c_int), ("verify", ct.c_int),
                ("bulk_switch", ct.c_double), ("stall_ratio", ct.c_double),
                ("poly", ct.c_double * 3), ("mlp_params", ct.c_void_p), ("timing", ct.c_int),
                ("tile", ct.c_int), ("scale_squarings", ct.c_int),
                ("dynamic_scaling", ct.c_int), ("evaluation", ct.c_int),
                ("emul_slices", ct.c_int), ("store_format", ct.c_int),
                ("store_bits", ct.c_int), ("store_regime", ct.c_int),
                ("hist_ref", ct.c_void_p), ("hist_err", ct.c_void_p), ("hist_rho", ct.c_void_p),
                ("hist_len", ct.c_int), ("bulk_force", ct.c_int), ("scale_lanczos", ct.c_int)]


class IprResult(ct.Structure):
    _fields_ = [("status", ct.c_int), ("iters_bulk", ct.c_int), ("iters_fp64", ct.c_int),
                ("fallback_used", ct.c_int), ("gemms", ct.c_int),
                ("residual_proxy", ct.c_double), ("residual_true", ct.c_double),
                ("init_bound", ct.c_double), ("norm1", ct.c_double), ("norminf", ct.c_double),
                ("poly_used", ct.c_double * 3), ("init_scale", ct.c_double),
                ("ms_norms", ct.c_double),
                ("ms_init", ct.c_double), ("ms_bulk", ct.c_double), ("ms_refine", ct.c_double),
                ("ms_verify", ct.c_double), ("gemm_launches", ct.c_int), ("ms_gemm", ct.c_double),
                ("gemm_flops", ct.c_double), ("lp_gemm_launches", ct.c_int),
                ("ms_lp_gemm", ct.c_double), ("lp_gemm_flops", ct.c_double),
                ("lmin_est", ct.c_double), ("reest_iter", ct.c_int),
                ("lmin_reest", ct.c_double), ("bulk_skipped", ct.c_int)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["poly_used"] = list(self.poly_used)
        d["status_name"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


class IprError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def library_path() -> str:
    return os.path.join(_HERE, "libipr.so")


_SIGS = {
    "ipr_schedule_default": (None, [ct.c_void_p]),
    "ipr_workspace_size": (ct.c_size_t, [ct.c_int, ct.c_int, ct.c_int, ct.c_void_p]),
    "ipr_solve": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int, ct.c_double,
                             ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "ipr_solve_batched": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                     ct.c_void_p, ct.c_int, ct.c_double, ct.c_void_p,
                                     ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "ipr_gemm": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int,
                            ct.c_double, ct.c_double, ct.c_double, ct.c_int, ct.c_void_p]),
    "ipr_gemm_lowp": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int,
                                 ct.c_int, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "ipr_gemm_lowp_workspace": (ct.c_size_t, [ct.c_int]),
    "ipr_gemm_emul": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int, ct.c_int,
                                 ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "ipr_gemm_emul_workspace": (ct.c_size_t, [ct.c_int, ct.c_int]),
    "ipr_lowdin": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int,
                              ct.c_double, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t,
                              ct.c_void_p]),
    "ipr_lowdin_workspace": (ct.c_size_t, [ct.c_int, ct.c_void_p]),
    "ipr_norms": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_size_t,
                             ct.c_void_p]),
    "ipr_features": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int,
                                ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "ipr_mlp_forward": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int,
                                   ct.c_void_p]),
    "ipr_mlp_train_step": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                      ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int, ct.c_float,
                                      ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]),
    "ipr_mlp_workspace": (ct.c_size_t, [ct.c_int]),
    "ipr_last_error": (ct.c_char_p, []),
    "ipr_tune_batched": (ct.c_int, [ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.c_void_p]),
    "ipr_spectral_counts": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                       ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int, ct.c_double,
                                       ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_size_t,
                                       ct.c_void_p]),
    "ipr_solve_noalloc": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int, ct.c_double,
                                     ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "ipr_eigvalsh": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_size_t,
                                ct.c_void_p]),
    "ipr_eigvalsh_workspace": (ct.c_size_t, [ct.c_int]),
    "ipr_get_batched_tiles": (ct.c_int, [ct.c_void_p]),
    "ipr_set_batched_tiles": (ct.c_int, [ct.c_void_p]),
}


def load():
    """Loads libipr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with "
                               "`python -m paper_1703_02283_amd.build`")
        lib = ct.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _fn(name):
    f = getattr(load(), name, None)
    if f is None:
        raise RuntimeError(f"{name} is not exported by {library_path()}")
    return f


def ipr_last_error() -> str:
    return _fn("ipr_last_error")().decode()


def _check(code, allow=()):
    if code != IPR_OK and code not in allow:
        raise IprError(code, ipr_last_error())
    return code


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _need(t, dtype, shape=None, name="tensor"):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")


def ipr_schedule_default(**overrides) -> IprSchedule:
    s = IprSchedule()
    _fn("ipr_schedule_default")(ct.byref(s))
    for k, v in overrides.items():
        if k == "poly":
            s.poly = (ct.c_double * 3)(*v)
        elif k == "mlp_params":
            if v is not None:
                _need(v, torch.float32, (IPR_MLP_NPARAM,), "mlp_params")
            s.mlp_params = None if v is None else v.data_ptr()
            s._mlp_ref = v  # the schedule holds only the pointer: keep the tensor alive
        else:
            setattr(s, k, v)
    return s


def ipr_workspace_size(n_max, p_max, batch=1, schedule=None) -> int:
    return int(_fn("ipr_workspace_size")(n_max, p_max, batch,
                                         ct.byref(schedule) if schedule else None))


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def ipr_solve(A, p, tol, schedule=None, out=None, workspace=None, stream=None,
              raise_on=(IPR_EARG, IPR_EHIP, IPR_EGUARD)):
    """A^{-1/p} of the SPD matrix A (n x n float64 device tensor).
    Returns (C, IprResult); numerical outcomes other than OK are reported in
    result.status (and raise only when listed in ``raise_on``). With
    init=IPR_INIT_USER, ``out`` holds C_0 on entry."""
    _need(A, torch.float64, name="A")
    n = A.shape[0]
    if A.dim() != 2 or A.shape[1] != n:
        raise ValueError("A must be square")
    sch = schedule if schedule is not None else ipr_schedule_default()
    if sch.init == IPR_INIT_USER and out is None:
        raise ValueError("init=IPR_INIT_USER takes C_0 in `out`")
    C = out if out is not None else torch.empty_like(A)
    _need(C, torch.float64, (n, n), "out")
    need = ipr_workspace_size(n, p, 1, sch)
    ws = workspace if workspace is not None else _workspace(need, A.device)
    res = IprResult()
    rc = _fn("ipr_solve")(_ptr(A), _ptr(C), n, p, tol, ct.byref(sch), ct.byref(res),
                          _ptr(ws), ws.numel(), _stream(stream))
    if rc in raise_on:
        raise IprError(rc, ipr_last_error())
    return C, res


IPR_NOALLOC_SCRATCH_BYTES = 64 << 20


def ipr_solve_noalloc(A, p, tol, schedule=None, out=None, stream=None,
                      raise_on=(IPR_EARG, IPR_EHIP, IPR_EGUARD)):
    """ipr_solve on the library's fixed device scratch instead of a caller
    workspace (see include/ipr.h). ``out`` (n x n float64 device tensor) is
    the caller's output buffer; the call itself allocates nothing."""
    _need(A, torch.float64, name="A")
    n = A.shape[0]
    if A.dim() != 2 or A.shape[1] != n:
        raise ValueError("A must be square")
    sch = schedule if schedule is not None else ipr_schedule_default()
    if sch.init == IPR_INIT_USER and out is None:
        raise ValueError("init=IPR_INIT_USER takes C_0 in `out`")
    C = out if out is not None else torch.empty_like(A)
    _need(C, torch.float64, (n, n), "out")
    res = IprResult()
    rc = _fn("ipr_solve_noalloc")(_ptr(A), _ptr(C), n, p, tol, ct.byref(sch), ct.byref(res),
                                  _stream(stream))
    if rc in raise_on:
        raise IprError(rc, ipr_last_error())
    return C, res


def ipr_lowdin(S, H, tol, schedule=None, out_x=None, out_h=None, workspace=None, stream=None,
               raise_on=(IPR_EARG, IPR_EHIP, IPR_EGUARD)):
    """(X, X H X, IprResult) with X = S^{-1/2} (see include/ipr.h)."""
    _need(S, torch.float64, name="S")
    n = S.shape[0]
    _need(H, torch.float64, (n, n), "H")
    sch = schedule if schedule is not None else ipr_schedule_default()
    X = out_x if out_x is not None else torch.empty_like(S)
    Ht = out_h if out_h is not None else torch.empty_like(S)
    ws = workspace if workspace is not None else _workspace(
        int(_fn("ipr_lowdin_workspace")(n, ct.byref(sch))), S.device)
    res = IprResult()
    rc = _fn("ipr_lowdin")(_ptr(S), _ptr(H), _ptr(X), _ptr(Ht), n, tol, ct.byref(sch),
                           ct.byref(res), _ptr(ws), ws.numel(), _stream(stream))
    if rc in raise_on:
        raise IprError(rc, ipr_last_error())
    return X, Ht, res


def ipr_solve_batched(A_packed, offsets, ns, ps, tol, schedule=None, out=None,
                      workspace=None, stream=None):
    """Independent solves of a packed batch (see include/ipr.h). offsets, ns,
    ps are Python sequences. Returns (C_packed, [IprResult])."""
    _need(A_packed, torch.float64, name="A_packed")
    batch = len(ns)
    off = (ct.c_int64 * batch)(*[int(o) for o in offsets])
    nn = (ct.c_int * batch)(*[int(v) for v in ns])
    pp = (ct.c_int * batch)(*[int(v) for v in ps])
    sch = schedule if schedule is not None else ipr_schedule_default()
    C = out if out is not None else torch.empty_like(A_packed)
    tot = sum(int(v) * int(v) for v in ns)
    need = ipr_workspace_size(int(max(ns)), int(max(ps)), batch, sch)
    need = max(need, int(_fn("ipr_workspace_size")(max(1, int(tot ** 0.5) + 1), int(max(ps)),
                                                     batch, ct.byref(sch))))
    ws = workspace if workspace is not None else _workspace(need, A_packed.device)
    res = (IprResult * batch)()
    rc = _fn("ipr_solve_batched")(_ptr(A_packed), _ptr(C), off, nn, pp, batch, tol,
                                  ct.byref(sch), res, _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, allow=(IPR_EMAXITER, IPR_EFLOOR, IPR_EDIVERGED))
    return C, list(res)


IPR_BATCH_BUCKETS = 6


def ipr_tune_batched(workspace_bytes=None, device="cuda", stream=None):
    """Runs the batched solver's tile autotuner; returns the table."""
    need = ipr_workspace_size(1024, 1, 1)
    ws = _workspace(max(need, workspace_bytes or 0), device)
    out = (ct.c_int * IPR_BATCH_BUCKETS)()
    _check(_fn("ipr_tune_batched")(_ptr(ws), ws.numel(), out, _stream(stream)))
    return list(out)


def ipr_get_batched_tiles():
    out = (ct.c_int * IPR_BATCH_BUCKETS)()
    _check(_fn("ipr_get_batched_tiles")(out))
    return list(out)


def ipr_set_batched_tiles(tiles):
    arr = (ct.c_int * IPR_BATCH_BUCKETS)(*[int(t) for t in tiles])
    _check(_fn("ipr_set_batched_tiles")(arr))


def ipr_gemm(L, R, X=None, alpha=1.0, beta=0.0, gamma=0.0, triangle=False, out=None,
             stream=None):
    """D = alpha L^T R + beta X + gamma I on the FP64 matrix cores."""
    n = L.shape[0]
    for t, nm in ((L, "L"), (R, "R")):
        _need(t, torch.float64, (n, n), nm)
    if X is not None:
        _need(X, torch.float64, (n, n), "X")
    D = out if out is not None else torch.empty_like(L)
    _check(_fn("ipr_gemm")(_ptr(L), _ptr(R), _ptr(X), _ptr(D), n, alpha, beta, gamma,
                           1 if triangle else 0, _stream(stream)))
    return D


def ipr_gemm_lowp_workspace(n) -> int:
    return int(_fn("ipr_gemm_lowp_workspace")(n))


def ipr_gemm_lowp(L, R, dtype, out=None, workspace=None, stream=None, triangle=False):
    """D = L^T R with operands stored in a low-precision format (fp32 accumulate);
    triangle: upper tiles computed, D mirrored from them."""
    n = L.shape[0]
    for t, nm in ((L, "L"), (R, "R")):
        _need(t, torch.float64, (n, n), nm)
    D = out if out is not None else torch.empty_like(L)
    ws = workspace if workspace is not None else _workspace(ipr_gemm_lowp_workspace(n), L.device)
    _check(_fn("ipr_gemm_lowp")(_ptr(L), _ptr(R), _ptr(D), n, int(dtype), 1 if triangle else 0,
                                _ptr(ws), ws.numel(), _stream(stream)))
    return D


def ipr_gemm_emul_workspace(n, slices=10) -> int:
    return int(_fn("ipr_gemm_emul_workspace")(n, slices))


def ipr_gemm_emul(L, R, slices=10, out=None, workspace=None, stream=None, triangle=False):
    """D = L^T R, FP64-accurate, from int8 digit slices on the matrix cores
    (triangle: upper tiles computed, D mirrored from them)."""
    n = L.shape[0]
    for t, nm in ((L, "L"), (R, "R")):
        _need(t, torch.float64, (n, n), nm)
    D = out if out is not None else torch.empty_like(L)
    ws = workspace if workspace is not None else _workspace(
        ipr_gemm_emul_workspace(n, slices), L.device)
    _check(_fn("ipr_gemm_emul")(_ptr(L), _ptr(R), _ptr(D), n, int(slices), 1 if triangle else 0,
                                _ptr(ws), ws.numel(), _stream(stream)))
    return D


def ipr_eigvalsh(A, out=None, workspace=None, stream=None):
    """Eigenvalues (ascending, float64 device tensor of n) of the symmetric A."""
    _need(A, torch.float64, name="A")
    n = A.shape[0]
    W = out if out is not None else torch.empty(n, dtype=torch.float64, device=A.device)
    _need(W, torch.float64, (n,), "out")
    ws = workspace if workspace is not None else _workspace(
        int(_fn("ipr_eigvalsh_workspace")(n)), A.device)
    _check(_fn("ipr_eigvalsh")(_ptr(A), n, _ptr(W), _ptr(ws), ws.numel(), _stream(stream)))
    return W


def ipr_norms(A, workspace=None, stream=None):
    """(||A||_1, ||A||_inf)."""
    _need(A, torch.float64, name="A")
    n = A.shape[0]
    ws = workspace if workspace is not None else _workspace(8 * (n * (n // 256 + 4) + 64),
                                                            A.device)
    out = (ct.c_double * 2)()
    _check(_fn("ipr_norms")(_ptr(A), n, out, _ptr(ws), ws.numel(), _stream(stream)))
    return out[0], out[1]


def ipr_features(A_packed, offsets, ns, ps, workspace=None, stream=None):
    """batch x 16 float32 features of a packed batch."""
    _need(A_packed, torch.float64, name="A_packed")
    batch = len(ns)
    off = (ct.c_int64 * batch)(*[int(o) for o in offsets])
    nn = (ct.c_int * batch)(*[int(v) for v in ns])
    pp = (ct.c_int * batch)(*[int(v) for v in ps])
    feat = torch.empty((batch, 16), dtype=torch.float32, device=A_packed.device)
    ws = workspace if workspace is not None else _workspace(16 * batch + 2048, A_packed.device)
    _check(_fn("ipr_features")(_ptr(A_packed), off, nn, pp, batch, _ptr(feat), _ptr(ws),
                               ws.numel(), _stream(stream)))
    return feat


def ipr_spectral_counts(lam_packed, offsets, ns, ps, scales, cands, tol, max_iter=200,
                        per_item=False, stream=None):
    """Exact-arithmetic iteration counts (batch x ncand numpy int array) of the
    coupled iteration per eigenvalue for candidate polynomial starts."""
    import numpy as np
    _need(lam_packed, torch.float64, name="lam_packed")
    batch = len(ns)
    cand = np.ascontiguousarray(np.asarray(cands, dtype=np.float64).reshape(-1, 3))
    ncand = 0 if per_item else cand.shape[0]
    if per_item and cand.shape[0] != batch:
        raise ValueError("per_item needs one candidate per matrix")
    off = (ct.c_int64 * batch)(*[int(o) for o in offsets])
    nn = (ct.c_int * batch)(*[int(v) for v in ns])
    pp = (ct.c_int * batch)(*[int(v) for v in ps])
    sc = (ct.c_double * batch)(*[float(v) for v in scales])
    cc = cand.ctypes.data_as(ct.c_void_p)
    out = np.zeros((batch, max(ncand, 1)), dtype=np.int32)
    nc = max(ncand, batch if per_item else 1)
    ws = _workspace(batch * (16 + 8) + 24 * nc + 4 * batch * max(ncand, 1) + 8192,
                    lam_packed.device)
    _check(_fn("ipr_spectral_counts")(_ptr(lam_packed), off, nn, pp, sc, batch, cc, ncand,
                                      float(tol), int(max_iter), out.ctypes.data_as(ct.c_void_p),
                                      _ptr(ws), ws.numel(), _stream(stream)))
    return out[:, 0] if per_item else out


def ipr_mlp_forward(params, X, stream=None):
    _need(params, torch.float32, (IPR_MLP_NPARAM,), "params")
    _need(X, torch.float32, None, "X")
    Y = torch.empty((X.shape[0], 3), dtype=torch.float32, device=X.device)
    _check(_fn("ipr_mlp_forward")(_ptr(params), _ptr(X), _ptr(Y), X.shape[0], _stream(stream)))
    return Y


def ipr_mlp_workspace(batch) -> int:
    return int(_fn("ipr_mlp_workspace")(batch))


def ipr_mlp_train_step(params, grad, m, v, X, T, step, lr, loss_out, workspace=None,
                       stream=None):
    for t, nm in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _need(t, torch.float32, (IPR_MLP_NPARAM,), nm)
    _need(X, torch.float32, None, "X")
    _need(T, torch.float32, (X.shape[0], 3), "T")
    ws = workspace if workspace is not None else _workspace(ipr_mlp_workspace(X.shape[0]),
                                                            X.device)
    _check(_fn("ipr_mlp_train_step")(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), _ptr(X),
                                     _ptr(T), X.shape[0], int(step), float(lr), _ptr(loss_out),
                                     _ptr(ws), ws.numel(), _stream(stream)))
