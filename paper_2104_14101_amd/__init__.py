"""Adaptive sketching-based least-squares solvers (Lacotte & Pilanci, arXiv 2104.14101) on
MI355X: torch-facing wrappers over the C ABI of libaes.so (include/aes.h).

Every step of the solve runs in the library's HIP kernels; torch provides device memory and
the current stream only.  Tensors must be float64 HIP tensors; matrices are row-major.

    x, info = solve(A, b, nu, lam=None, tol=1e-10, method="pcg", sketch="srht", ...)
    q, pHp  = hv(A, p, nu, lam)                 # A^T (A p) + nu^2 Lambda p, one pass over A
    SA      = sketch(A, m, kind="srht", seed=0, k=0)
    G, L    = factor(SA, nu, lam)               # H_S (or W_S when m < d) and its Cholesky factor
    v       = precond_apply(SA, nu, lam, z)     # H_S^{-1} z
    results = solve_batched(problems, tol, ...)
    x       = SketchSolve.apply(A, b, log_nu, lam, opts)   # autograd: adjoint-solve backward
"""
import ctypes
import threading
import weakref

import torch

from . import _binding as B

__all__ = ["solve", "solve_dual", "solve_batched", "hv", "hv_multi", "sketch", "factor", "precond_apply", "SketchSolve", "AesError"]

AesError = B.AesError
# One library handle per device, shared by every Python thread: a handle's workspace pool and
# pinned flag block are for one call at a time, so every call on it holds that handle's lock.
_handles = {}
_handles_lock = threading.Lock()


def _lib():
    return B.load()


class _Handle:
    __slots__ = ("ptr", "lock")

    def __init__(self, ptr):
        self.ptr = ptr
        self.lock = threading.Lock()


def _handle_entry(device):
    idx = device.index if device.index is not None else torch.cuda.current_device()
    with _handles_lock:
        e = _handles.get(idx)
        if e is None:
            hv_ = ctypes.c_void_p()
            st = _lib().aes_create(ctypes.byref(hv_), idx)
            if st != 0:
                raise AesError(st, "aes_create failed")
            e = _Handle(hv_)
            _handles[idx] = e
    return e


def _handle(device):
    return _handle_entry(device).ptr


def _call(device, fn, *args):
    """Run one library call on the device's handle under its lock; returns (handle, status)."""
    e = _handle_entry(device)
    with e.lock:
        return e.ptr, fn(e.ptr, *args)


def _check(h, st):
    if st != 0:
        msg = _lib().aes_last_error(h)
        raise AesError(st, msg.decode() if msg else "")


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _req(t, name, ndim=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor on a HIP device")
    if ndim is not None and t.dim() not in ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    return t


def _lam(lam, d, device):
    """Lambda's diagonal: None (identity) or a float64 (d,) tensor on `device`."""
    if lam is None:
        return None
    _req(lam, "lam", (1,))
    if lam.shape[0] != d:
        raise ValueError(f"lam must have shape ({d},), got {tuple(lam.shape)}")
    if lam.device != device:
        raise ValueError(f"lam is on {lam.device}, A on {device}")
    return lam.contiguous()


def _out(x, d, c, device, squeeze):
    """Caller-given output buffer: float64 on `device`, shape (d,) or (d, c), unit column stride."""
    if x is None:
        return torch.empty((d, c), dtype=torch.float64, device=device)
    _req(x, "x", (1, 2))
    if x.device != device:
        raise ValueError(f"x is on {x.device}, A on {device}")
    if x.dim() == 1:
        if c != 1 or x.shape[0] != d:
            raise ValueError(f"x must have shape ({d}, {c})")
        if x.stride(0) != 1:
            raise ValueError("x must be contiguous")
        return x.view(d, 1)
    if tuple(x.shape) != (d, c):
        raise ValueError(f"x must have shape ({d}, {c}), got {tuple(x.shape)}")
    if x.stride(1) != 1 or x.stride(0) < c:
        raise ValueError("x must be row-major with unit column stride")
    return x


def _vec(t, name, d, device):
    _req(t, name, (1,))
    if t.shape[0] != d:
        raise ValueError(f"{name} must have shape ({d},), got {tuple(t.shape)}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, A on {device}")
    return t.contiguous()


def _mat(t, name, d, device):
    _req(t, name, (2,))
    if t.shape[0] != d:
        raise ValueError(f"{name} must have {d} rows, got {tuple(t.shape)}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, A on {device}")
    return t.contiguous()


def _rowmajor(t):
    if t.dim() == 2 and t.stride(1) == 1 and t.stride(0) >= t.shape[1]:
        return t, t.stride(0)
    t = t.contiguous()
    return t, (t.shape[1] if t.dim() == 2 else 1)


def make_options(method="pcg", sketch="srht", precision="fp64", stop="xrel", rho=0.125, m_init=1, m_max=0,
                 max_iter=200, seed=0, problem=0, adaptive=True, force_reject_at=-1, inner_tol=1e-6, max_refine=20,
                 trace_cap=0, x0=None, profile=False, keep_fp32_copy=False):
    o = B.Options()
    _lib().aes_default_options(ctypes.byref(o))
    o.method = B.METHODS[method]
    o.sketch = B.SKETCHES[sketch]
    o.precision = B.PRECISIONS[precision]
    o.stop = B.STOPS[stop]
    o.rho = float(rho)
    o.m_init = int(m_init)
    o.m_max = int(m_max)
    o.max_iter = int(max_iter)
    o.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    o.problem = int(problem)
    o.adaptive = 1 if adaptive else 0
    o.force_reject_at = int(force_reject_at)
    o.inner_tol = float(inner_tol)
    o.max_refine = int(max_refine)
    buf = None
    if trace_cap:
        buf = (B.TraceEntry * int(trace_cap))()
        o.trace = ctypes.cast(buf, ctypes.POINTER(B.TraceEntry))
        o.trace_cap = int(trace_cap)
    o.x0 = ctypes.c_void_p(x0.data_ptr()) if x0 is not None else None
    o.profile = 1 if profile else 0
    o.keep_fp32_copy = 1 if keep_fp32_copy else 0
    return o, buf


def _info_dict(info, buf):
    d = info.as_dict()
    if buf is not None:
        d["trace"] = [dict(t=buf[i].t, m=buf[i].m, k=buf[i].k, log_ratio=buf[i].log_ratio,
                           threshold=buf[i].threshold, accept=bool(buf[i].accept), dtilde=buf[i].dtilde,
                           time_ms=buf[i].time_ms) for i in range(info.trace_len)]
    return d


def solve(A, b, nu, lam=None, tol=1e-10, x=None, check=True, **opts):
    """Adaptive PCG / IHS solve of (A^T A + nu^2 Lambda) x = b.  Returns (x, info dict).

    b: (d,) or (d, c) with c <= 32.  Options: method, sketch, precision, stop, rho, m_init,
    m_max, max_iter, seed, problem, adaptive, force_reject_at, inner_tol, max_refine,
    trace_cap (record the attempted steps), x0, profile (event-time the fused H.v kernel),
    keep_fp32_copy (mixed precision: reuse the handle's FP32 copy of this same, unchanged A).
    """
    _req(A, "A", (2,))
    _req(b, "b", (1, 2))
    A, lda = _rowmajor(A)
    n, d = A.shape
    squeeze = b.dim() == 1
    b2 = b.reshape(d, 1) if squeeze else b
    b2, ldb = _rowmajor(b2)
    c = b2.shape[1]
    if b2.device != A.device:
        raise ValueError(f"b is on {b2.device}, A on {A.device}")
    lam = _lam(lam, d, A.device)
    x0 = opts.pop("x0", None)
    if x0 is not None:
        x0 = _req(x0, "x0").reshape(d, c).contiguous()
    o, buf = make_options(x0=x0, **opts)
    given = x
    x = _out(x, d, c, A.device, squeeze)
    info = B.Info()
    h, st = _call(A.device, _lib().aes_solve, _stream(A.device), n, d, c, _ptr(A), lda, _ptr(b2), ldb, float(nu),
                  _ptr(lam), float(tol), ctypes.byref(o), _ptr(x), x.stride(0), ctypes.byref(info))
    out = _info_dict(info, buf)
    if check and st not in (B.AES_OK, B.AES_ERR_MAX_ITER):
        _check(h, st)
    if given is not None:
        return given, out
    return (x.reshape(d) if squeeze else x), out


def solve_dual(A, b, nu, lam=None, tol=1e-10, x=None, check=True, **opts):
    """H x = b through the dual problem in R^n (n < d, n <= 32768).  Returns (x, info dict).

    Same arguments as ``solve`` (no x0); info describes the dual solve over Lambda^{-1/2} A^T.
    """
    _req(A, "A", (2,))
    _req(b, "b", (1, 2))
    A, lda = _rowmajor(A)
    n, d = A.shape
    squeeze = b.dim() == 1
    b2 = b.reshape(d, 1) if squeeze else b
    b2, ldb = _rowmajor(b2)
    c = b2.shape[1]
    if b2.device != A.device:
        raise ValueError(f"b is on {b2.device}, A on {A.device}")
    lam = _lam(lam, d, A.device)
    if opts.get("x0") is not None:
        raise ValueError("the dual form takes no start point")
    opts.pop("x0", None)
    o, buf = make_options(**opts)
    given = x
    x = _out(x, d, c, A.device, squeeze)
    info = B.Info()
    h, st = _call(A.device, _lib().aes_solve_dual, _stream(A.device), n, d, c, _ptr(A), lda, _ptr(b2), ldb, float(nu),
                  _ptr(lam), float(tol), ctypes.byref(o), _ptr(x), x.stride(0), ctypes.byref(info))
    out = _info_dict(info, buf)
    if check and st not in (B.AES_OK, B.AES_ERR_MAX_ITER):
        _check(h, st)
    if given is not None:
        return given, out
    return (x.reshape(d) if squeeze else x), out


def solve_direct(A, b, nu, lam=None, x=None):
    """The direct baseline of Sec. 5: Cholesky of the full H = A^T A + nu^2 Lambda.  Returns x.

    A (n x d), b (d or d x c, c <= 32), lam and x as for ``solve``; FP64 only.
    """
    _req(A, "A", (2,))
    _req(b, "b", (1, 2))
    A, lda = _rowmajor(A)
    n, d = A.shape
    squeeze = b.dim() == 1
    b2 = b.reshape(d, 1) if squeeze else b
    b2, ldb = _rowmajor(b2)
    c = b2.shape[1]
    if b2.device != A.device:
        raise ValueError(f"b is on {b2.device}, A on {A.device}")
    lam = _lam(lam, d, A.device)
    given = x
    x = _out(x, d, c, A.device, squeeze)
    _check(*_call(A.device, _lib().aes_solve_direct, _stream(A.device), n, d, c, _ptr(A), lda, _ptr(b2), ldb,
                  float(nu), _ptr(lam), _ptr(x), x.stride(0)))
    if given is not None:
        return given
    return x.reshape(d) if squeeze else x


def solve_batched(problems, tol=1e-10, **opts):
    """Solve a list of problems dict(A, b, nu, lam=None); problem p uses Philox stream p.

    Returns a list of (x, info dict)."""
    if not problems:
        return []
    dev = problems[0]["A"].device
    arr = (B.Problem * len(problems))()
    keep = []
    outs = []
    for i, pr in enumerate(problems):
        A, lda = _rowmajor(_req(pr["A"], "A", (2,)))
        if A.device != dev:
            raise ValueError(f"problem {i}: A is on {A.device}, problem 0 on {dev}")
        b = _req(pr["b"], "b", (1, 2))
        n, d = A.shape
        b2 = b.reshape(d, 1) if b.dim() == 1 else b
        b2, ldb = _rowmajor(b2)
        if b2.device != dev:
            raise ValueError(f"problem {i}: b is on {b2.device}, A on {dev}")
        c = b2.shape[1]
        lam = _lam(pr.get("lam"), d, dev)
        x = torch.empty((d, c), dtype=torch.float64, device=dev)
        keep += [A, b2, lam, x]
        outs.append((x, b.dim() == 1))
        arr[i] = B.Problem(n, d, c, A.data_ptr(), lda, b2.data_ptr(), ldb, float(pr["nu"]),
                           lam.data_ptr() if lam is not None else None, x.data_ptr(), c)
    o, _ = make_options(**opts)
    infos = (B.Info * len(problems))()
    h, st = _call(dev, _lib().aes_solve_batched, _stream(dev), len(problems), arr, float(tol), ctypes.byref(o), infos)
    if st not in (B.AES_OK, B.AES_ERR_MAX_ITER):
        _check(h, st)
    return [(x.reshape(-1) if sq else x, infos[i].as_dict()) for i, (x, sq) in enumerate(outs)]


def hv(A, p, nu, lam=None):
    """(q, pHp): q = A^T (A p) + nu^2 Lambda p and pHp = ||A p||^2 + nu^2 p^T Lambda p."""
    _req(A, "A", (2,))
    A, lda = _rowmajor(A)
    n, d = A.shape
    p = _vec(p, "p", d, A.device)
    lam = _lam(lam, d, A.device)
    q = torch.empty(d, dtype=torch.float64, device=A.device)
    php = torch.empty(1, dtype=torch.float64, device=A.device)
    _check(*_call(A.device, _lib().aes_hv, _stream(A.device), n, d, _ptr(A), lda, float(nu), _ptr(lam), _ptr(p),
                  _ptr(q), _ptr(php)))
    return q, php


def hv_multi(A, P, nu, lam=None, precision="fp64"):
    """Q = A^T (A P) + nu^2 Lambda P for P of shape (d, c), c a power of two <= 32."""
    _req(A, "A", (2,))
    A, lda = _rowmajor(A)
    n, d = A.shape
    P = _mat(P, "P", d, A.device)
    c = P.shape[1]
    lam = _lam(lam, d, A.device)
    Q = torch.empty_like(P)
    _check(*_call(A.device, _lib().aes_hv_multi, _stream(A.device), n, d, c, _ptr(A), lda, float(nu), _ptr(lam),
                  _ptr(P), _ptr(Q), B.PRECISIONS[precision]))
    return Q


def sketch(A, m, kind="srht", seed=0, k=0, problem=0):
    """S A (m x d) for sketch index k (see include/aes.h for the random streams)."""
    _req(A, "A", (2,))
    A, lda = _rowmajor(A)
    n, d = A.shape
    SA = torch.empty((m, d), dtype=torch.float64, device=A.device)
    _check(*_call(A.device, _lib().aes_sketch, _stream(A.device), B.SKETCHES[kind], n, d, _ptr(A), lda, int(m),
                  int(seed), int(problem), int(k), _ptr(SA)))
    return SA


def factor(SA, nu, lam=None):
    """(G, L): G = SA^T SA + nu^2 Lambda (m >= d) or SA Lambda^-1 SA^T + nu^2 I (m < d), lower
    triangle, and its lower Cholesky factor."""
    SA = _req(SA, "SA", (2,)).contiguous()
    m, d = SA.shape
    dim = d if m >= d else m
    G = torch.empty((dim, dim), dtype=torch.float64, device=SA.device)
    L = torch.empty((dim, dim), dtype=torch.float64, device=SA.device)
    lam = _lam(lam, d, SA.device)
    _check(*_call(SA.device, _lib().aes_factor, _stream(SA.device), m, d, _ptr(SA), float(nu), _ptr(lam), _ptr(G),
                  _ptr(L)))
    return G, L


def precond_apply(SA, nu, lam, z):
    """H_S^{-1} z for z of shape (d,) or (d, c) with c a power of two <= 32."""
    SA = _req(SA, "SA", (2,)).contiguous()
    m, d = SA.shape
    squeeze = _req(z, "z", (1, 2)).dim() == 1
    z2 = _mat(z.reshape(d, -1) if z.shape[0] == d else z, "z", d, SA.device)
    c = z2.shape[1]
    v = torch.empty_like(z2)
    lam = _lam(lam, d, SA.device)
    _check(*_call(SA.device, _lib().aes_precond_apply, _stream(SA.device), m, d, c, _ptr(SA), float(nu), _ptr(lam),
                  _ptr(z2), _ptr(v)))
    return v.reshape(d) if squeeze else v


def _free_ctx(addr):
    _lib().aes_ctx_free(ctypes.c_void_p(addr))


class _KeptContext:
    """Owner of an aes_ctx (the forward solve's sketch, factor and x*): the context is freed
    when this object is collected (the autograd graph that holds it is released, after a
    backward without retain_graph, or when the output is dropped without one) or by free()."""

    def __init__(self, ptr, entry):
        self.ptr = ptr
        self.entry = entry  # the device handle entry: calls on the context hold its lock
        self._fin = weakref.finalize(self, _free_ctx, ptr.value)
        self._fin.atexit = False

    def free(self):
        self._fin()

    @property
    def alive(self):
        return self._fin.alive


class SketchSolve(torch.autograd.Function):
    """x* = argmin 1/2 x^T (A^T A + nu^2 Lambda) x - b^T x with nu = exp(log_nu).

    Forward: adaptive PCG (aes_solve_keep when a gradient is needed, plain aes_solve
    otherwise).  Backward: the adjoint solve H lam = dL/dx* by adaptive PCG reusing the forward
    sketch and factorisation (aes_adjoint_solve), then dL/db = lam,
    dL/dA = -(A x*) lam^T - (A lam) x*^T, dL/dlog_nu = -2 nu^2 lam^T Lambda x*.
    The kept context lives as long as the autograd graph (a second backward with
    retain_graph=True reuses it) and is freed with it.
    """

    @classmethod
    def apply(cls, A, b, log_nu, lam=None, opts=None):
        needs = torch.is_grad_enabled() and any(
            isinstance(t, torch.Tensor) and t.requires_grad for t in (A, b, log_nu, lam))
        if not needs:
            o = dict(opts or {})
            tol = o.pop("tol", 1e-10)
            nu = float(torch.exp(log_nu.detach()).item())
            x, _ = solve(A.detach(), b.detach(), nu, lam.detach() if lam is not None else None, tol=tol, **o)
            return x
        return super().apply(A, b, log_nu, lam, opts)

    @staticmethod
    def forward(ctx, A, b, log_nu, lam=None, opts=None):
        opts = dict(opts or {})
        tol = opts.pop("tol", 1e-10)
        A_c, lda = _rowmajor(_req(A.detach(), "A", (2,)))
        n, d = A_c.shape
        b_c = _vec(b.detach(), "b", d, A_c.device)
        nu = float(torch.exp(log_nu.detach()).item())
        lam_c = _lam(lam.detach() if lam is not None else None, d, A_c.device)
        o, _ = make_options(**opts)
        x = torch.empty(d, dtype=torch.float64, device=A.device)
        info = B.Info()
        cptr = ctypes.c_void_p()
        h, st = _call(A.device, _lib().aes_solve_keep, _stream(A.device), n, d, 1, _ptr(A_c), lda, _ptr(b_c), 1, nu,
                      _ptr(lam_c), float(tol), ctypes.byref(o), _ptr(x), 1, ctypes.byref(info), ctypes.byref(cptr))
        if st != B.AES_OK:
            _check(h, st)
        ctx.kept = _KeptContext(cptr, _handle_entry(A.device))
        ctx.keep = (A_c, lam_c)
        ctx.tol = tol
        ctx.info = info.as_dict()
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        kept = ctx.kept
        if kept is None or not kept.alive:
            raise RuntimeError("SketchSolve: the kept context was already released")
        g = _vec(gx.detach().to(torch.float64), "grad", x.shape[0], x.device)
        lamv = torch.empty_like(g)
        info = B.Info()
        lib = _lib()
        A_c, _ = ctx.keep
        dA = None
        if ctx.needs_input_grad[0]:
            dA = torch.empty((A_c.shape[0], A_c.shape[1]), dtype=torch.float64, device=A_c.device)
        dln = ctypes.c_double(0.0)
        with kept.entry.lock:
            st = lib.aes_adjoint_solve(kept.ptr, _stream(g.device), _ptr(g), float(ctx.tol), _ptr(lamv),
                                       ctypes.byref(info))
            if st != B.AES_OK:
                raise AesError(st, "adjoint solve failed")
            st = lib.aes_grad(kept.ptr, _stream(g.device), _ptr(lamv), _ptr(dA), ctypes.byref(dln))
        if st != B.AES_OK:
            raise AesError(st, "gradient kernel failed")
        dlognu = torch.tensor(dln.value, dtype=torch.float64, device=g.device)
        return dA, lamv, dlognu, None, None
