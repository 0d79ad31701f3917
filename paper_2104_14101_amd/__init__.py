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

import torch

from . import _binding as B

__all__ = ["solve", "solve_dual", "solve_batched", "hv", "hv_multi", "sketch", "factor", "precond_apply", "SketchSolve", "AesError"]

AesError = B.AesError
_handles = {}


def _lib():
    return B.load()


def _handle(device):
    idx = device.index if device.index is not None else torch.cuda.current_device()
    h = _handles.get(idx)
    if h is None:
        hv_ = ctypes.c_void_p()
        st = _lib().aes_create(ctypes.byref(hv_), idx)
        if st != 0:
            raise AesError(st, "aes_create failed")
        h = hv_
        _handles[idx] = h
    return h


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


def _rowmajor(t):
    if t.dim() == 2 and t.stride(1) == 1 and t.stride(0) >= t.shape[1]:
        return t, t.stride(0)
    t = t.contiguous()
    return t, (t.shape[1] if t.dim() == 2 else 1)


def make_options(method="pcg", sketch="srht", precision="fp64", stop="xrel", rho=0.125, m_init=1, m_max=0,
                 max_iter=200, seed=0, problem=0, adaptive=True, force_reject_at=-1, inner_tol=1e-6, max_refine=20,
                 trace_cap=0, x0=None, profile=False):
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
    return o, buf


def _info_dict(info, buf):
    d = info.as_dict()
    if buf is not None:
        d["trace"] = [dict(t=buf[i].t, m=buf[i].m, k=buf[i].k, log_ratio=buf[i].log_ratio,
                           threshold=buf[i].threshold, accept=bool(buf[i].accept)) for i in range(info.trace_len)]
    return d


def solve(A, b, nu, lam=None, tol=1e-10, x=None, check=True, **opts):
    """Adaptive PCG / IHS solve of (A^T A + nu^2 Lambda) x = b.  Returns (x, info dict).

    b: (d,) or (d, c) with c <= 32.  Options: method, sketch, precision, stop, rho, m_init,
    m_max, max_iter, seed, problem, adaptive, force_reject_at, inner_tol, max_refine,
    trace_cap (record the attempted steps), x0, profile (event-time the fused H.v kernel).
    """
    _req(A, "A", (2,))
    _req(b, "b", (1, 2))
    A, lda = _rowmajor(A)
    n, d = A.shape
    squeeze = b.dim() == 1
    b2 = b.reshape(d, 1) if squeeze else b
    b2, ldb = _rowmajor(b2)
    c = b2.shape[1]
    if lam is not None:
        _req(lam, "lam", (1,))
        lam = lam.contiguous()
    x0 = opts.pop("x0", None)
    if x0 is not None:
        x0 = _req(x0, "x0").reshape(d, c).contiguous()
    o, buf = make_options(x0=x0, **opts)
    if x is None:
        x = torch.empty((d, c), dtype=torch.float64, device=A.device)
    info = B.Info()
    h = _handle(A.device)
    st = _lib().aes_solve(h, _stream(A.device), n, d, c, _ptr(A), lda, _ptr(b2), ldb, float(nu), _ptr(lam), float(tol),
                          ctypes.byref(o), _ptr(x), x.stride(0), ctypes.byref(info))
    out = _info_dict(info, buf)
    if check and st not in (B.AES_OK, B.AES_ERR_MAX_ITER):
        _check(h, st)
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
    if lam is not None:
        _req(lam, "lam", (1,))
        lam = lam.contiguous()
    if opts.get("x0") is not None:
        raise ValueError("the dual form takes no start point")
    opts.pop("x0", None)
    o, buf = make_options(**opts)
    if x is None:
        x = torch.empty((d, c), dtype=torch.float64, device=A.device)
    info = B.Info()
    h = _handle(A.device)
    st = _lib().aes_solve_dual(h, _stream(A.device), n, d, c, _ptr(A), lda, _ptr(b2), ldb, float(nu), _ptr(lam),
                               float(tol), ctypes.byref(o), _ptr(x), x.stride(0), ctypes.byref(info))
    out = _info_dict(info, buf)
    if check and st not in (B.AES_OK, B.AES_ERR_MAX_ITER):
        _check(h, st)
    return (x.reshape(d) if squeeze else x), out


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
        b = _req(pr["b"], "b", (1, 2))
        n, d = A.shape
        b2 = b.reshape(d, 1) if b.dim() == 1 else b
        b2, ldb = _rowmajor(b2)
        c = b2.shape[1]
        lam = pr.get("lam")
        lam = lam.contiguous() if lam is not None else None
        x = torch.empty((d, c), dtype=torch.float64, device=dev)
        keep += [A, b2, lam, x]
        outs.append((x, b.dim() == 1))
        arr[i] = B.Problem(n, d, c, A.data_ptr(), lda, b2.data_ptr(), ldb, float(pr["nu"]),
                           lam.data_ptr() if lam is not None else None, x.data_ptr(), c)
    o, _ = make_options(**opts)
    infos = (B.Info * len(problems))()
    h = _handle(dev)
    st = _lib().aes_solve_batched(h, _stream(dev), len(problems), arr, float(tol), ctypes.byref(o), infos)
    if st not in (B.AES_OK, B.AES_ERR_MAX_ITER):
        _check(h, st)
    return [(x.reshape(-1) if sq else x, infos[i].as_dict()) for i, (x, sq) in enumerate(outs)]


def hv(A, p, nu, lam=None):
    """(q, pHp): q = A^T (A p) + nu^2 Lambda p and pHp = ||A p||^2 + nu^2 p^T Lambda p."""
    _req(A, "A", (2,))
    A, lda = _rowmajor(A)
    n, d = A.shape
    p = _req(p, "p", (1,)).contiguous()
    lam = lam.contiguous() if lam is not None else None
    q = torch.empty(d, dtype=torch.float64, device=A.device)
    php = torch.empty(1, dtype=torch.float64, device=A.device)
    h = _handle(A.device)
    _check(h, _lib().aes_hv(h, _stream(A.device), n, d, _ptr(A), lda, float(nu), _ptr(lam), _ptr(p), _ptr(q), _ptr(php)))
    return q, php


def hv_multi(A, P, nu, lam=None, precision="fp64"):
    """Q = A^T (A P) + nu^2 Lambda P for P of shape (d, c), c a power of two <= 32."""
    _req(A, "A", (2,))
    A, lda = _rowmajor(A)
    n, d = A.shape
    P = _req(P, "P", (2,)).contiguous()
    c = P.shape[1]
    lam = lam.contiguous() if lam is not None else None
    Q = torch.empty_like(P)
    h = _handle(A.device)
    _check(h, _lib().aes_hv_multi(h, _stream(A.device), n, d, c, _ptr(A), lda, float(nu), _ptr(lam), _ptr(P), _ptr(Q),
                                  B.PRECISIONS[precision]))
    return Q


def sketch(A, m, kind="srht", seed=0, k=0, problem=0):
    """S A (m x d) for sketch index k (see include/aes.h for the random streams)."""
    _req(A, "A", (2,))
    A, lda = _rowmajor(A)
    n, d = A.shape
    SA = torch.empty((m, d), dtype=torch.float64, device=A.device)
    h = _handle(A.device)
    _check(h, _lib().aes_sketch(h, _stream(A.device), B.SKETCHES[kind], n, d, _ptr(A), lda, int(m), int(seed),
                                int(problem), int(k), _ptr(SA)))
    return SA


def factor(SA, nu, lam=None):
    """(G, L): G = SA^T SA + nu^2 Lambda (m >= d) or SA Lambda^-1 SA^T + nu^2 I (m < d), lower
    triangle, and its lower Cholesky factor."""
    SA = _req(SA, "SA", (2,)).contiguous()
    m, d = SA.shape
    dim = d if m >= d else m
    G = torch.empty((dim, dim), dtype=torch.float64, device=SA.device)
    L = torch.empty((dim, dim), dtype=torch.float64, device=SA.device)
    lam = lam.contiguous() if lam is not None else None
    h = _handle(SA.device)
    _check(h, _lib().aes_factor(h, _stream(SA.device), m, d, _ptr(SA), float(nu), _ptr(lam), _ptr(G), _ptr(L)))
    return G, L


def precond_apply(SA, nu, lam, z):
    """H_S^{-1} z for z of shape (d,) or (d, c) with c a power of two <= 32."""
    SA = _req(SA, "SA", (2,)).contiguous()
    m, d = SA.shape
    squeeze = z.dim() == 1
    z2 = _req(z, "z").reshape(d, -1).contiguous()
    c = z2.shape[1]
    v = torch.empty_like(z2)
    lam = lam.contiguous() if lam is not None else None
    h = _handle(SA.device)
    _check(h, _lib().aes_precond_apply(h, _stream(SA.device), m, d, c, _ptr(SA), float(nu), _ptr(lam), _ptr(z2),
                                       _ptr(v)))
    return v.reshape(d) if squeeze else v


class SketchSolve(torch.autograd.Function):
    """x* = argmin 1/2 x^T (A^T A + nu^2 Lambda) x - b^T x with nu = exp(log_nu).

    Forward: adaptive PCG (aes_solve_keep).  Backward: the adjoint solve H lam = dL/dx* by
    adaptive PCG reusing the forward sketch and factorisation (aes_adjoint_solve), then
    dL/db = lam, dL/dA = -(A x*) lam^T - (A lam) x*^T, dL/dlog_nu = -2 nu^2 lam^T Lambda x*.
    """

    @staticmethod
    def forward(ctx, A, b, log_nu, lam=None, opts=None):
        opts = dict(opts or {})
        tol = opts.pop("tol", 1e-10)
        A_c, lda = _rowmajor(_req(A.detach(), "A", (2,)))
        n, d = A_c.shape
        b_c = _req(b.detach(), "b", (1,)).contiguous()
        nu = float(torch.exp(log_nu.detach()).item())
        lam_c = lam.detach().contiguous() if lam is not None else None
        o, _ = make_options(**opts)
        x = torch.empty(d, dtype=torch.float64, device=A.device)
        info = B.Info()
        cptr = ctypes.c_void_p()
        h = _handle(A.device)
        st = _lib().aes_solve_keep(h, _stream(A.device), n, d, 1, _ptr(A_c), lda, _ptr(b_c), 1, nu, _ptr(lam_c),
                                   float(tol), ctypes.byref(o), _ptr(x), 1, ctypes.byref(info), ctypes.byref(cptr))
        if st not in (B.AES_OK,):
            _check(h, st)
        ctx.aes_ctx = cptr
        ctx.keep = (A_c, lam_c)
        ctx.tol = tol
        ctx.info = info.as_dict()
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        g = _req(gx.detach().to(torch.float64), "grad").contiguous()
        lamv = torch.empty_like(g)
        info = B.Info()
        lib = _lib()
        st = lib.aes_adjoint_solve(ctx.aes_ctx, _stream(g.device), _ptr(g), float(ctx.tol), _ptr(lamv),
                                   ctypes.byref(info))
        if st != B.AES_OK:
            lib.aes_ctx_free(ctx.aes_ctx)
            raise AesError(st, "adjoint solve failed")
        A_c, _ = ctx.keep
        dA = None
        if ctx.needs_input_grad[0]:
            dA = torch.empty((A_c.shape[0], A_c.shape[1]), dtype=torch.float64, device=A_c.device)
        dln = ctypes.c_double(0.0)
        st = lib.aes_grad(ctx.aes_ctx, _stream(g.device), _ptr(lamv), _ptr(dA), ctypes.byref(dln))
        lib.aes_ctx_free(ctx.aes_ctx)
        ctx.aes_ctx = None
        if st != B.AES_OK:
            raise AesError(st, "gradient kernel failed")
        dlognu = torch.tensor(dln.value, dtype=torch.float64, device=g.device)
        return dA, lamv, dlognu, None, None
