"""Seeded synthetic inputs shaped like the paper's synthetic workloads.

This module is shared by the tests, the benchmark and the oracle's callers.  It holds none of
the solver's arithmetic: it only draws A = U diag(sigma) V^T (U from the QR factorisation of
an i.i.d. N(0,1) n x d matrix, V from the QR factorisation of an i.i.d. N(0,1) d x d matrix),
the diagonal Lambda and the right-hand sides b = A^T y.  The paper's synthetic design is a
data matrix with a prescribed singular-value decay and a sweep of nu (Sec. 5); the five named
workloads below fix those choices.

Two backends draw the same recipe:
  * 'numpy' (CPU): numpy.random.default_rng(SeedSequence([210414101, tag])), PCG64, in the
    order U, V, Lambda, y, x_t; used for small cases and CPU tests;
  * 'torch' (a torch device, typically the GPU): torch.Generator seeded with the same tag; used
    for large cases so that the QR factorisations do not dominate a run.  The two backends
    give different (equally valid) draws.
"""
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 210414101


@dataclass
class Workload:
    name: str
    n: int
    d: int
    decay: str            # 'geo:<q>' sigma_j = q^j, 'pow:<p>' sigma_j = j^-p
    nu: float
    lam: str = "identity"  # 'identity' | 'uniform1_10' (1 + U[0, 9])
    nrhs: int = 1
    sketch: str = "srht"
    m_init: int = 16
    method: str = "pcg"
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    # plain adaptive PCG, FP64, geometric decay 0.9^j
    "pcg_n4096_d256": Workload("pcg_n4096_d256", 4096, 256, "geo:0.9", 1e-2, m_init=8),
    # adaptive PCG and IHS, FP64, polynomial decay 1/j, Lambda = 1 + U[0,9]
    "pcg_n65536_d2048": Workload("pcg_n65536_d2048", 65536, 2048, "pow:1", 1e-3, lam="uniform1_10", m_init=16),
    # mixed precision, geometric decay 0.995^j (the paper's synthetic spectrum)
    "mixed_n262144_d4096": Workload("mixed_n262144_d4096", 262144, 4096, "geo:0.995", 1e-2, m_init=16),
    # differentiation, polynomial decay j^-1/2
    "adjoint_n131072_d1024": Workload("adjoint_n131072_d1024", 131072, 1024, "pow:0.5", 1e-2, m_init=16),
}


def singular_values(d, decay):
    kind, val = decay.split(":")
    j = np.arange(1, d + 1, dtype=np.float64)
    if kind == "geo":
        return float(val) ** j
    if kind == "pow":
        return j ** (-float(val))
    raise ValueError(decay)


def _tag(name):
    return int.from_bytes(name.encode()[:8].ljust(8, b"\0"), "little") & 0x7FFFFFFF


def make_matrix_numpy(n, d, sigma, rng):
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    V, _ = np.linalg.qr(rng.standard_normal((d, d)))
    A = (U * sigma[None, :]) @ V.T
    return np.ascontiguousarray(A), V


def _lower_inverse(torch, L, leaf=512):
    """Inverse of a lower-triangular matrix by 2 x 2 blocks (products only; small triangular
    solves at the leaves): inv([[L11, 0], [L21, L22]]) = [[X11, 0], [-X22 L21 X11, X22]]."""
    d = L.shape[0]
    if d <= leaf:
        return torch.linalg.solve_triangular(L, torch.eye(d, device=L.device, dtype=L.dtype), upper=False)
    h = d // 2
    X11 = _lower_inverse(torch, L[:h, :h].contiguous(), leaf)
    X22 = _lower_inverse(torch, L[h:, h:].contiguous(), leaf)
    X = torch.zeros_like(L)
    X[:h, :h] = X11
    X[h:, h:] = X22
    X[h:, :h] = -(X22 @ (L[h:, :h].contiguous() @ X11))
    return X


def make_problem(n, d, decay, nu, lam="identity", nrhs=1, seed=0, backend="numpy", device=None,
                 with_xt=False, dtype=np.float64, ortho="qr"):
    """Draw one problem.  Returns a dict with A, b, nu, lam, sigma, V (and y, xt).

    backend 'numpy' returns numpy arrays; backend 'torch' returns torch tensors on `device`
    (A, b, lam, V, xt) with sigma as numpy.  ortho (torch backend): how U is made orthonormal
    from the Gaussian matrix G — 'qr' (Householder QR) or 'cholqr' (U = G R^{-1} with
    R^T R = G^T G, two large products instead of a QR; accurate for the tall Gaussian G, whose
    condition number is about (sqrt n + sqrt d) / (sqrt n - sqrt d)).
    """
    sigma = singular_values(d, decay)
    if backend == "numpy":
        rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, seed]))
        A, V = make_matrix_numpy(n, d, sigma, rng)
        if lam == "identity":
            lv = np.ones(d)
        elif lam == "uniform1_10":
            lv = 1.0 + 9.0 * rng.random(d)
        else:
            raise ValueError(lam)
        Y = rng.standard_normal((n, nrhs))
        B = A.T @ Y
        out = dict(A=A, b=B[:, 0] if nrhs == 1 else B, nu=float(nu), lam=lv, sigma=sigma, V=V,
                   y=Y[:, 0] if nrhs == 1 else Y)
        if with_xt:
            out["xt"] = rng.standard_normal(d)
        return out
    if backend == "torch":
        import torch

        dev = torch.device(device or "cuda")
        g = torch.Generator(device=dev)
        g.manual_seed(SEED_BASE * 1000003 + int(seed))
        G = torch.randn((n, d), generator=g, device=dev, dtype=torch.float64)
        if ortho == "cholqr":
            L = torch.linalg.cholesky(G.T @ G)
            Rinv = _lower_inverse(torch, L).T.contiguous()
            del L
            U = G @ Rinv
            del Rinv
        else:
            U, _ = torch.linalg.qr(G, mode="reduced")
        del G
        Gv = torch.randn((d, d), generator=g, device=dev, dtype=torch.float64)
        V, _ = torch.linalg.qr(Gv, mode="reduced")
        del Gv
        s_t = torch.as_tensor(sigma, device=dev, dtype=torch.float64)
        U.mul_(s_t[None, :])
        A = U @ V.T.contiguous()
        del U
        if lam == "identity":
            lv = torch.ones(d, device=dev, dtype=torch.float64)
        elif lam == "uniform1_10":
            lv = 1.0 + 9.0 * torch.rand(d, generator=g, device=dev, dtype=torch.float64)
        else:
            raise ValueError(lam)
        Y = torch.randn((n, nrhs), generator=g, device=dev, dtype=torch.float64)
        B = A.T @ Y
        out = dict(A=A.contiguous(), b=B[:, 0].contiguous() if nrhs == 1 else B.contiguous(), nu=float(nu),
                   lam=lv, sigma=sigma, V=V, y=Y[:, 0] if nrhs == 1 else Y)
        if with_xt:
            out["xt"] = torch.randn(d, generator=g, device=dev, dtype=torch.float64)
        return out
    raise ValueError(backend)


def make_wide_problem(n, d, decay, nu, lam="identity", nrhs=1, seed=0, backend="numpy", device=None):
    """A problem with n < d (the dual form's shape, e.g. the paper's OVA-Lung n = 1545,
    d = 10936): A is the transpose of the matrix ``make_problem`` draws at d x n, so its n
    singular values follow ``decay``; Lambda (length d) and b = A^T y with y ~ N(0, I_n) are drawn
    afterwards.  Returns a dict with A (n x d), b, nu, lam, sigma, y."""
    if n > d:
        raise ValueError("make_wide_problem needs n <= d")
    if lam not in ("identity", "uniform1_10"):
        raise ValueError(lam)
    P = make_problem(d, n, decay, nu, "identity", 1, seed, backend, device)
    if backend == "numpy":
        A = np.ascontiguousarray(P["A"].T)
        rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, seed, 1]))
        lv = np.ones(d) if lam == "identity" else 1.0 + 9.0 * rng.random(d)
        Y = rng.standard_normal((n, nrhs))
        B = A.T @ Y
    else:
        import torch

        A = P["A"].T.contiguous()
        del P["A"]
        g = torch.Generator(device=A.device)
        g.manual_seed(SEED_BASE * 1000003 + int(seed) + 7919)
        lv = (torch.ones(d, device=A.device, dtype=torch.float64) if lam == "identity"
              else 1.0 + 9.0 * torch.rand(d, generator=g, device=A.device, dtype=torch.float64))
        Y = torch.randn((n, nrhs), generator=g, device=A.device, dtype=torch.float64)
        B = (A.T @ Y).contiguous()
    return dict(A=A, b=B[:, 0] if nrhs == 1 else B, nu=float(nu), lam=lv, sigma=P["sigma"],
                y=Y[:, 0] if nrhs == 1 else Y)


def make_workload(name, seed=0, backend="numpy", device=None, **kw):
    w = WORKLOADS[name]
    return make_problem(w.n, w.d, w.decay, w.nu, w.lam, w.nrhs, seed=seed, backend=backend, device=device, **kw)


def batched_specs(count=64, seed=0):
    """Sizes and nu of the batched workload: n = 256*U{32..512}, d = 256*U{1..8},
    nu log-uniform in [1e-4, 1e-1], sigma_j = 0.98^j, Lambda = I, 32 right-hand sides."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 3, seed]))
    ns = 256 * rng.integers(32, 513, size=count)
    ds = 256 * rng.integers(1, 9, size=count)
    nus = 10.0 ** rng.uniform(-4, -1, size=count)
    return [dict(n=int(n), d=int(d), nu=float(v), decay="geo:0.98", nrhs=32) for n, d, v in zip(ns, ds, nus)]
