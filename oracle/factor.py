"""Cached factorisation of the sketched Hessian H_S = (SA)^T SA + nu^2 Lambda.

Test infrastructure only.  Follows Sec. 4.1 ("Sketching and factorization costs"):

* m >= d: form H_S (d x d) and its Cholesky factor L; H_S v = z is two triangular solves.
* m <  d: form W_S = SA Lambda^{-1} (SA)^T + nu^2 I_m (m x m) and its Cholesky factor L_W;
  by the Woodbury identity v = (Lambda^{-1}/nu^2) (z - (SA)^T W_S^{-1} SA Lambda^{-1} z).

The branch at m == d is the Cholesky of H_S (the paper's "m >= d").
Pins (tests/test_oracle_factor.py): L L^T == H_S; apply(z) == numpy.linalg.solve of the
explicitly formed H_S for both branches (the Woodbury identity).
"""
import numpy as np
import scipy.linalg as sla


class NotSPDError(np.linalg.LinAlgError):
    pass


class SketchedHessian:
    """Factorisation of H_S for one sketch SA (m x d)."""

    def __init__(self, SA, nu, lam):
        SA = np.asarray(SA, dtype=np.float64)
        self.m, self.d = SA.shape
        self.nu = float(nu)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.SA = SA
        self.woodbury = self.m < self.d
        try:
            if not self.woodbury:
                G = SA.T @ SA + (self.nu ** 2) * np.diag(self.lam)
                self.L = np.linalg.cholesky(G)
            else:
                W = (SA / self.lam[None, :]) @ SA.T + (self.nu ** 2) * np.eye(self.m)
                self.L = np.linalg.cholesky(W)
        except np.linalg.LinAlgError as e:
            raise NotSPDError(str(e)) from e

    def matrix(self):
        """H_S formed explicitly (for tests)."""
        return self.SA.T @ self.SA + (self.nu ** 2) * np.diag(self.lam)

    def apply(self, z):
        """v = H_S^{-1} z for z of shape (d,) or (d, c)."""
        z = np.asarray(z, dtype=np.float64)
        if not self.woodbury:
            y = sla.solve_triangular(self.L, z, lower=True)
            return sla.solve_triangular(self.L.T, y, lower=False)
        lam = self.lam if z.ndim == 1 else self.lam[:, None]
        u = self.SA @ (z / lam)
        w = sla.solve_triangular(self.L, u, lower=True)
        w = sla.solve_triangular(self.L.T, w, lower=False)
        return (z - self.SA.T @ w) / (lam * self.nu ** 2)
