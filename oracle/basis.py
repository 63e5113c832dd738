"""Reference-element operators on Legendre-Gauss-Lobatto points (oracle).

Paper: Sec. Methodology, Eqs. lagrange_3d, lag (Lagrange basis on GLL
points), divergenc_quadrature (GLL quadrature), fluxes_discrete_strong
(derivative matrix), sbp and boundary_matrix.

Reading of garbled passages:
* Eq. sbp as printed is not an SBP identity under any index convention; the
  property used is  w_n D_nj + w_j D_jn = B_nj  with B = diag(-1, 0.., +1).
* The derivative at node n is sum_j D_nj F_j with D_nj = l_j'(xi_n)
  (row = evaluation node), which is the matrix of Eq. DGvec.
"""
import numpy as np


def legendre(n, x):
    """P_n(x) and P_n'(x) by the three-term recurrence."""
    x = np.asarray(x)
    if x.dtype.kind != "f":
        x = x.astype(float)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    d0 = np.zeros_like(x)
    d1 = np.ones_like(x)
    for k in range(2, n + 1):
        p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        d2 = d0 + (2 * k - 1) * p1
        p0, p1 = p1, p2
        d0, d1 = d1, d2
    return p1, d1


def lgl(N, dtype=np.float64):
    """LGL nodes (ascending) and weights for polynomial degree N.

    Nodes: -1, +1 and the N-1 roots of P_N', found by Newton's method on
    P_N' started from Chebyshev-Gauss-Lobatto points.  Weights:
    w_j = 2 / (N (N+1) P_N(xi_j)^2).  ``dtype`` (float64 or longdouble) is
    the precision of the iteration and the result.
    """
    x = -np.cos(np.pi * np.arange(N + 1, dtype=dtype) / N)
    inner = x[1:-1].copy()
    for _ in range(100):
        _, dp = legendre(N, inner)
        # P_N'' from the Legendre ODE: (1-x^2) P'' = 2x P' - N(N+1) P
        p, _ = legendre(N, inner)
        d2 = (2 * inner * dp - N * (N + 1) * p) / (1 - inner * inner)
        step = dp / d2
        inner = inner - step
        if np.max(np.abs(step)) < 1e-16:
            break
    x = np.concatenate((np.array([-1.0], dtype), inner, np.array([1.0], dtype)))
    p, _ = legendre(N, x)
    w = 2.0 / (N * (N + 1) * p * p)
    return x, w


def barycentric_weights(x):
    n = len(x)
    lam = np.ones(n, x.dtype)
    for j in range(n):
        for k in range(n):
            if k != j:
                lam[j] /= (x[j] - x[k])
    return lam


def derivative_matrix(x):
    """D_nj = l_j'(x_n) by the barycentric formula; diagonal = -sum of row."""
    lam = barycentric_weights(x)
    n = len(x)
    D = np.zeros((n, n), x.dtype)
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = lam[j] / lam[i] / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, np.arange(n) != i])
    return D


def interpolation_matrix(x, y):
    """I_ij = l_j(y_i): values at points y of the Lagrange basis on nodes x."""
    n = len(x)
    I = np.ones((len(y), n))
    for j in range(n):
        for k in range(n):
            if k != j:
                I[:, j] *= (y - x[k]) / (x[j] - x[k])
    return I


def legendre_vandermonde(x):
    """V_ij = phi_j(x_i) with orthonormal Legendre phi_j = sqrt((2j+1)/2) P_j."""
    n = len(x)
    V = np.zeros((n, n), x.dtype)
    for j in range(n):
        p, _ = legendre(j, x)
        V[:, j] = np.sqrt(x.dtype.type((2 * j + 1) / 2.0)) * p
    return V


def gauss_legendre(n):
    """n-point Gauss-Legendre rule (roots of P_n by Newton)."""
    x = -np.cos(np.pi * (np.arange(n) + 0.75) / (n + 0.5))
    for _ in range(100):
        p, dp = legendre(n, x)
        step = p / dp
        x = x - step
        if np.max(np.abs(step)) < 1e-16:
            break
    _, dp = legendre(n, x)
    w = 2.0 / ((1 - x * x) * dp * dp)
    return x, w


def inverse(A):
    """Matrix inverse in A's precision: LAPACK in float64, then Newton-Schulz
    refinement X <- X (2I - A X) (quadratic) for extended precision, which
    LAPACK does not offer."""
    X = np.linalg.inv(A.astype(np.float64)).astype(A.dtype)
    if A.dtype != np.float64:
        I2 = 2 * np.eye(A.shape[0], dtype=A.dtype)
        for _ in range(3):
            X = X @ (I2 - A @ X)
    return X


class Basis:
    """Everything the oracle needs for one polynomial degree N, in float64
    or, for rounding studies, in extended precision (np.longdouble)."""

    def __init__(self, N, dtype=np.float64):
        self.N = N
        self.n1 = N + 1
        self.dtype = dtype
        self.xi, self.w = lgl(N, dtype)
        self.D = derivative_matrix(self.xi)
        self.V = legendre_vandermonde(self.xi)
        self.Vinv = inverse(self.V)
