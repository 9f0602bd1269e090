"""Oracle grid: collocation nodes, 1D differentiation matrices, quadrature weights.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper expands F in Chebyshev polynomials in r and (for this hot path)
Fourier modes in the angles (Sect. 5.1); here the same bases are used in
nodal (collocation) form, so each 1D derivative is a dense N x N matrix.

Pins (tests/test_oracle_grid.py): exactness of the Chebyshev matrix on
polynomials (checked against numpy.polynomial.chebyshev), exactness of the
Fourier matrix on trigonometric polynomials (checked against numpy.fft),
textbook values of the 3-point Chebyshev matrix and of the Clenshaw-Curtis
and Fejer weights (tests/golden/), quadrature exactness on monomials.
"""

from dataclasses import dataclass, field

import numpy as np


def cgl_nodes(n_r, r_in, r_out):
    """Chebyshev-Gauss-Lobatto nodes in ascending order on [r_in, r_out].

    x_j = -cos(pi j / (n_r - 1)), r_j = (r_in + r_out)/2 + (r_out - r_in)/2 x_j,
    so r_0 = r_in and r_{n_r-1} = r_out (the shell of Sect. 4.1, R1 <= r <= R2).
    """
    j = np.arange(n_r)
    x = -np.cos(np.pi * j / (n_r - 1))
    return 0.5 * (r_in + r_out) + 0.5 * (r_out - r_in) * x


def cheb_diff_matrix(n_r, r_in, r_out):
    """Chebyshev-Gauss-Lobatto collocation derivative on [r_in, r_out].

    Off-diagonal: D_ij = (c_i / c_j) (-1)^(i+j) / (x_i - x_j), c_0 = c_N = 2,
    other c = 1 (the standard collocation matrix of the Chebyshev basis; the
    same formula holds for ascending nodes).  The node differences are taken
    in the trigonometric form x_i - x_j = 2 sin(pi (i+j)/(2N)) sin(pi (i-j)/(2N))
    to avoid cancellation, and the diagonal is minus the off-diagonal row sum,
    so D applied to a constant is exactly 0.  The result is scaled by
    dx/dr = 2 / (r_out - r_in).
    """
    n = n_r - 1
    c = np.ones(n_r)
    c[0] = 2.0
    c[-1] = 2.0
    D = np.zeros((n_r, n_r))
    for i in range(n_r):
        for k in range(n_r):
            if i != k:
                dx = 2.0 * np.sin(np.pi * (i + k) / (2 * n)) * np.sin(np.pi * (i - k) / (2 * n))
                D[i, k] = (c[i] / c[k]) * (-1.0) ** (i + k) / dx
    for i in range(n_r):
        D[i, i] = -(D[i, :].sum() - D[i, i])
    return D * (2.0 / (r_out - r_in))


def fourier_diff_matrix(n):
    """Periodic Fourier collocation derivative on n equispaced points (n even).

    D_jk = 0.5 (-1)^(j-k) cot((x_j - x_k)/2) for j != k, D_jj = 0, with
    x_j - x_k = 2 pi (j - k)/n.  The matrix is circulant and antisymmetric and
    gives the exact derivative of every trigonometric polynomial of degree
    below n/2; the Nyquist mode is mapped to zero.  Being shift invariant, the
    same matrix serves the half-shifted DFS lines.
    """
    if n % 2:
        raise ValueError("Fourier line length must be even")
    D = np.zeros((n, n))
    h = 2.0 * np.pi / n
    for j in range(n):
        for k in range(n):
            if j != k:
                D[j, k] = 0.5 * (-1.0) ** (j - k) / np.tan(0.5 * (j - k) * h)
    return D


def fejer_weights(n):
    """Fejer's first rule on mu_i = cos(t_i), t_i = (i + 1/2) pi / n.

    w_i = (2/n) [1 - 2 sum_{k=1}^{floor(n/2)} cos(2 k t_i) / (4 k^2 - 1)],
    sum w_i = 2, exact for polynomials in mu of degree <= n - 1.
    Used for the angular integrals over sin(Theta) dTheta and sin(theta)
    dtheta (App. A, Eqs. Npho and Flux; the paper itself gives no rule).
    """
    t = (np.arange(n) + 0.5) * np.pi / n
    w = np.ones(n)
    for k in range(1, n // 2 + 1):
        w -= 2.0 * np.cos(2.0 * k * t) / (4.0 * k * k - 1.0)
    return w * (2.0 / n)


def clenshaw_curtis_weights(n_r):
    """Clenshaw-Curtis weights on the n_r Chebyshev-Gauss-Lobatto nodes of [-1, 1].

    Written from the cosine-series form: with N = n_r - 1 and t_j = pi j / N,
    w_j = (c_j / N) [1 - sum_{k=1}^{floor(N/2)} b_k cos(2 k t_j) / (4 k^2 - 1)],
    c_0 = c_N = 1, other c_j = 2; b_k = 1 when 2k = N, else 2.
    Exact for polynomials of degree <= N.  Symmetric, so the ascending order
    used for r needs no re-ordering.
    """
    N = n_r - 1
    t = np.pi * np.arange(n_r) / N
    w = np.ones(n_r)
    for k in range(1, N // 2 + 1):
        b = 1.0 if 2 * k == N else 2.0
        w -= b * np.cos(2.0 * k * t) / (4.0 * k * k - 1.0)
    c = np.full(n_r, 2.0)
    c[0] = 1.0
    c[-1] = 1.0
    return w * c / N


@dataclass
class Grid:
    """The doubly spherical grid (r, theta, phi) x (Theta, Phi) x eps (Sect. 4.1).

    Array layout everywhere: [eps][r][theta][phi][Theta][Phi], C order.
    """

    n_eps: int
    n_r: int
    n_theta: int
    n_phi: int
    n_Theta: int
    n_Phi: int
    r_in: float = 1.0
    r_out: float = 3.0
    r: np.ndarray = field(init=False)
    theta: np.ndarray = field(init=False)
    phi: np.ndarray = field(init=False)
    Theta: np.ndarray = field(init=False)
    Phi: np.ndarray = field(init=False)
    D_r: np.ndarray = field(init=False)
    D_theta: np.ndarray = field(init=False)  # 2 n_theta DFS line
    D_phi: np.ndarray = field(init=False)
    D_Theta: np.ndarray = field(init=False)  # 2 n_Theta DFS line
    D_Phi: np.ndarray = field(init=False)
    w_Theta: np.ndarray = field(init=False)  # Fejer in cos(Theta)
    w_theta: np.ndarray = field(init=False)  # Fejer in cos(theta)
    w_r: np.ndarray = field(init=False)  # Clenshaw-Curtis in r (dr)

    def __post_init__(self):
        if self.n_r < 3 or self.n_theta < 1 or self.n_Theta < 1:
            raise ValueError("grid too small")
        if self.n_phi % 2 or self.n_Phi % 2:
            raise ValueError("n_phi and n_Phi must be even")
        self.r = cgl_nodes(self.n_r, self.r_in, self.r_out)
        self.theta = (np.arange(self.n_theta) + 0.5) * np.pi / self.n_theta
        self.phi = 2.0 * np.pi * np.arange(self.n_phi) / self.n_phi
        self.Theta = (np.arange(self.n_Theta) + 0.5) * np.pi / self.n_Theta
        self.Phi = 2.0 * np.pi * np.arange(self.n_Phi) / self.n_Phi
        self.D_r = cheb_diff_matrix(self.n_r, self.r_in, self.r_out)
        self.D_theta = fourier_diff_matrix(2 * self.n_theta)
        self.D_phi = fourier_diff_matrix(self.n_phi)
        self.D_Theta = fourier_diff_matrix(2 * self.n_Theta)
        self.D_Phi = fourier_diff_matrix(self.n_Phi)
        self.w_Theta = fejer_weights(self.n_Theta)
        self.w_theta = fejer_weights(self.n_theta)
        self.w_r = 0.5 * (self.r_out - self.r_in) * clenshaw_curtis_weights(self.n_r)

    @property
    def shape(self):
        return (self.n_eps, self.n_r, self.n_theta, self.n_phi, self.n_Theta, self.n_Phi)

    @property
    def size(self):
        return int(np.prod(self.shape))

    def mesh(self):
        """Broadcastable node arrays (r, theta, phi, Theta, Phi) of rank 6."""
        r = self.r[None, :, None, None, None, None]
        th = self.theta[None, None, :, None, None, None]
        ph = self.phi[None, None, None, :, None, None]
        Th = self.Theta[None, None, None, None, :, None]
        Ph = self.Phi[None, None, None, None, None, :]
        return r, th, ph, Th, Ph

    def dt_default(self):
        """0.2 times the smallest radial spacing, r_1 - r_0."""
        return 0.2 * (self.r[1] - self.r[0])


def make_grid(n_eps, n_r, n_theta, n_phi, n_Theta, n_Phi, r_in=1.0, r_out=3.0):
    return Grid(n_eps, n_r, n_theta, n_phi, n_Theta, n_Phi, r_in, r_out)
