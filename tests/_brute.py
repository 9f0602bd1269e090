"""Brute-force dense assembly of the right-hand side matrix on tiny grids.

An independent code path for the oracle pins: every matrix entry is written by
explicit index loops from the 1D matrices (which are pinned on their own) and
coefficients evaluated with the math module, following the definitions:
Eq. (Liouvsph) for the operator, the DFS identities
F(-theta, phi, Theta, Phi) = F(theta, phi + pi, Theta, Phi + pi) and
F(-Theta, Phi) = F(Theta, Phi + pi) for the theta and Theta lines, the collision
term (in-scattering written out as the double sum over directions of the phase
function p(omega . omega') = c0 + c1 mu + c2 mu^2, with omega from the angles by
the math module) and the inflow mask.  Sizes are kept at a few hundred nodes.
"""

import math

import numpy as np

from oracle import grid as og


def _omega(Th, Ph):
    return (math.cos(Th), math.sin(Th) * math.cos(Ph), math.sin(Th) * math.sin(Ph))


def assemble(g, kappa=None, sigma=None, bc=True, with_L=True, dtype=float, kernel=None):
    shp = g.shape
    n = int(np.prod(shp))
    A = np.zeros((n, n), dtype=dtype)
    idx = np.arange(n).reshape(shp)
    Dr = og.cheb_diff_matrix(g.n_r, g.r_in, g.r_out)
    Dth = og.fourier_diff_matrix(2 * g.n_theta)
    Dph = og.fourier_diff_matrix(g.n_phi)
    DTh = og.fourier_diff_matrix(2 * g.n_Theta)
    DPh = og.fourier_diff_matrix(g.n_Phi)
    wT = og.fejer_weights(g.n_Theta)
    nth, nph, nTh, nPh = g.n_theta, g.n_phi, g.n_Theta, g.n_Phi
    for e in range(g.n_eps):
        for j in range(g.n_r):
            r = g.r[j]
            for l in range(nth):
                th = (l + 0.5) * math.pi / nth
                for k in range(nph):
                    kp = (k + nph // 2) % nph
                    for i in range(nTh):
                        Th = (i + 0.5) * math.pi / nTh
                        inflow = bc and ((j == 0 and math.cos(Th) > 0) or (j == g.n_r - 1 and math.cos(Th) < 0))
                        for m in range(nPh):
                            row = idx[e, j, l, k, i, m]
                            if inflow:
                                continue
                            Ph = 2 * math.pi * m / nPh
                            mp = (m + nPh // 2) % nPh
                            if with_L:
                                c_r = math.cos(Th)
                                c_th = math.sin(Th) * math.cos(Ph) / r
                                c_ph = math.sin(Th) * math.sin(Ph) / (r * math.sin(th))
                                c_Th = -math.sin(Th) / r
                                c_Ph = -math.sin(Th) * math.sin(Ph) * math.cos(th) / (r * math.sin(th))
                                for jj in range(g.n_r):
                                    A[row, idx[e, jj, l, k, i, m]] -= c_r * Dr[j, jj]
                                for q in range(2 * nth):
                                    col = idx[e, j, q, k, i, m] if q < nth else idx[e, j, 2 * nth - 1 - q, kp, i, mp]
                                    A[row, col] -= c_th * Dth[l, q]
                                for kk in range(nph):
                                    A[row, idx[e, j, l, kk, i, m]] -= c_ph * Dph[k, kk]
                                for q in range(2 * nTh):
                                    col = idx[e, j, l, k, q, m] if q < nTh else idx[e, j, l, k, 2 * nTh - 1 - q, mp]
                                    A[row, col] -= c_Th * DTh[i, q]
                                for mm in range(nPh):
                                    A[row, idx[e, j, l, k, i, mm]] -= c_Ph * DPh[m, mm]
                            if kappa is not None:
                                ka = kappa[e, j, l, k]
                                si = sigma[e, j, l, k]
                                A[row, row] -= ka + si
                                c1, c2 = kernel if kernel is not None else (0.0, 0.0)
                                c0 = 1.0 - c2 / 3.0
                                om = _omega(Th, Ph)
                                for ii in range(nTh):
                                    for mm in range(nPh):
                                        op = _omega((ii + 0.5) * math.pi / nTh, 2 * math.pi * mm / nPh)
                                        mu = om[0] * op[0] + om[1] * op[1] + om[2] * op[2]
                                        ph = c0 + c1 * mu + c2 * mu * mu
                                        A[row, idx[e, j, l, k, ii, mm]] += si * ph * wT[ii] * (2 * math.pi / nPh) / (4 * math.pi)
    return A


def source(g, eta, bc=True):
    b = np.broadcast_to(np.asarray(eta)[:, :, :, :, None, None], g.shape).copy()
    if bc:
        for i in range(g.n_Theta):
            cT = math.cos((i + 0.5) * math.pi / g.n_Theta)
            if cT > 0:
                b[:, 0, :, :, i, :] = 0
            if cT < 0:
                b[:, -1, :, :, i, :] = 0
    return b.reshape(-1)


def rk4_polys(dtA):
    """P(dtA), Q(dtA) with y1 = P y + dt Q b for y' = A y + b under classical RK4."""
    n = dtA.shape[0]
    I = np.eye(n, dtype=dtA.dtype)
    Z2 = dtA @ dtA
    Z3 = Z2 @ dtA
    Z4 = Z3 @ dtA
    P = I + dtA + Z2 / 2 + Z3 / 6 + Z4 / 24
    Q = I + dtA / 2 + Z2 / 6 + Z3 / 24
    return P, Q
