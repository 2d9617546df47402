"""Two-grid local Fourier analysis (LFA) for red-black Gauss-Seidel with
full-weighting restriction and (bi/tri)linear interpolation on the 5-/7-point
Laplacian.  Test-only: it pins the convergence factor the oracle's V-cycle
must show, independently of the oracle's code.

Method (Trottenberg, Oosterlee, Schueller, "Multigrid", Sec. 4, cited by the
paper for its multigrid background): a low frequency theta in [-pi/2, pi/2)^d
couples with its 2^d harmonics theta + pi*alpha, alpha in {0,1}^d.  All
operators become 2^d x 2^d matrices on that space:

  A_hat        = diag( sum_i (2 - 2 cos th_i) / h^2 )
  Jacobi       = diag( (1/d) sum_i cos th_i )                (omega = 1)
  colour masks = (I +- Pi)/2, Pi swapping theta <-> theta + pi*(1..1)
                 (the red/black indicator is (1 +- (-1)^{sum of indices})/2)
  red half-sweep   S_r = E_black + E_red * Jacobi
  black half-sweep S_b = E_red + E_black * Jacobi
  FW restriction   R_hat[alpha] = prod_i (1 + cos th^alpha_i) / 2
  interpolation    P_hat = R_hat^T (linear interpolation of a coarse mode)
  coarse operator  Ac_hat = sum_i (2 - 2 cos 2 th_i) / (2h)^2
  two-grid         M = (S_r S_b)^nu2 (I - P_hat Ac^-1 R_hat A_hat) (S_b S_r)^nu1
"""
from __future__ import annotations

import itertools

import numpy as np


def _harmonics(d):
    return [np.array(a, dtype=float) for a in itertools.product((0, 1), repeat=d)]


def two_grid_matrix(theta, nu1, nu2, h=1.0, smoother="rbgs", omega=1.0):
    theta = np.asarray(theta, dtype=float)
    d = theta.size
    alphas = _harmonics(d)
    nh = len(alphas)
    ths = [theta + np.pi * a for a in alphas]
    Ahat = np.diag([np.sum(2 - 2 * np.cos(t)) / h ** 2 for t in ths])
    jac = np.diag([np.mean(np.cos(t)) for t in ths])
    # permutation alpha -> alpha xor (1,...,1)
    Pi = np.zeros((nh, nh))
    for i, a in enumerate(alphas):
        b = 1 - a
        j = next(q for q, c in enumerate(alphas) if np.array_equal(c, b))
        Pi[j, i] = 1.0
    I = np.eye(nh)
    Ered, Eblack = 0.5 * (I + Pi), 0.5 * (I - Pi)
    if smoother == "rbgs":
        Sr = Eblack + Ered @ jac
        Sb = Ered + Eblack @ jac
        pre = Sb @ Sr
        post = Sr @ Sb
    else:  # weighted Jacobi
        pre = post = (1 - omega) * I + omega * jac
    Rhat = np.array([[np.prod((1 + np.cos(t)) / 2) for t in ths]])
    Phat = Rhat.T
    Ac = np.sum(2 - 2 * np.cos(2 * theta)) / (2 * h) ** 2
    K = I - Phat @ Rhat @ Ahat / Ac
    return np.linalg.matrix_power(post, nu2) @ K @ np.linalg.matrix_power(pre, nu1)


def two_grid_factor(d, nu1, nu2, n=64, smoother="rbgs", omega=1.0):
    """max over low frequencies (theta != 0) of the spectral radius."""
    grid = -np.pi / 2 + np.pi * (np.arange(n) + 0.5) / n  # avoids theta = 0 exactly
    rho = 0.0
    for th in itertools.product(grid, repeat=d):
        M = two_grid_matrix(np.array(th), nu1, nu2, smoother=smoother, omega=omega)
        rho = max(rho, float(np.max(np.abs(np.linalg.eigvals(M)))))
    return rho


def smoothing_factor_jacobi(d, omega, n=256):
    """max over high frequencies of |1 - omega + omega * mean(cos th)|."""
    grid = -np.pi + 2 * np.pi * (np.arange(n) + 0.5) / n
    mu = 0.0
    for th in itertools.product(grid, repeat=d):
        th = np.array(th)
        if np.all(np.abs(th) < np.pi / 2):
            continue
        mu = max(mu, abs(1 - omega + omega * np.mean(np.cos(th))))
    return mu
