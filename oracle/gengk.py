"""Generalized Golub-Kahan bidiagonalization (Algorithm 1) and the genHyBR
projected solve (Sec. 3.2).

Test infrastructure only (see ``oracle/__init__``).

Problem (eq. eqv_opt1): w_hat = argmin (1/tau^2)||A Sigma w - b||^2 +
(1/sigma^2)||w||_Sigma^2, x_hat = Sigma w_hat.  Algorithm 1 builds U_{k+1},
V_k and the lower-bidiagonal B_k with (eq. exact_arith)
    A Sigma V_k = U_{k+1} B_k,  U^T U = tau^2 I,  V^T Sigma V = I.

Reading of a typo: Algorithm 1 writes the u-normalisation with a 1/tau^2
factor, but its first step uses ||b||/tau and eq. exact_arith requires
U^T U = tau^2 I; both hold only if every beta is the 2-norm divided by tau.
That reading is used here.

Posterior covariance (Sec. 3.5 and the appendix, eq. bgamma_approx):
Gamma = (Sigma^{-1}/sigma^2 + A^T A/tau^2)^{-1} is approximated from the same
bidiagonalization as sigma^2 (Sigma - Z_k Delta_k Z_k^T), Z_k = Sigma V_k W_k,
B_k^T B_k = W_k Theta_k W_k^T.  Reading of a garbled factor: the text gives
Delta_k = (I + lambda^{-2} Theta_k)^{-1}; the form that reproduces Gamma
exactly once the Krylov space is complete (k = p) is
Delta_k = (I + lambda^2 Theta_k^{-1})^{-1} = Theta_k (Theta_k + I/sigma^2)^{-1},
lambda^2 = 1/sigma^2, and that is the one used here.

Projected problem (eq. xhat_est): z_k = (B_k^T B_k + I/sigma^2)^{-1} B_k^T beta_1 e_1,
x_k* = Sigma V_k z_k, and the quadratic term x^T Sigma^{-1} x ~ ||z_k||^2.
The minimum value (1/tau^2)||A x - b||^2 + (1/sigma^2) x^T Sigma^{-1} x
equals ||B_k z_k - beta_1 e_1||^2 + ||z_k||^2/sigma^2 in exact arithmetic.
"""
import numpy as np


def gengk(A, Sigma, b, tau2, k, reorth=False):
    """k steps of Algorithm 1 with dense A (p x n) and Sigma (n x n).

    Returns beta1, U (p x (k+1)), V (n x k), B (k+1 x k), alphas, betas.
    """
    tau = np.sqrt(tau2)
    b = np.asarray(b, dtype=np.float64)
    beta1 = np.linalg.norm(b) / tau
    u = b / beta1
    t = A.T @ u / tau2
    alpha = np.sqrt(t @ Sigma @ t)
    v = t / alpha
    U, V, al, be = [u], [v], [alpha], [beta1]
    for i in range(k):
        s = A @ (Sigma @ V[-1]) - al[-1] * U[-1]
        if reorth:
            Um = np.array(U).T
            s = s - Um @ (Um.T @ s) / tau2
        beta = np.linalg.norm(s) / tau
        u = s / beta
        t = A.T @ u / tau2 - beta * V[-1]
        if reorth:
            Vm = np.array(V).T
            t = t - Vm @ (Vm.T @ (Sigma @ t))
        alpha = np.sqrt(t @ Sigma @ t)
        U.append(u)
        be.append(beta)
        if i < k - 1:
            v = t / alpha
            V.append(v)
            al.append(alpha)
    U = np.array(U).T
    V = np.array(V).T
    B = np.zeros((k + 1, k))
    for i in range(k):
        B[i, i] = al[i]
        B[i + 1, i] = be[i + 1]
    return beta1, U, V, B, np.array(al), np.array(be)


def projected_solve(B, beta1, sigma2):
    """z_k of eq. xhat_est and the projected objective value
    ||B z - beta1 e1||^2 + ||z||^2 / sigma^2."""
    k = B.shape[1]
    e1 = np.zeros(B.shape[0])
    e1[0] = beta1
    z = np.linalg.solve(B.T @ B + np.eye(k) / sigma2, B.T @ e1)
    J = float(np.sum((B @ z - e1) ** 2) + z @ z / sigma2)
    return z, J


def gengk_solve(A, Sigma, b, sigma2, tau2, k, reorth=False):
    """x_k* on every cell and the quadratic value J (Sec. 3.2)."""
    beta1, U, V, B, _, _ = gengk(A, Sigma, b, tau2, k, reorth=reorth)
    z, J = projected_solve(B, beta1, sigma2)
    x = Sigma @ (V @ z)
    return x, J, z


def posterior_variance(A, Sigma, b, sigma2, tau2, k, reorth=True):
    """Diagonal of the low-rank posterior covariance of eq. bgamma_approx
    (with the Delta_k reading in the module docstring) over every cell:
    var x_i = sigma2 (Sigma_ii - sum_j Z_ij^2 Delta_j)."""
    beta1, U, V, B, _, _ = gengk(A, Sigma, b, tau2, k, reorth=reorth)
    theta, W = np.linalg.eigh(B.T @ B)
    Z = Sigma @ V @ W
    delta = theta / (theta + 1.0 / sigma2)
    return sigma2 * (np.diag(Sigma) - (Z * Z) @ delta)
