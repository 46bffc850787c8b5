"""Stochastic limited-memory BFGS of App. D (Algorithm 2) — plain NumPy.

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see oracle/__init__.py).

Minimises an energy J(u) given only an estimator g(u, i) -> (F, G) of
(J(u), grad J(u)) whose stochastic approximation is fixed by the iteration
index i (both evaluations of one iteration use the same approximation, so
that the curvature pair (s, y) they produce is consistent).  Per iteration:

    F_u, G_u <- g(u, i)
    z   <- -H_k G_u                                (two-loop recursion)
    F_z, G_z <- g(u + nu z, i)                     (no line search)
    S <- [S, nu z], Y <- [Y, G_z - G_u]            (keep the last m_h pairs)
    z   <- z - H_k G_z                             (with the updated pairs)
    u   <- clip(u + nu z, u_min, u_max)            (projection)
    J_i <- min(F_u, F_z)
    averaging of the iterates with weights w(i) (paper: i^3), switched on
    after the first increase of the energy estimate J_i > J_{i-1}; the
    returned estimate is the weighted average once it is on, else u.

H_k is the L-BFGS inverse Hessian of the stored pairs with the initial
matrix H_0 = h0 I (Nocedal & Wright, Numerical Optimization, 2nd ed.,
Algorithm 7.4).  The paper gives H_0 as an input; h0 is that input here
(parity reading: a scalar multiple of the identity).
"""

from __future__ import annotations

from typing import Callable, List, Tuple

import numpy as np


def two_loop(g: np.ndarray, S: List[np.ndarray], Y: List[np.ndarray], h0: float) -> np.ndarray:
    """H g for the L-BFGS inverse Hessian of the pairs (S[j], Y[j]), oldest
    first, with H_0 = h0 I (Nocedal & Wright Algorithm 7.4)."""
    q = np.array(g, dtype=np.float64)
    m = len(S)
    rho = [1.0 / float(np.dot(Y[j], S[j])) for j in range(m)]
    alpha = [0.0] * m
    for j in range(m - 1, -1, -1):
        alpha[j] = rho[j] * float(np.dot(S[j], q))
        q = q - alpha[j] * Y[j]
    r = h0 * q
    for j in range(m):
        beta = rho[j] * float(np.dot(Y[j], r))
        r = r + (alpha[j] - beta) * S[j]
    return r


def dense_inverse_hessian(S, Y, h0: float, n: int) -> np.ndarray:
    """The same operator as an explicit matrix, from the BFGS update
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T applied to H_0 = h0 I
    for the pairs in order (textbook form; used only by the pins)."""
    H = h0 * np.eye(n)
    I = np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / float(np.dot(y, s))
        V = I - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


def slbfgs(g: Callable[[np.ndarray, int], Tuple[float, np.ndarray]], u0: np.ndarray, *, nu: float,
           n_evals: int, m_h: int = 64, h0: float = 1.0, u_min=-np.inf, u_max=np.inf,
           weight: Callable[[int], float] = lambda i: float(i) ** 3, history: bool = False):
    """Algorithm 2 without line search.  Returns (u_hat, J_list[, iterates])."""
    u = np.array(u0, dtype=np.float64)
    u_bar = np.zeros_like(u)
    w_bar = 0.0
    J_prev = np.inf
    S: List[np.ndarray] = []
    Y: List[np.ndarray] = []
    averaging = False
    n_evl = 0
    i = 0
    Js = []
    u_hat = u.copy()
    its = []
    while n_evl < n_evals:
        i += 1
        F_u, G_u = g(u, i)
        n_evl += 1
        z = -two_loop(G_u, S, Y, h0)
        F_z, G_z = g(u + nu * z, i)
        n_evl += 1
        S.append(nu * z)
        Y.append(np.asarray(G_z, dtype=np.float64) - np.asarray(G_u, dtype=np.float64))
        if len(S) > m_h:
            S.pop(0)
            Y.pop(0)
        z = z - two_loop(G_z, S, Y, h0)
        u = u + nu * z
        u = np.maximum(np.minimum(u, u_max), u_min)
        J_i = min(F_u, F_z)
        if averaging:
            u_bar = u_bar + weight(i) * u
            w_bar = w_bar + weight(i)
            u_hat = u_bar / w_bar
        else:
            if J_i > J_prev:
                averaging = True
            u_hat = u.copy()
        J_prev = J_i
        Js.append(J_i)
        if history:
            its.append(u_hat.copy())
    return (u_hat, Js, its) if history else (u_hat, Js)
