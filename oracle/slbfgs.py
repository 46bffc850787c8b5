"""Stochastic limited-memory BFGS of App. D (Algorithm 2) — plain NumPy.

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see oracle/__init__.py).

Minimises an energy J(u) given only an estimator g(u, i) -> (F, G) of
(J(u), grad J(u)) whose stochastic approximation is fixed by the index i.
The method is built from three parts:

* ``LbfgsMemory``: the last m_h curvature pairs (s, y) and the product of
  their L-BFGS inverse Hessian with a vector, initial matrix h0 I (Nocedal &
  Wright, Numerical Optimization, 2nd ed., Algorithm 7.4).  The paper gives
  the initial matrix as an input; a scalar multiple of the identity is the
  reading here.
* ``quasi_newton_step``: one step with a fixed approximation i.  Both
  estimator calls of the step use the same i, so the pair they produce
  (the step taken and the change of the gradient) is consistent; the pair
  enters the memory before the direction is corrected with the gradient at
  the trial point.  No line search: the step length is nu.
* ``IterateAverage``: the returned estimate, the plain iterate until the
  energy estimate first increases, afterwards the running mean of the later
  iterates weighted by w(i) (the paper: i^3).

``slbfgs`` composes them with the projection onto [u_min, u_max] and the
energy estimate min(F at u, F at the trial point) of each step.
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


class LbfgsMemory:
    """The last m_h pairs (s, y), oldest first, and H v for their L-BFGS
    inverse Hessian with H_0 = h0 I."""

    def __init__(self, m_h: int, h0: float):
        self.m_h = int(m_h)
        self.h0 = float(h0)
        self.S: List[np.ndarray] = []
        self.Y: List[np.ndarray] = []

    def push(self, s: np.ndarray, y: np.ndarray) -> None:
        self.S.append(np.asarray(s, dtype=np.float64))
        self.Y.append(np.asarray(y, dtype=np.float64))
        if len(self.S) > self.m_h:
            del self.S[0], self.Y[0]

    def apply(self, v: np.ndarray) -> np.ndarray:
        return two_loop(v, self.S, self.Y, self.h0)


def quasi_newton_step(g: Callable[[np.ndarray, int], Tuple[float, np.ndarray]], u: np.ndarray, i: int,
                      memory: LbfgsMemory, nu: float) -> Tuple[np.ndarray, float]:
    """One stochastic quasi-Newton step of length nu with approximation i of
    the estimator (App. D): the quasi-Newton direction d = -H G at u, the
    estimator at the trial point u + nu d, the pair (nu d, G_trial - G) added
    to the memory, the direction corrected by -H G_trial with the updated
    memory.  Returns (u + nu d before any projection, min of the two energy
    values)."""
    F_at_u, G_at_u = g(u, i)
    d = -memory.apply(G_at_u)
    F_trial, G_trial = g(u + nu * d, i)
    memory.push(nu * d, np.asarray(G_trial, dtype=np.float64) - np.asarray(G_at_u, dtype=np.float64))
    d = d - memory.apply(G_trial)
    return u + nu * d, min(F_at_u, F_trial)


class IterateAverage:
    """Estimate returned after each step: the iterate itself until the energy
    estimate increases for the first time, then the w(i)-weighted mean of the
    iterates of the following steps (App. D)."""

    def __init__(self, weight: Callable[[int], float]):
        self.weight = weight
        self.on = False
        self.total = None
        self.wsum = 0.0
        self.J_last = np.inf

    def update(self, i: int, u: np.ndarray, J: float) -> np.ndarray:
        if self.on:
            wi = self.weight(i)
            self.total = wi * u if self.total is None else self.total + wi * u
            self.wsum += wi
            est = self.total / self.wsum
        else:
            self.on = J > self.J_last
            est = u.copy()
        self.J_last = J
        return est


def slbfgs(g: Callable[[np.ndarray, int], Tuple[float, np.ndarray]], u0: np.ndarray, *, nu: float,
           n_evals: int, m_h: int = 64, h0: float = 1.0, u_min=-np.inf, u_max=np.inf,
           weight: Callable[[int], float] = lambda i: float(i) ** 3, history: bool = False):
    """Algorithm 2 without line search: steps i = 1, 2, ... until n_evals
    estimator calls (two per step) are spent.  Returns (u_hat, [J_i][, the
    estimate after each step])."""
    u = np.array(u0, dtype=np.float64)
    memory = LbfgsMemory(m_h, h0)
    average = IterateAverage(weight)
    Js, its = [], []
    u_hat = u.copy()
    i = 0
    while 2 * i < n_evals:
        i += 1
        u, J = quasi_newton_step(g, u, i, memory, nu)
        u = np.maximum(np.minimum(u, u_max), u_min)
        u_hat = average.update(i, u, J)
        Js.append(J)
        if history:
            its.append(u_hat.copy())
    return (u_hat, Js, its) if history else (u_hat, Js)
