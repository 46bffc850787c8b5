"""Pins of the oracle's stochastic L-BFGS (App. D, Algorithm 2).

The oracle is checked against what the mathematics fixes, not against itself:
the dense textbook BFGS inverse-Hessian update, the secant equation, the
closed-form minimiser of a convex quadratic (unconstrained and, for a
separable one, with the box of the projection step), the weighted averaging
switched on by the first energy increase, and finite differences of the
squared-slowness chain rule.
"""

import numpy as np

import oracle.slbfgs as sl


def _pairs(rng, n, m, A):
    S = [rng.standard_normal(n) for _ in range(m)]
    return S, [A @ s for s in S]


def test_two_loop_equals_dense_bfgs_update():
    rng = np.random.default_rng(0)
    n = 7
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)          # y = A s: positive curvature y^T s > 0
    S, Y = _pairs(rng, n, 5, A)
    g = rng.standard_normal(n)
    H = sl.dense_inverse_hessian(S, Y, 0.37, n)
    assert np.allclose(sl.two_loop(g, S, Y, 0.37), H @ g, rtol=0, atol=1e-12 * np.abs(H @ g).max())
    assert np.allclose(H, H.T, atol=1e-12)                   # BFGS keeps H symmetric
    # secant equation of the newest pair: H y_m = s_m
    assert np.allclose(sl.two_loop(Y[-1], S, Y, 0.37), S[-1], atol=1e-12 * np.abs(S[-1]).max())
    # no pairs: H = h0 I
    assert np.array_equal(sl.two_loop(g, [], [], 2.0), 2.0 * g)


def test_two_loop_recovers_inverse_of_quadratic_with_n_conjugate_pairs():
    # hereditary property of BFGS: after n steps along A-conjugate directions
    # (s_i^T A s_j = 0, i != j) with y = A s, H = A^-1 whatever H_0
    rng = np.random.default_rng(1)
    n = 6
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)
    lam, V = np.linalg.eigh(A)
    A_mhalf = V @ np.diag(lam ** -0.5) @ V.T
    Qo, _ = np.linalg.qr(rng.standard_normal((n, n)))
    S = [A_mhalf @ Qo[:, j] * (1 + j) for j in range(n)]
    Y = [A @ s for s in S]
    g = rng.standard_normal(n)
    want = np.linalg.solve(A, g)
    assert np.abs(sl.two_loop(g, S, Y, 1.0) - want).max() < 1e-9 * np.abs(want).max()


def test_slbfgs_converges_to_quadratic_minimiser():
    rng = np.random.default_rng(3)
    n = 20
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(1, 10, n)) @ Q.T
    b = rng.standard_normal(n)
    u_star = np.linalg.solve(A, b)

    def g(u, i):
        return 0.5 * u @ A @ u - b @ u, A @ u - b

    u_hat, J = sl.slbfgs(g, np.zeros(n), nu=1.0, n_evals=40, m_h=64, h0=0.1)
    assert np.linalg.norm(u_hat - u_star) < 1e-10 * np.linalg.norm(u_star)
    assert J[-1] <= J[0]
    assert len(J) == 20                   # two evaluations per iteration


def test_slbfgs_projection_reaches_box_minimiser():
    rng = np.random.default_rng(4)
    n = 20
    a = np.linspace(1, 5, n)
    b = 3.0 * rng.standard_normal(n)

    def g(u, i):
        return 0.5 * np.sum(a * u * u) - b @ u, a * u - b

    u_hat, _, its = sl.slbfgs(g, np.zeros(n), nu=1.0, n_evals=60, h0=0.2, u_min=-0.5, u_max=0.5, history=True)
    assert all(np.all((x >= -0.5) & (x <= 0.5)) for x in its)
    assert np.abs(u_hat - np.clip(b / a, -0.5, 0.5)).max() < 1e-4


def test_averaging_starts_after_first_energy_increase():
    # an estimator whose energy rises at iteration 3: from then on the
    # estimate is the i^3-weighted mean of the iterates of iterations >= 4
    n = 3
    raw = []

    def g(u, i):
        F = {1: 5.0, 2: 4.0, 3: 4.5}.get(i, 1.0)
        return F, u - 0.1 * i

    def weight(i):
        return float(i) ** 3

    u = np.zeros(n)
    u_hat, J, its = sl.slbfgs(g, u, nu=0.5, n_evals=12, h0=1.0, weight=weight, history=True)
    assert J[:3] == [5.0, 4.0, 4.5]
    # rerun recording the raw iterates to form the expected average
    u_raw = []
    S, Y = [], []
    for i in range(1, 7):
        F_u, G_u = g(u, i)
        z = -sl.two_loop(G_u, S, Y, 1.0)
        F_z, G_z = g(u + 0.5 * z, i)
        S.append(0.5 * z)
        Y.append(G_z - G_u)
        z = z - sl.two_loop(G_z, S, Y, 1.0)
        u = u + 0.5 * z
        u_raw.append(u.copy())
    assert np.allclose(its[2], u_raw[2])               # not averaged yet at the activating iteration
    w = np.array([weight(i) for i in range(4, 7)])
    want = (w[:, None] * np.array(u_raw[3:6])).sum(0) / w.sum()
    assert np.allclose(u_hat, want, rtol=1e-13, atol=0)


def test_squared_slowness_chain_rule():
    # J(c) = sum (c - c*)^2 / 2 with c = u^-1/2: dJ/du = -c^3/2 dJ/dc (central FD)
    rng = np.random.default_rng(5)
    c_star = 1500 + 50 * rng.standard_normal(8)
    c = 1500 + 30 * rng.standard_normal(8)
    u = 1.0 / c ** 2

    def J(uu):
        cc = 1.0 / np.sqrt(uu)
        return 0.5 * np.sum((cc - c_star) ** 2)

    G_u = -0.5 * c ** 3 * (c - c_star)
    h = 1e-6 * u
    fd = np.array([(J(u + h[k] * np.eye(8)[k]) - J(u - h[k] * np.eye(8)[k])) / (2 * h[k]) for k in range(8)])
    assert np.allclose(fd, G_u, rtol=1e-6)
