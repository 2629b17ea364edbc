"""d loss / d kappa of the sampled field (oracle, test infrastructure only).

Loss over samples s and points x_i with shared targets y_i:
    L = sum_s 1/2 sum_i (u_s(x_i) - y_i)^2 = sum_s 1/2 |Phi u_s - y|^2.

The field is u = sum_k omega_k x_k with (sigma_k M + S) x_k = r, sigma_k = kappa^2 + t_k,
r = M w_n and the chain A w_1 = b, A w_i = M w_{i-1}, A = kappa^2 M + S (Sec. 3.4).
omega_k and t_k do not depend on kappa.  Differentiating and transposing
(the matrices are symmetric) gives, with g_s = Phi^T (Phi u_s - y):
    lambda_k = (sigma_k M + S)^-1 g_s,      mu = sum_k omega_k lambda_k,
    nu_n = A^-1 M mu,   nu_{i-1} = A^-1 M nu_i,
    dL/dkappa = -2 kappa sum_s [ sum_k omega_k lambda_k^T M x_k + sum_i nu_i^T M w_i ].
Improved split (two passes of the rule, Sec. 3.4): u = sum_k omega_k x2_k with
(sigma_k M + S) x2_k = M u1, u1 = sum_k omega_k x1_k, (sigma_k M + S) x1_k = r.  The adjoint runs
the passes backwards: lambda2_k = (sigma_k M + S)^-1 g, mu2 = sum_k omega_k lambda2_k, then the load
of the first pass is M mu2: lambda1_k = (sigma_k M + S)^-1 M mu2, mu1 = sum_k omega_k lambda1_k, and the
chain continues from mu1; dL/dkappa gains sum_k omega_k lambda_k^T M x_k for both passes.
Three independent routes are provided: that adjoint formula with direct solves,
central finite differences of the whole sampler, and the dense generalised
eigen-expansion on tiny meshes.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import fractional


def loss(U, Phi, y):
    """Per-sample losses 1/2 |Phi u_s - y|^2, shape (nsamp,)."""
    R = np.stack([Phi @ u for u in U]) - y[None, :]
    return 0.5 * np.sum(R * R, axis=1)


def adjoint_two_pass(M, S, kappa, beta, h, k_minus, k_plus, b, Phi, y):
    """dL_s/dkappa for the improved split when it applies the rule twice (see the module text);
    returns (grad (nsamp,), u)."""
    n, bf, passes = fractional.split(beta, "improved")
    if passes != 2:
        raise ValueError("the improved split applies the rule once here; use adjoint")
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    ws = fractional.integer_chain(M, S, kappa, n, b)
    r = b if n == 0 else np.stack([M @ w for w in ws[-1]])
    sigma, omega, _ = fractional.nodes(kappa, bf, h, k_minus, k_plus)
    x1 = fractional.node_solutions(M, S, sigma, r)
    u1 = sum(omega[k] * x1[k] for k in range(len(sigma)))
    x2 = fractional.node_solutions(M, S, sigma, np.stack([M @ v for v in u1]))
    u = sum(omega[k] * x2[k] for k in range(len(sigma)))
    g = np.stack([Phi.T @ (Phi @ us - y) for us in u])
    grad = np.zeros(len(u))
    load = g
    for xs in (x2, x1):  # passes backwards
        lam = fractional.node_solutions(M, S, sigma, load)
        for k in range(len(sigma)):
            for s in range(len(u)):
                grad[s] += omega[k] * (lam[k, s] @ (M @ xs[k, s]))
        mu = sum(omega[k] * lam[k] for k in range(len(sigma)))
        load = np.stack([M @ v for v in mu])
    A_lu = spla.splu((kappa * kappa * M + S).tocsc())
    if n > 0:
        nu = np.stack([A_lu.solve(M @ v) for v in mu])
        for i in range(n, 0, -1):
            for s in range(len(u)):
                grad[s] += nu[s] @ (M @ ws[i - 1][s])
            if i > 1:
                nu = np.stack([A_lu.solve(M @ v) for v in nu])
    return -2.0 * kappa * grad, u


def adjoint(M, S, kappa, beta, h, k_minus, k_plus, b, Phi, y):
    """Per-sample dL_s/dkappa by the adjoint formula above; returns (grad (nsamp,), u)."""
    u, ws, xs, omega = fractional.sample(M, S, kappa, beta, h, k_minus, k_plus, b, keep=True)
    n, bf = fractional.split_plain(beta)
    g = np.stack([Phi.T @ (Phi @ us - y) for us in u])
    grad = np.zeros(len(u))
    A_lu = spla.splu((kappa * kappa * M + S).tocsc())
    if bf != 0.0:
        sigma, omega, _ = fractional.nodes(kappa, bf, h, k_minus, k_plus)
        lam = fractional.node_solutions(M, S, sigma, g)
        for k in range(len(sigma)):
            for s in range(len(u)):
                grad[s] += omega[k] * (lam[k, s] @ (M @ xs[k, s]))
        mu = np.zeros_like(g)
        for k in range(len(sigma)):
            mu = mu + omega[k] * lam[k]
        adj = mu
    else:
        adj = g
    # chain adjoint: nu_n = A^-1 M adj (fractional case) or A^-1 g (pure integer case)
    if n > 0:
        if bf != 0.0:
            nu = np.stack([A_lu.solve(M @ v) for v in adj])
        else:
            nu = np.stack([A_lu.solve(v) for v in adj])
        for i in range(n, 0, -1):
            for s in range(len(u)):
                grad[s] += nu[s] @ (M @ ws[i - 1][s])
            if i > 1:
                nu = np.stack([A_lu.solve(M @ v) for v in nu])
    return -2.0 * kappa * grad, u


def finite_difference(M, S, kappa, beta, h, k_minus, k_plus, b, Phi, y, delta=1e-5, mode="plain"):
    """Central difference [L(kappa+delta) - L(kappa-delta)] / (2 delta), per sample."""
    up = fractional.sample(M, S, kappa + delta, beta, h, k_minus, k_plus, b, mode=mode)
    um = fractional.sample(M, S, kappa - delta, beta, h, k_minus, k_plus, b, mode=mode)
    return (loss(up, Phi, y) - loss(um, Phi, y)) / (2.0 * delta)


def eigen_expansion(M, S, kappa, beta, h, k_minus, k_plus, b, Phi, y, mode="plain"):
    """Dense route: u = V diag(G(kappa^2+mu)) V^T b, du/dkappa = V diag(2 kappa G'(.)) V^T b,
    G(lam) = lam^-n Q(lam)^P (P passes of the rule), Q = sum_k omega_k/(t_k+lam),
    G' = -n lam^{-n-1} Q^P + P lam^-n Q^{P-1} Q'."""
    mu, V = sla.eigh(S.toarray(), M.toarray())
    n, bf, passes = fractional.split(beta, mode)
    lam = kappa * kappa + mu
    if bf != 0.0:
        _, omega, t = fractional.nodes(kappa, bf, h, k_minus, k_plus)
        Q = np.sum(omega[:, None] / (t[:, None] + lam[None, :]), axis=0)
        dQ = -np.sum(omega[:, None] / (t[:, None] + lam[None, :]) ** 2, axis=0)
    else:
        Q, dQ = np.ones_like(lam), np.zeros_like(lam)
    G = lam ** (-n) * Q ** passes
    dG = -n * lam ** (-n - 1.0) * Q ** passes + passes * lam ** (-n) * Q ** (passes - 1) * dQ
    b = np.atleast_2d(b)
    c = V.T @ b.T
    U = (V @ (G[:, None] * c)).T
    dU = (V @ ((2.0 * kappa * dG)[:, None] * c)).T
    R = np.stack([Phi @ u for u in U]) - y[None, :]
    return np.array([R[s] @ (Phi @ dU[s]) for s in range(len(U))]), U
