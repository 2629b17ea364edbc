"""Fractional solve u ~ (M^-1 A)^-beta M^-1 b with A = kappa^2 M + S (oracle, test infrastructure only).

Sec. 3.4.  Plain split beta = n + beta' (n integer, 0 <= beta' < 1):
  * integer chain (Sec. 3.4, first display): A w_1 = b, A w_i = M w_{i-1}, i = 2..n;
  * fractional part by the sinc rule of eq. (beta-approx) applied to r = M w_n
    (r = b if n = 0).  In Galerkin form the identity of that display is the
    mass matrix M, so each node solves (M + e^{2 y_k} A) z = r, i.e.
        (t_k M + A) x_k = r,  t_k = e^{-2 y_k},  sigma_k = kappa^2 + t_k,
        u = sum_k omega_k x_k,  omega_k = (2 h sin(pi beta')/pi) t_k^{1-beta'},
    with y_k = k h for k = -k_minus..k_plus (the paper: h = 1/sqrt(K), k_minus = k_plus = K).
  * if beta' = 0 the result is w_n.
The integer chain runs first, then the node solves (both orders give the same
matrix function).  Every linear solve is a sparse LU (SuperLU) factorisation.
The quadrature sum runs over k in ascending order.

Improved split (Sec. 3.4, the modification for beta close to an integer): with
beta = n + beta', if beta' < 1/3 (and n >= 1) then beta = (n-1) + 2 beta'' with
beta'' = (beta'+1)/2; if beta' > 2/3 then beta = n + 2 beta'' with beta'' = beta'/2;
otherwise the plain split.  "2 beta''" means the sinc rule for beta'' applied twice:
v = sum_k omega_k x_k on r, then the same rule on M v.
"""
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def split_plain(beta):
    """beta = n + beta' with n = floor(beta) and beta' in [0, 1) (Sec. 3.4)."""
    n = int(math.floor(beta))
    return n, beta - n


def split(beta, mode="plain"):
    """(n, beta'', passes): n integer solves, then the rule for beta'' applied `passes` times.

    mode "plain": beta = n + beta' (one pass); mode "improved": Sec. 3.4's modification."""
    n, bf = split_plain(beta)
    if mode == "improved":
        if 0.0 < bf < 1.0 / 3.0 and n >= 1:
            return n - 1, (bf + 1.0) / 2.0, 2
        if bf > 2.0 / 3.0:
            return n, bf / 2.0, 2
    elif mode != "plain":
        raise ValueError(mode)
    return n, bf, 1


def nodes(kappa, beta_frac, h, k_minus, k_plus):
    """Shifts sigma_k = kappa^2 + t_k and weights omega_k of the sinc rule (eq. beta-approx)."""
    ks = np.arange(-k_minus, k_plus + 1)
    t = np.exp(-2.0 * ks * h)
    sigma = kappa * kappa + t
    omega = 2.0 * h * math.sin(math.pi * beta_frac) / math.pi * t ** (1.0 - beta_frac)
    return sigma, omega, t


def integer_chain(M, S, kappa, n, b):
    """w_1..w_n for right-hand sides b of shape (nsamp, N); returns a list of n arrays."""
    A = (kappa * kappa * M + S).tocsc()
    lu = spla.splu(A)
    ws = []
    rhs = b
    for _ in range(n):
        w = np.stack([lu.solve(r) for r in rhs])
        ws.append(w)
        rhs = np.stack([M @ x for x in w])
    return ws


def node_solutions(M, S, sigma, r):
    """x_k = (sigma_k M + S)^-1 r for every node k and sample; shape (K, nsamp, N)."""
    out = []
    for s in sigma:
        lu = spla.splu((s * M + S).tocsc())
        out.append(np.stack([lu.solve(v) for v in r]))
    return np.array(out)


def sample(M, S, kappa, beta, h, k_minus, k_plus, b, keep=False, mode="plain"):
    """u for loads b of shape (nsamp, N) by the plain split (mode "plain") or the improved split
    (mode "improved", two passes of the rule when it applies).

    With keep=True (plain split only) also returns the intermediate w_i and x_k (for the adjoint)."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    n, bf, passes = split(beta, mode)
    if keep and passes != 1:
        raise ValueError("keep=True is for the one-pass rule")
    ws = integer_chain(M, S, kappa, n, b)
    if bf == 0.0:
        u = ws[-1]
        return (u, ws, None, None) if keep else u
    r = b if n == 0 else np.stack([M @ w for w in ws[-1]])
    sigma, omega, _ = nodes(kappa, bf, h, k_minus, k_plus)
    for pas in range(passes):
        if pas > 0:
            r = np.stack([M @ v for v in u])
        xs = node_solutions(M, S, sigma, r)
        u = np.zeros_like(r)
        for k in range(len(sigma)):  # ascending k
            u = u + omega[k] * xs[k]
    return (u, ws, xs, omega) if keep else u


def scalar_filter(lam, kappa, beta, h, k_minus, k_plus, mode="plain"):
    """G(mu) = lam^-n Q(lam)^passes, Q(lam) = sum_k omega_k / (t_k + lam), lam = kappa^2 + mu: the
    rule as a function of a generalised eigenvalue mu of (S, M)."""
    n, bf, passes = split(beta, mode)
    if bf == 0.0:
        return lam ** (-n)
    _, omega, t = nodes(kappa, bf, h, k_minus, k_plus)
    return lam ** (-n) * np.sum(omega[:, None] / (t[:, None] + lam[None, :]), axis=0) ** passes


def dense_quadrature(M, S, kappa, beta, h, k_minus, k_plus, b, mode="plain"):
    """Brute force on tiny meshes: S V = M V Lambda, V^T M V = I gives the exact image of the
    quadrature rule, u_Q = V diag(G(kappa^2 + mu)) V^T b."""
    mu, V = sla.eigh(S.toarray(), M.toarray())
    G = scalar_filter(kappa * kappa + mu, kappa, beta, h, k_minus, k_plus, mode)
    b = np.atleast_2d(b)
    return (V @ (G[:, None] * (V.T @ b.T))).T


def dense_exact(M, S, kappa, beta, b):
    """Exact discrete fractional power u = V diag((kappa^2 + mu)^-beta) V^T b."""
    mu, V = sla.eigh(S.toarray(), M.toarray())
    G = (kappa * kappa + mu) ** (-beta)
    b = np.atleast_2d(b)
    return (V @ (G[:, None] * (V.T @ b.T))).T
