"""Scalar sinc quadrature of the Balakrishnan integral (oracle, test infrastructure only).

Sec. 1, eq. (integral) and Sec. 3.4, eq. (beta-approx).  For lambda > 0 and
0 < beta < 1 the Balakrishnan formula gives

    lambda^(-beta) = sin(pi beta)/pi * int_0^inf t^(-beta) (t + lambda)^(-1) dt.

(The paper prints the left-hand exponent as +beta; the identity only holds
with -beta, which is the reading used throughout.)  Substituting t = e^(-2y)
and sampling y on the grid y_k = k h turns it into the sinc rule

    lambda^(-beta) ~ (2 h sin(pi beta)/pi) sum_k e^(2 beta y_k) / (1 + e^(2 y_k) lambda),

which is the paper's rule with h = 1/sqrt(K) and k = -K..K.  The matrix rule
applies the same weights to the shifted systems (t_k M + A) with t_k = e^(-2 y_k),
see fractional.py.
"""
import math

import numpy as np


def sinc_sum(lam, beta, h, k_minus, k_plus):
    """(2 h sin(pi beta)/pi) * sum_{k=-k_minus}^{k_plus} e^{2 beta k h} / (1 + e^{2 k h} lam).

    Sec. 3.4, eq. (beta-approx), scalar form (lam may be an array)."""
    lam = np.asarray(lam, dtype=np.float64)
    total = np.zeros_like(lam)
    for k in range(-k_minus, k_plus + 1):
        y = k * h
        total = total + math.exp(2.0 * beta * y) / (1.0 + math.exp(2.0 * y) * lam)
    return 2.0 * h * math.sin(math.pi * beta) / math.pi * total


def paper_rule(lam, beta, K):
    """Q_K(lam; beta): the paper's rule with 2K+1 nodes and step 1/sqrt(K) (eq. beta-approx)."""
    return sinc_sum(lam, beta, 1.0 / math.sqrt(K), K, K)


def plain_split_error(lam, beta, K, norm=2.0):
    """Error of the plain split beta = 1 + (beta-1) on an eigenfunction with eigenvalue lam.

    One exact integer solve (factor 1/lam) followed by the sinc rule for beta-1.
    The node budget K counts the integer solve, so the rule keeps K-1 (Sec. 4.1.3,
    comparison of the two splittings at equal total node count).  `norm` is the L2
    norm of the load eigenfunction (2 for the paper's Y_{1,-1})."""
    approx = paper_rule(lam, beta - 1.0, K - 1) / lam
    return norm * abs(approx - lam ** (-beta))


def improved_split_error(lam, beta, K, norm=2.0):
    """Error of the improved split beta = 2 x (beta/2): the rule for beta/2 applied twice,
    each time with K/2 (Sec. 3.4, improved splitting; Sec. 4.1.3)."""
    q = paper_rule(lam, beta / 2.0, K // 2)
    return norm * abs(q * q - lam ** (-beta))


def fractional_error(lam, beta, K, norm=2.0):
    """Error of the paper's rule for 0 < beta < 1 on an eigenfunction (Sec. 4.1.3, Fig. 5)."""
    return norm * abs(paper_rule(lam, beta, K) - lam ** (-beta))
