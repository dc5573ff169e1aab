"""Growth rate and coefficient of determination of crystal-size histories (host side).

TEST INFRASTRUCTURE ONLY (part of the oracle; see oracle/oracle.py).

Paper, Section 4.1.2: the average length L_avg = (L_1 + ... + L_6)/6 is recorded over time and
fitted with a linear function whose slope is the growth rate G; R^2 = 1 - A_res / A_tot with
A_res the residual and A_tot the total sum of squares about the mean.
"""
from __future__ import annotations

import numpy as np


def linear_fit(t, L):
    """Least-squares line through the points (t_j, L_j) for every column of L.

    t: [S]; L: [S] or [S, K]. Returns (slope, intercept, R2), each [K] (or scalar).
    R2 is 1 when the data are exactly constant (A_tot = 0 and A_res = 0).
    """
    t = np.asarray(t, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    one = L.ndim == 1
    if one:
        L = L[:, None]
    S = t.shape[0]
    # Normal equations of min sum_j (L_j - (b + G t_j))^2, solved with numpy's lstsq.
    A = np.stack([np.ones(S), t], axis=1)
    coef, *_ = np.linalg.lstsq(A, L, rcond=None)
    b, G = coef[0], coef[1]
    Lfit = b[None, :] + G[None, :] * t[:, None]
    A_res = ((L - Lfit) ** 2).sum(axis=0)
    A_tot = ((L - L.mean(axis=0)) ** 2).sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        R2 = np.where(A_tot > 0, 1.0 - A_res / np.where(A_tot > 0, A_tot, 1.0),
                      np.where(A_res == 0, 1.0, 0.0))
    if one:
        return G[0], b[0], R2[0]
    return G, b, R2


def growth_rates(t, L):
    """Per-direction growth rates G_k, their R^2, and G_avg, the slope of L_avg(t)."""
    G, _, R2 = linear_fit(t, L)
    L = np.asarray(L, dtype=np.float64)
    G_avg, _, _ = linear_fit(t, L.mean(axis=1))
    return G, R2, G_avg
