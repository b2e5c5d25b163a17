"""Chebyshev time propagation with the MPK (Sec. 7).

One time step applies U(dt) = sum_{k=0..M} c_k T_k(A) to the state:
v_0 = x, v_1 = A x, v_{k+1} = 2 A v_k - v_{k-1} (Eq. 7-8), x' = sum c_k v_k.
The M products are split into blocks of p powers; every block is one mpk_run
whose recurrence epilogue forms v_k and accumulates c_k v_k (Sec. 7: M/p MPK
batches).  For the Schroedinger equation the coefficients are complex and
the state is a complex vector held as two real columns (k = 2).

Host-side set-up only: the coefficients are computed here once per (M, dt);
every vector operation of a step runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np
from scipy.special import jv

from .mpk import Plan, Recurrence


def schroedinger_coefficients(M: int, r_dt: float, c_dt: float = 0.0) -> np.ndarray:
    """c_k of exp(-i H dt) for H = r A + c (spectrum of A in [-1, 1]):
    (2 - delta_k0) (-i)^k J_k(r dt) exp(-i c dt) (Jacobi-Anger expansion)."""
    k = np.arange(M + 1)
    return (2.0 - (k == 0)) * ((-1j) ** k) * jv(k, r_dt) * np.exp(-1j * c_dt)


def degree_for_cutoff(r_dt: float, cutoff: float = 1e-4, max_degree: int = 4096) -> int:
    """Smallest M with |c_k| < cutoff for every k > M (the paper's cut-off rule)."""
    M = int(np.ceil(r_dt))
    while M < max_degree and np.max(np.abs(2 * jv(np.arange(M + 1, M + 40), r_dt))) >= cutoff:
        M += 1
    return M


class ChebPropagator:
    """Chebyshev propagator on a plan built with nrhs = 2 (complex state).

    ``step(X, acc)``: X (device, N x 2, plan order) is the state; acc receives
    the new state.  ``baseline`` selects p back-to-back SpMV launches per
    block instead of the level-blocked MPK.
    """

    def __init__(self, plan: Plan, M: int, r_dt: float, c_dt: float = 0.0):
        if plan.nrhs != 2:
            raise ValueError("complex propagation needs a plan with nrhs = 2")
        if M % plan.p != 0:
            raise ValueError("the degree must be a multiple of the plan's p")
        self.plan = plan
        self.M = M
        self.p = plan.p
        self.c = schroedinger_coefficients(M, r_dt, c_dt)
        p = self.p
        coef = np.stack([self.c[1:].real, self.c[1:].imag], 1).reshape(M // p, 2 * p)
        self._rec = []
        for b in range(M // p):
            if b == 0:
                alpha = np.array([1.0] + [2.0] * (p - 1))
                gamma = np.array([0.0] + [-1.0] * (p - 1))
            else:
                alpha = np.full(p, 2.0)
                gamma = np.full(p, -1.0)
            self._rec.append((alpha, gamma, coef[b].copy()))
        self._Y = None

    def step(self, X, acc, baseline: bool = False, stream=None):
        import torch

        p = self.p
        if self._Y is None or self._Y.shape[1:] != X.shape:
            self._Y = torch.empty((2, p) + tuple(X.shape), dtype=torch.float64, device=X.device)
        c0 = self.c[0]
        # acc = c_0 v_0 (complex scale of the two real columns)
        torch.mul(X, c0.real, out=acc)
        if c0.imag != 0.0:
            acc[:, 0].add_(X[:, 1], alpha=-c0.imag)
            acc[:, 1].add_(X[:, 0], alpha=c0.imag)
        run = self.plan.run_baseline if baseline else self.plan.run
        x_in, y_prev = X, None
        for b, (alpha, gamma, coef) in enumerate(self._rec):
            Yb = self._Y[b % 2]
            run(x_in, Yb, Recurrence(alpha, None, gamma, coef, True, y_prev, acc), stream=stream)
            # the next block starts from v_{(b+1)p} with v_{(b+1)p - 1} before it
            x_in, y_prev = Yb[p - 1], Yb[p - 2]
        return acc
