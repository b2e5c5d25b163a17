"""Chebyshev time propagation with the MPK (Sec. 7).

One time step applies U(dt) = sum_{k=0..M} c_k T_k(A) to the state:
v_0 = x, v_1 = A x, v_{k+1} = 2 A v_k - v_{k-1} (Eq. 7-8), x' = sum c_k v_k.
The M products are split into blocks of p powers; every block is one mpk_run
whose recurrence epilogue forms v_k and accumulates c_k v_k (Sec. 7: M/p MPK
batches); the first block also starts the sum with c_0 v_0.  Two equations:

* Schroedinger, i dpsi/dt = H psi with H = r A + c: complex coefficients
  (Bessel functions J_k), the state is a complex vector held as two real
  columns (k = 2).
* Heat, dpsi/dt = a Laplacian(psi), discretised as L = -Laplacian_h with
  spectrum in [0, 2r] and stored as A = L / r - I: real coefficients
  (modified Bessel functions I_k), one real column.

Host-side set-up only: the coefficients are computed here once per (M, dt);
every vector operation of a step runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ive, jv

from .mpk import Plan, Recurrence


def schroedinger_coefficients(M: int, r_dt: float, c_dt: float = 0.0) -> np.ndarray:
    """c_k of exp(-i H dt) for H = r A + c (spectrum of A in [-1, 1]):
    (2 - delta_k0) (-i)^k J_k(r dt) exp(-i c dt) (Jacobi-Anger expansion)."""
    k = np.arange(M + 1)
    return (2.0 - (k == 0)) * ((-1j) ** k) * jv(k, r_dt) * np.exp(-1j * c_dt)


def heat_coefficients(M: int, tau: float) -> np.ndarray:
    """c_k of exp(-tau (A + I)) = exp(-a dt L) for L = r (A + I), tau = a dt r:
    the generating function of the modified Bessel functions gives
    exp(-tau x) = I_0(tau) + 2 sum_k (-1)^k I_k(tau) T_k(x), so
    c_k = (2 - delta_k0) (-1)^k exp(-tau) I_k(tau) (scipy's ive)."""
    k = np.arange(M + 1)
    return (2.0 - (k == 0)) * np.where(k % 2 == 0, 1.0, -1.0) * ive(k, tau)


def degree_for_cutoff(x: float, cutoff: float = 1e-4, max_degree: int = 4096, kind: str = "schroedinger") -> int:
    """Smallest M with |c_k| < cutoff for every k > M (the paper's cut-off
    rule); x is r dt (Schroedinger) or tau (heat)."""
    if kind == "schroedinger":
        f = lambda k: 2 * np.abs(jv(k, x))  # noqa: E731
        M = int(np.ceil(x))  # J_k(x) is not small before k > x
    else:
        f = lambda k: 2 * ive(k, x)  # noqa: E731
        M = 1
    while M < max_degree and np.max(f(np.arange(M + 1, M + 40))) >= cutoff:
        M += 1
    return M


class ChebPropagator:
    """Chebyshev propagator: ``step(X, acc)`` writes U(dt) X to acc (both
    device, N x k, plan order).  Complex coefficients need a plan with
    nrhs = 2 (re, im columns of one complex state); real coefficients act
    on every column.  ``baseline`` selects p back-to-back SpMV launches per
    block instead of the level-blocked MPK."""

    def __init__(self, plan: Plan, coeffs):
        c = np.asarray(coeffs)
        self.complex = np.iscomplexobj(c)
        if self.complex and plan.nrhs != 2:
            raise ValueError("complex propagation needs a plan with nrhs = 2")
        if plan.nrhs > 2:
            raise ValueError("the recurrence epilogue handles nrhs <= 2")
        M = len(c) - 1
        if M < 1 or M % plan.p != 0:
            raise ValueError("the degree must be a positive multiple of the plan's p")
        self.plan, self.M, self.p, self.c = plan, M, plan.p, c
        p = self.p
        if self.complex:
            coef = np.stack([c[1:].real, c[1:].imag], 1).reshape(M // p, 2 * p)
            self.c0 = np.array([c[0].real, c[0].imag])
        else:
            coef = np.asarray(c[1:], dtype=np.float64).reshape(M // p, p)
            self.c0 = np.array([float(c[0])])
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

    @classmethod
    def schroedinger(cls, plan: Plan, M: int, r_dt: float, c_dt: float = 0.0):
        return cls(plan, schroedinger_coefficients(M, r_dt, c_dt))

    @classmethod
    def heat(cls, plan: Plan, M: int, tau: float):
        return cls(plan, heat_coefficients(M, tau))

    def step(self, X, acc, baseline: bool = False, stream=None):
        import torch

        p = self.p
        if self._Y is None or self._Y.shape[1:] != X.shape:
            self._Y = torch.empty((2, p) + tuple(X.shape), dtype=torch.float64, device=X.device)
        run = self.plan.run_baseline if baseline else self.plan.run
        x_in, y_prev = X, None
        for b, (alpha, gamma, coef) in enumerate(self._rec):
            Yb = self._Y[b % 2]
            rec = Recurrence(alpha, None, gamma, coef, self.complex, y_prev, acc,
                             coef0=self.c0 if b == 0 else None)
            run(x_in, Yb, rec, stream=stream)
            # the next block starts from v_{(b+1)p} with v_{(b+1)p - 1} before it
            x_in, y_prev = Yb[p - 1], Yb[p - 2]
        return acc
