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
    on every column.  ``baseline`` selects back-to-back SpMV launches per
    block instead of the level-blocked MPK.

    The degree M is covered by floor(M/p) blocks of the plan's p powers and,
    when p does not divide M, one block of the remaining M mod p powers on
    the same plan (Sec. 5: powers beyond p_m run as a further, shorter MPK
    call).  Every block after the first continues the three-term recurrence
    from the last two vectors of the previous blocks, v_{b p} and
    v_{b p - 1}; with p = 1 the older one is the previous block's input."""

    def __init__(self, plan: Plan, coeffs):
        c = np.asarray(coeffs)
        self.complex = np.iscomplexobj(c)
        if self.complex and plan.nrhs != 2:
            raise ValueError("complex propagation needs a plan with nrhs = 2")
        if plan.nrhs > 2:
            raise ValueError("the recurrence epilogue handles nrhs <= 2")
        M = len(c) - 1
        if M < 1:
            raise ValueError("the degree must be at least 1")
        self.plan, self.M, self.p, self.c = plan, M, plan.p, c
        p = self.p
        if self.complex:
            self.c0 = np.array([c[0].real, c[0].imag])
        else:
            self.c0 = np.array([float(c[0])])
        # blocks: (first power index k0 of the block, number of powers)
        self.blocks = [(1 + b * p, p) for b in range(M // p)]
        if M % p:
            self.blocks.append((1 + (M // p) * p, M % p))
        self._rec = []
        for b, (k0, n) in enumerate(self.blocks):
            ck = c[k0:k0 + n]
            coef = (np.stack([ck.real, ck.imag], 1).reshape(-1) if self.complex
                    else np.asarray(ck, dtype=np.float64))
            alpha = np.full(n, 2.0)
            gamma = np.full(n, -1.0)
            if b == 0:
                alpha[0], gamma[0] = 1.0, 0.0  # v_1 = A v_0
            self._rec.append((alpha, gamma, coef.copy()))
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
        if self._Y is None or self._Y.shape[2:] != X.shape:
            # three power blocks in turn: the block being written never
            # overlaps the two vectors it continues from
            self._Y = torch.empty((3, p) + tuple(X.shape), dtype=torch.float64, device=X.device)
        run = self.plan.run_baseline if baseline else self.plan.run
        x_in, y_prev = X, None
        for b, ((k0, n), (alpha, gamma, coef)) in enumerate(zip(self.blocks, self._rec)):
            Yb = self._Y[b % 3]
            rec = Recurrence(alpha, None, gamma, coef, self.complex, y_prev, acc,
                             coef0=self.c0 if b == 0 else None)
            run(x_in, Yb, rec, stream=stream, powers=n)
            # the next block continues from v_{k0+n-1} and the vector before it
            y_prev = Yb[n - 2] if n >= 2 else x_in
            x_in = Yb[n - 1]
        return acc
