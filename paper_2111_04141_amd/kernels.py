"""Gridding-kernel design on the host: least-misfit gridding functions.

Design-time configuration, not a step of the gridding path: it produces the
kernel table that the device gridders, the pruner and the corrector take as
input (the thesis, too, takes its kernels as given inputs: Ye's script for
the least-misfit functions, Section 7.6, and CASA's prolate spheroidal,
Section 3.4.3).

Least-misfit gridding function (Section 2.3.4 after Ye et al.; corrector of
Section 2.3.5).  A record at sub-cell offset nu, gridded with kernel C of
support W cells and imaged, gives at image coordinate x (field units)
r(x, nu) = sum_b c(x + b) exp(+j2pi b nu) (Poisson summation), c the
transform of C.  With the corrector h(x) the error averaged over nu is
    e(x; C, h) = h(x)^2 sum_b c(x + b)^2 - 2 h(x) c(x) + 1,
least for h = c / sum_b c(x + b)^2 (the corrector the thesis prints),
leaving the map error 1 - c(x)^2 / sum_b c(x + b)^2.  The least-misfit
function of support W and central half-width x0 minimises the integral of
e over |x| <= x0.

Two forms of c (a reading; the thesis gives only the objective):
  * continuous: c the transform of C itself and b over all integers (a
    kernel used at very fine oversampling, the regime Ye et al. target);
  * sampled: C is used only through its table at 1/beta cells, as by the
    column pruner, whose input grid is itself sampled at 1/beta output cells
    (Convolution-Based FFT Pruning, Section 2.5); then c is the table's
    discrete transform (1/beta) sum_e T[e] cos(2pi nu_e x), periodic with
    period beta, and b runs over one period (the beta images that fold onto
    the pruned field).
Method: C is a half-wave cosine series on [-W/2, W/2], zero at the edges,
    C(nu) = sum_{m odd} a_m cos(m pi nu / W),
so c is linear in a and the map error is a ratio of quadratic forms,
    l2(x) = a' B(x) a / a' A(x) a,   B(x) = sum_{b != 0} phi(x + b) phi(x + b)',
    A(x) = B(x) + phi(x) phi(x)',
with phi(x) the transforms of the basis functions (no cancellation: the
alias terms are summed on their own).  With the denominators frozen at the
current iterate the weighted objective sum_q w_q a'B_q a / d_q is a
generalised Rayleigh quotient, minimised by the extreme eigenvector of the
pair (sum_q w_q phi_q phi_q' / d_q, sum_q w_q A_q / d_q); the iteration
refreezes d_q = a'A_q a and keeps the best iterate.  The pencil is solved
in the numerically non-null range of its second matrix.  The integral is a
Gauss-Legendre sum.  The table samples C every 1/beta cells (its end
entries are 0) and is scaled to C(0) = 1.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class LeastMisfit:
    table: np.ndarray        # beta * W + 1 samples, entry t at (t - beta W / 2)/beta cells
    coeffs: np.ndarray       # coefficients a_m of cos(m pi nu / W), m = 1, 3, 5, ...
    support: int
    x0: float
    beta: int
    sampled: bool
    mean_error: float        # mean of the map error over |x| <= x0 (model)
    max_error: float         # largest map error on the quadrature nodes (model)
    iterations: int


def _harmonics(N: int) -> np.ndarray:
    return 2 * np.arange(N) + 1


def _transform(W: int, N: int, beta: int, sampled: bool, x: np.ndarray) -> np.ndarray:
    """Transform of each basis function at x, shape [len(x), N]."""
    m = _harmonics(N)
    x = np.asarray(x, np.float64)
    if not sampled:
        wx = W * x[:, None]
        return 0.5 * W * (np.sinc(wx + m / 2) + np.sinc(wx - m / 2))
    nu = (np.arange(beta * W + 1) - beta * W / 2) / beta
    basis = np.cos(np.pi * np.outer(nu, m) / W)            # [E + 1, N]
    return (np.cos(2.0 * np.pi * np.outer(x, nu)) @ basis) / beta


def _top_eigvec(P: np.ndarray, A: np.ndarray, rcond: float = 1e-15) -> np.ndarray:
    """Vector maximising a'Pa / a'Aa (A symmetric positive semi-definite),
    solved in the range of A above rcond times its largest eigenvalue."""
    lam, U = np.linalg.eigh(A)
    keep = lam > rcond * lam.max()
    Ur = U[:, keep] / np.sqrt(lam[keep])
    mu, Y = np.linalg.eigh(Ur.T @ P @ Ur)
    return Ur @ Y[:, -1]


def least_misfit(support: int, x0: float, beta: int, sampled: bool = False,
                 nbasis: int | None = None, nodes: int = 96, alias_terms: int = 400,
                 iterations: int = 60) -> LeastMisfit:
    """Least-misfit gridding function of `support` cells for the central
    region |x| <= x0 (field units), tabulated at oversampling `beta` (see
    the module docstring for `sampled`)."""
    W = int(support)
    if W < 1 or not (0.0 < x0 < 0.5) or beta < 1 or (beta * W) % 2:
        raise ValueError("support >= 1, 0 < x0 < 0.5, beta >= 1 with beta * support even")
    N = int(nbasis) if nbasis is not None else W + 4
    g, gw = np.polynomial.legendre.leggauss(nodes)
    xq = x0 * g
    wq = x0 * gw
    phi = _transform(W, N, beta, sampled, xq)               # c(x_q) = phi a
    bs = (np.arange(beta) - beta // 2) if sampled else np.arange(-alias_terms, alias_terms + 1)
    Bq = np.zeros((nodes, N, N))
    for b in bs:
        if b == 0:
            continue
        pb = _transform(W, N, beta, sampled, xq + b)
        Bq += pb[:, :, None] * pb[:, None, :]
    Pq = phi[:, :, None] * phi[:, None, :]

    def map_error(a):
        num = np.einsum("i,qij,j->q", a, Bq, a)
        return num / (num + (phi @ a) ** 2)

    d = np.ones(nodes)
    best_obj, best_a = np.inf, None
    it = 0
    for it in range(1, iterations + 1):
        P = np.einsum("q,qij->ij", wq / d, Pq)
        A = P + np.einsum("q,qij->ij", wq / d, Bq)
        a = _top_eigvec(P, A)
        a = a / a.sum()
        err = map_error(a)
        obj = float(wq @ err)
        if obj < best_obj * (1.0 - 1e-9):
            best_obj, best_a = obj, a
        elif it > 3:
            break
        d = (phi @ a) ** 2 + np.einsum("i,qij,j->q", a, Bq, a)
    a = best_a
    err = map_error(a)
    nu = (np.arange(beta * W + 1) - beta * W / 2) / beta
    table = np.cos(np.pi * np.outer(nu, _harmonics(N)) / W) @ a
    table[0] = table[-1] = 0.0                              # cos(m pi / 2) = 0 for odd m
    return LeastMisfit(table=table, coeffs=a, support=W, x0=float(x0), beta=int(beta),
                       sampled=bool(sampled), mean_error=float(wq @ err) / (2 * x0),
                       max_error=float(err.max()), iterations=it)


def corrector(lm: LeastMisfit, x, alias_terms: int = 400) -> np.ndarray:
    """The least-misfit corrector h(x) = c(x) / sum_b c(x + b)^2 of the
    designed function at image coordinates x (field units)."""
    x = np.asarray(x, np.float64)
    N = lm.coeffs.shape[0]
    f = lambda y: _transform(lm.support, N, lm.beta, lm.sampled, y) @ lm.coeffs
    bs = (np.arange(lm.beta) - lm.beta // 2) if lm.sampled else range(-alias_terms, alias_terms + 1)
    s = np.zeros_like(x)
    for b in bs:
        s += f(x + b) ** 2
    return f(x) / s
