"""FP64 oracle for iterative reconstruction on the matched projector pair.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's
CPU-baseline leg; the product library never imports it.

The system is  A x = p  with
  A   = the forward projector, the exact adjoint of the backprojection of the
        paper's Listing 1 (``oracle.forwardproject``: volume -> projections),
  A^T = that backprojection (``oracle.backproject``: projections -> volume),
so one iteration costs one backprojection and one forward projection.  The
paper itself is about the backprojection only; these solvers are standard
algorithms written out from their published definitions, with the two
oracle projectors and numpy vector arithmetic as their only steps.

CGLS (conjugate gradients applied to the normal equations A^T A x = A^T p in
the residual form of Hestenes & Stiefel, 1952; Bjorck, "Numerical Methods for
Least Squares Problems", 1996, Sec. 7.4):
    r0 = p - A x0,  s0 = A^T r0,  d0 = s0,  gamma0 = ||s0||^2
    for k = 0, 1, ...:
        q      = A d_k
        alpha  = gamma_k / ||q||^2               (0 if ||q|| = 0)
        x     += alpha d_k
        r     -= alpha q
        s      = A^T r
        gamma' = ||s||^2
        beta   = gamma' / gamma_k                (0 if gamma_k = 0)
        d      = s + beta d_k
The k-th iterate minimises ||A x - p|| over x0 + K_k(A^T A, A^T r0).

Landweber (1951), plain gradient descent on 0.5 ||A x - p||^2 with a fixed step:
    x_{k+1} = x_k + lambda A^T (p - A x_k)

SIRT (simultaneous iterative reconstruction, Gilbert 1972, in the row/column
normalised form used for cone-beam CT, e.g. Gregor & Benson 2008):
    x_{k+1} = x_k + lambda * C (A^T (R (p - A x_k)))     [then max(., 0) if nonneg]
with R = diag(1 / row sums of A), C = diag(1 / column sums of A).  Row sums
are A applied to a volume of ones, column sums A^T applied to projections of
ones.  Reading of this implementation (the published form divides by the sums
and leaves zero sums out): each sum is floored at SIRT_FLOOR times the largest
sum before it is inverted, 1 / max(s, SIRT_FLOOR * max(s)).  Rows and columns
with a zero sum then contribute exactly zero, as in the published form, and
the weights stay continuous in the sums, so rays that graze the volume with a
vanishing row sum cannot turn rounding differences into O(1) updates.
"""
from __future__ import annotations

import numpy as np

from . import backproject, forwardproject, _f64

SIRT_FLOOR = 1e-3


def _ops(L, voxel, mats, shape, origin):
    N, H, W = shape

    def A(x):
        return forwardproject(L, voxel, mats, x, W, H, origin)

    def At(r):
        return backproject(L, voxel, mats, r, origin)

    return A, At


def _dot(a, b) -> float:
    return float(np.dot(a.ravel(), b.ravel()))


def cgls(L: int, voxel: float, mats, proj, n_iter: int, x0=None, origin=None):
    """CGLS for min ||A x - p||_2 (FP64).

    Returns (x, res2) where res2[k] = ||r_k||^2, k = 0 .. n_iter, the squared
    norm of the residual as carried by the recursion (equal to ||p - A x_k||^2
    in exact arithmetic)."""
    p = _f64(proj)
    A, At = _ops(L, voxel, mats, p.shape, origin)
    if x0 is None:
        x = np.zeros((L, L, L))
        r = p.copy()
    else:
        x = _f64(x0).reshape(L, L, L).copy()
        r = p - A(x)
    s = At(r)
    d = s.copy()
    gamma = _dot(s, s)
    res2 = [_dot(r, r)]
    for _ in range(n_iter):
        q = A(d)
        qq = _dot(q, q)
        alpha = gamma / qq if qq > 0.0 else 0.0
        x += alpha * d
        r -= alpha * q
        res2.append(_dot(r, r))
        s = At(r)
        gamma_new = _dot(s, s)
        beta = gamma_new / gamma if gamma > 0.0 else 0.0
        d = s + beta * d
        gamma = gamma_new
    return x, np.array(res2)


def sirt_weights(L: int, voxel: float, mats, shape, origin=None):
    """(R, C): the inverted, floored row sums (N, H, W) and column sums (L, L, L)."""
    A, At = _ops(L, voxel, mats, shape, origin)
    rows = A(np.ones((L, L, L)))
    cols = At(np.ones(shape))

    def inv(s):
        floor = SIRT_FLOOR * s.max()
        return 1.0 / np.maximum(s, floor) if floor > 0.0 else np.zeros_like(s)

    return inv(rows), inv(cols)


def sirt(L: int, voxel: float, mats, proj, n_iter: int, lam: float = 1.0, x0=None,
         nonneg: bool = False, origin=None):
    """SIRT (FP64).  Returns (x, res2) with res2[k] = ||p - A x_k||^2 for
    k = 0 .. n_iter - 1 (the residual each update starts from)."""
    p = _f64(proj)
    A, At = _ops(L, voxel, mats, p.shape, origin)
    R, C = sirt_weights(L, voxel, mats, p.shape, origin)
    x = np.zeros((L, L, L)) if x0 is None else _f64(x0).reshape(L, L, L).copy()
    res2 = []
    for _ in range(n_iter):
        r = p - A(x)
        res2.append(_dot(r, r))
        x = x + lam * C * At(R * r)
        if nonneg:
            x = np.maximum(x, 0.0)
    return x, np.array(res2)


def landweber(L: int, voxel: float, mats, proj, n_iter: int, lam: float, x0=None, origin=None):
    """Landweber iteration (FP64).  Returns (x, res2) with res2[k] =
    ||p - A x_k||^2, k = 0 .. n_iter - 1."""
    p = _f64(proj)
    A, At = _ops(L, voxel, mats, p.shape, origin)
    x = np.zeros((L, L, L)) if x0 is None else _f64(x0).reshape(L, L, L).copy()
    res2 = []
    for _ in range(n_iter):
        r = p - A(x)
        res2.append(_dot(r, r))
        x = x + lam * At(r)
    return x, np.array(res2)
