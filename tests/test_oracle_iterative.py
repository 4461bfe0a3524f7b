"""Pins for the iterative-reconstruction oracle (CGLS and SIRT on the matched
projector pair), each against dense linear algebra rather than the oracle's
own recursion:

* CGLS: the k-th iterate is the least-squares minimiser over the Krylov space
  x0 + K_k(A^T A, A^T r0) (built by Gram-Schmidt from the dense matrix and
  solved with numpy's lstsq); run to convergence it reaches the minimum-norm
  least-squares solution (lstsq); its recursive residual equals the direct
  one; the residual never grows; degenerate and consistent cases;
* Landweber: the same closed form with unit weights;
* SIRT: a closed form through the eigen-decomposition of the symmetrised
  iteration matrix; the row/column weights against the dense matrix's sums;
  a consistent solution is a fixed point; the non-negative variant.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import iterative as IT
from oracle import forwardproject
from tests.test_oracle import dense_B


def _case(L, W, H, N, seed):
    mats = S.tiny_cone_matrices(N, W, H, L, 1.0, seed)
    A = dense_B(L, 1.0, mats, W, H).T          # (N*H*W, L^3): the forward projector
    p = S.random_projections(N, H, W, seed + 7).astype(np.float64)
    return mats, A, p


def _krylov_min(A, r0, k):
    """argmin over span{A^T r0, (A^T A) A^T r0, ...} (k vectors) of ||A y - r0||."""
    AtA = A.T @ A
    basis = []
    v = A.T @ r0
    for _ in range(k):
        for b in basis:                       # two passes of Gram-Schmidt
            v = v - (b @ v) * b
        for b in basis:
            v = v - (b @ v) * b
        n = np.linalg.norm(v)
        if n == 0.0:
            break
        basis.append(v / n)
        v = AtA @ basis[-1]
    V = np.stack(basis, 1)
    c = np.linalg.lstsq(A @ V, r0, rcond=None)[0]
    return V @ c


@pytest.mark.parametrize("L,W,H,N,seed", [(4, 7, 5, 3, 1), (5, 9, 7, 4, 2)])
def test_cgls_krylov_optimality(L, W, H, N, seed):
    mats, A, p = _case(L, W, H, N, seed)
    for k in range(1, 7):
        x, _ = IT.cgls(L, 1.0, mats, p, k)
        ref = _krylov_min(A, p.ravel(), k)
        assert np.linalg.norm(x.ravel() - ref) <= 1e-8 * np.linalg.norm(ref), k


def test_cgls_krylov_optimality_with_start():
    L, W, H, N = 4, 7, 5, 3
    mats, A, p = _case(L, W, H, N, 11)
    x0 = np.random.default_rng(4).standard_normal((L, L, L)) * 50.0
    r0 = p.ravel() - A @ x0.ravel()
    for k in (1, 3, 5):
        x, res = IT.cgls(L, 1.0, mats, p, k, x0=x0)
        ref = x0.ravel() + _krylov_min(A, r0, k)
        assert np.linalg.norm(x.ravel() - ref) <= 1e-8 * np.linalg.norm(ref), k
        assert res[0] == pytest.approx(float(r0 @ r0), rel=1e-12)


@pytest.mark.parametrize("L,W,H,N,seed", [(4, 7, 5, 3, 1), (5, 9, 7, 4, 2)])
def test_cgls_converges_to_min_norm_lstsq(L, W, H, N, seed):
    mats, A, p = _case(L, W, H, N, seed)
    x, res = IT.cgls(L, 1.0, mats, p, 200)
    ref = np.linalg.lstsq(A, p.ravel(), rcond=None)[0]     # minimum-norm solution
    assert np.linalg.norm(x.ravel() - ref) <= 1e-10 * np.linalg.norm(ref)
    # the residual is orthogonal to the range: A^T r = 0 at the solution
    r = p.ravel() - A @ x.ravel()
    assert np.linalg.norm(A.T @ r) <= 1e-10 * np.linalg.norm(A.T @ p.ravel())


def test_cgls_residual_history():
    L, W, H, N = 5, 9, 7, 4
    mats, A, p = _case(L, W, H, N, 3)
    n = 12
    _, res = IT.cgls(L, 1.0, mats, p, n)
    assert res.shape == (n + 1,)
    assert np.all(np.diff(res) <= 1e-12 * res[0])          # never grows
    for k in (0, 1, 4, 12):
        x, _ = IT.cgls(L, 1.0, mats, p, k)
        direct = float(np.sum((p.ravel() - A @ x.ravel()) ** 2))
        assert res[k] == pytest.approx(direct, rel=1e-10)


def test_cgls_degenerate_cases():
    L, W, H, N = 4, 7, 5, 3
    mats, A, p = _case(L, W, H, N, 5)
    x, res = IT.cgls(L, 1.0, mats, np.zeros_like(p), 4)
    assert np.all(x == 0.0) and np.all(res == 0.0)
    # consistent data started at the solution stays there
    xt = np.random.default_rng(6).standard_normal((L, L, L))
    pt = forwardproject(L, 1.0, mats, xt, W, H)
    x, res = IT.cgls(L, 1.0, mats, pt, 3, x0=xt)
    assert np.array_equal(x, xt)
    assert res[0] == 0.0
    # a volume entirely off the detector: A = 0, nothing moves
    far = mats.copy()
    far[:, 0, 3] += 1e4 * far[:, 2, 3]
    x, res = IT.cgls(L, 1.0, far, p, 3)
    assert np.all(x == 0.0)
    assert np.all(res == res[0])


def test_sirt_weights_are_floored_dense_sums():
    L, W, H, N = 5, 9, 7, 4
    mats, A, p = _case(L, W, H, N, 8)
    R, C = IT.sirt_weights(L, 1.0, mats, p.shape)
    rows, cols = A.sum(1), A.sum(0)
    assert (rows == 0).any() and (cols == 0).any()   # the case has empty rows and columns
    np.testing.assert_allclose(R.ravel(), 1.0 / np.maximum(rows, 1e-3 * rows.max()), rtol=1e-12)
    np.testing.assert_allclose(C.ravel(), 1.0 / np.maximum(cols, 1e-3 * cols.max()), rtol=1e-12)


@pytest.mark.parametrize("lam", [1.0, 1.7])
def test_sirt_spectral_closed_form(lam):
    """x_k = x0 + lam C A^T R (p - A x_{k-1}) is linear: with y = C^(-1/2) x and
    M = C^(1/2) A^T R A C^(1/2) = V diag(mu) V^T, each coordinate z = V^T y obeys
    z_k = (1 - lam mu)^k z_0 + (b / mu) (1 - (1 - lam mu)^k),  b = V^T C^(1/2) A^T R p."""
    L, W, H, N = 4, 7, 5, 3
    mats, A, p = _case(L, W, H, N, 9)
    rows, cols = A.sum(1), A.sum(0)
    R = 1.0 / np.maximum(rows, 1e-3 * rows.max())
    Ch = np.sqrt(1.0 / np.maximum(cols, 1e-3 * cols.max()))
    M = (Ch[:, None] * A.T) @ (R[:, None] * A * Ch[None, :])
    mu, V = np.linalg.eigh(M)
    x0 = np.random.default_rng(10).standard_normal(L ** 3) * 30.0
    z0 = V.T @ (x0 / Ch)
    b = V.T @ (Ch * (A.T @ (R * p.ravel())))
    for k in (1, 2, 5):
        f = (1.0 - lam * mu) ** k
        live = mu > 1e-12 * mu.max()
        zk = np.where(live, f * z0 + np.divide(b, mu, where=live, out=np.zeros_like(b)) * (1.0 - f),
                      z0 + k * lam * b)
        ref = Ch * (V @ zk)
        x, res = IT.sirt(L, 1.0, mats, p, k, lam=lam, x0=x0.reshape(L, L, L))
        assert np.linalg.norm(x.ravel() - ref) <= 1e-10 * np.linalg.norm(ref), k
        assert res.shape == (k,)


def test_sirt_fixed_point_and_nonneg():
    L, W, H, N = 5, 9, 7, 4
    mats, A, p = _case(L, W, H, N, 12)
    xt = np.random.default_rng(13).standard_normal((L, L, L))
    pt = (A @ xt.ravel()).reshape(p.shape)
    x, res = IT.sirt(L, 1.0, mats, pt, 3, x0=xt)
    np.testing.assert_allclose(x, xt, rtol=0, atol=1e-12 * np.abs(xt).max())
    assert max(res) <= 1e-20 * float(np.sum(pt ** 2))
    # non-negative variant: each update is clamped at zero
    x1, _ = IT.sirt(L, 1.0, mats, p, 1)
    x1n, _ = IT.sirt(L, 1.0, mats, p, 1, nonneg=True)
    assert (x1 < 0).any()
    np.testing.assert_array_equal(x1n, np.maximum(x1, 0.0))
    x5n, res = IT.sirt(L, 1.0, mats, p, 5, nonneg=True)
    assert np.all(x5n >= 0.0)


def test_landweber_spectral_closed_form():
    """x_k = x_{k-1} + lam A^T (p - A x_{k-1}); with A^T A = V diag(mu) V^T,
    z = V^T x obeys z_k = (1 - lam mu)^k z_0 + (b / mu)(1 - (1 - lam mu)^k), b = V^T A^T p."""
    L, W, H, N = 4, 7, 5, 3
    mats, A, p = _case(L, W, H, N, 14)
    mu, V = np.linalg.eigh(A.T @ A)
    lam = 1.5 / mu.max()
    x0 = np.random.default_rng(15).standard_normal(L ** 3)
    z0 = V.T @ x0
    b = V.T @ (A.T @ p.ravel())
    live = mu > 1e-12 * mu.max()
    for k in (1, 3, 6):
        f = (1.0 - lam * mu) ** k
        zk = np.where(live, f * z0 + np.divide(b, mu, where=live, out=np.zeros_like(b)) * (1.0 - f), z0 + k * lam * b)
        x, res = IT.landweber(L, 1.0, mats, p, k, lam, x0=x0.reshape(L, L, L))
        ref = V @ zk
        assert np.linalg.norm(x.ravel() - ref) <= 1e-10 * np.linalg.norm(ref), k
        assert res[0] == pytest.approx(float(np.sum((p.ravel() - A @ x0) ** 2)), rel=1e-12)
