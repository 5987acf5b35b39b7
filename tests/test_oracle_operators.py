"""Pins of the oracle's grid operators against brute-force index loops and dense
linear algebra written directly from the paper's definitions (Sec. 2.2, Sec. 3.1)."""

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

from oracle import ccmf_oracle as O

from dense_ops import (_lin, _voxels, dense_A, dense_div_minus, dense_grad_plus,
                       dense_proj_K, dense_shift_back)

DIMS = (3, 4, 5)


def test_shift_operators_match_index_definition(rng):
    v = rng.standard_normal((3,) + DIMS)
    S = dense_shift_back(DIMS)
    np.testing.assert_allclose(O.shift_back(v).ravel(), S @ v.ravel(), atol=0)
    # S* is the adjoint of S under the 1/N inner product, i.e. the transpose
    np.testing.assert_allclose(O.shift_fwd(v).ravel(), S.T @ v.ravel(), atol=0)
    np.testing.assert_allclose(O.shift_fwd(O.shift_back(v)), v, atol=0)


def test_div_and_grad_match_index_definition(rng):
    v = rng.standard_normal((3,) + DIMS)
    phi = rng.standard_normal(DIMS)
    D = dense_div_minus(DIMS)
    G = dense_grad_plus(DIMS)
    np.testing.assert_allclose(O.div_minus(v).ravel(), D @ v.ravel(), atol=1e-13)
    np.testing.assert_allclose(O.grad_plus(phi).ravel(), G @ phi.ravel(), atol=1e-13)
    # summation by parts: <div^- v, phi> = -<v, grad^+ phi>  (so grad^+ = -(div^-)*)
    np.testing.assert_allclose(D, -G.T, atol=0)
    assert abs(O.inner(O.div_minus(v)[None], phi[None]) + O.inner(v, O.grad_plus(phi))) < 1e-13


def test_A_adjoint_isometry_and_projector(rng):
    v = rng.standard_normal((3,) + DIMS)
    w = rng.standard_normal((6,) + DIMS)
    A = dense_A(DIMS)
    np.testing.assert_allclose(O.A_op(v).ravel(), A @ v.ravel(), atol=1e-14)
    np.testing.assert_allclose(O.A_adj(w).ravel(), A.T @ w.ravel(), atol=1e-14)
    # A*A = Id (Sec. 3.1), A A* an orthogonal projector
    np.testing.assert_allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-14)
    P = A @ A.T
    np.testing.assert_allclose(P @ P, P, atol=1e-14)
    np.testing.assert_allclose(O.A_adj(O.A_op(v)), v, atol=1e-14)


def test_node_constraint_equals_face_sum(rng):
    """|(A v)[x]|^2 equals half the sum of squares of the six face fluxes incident
    to voxel x (eq:theory_CCMF_original_bound, eq:CCMF_FFT_problemA)."""
    v = rng.standard_normal((3,) + DIMS)
    Av = O.A_op(v)
    n1, n2, n3 = DIMS
    for (i, j, k) in _voxels(DIMS):
        faces = [v[0, i, j, k], v[0, (i - 1) % n1, j, k],
                 v[1, i, j, k], v[1, i, (j - 1) % n2, k],
                 v[2, i, j, k], v[2, i, j, (k - 1) % n3]]
        assert abs(np.sum(Av[:, i, j, k] ** 2) - 0.5 * np.sum(np.square(faces))) < 1e-13


def test_laplace_pinv_equals_dense_pseudoinverse(rng):
    r = rng.standard_normal(DIMS)
    L = dense_div_minus(DIMS) @ dense_grad_plus(DIMS)
    phi_dense = np.linalg.pinv(L) @ r.ravel()
    np.testing.assert_allclose(O.laplace_pinv(r).ravel(), phi_dense, atol=1e-12)
    # the symbol vanishes only at q = 0
    lam = O.laplace_symbol((4, 6, 7))
    assert lam[0, 0, 0] == 0.0 and np.count_nonzero(lam == 0.0) == 1


@pytest.mark.parametrize("dims", [(3, 4, 5), (4, 4, 1), (1, 1, 1), (2, 3, 2)])
def test_gamma_is_orthogonal_projector_onto_gradients(rng, dims):
    n = int(np.prod(dims))
    G = dense_grad_plus(dims)
    basis = np.zeros((3 * n, 3 * n))
    for col in range(3 * n):
        e = np.zeros(3 * n)
        e[col] = 1.0
        basis[:, col] = O.Gamma_op(e.reshape((3,) + dims)).ravel()
    # projector onto range(grad^+), computed independently by dense least squares
    Q = scipy.linalg.orth(G) if np.any(G) else np.zeros((3 * n, 0))
    np.testing.assert_allclose(basis, Q @ Q.T, atol=1e-12)


@pytest.mark.parametrize("dims", [(3, 4, 5), (2, 3, 1)])
def test_proj_K_matches_dense_projection(rng, dims):
    xibar = rng.standard_normal(3)
    xibar /= np.linalg.norm(xibar)
    w = rng.standard_normal((6,) + dims)
    xi, phi = O.proj_K(w, xibar)
    np.testing.assert_allclose(xi.ravel(), dense_proj_K(w, xibar, dims), atol=1e-12)
    # xi lies in K with the returned potential: A* xi = xibar + grad^+ phi
    lhs = O.A_adj(xi)
    rhs = np.stack([xibar[c] + O.grad_plus(phi)[c] for c in range(3)])
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)
    assert abs(phi.mean()) < 1e-13
    # idempotent
    xi2, _ = O.proj_K(xi, xibar)
    np.testing.assert_allclose(xi2, xi, atol=1e-12)


def test_proj_C_is_the_ball_projection(rng):
    dims = (2, 3, 2)
    gamma = rng.uniform(0.0, 2.0, dims)
    gamma[0, 0, 0] = 0.0
    w = rng.standard_normal((6,) + dims) * 1.5
    p = O.proj_C(w, gamma)
    nrm = np.sqrt(np.sum(p * p, axis=0))
    assert np.all(nrm <= gamma * (1 + 1e-14) + 1e-300)
    # variational inequality <w - P w, y - P w> <= 0 for points y of the ball
    for _ in range(50):
        y = rng.standard_normal((6,) + dims)
        ny = np.sqrt(np.sum(y * y, axis=0))
        y *= (gamma * rng.uniform(0, 1, dims) / np.maximum(ny, 1e-300))[None]
        assert np.all(np.sum((w - p) * (y - p), axis=0) <= 1e-12)
    # continuity at the sphere |w| = gamma and identity inside
    w_in = w * (0.5 * gamma / np.maximum(np.sqrt(np.sum(w * w, axis=0)), 1e-300))[None]
    np.testing.assert_allclose(O.proj_C(w_in, gamma), w_in, atol=0)
    w_on = w * (gamma / np.sqrt(np.sum(w * w, axis=0)))[None]
    np.testing.assert_allclose(O.proj_C(w_on * (1 + 1e-12), gamma), w_on, atol=1e-11)


def test_admm_step_e_update_is_the_augmented_lagrangian_minimiser(rng):
    """e^{k+1} = argmin_e g(e) + <v, xi^{k+1} - e> + rho/2 |xi^{k+1} - e|^2
    (eq:CCMF_FFT_ADMM_abstract, second line), checked per voxel with a direct
    numerical minimisation; the xi-step against the dense projection."""
    dims = (2, 2, 3)
    gamma = rng.uniform(0.3, 2.0, dims)
    xibar = np.array([0.6, -0.8, 0.0])
    e = rng.standard_normal((6,) + dims)
    v = O.proj_C(rng.standard_normal((6,) + dims), gamma)
    rho, delta = 0.7, 0.25
    xi_half, phi, e_new, v_new = O.admm_step(e, v, rho, xibar, gamma, delta)
    np.testing.assert_allclose(xi_half.ravel(), dense_proj_K(e - v / rho, xibar, dims), atol=1e-12)
    xi_new = 2 * (1 - delta) * xi_half - (1 - 2 * delta) * e
    for (i, j, k) in _voxels(dims):
        g, vv, xx = gamma[i, j, k], v[:, i, j, k], xi_new[:, i, j, k]

        def f(y):
            return g * np.sqrt(np.sum(y * y) + 1e-300) - vv @ y + 0.5 * rho * np.sum((xx - y) ** 2)

        best = min((scipy.optimize.minimize(f, x0, method="Nelder-Mead",
                                            options=dict(xatol=1e-12, fatol=1e-14, maxiter=40000))
                    for x0 in (e_new[:, i, j, k] + 1e-3, np.zeros(6) + 1e-6)), key=lambda r: r.fun)
        assert f(e_new[:, i, j, k]) <= best.fun + 1e-9
        np.testing.assert_allclose(best.x, e_new[:, i, j, k], atol=2e-4)
    np.testing.assert_allclose(v_new, v + rho * (xi_new - e_new), atol=0)
