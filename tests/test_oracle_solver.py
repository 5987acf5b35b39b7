"""Pins of the oracle's ADMM solve against closed forms of the discrete problem,
bounds, an independent SciPy solver, a certified primal-dual bracket and
finite differences (none of them re-uses the oracle's own arithmetic)."""

import math

import numpy as np
import pytest
import scipy.optimize

from oracle import ccmf_oracle as O
from paper_2103_05968_amd import microstructures as M

from closed_forms import laminate_oblique_gradient
from dense_ops import dense_div_minus, dense_shift_back

TIGHT = 1e-9


def solve(gamma, xibar, tol=TIGHT, **kw):
    kw.setdefault("max_iter", 40000)
    return O.admm_solve(gamma, xibar, tol=tol, **kw)


# --- homogeneous medium: geff = kappa |xibar| (spec closed form) ------------

@pytest.mark.parametrize("xibar", [(1, 0, 0), (0, 0, 1), (0.3, -0.4, 0.866), (2.0, 1.0, -2.0)])
def test_homogeneous_gives_kappa(xibar):
    gamma = np.full((5, 4, 3), 2.5)
    r = solve(gamma, xibar)
    assert r.converged and r.iterations == 1
    assert r.residual == 0.0 or r.residual < 1e-15
    assert abs(r.geff - 2.5) < 1e-14
    assert abs(r.dual_est - 2.5) < 1e-14


# --- laminates (translation averaging in the plane of the layers) ---------------

def laminate_oblique(profile, xibar):
    """max over 0 <= c <= min gamma of |xi_1| c + |xi_perp| mean sqrt(gamma^2 - c^2):
    the reduced one-dimensional max-flow of a medium layered along e1."""
    xb = np.asarray(xibar, float) / np.linalg.norm(xibar)
    a, b = abs(xb[0]), math.hypot(xb[1], xb[2])
    gmin = profile.min()

    def neg(c):
        return -(a * c + b * np.mean(np.sqrt(np.maximum(profile ** 2 - c * c, 0.0))))

    res = scipy.optimize.minimize_scalar(neg, bounds=(0.0, gmin), method="bounded",
                                         options=dict(xatol=1e-14))
    cands = [0.0, gmin, res.x]
    return max(-neg(c) for c in cands)


@pytest.mark.parametrize("n1", [6, 7])
def test_laminate_normal_to_layers_gives_min(rng, n1):
    prof = rng.uniform(0.5, 3.0, n1)
    gamma = M.laminate(prof, (n1, 3, 2), axis=0)
    r = solve(gamma, (1, 0, 0))
    assert r.converged
    assert abs(r.geff - prof.min()) < 2e-8 * prof.min()


@pytest.mark.parametrize("xibar", [(0, 1, 0), (0, 0, 1), (0, 0.6, 0.8)])
def test_laminate_in_plane_gives_mean(rng, xibar):
    prof = rng.uniform(0.5, 3.0, 6)
    gamma = M.laminate(prof, (6, 3, 4), axis=0)
    r = solve(gamma, xibar)
    assert r.converged
    assert abs(r.geff - prof.mean()) < 2e-8 * prof.mean()


@pytest.mark.parametrize("xibar", [(0.8, 0.6, 0.0), (0.5, 0.5, 0.7071067811865476), (0.2, 0.0, 0.98)])
def test_laminate_oblique_matches_1d_maximisation(rng, xibar):
    prof = rng.uniform(0.5, 3.0, 6)
    gamma = M.laminate(prof, (6, 2, 2), axis=0)
    r = solve(gamma, xibar, tol=1e-10, max_iter=80000)
    want = laminate_oblique(prof, xibar)
    assert abs(r.geff - want) < 1e-7 * want


# --- extrusion: a field independent of x3 is a 2-d problem ---------------------

def test_extrusion_equals_single_slice(rng):
    g2 = rng.uniform(0.4, 3.0, (5, 6))
    g3 = np.repeat(g2[:, :, None], 4, axis=2)
    for xibar in [(1, 0, 0), (0.6, 0.8, 0.0), (0.3, 0.4, 0.866)]:
        a = solve(g3, xibar)
        b = solve(g2[:, :, None], xibar)
        assert abs(a.geff - b.geff) < 1e-7 * b.geff
    e3 = solve(g3, (0, 0, 1))
    assert abs(e3.geff - g2.mean()) < 1e-9 * g2.mean()


# --- bounds and the single-sphere result of Sec. 4.2 ---------------------------

def test_bounds_and_planar_cut(rng):
    gamma = rng.uniform(0.3, 4.0, (5, 4, 6))
    r = solve(gamma, (1, 0, 0))
    assert gamma.min() - 1e-9 <= r.geff <= gamma.mean() + 1e-9
    planar = min(gamma[i].mean() for i in range(gamma.shape[0]))
    assert r.geff <= planar + 1e-8
    r2 = solve(gamma, (0.2, -0.5, 0.84))
    assert gamma.min() - 1e-9 <= r2.geff <= gamma.mean() + 1e-9


def test_single_sphere_golden_fixture_scaled_down():
    """The printed result of Sec. 4.2 (tests/golden/single_sphere_sec4_2.json) on a
    cell scaled by 1/4 (16^3, diameter 8): geff = gamma_matrix."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "single_sphere_sec4_2.json")))
    n = gold["grid"][0] // 4
    gamma = M.single_sphere(n, gold["sphere_diameter"] / 4, gold["gamma_sphere"], gold["gamma_matrix"])
    r = solve(gamma, gold["load"], tol=gold["tol"])
    assert r.converged
    assert abs(r.geff - gold["geff"]) <= 1e-3 * gold["geff"]


def test_single_tough_sphere_gives_matrix_value():
    """A tough sphere (10x the matrix) is bypassed by a planar crack: geff equals
    the matrix value (Sec. 4.2).  Scaled-down cell (16^3, diameter 8)."""
    gamma = M.single_sphere(16, 8.0, 10.0, 1.0)
    r = solve(gamma, (1, 0, 0), tol=1e-8)
    assert r.converged
    assert abs(r.geff - 1.0) < 1e-6


# --- invariances ------------------------------------------------------------------

def test_invariances(rng):
    gamma = rng.uniform(0.3, 3.0, (4, 5, 3))
    xb = np.array([0.48, 0.6, 0.64])
    base = solve(gamma, xb).geff
    tol = 2e-7 * base
    # lattice translation
    assert abs(solve(np.roll(gamma, (1, 2, 1), axis=(0, 1, 2)), xb).geff - base) < tol
    # axis permutation together with the load
    perm = (2, 0, 1)
    assert abs(solve(np.transpose(gamma, perm), xb[list(perm)]).geff - base) < tol
    # reflection x1 -> -x1 together with xi_1 -> -xi_1
    assert abs(solve(gamma[::-1].copy(), xb * np.array([-1, 1, 1])).geff - base) < tol
    # antipodal load
    assert abs(solve(gamma, -xb).geff - base) < tol
    # 1-homogeneity in gamma
    assert abs(solve(3.0 * gamma, xb).geff - 3.0 * base) < 3 * tol
    # monotone and concave in gamma
    g2 = gamma + rng.uniform(0.0, 1.0, gamma.shape)
    assert solve(g2, xb).geff >= base - tol
    mid = solve(0.5 * (gamma + g2), xb).geff
    assert mid >= 0.5 * (base + solve(g2, xb).geff) - tol


# --- independent solver on tiny grids -------------------------------------------

def slsqp_max_flow(gamma, xibar):
    """The discrete max-flow of eq:CCMF_FFT_problem solved by SciPy's SLSQP on
    the face fluxes: max <xibar, v> s.t. div^- v = 0, |v|^2 + |Sv|^2 <= 2 gamma^2."""
    dims = gamma.shape
    n = gamma.size
    D = dense_div_minus(dims)
    S = dense_shift_back(dims)
    xb = np.asarray(xibar, float) / np.linalg.norm(xibar)
    cobj = np.concatenate([np.full(n, xb[c]) for c in range(3)]) / n
    g2 = 2.0 * gamma.ravel() ** 2

    def node(v):
        v3 = v.reshape(3, n)
        s3 = (S @ v).reshape(3, n)
        return g2 - np.sum(v3 ** 2, axis=0) - np.sum(s3 ** 2, axis=0)

    def node_jac(v):
        J = np.zeros((n, 3 * n))
        sv = S @ v
        for x in range(n):
            for c in range(3):
                J[x, c * n + x] -= 2 * v[c * n + x]
                J[x] -= 2 * sv[c * n + x] * S[c * n + x]
        return J

    Dr = D[:-1]       # one balance equation is implied by the others
    cons = [dict(type="eq", fun=lambda v: Dr @ v, jac=lambda v: Dr),
            dict(type="ineq", fun=node, jac=node_jac)]
    best = None
    for start in (np.zeros(3 * n), 0.5 * gamma.min() * np.concatenate([np.full(n, xb[c]) for c in range(3)])):
        res = scipy.optimize.minimize(lambda v: -cobj @ v, start, jac=lambda v: -cobj,
                                      constraints=cons, method="SLSQP",
                                      options=dict(ftol=1e-15, maxiter=2000))
        if best is None or -res.fun > -best.fun:
            best = res
    return -best.fun


@pytest.mark.parametrize("dims,xibar", [((2, 2, 2), (1, 0, 0)), ((2, 2, 2), (0.3, 0.5, 0.8)),
                                        ((3, 3, 3), (1, 0, 0)), ((3, 3, 3), (0.3, -0.5, 0.8)),
                                        ((3, 2, 1), (0.6, 0.8, 0.0))])
def test_matches_independent_socp_solver(rng, dims, xibar):
    gamma = rng.uniform(0.2, 5.0, dims)
    r = solve(gamma, xibar, tol=1e-10)
    want = slsqp_max_flow(gamma, xibar)
    assert abs(r.geff - want) < 1e-7 * want


def test_degenerate_cells():
    g = np.array([[[1.7]]])
    assert abs(solve(g, (0.3, 0.4, 0.5)).geff - 1.7) < 1e-14
    g2 = np.array([1.0, 3.0]).reshape(2, 1, 1)
    assert abs(solve(g2, (1, 0, 0)).geff - 1.0) < 1e-8
    assert abs(solve(g2, (0, 1, 0)).geff - 2.0) < 1e-8


# --- certified primal-dual bracket ------------------------------------------------

def test_certificate_brackets_and_gap_vanishes(rng):
    gamma = rng.uniform(0.3, 3.0, (4, 3, 5))
    xb = (0.36, 0.48, 0.8)
    loose = solve(gamma, xb, tol=1e-3)
    tight = solve(gamma, xb, tol=1e-10)
    truth = tight.geff
    for r in (loose, tight):
        cert, sigma = O.dual_certificate(gamma, xb, r.v)
        assert cert <= truth + 1e-10
        assert r.geff >= truth - 1e-10
    c_loose, _ = O.dual_certificate(gamma, xb, loose.v)
    c_tight, _ = O.dual_certificate(gamma, xb, tight.v)
    assert tight.geff - c_tight < 1e-7 * truth
    assert (tight.geff - c_tight) < (loose.geff - c_loose)


# --- penalty rules and damping reach the same limit ----------------------------

@pytest.mark.parametrize("rule,delta", [("bb", 0.25), ("ltd", 0.25), ("const", 0.25), ("bb", 0.5)])
def test_rules_converge_to_the_same_geff(rng, rule, delta):
    gamma = M.boolean_spheres((8, 8, 8), 2.0, 0.2, 0.3, 1.0, seed=3)
    ref = solve(gamma, (1, 0, 0), tol=1e-10, max_iter=100000)
    r = solve(gamma, (1, 0, 0), tol=1e-9, rule=rule, delta=delta, max_iter=100000)
    assert r.converged
    assert abs(r.geff - ref.geff) < 1e-6 * ref.geff


# --- pores (gamma = 0) and the all-zero field -----------------------------------

def test_pores_and_zero_field():
    g = M.boolean_spheres((8, 8, 8), 2.0, 0.25, 0.0, 1.0, seed=7)
    r = solve(g, (1, 0, 0), tol=1e-5, max_iter=20000)
    assert r.converged and 0.0 <= r.geff <= g.mean()
    planar = min(g[i].mean() for i in range(8))
    assert r.geff <= planar * (1 + 1e-4)
    z = solve(np.zeros((3, 3, 3)), (1, 0, 0))
    assert z.converged and z.iterations == 1 and z.geff == 0.0


def test_invalid_inputs_raise():
    with pytest.raises(ValueError):
        O.admm_solve(-np.ones((2, 2, 2)), (1, 0, 0))
    with pytest.raises(ValueError):
        O.admm_solve(np.full((2, 2, 2), np.nan), (1, 0, 0))
    with pytest.raises(ValueError):
        O.admm_solve(np.ones((2, 2, 2)), (0, 0, 0))
    with pytest.raises(ValueError):
        O.admm_solve(np.ones((2, 2, 2)), (1, 0, 0), delta=1.0)


# --- envelope gradient against central finite differences ---------------------

def test_envelope_gradient_matches_finite_differences(rng):
    gamma = rng.uniform(0.5, 2.5, (4, 3, 3))
    xb = (0.48, 0.6, 0.64)
    r = solve(gamma, xb, tol=1e-12, max_iter=200000)
    grad = O.envelope_gradient(gamma, r.xi_half)
    assert np.all(grad >= 0)
    # Euler's identity for the 1-homogeneous geff
    assert abs(np.sum(gamma * grad) - r.geff) < 1e-12
    h = 1e-4
    for idx in [(0, 0, 0), (1, 2, 1), (3, 1, 2), tuple(np.unravel_index(np.argmax(grad), grad.shape))]:
        gp = gamma.copy()
        gm = gamma.copy()
        gp[idx] += h
        gm[idx] -= h
        fd = (solve(gp, xb, tol=1e-12, max_iter=200000).geff
              - solve(gm, xb, tol=1e-12, max_iter=200000).geff) / (2 * h)
        assert abs(fd - grad[idx]) < 2e-4 * max(grad.max(), 1e-3)


# --- load gradient: mean face flux ------------------------------------------------

@pytest.mark.parametrize("xibar", [(0.8, 0.6, 0.0), (-0.5, 0.5, 0.7071067811865476)])
def test_mean_flux_is_the_laminate_load_gradient(rng, xibar):
    prof = rng.uniform(0.5, 3.0, 6)
    gamma = M.laminate(prof, (6, 2, 2), axis=0)
    r = solve(gamma, xibar, tol=1e-11, max_iter=200000)
    want = laminate_oblique_gradient(prof, xibar)
    assert np.abs(r.mean_flux - want).max() < 1e-6 * np.abs(want).max()
    # Euler's identity of the support function: <xibar, grad> = geff
    xb = np.asarray(xibar, float) / np.linalg.norm(xibar)
    assert abs(xb @ r.mean_flux - r.geff) < 1e-8 * r.geff


def test_mean_flux_matches_load_finite_differences(rng):
    gamma = rng.uniform(0.5, 2.5, (4, 3, 3))
    xb = np.array([0.48, 0.6, 0.64])
    r = solve(gamma, xb, tol=1e-12, max_iter=200000)
    m = r.mean_flux
    h = 1e-4
    for t in (np.array([0.6, -0.48, 0.0]), np.array([0.0, 0.64, -0.6]) / 0.8772684879784524):
        t = t - (t @ xb) * xb      # tangent to the unit sphere at xibar
        fp = solve(gamma, xb + h * t, tol=1e-12, max_iter=200000).geff
        fm = solve(gamma, xb - h * t, tol=1e-12, max_iter=200000).geff
        # d/dh geff((xibar + h t)/|xibar + h t|) = <t, m> for t orthogonal to xibar
        assert abs((fp - fm) / (2 * h) - t @ m) < 1e-6


# --- warm start ------------------------------------------------------------------

@pytest.mark.parametrize("rule", [O.RHO_BB, O.RHO_LTD])
def test_resuming_a_stopped_solve_continues_the_same_sequence(rng, rule):
    gamma = M.laminate(rng.uniform(0.5, 3.0, 5), (5, 4, 3), axis=0) * rng.uniform(0.8, 1.2, (5, 4, 3))
    xb = (0.3, -0.5, 0.81)
    k1, k2 = 17, 25
    whole = O.admm_solve(gamma, xb, tol=1e-300, rule=rule, max_iter=k1 + k2 - 1)
    first = O.admm_solve(gamma, xb, tol=1e-300, rule=rule, max_iter=k1)
    assert first.k == k1 - 1 and first.iterations == k1
    rest = O.admm_solve(gamma, xb, tol=1e-300, rule=rule, max_iter=k2,
                        start=(first.e, first.v, first.rho, first.k))
    assert rest.k == whole.k and rest.iterations == k2
    assert rest.geff == whole.geff and rest.rho == whole.rho
    assert np.array_equal(rest.v, whole.v) and np.array_equal(rest.e, whole.e)
    # a converged state stays converged: resuming it stops after one step
    conv = solve(gamma, xb, tol=1e-8, rule=rule)
    again = O.admm_solve(gamma, xb, tol=1e-8, rule=rule, start=(conv.e, conv.v, conv.rho, conv.k))
    assert again.iterations == 1 and again.geff == conv.geff
