"""Plain FP64 NumPy oracle for the FFT-based ADMM of the CCMF discretization
of the effective crack energy (Ernesti & Schneider, arXiv 2103.05968).

THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite,
the smoke check of the package entry module and the ``cpu_baseline`` leg of
the benchmark may import or call anything in this directory.  It shares no
code with the HIP path (no kernels, tables, constants or helpers) and imports
nothing from the product package.

Everything here is written for a reader holding the paper, in its notation:

* ``gamma``   crack resistance sampled at voxel centres, shape (N1, N2, N3)
              (Sec. 2.2, the sampling below the mass-conservation equation).
* flux ``v``  3 components on the faces i+1/2, j+1/2, k+1/2, stored at the
              voxel centre (the cell-centred identification of Sec. 2.2).
* ``xi``, ``e``, ADMM multiplier ``v``: 6 components per voxel (Sec. 3.2).
* inner product with the 1/(N1 N2 N3) normalisation (eq:theory_CCMF_inner_product).

Arrays of vector fields carry the component on axis 0: 3-fields (3, N1, N2, N3),
6-fields (6, N1, N2, N3) with rows 0..2 = first block, rows 3..5 = second block.

Readings of points the paper leaves open are marked "READING" below; each is
listed, with its justification, in the design notes of the repository.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
something other than itself (brute-force index loops, dense linear algebra,
closed forms derived from the discrete problem, an independent SciPy solver,
bounds and a certified primal-dual bracket).  The iteration path of the
adaptive penalty rules (the Barzilai-Borwein safeguard, READING 4) has no
independent pin: "parity unpinned" for the penalty trajectory itself; the
limit it converges to (geff) is pinned.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SQRT2 = math.sqrt(2.0)


# ---------------------------------------------------------------------------
# Grid operators of the CCMF discretization (Sec. 2.2 and Sec. 3.1)
# ---------------------------------------------------------------------------

def shift_back(v: np.ndarray) -> np.ndarray:
    """Backward shift S (eq:theory_CCMF_shift_operator): (Sv)_c[x] = v_c[x - e_c], periodic."""
    return np.stack([np.roll(v[c], 1, axis=c) for c in range(3)])


def shift_fwd(v: np.ndarray) -> np.ndarray:
    """Forward shift S* (eq:CCMF_FFT_SOperator_adjoint): (S*v)_c[x] = v_c[x + e_c], periodic."""
    return np.stack([np.roll(v[c], -1, axis=c) for c in range(3)])


def A_op(v: np.ndarray) -> np.ndarray:
    """Dimension-doubling operator A v = [v; S v]/sqrt(2) (eq:CCMF_FFT_AOperator)."""
    return np.concatenate([v, shift_back(v)]) / SQRT2


def A_adj(w: np.ndarray) -> np.ndarray:
    """Adjoint A*[w1; w2] = (w1 + S* w2)/sqrt(2) (eq:CCMF_FFT_AOperator_adjoint)."""
    return (w[:3] + shift_fwd(w[3:])) / SQRT2


def div_minus(v: np.ndarray) -> np.ndarray:
    """Backward divergence div^- (Sec. 2.2): sum_c v_c[x] - v_c[x - e_c]."""
    return sum(v[c] - np.roll(v[c], 1, axis=c) for c in range(3))


def grad_plus(phi: np.ndarray) -> np.ndarray:
    """Forward difference gradient nabla^+ (first used in the dual function of Sec. 3.1).

    READING 1: (nabla^+ phi)_c[x] = phi[x + e_c] - phi[x], no 1/h; this is the
    operator for which <div^- v, phi> = -<v, nabla^+ phi> under the 1/N inner
    product, which is what the derivation of the projector requires.
    """
    return np.stack([np.roll(phi, -1, axis=c) - phi for c in range(3)])


def inner(a: np.ndarray, b: np.ndarray) -> float:
    """Inner product with the 1/(N1 N2 N3) normalisation (eq:theory_CCMF_inner_product)."""
    n = a.shape[-1] * a.shape[-2] * a.shape[-3]
    return float(np.sum(a * b)) / n


def laplace_symbol(dims) -> np.ndarray:
    """Fourier symbol of div^- nabla^+ on the rfftn grid.

    READING 2: with the DFT convention f^(q) = sum_x f[x] exp(-2 pi i q.x/N),
    the forward difference has symbol exp(2 pi i q_c/N_c) - 1, so the periodic
    7-point Laplacian div^- nabla^+ has the real symbol
    lambda(q) = -sum_c 4 sin^2(pi q_c / N_c), zero only at q = 0.
    """
    n1, n2, n3 = dims
    q1 = np.arange(n1)[:, None, None]
    q2 = np.arange(n2)[None, :, None]
    q3 = np.arange(n3 // 2 + 1)[None, None, :]
    return -(4.0 * np.sin(np.pi * q1 / n1) ** 2
             + 4.0 * np.sin(np.pi * q2 / n2) ** 2
             + 4.0 * np.sin(np.pi * q3 / n3) ** 2)


def laplace_pinv(r: np.ndarray) -> np.ndarray:
    """phi = (div^- nabla^+)^dagger r, solved in Fourier space (the pseudo-inverse in
    eq:CCMF_FFT_Gamma_2; the mean mode is set to zero, so phi has zero mean)."""
    lam = laplace_symbol(r.shape)
    rh = np.fft.rfftn(r)
    lam0 = lam.copy()
    lam0[0, 0, 0] = 1.0
    ph = rh / lam0
    ph[0, 0, 0] = 0.0
    return np.fft.irfftn(ph, s=r.shape, axes=(0, 1, 2))


def Gamma_op(v: np.ndarray) -> np.ndarray:
    """Gamma = nabla^+ (div^- nabla^+)^dagger div^- (eq:CCMF_FFT_Gamma_2), on 3-fields."""
    return grad_plus(laplace_pinv(div_minus(v)))


def A_xibar(xibar, dims) -> np.ndarray:
    """A applied to the constant field xibar (a 6-field)."""
    const = np.empty((3,) + tuple(dims))
    for c in range(3):
        const[c] = xibar[c]
    return A_op(const)


def proj_K(w: np.ndarray, xibar) -> tuple[np.ndarray, np.ndarray]:
    """Orthogonal projection onto K_xibar (eq:CCMF_FFT_Gamma_2):

        P_K(w) = A xibar + (Id - A A* + A Gamma A*) w.

    Returns (P_K(w), phi) with phi = (div^- nabla^+)^dagger div^- A* w the node
    potential of eq:CCMF_FFT_Gamma_1 (zero mean).
    """
    dims = w.shape[1:]
    Aw = A_adj(w)
    phi = laplace_pinv(div_minus(Aw))
    gphi = grad_plus(phi)                  # = Gamma A* w
    xi = A_xibar(xibar, dims) + w - A_op(Aw) + A_op(gphi)
    return xi, phi


def proj_C(w: np.ndarray, gamma: np.ndarray) -> np.ndarray:
    """Node-wise projection onto C_gamma (eq:CCMF_FFT_Cgamma and the formula after
    Moreau's identity): gamma w/|w| where |w| > gamma, else w (6-vectors)."""
    nw = np.sqrt(np.sum(w * w, axis=0))
    out = w.copy()
    big = nw > gamma
    scale = np.zeros_like(nw)
    scale[big] = gamma[big] / nw[big]
    out[:, big] = w[:, big] * scale[big]
    return out


def energy(xi: np.ndarray, gamma: np.ndarray) -> float:
    """g(xi) = (1/N) sum gamma |xi| (eq:CCMF_FFT_problem_primal_final)."""
    return float(np.mean(gamma * np.sqrt(np.sum(xi * xi, axis=0))))


# ---------------------------------------------------------------------------
# The damped ADMM with adaptive penalty (eq:CCMF_FFT_ADMM, second form)
# ---------------------------------------------------------------------------

RHO_BB, RHO_CONST, RHO_LTD = "bb", "const", "ltd"
BB_MIN_CORRELATION = 0.2   # READING 4: reliability test of the Barzilai-Borwein estimate
RHO_CLAMP = 1e6            # READING 4: adaptive penalties kept within [1/RHO_CLAMP, RHO_CLAMP] * rho0
ETA0, K0 = 1.0, 100.0      # READING 4: rho^{k+1}/rho^k within [1/g_k, g_k], g_k = 1 + ETA0/(1 + k/K0)^2


@dataclass
class AdmmResult:
    geff: float                 # primal energy g(xi^{k+1/2}) at the stopping iterate (READING 6)
    iterations: int             # number of xi-steps taken
    converged: bool
    residual: float             # |e^k - xi^{k+1/2}|_{L2} at the stopping iterate
    mean_v_norm: float          # |<v^k>| at the stopping iterate
    dual_est: float             # <A xibar, v^k>
    phi: np.ndarray             # node potential of the stopping iterate (zero mean)
    flux: np.ndarray            # A* v^k: the face fluxes, 3-field
    xi_half: np.ndarray         # xi^{k+1/2} at the stopping iterate
    v: np.ndarray               # multiplier v^k at the stopping iterate
    e: np.ndarray               # e^k at the stopping iterate
    rho: float                  # rho^k used in the stopping iterate
    history: list = field(default_factory=list)   # (k, residual, rho^k, energy) per iteration
    k: int = 0                  # global iteration index of the stopping state

    @property
    def mean_flux(self) -> np.ndarray:
        """<A* v^k>: geff is the support function of the mean fluxes of the admissible
        flows (max-flow form eq:CCMF_FFT_problemA), so at the optimum this is the
        gradient of its 1-homogeneous extension in the load xibar."""
        return self.flux.reshape(3, -1).mean(axis=1)


def rho_initial(gamma: np.ndarray) -> float:
    """READING 3: rho^0 = smallest positive crack resistance, the 'lower bound'
    penalty the paper uses for its constant-penalty runs (Sec. 4.2, Sec. 4.3)."""
    pos = gamma[gamma > 0]
    if pos.size == 0:
        return 1.0
    return float(pos.min())


def ltd_penalty(v_new, e_new):
    """Lorenz-Tran-Dinh scaling of Sec. 3.2: rho = |v|/|e| (None if undefined)."""
    ne = inner(e_new, e_new)
    nv = inner(v_new, v_new)
    if ne > 0.0 and nv > 0.0:
        return math.sqrt(nv / ne)
    return None


def bb_penalty(v_new, v, e_new, e):
    """Barzilai-Borwein scaling of Sec. 3.2, rho = <dv, de>/|de|^2, with the
    safeguard of READING 4: the estimate is used only where it is a reliable
    curvature estimate, i.e. the correlation <dv, de>/(|dv| |de|) is at least
    BB_MIN_CORRELATION; otherwise the Lorenz-Tran-Dinh scaling is used."""
    dv = v_new - v
    de = e_new - e
    num = inner(dv, de)
    den = inner(de, de)
    dvv = inner(dv, dv)
    if num > 0.0 and den > 0.0 and num >= BB_MIN_CORRELATION * math.sqrt(den * dvv):
        return num / den
    return ltd_penalty(v_new, e_new)


def admm_step(e, v, rho, xibar, gamma, delta):
    """One step of the damped ADMM (eq:CCMF_FFT_ADMM, second form) for a unit
    load ``xibar``; returns (xi^{k+1/2}, phi, e^{k+1}, v^{k+1}).

        xi^{k+1/2} = A xibar - (1/rho)(Id - A A* + A Gamma A*)(v - rho e) = P_K(e - v/rho)
        xi^{k+1}   = 2(1-delta) xi^{k+1/2} - (1-2 delta) e
        e^{k+1}    = [v + rho xi^{k+1} - P_C(v + rho xi^{k+1})] / rho   (Moreau's identity)
        v^{k+1}    = v + rho (xi^{k+1} - e^{k+1})
    """
    xi_half, phi = proj_K(e - v / rho, xibar)
    xi_new = 2.0 * (1.0 - delta) * xi_half - (1.0 - 2.0 * delta) * e
    z = v + rho * xi_new
    e_new = (z - proj_C(z, gamma)) / rho
    v_new = v + rho * (xi_new - e_new)
    return xi_half, phi, e_new, v_new


def admm_solve(gamma, xibar, tol=1e-4, delta=0.25, rule=RHO_BB, rho0=None,
               max_iter=20000, record=False, start=None) -> AdmmResult:
    """Solve the CCMF min-cut / max-flow pair by the damped ADMM of Sec. 3.2.

    Scheme (eq:CCMF_FFT_ADMM, damped form), with w^k = e^k - v^k/rho^k:
        xi^{k+1/2} = P_K(w^k)
        xi^{k+1}   = 2(1-delta) xi^{k+1/2} - (1-2 delta) e^k
        e^{k+1}    = [v^k + rho^k xi^{k+1} - P_C(v^k + rho^k xi^{k+1})] / rho^k
        v^{k+1}    = v^k + rho^k (xi^{k+1} - e^{k+1})
    stopped by the criterion of eq:convergence_criterion,
        |e^k - xi^{k+1/2}|_{L2} <= tol |<v^k>|,
    checked on the pair (e^k, xi^{k+1/2}) of the same iteration (READING 5).
    Penalty rules of Sec. 3.2: Barzilai-Borwein (default), Lorenz-Tran-Dinh,
    or constant rho^0; the Barzilai-Borwein safeguard is ``bb_penalty``'s.

    ``start = (e, v, rho, k)`` resumes from the state (e^k, v^k) with penalty
    rho^k at global iteration index k (a warm start); ``max_iter`` then counts
    the steps of this call and ``iterations`` reports them.
    """
    gamma = np.asarray(gamma, dtype=np.float64)
    if gamma.ndim != 3:
        raise ValueError("gamma must be a 3-d array")
    if not np.all(np.isfinite(gamma)) or np.any(gamma < 0):
        raise ValueError("gamma must be finite and non-negative")
    xb = np.asarray(xibar, dtype=np.float64).reshape(3)
    nrm = float(np.linalg.norm(xb))
    if not math.isfinite(nrm) or nrm == 0.0:
        raise ValueError("xibar must be a finite non-zero vector")
    xb = xb / nrm                       # the load is a unit normal (Sec. 2.1)
    if not (0.0 < delta < 1.0):
        raise ValueError("delta must lie in (0, 1)")
    dims = gamma.shape

    # READING 3: start on the planar crack e^0 = A xibar (phi = 0, so e^0 in K)
    # with a multiplier in the subdifferential of g at e^0: v^0 = gamma A xibar.
    e = A_xibar(xb, dims)
    v = gamma[None] * e
    r0 = rho_initial(gamma) if rho0 is None else float(rho0)
    if not (r0 > 0.0 and math.isfinite(r0)):
        raise ValueError("rho0 must be positive and finite")
    rho = r0
    k = 0
    if start is not None:
        e = np.array(start[0], dtype=np.float64).reshape((6,) + dims)
        v = np.array(start[1], dtype=np.float64).reshape((6,) + dims)
        rho = float(start[2])
        k = int(start[3])
    history = []
    # READING 7: if gamma vanishes identically, g = 0 on all of K and the first
    # xi-step is optimal; the criterion (right-hand side 0) is then taken as met.
    all_zero = not np.any(gamma > 0)

    steps = 0
    while True:
        xi_half, phi, e_new, v_new = admm_step(e, v, rho, xb, gamma, delta)
        d = e - xi_half
        res = math.sqrt(inner(d, d))
        mean_v = v.reshape(6, -1).mean(axis=1)
        mvn = float(np.linalg.norm(mean_v))
        E = energy(xi_half, gamma)
        if record:
            history.append((k, res, rho, E))
        last = (steps + 1 >= max_iter)
        done = res <= tol * mvn or all_zero
        if done or last:
            return AdmmResult(
                geff=E, iterations=steps + 1, converged=bool(done),
                residual=res, mean_v_norm=mvn,
                dual_est=inner(A_xibar(xb, dims), v),
                phi=phi, flux=A_adj(v), xi_half=xi_half, v=v, e=e, rho=rho,
                history=history, k=k)

        rho_new = rho
        if rule == RHO_BB:
            cand = bb_penalty(v_new, v, e_new, e)
        elif rule == RHO_LTD:
            cand = ltd_penalty(v_new, e_new)
        elif rule == RHO_CONST:
            cand = None
        else:
            raise ValueError(f"unknown penalty rule {rule!r}")
        if cand is not None and math.isfinite(cand) and cand > 0.0:
            # READING 4: a summable relative variation of the penalty (the
            # convergence condition of non-stationary Douglas-Rachford / ADMM)
            g = 1.0 + ETA0 / (1.0 + k / K0) ** 2
            rho_new = min(max(cand, rho / g), rho * g)
            rho_new = min(max(rho_new, r0 / RHO_CLAMP), r0 * RHO_CLAMP)

        e, v, rho = e_new, v_new, rho_new
        k += 1
        steps += 1


# ---------------------------------------------------------------------------
# Certified dual bound (strong duality, Sec. 2.1; max-flow form eq:CCMF_FFT_problemA)
# ---------------------------------------------------------------------------

def dual_certificate(gamma, xibar, v) -> tuple[float, float]:
    """Certified lower bound on geff from a multiplier v (6-field).

    y = A* v is a face flux.  Its div^- free part y_df = y - nabla^+ L^dagger div^- y
    (Helmholtz projection with the same spectral solve) has the same mean.  With
    sigma = max_x |A y_df|/gamma over gamma > 0, y_df / max(1, sigma) is feasible
    for the max-flow problem of eq:CCMF_FFT_problemA, so its objective
    <xibar, y_df>/max(1, sigma) is at most geff.  Returns (bound, sigma);
    the bound is -inf if a voxel with gamma = 0 carries flux.
    """
    gamma = np.asarray(gamma, dtype=np.float64)
    xb = np.asarray(xibar, dtype=np.float64).reshape(3)
    xb = xb / np.linalg.norm(xb)
    y = A_adj(v)
    y_df = y - grad_plus(laplace_pinv(div_minus(y)))
    ny = np.sqrt(np.sum(A_op(y_df) ** 2, axis=0))
    pos = gamma > 0
    if np.any(ny[~pos] > 1e-12 * max(1.0, float(ny.max()))):
        return -math.inf, math.inf
    sigma = float(np.max(ny[pos] / gamma[pos])) if np.any(pos) else 0.0
    obj = float(sum(xb[c] * y_df[c].mean() for c in range(3)))
    return obj / max(1.0, sigma), sigma


def envelope_gradient(gamma, xi_half) -> np.ndarray:
    """d geff / d gamma[x] = |xi*[x]| / N (Danskin / envelope theorem applied to
    the min-cut form eq:CCMF_FFT_problem_primal_final, whose objective is linear
    in gamma).  A supergradient where the optimal |xi*| is not unique."""
    n = gamma.size
    return np.sqrt(np.sum(xi_half * xi_half, axis=0)) / n
