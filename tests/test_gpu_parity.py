"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: FP64 mode matches the oracle to 1e-6 relative on geff (fields of a
fixed number of iterations to ~1e-9); FP32 mode (FP32 fields, FP64
reductions) matches the FP64 oracle to 1e-4 relative on geff.
"""

import math
import sys

import numpy as np
import pytest
import torch

from oracle import ccmf_oracle as O
from paper_2103_05968_amd import microstructures as M

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_05968_amd import ccmf  # noqa: F401  (fails loudly if the library is missing)


def plan_of(kappa, dtype=torch.float64):
    from paper_2103_05968_amd.ccmf import Plan
    return Plan(torch.as_tensor(np.ascontiguousarray(kappa), dtype=dtype, device=DEV))


def dht_axis_np(x, axis):
    X = np.fft.fft(x, axis=axis)
    return X.real - X.imag


SIZES = [(16, 16, 16), (24, 20, 18), (15, 12, 10), (8, 1, 5), (1, 6, 7), (7, 9, 1)]


# --- the spectral solve ------------------------------------------------------------

@pytest.mark.parametrize("dims", SIZES + [(32, 32, 32)])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
def test_hartley_pass_matches_numpy(dims, dtype, tol, rng):
    banner(f"hartley {dims} {dtype}")
    p = plan_of(np.ones(dims), dtype)
    x = rng.standard_normal((2,) + dims)
    xt = torch.as_tensor(x, dtype=dtype, device=DEV)
    for axis in range(3):
        got = p.hartley_axis(xt, axis).double().cpu().numpy()
        want = dht_axis_np(x, axis + 1)
        scale = np.abs(want).max() + 1e-30
        assert np.abs(got - want).max() <= tol * scale * max(1, math.log2(dims[axis] + 1)), axis


@pytest.mark.parametrize("dims", SIZES + [(32, 32, 32), (64, 48, 40)])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 5e-5)])
def test_laplace_pinv_matches_oracle(dims, dtype, tol, rng):
    banner(f"laplace {dims} {dtype}")
    p = plan_of(np.ones(dims), dtype)
    r = rng.standard_normal((3,) + dims)
    got = p.laplace_pinv(torch.as_tensor(r, dtype=dtype, device=DEV)).double().cpu().numpy()
    for q in range(3):
        want = O.laplace_pinv(r[q])
        assert np.abs(got[q] - want).max() <= tol * (np.abs(want).max() + 1e-30)


# --- fixed number of iterations: iterate-level parity in FP64 ------------------------

def fixed_k(gamma, xibar, K, dtype=torch.float64, rule="bb", delta=0.25):
    p = plan_of(gamma, dtype)
    res = p.solve([xibar], tol=1e-300, max_iter=K, rule=rule, delta=delta, want_phi=True, want_flux=True)
    assert res.iterations[0, 0] == K and not res.converged
    ora = O.admm_solve(gamma, xibar, tol=1e-300, max_iter=K, rule=rule, delta=delta)
    return res, ora


@pytest.mark.parametrize("dims", [(16, 16, 16), (24, 20, 18), (15, 12, 10), (8, 1, 5), (12, 20, 16), (6, 40, 32)])
@pytest.mark.parametrize("rule,delta", [("bb", 0.25), ("ltd", 0.25), ("const", 0.5)])
def test_fixed_iterations_fp64_match_oracle(dims, rule, delta):
    banner(f"fixedK {dims} {rule} {delta}")
    gamma = M.boolean_spheres(dims, 3.0, 0.2, 10.0, 1.0, seed=11)
    xb = (0.48, 0.6, 0.64)
    res, ora = fixed_k(gamma, xb, 30, rule=rule, delta=delta)
    assert abs(res.geff[0, 0] - ora.geff) <= 1e-10 * ora.geff
    assert abs(res.residual[0, 0] - ora.residual) <= 1e-8 * ora.residual
    assert abs(res.dual_est[0, 0] - ora.dual_est) <= 1e-10 * abs(ora.dual_est)
    phi = res.phi[0, 0].cpu().numpy()
    assert np.abs(phi - ora.phi).max() <= 1e-9 * np.abs(ora.phi).max()
    flux = res.flux[0, 0].cpu().numpy()
    assert np.abs(flux - ora.flux).max() <= 1e-9 * np.abs(ora.flux).max()


# --- converged solves --------------------------------------------------------------

def test_converged_fp64_matches_oracle():
    banner("converged fp64 16^3")
    gamma = M.boolean_spheres((16, 16, 16), 3.0, 0.15, 0.3, 1.0, seed=1)
    ora = O.admm_solve(gamma, (1, 0, 0), tol=1e-6, max_iter=20000)
    res = plan_of(gamma).solve([(1, 0, 0)], tol=1e-6, max_iter=20000)
    assert res.converged and ora.converged
    assert abs(res.geff[0, 0] - ora.geff) <= 1e-6 * ora.geff
    # the penalty trajectory is rounding-sensitive over thousands of steps, so the
    # stopping iteration is compared loosely; geff is the parity quantity
    assert abs(int(res.iterations[0, 0]) - ora.iterations) <= 0.25 * ora.iterations


@pytest.mark.parametrize("dims", [(24, 20, 18), (16, 16, 16)])
def test_fp32_matches_fp64_oracle(dims):
    banner(f"fp32 vs oracle {dims}")
    gamma = M.boolean_spheres(dims, 3.0, 0.2, 10.0, 1.0, seed=5)
    xb = (1, 0, 0)
    ora = O.admm_solve(gamma, xb, tol=1e-7, max_iter=40000)
    res = plan_of(gamma, torch.float32).solve([xb], tol=1e-6, max_iter=40000)
    assert res.converged
    assert abs(res.geff[0, 0] - ora.geff) <= 1e-4 * ora.geff


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
def test_closed_forms(dtype, tol, rng):
    banner(f"closed forms {dtype}")
    # homogeneous: geff = kappa, converged after one step
    r = plan_of(np.full((20, 12, 10), 2.5), dtype).solve([(0.3, -0.4, 0.866)], tol=1e-8)
    assert r.converged and r.iterations[0, 0] == 1 and abs(r.geff[0, 0] - 2.5) <= tol * 2.5
    # laminate along e1: min for e1, mean for in-plane loads
    prof = rng.uniform(0.5, 3.0, 12)
    lam = M.laminate(prof, (12, 8, 6), axis=0)
    r = plan_of(lam, dtype).solve([(1, 0, 0), (0, 0.6, 0.8)], tol=1e-9 if dtype == torch.float64 else 1e-6)
    assert abs(r.geff[0, 0] - prof.min()) <= (1e-7 if dtype == torch.float64 else 1e-4) * prof.min()
    assert abs(r.geff[0, 1] - prof.mean()) <= (1e-7 if dtype == torch.float64 else 1e-4) * prof.mean()
    # extrusion along e3: the e3 load gives the mean
    g2 = rng.uniform(0.4, 3.0, (16, 12))
    ext = np.repeat(g2[:, :, None], 8, axis=2)
    r = plan_of(ext, dtype).solve([(0, 0, 1)], tol=1e-6)
    assert abs(r.geff[0, 0] - g2.mean()) <= (1e-10 if dtype == torch.float64 else 1e-5) * g2.mean()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_equals_single(dtype):
    banner(f"batched {dtype}")
    fields = np.stack([M.boolean_spheres((16, 12, 20), 3.0, 0.2, 5.0, 1.0, seed=s) for s in (21, 22)])
    loads = [(1, 0, 0), (0, 1, 0), (0.36, 0.48, 0.8)]
    batched = plan_of(fields, dtype).solve(loads, tol=1e-5, max_iter=5000)
    for f in range(2):
        single_plan = plan_of(fields[f], dtype)
        for l, xb in enumerate(loads):
            s = single_plan.solve([xb], tol=1e-5, max_iter=5000)
            assert s.geff[0, 0] == batched.geff[f, l]
            assert s.iterations[0, 0] == batched.iterations[f, l]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_graph_replay_equals_eager_launches(dtype):
    banner(f"graph vs eager {dtype}")
    g = M.boolean_spheres((20, 16, 12), 3.0, 0.2, 5.0, 1.0, seed=9)
    p = plan_of(g, dtype)
    loads = [(1, 0, 0), (0.36, 0.48, 0.8)]
    for K, tol in [(7, 1e-300), (400, 1e-5)]:
        a = p.solve(loads, tol=tol, max_iter=K, check_every=6, want_phi=True)
        b = p.solve(loads, tol=tol, max_iter=K, check_every=6, want_phi=True, eager=True)
        assert np.array_equal(a.geff, b.geff) and np.array_equal(a.iterations, b.iterations)
        assert torch.equal(a.phi, b.phi)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_single_sphere_golden_full_size(dtype):
    """Sec. 4.2 at the paper's size: 64^3, sphere of diameter 32, contrast 10, e_x,
    tol 1e-4 -> geff = gamma_matrix (tests/golden/single_sphere_sec4_2.json)."""
    import json
    import os
    banner(f"single sphere 64^3 {dtype}")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "single_sphere_sec4_2.json")))
    g = M.single_sphere(gold["grid"][0], gold["sphere_diameter"], gold["gamma_sphere"], gold["gamma_matrix"])
    p = plan_of(g, dtype)
    r = p.solve([gold["load"]], tol=gold["tol"], max_iter=40000)
    cert, _ = p.certificate()
    assert r.converged
    assert abs(r.geff[0, 0] - gold["geff"]) <= 1e-3 * gold["geff"]
    assert cert[0, 0] <= gold["geff"] * (1 + 1e-6)


def test_certificate_matches_oracle_and_brackets():
    banner("certificate")
    g = M.boolean_spheres((16, 12, 10), 3.0, 0.2, 5.0, 1.0, seed=13)
    xb = (0.48, 0.6, 0.64)
    # fixed iterations: the GPU certificate equals the oracle's for the same iterate
    p = plan_of(g)
    res = p.solve([xb], tol=1e-300, max_iter=25)
    cert, sig = p.certificate()
    ora = O.admm_solve(g, xb, tol=1e-300, max_iter=25)
    ocert, osig = O.dual_certificate(g, xb, ora.v)
    assert abs(sig[0, 0] - osig) <= 1e-9 * osig
    assert abs(cert[0, 0] - ocert) <= 1e-9 * abs(ocert)
    # converged: cert <= geff with a small gap, in both precisions
    for dtype, gap in [(torch.float64, 1e-5), (torch.float32, 1e-4)]:
        p = plan_of(g, dtype)
        res = p.solve([xb, (1, 0, 0)], tol=1e-7 if dtype == torch.float64 else 1e-6, max_iter=40000)
        cert, sig = p.certificate()
        assert np.all(cert <= res.geff * (1 + 1e-6))
        assert np.all(res.geff - cert <= gap * res.geff)


def test_gradient_fp64_matches_oracle_and_fd():
    banner("gradient fp64")
    rng = np.random.default_rng(3)
    gamma = rng.uniform(0.5, 2.5, (6, 5, 4))
    xb = (0.48, 0.6, 0.64)
    p = plan_of(gamma)
    res = p.solve([xb], tol=1e-12, max_iter=200000)
    ora = O.admm_solve(gamma, xb, tol=1e-12, max_iter=200000)
    g = p.grad_kappa([1.0])[0].cpu().numpy()
    want = O.envelope_gradient(gamma, ora.xi_half)
    assert abs(res.geff[0, 0] - ora.geff) <= 1e-9 * ora.geff
    assert np.abs(g - want).max() <= 1e-6 * want.max()
    assert abs(np.sum(gamma * g) - res.geff[0, 0]) <= 1e-10
    h = 1e-4
    for idx in [(0, 0, 0), (2, 3, 1), tuple(np.unravel_index(np.argmax(g), g.shape))]:
        gp, gm = gamma.copy(), gamma.copy()
        gp[idx] += h
        gm[idx] -= h
        fp = plan_of(gp).solve([xb], tol=1e-12, max_iter=200000).geff[0, 0]
        fm = plan_of(gm).solve([xb], tol=1e-12, max_iter=200000).geff[0, 0]
        assert abs((fp - fm) / (2 * h) - g[idx]) <= 2e-4 * g.max()


def test_gradient_single_voxel_fd_lognormal_fp64():
    """Central differences of geff at 20 voxels (10 uniform, 10 from the top decile
    of |xi*|) of a log-normal field, FP64, scaled-down cell of the differentiation
    workload; the FP32 gradient is compared with the FP64 one."""
    banner("gradient fd lognormal")
    k = M.gaussian_lognormal(8, 2.0, 0.5, seed=4)
    xb = tuple(np.ones(3) / np.sqrt(3.0))
    p = plan_of(k)
    p.solve([xb], tol=1e-10, max_iter=100000)
    g = p.grad_kappa([1.0])[0].cpu().numpy()
    g32 = plan_of(k, torch.float32)
    g32.solve([xb], tol=1e-6, max_iter=100000)
    gr32 = g32.grad_kappa([1.0])[0].cpu().numpy()
    assert np.abs(gr32 - g).max() <= 5e-3 * g.max()
    rng = np.random.default_rng(40)
    flat = np.argsort(g.ravel())
    idx = list(rng.choice(k.size, 10, replace=False)) + list(rng.choice(flat[-k.size // 10:], 10, replace=False))
    h = 1e-2
    for n, q in enumerate(idx):
        v = np.unravel_index(q, k.shape)
        kp, km = k.copy(), k.copy()
        kp[v] += h * k[v]
        km[v] -= h * k[v]
        fp = plan_of(kp).solve([xb], tol=1e-9, max_iter=100000).geff[0, 0]
        fm = plan_of(km).solve([xb], tol=1e-9, max_iter=100000).geff[0, 0]
        fd = (fp - fm) / (2 * h * k[v])
        banner(f"  voxel {n} {v}: fd {fd:.6e} grad {g[v]:.6e}")
        assert abs(fd - g[v]) <= 1e-2 * g.max(), (v, fd, g[v])


def test_autograd_function():
    banner("autograd")
    from paper_2103_05968_amd.ccmf import effective_crack_energy
    rng = np.random.default_rng(4)
    k = torch.as_tensor(rng.uniform(0.5, 2.0, (8, 6, 5)), dtype=torch.float64, device=DEV).requires_grad_(True)
    ge = effective_crack_energy(k, [(1, 0, 0), (0, 0, 1)], tol=1e-10, max_iter=100000)
    (ge[0] + 2.0 * ge[1]).backward()
    assert k.grad is not None and k.grad.shape == k.shape
    # Euler's identity for the 1-homogeneous sum
    total = float(ge[0] + 2.0 * ge[1])
    assert abs(float((k.detach() * k.grad).sum()) - total) <= 1e-8 * total


def test_invalid_inputs_are_rejected():
    banner("errors")
    from paper_2103_05968_amd._lib import CcmfError
    bad = np.ones((4, 4, 4))
    bad[1, 2, 3] = -1.0
    with pytest.raises(CcmfError, match="negative or non-finite"):
        plan_of(bad)
    bad[1, 2, 3] = np.nan
    with pytest.raises(CcmfError):
        plan_of(bad)
    p = plan_of(np.ones((4, 4, 4)))
    with pytest.raises(CcmfError, match="zero"):
        p.solve([(0, 0, 0)], tol=1e-4)
    with pytest.raises(CcmfError, match="tol"):
        p.solve([(1, 0, 0)], tol=0.0)
    with pytest.raises(CcmfError, match="delta"):
        p.solve([(1, 0, 0)], tol=1e-4, delta=1.5)
    with pytest.raises(CcmfError):
        p.grad_kappa([1.0])   # no solve yet


def test_pores_and_all_zero_field():
    banner("pores")
    z = plan_of(np.zeros((6, 5, 4))).solve([(1, 0, 0)], tol=1e-6)
    assert z.converged and z.iterations[0, 0] == 1 and z.geff[0, 0] == 0.0
    g = M.boolean_spheres((12, 12, 12), 2.5, 0.2, 0.0, 1.0, seed=7)
    ora = O.admm_solve(g, (1, 0, 0), tol=1e-300, max_iter=40)
    res = plan_of(g).solve([(1, 0, 0)], tol=1e-300, max_iter=40)
    assert abs(res.geff[0, 0] - ora.geff) <= 1e-10 * ora.geff


def test_not_converged_is_reported():
    banner("not converged")
    from paper_2103_05968_amd._lib import CcmfError
    g = M.boolean_spheres((8, 8, 8), 2.0, 0.2, 5.0, 1.0, seed=2)
    p = plan_of(g)
    r = p.solve([(1, 0, 0)], tol=1e-12, max_iter=7)
    assert not r.converged and r.iterations[0, 0] == 7
    with pytest.raises(CcmfError):
        p.solve([(1, 0, 0)], tol=1e-12, max_iter=7, raise_not_converged=True)


@pytest.mark.parametrize("walk", ["2", "3"])
def test_tile_walk(walk, rng, monkeypatch):
    """Transform passes with each block walking several tiles (forced through the
    diagnostic CCMF_TILE_WALK; the autotuner picks the walk by time, so small cases
    may never take it): ragged last tiles (24 and 6 lines per outer index), a last
    walk shorter than the others, and odd line counts (no vector loads).  Results
    must equal the single-tile walk bit for bit and match numpy and the oracle."""
    banner(f"tile walk {walk}")
    for dims in [(32, 64, 24), (16, 32, 6), (16, 32, 5), (64, 16, 32)]:
        for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 2e-5)):
            x = rng.standard_normal((2,) + dims)
            xt = torch.as_tensor(x, dtype=dtype, device=DEV)
            monkeypatch.setenv("CCMF_TILE_WALK", "1")
            p1 = plan_of(np.ones(dims), dtype)
            one = [p1.hartley_axis(xt, axis) for axis in range(3)] + [p1.laplace_pinv(xt)]
            monkeypatch.setenv("CCMF_TILE_WALK", walk)
            p = plan_of(np.ones(dims), dtype)
            for axis in range(3):
                got = p.hartley_axis(xt, axis)
                assert torch.equal(got, one[axis]), (dims, axis)
                want = dht_axis_np(x, axis + 1)
                got = got.double().cpu().numpy()
                assert np.abs(got - want).max() <= tol * np.abs(want).max() * 8, (dims, axis)
            got = p.laplace_pinv(xt)
            assert torch.equal(got, one[3]), dims
            want = O.laplace_pinv(x[0])
            assert np.abs(got[0].double().cpu().numpy() - want).max() <= 5 * tol * np.abs(want).max(), dims
        gamma = M.boolean_spheres(dims, 2.0, 0.2, 5.0, 1.0, seed=3)
        res = plan_of(gamma).solve([(0.48, 0.6, 0.64)], tol=1e-300, max_iter=12, autotune=False, want_phi=True)
        ora = O.admm_solve(gamma, (0.48, 0.6, 0.64), tol=1e-300, max_iter=12)
        assert abs(res.geff[0, 0] - ora.geff) <= 1e-10 * ora.geff, dims
        assert np.abs(res.phi[0, 0].cpu().numpy() - ora.phi).max() <= 1e-9 * np.abs(ora.phi).max(), dims


@pytest.mark.parametrize("variant", ["0", "1", "2"])
def test_fft_plan_variants(variant, rng, monkeypatch):
    """Every register-blocked FFT plan variant (forced through the diagnostic
    CCMF_FFT_VARIANT) in every pass: single Hartley passes against numpy, the
    pseudo-inverse against the oracle, and a fixed-K solve against the oracle."""
    banner(f"fft plan variant {variant}")
    monkeypatch.setenv("CCMF_FFT_VARIANT", variant)
    for dims in [(32, 16, 8), (4, 128, 256), (256, 2, 4)]:
        for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 2e-5)):
            p = plan_of(np.ones(dims), dtype)
            x = rng.standard_normal((2,) + dims)
            xt = torch.as_tensor(x, dtype=dtype, device=DEV)
            for axis in range(3):
                got = p.hartley_axis(xt, axis).double().cpu().numpy()
                want = dht_axis_np(x, axis + 1)
                assert np.abs(got - want).max() <= tol * np.abs(want).max() * 8, (dims, axis)
            got = p.laplace_pinv(xt).double().cpu().numpy()
            want = O.laplace_pinv(x[0])
            assert np.abs(got[0] - want).max() <= 5 * tol * np.abs(want).max(), dims
        gamma = M.boolean_spheres(dims, 2.0, 0.2, 5.0, 1.0, seed=3)
        res = plan_of(gamma).solve([(0.48, 0.6, 0.64)], tol=1e-300, max_iter=12, autotune=False)
        ora = O.admm_solve(gamma, (0.48, 0.6, 0.64), tol=1e-300, max_iter=12)
        assert abs(res.geff[0, 0] - ora.geff) <= 1e-10 * ora.geff, dims
