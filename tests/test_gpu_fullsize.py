"""Parity at the full sizes of the five workloads, through the C ABI, in the launch
configuration the benchmark uses (loads batched in one launch sequence, graph
replay, autotuned transform tiles).

A few iterations are compared element by element (on sampled voxels where the
field is large) with the FP64 oracle run on the host; converged results are
compared with stored oracle values (tests/golden/, written by
tests/golden/make_oracle_goldens.py), closed forms, or properties that hold at
any size (bounds, certificate, batch invariance, FP32 against FP64).
"""

import json
import os
import sys
import time

import numpy as np
import pytest
import torch

from oracle import ccmf_oracle as O
from paper_2103_05968_amd import microstructures as M

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_05968_amd import ccmf  # noqa: F401  (fails loudly if the library is missing)


def plan_of(kappa, dtype):
    from paper_2103_05968_amd.ccmf import Plan
    return Plan(torch.as_tensor(np.ascontiguousarray(kappa), dtype=dtype, device=DEV))


def planar_cut_bound(kappa, axis):
    """geff(e_axis) <= min over layers normal to e_axis of the layer mean (a flat cut)."""
    other = tuple(a for a in range(3) if a != axis)
    return float(kappa.mean(axis=other).min())


def sample_rel_err(got, want, rng, count=4096):
    idx = rng.choice(want.size, size=min(count, want.size), replace=False)
    g, w = got.ravel()[idx], want.ravel()[idx]
    return float(np.abs(g - w).max() / np.abs(want).max())


# --- 32^3 spheres, FP64, tol 1e-6 --------------------------------------------------

def test_spheres32_f64():
    cfg = M.CONFIGS["c1"]
    kap = M.config_c1()
    xb = cfg["loads"][0]
    banner("32^3 FP64: 40 iterations vs oracle")
    p = plan_of(kap, torch.float64)
    res = p.solve([xb], tol=1e-300, max_iter=40, want_phi=True, want_flux=True)
    ora = O.admm_solve(kap, xb, tol=1e-300, max_iter=40)
    assert abs(res.geff[0, 0] - ora.geff) <= 1e-10 * ora.geff
    phi = res.phi[0, 0].cpu().numpy()
    assert np.abs(phi - ora.phi).max() <= 1e-9 * np.abs(ora.phi).max()
    flux = res.flux[0, 0].cpu().numpy()
    assert np.abs(flux - ora.flux).max() <= 1e-9 * np.abs(ora.flux).max()
    banner("32^3 FP64: converged vs stored oracle value")
    gold = json.load(open(os.path.join(GOLDEN, "oracle_spheres32_f64.json")))
    res = p.solve([xb], tol=cfg["tol"], max_iter=100000)
    assert res.converged and gold["converged"]
    assert abs(res.geff[0, 0] - gold["geff"]) <= 1e-6 * gold["geff"]
    assert abs(int(res.iterations[0, 0]) - gold["iterations"]) <= 0.25 * gold["iterations"]
    assert np.abs(res.mean_flux[0, 0] - gold["mean_flux"]).max() <= 1e-5 * np.abs(gold["mean_flux"]).max()


# --- 256^3 UD fibres, FP32, loads e1 e2 e3 (the benchmark workload) ------------------

def test_ud_fibres256_f32_bench_configuration():
    cfg = M.CONFIGS["c2"]
    kap = M.config_c2()
    loads = cfg["loads"]
    rng = np.random.default_rng(7)
    banner("256^3: 2 iterations, FP32 and FP64, three loads batched")
    r32 = plan_of(kap, torch.float32).solve(loads, tol=1e-300, max_iter=2, want_phi=True)
    r64 = plan_of(kap, torch.float64).solve(loads, tol=1e-300, max_iter=2, want_phi=True)
    banner("256^3: oracle, 2 iterations of load e1 (FP64 NumPy, ~30 s)")
    t = time.perf_counter()
    ora = O.admm_solve(kap, loads[0], tol=1e-300, max_iter=2)
    banner(f"  oracle done in {time.perf_counter() - t:.0f} s")
    assert abs(r64.geff[0, 0] - ora.geff) <= 1e-10 * ora.geff
    assert sample_rel_err(r64.phi[0, 0].cpu().numpy(), ora.phi, rng) <= 1e-9
    assert abs(r32.geff[0, 0] - ora.geff) <= 1e-5 * ora.geff
    assert sample_rel_err(r32.phi[0, 0].cpu().numpy(), ora.phi, rng) <= 2e-5
    # e3 runs along the fibres: geff = mean kappa, reached at the first step
    banner("256^3: e3 closed form, converged")
    r = plan_of(kap, torch.float32).solve(loads, tol=cfg["tol"], max_iter=2)
    assert r.iterations[0, 2] == 1
    assert abs(r.geff[0, 2] - kap.mean()) <= 1e-6 * kap.mean()


# --- 64 x 128^3 polydisperse spheres x 3 loads, FP32, one batched launch ------------

@pytest.fixture(scope="module")
def poly_batch():
    t = time.perf_counter()
    kap = np.stack([M.config_c3(r) for r in range(64)])
    banner(f"generated 64 realizations of 128^3 in {time.perf_counter() - t:.0f} s")
    return kap


def test_poly_spheres_batch_invariance_and_oracle(poly_batch):
    cfg = M.CONFIGS["c3"]
    loads = cfg["loads"]
    banner("64 x 128^3 x 3: 10 iterations batched")
    batch = plan_of(poly_batch, torch.float32).solve(loads, tol=1e-300, max_iter=10, want_phi=True)
    for f, l in ((0, 1), (33, 0), (63, 2)):
        alone = plan_of(poly_batch[f], torch.float32).solve([loads[l]], tol=1e-300, max_iter=10, want_phi=True)
        assert alone.geff[0, 0] == batch.geff[f, l]
        assert torch.equal(alone.phi[0, 0], batch.phi[f, l])
    banner("128^3: oracle, 10 iterations of realization 0, load e2 (~20 s)")
    ora = O.admm_solve(poly_batch[0], loads[1], tol=1e-300, max_iter=10)
    assert abs(batch.geff[0, 1] - ora.geff) <= 1e-5 * ora.geff
    assert sample_rel_err(batch.phi[0, 1].cpu().numpy(), ora.phi, np.random.default_rng(3)) <= 2e-5


def test_poly_spheres_batch_converged(poly_batch):
    cfg = M.CONFIGS["c3"]
    loads = cfg["loads"]
    # most problems stop within 2000-8000 iterations; with the penalty safeguard of
    # the design notes (reading 4) a few percent stagnate just above the tolerance
    # for 20000-40000 iterations while geff has long settled
    banner("64 x 128^3 x 3: converged, tol 1e-4, one batched solve")
    t = time.perf_counter()
    p = plan_of(poly_batch, torch.float32)
    r = p.solve(loads, tol=cfg["tol"], max_iter=60000)
    el = time.perf_counter() - t
    its = r.iterations
    banner(f"  iterations min {its.min()} max {its.max()}, {el:.1f} s, "
           f"{poly_batch[0].size * its.sum() / el / 1e9:.1f} G voxel-iters/s")
    assert r.converged
    cert, _ = p.certificate()
    for f in range(64):
        for l in range(3):
            g = r.geff[f, l]
            assert poly_batch[f].min() * (1 - 1e-5) <= g <= planar_cut_bound(poly_batch[f], l) * (1 + 1e-5)
            assert cert[f, l] <= g * (1 + 1e-6)
    banner("128^3: realization 5 in FP64 to tol 1e-6 vs FP32 to tol 1e-5")
    g64 = plan_of(poly_batch[5], torch.float64).solve(loads, tol=1e-6, max_iter=40000)
    g32 = plan_of(poly_batch[5], torch.float32).solve(loads, tol=1e-5, max_iter=40000)
    assert np.abs(g32.geff - g64.geff).max() <= 1e-4 * g64.geff.max()


# --- 128^3 log-normal field, FP32 gradient ------------------------------------------

def test_lognormal128_gradient():
    cfg = M.CONFIGS["c4"]
    kap = M.config_c4()
    xb = cfg["loads"]
    banner("128^3 log-normal: FP32 solve to tol 1e-5, envelope gradient")
    p = plan_of(kap, torch.float32)
    r = p.solve(xb, tol=cfg["tol"], max_iter=60000)
    assert r.converged
    g = p.grad_kappa([1.0])[0].double().cpu().numpy()
    assert g.min() >= 0.0
    # Euler's identity of the 1-homogeneous energy
    assert abs(float((kap * g).sum()) - r.geff[0, 0]) <= 1e-5 * r.geff[0, 0]
    # directional central difference along a smooth perturbation of log kappa
    eta = np.log(M.gaussian_lognormal(128, 8.0, 1.0, seed=41))
    h = 0.02
    banner("128^3 log-normal: directional difference (two FP32 solves)")
    fp = plan_of(kap * np.exp(h * eta), torch.float32).solve(xb, tol=cfg["tol"], max_iter=60000).geff[0, 0]
    fm = plan_of(kap * np.exp(-h * eta), torch.float32).solve(xb, tol=cfg["tol"], max_iter=60000).geff[0, 0]
    want = float((g * kap * eta).sum())
    banner(f"  fd {(fp - fm) / (2 * h):.6e} envelope {want:.6e}")
    assert abs((fp - fm) / (2 * h) - want) <= 2e-3 * abs(r.geff[0, 0])


# --- 512^3 short fibres, FP32, tol 1e-4 ----------------------------------------------

def test_short_fibres512_f32():
    cfg = M.CONFIGS["c5"]
    t = time.perf_counter()
    kap = M.config_c5()
    banner(f"generated 512^3 short fibres in {time.perf_counter() - t:.0f} s")
    xb = cfg["loads"]
    rng = np.random.default_rng(11)
    banner("512^3: 20 iterations FP32 vs FP64 (FP64 pinned to the oracle at the smaller sizes)")
    r32 = plan_of(kap, torch.float32).solve(xb, tol=1e-300, max_iter=20, want_phi=True)
    r64 = plan_of(kap, torch.float64).solve(xb, tol=1e-300, max_iter=20, want_phi=True)
    assert abs(r32.geff[0, 0] - r64.geff[0, 0]) <= 1e-5 * r64.geff[0, 0]
    assert sample_rel_err(r32.phi[0, 0].cpu().numpy(), r64.phi[0, 0].cpu().numpy(), rng) <= 2e-5
    del r64
    torch.cuda.empty_cache()
    banner("512^3: converged FP32, tol 1e-4")
    t = time.perf_counter()
    p = plan_of(kap, torch.float32)
    r = p.solve(xb, tol=cfg["tol"], max_iter=20000)
    el = time.perf_counter() - t
    banner(f"  {int(r.iterations[0, 0])} iterations, {el:.1f} s, "
           f"{kap.size * int(r.iterations[0, 0]) / el / 1e9:.1f} G voxel-iters/s, geff {r.geff[0, 0]:.6f}")
    assert r.converged
    assert kap.min() <= r.geff[0, 0] <= planar_cut_bound(kap, 0) * (1 + 1e-5)
    cert, _ = p.certificate()
    assert cert[0, 0] <= r.geff[0, 0] * (1 + 1e-6)
