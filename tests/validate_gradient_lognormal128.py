"""Full-size validation of the envelope gradient on the 128^3 log-normal workload
(kappa = exp(0.5 G), squared-exponential covariance, length 8, load (1,1,1)/sqrt3).

Not collected by pytest (it takes minutes of GPU time): run it directly on a GPU.
It solves in FP32 (tol 1e-5) and FP64, takes the envelope gradients, and checks
them against central finite differences of FP64 solves at 20 voxels (10 uniform,
10 from the top decile of |xi*|, seed 40) and along a smooth random direction.
Each FP64 geff is bracketed by the certified dual bound, so every difference
quotient carries an error bar.  Prints one JSON line per check and a summary.
"""

import json
import os
import sys
import time

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2103_05968_amd import microstructures as M  # noqa: E402
from paper_2103_05968_amd.ccmf import Plan  # noqa: E402

DEV = "cuda:0"
XB = [tuple(np.ones(3) / np.sqrt(3.0))]


def solve64(k, tol=1e-9, max_iter=60000):
    p = Plan(torch.as_tensor(k, dtype=torch.float64, device=DEV))
    r = p.solve(XB, tol=tol, max_iter=max_iter)
    cert, _ = p.certificate()
    g = p.grad_kappa([1.0])[0].cpu().numpy()
    p.close()
    return float(r.geff[0, 0]), float(cert[0, 0]), g, int(r.iterations[0, 0])


def main():
    k = M.config_c4()
    t0 = time.time()
    p32 = Plan(torch.as_tensor(k, dtype=torch.float32, device=DEV))
    r32 = p32.solve(XB, tol=1e-5, max_iter=40000)
    g32 = p32.grad_kappa([1.0])[0].double().cpu().numpy()
    f64, c64, g64, it64 = solve64(k)
    print(json.dumps(dict(check="base", geff32=float(r32.geff[0, 0]), iters32=int(r32.iterations[0, 0]),
                          geff64=f64, cert64=c64, iters64=it64, euler64=float((k * g64).sum()),
                          grad32_vs_64=float(np.abs(g32 - g64).max() / g64.max()),
                          seconds=time.time() - t0)), flush=True)
    rng = np.random.default_rng(40)
    order = np.argsort(g64.ravel())
    picks = list(rng.choice(k.size, 10, replace=False)) + list(rng.choice(order[-k.size // 10:], 10, replace=False))
    h = 0.05
    worst = 0.0
    for q in picks:
        v = np.unravel_index(int(q), k.shape)
        kp, km = k.copy(), k.copy()
        kp[v] *= 1 + h
        km[v] *= 1 - h
        fp, cp, _, _ = solve64(kp)
        fm, cm, _, _ = solve64(km)
        fd = (fp - fm) / (2 * h * k[v])
        bar = ((fp - cp) + (fm - cm)) / (2 * h * k[v])
        dev = abs(fd - g64[v]) / g64.max()
        worst = max(worst, dev)
        print(json.dumps(dict(check="voxel", voxel=[int(i) for i in v], fd=fd, fd_error_bar=bar,
                              grad64=float(g64[v]), grad32=float(g32[v]), rel_to_max=dev)), flush=True)
    # smooth direction: eta = a low-pass random field, relative step 1e-3
    eta = M.gaussian_lognormal(128, 8.0, 1.0, seed=41)
    eta = np.log(eta) * k
    t = 1e-3
    fp, cp, _, _ = solve64(k + t * eta)
    fm, cm, _, _ = solve64(k - t * eta)
    fd = (fp - fm) / (2 * t)
    dd64 = float((g64 * eta).sum())
    dd32 = float((g32 * eta).sum())
    print(json.dumps(dict(check="direction", fd=fd, fd_error_bar=((fp - cp) + (fm - cm)) / (2 * t),
                          grad64_dot=dd64, grad32_dot=dd32, rel=abs(fd - dd64) / abs(dd64))), flush=True)
    print(json.dumps(dict(check="summary", worst_voxel_dev_rel_to_max=worst, seconds=time.time() - t0)), flush=True)


if __name__ == "__main__":
    main()
