"""Seeded synthetic crack-resistance fields (voxel images of kappa = gamma).

This module only builds inputs: it holds none of the solver's arithmetic and
is shared by the solver's tests, the benchmark and the checks that run the
plain reference implementation, so that both sides consume identical bytes.

The paper's own microstructures (mechanical-contraction fibre packings, SAM
short-fibre composites, sand-core scans) are not available; the recipes below
are synthetic stand-ins with the shapes, phase contrasts and volume fractions
of its workloads (single sphere of Sec. 4.2, UD fibres of Sec. 4.3, short
fibres of Sec. 4.4, porous spheres of Sec. 4.5).

Conventions shared by all generators:

* the grid is periodic, voxel (i, j, k) has its centre at (i+1/2, j+1/2, k+1/2)
  (Sec. 2.2: the crack resistance is sampled at voxel centres);
* a voxel belongs to an inclusion iff its centre lies in it, measured with
  periodic minimum-image distances ("interface-free": binary phases);
* randomness comes from ``numpy.random.default_rng(seed)`` only.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "voxel_centres", "boolean_spheres", "rsa_discs_extruded", "rsa_polydisperse_spheres",
    "hard_particle_packing", "packed_discs_extruded", "packed_spheres",
    "gaussian_lognormal", "boolean_cylinders", "single_sphere", "laminate",
    "config_c1", "config_c2", "config_c3", "config_c4", "config_c5", "CONFIGS",
]


def voxel_centres(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) + 0.5


def _periodic_sq_dist_axis(centres: np.ndarray, c: float, n: int) -> np.ndarray:
    d = np.abs(centres - c)
    d = np.minimum(d, n - d)
    return d * d


def _ball_mask(dims, centre, radius) -> np.ndarray:
    """Voxels whose centre lies within `radius` of `centre` (periodic), full grid."""
    n1, n2, n3 = dims
    d1 = _periodic_sq_dist_axis(voxel_centres(n1), centre[0], n1)
    d2 = _periodic_sq_dist_axis(voxel_centres(n2), centre[1], n2)
    d3 = _periodic_sq_dist_axis(voxel_centres(n3), centre[2], n3)
    return (d1[:, None, None] + d2[None, :, None] + d3[None, None, :]) <= radius * radius


def _mark_ball(mask: np.ndarray, centre, radius) -> int:
    """Set `mask` on the voxels of the periodic ball (centre, radius); visits only the
    ball's bounding box.  Same voxel set as _ball_mask.  Returns the number of
    voxels newly set."""
    idx = []
    for c, n in zip(centre, mask.shape):
        lo = int(np.floor(c - radius - 0.5))
        hi = int(np.ceil(c + radius - 0.5))
        ii = np.arange(lo, hi + 1)
        if ii.size >= n:
            ii = np.arange(n)
        ii = np.unique(ii % n)
        d = np.abs(ii + 0.5 - c)
        d = np.minimum(d, n - d)
        idx.append((ii, d * d))
    (i1, q1), (i2, q2), (i3, q3) = idx
    inside = (q1[:, None, None] + q2[None, :, None] + q3[None, None, :]) <= radius * radius
    sub = mask[np.ix_(i1, i2, i3)]
    added = int(np.count_nonzero(inside & ~sub))
    mask[np.ix_(i1, i2, i3)] = sub | inside
    return added


def boolean_spheres(dims, radius, target_fraction, kappa_incl, kappa_matrix, seed):
    """Overlapping spheres with centres uniform in the cell, added one at a time
    until the inclusion voxel fraction reaches `target_fraction`."""
    rng = np.random.default_rng(seed)
    dims = tuple(int(d) for d in dims)
    incl = np.zeros(dims, dtype=bool)
    count, total = 0, incl.size
    while count < target_fraction * total:
        c = rng.uniform(0.0, 1.0, 3) * np.array(dims, dtype=np.float64)
        count += _mark_ball(incl, c, radius)
    return np.where(incl, kappa_incl, kappa_matrix).astype(np.float64)


def _periodic_dist(a: np.ndarray, b: np.ndarray, box: np.ndarray) -> np.ndarray:
    d = np.abs(a - b)
    d = np.minimum(d, box - d)
    return np.sqrt(np.sum(d * d, axis=-1))


def rsa_discs_extruded(n12, n3, radius, target_fraction, kappa_fibre, kappa_matrix, seed):
    """Aligned cylindrical fibres along e3: random sequential addition of discs of
    `radius` in the e1-e2 plane (centres uniform, accepted if the periodic
    distance to every accepted centre is at least 2*radius), stopped once the
    voxel area fraction reaches `target_fraction`, then extruded along e3."""
    rng = np.random.default_rng(seed)
    box = np.array([n12, n12], dtype=np.float64)
    area = np.zeros((n12, n12), dtype=bool)
    xc = voxel_centres(n12)
    centres = np.empty((0, 2))
    attempts = 0
    while area.mean() < target_fraction:
        attempts += 1
        if attempts > 10_000_000:
            raise RuntimeError("RSA did not reach the target fraction")
        c = rng.uniform(0.0, 1.0, 2) * box
        if centres.shape[0] and np.any(_periodic_dist(centres, c, box) < 2.0 * radius):
            continue
        centres = np.vstack([centres, c])
        d1 = _periodic_sq_dist_axis(xc, c[0], n12)
        d2 = _periodic_sq_dist_axis(xc, c[1], n12)
        area |= (d1[:, None] + d2[None, :]) <= radius * radius
    kap2 = np.where(area, kappa_fibre, kappa_matrix).astype(np.float64)
    return np.repeat(kap2[:, :, None], n3, axis=2), centres


def hard_particle_packing(ndim, count, box, fraction, seed, equilibrate=50, max_sweeps=50_000):
    """Random non-overlapping packing of `count` equal discs (ndim 2) or spheres
    (ndim 3) filling `fraction` of the periodic cube [0, box)^ndim, by Monte-Carlo
    compression: random sequential addition at a radius giving 20 % fill, then
    sweeps of random single-particle moves (rejected on overlap, step adapted to
    ~40 % acceptance), after each of which the radius grows to half the smallest
    centre distance, capped at the target; `equilibrate` further sweeps at the
    target radius.  A stand-in for the mechanical-contraction packings of Sec. 4.3
    and Sec. 4.5 (dense random packings of equal particles).
    Returns (centres [count, ndim], radius)."""
    rng = np.random.default_rng(seed)
    unit = math.pi if ndim == 2 else 4.0 * math.pi / 3.0
    big = (fraction * box ** ndim / (count * unit)) ** (1.0 / ndim)
    r = big * min(1.0, (0.2 / fraction) ** (1.0 / ndim))

    def sq_dists(x, c):
        d = np.abs(x - c)
        d = np.minimum(d, box - d)
        return np.sum(d * d, axis=-1)

    x = np.empty((0, ndim))
    attempts = 0
    while x.shape[0] < count:
        attempts += 1
        if attempts > 10_000_000:
            raise RuntimeError("initial insertion failed")
        c = rng.uniform(0.0, box, ndim)
        if x.shape[0] and np.min(sq_dists(x, c)) < 4.0 * r * r:
            continue
        x = np.vstack([x, c])
    step, settled = r, 0
    for _ in range(max_sweeps):
        accepted = 0
        for i in rng.permutation(count):
            t = (x[i] + rng.uniform(-step, step, ndim)) % box
            q = sq_dists(x, t)
            q[i] = np.inf
            if q.min() >= 4.0 * r * r:
                x[i] = t
                accepted += 1
        q = sq_dists(x[:, None, :], x[None, :, :])
        np.fill_diagonal(q, np.inf)
        r = min(big, 0.5 * math.sqrt(q.min()))
        step = min(big, step * (1.2 if accepted > 0.4 * count else 0.8))
        if r >= big:
            settled += 1
            if settled >= equilibrate:
                return x, big
    raise RuntimeError("packing did not reach the target fraction")


def packed_discs_extruded(n12, n3, count, fraction, kappa_fibre, kappa_matrix, seed):
    """Aligned fibres along e3: a dense random packing of `count` equal discs
    (hard_particle_packing) in the e1-e2 plane, voxelised and extruded along e3
    (the unidirectional composite of Sec. 4.3)."""
    centres, radius = hard_particle_packing(2, count, float(n12), fraction, seed)
    xc = voxel_centres(n12)
    area = np.zeros((n12, n12), dtype=bool)
    for c in centres:
        area |= (_periodic_sq_dist_axis(xc, c[0], n12)[:, None]
                 + _periodic_sq_dist_axis(xc, c[1], n12)[None, :]) <= radius * radius
    kap2 = np.where(area, kappa_fibre, kappa_matrix).astype(np.float64)
    return np.repeat(kap2[:, :, None], n3, axis=2)


def packed_spheres(n, count, fraction, kappa_incl, kappa_matrix, seed):
    """n^3 cell with a dense random packing of `count` equal spheres
    (hard_particle_packing); kappa_incl = 0 gives the pores of Sec. 4.5."""
    centres, radius = hard_particle_packing(3, count, float(n), fraction, seed)
    incl = np.zeros((n, n, n), dtype=bool)
    for c in centres:
        _mark_ball(incl, c, radius)
    return np.where(incl, kappa_incl, kappa_matrix).astype(np.float64)


def rsa_polydisperse_spheres(n, rmin, rmax, target_fraction, kappa_incl, kappa_matrix, seed):
    """Non-overlapping spheres, radii uniform in [rmin, rmax], random sequential
    addition (accepted if the periodic centre distance is at least r_a + r_b),
    stopped once the inclusion voxel fraction reaches `target_fraction`."""
    rng = np.random.default_rng(seed)
    dims = (n, n, n)
    box = np.array(dims, dtype=np.float64)
    incl = np.zeros(dims, dtype=bool)
    centres = np.zeros((0, 3))
    radii = np.zeros((0,))
    count, total = 0, incl.size
    attempts = 0
    while count < target_fraction * total:
        attempts += 1
        if attempts > 10_000_000:
            raise RuntimeError("RSA did not reach the target fraction")
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0.0, 1.0, 3) * box
        if centres.shape[0] and np.any(_periodic_dist(centres, c, box) < radii + r):
            continue
        centres = np.vstack([centres, c])
        radii = np.append(radii, r)
        count += _mark_ball(incl, c, r)
    return np.where(incl, kappa_incl, kappa_matrix).astype(np.float64)


def gaussian_lognormal(n, corr_len, sigma, seed):
    """kappa = exp(sigma * G), G a periodic Gaussian random field with covariance
    C(r) = exp(-r^2 / (2 corr_len^2)): white noise N(0, 1) filtered in Fourier
    space by the square root of the (non-negative part of the) periodic spectrum
    of C, then normalised to sample mean 0 and sample variance 1."""
    rng = np.random.default_rng(seed)
    x = np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64)
    r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    cov = np.exp(-r2 / (2.0 * corr_len * corr_len))
    spec = np.fft.rfftn(cov).real
    spec = np.maximum(spec, 0.0)
    noise = rng.standard_normal((n, n, n))
    g = np.fft.irfftn(np.fft.rfftn(noise) * np.sqrt(spec), s=(n, n, n))
    g = (g - g.mean()) / g.std()
    return np.exp(sigma * g)


def boolean_cylinders(n, radius, length, target_fraction, kappa_fibre, kappa_matrix, seed):
    """Overlapping flat-capped cylinders (radius, length) with isotropic axis
    directions (uniform on the sphere) and uniform centres, added until the
    fibre voxel fraction reaches `target_fraction`."""
    rng = np.random.default_rng(seed)
    incl = np.zeros((n, n, n), dtype=bool)
    total = n ** 3
    count = 0
    half = 0.5 * length
    reach = int(math.ceil(radius)) + 1
    off = np.arange(-reach, reach + 1)
    o1, o2, o3 = np.meshgrid(off, off, off, indexing="ij")
    o1, o2, o3 = o1.ravel(), o2.ravel(), o3.ravel()
    while count < target_fraction * total:
        u = rng.standard_normal(3)
        d = u / np.linalg.norm(u)
        c = rng.uniform(0.0, 1.0, 3) * n
        steps = np.arange(-half, half + 1.0, 1.0)
        pts = c[None, :] + steps[:, None] * d[None, :]
        base = np.floor(pts).astype(np.int64)
        # candidate voxels: a small cube around each sample point on the axis
        ci = (base[:, 0:1] + o1[None, :]).ravel()
        cj = (base[:, 1:2] + o2[None, :]).ravel()
        ck = (base[:, 2:3] + o3[None, :]).ravel()
        lin = np.unique(((ci % n) * n + (cj % n)) * n + (ck % n))
        # rebuild unwrapped candidate coordinates nearest to the centre
        vi = lin // (n * n)
        vj = (lin // n) % n
        vk = lin % n
        p = np.stack([vi, vj, vk], axis=1).astype(np.float64) + 0.5 - c[None, :]
        p -= n * np.round(p / n)
        t = p @ d
        perp = p - t[:, None] * d[None, :]
        inside = (np.abs(t) <= half) & (np.sum(perp * perp, axis=1) <= radius * radius)
        sel = lin[inside]
        flat = incl.reshape(-1)
        new = ~flat[sel]
        count += int(np.count_nonzero(new))
        flat[sel] = True
    return np.where(incl, kappa_fibre, kappa_matrix).astype(np.float64)


def single_sphere(n, diameter, kappa_sphere, kappa_matrix):
    """One sphere of the given diameter at the cell centre (Sec. 4.2's setup)."""
    c = np.array([n / 2.0] * 3)
    m = _ball_mask((n, n, n), c, diameter / 2.0)
    return np.where(m, kappa_sphere, kappa_matrix).astype(np.float64)


def laminate(profile, dims, axis=0):
    """A field that depends on one coordinate only (a layered medium)."""
    profile = np.asarray(profile, dtype=np.float64)
    shape = [1, 1, 1]
    shape[axis] = profile.size
    reps = list(dims)
    reps[axis] = 1
    return np.tile(profile.reshape(shape), reps)


# --- the five workloads --------------------------------------------------------

def config_c1():
    """32^3, overlapping spheres r = 4, ~15 % inclusions with kappa 0.3 in a matrix of 1."""
    return boolean_spheres((32, 32, 32), 4.0, 0.15, 0.3, 1.0, seed=1)


def config_c2(n=256):
    """n^3, aligned fibres along e3 (r = 5, non-overlapping, 20 %), kappa 10 / 1."""
    kap, _ = rsa_discs_extruded(n, n, 5.0, 0.20, 10.0, 1.0, seed=2)
    return kap


def config_c3(realization, n=128):
    """n^3 polydisperse non-overlapping spheres (r ~ U(3, 8), 25 %), kappa 0.2 / 1."""
    return rsa_polydisperse_spheres(n, 3.0, 8.0, 0.25, 0.2, 1.0, seed=1000 + int(realization))


def config_c4(n=128):
    """n^3 log-normal field exp(0.5 G), squared-exponential covariance, length 8."""
    return gaussian_lognormal(n, 8.0, 0.5, seed=4)


def config_c5(n=512):
    """n^3 isotropic short fibres (r = 2, length 80, 15 %), kappa 5 / 1."""
    return boolean_cylinders(n, 2.0, 80.0, 0.15, 5.0, 1.0, seed=5)


CONFIGS = {
    "c1": dict(name="spheres32_f64", dims=(32, 32, 32), loads=[(1.0, 0.0, 0.0)], tol=1e-6),
    "c2": dict(name="ud_fibres256_f32", dims=(256, 256, 256),
               loads=[(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)], tol=1e-5),
    "c3": dict(name="poly_spheres128x64_f32", dims=(128, 128, 128),
               loads=[(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)], tol=1e-4),
    "c4": dict(name="lognormal128_f32", dims=(128, 128, 128),
               loads=[tuple(np.ones(3) / math.sqrt(3.0))], tol=1e-5),
    "c5": dict(name="short_fibres512_f32", dims=(512, 512, 512), loads=[(1.0, 0.0, 0.0)], tol=1e-4),
}
