"""Closed forms of the discrete problem shared by the oracle pins and the GPU tests."""

import math

import numpy as np
import scipy.optimize


def laminate_oblique_gradient(profile, xibar):
    """Gradient in xibar of the 1-homogeneous laminate formula |xi_1| c + |xi_perp| mean
    sqrt(gamma^2 - c^2) maximised over c (envelope theorem at the maximiser c*)."""
    xb = np.asarray(xibar, float) / np.linalg.norm(xibar)
    a, b = abs(xb[0]), math.hypot(xb[1], xb[2])
    gmin = profile.min()

    def neg(c):
        return -(a * c + b * np.mean(np.sqrt(np.maximum(profile ** 2 - c * c, 0.0))))

    res = scipy.optimize.minimize_scalar(neg, bounds=(0.0, gmin), method="bounded",
                                         options=dict(xatol=1e-14))
    c = min([0.0, gmin, res.x], key=neg)
    s = np.mean(np.sqrt(np.maximum(profile ** 2 - c * c, 0.0)))
    return np.array([math.copysign(c, xb[0]), s * xb[1] / b, s * xb[2] / b])
