"""Trapezoid-rule discretization of a closed curve for the C ABI (Sec. 2.3).

Nodes y_j = z(2 pi j / N), weights w_j = (2 pi / N) |z'(t_j)|, outward normals
(z2', -z1') / |z'| of a counter-clockwise curve, and the signed curvature needed by the
Kress quadrature.  The curve object supplies z, z', z'' at parameter values.
"""
from __future__ import annotations

import math

import numpy as np


def discretize(curve, N: int):
    t = 2.0 * math.pi * np.arange(N) / N
    z, dz, d2z = curve.sample(t)
    sp = np.sqrt(dz[:, 0] ** 2 + dz[:, 1] ** 2)
    nodes = np.ascontiguousarray(z)
    weights = (2.0 * math.pi / N) * sp
    normals = np.ascontiguousarray(np.stack([dz[:, 1] / sp, -dz[:, 0] / sp], axis=1))
    curvature = (dz[:, 0] * d2z[:, 1] - dz[:, 1] * d2z[:, 0]) / sp ** 3
    return nodes, weights, normals, curvature
