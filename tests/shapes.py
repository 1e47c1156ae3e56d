"""Shape measurements of a grown crystal (test helpers): distances along rays to the phi = 0 contour."""
import math

import numpy as np


def ray_radius(phi, cx, cy, theta, ds=0.05):
    """Distance from (cx, cy) to the outermost phi = 0 crossing along the ray at angle theta
    (bilinear interpolation of phi on the periodic lattice, linear interpolation of the crossing),
    searched up to half the box."""
    n = phi.shape[0]
    s = np.arange(0.0, n / 2 - 1, ds)
    x, y = cx + s * math.cos(theta), cy + s * math.sin(theta)
    x0, y0 = np.floor(x).astype(int), np.floor(y).astype(int)
    fx, fy = x - x0, y - y0
    v = (phi[y0 % n, x0 % n] * (1 - fx) * (1 - fy) + phi[y0 % n, (x0 + 1) % n] * fx * (1 - fy) +
         phi[(y0 + 1) % n, x0 % n] * (1 - fx) * fy + phi[(y0 + 1) % n, (x0 + 1) % n] * fx * fy)
    idx = np.nonzero(v >= 0)[0]
    if len(idx) == 0:
        return 0.0
    i = idx[-1]
    if i + 1 == len(s):
        return float(s[i])  # the contour lies beyond the sampled half-box
    return s[i] + ds * v[i] / (v[i] - v[i + 1])


def hexagon_descriptors(phi, cx, cy):
    """Mean distance to the contour along the six tip directions (0, 60, ..., 300 degrees) and along
    the six directions between them (30, 90, ...), and the solid area as a fraction of the regular
    hexagon whose vertices are at the mean tip distance: a faceted plate has side/tip = cos 30 deg and
    fill 1; branched crystals have less of both."""
    tip = float(np.mean([ray_radius(phi, cx, cy, math.radians(a)) for a in range(0, 360, 60)]))
    side = float(np.mean([ray_radius(phi, cx, cy, math.radians(a)) for a in range(30, 360, 60)]))
    area = float((phi > 0).sum())
    return tip, side / tip, area / (1.5 * math.sqrt(3.0) * tip * tip)
