"""String method for minimum energy paths: the second workload of the paper
(Section 3.2, a reaction path discretised into images, each image's BO
energy and force computed in parallel, the path updated between force calls).

TEST INFRASTRUCTURE (see the package docstring).  Plain NumPy, written from
the simplified string method of E, Ren and Vanden-Eijnden (J. Chem. Phys.
126, 164103 (2007)); it shares no code with the HIP path.

One iteration of a string of n images x_0 .. x_{n-1} (each a vector of all
atomic coordinates, bohr):
  1. evolution: every movable image takes a steepest-descent step along its
     force, x_i <- x_i + h F_i (F = -dE/dx, h in bohr^2/Eh); with fixed ends
     the first and last image stay;
  2. reparametrisation: the images are redistributed to equal arc length
     along the piecewise-linear curve through them: with cumulative chord
     lengths s_0 = 0 <= s_1 <= ... <= s_{n-1} = L, image i moves to the
     point at arc length i L / (n - 1), found by linear interpolation on the
     segment that contains it (s_j <= i L/(n-1) < s_{j+1}, the last target on
     the last segment); a zero-length segment gives weight 0; a string of
     zero length is left as it is.  The end images keep their positions.
"""

from __future__ import annotations

import numpy as np


def arc_positions(x) -> np.ndarray:
    """Normalised cumulative chord lengths s_i / L of the images (zeros if L = 0)."""
    flat = np.asarray(x, float).reshape(len(x), -1)
    seg = np.sqrt(np.sum(np.diff(flat, axis=0) ** 2, axis=1))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    return s / s[-1] if s[-1] > 0 else s


def reparametrize(x) -> np.ndarray:
    x = np.asarray(x, float)
    n = len(x)
    flat = x.reshape(n, -1)
    seg = np.sqrt(np.sum(np.diff(flat, axis=0) ** 2, axis=1))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    L = s[-1]
    if n < 3 or L == 0.0:
        return x.copy()
    out = flat.copy()
    for i in range(1, n - 1):
        t = i * L / (n - 1)
        j = 0
        while j < n - 2 and s[j + 1] <= t:
            j += 1
        d = s[j + 1] - s[j]
        w = (t - s[j]) / d if d > 0 else 0.0
        out[i] = (1.0 - w) * flat[j] + w * flat[j + 1]
    return out.reshape(x.shape)


def evolve(x, forces, h, fix_ends=False) -> np.ndarray:
    x = np.asarray(x, float)
    out = x + h * np.asarray(forces, float)
    if fix_ends:
        out[0], out[-1] = x[0], x[-1]
    return out


def step(x, forces, h, fix_ends=False) -> np.ndarray:
    """One iteration: evolution, then reparametrisation."""
    return reparametrize(evolve(x, forces, h, fix_ends))
