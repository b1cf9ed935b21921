"""Exact Euclidean projections onto the prox-friendly sets (Sec. II assumption; Sec. III-B Step 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Step 3 of the ADMM evaluates the proximal operator of an indicator function,
which is the Euclidean projection onto the set.  The paper gives the box clamp
and norm scaling as its examples; half-spaces (linearized obstacles), second-
order cones (||T|| <= Gamma) and scaled cones (glide slope) follow from the
standard closed forms.  All functions act row-wise on (n, m) arrays.
"""
from __future__ import annotations

import numpy as np


def proj_box(v: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Clamp(v, lo, hi), element-wise (Step 3 box case)."""
    return np.minimum(np.maximum(v, lo), hi)


def proj_halfspace(v: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Projection onto {y : a'y >= b}: v + max(0, b - a'v) / (a'a) * a."""
    viol = np.maximum(0.0, b - np.sum(a * v, axis=-1))
    return v + (viol / np.sum(a * a, axis=-1))[..., None] * a


def proj_ball(v: np.ndarray, radius: float) -> np.ndarray:
    """Projection onto {y : ||y|| <= radius}: norm scaling v * min(1, radius/||v||)."""
    nv = np.sqrt(np.sum(v * v, axis=-1))
    scale = np.ones_like(nv)
    big = nv > radius
    scale[big] = radius / nv[big]
    return v * scale[..., None]


def proj_soc(v: np.ndarray) -> np.ndarray:
    """Projection onto the second-order cone {(t, s) : ||t|| <= s}; s is the last column."""
    return proj_cone(v, 1.0)


def proj_cone(v: np.ndarray, kappa: float) -> np.ndarray:
    """Projection onto {(y, s) : ||y|| <= kappa s}; s is the last column.

    Inside: v.  Polar side (kappa ||y|| <= -s): 0.  Otherwise the point on the
    boundary ray: c (kappa y/||y||, 1) with c = (kappa ||y|| + s)/(1 + kappa^2).
    A zero radial part on the boundary branch cannot occur (it would be inside
    or polar), so the division by ||y|| is safe.
    """
    y, s = v[..., :-1], v[..., -1]
    ny = np.sqrt(np.sum(y * y, axis=-1))
    out = np.array(v, dtype=float, copy=True)
    inside = ny <= kappa * s
    polar = (~inside) & (kappa * ny <= -s)
    edge = ~(inside | polar)
    out[polar] = 0.0
    if np.any(edge):
        c = (kappa * ny[edge] + s[edge]) / (1.0 + kappa * kappa)
        out[edge, :-1] = (c * kappa / ny[edge])[:, None] * y[edge]
        out[edge, -1] = c
    return out
