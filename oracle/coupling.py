"""TEST INFRASTRUCTURE ONLY: plain float64 oracle of the steps that couple the
IMF to a density-based TO loop (Sec. 2.2 of the paper), written from their
definitions:

* Heaviside projection (Eq. Heaviside): rho = 1 - exp(-beta xi) + xi exp(-beta).
  For use as the design of an IMF request the result is rounded to the nearest
  multiple of 2^-24 (halves up) and clamped to [0, 1]; xi is clamped to [0, 1].
* Accessibility filter (Eq. accFilter): fbar (the allowance-applied normalized
  IMF of Algorithm 1) inside the design Omega = [rho > tau], 1 on the secluded
  set Gamma, 0 elsewhere.
* Filtered sensitivity (Eq. filtered_sens): (1 - w) Sbar_phi + w Sbar_IMF, with
  Sbar_phi the objective sensitivity divided by its maximum magnitude over
  Omega_0 (the paper says "normalized" without the norm; 0 when that maximum
  is 0).
* Greedy machining plan (Sec. 3.4.1, post-processing): repeatedly the orientation
  whose accessible set covers the most of the remaining negative space.

Only the tests may import this module.
"""
from __future__ import annotations

import numpy as np

Q24 = float(1 << 24)


def heaviside(xi, beta: float) -> np.ndarray:
    """Eq. Heaviside in float64, then the 2^-24 grid (round half up), float32."""
    x = np.clip(np.asarray(xi, np.float64), 0.0, 1.0)
    r = 1.0 - np.exp(-beta * x) + x * np.exp(-beta)
    q = np.floor(r * Q24 + 0.5) / Q24
    return np.clip(q, 0.0, 1.0).astype(np.float32)


def omega0_of(shape, fixture=None, domain=None) -> np.ndarray:
    if domain is not None:
        return np.asarray(domain) != 0
    if fixture is not None:
        return np.asarray(fixture) == 0
    return np.ones(shape, bool)


def access_filter(design, imf_norm, secluded, tau: float = 0.5) -> np.ndarray:
    """Eq. accFilter: fbar on Omega = [rho > tau], 1 on Gamma, 0 elsewhere."""
    rho = np.asarray(design, np.float64)
    out = np.zeros(rho.shape, np.float32)
    sec = np.asarray(secluded) != 0
    out[sec] = 1.0
    inside = rho > tau
    out[inside] = np.asarray(imf_norm, np.float32)[inside]
    return out


def filtered_sensitivity(sens_phi, filt, w: float, omega0) -> np.ndarray:
    """Eq. filtered_sens with Sbar_phi = S_phi / max_{Omega_0} |S_phi|."""
    s = np.asarray(sens_phi, np.float64)
    om = np.asarray(omega0, bool)
    m = float(np.abs(s[om]).max()) if om.any() else 0.0
    sbar = s / m if m > 0 else np.zeros_like(s)
    return ((1.0 - w) * sbar + w * np.asarray(filt, np.float64)).astype(np.float32)


def plan_greedy(masks_bool, design, tau: float = 0.5, omega0=None, max_steps=None):
    """Greedy machining plan (Sec. 3.4.1): from the negative space
    N = Omega_0 and [rho <= tau], repeatedly take the orientation whose
    accessible set covers the most of what remains (lowest index on ties),
    remove it, until nothing more is removable.  masks_bool: [n_orient, ...]
    booleans of the grid's shape.  Returns ([(orientation, removed), ...],
    remaining)."""
    A = np.asarray(masks_bool, bool).reshape(len(masks_bool), -1)
    rho = np.asarray(design, np.float64).reshape(-1)
    om = np.ones_like(rho, bool) if omega0 is None else np.asarray(omega0, bool).reshape(-1)
    R = om & (rho <= tau)
    steps = []
    limit = len(A) if max_steps is None else max_steps
    while len(steps) < limit:
        cover = [int(np.count_nonzero(A[q] & R)) for q in range(len(A))]
        best = int(np.argmax(cover))  # first maximum
        if cover[best] == 0:
            break
        steps.append((best, cover[best]))
        R &= ~A[best]
    return steps, int(np.count_nonzero(R))
