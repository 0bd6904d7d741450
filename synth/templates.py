"""Single-event shapes for the last column of the linear-search design.

The paper proposes replacing the box in the last column of the design
matrix by other base models: limb-darkened transits and the asymmetric dips
of transiting exocomets (Section 4.4, prospects). It gives no formula for
either, so the shapes here are stated choices. Each is a vector of d values,
one per lattice slot of the event window (slot k of the window sits at
u = (k + 1/2) / d of its duration), with peak value 1, so the fitted depth is
the depth at the deepest point. A shape is an input of the search like the
durations: the search takes any vector.

* ``box``: 1 everywhere (the search of Section 2.2).
* ``limb_darkened``: a planet small against its star crossing on a chord of
  impact parameter b, with quadratic limb darkening
  I(mu) = 1 - u1 (1 - mu) - u2 (1 - mu)^2: the dip follows the surface
  brightness under the planet, I(mu(r(u))), r(u) the projected separation
  along the chord (r = b at mid-event, 1 at the window edges).
* ``exocomet``: a linear ingress over the first ``rise`` of the window, then
  an exponential egress exp(-(u - rise) / tail).
"""
from __future__ import annotations

import numpy as np


def _centres(d: int) -> np.ndarray:
    if d < 1:
        raise ValueError("a window needs at least one slot")
    return (np.arange(d, dtype=np.float64) + 0.5) / d


def box(d: int) -> np.ndarray:
    return np.ones_like(_centres(int(d)))


def limb_darkened(d: int, u1: float = 0.4, u2: float = 0.25, b: float = 0.0) -> np.ndarray:
    if not 0.0 <= b < 1.0:
        raise ValueError("impact parameter must be in [0, 1)")
    u = _centres(d)
    half_chord = np.sqrt(1.0 - b * b)
    r = np.sqrt(b * b + ((2.0 * u - 1.0) * half_chord) ** 2)
    mu = np.sqrt(np.clip(1.0 - r * r, 0.0, None))
    intensity = 1.0 - u1 * (1.0 - mu) - u2 * (1.0 - mu) ** 2
    mu_mid = np.sqrt(1.0 - b * b)
    peak = 1.0 - u1 * (1.0 - mu_mid) - u2 * (1.0 - mu_mid) ** 2
    return intensity / peak


def exocomet(d: int, rise: float = 0.1, tail: float = 0.3) -> np.ndarray:
    if not (0.0 < rise < 1.0 and tail > 0.0):
        raise ValueError("need 0 < rise < 1 and tail > 0")
    u = _centres(d)
    s = np.where(u < rise, u / rise, np.exp(-(u - rise) / tail))
    return s / np.max(s)


def shapes_for(kind: str, durations, **kw) -> list:
    """One shape per duration (slots), by name: box, limb_darkened, exocomet."""
    fn = {"box": box, "limb_darkened": limb_darkened, "exocomet": exocomet}[kind]
    return [fn(int(d), **kw) for d in durations]
