"""Oracle: the periodic search over several segments of a light curve, each
with its own linear search (Sections 3.3 and 4.1: sectors observed years apart
are searched with one GP and one linear search per sector, and the periodic
search combines them).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The definition: segment s covers the lattice slots [off_s, off_s + n_s) of one
global lattice of cadence dt (from the first slot of the first segment); its
linear-search grid is placed there, every slot of no segment is an invalid
cell, and the periodic search of ``oracle.periodic`` runs on that global grid.
Phases and events are in global slots, so a transit train continues across
the gaps.

Reading: the segments share dt, the durations and the phase origin (global
slot 0); their offsets are integers (sectors on one lattice).
"""
from __future__ import annotations

import numpy as np

from . import periodic


def assemble(grids, offsets):
    """Global (depth, var, dll, valid) from per-segment grids [(depth, var, dll, valid), ...] at slot offsets."""
    offsets = [int(o) for o in offsets]
    n_d = np.asarray(grids[0][0]).shape[0]
    n_t = max(o + np.asarray(g[0]).shape[1] for g, o in zip(grids, offsets))
    depth = np.zeros((n_d, n_t))
    var = np.full((n_d, n_t), np.inf)
    dll = np.zeros((n_d, n_t))
    valid = np.zeros((n_d, n_t), dtype=np.uint8)
    for (d, v, l, ok), o in zip(grids, offsets):
        n = np.asarray(d).shape[1]
        if np.any(valid[:, o:o + n]):
            raise ValueError("segments overlap")
        depth[:, o:o + n] = d
        var[:, o:o + n] = v
        dll[:, o:o + n] = l
        valid[:, o:o + n] = ok
    return depth, var, dll, valid


def periodic_search_segments(grids, offsets, dt: float, periods, sign: int = 1) -> dict:
    """Periodic search of the segments combined (phases in global slots)."""
    return periodic.periodic_search(*assemble(grids, offsets), dt, periods, sign)
