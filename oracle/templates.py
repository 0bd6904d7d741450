"""Oracle: the single-event search with a non-box base model (Section 4.4,
prospects: limb-darkened transits and exocomets in the last column of the
design matrix).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

For cell (duration j, slot i) the design is X = [A | b_ij] as in Section
2.2, with the box replaced by a shape: with a_ij = i - floor(d_j/2),

    b_ij[m] = -s_j[l_m - a_ij]   if a_ij <= l_m < a_ij + d_j,   else 0,

where l_m is the lattice slot of sample m and s_j (d_j values) is the shape
of duration j. The unit shape is the box of ``oracle.linear``. The fit is
the same generalised least squares of Eqs. 5-6, solved in full for each
cell (``oracle.linear._fit_cells``); dll is the gain of ln L over the
trend-only fit.

Readings: the window convention is the box's (the shape's slot k sits at
slot a_ij + k); the shape values are given per slot, so a sample's weight
is the shape value of its slot; invalid cells as for the box.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import linear as olin


def template_column(lattice: np.ndarray, slot: int, shape: np.ndarray) -> np.ndarray:
    """b of the cell at ``slot`` with the shape ``shape`` (written as an explicit scan)."""
    lattice = np.asarray(lattice, dtype=np.int64)
    d = len(shape)
    a = slot - d // 2
    b = np.zeros(lattice.shape[0])
    for m, l in enumerate(lattice):
        if a <= l < a + d:
            b[m] = -float(shape[l - a])
    return b


def linear_search_template(f: np.ndarray, A: np.ndarray, L: np.ndarray, lattice: np.ndarray, shapes,
                           n_epochs: Optional[int] = None, cells=None, batch: int = 256) -> dict:
    """The search over all (duration j, slot i) cells (or the listed ``cells``), duration j having the
    shape ``shapes[j]``. Same outputs as ``oracle.linear.linear_search``."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    A = np.asarray(A, dtype=np.float64).reshape(n, -1)
    lattice = np.asarray(lattice, dtype=np.int64)
    shapes = [np.asarray(s, dtype=np.float64) for s in shapes]
    if n_epochs is None:
        n_epochs = int(lattice[-1]) + 1
    if cells is None:
        cells = [(j, i) for j in range(len(shapes)) for i in range(n_epochs)]
        out_shape = (len(shapes), n_epochs)
    else:
        out_shape = (len(cells),)
    ft = olin.whiten(L, f)
    At = olin.whiten(L, A) if A.shape[1] else np.zeros((n, 0))
    chi2_0, _ = olin.null_fit(L, f, A)
    ld = float(2.0 * np.sum(np.log(np.diag(L))))
    lnl0 = -0.5 * chi2_0 - 0.5 * ld - 0.5 * n * math.log(2.0 * math.pi)
    ncell = len(cells)
    depth = np.zeros(ncell)
    var = np.full(ncell, np.inf)
    dll = np.zeros(ncell)
    valid = np.zeros(ncell, dtype=np.uint8)
    cols = {}
    todo = []
    for c, (j, i) in enumerate(cells):
        b = template_column(lattice, i, shapes[j])
        if np.any(b != 0.0):
            cols[c] = b
            todo.append(c)
    for s in range(0, len(todo), batch):
        idx = todo[s:s + batch]
        B = np.stack([cols[c] for c in idx], axis=1)
        d, v, c2, ok = olin._fit_cells(At, ft, olin.whiten(L, B))
        for col, c in enumerate(idx):
            if ok[col]:
                depth[c] = d[col]
                var[c] = v[col]
                dll[c] = 0.5 * (chi2_0 - c2[col])
                valid[c] = 1
    return {"depth": depth.reshape(out_shape), "var": var.reshape(out_shape), "dll": dll.reshape(out_shape),
            "valid": valid.reshape(out_shape), "lnl0": lnl0, "chi2_0": chi2_0, "logdet": ld}
