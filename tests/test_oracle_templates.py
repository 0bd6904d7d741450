"""Pins of the oracle's single-event search with a non-box base model
(``oracle.templates``) and of the shape inputs (``synth.templates``).

The template search is pinned by what the mathematics fixes, not by itself:

* the unit shape is the box search of ``oracle.linear`` (pinned on its own);
* scaling the shape by c divides the depth by c and the variance by c^2 and
  leaves dll unchanged; a negated shape negates the depth;
* noise-free data made of a trend plus delta times one cell's column give
  depth = delta and a zero chi^2 at that cell (dll = chi2_0 / 2);
* dll, depth and var equal Eq. 5 and Eq. 6 evaluated with K itself (dense
  solves with K, no factor, no whitening);
* the column of a window straddling a gap, written out by hand.
"""
import math

import numpy as np
import pytest

from oracle import gp as ogp, linear as olin, templates as otpl
from synth import make_workload, sho_omega_from_rotation
from synth import templates as stpl


def _small(n=160, gap=(70, 9), seed=3, durations=(1, 4, 7)):
    th = {"amp": 0.006, "omega": sho_omega_from_rotation(0.5, 3.0), "q": 3.0, "sigma_w": 1e-3}
    w = make_workload(f"tpl-{n}", seed, n, 10 / 1440, th, list(durations), np.linspace(0.3, 1.0, 5),
                      gaps=[gap] if gap else [],
                      injection={"depth": 2e-3, "period": 0.37, "t0": 0.1, "duration": 0.03})
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    return w, L


def test_unit_shape_is_the_box():
    w, L = _small()
    box = olin.linear_search(w.f, w.A, L, w.lattice, w.durations, n_epochs=w.n_epochs)
    tpl = otpl.linear_search_template(w.f, w.A, L, w.lattice, stpl.shapes_for("box", w.durations),
                                      n_epochs=w.n_epochs)
    np.testing.assert_array_equal(tpl["valid"], box["valid"])
    v = box["valid"].astype(bool)
    for k in ("depth", "var", "dll"):
        np.testing.assert_allclose(tpl[k][v], box[k][v], rtol=1e-12, atol=1e-18)


def test_scaling_and_sign():
    w, L = _small()
    shapes = stpl.shapes_for("limb_darkened", w.durations)
    base = otpl.linear_search_template(w.f, w.A, L, w.lattice, shapes, n_epochs=w.n_epochs)
    c = 2.5
    scaled = otpl.linear_search_template(w.f, w.A, L, w.lattice, [c * s for s in shapes], n_epochs=w.n_epochs)
    neg = otpl.linear_search_template(w.f, w.A, L, w.lattice, [-s for s in shapes], n_epochs=w.n_epochs)
    v = base["valid"].astype(bool)
    assert v.sum() > 100
    np.testing.assert_allclose(scaled["depth"][v], base["depth"][v] / c, rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(scaled["var"][v], base["var"][v] / c ** 2, rtol=1e-9)
    np.testing.assert_allclose(scaled["dll"][v], base["dll"][v], rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(neg["depth"][v], -base["depth"][v], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(neg["dll"][v], base["dll"][v], rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("kind", ["limb_darkened", "exocomet"])
def test_noise_free_recovery(kind):
    w, L = _small()
    shapes = stpl.shapes_for(kind, w.durations)
    j, i, delta = 2, 73, 3e-3          # a window that straddles the gap
    b = otpl.template_column(w.lattice, i, shapes[j])
    f = w.A @ np.array([1.0, 2e-3, -1e-3])[:w.A.shape[1]] + delta * b
    out = otpl.linear_search_template(f, w.A, L, w.lattice, shapes, cells=[(j, i), (0, 20)])
    assert out["valid"][0] == 1
    assert out["depth"][0] == pytest.approx(delta, rel=1e-9)
    assert out["dll"][0] == pytest.approx(0.5 * out["chi2_0"], rel=1e-9)
    assert out["dll"][0] == pytest.approx(0.5 * delta ** 2 / out["var"][0], rel=1e-8)


def test_matches_eq5_with_dense_solves():
    w, L = _small()
    shapes = stpl.shapes_for("exocomet", w.durations)
    K = ogp.covariance(w.t, w.theta)
    cells = [(0, 5), (1, 69), (2, 73), (2, 150), (1, 0), (2, w.n_epochs - 1)]
    out = otpl.linear_search_template(w.f, w.A, L, w.lattice, shapes, cells=cells)
    n = w.n
    _, logdet = np.linalg.slogdet(K)

    def lnl(X):
        KiX = np.linalg.solve(K, X)
        G = X.T @ KiX
        wfit = np.linalg.solve(G, KiX.T @ w.f)
        r = w.f - X @ wfit
        chi2 = float(r @ np.linalg.solve(K, r))
        return -0.5 * chi2 - 0.5 * logdet - 0.5 * n * math.log(2 * math.pi), wfit, G

    l0, _, _ = lnl(w.A)
    assert out["lnl0"] == pytest.approx(l0, rel=1e-10)
    for c, (j, i) in enumerate(cells):
        X = np.column_stack([w.A, otpl.template_column(w.lattice, i, shapes[j])])
        l1, wfit, G = lnl(X)
        assert out["valid"][c] == 1
        assert out["dll"][c] == pytest.approx(l1 - l0, rel=1e-7, abs=1e-9)
        assert out["depth"][c] == pytest.approx(wfit[-1], rel=1e-7, abs=1e-12)
        assert out["var"][c] == pytest.approx(np.linalg.inv(G)[-1, -1], rel=1e-7)


def test_template_column_by_hand():
    lattice = np.array([0, 1, 2, 5, 6, 7, 8])   # slots 3 and 4 are a gap
    shape = np.array([1.0, 2.0, 3.0, 4.0])
    # slot 4, d = 4: window [2, 6) holds samples at slots 2 (k = 0) and 5 (k = 3)
    np.testing.assert_array_equal(otpl.template_column(lattice, 4, shape), [0, 0, -1, -4, 0, 0, 0])
    # slot 0: window [-2, 2) holds slots 0 (k = 2) and 1 (k = 3)
    np.testing.assert_array_equal(otpl.template_column(lattice, 0, shape), [-3, -4, 0, 0, 0, 0, 0])
    # an empty window gives an invalid cell
    out = otpl.linear_search_template(np.ones(7), np.ones((7, 1)), np.eye(7), lattice, [np.ones(1)],
                                      cells=[(0, 3), (0, 4)])
    assert out["valid"].tolist() == [0, 0]
    assert out["var"][0] == np.inf and out["dll"][0] == 0.0


def test_shapes():
    np.testing.assert_array_equal(stpl.limb_darkened(9, u1=0.0, u2=0.0), np.ones(9))
    s = stpl.limb_darkened(11)
    np.testing.assert_allclose(s, s[::-1], rtol=1e-15)
    assert s[5] == pytest.approx(1.0) and np.all(s <= 1.0 + 1e-15) and np.all(np.diff(s[:6]) > 0)
    g = stpl.limb_darkened(20, b=0.6)
    assert np.all(g > 0) and np.max(g) <= 1.0 + 1e-15
    e = stpl.exocomet(30)
    assert np.max(e) == pytest.approx(1.0)
    k = int(np.argmax(e))
    assert np.all(np.diff(e[:k + 1]) > 0) and np.all(np.diff(e[k:]) < 0)
    for bad in (lambda: stpl.limb_darkened(5, b=1.0), lambda: stpl.exocomet(5, rise=0.0),
                lambda: stpl.box(0)):
        with pytest.raises(ValueError):
            bad()
