"""Pins of the surrogate's FP64 reference (oracle/mlp.py) and of its training
labels: back-propagation against central finite differences, the bfloat16
rounding against its bit-level definition, the quadrature of the screening
function against the closed form, and the labels against the rates they are
built from."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.mlp as M
from paper_2604_24627_amd import inputs as I


def test_bf16_rounding_definition():
    # values exactly between two bfloat16 numbers round to the even mantissa
    one = 1.0
    ulp = 2.0 ** -7
    assert M.to_bf16(one + ulp / 2)[()] == one                  # tie -> even (1.0)
    assert M.to_bf16(one + 3 * ulp / 2)[()] == one + 2 * ulp     # tie -> even
    assert M.to_bf16(one + ulp * 0.51)[()] == one + ulp
    assert M.to_bf16(-3.0)[()] == -3.0
    x = np.random.default_rng(0).standard_normal(1000)
    q = M.to_bf16(x)
    assert np.all(np.abs(q - x) <= np.abs(x) * 2 ** -8 + 1e-300)
    assert np.all(M.to_bf16(q) == q)


def test_backprop_matches_central_differences():
    rng = np.random.default_rng(1)
    P = M.init_params(3)
    X = rng.standard_normal((16, 8))
    Y = rng.standard_normal(16)
    loss, G = M.loss_and_grads(P, X, Y)
    h = 1e-6
    for l in (0, 2, 4):
        W = P[l][0]
        for (i, j) in [(0, 0), (3, min(5, W.shape[1] - 1)), (W.shape[0] - 1, W.shape[1] - 1)]:
            old = W[i, j]
            W[i, j] = old + h; lp, _ = M.loss_and_grads(P, X, Y)
            W[i, j] = old - h; lm, _ = M.loss_and_grads(P, X, Y)
            W[i, j] = old
            assert G[l][0][i, j] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-10)
        b = P[l][1]
        old = b[0]
        b[0] = old + h; lp, _ = M.loss_and_grads(P, X, Y)
        b[0] = old - h; lm, _ = M.loss_and_grads(P, X, Y)
        b[0] = old
        assert G[l][1][0] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-10)


def test_screening_function_quadrature_matches_closed_form():
    for s in (1e-6, 1e-3, 0.3, 1.0, 7.0, 1e2, 1e4, 1e7):
        assert M.F_quad(s) == pytest.approx(O.F(s), rel=1e-12)


def test_labels_equal_the_rates_they_sample():
    p = I.Params(g_agg_GeV=1.0, g_ae=1.0, inverse=1)
    T, ne, Z, x, ch = M.sample_domain(64, 7)
    y, lk = M.labels(p, T, ne, Z, x, ch)
    grid = dict(ndim=1, n=(1, 1, 1), dx=0.2, dt=0.1, omega0=1e17)
    for i in range(64):
        A = 1.0 if Z[i] == 1 else 4.0
        cell_p = dict(p.as_dict(), channels=[1, 2, 4, 4][ch[i]], brems_ee=1 if ch[i] == 3 else 0)
        c = O.cell_state(grid, cell_p, np.array([T[i]]), np.array([ne[i]]),
                         [np.array([ne[i] / Z[i]])], [Z[i]], [A])[0]
        E = x[i] * T[i]
        if ch[i] == 0:
            R = O.gamma_prim(c, cell_p, E)
        elif ch[i] in (1, 2):
            R = O.gamma_abs(c, cell_p, E)[0]
        else:
            cz = O.cell_state(grid, dict(cell_p, brems_ee=0), np.array([T[i]]), np.array([ne[i]]),
                              [np.array([ne[i] / Z[i]])], [Z[i]], [A])[0]
            R = O.gamma_abs(c, cell_p, E)[0] - O.gamma_abs(cz, dict(cell_p, brems_ee=0), E)[0]
        if ch[i] >= 2:
            # brems targets exclude the cell's screening factor 1 - a eta in (0, 1]
            if not np.isfinite(y[i]):
                assert R == 0.0
                continue
            assert 0.0 <= y[i] - math.log(R) < -math.log(1e-6)
            R = math.exp(y[i])
        assert y[i] == pytest.approx(math.log(R), abs=1e-10)
        assert lk[i] == pytest.approx(0.5 * math.log(c["kappa2"]) - math.log(T[i]), abs=1e-12)


def test_brems_labels_scale_as_density_squared_through_the_screening_region():
    """Without its screening factor a brems rate is base * rho / n_e * n_e with
    base proportional to rho: doubling n_e (and the ions with it) adds exactly
    ln 4 to log R, although the factor itself changes strongly between the two
    densities (cold, dense cells).  The Compton-like target scales as rho."""
    p = I.Params(g_ae=1.0, inverse=1)
    n = 24
    rng = np.random.default_rng(5)
    T = rng.uniform(0.5, 1.5, n)
    ne = np.exp(rng.uniform(np.log(1e25), np.log(4e25), n))
    Z = np.where(np.arange(n) % 2 == 0, 1.0, 2.0)
    x = np.exp(rng.uniform(np.log(0.1), np.log(20.0), n))
    for chan, slope in ((1, math.log(2.0)), (2, math.log(4.0)), (3, math.log(4.0))):
        ch = np.full(n, chan, dtype=np.int32)
        y1, _ = M.labels(p, T, ne, Z, x, ch)
        y2, _ = M.labels(p, T, 2 * ne, Z, x, ch)
        ok = np.isfinite(y1) & np.isfinite(y2)
        assert ok.sum() >= n // 2
        np.testing.assert_allclose(y2[ok] - y1[ok], slope, atol=1e-9)
    # and the plain rates themselves do not (the factor is a strong function of rho)
    grid = dict(ndim=1, n=(1, 1, 1), dx=0.2, dt=0.1, omega0=1e17)
    cp = dict(p.as_dict(), channels=4, brems_ee=0)
    r = []
    for f in (1.0, 2.0):
        c = O.cell_state(grid, cp, np.array([0.7]), np.array([f * 2e25]), [np.array([f * 2e25])],
                         [1.0], [1.0])[0]
        r.append(O.gamma_abs(c, cp, 2.0)[0])
    assert abs(math.log(r[1] / r[0]) - math.log(4.0)) > 0.05
