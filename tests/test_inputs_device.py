"""The device-side plasma generator (used for plasmas too large for the host)
follows the same recipe as the host generator: layout invariants exactly, and
the distributions within sampling error (run here on the CPU device)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2604_24627_amd import inputs as I  # noqa: E402


@pytest.mark.parametrize("graded", [False, True])
def test_device_generator_matches_host_recipe(graded):
    if graded:
        wl = I.config5(n=(16, 12, 10))
    else:
        wl = I.Workload("u", ndim=2, n=(40, 30), ppc=32, dtype="f32", T_keV=3.0, n_e=6e25,
                        lognormal_sigma=0.5)
    h = I.make_plasma(wl, 1)
    d = I.make_plasma_device(wl, 1, "cpu")
    for name in ("electrons", "ions", "photons"):
        a, b = h["species"][name], d["species"][name]
        off = b["off"].numpy()
        cell = b["cell"].numpy()
        assert off[0] == 0 and off[-1] == b["n"] and np.all(np.diff(off) >= 0)
        np.testing.assert_array_equal(cell, np.repeat(np.arange(wl.ncell), np.diff(off)))
        x = b["x"].numpy()
        nfull = tuple(wl.n) + (1,) * (3 - len(wl.n))
        idx = [cell % nfull[0], (cell // nfull[0]) % nfull[1], cell // (nfull[0] * nfull[1])]
        for k in range(wl.ndim):
            np.testing.assert_array_equal(np.floor(x[k]).astype(np.int64), idx[k])
        assert b["w_ref"] == a["w_ref"] and b["kind"] == a["kind"]
        n = b["n"]
        assert abs(n - a["n"]) < 6 * math.sqrt(a["n"]) + 1
        wa, wb = a["w"].astype(np.float64), b["w"].numpy().astype(np.float64)
        assert wb.mean() == pytest.approx(wa.mean(), rel=6 * wa.std() / wa.mean() / math.sqrt(n) + 1e-6)
        if a["p"] is not None:
            ea = np.sqrt((a["p"].astype(np.float64) ** 2).sum(0))
            eb = np.sqrt((b["p"].numpy().astype(np.float64) ** 2).sum(0))
            assert eb.mean() == pytest.approx(ea.mean(), rel=6 * ea.std() / ea.mean() / math.sqrt(n))
            assert eb.std() == pytest.approx(ea.std(), rel=0.05)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_seeded_axions_and_means_for_operator_tests(dtype):
    """The axion population and the rate-fed means that both sides of the operator
    tests consume: layout, ids, dtype and ranges."""
    wl = I.Workload("a", ndim=2, n=(24, 20), ppc=37, dtype=dtype, T_keV=3.0, n_e=6e25)
    pl = I.make_plasma(wl, 0)
    a = I.make_axions(wl, pl, 8.0, seed=11)
    dt = np.float32 if dtype == "f32" else np.float64
    n = a["n"]
    assert a["x"].dtype == dt and a["p"].dtype == dt and a["w"].dtype == dt
    assert a["w_ref"] == wl.params.w_a and a["off"][-1] == n
    np.testing.assert_array_equal(a["cell"], np.repeat(np.arange(wl.ncell), np.diff(a["off"])))
    np.testing.assert_array_equal(a["id"], np.arange(n, dtype=np.uint64) + np.uint64(pl["next_id"]))
    assert a["next_id"] == pl["next_id"] + n
    ix, iy = np.floor(a["x"][0]).astype(int), np.floor(a["x"][1]).astype(int)
    np.testing.assert_array_equal(ix + wl.n[0] * iy, a["cell"])
    zero = a["w"] == 0
    assert 0.005 < zero.mean() < 0.04 and np.all(a["w"][~zero] > 0)
    E = 510.99895 * np.sqrt((a["p"].astype(np.float64) ** 2).sum(axis=0))
    # blackbody mean energy 3 zeta(4)/zeta(3) T = 2.701 T
    assert E.mean() / 3.0 == pytest.approx(2.701, rel=0.05)
    lam = I.means(1000, 3, rows=2, lo=1e-4, hi=3.0, dtype=dtype)
    assert lam.shape == (2, 1000) and lam.dtype == dt
    z = lam == 0
    assert 0 < z.sum() < 80 and lam[~z].min() >= 1e-4 * (1 - 1e-6) and lam.max() <= 3.0 * (1 + 1e-6)
    np.testing.assert_array_equal(I.means(1000, 3, rows=2, dtype=dtype), lam)
