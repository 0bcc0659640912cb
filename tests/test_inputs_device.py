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
