"""Checkpoint and resume: a run stopped after k steps, saved, loaded into a fresh sim
built from the same plasma and continued, equals the uninterrupted run bit for bit --
particle buffers, temperatures, statistics and histograms -- because every draw is keyed
by (seed, particle id, step) and no other state carries over (needs an MI355X)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_24627_amd import inputs as I  # noqa: E402
from paper_2604_24627_amd.sim import AxpicSim  # noqa: E402


def _snapshot(g):
    out = {"T": g.T.cpu().numpy(), "stats": g.stats.cpu().numpy(),
           "hist": g.hist.cpu().numpy(), "step": g.step_index, "next_id": g.next_id}
    for name in ("el", "ph", "ax"):
        sp = getattr(g, name)
        d = sp.to_numpy()
        out[name] = (sp.n, sp.n_sorted, d)
    return out


@pytest.mark.parametrize("thermal", ["particle", "cells"])
def test_resume_from_a_checkpoint_is_bit_identical(tmp_path, thermal):
    p = I.Params(g_agg_GeV=1e-10, g_ae=1e-13, channels=7, inverse=1, w_a=1e-36, boost=4e33,
                 lambda_cap=1.0, feedback=1, T_mode=2, r_relax=0.3)
    wl = I.Workload("ckpt", ndim=2, n=(16, 12), ppc=24, dtype="f32", T_keV=3.0, n_e=6e25,
                    params=p)
    pl = I.make_plasma(wl, 5)
    print(f"[ckpt] thermal={thermal}", flush=True)
    whole = AxpicSim(pl, wl.params, thermal=thermal)
    for _ in range(6):
        whole.step()
    first = AxpicSim(pl, wl.params, thermal=thermal)
    for _ in range(3):
        first.step()
    first.save(str(tmp_path))
    resumed = AxpicSim(pl, wl.params, thermal=thermal)
    resumed.load(str(tmp_path))
    for _ in range(3):
        resumed.step()
    a, b = _snapshot(whole), _snapshot(resumed)
    assert a["step"] == b["step"] == 6 and a["next_id"] == b["next_id"]
    for key in ("T", "stats", "hist"):
        np.testing.assert_array_equal(a[key], b[key])
    for name in ("el", "ph", "ax"):
        (na, sa, da), (nb, sb, db) = a[name], b[name]
        assert (na, sa) == (nb, sb), name
        for k in ("w", "id", "cell", "p", "x"):
            np.testing.assert_array_equal(da[k], db[k], err_msg=f"{name}.{k}")
    assert a["ax"][0] > 50 and a["stats"].any()
