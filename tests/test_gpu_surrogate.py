"""The rate surrogate on the GPU (needs an MI355X).

* the library's training samples (its plain rates, FP64) equal the oracle's
  independently computed labels;
* the BF16-MFMA training forward pass and gradients agree with the FP64
  reference that emulates the same bfloat16 rounding points (oracle/mlp.py);
* the fused inference kernel (weights in LDS, layers chained in registers)
  reproduces the training forward pass;
* a network trained on the GPU by these kernels reproduces the oracle's
  rates on held-out samples, and the rates it feeds the sampling operators
  keep the integrated power within 1% of the plain path; the test reports
  what it gains over the plain path (time per evaluation).
"""
import math
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
import oracle.mlp as M  # noqa: E402
from paper_2604_24627_amd import inputs as I  # noqa: E402
from paper_2604_24627_amd import axpic as B  # noqa: E402
from paper_2604_24627_amd.sim import AxpicSim  # noqa: E402
from paper_2604_24627_amd.surrogate import Surrogate, init_master  # noqa: E402


def unpad(master):
    """Padded FP32 master vector -> oracle parameter list (live entries only)."""
    P = np.asarray(master, dtype=np.float64)
    dims = [(32, 128), (128, 128), (128, 128), (128, 128), (128, 32)]
    out, off = [], 0
    for li, (din, dout) in enumerate(dims):
        W = P[off: off + din * dout].reshape(din, dout); off += din * dout
        b = P[off: off + dout]; off += dout
        if li == 0:
            W = W[:8]
        if li == 4:
            W, b = W[:, :1], b[:1]
        out.append([W.copy(), b.copy()])
    return out


def grads_unpad(g):
    return unpad(g)


def random_design(n, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, 32), dtype=np.float32)
    X[:, :4] = rng.uniform(-1, 1, (n, 4))
    X[np.arange(n), 4 + rng.integers(0, 4, n)] = 1.0
    Y = rng.standard_normal(n).astype(np.float32)
    return X, Y


def test_training_samples_match_oracle_labels():
    p = I.Params()
    S = Surrogate(p)
    feat, logR, ch = S.samples(4096, 5)
    T, ne, Z, x, chn = I.surrogate_samples(4096, 5)
    ref, lk = M.labels(p, T, ne, Z, x, chn)
    np.testing.assert_array_equal(ch.cpu().numpy(), chn)
    np.testing.assert_array_equal(np.isfinite(logR.cpu().numpy()), np.isfinite(ref))
    assert np.isfinite(ref).mean() > 0.99
    np.testing.assert_allclose(logR.cpu().numpy(), ref, rtol=0, atol=2e-11)
    f = feat.cpu().numpy()
    np.testing.assert_allclose(f[:, 0], np.log(x), atol=1e-13)
    np.testing.assert_allclose(f[:, 1], lk, atol=1e-12)
    np.testing.assert_allclose(f[:, 2], np.log(ne), atol=1e-12)
    np.testing.assert_array_equal(f[:, 3], Z)


def test_mlp_forward_and_gradients_match_fp64_reference():
    S = Surrogate(I.Params(), seed=3)
    X, Y = random_design(512, 9)
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    y = S.forward(Xt).cpu().numpy().astype(np.float64)
    P = unpad(S.master.cpu().numpy())
    yref, _ = M.forward(P, X[:, :8].astype(np.float64), quantize=True)
    assert np.max(np.abs(y - yref)) < 2e-2 * (1 + np.abs(yref).max())
    assert np.mean(np.abs(y - yref)) < 2e-3
    g, loss = S.loss_grad(Xt, Yt)
    torch.cuda.synchronize()
    lref, gref = M.loss_and_grads(P, X[:, :8].astype(np.float64), Y.astype(np.float64),
                                  quantize=True)
    assert float(loss.item()) == pytest.approx(lref, rel=2e-2)
    G = grads_unpad(g.cpu().numpy())
    for l in range(5):
        for k in range(2):
            a, b = G[l][k], gref[l][k]
            err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            assert err < 2e-2, (l, k, err)
    # padded entries carry no gradient
    gfull = g.cpu().numpy()
    assert np.all(gfull[8 * 128: 32 * 128] == 0.0)


def _small_plasma(T=3.0, ne=6e25, **pk):
    p = I.Params(g_agg_GeV=1e-10, g_ae=1e-13, channels=7, inverse=1, w_a=1e-36, lambda_cap=1.0,
                 boost=1e33, **pk)
    wl = I.Workload("sur", ndim=2, n=(32, 24), ppc=48, dtype="f32", T_keV=T, n_e=ne, n_ref=6e25,
                    params=p)
    return wl, I.make_plasma(wl, 4)


@pytest.fixture(scope="module")
def trained():
    S = Surrogate(I.Params(), seed=0)
    t0 = time.time()
    log = S.train(n_samples=1_000_000, steps=20000, batch=4096, lr=2e-3, lr_end=2e-5, seed=1,
                  log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    print(f"[surrogate] trained in {time.time() - t0:.1f} s, final loss {log[-1][1]:.3e}", flush=True)
    return S


def test_inference_kernel_reproduces_training_forward(trained):
    S = trained
    wl, pl = _small_plasma()
    g = AxpicSim(pl, wl.params)
    lam_mlp = S.rates(g, g.ph, B.PRIMAKOFF).double().cpu().numpy()
    # the same features through the training forward pass
    st = g.state.cpu().numpy().reshape(-1, B.STATE_N)
    ph = g.ph.to_numpy()
    c = ph["cell"]
    Tc, nec, k2 = st[c, 0], st[c, 1], st[c, 7]
    om = 510.99895 * np.sqrt((ph["p"].astype(np.float64) ** 2).sum(axis=0))
    feat = np.stack([np.log(om / Tc), 0.5 * np.log(k2) - np.log(Tc), np.log(nec),
                     np.full(om.size, 1.0)], axis=1)
    n = om.size
    logR = S.predict_log(torch.from_numpy(feat).cuda(),
                         torch.zeros(n, dtype=torch.int32, device="cuda")).cpu().numpy()
    G = 1e-20 * 1e33 * np.exp(logR) * (0.1 / g.grid_d["omega0"])
    lam_ref = ph["w"] * (g.ph.w_ref / (g.pdict["w_a"] * g.pdict["wa_mul"][0])) * -np.expm1(-G)
    inside = (om / Tc > 0.01) & (om / Tc < 100)
    assert inside.mean() > 0.9
    rel = np.abs(np.log(lam_mlp[inside]) - np.log(lam_ref[inside]))
    print(f"[surrogate] inference vs training forward: median |d log lambda| {np.median(rel):.2e}, "
          f"max {rel.max():.2e}", flush=True)
    assert np.median(rel) < 2e-3 and rel.max() < 5e-2 * S.norm["sigma"][0]


def test_trained_surrogate_matches_oracle_rates(trained):
    S = trained
    p = I.Params()
    T, ne, Z, x, ch = I.surrogate_samples(20000, 99)      # held out
    ref, lk = M.labels(p, T, ne, Z, x, ch)
    keep = np.isfinite(ref)                                 # brems with a zero screening factor
    T, ne, Z, x, ch, ref, lk = (a[keep] for a in (T, ne, Z, x, ch, ref, lk))
    feat = np.stack([np.log(x), lk, np.log(ne), Z], axis=1)
    pred = S.predict_log(torch.from_numpy(feat).cuda(), torch.from_numpy(ch).cuda()).cpu().numpy()
    err = pred - ref
    for c in range(4):
        e = err[ch == c]
        print(f"[surrogate] channel {c}: rms log-rate error {np.sqrt(np.mean(e * e)):.2e}, "
              f"max {np.abs(e).max():.2e}", flush=True)
        assert np.sqrt(np.mean(e * e)) < 0.02
        assert abs(np.mean(e)) < 0.005


def test_surrogate_power_within_one_percent_and_gain_reported(trained):
    S = trained
    wl, pl = _small_plasma()
    g = AxpicSim(pl, wl.params)
    lam_plain = g.rates(g.ph, B.PRIMAKOFF).double()
    lam_mlp = S.rates(g, g.ph, B.PRIMAKOFF).double()
    E = torch.sqrt(g.ph.p[0][: g.ph.n].double() ** 2 + g.ph.p[1][: g.ph.n].double() ** 2 +
                   g.ph.p[2][: g.ph.n].double() ** 2)
    Pp, Pm = float((lam_plain * E).sum()), float((lam_mlp * E).sum())
    assert Pm == pytest.approx(Pp, rel=0.01)
    for _ in range(3):
        g.step()
    pab_plain = g.rates(g.ax, B.COMPTON | B.BREMS).double()
    pab_mlp = S.rates(g, g.ax, B.COMPTON | B.BREMS).double()
    Ea = torch.sqrt(g.ax.p[0][: g.ax.n].double() ** 2 + g.ax.p[1][: g.ax.n].double() ** 2 +
                    g.ax.p[2][: g.ax.n].double() ** 2)
    wa = g.ax.w[: g.ax.n].double()
    Ap, Am = float((pab_plain * wa * Ea).sum()), float((pab_mlp * wa * Ea).sum())
    assert Am == pytest.approx(Ap, rel=0.01)
    # time per evaluation, plain vs surrogate (photons)
    def timed(fn, reps=20):
        fn(); torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record(); torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    tp = timed(lambda: g.rates(g.ph, B.PRIMAKOFF))
    tm = timed(lambda: S.rates(g, g.ph, B.PRIMAKOFF))
    print(f"[surrogate] photon rates: plain {tp * 1e3:.1f} us, surrogate {tm * 1e3:.1f} us "
          f"for {g.ph.n} photons; gain (plain/surrogate time) {tp / tm:.3f}", flush=True)


def test_out_of_box_particles_use_the_plain_rate(trained):
    S = trained
    wl, pl = _small_plasma(T=0.3)          # below the 0.5 keV edge of the training box
    g = AxpicSim(pl, wl.params)
    fb = torch.zeros(1, dtype=torch.int64, device="cuda")
    lam_mlp = S.rates(g, g.ph, B.PRIMAKOFF, fallback=fb)
    lam_plain = g.rates(g.ph, B.PRIMAKOFF)
    torch.cuda.synchronize()
    assert int(fb.item()) == g.ph.n
    np.testing.assert_array_equal(lam_mlp.cpu().numpy(), lam_plain.cpu().numpy())
