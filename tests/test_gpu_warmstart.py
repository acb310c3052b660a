"""The learned warm start end to end on a small member of the parametric
portfolio family: batched solves give the training targets, the network is
trained on the GPU, and on held-out parameters its predicted starting points
are compared with cold starts (the fallback and the yardstick)."""
import numpy as np
import pytest

from paper_2505_00311_amd import instances as I

pytestmark = pytest.mark.gpu


def test_warm_start_saves_iterations_on_held_out_parameters(pd, orc):
    from paper_2505_00311_amd import warmstart as W
    fam = I.PortfolioFamily(11, n_assets=1000, k=20)
    train_th = fam.thetas(12, 512)
    test_th = fam.thetas(13, 64)
    res, _ = W.solve_family(fam, train_th)
    assert all(r["status"] == 0 for r in res)
    T = W.targets_of(res)
    net, norm, hist, _ = W.train(train_th, T, hidden=256, epochs=120, batch=128, lr=1e-3)
    assert hist[-1] < 0.5 * hist[0], (hist[0], hist[-1])
    cold, _ = W.solve_family(fam, test_th)
    starts = W.predict(net, norm, test_th, fam.n, fam.m)
    warm, _ = W.solve_family(fam, test_th, starts=starts)
    assert all(r["status"] == 0 for r in cold + warm)
    it_cold = np.mean([r["iterations"] for r in cold])
    it_warm = np.mean([r["iterations"] for r in warm])
    print("held-out mean iterations: cold", it_cold, "warm", it_warm, flush=True)
    assert it_warm < 0.9 * it_cold, (it_cold, it_warm)
    # the warm answers are as good as the cold ones by the oracle's measures
    for t, r, c in list(zip(test_th, warm, cold))[:4]:
        inst = fam.instance(t)
        k = orc.kkt(inst, r["x"], r["y"])
        assert max(k["err_p"], k["err_d"], k["err_gap"]) <= 1.01e-6, k
        assert r["pobj"] == pytest.approx(c["pobj"], rel=1e-5, abs=1e-5)
    net.close()
