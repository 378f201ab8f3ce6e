"""The learned initialiser pipeline on the 256 x 256 slice workload: pairs
made by split SART agree with the FP64 oracle, a network whose start is worse
is rejected (fallback to the 5-iteration image), and a briefly trained
network gives starts with a lower residual than the image it starts from.
The last is a property of training, stochastic: parity unpinned."""
import numpy as np
import pytest

from gpu_util import banner, rel_l2, to_np
from oracle import geometry as G
from oracle import sart as OS
from paper_1902_10559_amd import inputs, learned, unet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    return learned.scan()


def test_training_pairs_match_the_oracle(sc):
    banner("learned: pairs vs oracle")
    X, Y = learned.make_pairs(sc, [0, 1, 2], iters_in=5, iters_out=20)
    g = inputs.geometry_cfg5()
    A = G.to_fp32(G.system_matrix(g))
    f_true = G.image_to_snake(inputs.phantom_for(5, 1, g))
    p = (A.astype(np.float64) @ f_true).astype(np.float32)
    for k, img in ((5, X[1]), (20, Y[1])):
        f_ref, _ = OS.sart_full(A, p, 0.5, k)
        got = to_np(img).reshape(g.nz, g.nx)
        assert rel_l2(got, G.snake_to_image(f_ref, g.nx, g.nz)) <= 1e-5


def test_a_worse_learned_start_is_rejected(sc):
    import torch
    banner("learned: fallback")
    net = unet.UNet(sc.geom.nz, sc.geom.nx, seed=3)
    L = net.layers["out"]
    L.b.fill_(50.0)          # the network now adds a large constant: a bad start
    net.prep()
    items = [7, 8]
    systems = learned.systems_for(sc, learned.folded_projections(sc, items))
    f5 = [sc.S.new_image() for _ in items]
    h5 = [torch.empty(6, dtype=torch.float64, device="cuda") for _ in items]
    learned.solve(systems, f5, 5, zero_start=True, res=h5)
    res5 = [h[5].item() for h in h5]
    starts, acc, res_l = learned.learned_starts(net, sc, systems, f5, res5)
    assert acc == [False, False] and all(r > q for r, q in zip(res_l, res5))
    for s, f in zip(starts, f5):
        assert np.array_equal(to_np(s), to_np(f))


def test_brief_training_lowers_the_start_residual(sc):
    banner("learned: brief training")
    X, Y = learned.make_pairs(sc, list(range(100, 356)), iters_in=5, iters_out=200)
    net = unet.UNet(sc.geom.nz, sc.geom.nx, seed=0)
    losses = learned.train(net, X, Y, epochs=3, batch=8, lr=1e-3)
    banner(f"losses {losses[0]:.3e} -> {losses[-1]:.3e}")
    rep = learned.evaluate(net, sc, list(range(10 ** 6, 10 ** 6 + 16)), tols=(1e-2,), cap=3000)
    banner(f"report {rep}")
    assert rep["res_learned_start"] < rep["res_after_5"]
    assert rep["accepted"] >= 8
    # and the learned start saves iterations to 1e-2 (median over the 16)
    t = rep["tolerances"]["0.01"]
    assert t["learned_reached"] == t["plain_reached"] == 16
    assert t["learned_median_iters"] < t["plain_median_iters"], t
