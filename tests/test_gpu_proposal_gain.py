"""What the trained proposal gains: on held-out corridor states (seeds
disjoint from training), one MPPI update at K = 1024 around the network's
mean (with the plain shifted nominal as fallback) against the same update
around the plain shifted nominal at K = 1024 and at K = 4096, scored by the
noise-free cost of the updated nominal.  Uses the shipped weights, trained
on the GPU by the library's own kernels (paper_2605_29663_amd.train_proposal)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2605_29663_amd", "proposal_c2.bin")


@pytest.fixture(scope="module")
def pkg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29663_amd as p
    p.load()
    return p


def test_trained_proposal_beats_plain_at_equal_rollouts(pkg):
    from paper_2605_29663_amd import learn
    assert os.path.exists(WEIGHTS)
    net = pkg.Proposal(40, 2, hidden=256, max_batch=64)
    net.load(WEIGHTS)
    costs, fallback = learn.evaluate(net, n_states=96, n_parallel=16, warm_steps=20, repeats=2,
                                     seed0=learn.HELDOUT_SEED0 + 500000, log=lambda m: None)
    s = learn.summarize(costs, fallback, n_boot=500)
    print(s)
    g = s["learned_small_over_plain_small"]
    # at the same number of rollouts the learned mean lowers the final cost
    # in more states than it raises it (1000 held-out states: 676 lower, 74
    # equal (fallback), 225 higher) ...
    assert g["states_lower"] > g["states_higher"], s
    # ... while the ratio of mean costs stays level with plain MPPI at K =
    # 1024 (1000 states: 1.0004, 95 % interval 0.988 - 1.012; both are 1.028
    # of plain K = 4096, so the 2 % target at a quarter of the rollouts is not
    # met on this workload); on 96 states the bound is loose
    assert g["ratio"] < 1.05, s


def test_broken_network_falls_back_to_plain(pkg):
    """NaN weights: the mean maps to the box edge, loses the noise-free cost
    comparison, and the update is the plain one from the shifted nominal, bit
    for bit."""
    import torch
    from paper_2605_29663_amd import learn, scenes
    sc = learn.corridor_scene(learn.HELDOUT_SEED0 + 42)
    prm = learn.scene_params(sc, 512)
    ctx = learn.make_context(sc)
    net = pkg.Proposal(40, 2, hidden=256, max_batch=8)
    net.set_params(np.full(net.n_params, np.nan, dtype=np.float32))
    q = np.float32([0.1, 0.0, 0.05])
    U_shift = torch.zeros((40, 2), device="cuda")
    u, v, D, fb = learn.learned_update(net, ctx, prm, q, U_shift, seed=3, K=512)
    assert fb
    U = U_shift.clone()
    u2, v2, D2 = ctx.mppi_step(dict(prm, K=512, validate=1), q, U, 3, 0, diag=True)
    np.testing.assert_array_equal(u, u2)
    assert v == v2
    assert torch.equal(D["U_upd"], D2["U_upd"])
