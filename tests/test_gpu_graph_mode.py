"""Graph mode of the single-scene step (a captured one-scene batch): the
same commands, validation flags and nominals as eager steps, bit for bit,
over chained steps; rebuilt on a parameter change, re-planned after new
points."""
import numpy as np
import pytest

from paper_2605_29663_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29663_amd as p
    p.load()
    return p


def _ctx(pkg, sc, kind=0):
    c = pkg.Context(0)
    c.set_footprint(kind, sc["polygon"] if kind == 0 else sc["rects"])
    c.set_points(sc["ox"], sc["oy"], sc.get("ovx"), sc.get("ovy"))
    return c


@pytest.mark.parametrize("name", ["c1", "c3", "c1-quad"])
def test_graph_mode_equals_eager(pkg, name):
    """c1-quad: the c1 scene with a 64-vertex footprint (lane quads)."""
    import torch
    prm, sc = scenes.config(name.split("-")[0], K=256, T=20)
    if name.endswith("quad"):
        sc = dict(sc, polygon=scenes.star_polygon(np.random.default_rng(64), 64, 0.15, 0.4))
    kind = prm["footprint_kind"]
    eager, graph = _ctx(pkg, sc, kind), _ctx(pkg, sc, kind)
    graph.mppi_set_graph(True)
    Ue = torch.zeros((prm["T"], prm["nu"]), device="cuda")
    Ug = torch.zeros_like(Ue)
    q = np.zeros(3, np.float32)
    for t in range(5):
        ue, ve, _ = eager.mppi_step(prm, q, Ue, 9, t)
        ug, vg, _ = graph.mppi_step(prm, q, Ug, 9, t)
        np.testing.assert_array_equal(ue, ug)
        assert ve == vg
        assert torch.equal(Ue, Ug)
        q = q + np.float32([0.05, 0.01, 0.02])
    # a parameter change rebuilds the graph
    prm2 = dict(prm, K=128, lambda_=0.5)
    ue, ve, _ = eager.mppi_step(prm2, q, Ue, 9, 7)
    ug, vg, _ = graph.mppi_step(prm2, q, Ug, 9, 7)
    np.testing.assert_array_equal(ue, ug)
    assert torch.equal(Ue, Ug)
    # new points: the graph path re-plans
    for c in (eager, graph):
        c.set_points(sc["ox"][:300], sc["oy"][:300],
                     None if sc.get("ovx") is None else sc["ovx"][:300],
                     None if sc.get("ovy") is None else sc["ovy"][:300])
    ue, ve, _ = eager.mppi_step(prm2, q, Ue, 9, 8)
    ug, vg, _ = graph.mppi_step(prm2, q, Ug, 9, 8)
    np.testing.assert_array_equal(ue, ug)
    assert torch.equal(Ue, Ug)
    # diagnostics take the eager path even in graph mode
    _, _, D = graph.mppi_step(prm2, q, Ug.clone(), 9, 9, diag=True)
    assert D["d_min"].shape == (prm2["K"], prm2["T"])
    graph.mppi_set_graph(False)
    eager.close()
    graph.close()


def test_graph_mode_profiling_times_the_batch(pkg):
    """With profiling on, graph mode runs its one-scene batch eagerly (same
    bits as the replay) and reports one timed distance pass per step."""
    import torch
    prm, sc = scenes.config("c1", K=256, T=20)
    a, b = _ctx(pkg, sc), _ctx(pkg, sc)
    a.mppi_set_graph(True)
    b.mppi_set_graph(True)
    Ua = torch.zeros((prm["T"], prm["nu"]), device="cuda")
    Ub = torch.zeros_like(Ua)
    q = np.zeros(3, np.float32)
    b.mppi_set_profiling(True)
    for t in range(3):
        ua, va, _ = a.mppi_step(prm, q, Ua, 4, t)
        ub, vb, _ = b.mppi_step(prm, q, Ub, 4, t)
        np.testing.assert_array_equal(ua, ub)
        assert va == vb
        assert torch.equal(Ua, Ub)
    ms, n = b.mppi_get_profile()
    assert n == 3 and ms > 0.0
    b.mppi_set_profiling(False)
    a.close()
    b.close()
