"""Host-side pieces of the closed-loop docking benchmark (CPU only)."""
import numpy as np


def test_convex_hull_of_fork_and_star():
    from paper_2605_29663_amd import closed_loop, scenes
    h = closed_loop.convex_hull(closed_loop.FOOTPRINT_FORK)
    np.testing.assert_allclose(sorted(map(tuple, h)),
                               sorted([(-0.5, -0.4), (1.1, -0.4), (1.1, 0.4), (-0.5, 0.4)]))
    # a hull contains every vertex and is convex (all turns to the left)
    rng = np.random.default_rng(3)
    V = scenes.star_polygon(rng, 23)
    H = closed_loop.convex_hull(V)
    n = len(H)
    for k in range(n):
        a, b, c = H[k], H[(k + 1) % n], H[(k + 2) % n]
        assert (b[0] - a[0]) * (c[1] - b[1]) - (b[1] - a[1]) * (c[0] - b[0]) > 0
        for v in V:
            e = (b[0] - a[0]) * (v[1] - a[1]) - (b[1] - a[1]) * (v[0] - a[0])
            assert e >= -1e-12


def test_docking_goal_puts_the_post_in_the_concavity():
    from oracle import oracle as orc
    from paper_2605_29663_amd import closed_loop as cl
    # the post centre, seen from the docked pose, lies between the forks:
    # outside the footprint, inside its hull
    p = (cl.POST[0] - cl.GOAL[0], cl.POST[1] - cl.GOAL[1])
    assert orc.sdf_polygon(cl.FOOTPRINT_FORK, [p[0]], [p[1]])[0] > cl.POST_R
    assert orc.sdf_polygon(cl.convex_hull(cl.FOOTPRINT_FORK), [p[0]], [p[1]])[0] < -cl.POST_R
