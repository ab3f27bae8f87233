"""Graph replays of the step launch (jg_params.use_graph) against direct launches.

The graph holds the same kernels with the same arguments but the first step's index, which a
replay rewrites, so every replay must give the bits of the direct launch.  The calls cross the
start of the seeded pushes (the index decides when a force acts), change the step count (one
graph per count), run back to back without waiting, and alternate with eager work: state
downloads, a state upload and warm-store clears."""
import sys

import numpy as np
import pytest

from paper_2606_28394_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    from paper_2606_28394_amd import jenga
    jenga.load_library()
    return jenga


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mixed_scene():
    """Removal towers (pushes from step 60) beside a 9 x 32 wall kept in device memory: two
    launch classes in one graph."""
    towers = W.cfg2(0, n_per_mu=2, n_steps=200)
    wall = W.masonry_wall(9, 32, seed=4)
    sb = W.SceneBuilder(W.default_params(), 200)
    ptr = towers["tower_ptr"]
    for t in range(towers["n_towers"]):
        a, b = int(ptr[t]), int(ptr[t + 1])
        sb.add_tower(towers["half_extents"][a:b], towers["mass"][a:b], towers["pos"][a:b], towers["quat"][a:b],
                     towers["mu"][t], towers["linvel"][a:b], towers["angvel"][a:b])
    for i in range(len(towers["push_body"])):
        b = int(towers["push_body"][i])
        sb.add_push(b, towers["push_force"][i], int(towers["push_start"][i]), int(towers["push_steps"][i]),
                    float(towers["push_withdraw"][i]))
    wp = wall["tower_ptr"]
    for t in range(wall["n_towers"]):
        a, b = int(wp[t]), int(wp[t + 1])
        sb.add_tower(wall["half_extents"][a:b], wall["mass"][a:b], wall["pos"][a:b], wall["quat"][a:b],
                     wall["mu"][t], wall["linvel"][a:b], wall["angvel"][a:b])
    return sb.build()


def _same(a, b, what):
    for x, y in zip(a, b):
        assert np.array_equal(x, y), what


@pytest.mark.parametrize("warm_start", [0, 1])
def test_graph_replays_match_direct_launches(J, warm_start):
    sc = _mixed_scene()
    assert len(sc["push_body"]) > 0 and min(sc["push_start"]) == 60
    _say(f"graph vs direct, warm_start {warm_start}: {sc['n_towers']} towers, {int(sc['tower_ptr'][-1])} bodies")
    direct = J.World(sc, warm_start=warm_start)
    graph = J.World(sc, warm_start=warm_start, use_graph=True)
    init = direct.state()
    done = 0
    for calls in ([20, 20], [10, 10, 10], [20, 5, 5]):   # back to back, then compared
        for n in calls:
            direct.step(n)
            graph.step(n)
            done += n
        _say(f"  after {done} steps")
        _same(direct.state(), graph.state(), f"state after {done} steps")
    s_d, s_g = direct.stats(), graph.stats()
    assert s_d.error_word == 0 and s_g.error_word == 0
    assert (s_d.manifolds, s_d.points, s_d.contact_iters) == (s_g.manifolds, s_g.points, s_g.contact_iters)
    for t in (0, 3, sc["n_towers"] - 1):
        cd, cg = direct.contacts(t), graph.contacts(t)
        assert len(cd) == len(cg)
        for f in ("body_a", "body_b", "slot", "point", "lambda_n", "lambda_t1", "lambda_t2"):
            assert np.array_equal(cd[f], cg[f]), f"tower {t} contact field {f}"
    # an upload between replays (the layout and buffers stay, so the graphs are reused)
    direct.set_state(*init)
    graph.set_state(*init)
    for n in (20, 20, 5):
        direct.step(n)
        graph.step(n)
    _same(direct.state(), graph.state(), "state after the restored start")
    direct.close()
    graph.close()


def test_graph_follows_a_changed_layout(J):
    """A push added between calls changes the layout (pushes per pack, LDS): the graph built
    before it is rebuilt, and the push acts from the step it names."""
    sc = W.tilted_towers(3, 12, seed=21, n_steps=40)
    direct = J.World(sc)
    graph = J.World(sc, use_graph=True)
    for w in (direct, graph):
        w.step(10)
        w.step(10)
    body = int(sc["tower_ptr"][5]) + 4
    for w in (direct, graph):
        J.jg_set_push(w.h, body, [0.02, 0.0, 0.0], 20, 15)
        w.step(10)
        w.step(10)
    _same(direct.state(), graph.state(), "state after the layout change")
    direct.close()
    graph.close()
