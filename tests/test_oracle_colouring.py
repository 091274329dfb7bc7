"""Pins of the oracle's nearest-point colouring of Sigma with flood fill over the
lattice's convex hull (Sec. 3), against independent constructions: qhull's convex
hull, graph distances from scipy's shortest paths, exact seeds on lattice points."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components, shortest_path
from scipy.spatial import ConvexHull

import oracle


def qhull_edges(p):
    e = set()
    for t in ConvexHull(p).simplices:
        a, b, c = sorted(int(x) for x in t)
        e |= {(a, b), (a, c), (b, c)}
    return e


@pytest.mark.parametrize("N", [4, 10, 37, 100, 128])
def test_hull_edges_match_qhull(N):
    nb = oracle.hull_adjacency(N)
    ours = {(i, j) for i in range(N) for j in nb[i] if i < j}
    assert ours == qhull_edges(oracle.lattice(N))
    assert all(nb[i] == sorted(nb[i]) for i in range(N))


def hull_graph(N):
    nb = oracle.hull_adjacency(N)
    r = [i for i in range(N) for _ in nb[i]]
    c = [j for i in range(N) for j in nb[i]]
    return csr_matrix((np.ones(len(r)), (r, c)), shape=(N, N))


def test_one_direction_colours_everything():
    assert np.all(oracle.colours(None, np.array([[0.3, -0.2, 0.9327379053]]), 100) == 0)


def test_seeds_sit_on_their_lattice_points():
    p = oracle.lattice(100)
    ks = [3, 41, 77, 90]
    col = oracle.colours(None, p[ks], 100)
    for m, k in enumerate(ks):
        assert col[k] == m


def test_fill_follows_graph_distance_from_the_seeds():
    N = 100
    p = oracle.lattice(N)
    col = oracle.colours(None, np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]), N)
    dist = shortest_path(hull_graph(N), unweighted=True, indices=[int(np.argmax(p[:, 2])),
                                                                  int(np.argmin(p[:, 2]))])
    for i in range(N):
        if dist[0, i] < dist[1, i]:
            assert col[i] == 0
        elif dist[1, i] < dist[0, i]:
            assert col[i] == 1
    # every colour class is connected along the hull
    G = hull_graph(N).tolil()
    for c in (0, 1):
        idx = np.flatnonzero(col == c)
        n, _ = connected_components(G[idx][:, idx], directed=False)
        assert n == 1


def test_a_point_claimed_twice_goes_to_the_closer_direction():
    p = oracle.lattice(100)
    k = 50
    near = p[k]
    off = p[k] + 0.01 * np.cross(p[k], [0.0, 0.0, 1.0])
    off /= np.linalg.norm(off)
    col = oracle.colours(None, np.array([off, near]), 100)  # the later one is closer
    assert col[k] == 1
    # the farther direction owns nothing: its only seed was taken
    assert np.count_nonzero(col == 0) == 0


def test_rotation_is_applied():
    # incoming direction +x: the lattice's pole turns to +x, so the direction along
    # +x owns the pole's neighbourhood in the rotated frame
    dirs = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    col = oracle.colours(np.array([1.0, 0.0, 0.0]), dirs, 100)
    p = oracle.lattice(100)
    assert col[int(np.argmax(p[:, 2]))] == 0 and col[int(np.argmin(p[:, 2]))] == 1


def test_pipeline_reads_the_mode_and_stays_close_to_voronoi():
    # the colouring and the Voronoi cells discretise the same Sigma: the radiances
    # differ, by a fraction of a percent on average
    from paper_2503_16037_amd import scenes
    sc = scenes.make_plain()
    a = oracle.run(sc)["radiance"]
    b = oracle.run(sc.with_(sigma_mode=1))["radiance"]
    d = np.abs(a - b) / a
    assert d.max() > 1e-3 and d.mean() < 0.02
