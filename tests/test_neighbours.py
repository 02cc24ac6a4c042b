"""Nearest-neighbour selection for the inter-site V (Eq. 9 in the q-supercell of Eq. 12).

The oracle's brute-force selection is pinned to closed-form geometries, and to a wider
image search on random sheared cells; the library's host routine (hp_neighbours, no GPU
needed) is then held to the oracle on random geometries and on the workload cells."""
import itertools

import numpy as np
import pytest

import oracle

A8 = np.eye(3) * 8.0


def test_oracle_simple_cubic_chain():
    # one site, q mesh 2x1x1: the only other supercell site is the copy one cell along a1
    assert oracle.nearest_neighbours(A8, [[0, 0, 0]], (2, 1, 1)) == [(0, 1, 8.0)]


def test_oracle_lone_site_has_no_neighbours():
    assert oracle.nearest_neighbours(A8, [[1, 2, 3]], (1, 1, 1)) == []


def test_oracle_simple_cubic_square():
    # q mesh 2x2x1: cells (0,1,0) -> 1 and (1,0,0) -> 2 at distance a; (1,1,0) -> 3 at a sqrt 2
    assert oracle.nearest_neighbours(A8, [[0, 0, 0]], (2, 2, 1)) == [(0, 1, 8.0), (0, 2, 8.0)]


def test_oracle_two_sites_in_cell():
    nn = oracle.nearest_neighbours(A8, [[0, 0, 0], [4, 0, 0]], (1, 1, 1))
    assert nn == [(0, 1, 4.0), (1, 0, 4.0)]
    # off-centre second site: distance to the nearer image
    nn = oracle.nearest_neighbours(A8, [[0, 0, 0], [5.5, 1, 0]], (1, 1, 1))
    assert nn[0][:2] == (0, 1) and abs(nn[0][2] - np.hypot(2.5, 1.0)) < 1e-14


def test_oracle_threshold_groups_near_ties():
    tau = [[0, 0, 0], [3.0, 0, 0], [0, 3.0 + 4e-4, 0]]
    ids = {j for i, j, _ in oracle.nearest_neighbours(A8, tau, (1, 1, 1)) if i == 0}
    assert ids == {1, 2}
    ids = {j for i, j, _ in oracle.nearest_neighbours(A8, tau, (1, 1, 1), dist_thr=1e-4) if i == 0}
    assert ids == {1}


def _wide_search(cell, tau, qmesh, dist_thr=6e-4, reach=4):
    """Same definition with supercell images `reach` shells out, plain loops."""
    A = np.asarray(cell).reshape(3, 3)
    tau = np.asarray(tau)
    nh = len(tau)
    cells = [(a, b, c) for a in range(qmesh[0]) for b in range(qmesh[1]) for c in range(qmesh[2])]
    pos = [tau[s] + np.array(c) @ A for c in cells for s in range(nh)]
    asc = np.diag(qmesh) @ A
    out = []
    for i in range(nh):
        d = []
        for j in range(len(pos)):
            best = np.inf
            for u, v, w in itertools.product(range(-reach, reach + 1), repeat=3):
                best = min(best, np.linalg.norm(pos[j] - pos[i] + np.array([u, v, w]) @ asc))
            d.append(best if j != i else np.inf)
        dmin = min(d)
        out += [(i, j, d[j]) for j in range(len(pos)) if np.isfinite(dmin) and d[j] <= dmin + dist_thr]
    return out


def _random_case(seed):
    rng = np.random.default_rng(seed)
    cell = np.diag(rng.uniform(6, 12, 3)) + np.triu(rng.uniform(-1.5, 1.5, (3, 3)), 1)
    nh = int(rng.integers(1, 4))
    tau = rng.uniform(0, 1, (nh, 3)) @ cell
    qmesh = tuple(int(x) for x in rng.integers(1, 3, 3))
    return cell, tau, qmesh


@pytest.mark.parametrize("seed", range(6))
def test_oracle_against_wide_search(seed):
    cell, tau, qmesh = _random_case(seed)
    a = oracle.nearest_neighbours(cell, tau, qmesh)
    b = _wide_search(cell, tau, qmesh)
    assert [x[:2] for x in a] == [x[:2] for x in b]
    assert np.allclose([x[2] for x in a], [x[2] for x in b], rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(10))
def test_library_matches_oracle(seed):
    from paper_2203_15684_amd import hp
    cell, tau, qmesh = _random_case(100 + seed)
    a = hp.hp_neighbours(cell, tau, qmesh)
    b = oracle.nearest_neighbours(cell, tau, qmesh)
    assert [x[:2] for x in a] == [x[:2] for x in b]
    assert np.allclose([x[2] for x in a], [x[2] for x in b], rtol=0, atol=1e-12)


@pytest.mark.parametrize("name,rep", [("duo_k221", 1), ("olivine28", 1), ("olivine28", 2)])
def test_library_matches_oracle_workload_cells(name, rep):
    """The Hubbard sites of the workload cells (first draw), and of the 2x1x1 supercell."""
    from paper_2203_15684_amd import hp
    from synth import spec_by_name
    from synth.system import _draw_atoms
    spec = spec_by_name(name)
    atoms, _, _ = _draw_atoms(spec, 0)
    tau = np.asarray(atoms.tau)[: spec.n_hub]
    cell = np.diag(spec.cell).astype(float)
    if rep == 2:
        tau = np.vstack([tau, tau + cell[0]])
        cell[0] *= 2
    a = hp.hp_neighbours(cell, tau, spec.qmesh)
    b = oracle.nearest_neighbours(cell, tau, spec.qmesh)
    assert [x[:2] for x in a] == [x[:2] for x in b]
    assert np.allclose([x[2] for x in a], [x[2] for x in b], rtol=0, atol=1e-12)


def test_library_rejects_bad_arguments():
    from paper_2203_15684_amd import hp
    with pytest.raises(hp.HpError):
        hp.hp_neighbours(A8, [[0, 0, 0]], (0, 1, 1))
    with pytest.raises(hp.HpError):
        hp.hp_neighbours(A8, [[0, 0, 0]], (1, 1, 1), dist_thr=-1.0)
