"""Seeded generators: determinism and the geometric recipe (closed-form checks)."""
import numpy as np
import pytest

from paper_1901_06229_amd import synth


def bonds_of(xyz):
    d = np.linalg.norm(xyz[:, None] - xyz[None], axis=-1)
    i, j = np.nonzero(np.triu(np.abs(d - 1.5) < 1e-4, 1))
    return list(zip(i.tolist(), j.tolist())), d


def graph_dist(n, bonds):
    INF = 10 ** 6
    D = np.full((n, n), INF, np.int64)
    np.fill_diagonal(D, 0)
    adj = [[] for _ in range(n)]
    for a, b in bonds:
        adj[a].append(b)
        adj[b].append(a)
    for s in range(n):
        q = [s]
        while q:
            x = q.pop(0)
            for y in adj[x]:
                if D[s, y] == INF:
                    D[s, y] = D[s, x] + 1
                    q.append(y)
    return D, adj


def test_deterministic_and_counter_based():
    a = synth.ligands(2, count=40)
    b = synth.ligands(2, count=40)
    for f in ("atom_offset", "xyz", "rot_offset", "rot_axis", "move_offset", "move_atoms"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = synth.ligands(2, count=10, first=20)
    for l in range(10):
        x, y = a.ligand(20 + l), c.ligand(l)
        for k in x:
            assert np.array_equal(x[k], y[k])
    assert np.array_equal(synth.orientations(2, 16), synth.orientations(2, 16))
    assert not np.array_equal(synth.ligands(2, count=3, seed=99).xyz, a.subset([0, 1, 2]).xyz)


@pytest.mark.parametrize("config", [1, 2, 3, 5])
def test_tree_geometry_and_clash_free(config):
    ligs = synth.ligands(config, count=6 if config == 5 else 25)
    for l in range(ligs.n_ligands):
        lig = ligs.ligand(l)
        xyz = lig["xyz"].astype(np.float64)
        n = len(xyz)
        bonds, d = bonds_of(xyz)
        assert len(bonds) == n - 1, "a tree has n-1 bonds of 1.5 A"
        D, adj = graph_dist(n, bonds)
        assert (D < 10 ** 6).all(), "connected"
        assert max(len(x) for x in adj) <= 4, "valence <= 4"
        # bond angles: every angle at an atom is near tetrahedral
        for p in range(n):
            for i in range(len(adj[p])):
                for j in range(i + 1, len(adj[p])):
                    u = xyz[adj[p][i]] - xyz[p]
                    v = xyz[adj[p][j]] - xyz[p]
                    ang = np.degrees(np.arccos(np.dot(u, v) / np.linalg.norm(u) / np.linalg.norm(v)))
                    assert 95.0 < ang < 125.0
        # atoms >= 3 bonds apart are >= r_bump + 0.1 apart
        far = D >= 3
        assert (d[far] >= synth.R_BUMP + 0.1 - 1e-4).all()
        assert abs(xyz.mean(0)).max() < 1e-4, "centred on the centroid"


@pytest.mark.parametrize("config", [1, 2, 3, 5])
def test_rotamers_are_subtrees(config):
    ligs = synth.ligands(config, count=4 if config == 5 else 20)
    for l in range(ligs.n_ligands):
        lig = ligs.ligand(l)
        xyz = lig["xyz"].astype(np.float64)
        n = len(xyz)
        bonds, _ = bonds_of(xyz)
        D, adj = graph_dist(n, bonds)
        R = len(lig["rot_axis"])
        assert R == min(int(ligs.r_target[l]), int(ligs.eligible[l]))
        depth = D[0]
        prev = (-1, -1)
        for r in range(R):
            a, b = (int(v) for v in lig["rot_axis"][r])
            assert (min(a, b), max(a, b)) in bonds
            assert depth[b] == depth[a] + 1, "b is the child end"
            key = (int(depth[b]), b)
            assert key > prev, "ordered by depth of b, then index"
            prev = key
            M = lig["move_atoms"][lig["move_offset"][r]:lig["move_offset"][r + 1]].tolist()
            assert M == sorted(M) and len(M) >= 1
            # the moving set: atoms reached from b without crossing a, minus b
            seen, stack = {b}, [b]
            while stack:
                x = stack.pop()
                for y in adj[x]:
                    if y != a and y not in seen:
                        seen.add(y)
                        stack.append(y)
            assert set(M) == seen - {b}


def test_config_distributions():
    c2 = synth.ligands(2, count=2000)
    n = np.diff(c2.atom_offset)
    R = np.diff(c2.rot_offset)
    assert n.min() >= 20 and n.max() <= 80 and abs(n.mean() - 50) < 2
    assert R.min() >= 2 - 2 and R.max() <= 12
    c3 = synth.ligands(3, count=4000)
    n3 = np.diff(c3.atom_offset)
    assert n3.min() >= 8 and n3.max() <= 150 and abs(np.median(n3) - 40) <= 2
    r3 = np.round(40 * (n3 - 8) / 142)
    assert (np.diff(c3.rot_offset) <= r3).all()
    c1 = synth.ligands(1)
    assert c1.n_ligands == 1 and c1.n_atoms(0) == 32 and c1.n_rot(0) == 4


@pytest.mark.parametrize("config", [1, 2])
def test_pocket_recipe(config):
    p = synth.pocket(config)
    G = p.grid.shape[0]
    h = p.spacing
    c = p.origin[0] + (np.arange(G) + 0.5) * h
    X, Y, Z = np.meshgrid(c, c, c, indexing="xy")  # [y, x, z]
    inside = (X / 10) ** 2 + (Y / 8) ** 2 + (Z / 6) ** 2 <= 1
    inside = np.transpose(inside, (2, 0, 1))  # -> [z, y, x]
    assert np.all(p.grid[~inside] == -1000.0)
    v = p.grid[inside]
    assert v.min() > 0 and v.max() <= 8.0
    assert p.origin[0] == -G * h / 2


def test_orientations_are_rotations():
    o = synth.orientations(2, 64).astype(np.float64)
    R = o[:, :9].reshape(-1, 3, 3)
    assert np.abs(R @ R.transpose(0, 2, 1) - np.eye(3)).max() < 1e-6
    assert np.abs(np.linalg.det(R) - 1).max() < 1e-6
    assert np.all(o[:, 9:] == 0)
