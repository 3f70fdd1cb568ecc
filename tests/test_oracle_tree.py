"""Pins for the oracle's reference octree and interaction lists (Sec. 2.5).

Invariants that any correct octree/dual traversal must satisfy, checked
by brute force on small meshes: keys sorted stably, boxes partition their
parent, leaves hold at most N_CRIT panels, box radii cover their points, every
(target panel, source panel) pair is covered exactly once by one P2P pair or
one M2L pair, every M2L pair meets the acceptance test, and no near-singular
pair (Sec. 2.3) lands in an M2L pair.
"""
import numpy as np
import pytest

import synthetic as syn


def leaf_of(T):
    leaf = np.full(T.perm.shape[0], -1)
    for b in range(T.nbox):
        lv, beg, end, par, c0, nc = T.boxes[b]
        if nc == 0:
            assert (leaf[beg:end] == -1).all()
            leaf[beg:end] = b
    assert (leaf >= 0).all()
    return leaf


def ancestors(T):
    anc = []
    for b in range(T.nbox):
        chain = [b]
        p = T.boxes[b, 3]
        while p >= 0:
            chain.append(p)
            p = T.boxes[p, 3]
        anc.append(set(chain))
    return anc


@pytest.mark.parametrize("mesh_fn,ncrit", [(lambda: syn.sphere(3), 16), (lambda: syn.rbc(3), 24),
                                           (lambda: syn.rbc_scene(3, 2, 5), 16)])
def test_tree_structure_and_completeness(orc, mesh_fn, ncrit):
    mesh = mesh_fn()
    theta = 0.5
    T = orc.Tree(mesh.xyz, mesh.tri, ncrit, theta)
    nt = mesh.n_panels
    assert np.array_equal(np.sort(T.perm), np.arange(nt))
    assert (np.diff(T.keys.astype(np.float64)) >= 0).all()
    same = T.keys[1:] == T.keys[:-1]
    assert (T.perm[1:][same] > T.perm[:-1][same]).all()  # stable on ties

    # keys from the stated definition
    c, S, _ = orc.panels(mesh.xyz, mesh.tri)
    lo, side = T.cube[:3], T.cube[3]
    cell = np.minimum(np.floor((c - lo) * (2.0 ** 21 / side)), 2 ** 21 - 1).astype(np.uint64)
    key = np.zeros(nt, dtype=np.uint64)
    for b in range(20, -1, -1):
        for a in range(3):
            key = (key << np.uint64(1)) | ((cell[:, a] >> np.uint64(b)) & np.uint64(1))
    assert np.array_equal(key[T.perm], T.keys)

    # boxes
    assert tuple(T.boxes[0, :4]) == (0, 0, nt, -1)
    for b in range(T.nbox):
        lv, beg, end, par, c0, nc = T.boxes[b]
        assert end > beg
        if nc:
            kids = T.boxes[c0:c0 + nc]
            assert kids[0, 1] == beg and kids[-1, 2] == end
            assert (kids[1:, 1] == kids[:-1, 2]).all()
            assert (kids[:, 3] == b).all() and (kids[:, 0] == lv + 1).all()
            assert end - beg > ncrit
        else:
            assert end - beg <= ncrit or lv == 21
        h = side / 2 ** lv
        ctr = T.box_real[b, :3]
        pts = c[T.perm[beg:end]]
        assert np.max(np.abs(pts - ctr)) <= 0.5 * h * (1 + 1e-12)
        # radius covers centroids and far-rule points
        bary, _ = orc.far_rule()
        v = mesh.xyz[mesh.tri[T.perm[beg:end]]]
        gp = np.einsum("kc,pcd->pkd", bary, v).reshape(-1, 3)
        r = np.sqrt(max(np.max(np.sum((pts - ctr) ** 2, 1)), np.max(np.sum((gp - ctr) ** 2, 1))))
        assert abs(r - T.box_real[b, 3]) <= 1e-14 * max(r, 1.0)
        assert abs(T.box_real[b, 4] - np.sqrt(8 * np.max(S[T.perm[beg:end]]))) < 1e-14 * T.box_real[b, 4]

    # lists sorted, unique
    for L in (T.m2l, T.p2p):
        k = L[:, 0].astype(np.int64) * T.nbox + L[:, 1]
        assert (np.diff(k) > 0).all()
    leaves = T.boxes[:, 5] == 0
    assert leaves[T.p2p[:, 0]].all() and leaves[T.p2p[:, 1]].all()

    # coverage: each (target panel, source panel) exactly once
    cover = np.zeros((nt, nt), dtype=np.int32)  # in sorted order
    for (a, b) in np.concatenate([T.m2l, T.p2p]):
        ba, ea = T.boxes[a, 1:3]
        bb, eb = T.boxes[b, 1:3]
        cover[ba:ea, bb:eb] += 1
    assert (cover == 1).all()

    # acceptance test and near-pair guard on M2L pairs
    R = T.box_real[:, 3]
    for (a, b) in T.m2l:
        d = np.linalg.norm(T.box_real[a, :3] - T.box_real[b, :3])
        assert R[a] + R[b] < theta * d
        ia = T.perm[T.boxes[a, 1]:T.boxes[a, 2]]
        ib = T.perm[T.boxes[b, 1]:T.boxes[b, 2]]
        d2 = np.sum((c[ia][:, None, :] - c[ib][None, :, :]) ** 2, axis=2)
        assert (d2 >= 8 * S[ib][None, :]).all()


def test_tiny_theta_gives_only_p2p(orc):
    mesh = syn.sphere(2)
    T = orc.Tree(mesh.xyz, mesh.tri, 8, 1e-9)
    assert T.m2l.shape[0] == 0
    nleaf = int((T.boxes[:, 5] == 0).sum())
    assert T.p2p.shape[0] == nleaf * nleaf


def test_single_panel_and_flat_cases(orc):
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    T = orc.Tree(xyz, tri, 4, 0.5)
    assert T.nbox == 1 and T.p2p.tolist() == [[0, 0]] and T.m2l.shape[0] == 0
    assert T.cube[3] == 1.0


def test_ncrit_one_reaches_depth(orc):
    mesh = syn.sphere(2)
    T = orc.Tree(mesh.xyz, mesh.tri, 1, 0.5)
    counts = T.boxes[:, 2] - T.boxes[:, 1]
    leaves = T.boxes[:, 5] == 0
    assert (counts[leaves] == 1).all()
