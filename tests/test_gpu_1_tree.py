"""GPU octree and interaction lists equal the CPU reference bit for bit."""
import numpy as np
import pytest

from gpu_util import MESHES, announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,ncrit,theta", [("sphere512", 16, 0.5), ("sphere8192", 64, 0.5),
                                              ("rbc2048", 32, 0.5), ("cells8x512", 24, 0.5),
                                              ("ellipsoid2048", 64, 0.3), ("sphere512", 1, 0.5),
                                              ("sphere2048", 300, 0.7)])
def test_tree_bitexact(orc, name, ncrit, theta):
    from paper_1506_05957_amd import fmmbem as fb
    announce(f"tree {name} ncrit={ncrit} theta={theta}")
    m = MESHES[name]()
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE, fb.params(theta=theta, ncrit=ncrit))
    g = fb.fmmbem_tree(ctx)
    c = orc.Tree(m.xyz, m.tri, ncrit, theta)
    assert np.array_equal(g["cube"].view(np.uint64), c.cube.view(np.uint64))
    assert np.array_equal(g["keys"], c.keys)
    assert np.array_equal(g["perm"], c.perm)
    assert np.array_equal(g["boxes"], c.boxes)
    assert g["nlevels"] == c.nlevels
    assert np.array_equal(g["box_real"].view(np.uint64), c.box_real.view(np.uint64))
    assert np.array_equal(g["m2l"], c.m2l)
    assert np.array_equal(g["p2p"], c.p2p)
    st = fb.fmmbem_get_stats(ctx)
    assert st["n_boxes"] == c.nbox and st["n_m2l"] == c.m2l.shape[0] and st["n_p2p"] == c.p2p.shape[0]
    fb.fmmbem_destroy(ctx)


def test_zero_area_triangle_rejected():
    from paper_1506_05957_amd import fmmbem as fb
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]])
    tri = np.array([[0, 1, 2], [0, 1, 3]], dtype=np.int32)
    with pytest.raises(fb.FmmbemError) as e:
        fb.fmmbem_build(xyz, tri, fb.LAPLACE)
    assert e.value.code == fb.EINVAL


def test_single_triangle():
    from paper_1506_05957_amd import fmmbem as fb
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    ctx = fb.fmmbem_build(xyz, tri, fb.LAPLACE)
    st = fb.fmmbem_get_stats(ctx)
    assert st["n_boxes"] == 1 and st["n_p2p"] == 1 and st["n_m2l"] == 0 and st["nnz_correction"] == 1
    fb.fmmbem_destroy(ctx)
