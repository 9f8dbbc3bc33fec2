"""The synthetic workloads have the structure the scene builder's big-triangle
rule is described against: the lattice's room walls, floor and roof are its
only big triangles, and the displaced spheres have none (host only)."""

import numpy as np

from tests.parity_util import big_tris
from workloads import make_workload
from workloads.lattice import room_mesh


def test_lattice_big_triangles_are_the_room():
    w = make_workload("lattice", H=8, W=8, n_views=1)
    big = big_tris(w.verts, w.tris)
    n_room = len(room_mesh()[1])
    assert n_room == 36
    # the room is merged after the beams: its triangles are the last ones
    assert np.array_equal(np.nonzero(big)[0], np.arange(len(w.tris) - n_room, len(w.tris)))


def test_displaced_spheres_have_no_big_triangles():
    for freq in (12, 40):
        w = make_workload("sphere8", H=8, W=8, n_views=1, freq=freq)
        assert not big_tris(w.verts, w.tris).any()
