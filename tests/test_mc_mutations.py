"""Plant plausible mistakes in the Marching Cubes oracle (on the CPU) and
check that at least one pin of ``test_mc_oracle`` fails under each."""
import numpy as np
import pytest

from oracle import mc
import test_mc_oracle as pins

_backward = mc.mc_backward
_normals = mc.grid_normals
_polygons = mc._case_polygons
_apex = mc._fan_apex


def backward_sign(mesh, dverts, r):
    return -_backward(mesh, dverts, r)


def backward_weights_swapped(mesh, dverts, r):
    m = dict(mesh)
    m["t"] = 1.0 - mesh["t"]
    return _backward(m, dverts, r)


def normals_flipped(chi):
    return -_normals(chi)


def normals_unscaled_axis(chi):
    g = _normals(chi)
    g[2] *= 2.0  # a wrong spacing along one axis
    return g


def polygons_reversed(case):
    return [loop[::-1] for loop in _polygons(case)]


def fan_from_first(loop):
    return 0


MUTATIONS = {
    "backward sign": ("mc_backward", backward_sign),
    "backward weights swapped": ("mc_backward", backward_weights_swapped),
    "normals flipped": ("grid_normals", normals_flipped),
    "normal spacing": ("grid_normals", normals_unscaled_axis),
    "triangles inward": ("_case_polygons", polygons_reversed),
    "fan apex on a face": ("_fan_apex", fan_from_first),
}

PINS = [
    lambda: pins.test_every_case_closed_and_manifold_on_random_fields(),
    lambda: pins.test_vertices_on_the_level_and_on_their_edges(),
    lambda: pins.test_plane(),
    lambda: pins.test_euler_characteristic("sphere", 2),
    lambda: pins.test_sphere_area_volume_converge_and_face_outward(),
    lambda: pins.test_backward_is_the_normal_derivative_on_a_plane(),
    lambda: pins.test_uniform_increase_moves_vertices_inward(),
]


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(mc, attr, fn)
    caught = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, f"no pin caught: {name}"


def test_pins_pass_unmutated():
    for pin in PINS:
        pin()
