"""Pins for the oracle's marching-tetrahedra extraction, on fields whose zero
set is known in closed form: planes (linear fields, which linear interpolation
reproduces exactly), a sphere (closed, consistently oriented, genus 0, its
volume), and the rules for missing weights and truncation jumps."""
import math

import numpy as np
import pytest

from oracle import oracle as O

# the volume keeps its voxel edge in float32: centres are (i + 1/2) * fl32(0.01)
V = float(np.float32(0.01))
TAU = 0.04


def centres(bx, by, bz, v=V):
    """(512, 3) voxel-centre coordinates of block (bx, by, bz), x fastest."""
    loc = np.arange(512)
    g = np.stack([bx * 8 + (loc & 7), by * 8 + ((loc >> 3) & 7), bz * 8 + (loc >> 6)], axis=1)
    return (g + 0.5) * v


def field_volume(fn, blocks, v=V, tau=TAU, weight_fn=None):
    vol = O.OracleVolume(np.float32(v), np.float32(tau), 1 << 20)
    for b in blocks:
        p = centres(*b, v=v)
        w = np.ones(512, dtype=np.uint32) if weight_fn is None else weight_fn(p)
        vol.set_block(O.pack_key(*b), fn(p), w)
    return vol


def grid(lo, hi):
    return [(x, y, z) for x in range(lo, hi) for y in range(lo, hi) for z in range(lo, hi)]


def tri_areas(verts):
    a = verts[:, 1] - verts[:, 0]
    b = verts[:, 2] - verts[:, 0]
    return 0.5 * np.linalg.norm(np.cross(a, b), axis=1)


def test_horizontal_plane_closed_form():
    # blocks (0..1)^3 span voxels 0..15: centres 0.005 .. 0.155; the plane z0 = 0.0731 lies
    # between centre layers 6 and 7 (0.065, 0.075)
    z0 = 0.0731
    m = field_volume(lambda p: z0 - p[:, 2], grid(0, 2)).mesh()
    cubes = 15 * 15  # every cube of that layer has all 8 corners in the blocks
    assert m.ids.shape[0] == 8 * cubes
    assert np.max(np.abs(m.verts[:, :, 2] - z0)) < 1e-12
    assert math.isclose(tri_areas(m.verts).sum(), cubes * V * V, rel_tol=1e-9)
    # the normals point to the outside (f > 0, below the plane): -z
    n = np.cross(m.verts[:, 1] - m.verts[:, 0], m.verts[:, 2] - m.verts[:, 0])
    assert np.all(n[:, 2] < 0)


def test_tilted_plane_vertices_lie_on_the_plane():
    nrm = np.array([0.3, -0.5, 0.81])
    nrm /= np.linalg.norm(nrm)
    c = 0.0317
    m = field_volume(lambda p: c - p @ nrm, grid(-1, 2)).mesh()
    assert m.ids.shape[0] > 1000
    assert np.max(np.abs(m.verts.reshape(-1, 3) @ nrm - c)) < 1e-12
    # vertices sit on grid edges between their two corners
    a = (m.edges[:, :, 0].astype(np.float64) + 0.5) * V
    b = (m.edges[:, :, 1].astype(np.float64) + 0.5) * V
    t = np.einsum("tvd,tvd->tv", m.verts - a, b - a) / np.einsum("tvd,tvd->tv", b - a, b - a)
    assert np.all((t >= -1e-12) & (t <= 1 + 1e-12))
    assert np.allclose(a + t[..., None] * (b - a), m.verts, atol=1e-12)
    assert np.all(np.abs(m.edges[:, :, 1] - m.edges[:, :, 0]).sum(axis=2) >= 1)


def sphere_mesh(r=0.1, centre=(0.003, -0.002, 0.001)):
    c = np.array(centre)
    return field_volume(lambda p: np.linalg.norm(p - c, axis=1) - r, grid(-2, 2)).mesh(), r, c


def test_sphere_is_closed_oriented_genus_zero():
    m, r, c = sphere_mesh()
    T = m.ids.shape[0]
    # vertices are identified by their grid edge
    vid = {}
    tri_v = np.zeros((T, 3), dtype=np.int64)
    for i in range(T):
        for j in range(3):
            e = tuple(m.edges[i, j].reshape(-1))
            tri_v[i, j] = vid.setdefault(e, len(vid))
    directed = {}
    for a, b, cc in tri_v:
        for u, w in ((a, b), (b, cc), (cc, a)):
            assert u != w, "degenerate triangle"
            directed[(u, w)] = directed.get((u, w), 0) + 1
    assert max(directed.values()) == 1, "an edge is used twice in one direction"
    for (u, w) in directed:
        assert (w, u) in directed, "an edge borders one triangle only"
    E = len(directed) // 2
    assert len(vid) - E + T == 2  # Euler characteristic of a sphere
    # outward winding encloses a positive volume close to the sphere's
    vol = np.einsum("ij,ij->i", m.verts[:, 0], np.cross(m.verts[:, 1], m.verts[:, 2])).sum() / 6
    assert 0.97 * (4 / 3) * math.pi * r ** 3 < vol < (4 / 3) * math.pi * r ** 3
    # linear interpolation of the distance field along an edge of length <= sqrt(3) v
    # errs by at most (3 v^2) / (8 r) towards the inside
    d = np.linalg.norm(m.verts.reshape(-1, 3) - c, axis=1) - r
    assert np.all(d <= 1e-12) and np.all(d >= -3 * V * V / (8 * r))


def test_missing_weight_removes_the_cubes_that_use_it():
    z0 = 0.0731
    full = field_volume(lambda p: z0 - p[:, 2], grid(0, 2)).mesh()
    hole = (np.array([3, 4, 6]) + 0.5) * V  # a centre of the layer just below the plane

    def weights(p):
        return np.where(np.all(np.abs(p - hole) < 1e-9, axis=1), 0, 1).astype(np.uint32)

    m = field_volume(lambda p: z0 - p[:, 2], grid(0, 2), weight_fn=weights).mesh()
    assert m.ids.shape[0] == full.ids.shape[0] - 4 * 8


@pytest.mark.parametrize("step,expect", [(TAU, 0), ((1 - 2 ** -11) * TAU, 0), (0.99 * TAU, 8 * 15 * 15),
                                         (0.5 * TAU, 8 * 15 * 15)])
def test_jumps_at_the_truncation_limit_are_not_surfaces(step, expect):
    z0 = 0.0731
    m = field_volume(lambda p: np.where(p[:, 2] < z0, step, -step), grid(0, 2)).mesh()
    assert m.ids.shape[0] == expect


def test_triangle_ids_are_unique_and_in_order():
    m, _, _ = sphere_mesh()
    order = np.lexsort((m.ids[:, 1], m.ids[:, 0]))
    assert np.array_equal(order, np.arange(m.ids.shape[0]))
    pairs = {(int(a), int(b)) for a, b in m.ids}
    assert len(pairs) == m.ids.shape[0]
    code = m.ids[:, 1]
    assert np.all(((code >> 1) & 7) < 6) and np.all((code >> 4) < 512)
