"""Pins for the oracle's surface evaluation (marching tetrahedra, area
sampling, HD / CD / CS of Section 4): closed forms on planes and spheres,
brute force on small sets, and the inverse of eq. 3-10."""

import math

import numpy as np
import pytest

import oracle as O
from oracle import metrics as Mx


def _axis(n):
    return (-1.0 + (2.0 * np.arange(n) + 1.0) / n).astype(np.float32)


def _field(n, fn):
    a = _axis(n).astype(np.float64)
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    return _axis(n), fn(x, y, z).astype(np.float32).reshape(-1)


def test_plane_is_extracted_exactly():
    # a linear field: linear interpolation puts every vertex on the plane, and
    # the surface is the plane over the square of the outer cell centres
    n = 10
    ax, F = _field(n, lambda x, y, z: x - 0.13)
    T = Mx.marching_tets(F, ax)
    assert np.allclose(T[:, :, 0], 0.13, atol=1e-6)
    side = float(ax[-1]) - float(ax[0])
    assert Mx.triangle_areas(T).sum() == pytest.approx(side * side, rel=1e-6)


def test_sphere_vertices_and_area():
    n, R = 40, 0.6
    ax, F = _field(n, lambda x, y, z: np.sqrt(x * x + y * y + z * z) - R)
    T = Mx.marching_tets(F, ax)
    h = 2.0 / n
    r = np.linalg.norm(T.reshape(-1, 3), axis=1)
    # linear interpolation of the exact distance along an edge of length <=
    # sqrt(3) h stays within h^2 of the sphere
    assert np.abs(r - R).max() <= h * h
    assert Mx.triangle_areas(T).sum() == pytest.approx(4 * math.pi * R * R, rel=0.02)


def test_cube_cases_give_closed_surfaces():
    # a single inside corner of a 2x2x2 grid: the surface cuts the cube's
    # corner; every triangle vertex lies on an edge from that corner
    ax = np.array([-0.5, 0.5], np.float32)
    F = np.ones(8, np.float32)
    F[0] = -1.0
    T = Mx.marching_tets(F, ax)
    assert T.shape[0] > 0
    v = T.reshape(-1, 3)
    # vertices are the midpoints of edges leaving corner 0 (values -1 and 1)
    on_edge = (np.isclose(v, 0.0) | np.isclose(v, -0.5)).all(axis=1)
    assert on_edge.all()


def test_sampling_is_on_triangles_and_uniform_by_area():
    rng = np.random.default_rng(3)
    T = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[0, 0, 1], [3, 0, 1], [0, 1, 1]]], np.float64)
    u = rng.random((60000, 3))
    P, N, tri = Mx.sample_surface(T, u)
    # area 0.5 and 1.5: a quarter of the samples on the first triangle
    assert abs((tri == 0).mean() - 0.25) < 0.01
    assert np.allclose(P[tri == 0, 2], 0.0) and np.allclose(P[tri == 1, 2], 1.0)
    assert np.all(P[:, 0] >= -1e-12) and np.all(P[:, 1] >= -1e-12)
    assert np.all(P[tri == 0, 0] + P[tri == 0, 1] <= 1 + 1e-12)
    assert np.allclose(np.abs(N[:, 2]), 1.0)


def test_sampling_is_uniform_within_a_triangle():
    # a uniform density on a triangle has the centroid as its mean, and each
    # of the four half-scale sub-triangles (three corners, the middle one)
    # holds a quarter of the samples
    rng = np.random.default_rng(11)
    A, B, C = np.array([0.2, -0.1, 0.3]), np.array([1.4, 0.2, 0.1]), np.array([0.5, 1.3, -0.4])
    T = np.array([[A, B, C]], np.float64)
    n = 200000
    P, _, _ = Mx.sample_surface(T, rng.random((n, 3)))
    side = max(np.linalg.norm(B - A), np.linalg.norm(C - A), np.linalg.norm(C - B))
    assert np.linalg.norm(P.mean(0) - (A + B + C) / 3.0) < 5e-3 * side
    # barycentric coordinates of the samples
    M = np.stack([B - A, C - A], 1)
    lb, lc = np.linalg.lstsq(M, (P - A).T, rcond=None)[0]
    la = 1.0 - lb - lc
    for frac in ((la > 0.5).mean(), (lb > 0.5).mean(), (lc > 0.5).mean()):
        assert abs(frac - 0.25) < 0.005


def test_metrics_brute_force_and_concentric_spheres():
    rng = np.random.default_rng(5)
    A = rng.normal(size=(300, 3))
    B = rng.normal(size=(200, 3))
    NA = A / np.linalg.norm(A, axis=1, keepdims=True)
    NB = B / np.linalg.norm(B, axis=1, keepdims=True)
    hd, cd, cs = Mx.surface_metrics(A, NA, B, NB)
    D = np.linalg.norm(A[:, None, :] - B[None, :, :], axis=2)
    ab, ba = D.min(1), D.min(0)
    assert hd == pytest.approx(max(ab.max(), ba.max()), rel=1e-12)
    assert cd == pytest.approx(0.5 * ab.mean() + 0.5 * ba.mean(), rel=1e-12)
    csb = 0.5 * np.abs(np.sum(NA * NB[D.argmin(1)], 1)).mean() + 0.5 * np.abs(np.sum(NB * NA[D.argmin(0)], 1)).mean()
    assert cs == pytest.approx(csb, rel=1e-12)
    # identical sets
    assert Mx.surface_metrics(A, NA, A, NA) == (0.0, 0.0, 1.0)
    # dense samples of two concentric spheres: every closest distance is
    # about the radius gap, normals agree
    v = rng.normal(size=(4000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    hd, cd, cs = Mx.surface_metrics(0.5 * v, v, 0.52 * v, v)
    assert cd == pytest.approx(0.02, rel=0.02) and hd < 0.05 and cs > 0.999


def test_sdf_from_targets_inverts_eq_3_10():
    m = -0.4
    S = np.linspace(m, 0.9, 50)
    t = O.targets_from_sdf(S, m)
    assert np.allclose(Mx.sdf_from_targets(t, m), S, atol=1e-9)
    assert Mx.sdf_from_targets(np.array([2.5]), m)[0] == m
    assert Mx.sdf_from_targets(np.array([1.0]), m)[0] == pytest.approx(0.0, abs=1e-15)


def test_infinite_corner_puts_the_vertex_on_the_finite_corner():
    # eq. 3-10 inverted gives +inf where the network output is <= 0; such a
    # corner is infinitely far outside, so the surface passes through the
    # finite (inside) corner
    ax = np.array([-0.5, 0.5], np.float32)
    F = np.full(8, np.inf, np.float32)
    F[0] = -1.0
    T = Mx.marching_tets(F, ax)
    assert T.shape[0] > 0 and np.all(np.isfinite(T))
    assert np.allclose(T.reshape(-1, 3), [-0.5, -0.5, -0.5])
