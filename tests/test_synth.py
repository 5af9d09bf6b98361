"""The seeded input generators: sampling a signed distance over worker
processes gives exactly what one process gives, and a saved workload reads
back unchanged."""

import numpy as np

import synth
from synth import sdf


def test_pooled_sdf_sampling_is_bitwise_the_single_process_one():
    prims = synth.random_shape(["box", "capsule", "torus", "ellipsoid"], np.random.default_rng(3))
    ax = synth.axis_coords(48)
    one = sdf.sample_sdf(prims, ax, workers=1)
    four = sdf.sample_sdf(prims, ax, workers=4)
    assert one.dtype == np.float32 and np.array_equal(one.view(np.uint32), four.view(np.uint32))


def test_workload_save_and_load_round_trip(tmp_path):
    p = synth.make_custom(3, [12, 20], 10, (1.5, 2.5), bands=[None, 0.2], samples=(1, 300, 16, 310))
    path = str(tmp_path / "w.npz")
    synth.save_problem(p, path)
    q = synth.load_problem(path)
    assert np.array_equal(p.params, q.params) and (p.m, p.cap, p.cull_k, p.lr) == (q.m, q.cap, q.cull_k, q.lr)
    for a, b in zip(p.levels, q.levels):
        assert a.n == b.n and a.band == b.band and a.octree == b.octree and a.sample_cap == b.sample_cap
        assert (a.axis is None) == (b.axis is None)
        if a.axis is not None:
            assert np.array_equal(a.axis, b.axis) and np.array_equal(a.S, b.S)
        assert (a.samples is None) == (b.samples is None)
        if a.samples is not None:
            assert np.array_equal(a.samples, b.samples)
