"""Checks of the seeded input generator (not part of the method): Philox-4x32-10
against its published known-answer vectors, and the moments of its normals."""

import numpy as np

from conftest import read_golden
from paper_1412_0781_amd import synth


def test_philox_known_answer_vectors():
    for row in read_golden("philox4x32_10_kat.txt"):
        v = [int(t, 16) for t in row.split()]
        ctr = np.array(v[0:4], dtype=np.uint32)
        key = np.array(v[4:6], dtype=np.uint32)
        out = synth.philox4x32_10(ctr, key)
        assert [int(x) for x in out] == v[6:10]


def test_normals_moments_and_independence_of_index():
    z = synth.normals(0, synth.STREAM_NOISE, np.arange(64), 4096)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1) < 0.01
    # any image can be regenerated on its own
    z5 = synth.normals(0, synth.STREAM_NOISE, np.array([5]), 4096)
    assert np.array_equal(z5[0], z[5])
    # streams and seeds differ
    assert not np.allclose(z[0], synth.normals(0, synth.STREAM_COEF, np.array([0]), 4096)[0])
    assert not np.allclose(z[0], synth.normals(1, synth.STREAM_NOISE, np.array([0]), 4096)[0])


def test_coefficient_variance_profile():
    k = np.array([0, 0, 1, 3])
    q = np.array([1, 2, 1, 2])
    v = synth.coef_variance(k, q)
    assert np.allclose(v, [1 / 4, 1 / 9, 1 / 8, 1 / 36])
    a = synth.random_coefficients(0, np.arange(20000), k, q)
    assert np.all(a[:, :2].imag == 0)
    assert np.allclose(np.mean(np.abs(a) ** 2, axis=0), v, rtol=0.05)
