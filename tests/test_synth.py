import numpy as np

import synth


def test_splitmix64_reference_value():
    # first output of SplitMix64 from seed 0 (published reference stream)
    assert int(synth.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF


def test_icosphere_counts_and_orientation():
    for s in range(4):
        V, T = synth.icosphere(s)
        assert V.shape[0] == 10 * 4 ** s + 2 and T.shape[0] == 20 * 4 ** s
        a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
        assert np.all(np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0)
        assert np.allclose(np.linalg.norm(V, axis=1), synth.DIAMETER / 2)


def test_jitter_bounds():
    V0, T = synth.icosphere(3)
    V1, T1 = synth.icosphere(3, jitter=0.05, seed=2)
    assert np.array_equal(T, T1)
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    L = np.linalg.norm(V0[e[:, 0]] - V0[e[:, 1]], axis=1)
    assert np.max(np.abs(V1 - V0)) <= 0.05 * L.max()
    assert np.max(np.abs(V1 - V0)) > 0.0
