"""Host logic of the surrogate driver, on the CPU: the stretch history that forms the 153 features
(17 load steps of R, newest first, padded with the identity) and the out-of-distribution score."""
import numpy as np

from paper_1902_09171_amd.surrogate import FEATURES, HISTORY, History, spread


def test_history_pads_with_identity_and_keeps_the_newest_first():
    assert HISTORY == 17 and FEATURES == 153
    h = History(2)
    eye = np.tile(np.eye(3).reshape(1, 1, 9), (2, HISTORY, 1))
    assert np.array_equal(h.features().reshape(2, HISTORY, 9), eye)
    rng = np.random.default_rng(1)
    Rs = [np.triu(rng.normal(size=(2, 3, 3))) for _ in range(HISTORY + 2)]
    for k, R in enumerate(Rs):
        h.push(R)
        f = h.features()
        assert f.shape == (2, FEATURES) and f.flags["C_CONTIGUOUS"]
        f = f.reshape(2, HISTORY, 9)
        for j in range(HISTORY):                 # slot j holds the stretch of j load steps ago
            want = Rs[k - j].reshape(2, 9) if j <= k else eye[:, 0]
            assert np.array_equal(f[:, j], want), (k, j)


def test_spread_is_the_largest_normalised_standard_deviation():
    var = np.array([[4.0, 1.0, 0.0], [0.25, 9.0, -1e-12]])   # a rounding-negative variance counts as 0
    y_sd = np.array([2.0, 1.0, 1.0])
    assert np.array_equal(spread(var, y_sd), np.array([1.0, 3.0]))
