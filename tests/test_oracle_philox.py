"""Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) in the oracle: published known-answer
vectors of the Random123 distribution, and uniformity of the derived 24-bit uniforms."""
import numpy as np

from oracle import core

KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 0xFFFFFFFF),
     (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_known_answers():
    for ctr, key, want in KAT:
        assert tuple(int(v) for v in core.philox4x32_10(ctr, key)) == want


def test_uniforms_are_uniform():
    key = (1902, 0)
    u = []
    for i in range(4000):
        w = core.philox4x32_10((i, 3, 17, 0), key)
        u.extend(((w[:3] >> 8).astype(np.float64) * 2.0 ** -24).tolist())
    u = np.array(u)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / len(u))
    assert abs(u.var() - 1 / 12) < 0.004
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    chi2 = ((hist - len(u) / 20) ** 2 / (len(u) / 20)).sum()
    assert chi2 < 45.3   # 19 dof, p ~ 0.999


def test_cell_ids_select_the_noise_stream():
    # a cell run alone with its batch index as noise id follows exactly the trajectory it has
    # inside the batch; with another id it draws other noise
    from synth import configs
    cells = [configs.kg_cell([20] * 10, 40 + k) for k in range(3)]
    p = configs.kg_params(precision="fp64")
    full = core.OracleBatch(p, cells)
    alone = core.OracleBatch(p, [cells[2]], cell_ids=[2])
    other = core.OracleBatch(p, [cells[2]])
    for b in (full, alone, other):
        b.run(5)
    xf = full.get_state(2)["x"]
    assert np.array_equal(alone.get_state(0)["x"], xf)
    assert not np.array_equal(other.get_state(0)["x"], xf)
