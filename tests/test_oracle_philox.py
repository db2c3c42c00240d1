"""Pins the oracle's Philox4x32-10 to known-answer vectors of the generator's published
definition (Salmon et al., SC'11, Random123 known-answer tests) and checks the uniforms
built from it."""
import numpy as np
from scipy.stats import kstest


def test_known_answers(orc):
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = orc.philox4x32_10(np.array(ctr, dtype=np.uint32), np.array(key, dtype=np.uint32))
        assert [int(v) for v in got] == list(want), [hex(int(v)) for v in got]


def test_uniforms_are_uniform_and_seeded(orc):
    u = orc.draw_uniforms(1234, 200000)
    assert u.min() >= 0.0 and u.max() < 1.0
    for j in range(3):
        assert kstest(u[:, j], "uniform").pvalue > 1e-4
    assert abs(np.corrcoef(u[:, 0], u[:, 1])[0, 1]) < 0.01
    assert not np.array_equal(u[:100], orc.draw_uniforms(1235, 100))
    assert np.array_equal(u[:100], orc.draw_uniforms(1234, 100))
