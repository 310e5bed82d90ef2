"""The seeded input generators (CPU): exact sizes, valid text, determinism, and the
run structure of the run-structured profiles."""
import numpy as np
import pytest

from paper_2212_05098_amd import synth


@pytest.mark.parametrize("prof", synth.SCRIPT_PROFILES)
def test_run_structured_buffers(prof):
    for n in (1, 7, 255, 4096, 100_003):
        b = synth.run_utf8_buffer(prof, n, synth.rng_for(3, n))
        assert b.size == n and b.dtype == np.uint8
        text = bytes(b).decode("utf-8")  # valid
        w = synth.run_utf16_buffer(prof, n, synth.rng_for(4, n))
        assert w.size == n and w.dtype == np.uint16
        w.astype("<u2").tobytes().decode("utf-16-le")  # valid, no split pair
        assert np.array_equal(b, synth.run_utf8_buffer(prof, n, synth.rng_for(3, n)))  # seeded
    words = text.split(" ")
    assert len(words) > 1000
    lens = np.array([len(x) for x in words[1:-1]])
    assert lens.min() >= 1 and lens.max() <= 9 and 4.0 < lens.mean() < 6.0


def test_run_structured_ascii_is_pure():
    b = synth.run_utf8_buffer("ascii", 1 << 20, synth.rng_for(5))
    assert (b < 0x80).all()


def test_config_buffers_exact_and_valid():
    for prof in synth.SCRIPT_PROFILES:
        b = synth.config_buffer(prof, synth.DIR_8TO16, 1 << 16, config=9)
        assert b.size == 1 << 16
        bytes(b).decode("utf-8")
        w = synth.config_buffer(prof, synth.DIR_16TO8, 1 << 16, config=9)
        assert w.size == 1 << 15
        w.astype("<u2").tobytes().decode("utf-16-le")


def test_stream_cuts_cover_the_buffer():
    rng = synth.rng_for(5, 1)
    for n, mx, mn in ((0, 3, 0), (1, 1, 0), (1000, 7, 0), (1000, 50, 1), (10 ** 6, 200_000, 1 << 10)):
        cuts = synth.stream_cuts(n, rng, mx, min_chunk=mn)
        assert cuts[0] == 0 and cuts[-1] == n
        steps = np.diff(cuts)
        assert np.all(steps >= 0) and np.all(steps <= mx)
        assert np.all(steps[:-1] >= mn)


def test_utf32_buffers_and_injection():
    rng = synth.rng_for(5, 2)
    for prof in synth.SCRIPT_PROFILES + ("mixed4",):
        u = synth.utf32_buffer(prof, 5000, rng)
        assert u.dtype == np.uint32 and u.size == 5000
        u.astype("<u4").tobytes().decode("utf-32-le")  # every unit a scalar value
        bad, pos = synth.inject_utf32(u, 1e-2, rng)
        assert pos == sorted(pos) and len(pos) >= 1
        assert np.array_equal(np.delete(bad, pos), np.delete(u, pos))
        assert all((0xD800 <= bad[p] <= 0xDFFF) or bad[p] > 0x10FFFF for p in pos)
