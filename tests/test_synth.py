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


def test_batch_injection_lands_in_every_flagged_string():
    """Every string the batch generator flags carries its error at the recorded offset,
    short strings included (log-normal lengths, median 256 B: a quarter are under
    90 B), and the number of erroring strings is binomial(n, err_frac)."""
    import oracle as O

    n, frac = 20000, 0.05
    b = synth.make_batch(n, seed_key=(0, 4, 99), median=256, sigma=2.0, hi=64 << 10, err_frac=frac)
    flagged = np.nonzero(b.err_pos >= 0)[0]
    mean, sd = n * frac, (n * frac * (1 - frac)) ** 0.5
    assert abs(flagged.size - mean) < 4 * sd, flagged.size
    for i in flagged:
        a, L = int(b.in_off[i]), int(b.in_len[i])
        if b.direction[i] == 0:
            r = O.validate_utf8(b.arena[a:a + L])
        else:
            r = O.validate_utf16le(b.arena[a:a + 2 * L].view(np.uint16))
        assert r.status != O.OK and r.count == b.err_pos[i], (i, L, r, b.err_pos[i])
    # unflagged strings are valid
    for i in np.nonzero(b.err_pos < 0)[0][:2000]:
        a, L = int(b.in_off[i]), int(b.in_len[i])
        if b.direction[i] == 0:
            assert O.validate_utf8(b.arena[a:a + L]).status == O.OK
        else:
            assert O.validate_utf16le(b.arena[a:a + 2 * L].view(np.uint16)).status == O.OK


@pytest.mark.parametrize("direction", [synth.DIR_8TO16, synth.DIR_16TO8])
def test_single_injection_in_short_buffers(direction):
    """One injected error per buffer of 8..300 units always lands inside it."""
    import oracle as O

    rng = synth.rng_for(6, direction)
    for L in list(range(8, 64)) + [100, 255, 256, 300]:
        for prof in synth.SCRIPT_PROFILES:
            if direction == synth.DIR_8TO16:
                inj = synth.inject_utf8(prof, L, 1.0 / L, rng)
                assert inj.data.size == L
                r = O.validate_utf8(inj.data)
            else:
                inj = synth.inject_utf16(prof, L, 1.0 / L, rng)
                assert inj.data.size == L
                r = O.validate_utf16le(inj.data)
            assert inj.positions.size == 1 and r.status != O.OK and r.count == inj.positions[0], (L, prof, r)
