"""The stream reading checked on the CPU against the oracle alone: cutting a buffer into
chunks, carrying the unfinished character at each chunk's end (a lead byte within the
last 3 bytes that wants more bytes than remain, or a final high surrogate), judging the
character across each cut from its own units, and running the rest of each chunk to its
end with a truncation error at the carried tail taken as the cut, gives exactly the
oracle's result on the whole buffer: the same output, error kind and offset.  The
pieces are transcoded by the oracle; error-dense alphabets make most cuts land on or
next to an error.  This is the rule the GPU stream path follows; the GPU tests check
the library against the oracle directly."""
import numpy as np

import oracle as O
from paper_2212_05098_amd import synth


def lead_len(b):
    return 4 if b >= 0xF0 else 3 if b >= 0xE0 else 2


def run_stream(data, cuts, in16):
    fn = O.utf16le_to_utf8 if in16 else O.utf8_to_utf16le
    dt = np.uint16 if in16 else np.uint8
    carry, need, in_units, out = [], 0, 0, []
    for i in range(len(cuts) - 1):
        chunk = [int(v) for v in data[cuts[i]:cuts[i + 1]]]
        final = i == len(cuts) - 2
        n, nc = len(chunk), len(carry)
        h = min(need, n) if nc else 0
        if nc and not final and h < need:          # the chunk does not finish the carried character
            carry, need, in_units = carry + chunk, need - n, in_units + n
            continue
        t = n                                      # start of the unfinished character at the end
        if not final:
            if in16:
                if n > h and (chunk[n - 1] & 0xFC00) == 0xD800:
                    t = n - 1
            else:
                for k in range(1, min(3, n - h) + 1):
                    b = chunk[n - k]
                    if b < 0x80:
                        break
                    if b >= 0xC0:
                        if lead_len(b) > k:
                            t = n - k
                        break
        if nc:                                     # piece 1: the character across the cut
            r1, o1 = fn(np.array(carry + chunk[:h], dt))
            if r1.status:
                return r1.status, in_units - nc + r1.count, out + list(o1[:r1.written])
            out += list(o1[:r1.written])
        if n > h:                                  # piece 2: the rest, to the chunk's end
            r2, o2 = fn(np.array(chunk[h:], dt))
            if r2.status and not (t < n and r2.count == t - h):
                return r2.status, in_units + h + r2.count, out + list(o2[:r2.written])
            out += list(o2[:r2.written])
        carry = chunk[t:]
        need = (1 if in16 else lead_len(carry[0]) - len(carry)) if carry else 0
        in_units += n
    return O.OK, None, out


def test_stream_rule_matches_whole_buffer():
    rng = synth.rng_for(77)
    a8 = np.array([0x41, 0x80, 0xBF, 0xC2, 0xC0, 0xE0, 0xE4, 0xED, 0xA0, 0xF0, 0xF4, 0x90, 0x8F, 0xF5, 0x9F, 0xB8],
                  np.uint8)
    a16 = np.array([0x41, 0xE9, 0x4E2D, 0xD83D, 0xDE00, 0xDBFF, 0xDC00, 0xFFFF], np.uint16)
    for trial in range(4000):
        in16 = trial % 2 == 1
        n = int(rng.integers(0, 40))
        if trial % 4 < 2:
            data = rng.choice(a16 if in16 else a8, size=n)
        else:
            data = synth.utf16_buffer("emoji", n, rng) if in16 else synth.utf8_buffer("mixed4", n, rng)
        cuts = synth.stream_cuts(n, rng, int(rng.integers(1, 8))) if n else [0, 0]
        st, off, out = run_stream(data, cuts, in16)
        want, ref = (O.utf16le_to_utf8 if in16 else O.utf8_to_utf16le)(data)
        assert st == want.status, (trial, data, cuts)
        if st:
            assert off == want.count, (trial, data, cuts)
        assert len(out) == want.written and list(out) == list(ref[:want.written]), (trial, data, cuts)
