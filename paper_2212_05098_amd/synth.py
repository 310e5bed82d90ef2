"""Seeded synthetic inputs: the script profiles, error injection, batches, traces.

This module only draws random code points and strings.  It holds none of the
transcoding arithmetic: code points are serialized to UTF-8 / UTF-16LE with
Python's own codecs, and truncation to an exact byte length goes through the codecs
as well (decode with ``errors="ignore"`` drops a trailing partial character).  Both
the GPU tests and the oracle tests draw their inputs here; the expected values
always come from the oracle.

The profiles stand in for the paper's "lipsum" corpus (section 8.1), which is not
available: code points are i.i.d. per profile with the mixes below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# (weight, lo, hi) code-point ranges, inclusive.  Weights within a profile sum to 1.
# "bmp3" is U+0800..FFFF without the surrogate block, handled in _draw_range.
PROFILES: Dict[str, List[Tuple[float, int, int]]] = {
    # 64 KiB mixed buffer: 40 % ASCII, 25 % 2-byte, 25 % 3-byte, 10 % 4-byte
    "mixed4": [(0.40, 0x20, 0x7E), (0.25, 0x80, 0x7FF), (0.25, 0x800, 0xFFFF), (0.10, 0x10000, 0x10FFFF)],
    "ascii": [(0.95, 0x20, 0x7E), (0.05, 0xA0, 0xFF)],
    # Latin / Cyrillic / Arabic: 40 % ASCII, 60 % uniform over three 2-byte blocks
    "latin": [(0.40, 0x20, 0x7E), (0.20, 0xC0, 0xFF), (0.20, 0x400, 0x4FF), (0.20, 0x600, 0x6FF)],
    "cjk": [(0.90, 0x4E00, 0x9FFF), (0.10, 0x20, 0x7E)],
    "emoji": [(0.30, 0x1F300, 0x1FAFF), (0.70, 0x20, 0x7E)],
}
SCRIPT_PROFILES = ("ascii", "latin", "cjk", "emoji")
PROFILE_IDS = {"mixed4": 0, "ascii": 1, "latin": 2, "cjk": 3, "emoji": 4}
DIR_8TO16 = 0
DIR_16TO8 = 1

# Approximate UTF-8 / UTF-16 bytes per character, used only to size the draws.
_APPROX_BPC = {"mixed4": (2.05, 2.2), "ascii": (1.05, 2.0), "latin": (1.6, 2.0),
               "cjk": (2.8, 2.0), "emoji": (1.9, 2.6)}


def rng_for(*key: int) -> np.random.Generator:
    """PCG64 generator seeded from a SeedSequence over the given integers."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _draw_range(rng: np.random.Generator, lo: int, hi: int, k: int) -> np.ndarray:
    if lo == 0x800 and hi == 0xFFFF:
        # U+0800..FFFF without U+D800..DFFF: 61,440 values
        v = rng.integers(0, 0xFFFF - 0x800 + 1 - 0x800, size=k, dtype=np.int64) + 0x800
        v = v + np.where(v >= 0xD800, 0x800, 0)
        return v
    return rng.integers(lo, hi + 1, size=k, dtype=np.int64)


def draw_codepoints(profile: str, k: int, rng: np.random.Generator) -> np.ndarray:
    """k i.i.d. code points of the profile, as uint32."""
    ranges = PROFILES[profile]
    w = np.array([r[0] for r in ranges], dtype=np.float64)
    which = rng.choice(len(ranges), size=k, p=w / w.sum())
    out = np.empty(k, dtype=np.int64)
    for j, (_, lo, hi) in enumerate(ranges):
        idx = np.nonzero(which == j)[0]
        out[idx] = _draw_range(rng, lo, hi, idx.size)
    return out.astype(np.uint32)


def cps_to_str(cps: np.ndarray) -> str:
    return np.ascontiguousarray(cps, dtype="<u4").tobytes().decode("utf-32-le")


def _ascii_pad(rng: np.random.Generator, k: int) -> bytes:
    return rng.integers(0x20, 0x7F, size=k, dtype=np.uint8).tobytes()


def utf8_buffer(profile: str, n_bytes: int, rng: np.random.Generator) -> np.ndarray:
    """Exactly n_bytes of valid UTF-8: i.i.d. characters of the profile, cut at the
    last whole character, then padded with printable ASCII."""
    if n_bytes == 0:
        return np.zeros(0, dtype=np.uint8)
    bpc = _APPROX_BPC[profile][0]
    k = int(n_bytes / bpc * 1.02) + 16
    b = cps_to_str(draw_codepoints(profile, k, rng)).encode("utf-8")
    while len(b) < n_bytes:
        b += cps_to_str(draw_codepoints(profile, k // 4 + 16, rng)).encode("utf-8")
    cut = b[:n_bytes].decode("utf-8", errors="ignore").encode("utf-8")
    cut += _ascii_pad(rng, n_bytes - len(cut))
    return np.frombuffer(cut, dtype=np.uint8).copy()


def utf16_buffer(profile: str, n_words: int, rng: np.random.Generator) -> np.ndarray:
    """Exactly n_words of valid UTF-16LE (never splitting a surrogate pair)."""
    if n_words == 0:
        return np.zeros(0, dtype=np.uint16)
    bpc = _APPROX_BPC[profile][1]
    k = int(2 * n_words / bpc * 1.02) + 16
    b = cps_to_str(draw_codepoints(profile, k, rng)).encode("utf-16-le")
    while len(b) < 2 * n_words:
        b += cps_to_str(draw_codepoints(profile, k // 4 + 16, rng)).encode("utf-16-le")
    cut = b[: 2 * n_words].decode("utf-16-le", errors="ignore").encode("utf-16-le")
    pad = np.frombuffer(_ascii_pad(rng, n_words - len(cut) // 2), dtype=np.uint8).astype("<u2")
    out = np.concatenate([np.frombuffer(cut, dtype="<u2"), pad])
    return out.astype(np.uint16)


# Run-structured text, closer to the paper's lipsum files than the i.i.d. profiles:
# words of 1..9 characters (mean 5) separated by single spaces, sentences of 5..20 words
# each written in one script drawn from the profile's ranges (lower-case Latin letters for
# the ASCII profile).  Waves of such text are often uniform in their byte classes.
RUN_SCRIPTS: Dict[str, List[Tuple[int, int]]] = {
    "ascii": [(0x61, 0x7A)],
    "latin": [(0xC0, 0xFF), (0x400, 0x4FF), (0x600, 0x6FF)],
    "cjk": [(0x4E00, 0x9FFF)],
    "emoji": [(0x1F300, 0x1FAFF)],
}


def run_codepoints(profile: str, k: int, rng: np.random.Generator) -> np.ndarray:
    """At least k code points of run-structured text of the profile, as uint32."""
    scripts = RUN_SCRIPTS[profile]
    n_words = k // 5 + 16
    wl = rng.integers(1, 10, size=n_words)                      # word lengths
    sl = rng.integers(5, 21, size=n_words // 5 + 2)             # sentence lengths in words
    sent = np.repeat(np.arange(sl.size), sl)[:n_words]          # sentence of each word
    script = rng.integers(0, len(scripts), size=sl.size)[sent]  # script of each word
    lo = np.array([a for a, _ in scripts], dtype=np.int64)[script]
    hi = np.array([b for _, b in scripts], dtype=np.int64)[script]
    per_char_lo = np.repeat(lo, wl)
    per_char_hi = np.repeat(hi, wl)
    chars = per_char_lo + (rng.random(per_char_lo.size) * (per_char_hi - per_char_lo + 1)).astype(np.int64)
    # a space after every word
    ends = np.cumsum(wl)
    out = np.insert(chars, ends, 0x20)
    return out.astype(np.uint32)


def run_utf8_buffer(profile: str, n_bytes: int, rng: np.random.Generator) -> np.ndarray:
    """Exactly n_bytes of valid run-structured UTF-8 (cut at a character, ASCII pad)."""
    if n_bytes == 0:
        return np.zeros(0, dtype=np.uint8)
    b = b""
    while len(b) < n_bytes:
        b += cps_to_str(run_codepoints(profile, max(n_bytes // 2, 64), rng)).encode("utf-8")
    cut = b[:n_bytes].decode("utf-8", errors="ignore").encode("utf-8")
    cut += _ascii_pad(rng, n_bytes - len(cut))
    return np.frombuffer(cut, dtype=np.uint8).copy()


def run_utf16_buffer(profile: str, n_words: int, rng: np.random.Generator) -> np.ndarray:
    """Exactly n_words of valid run-structured UTF-16LE."""
    if n_words == 0:
        return np.zeros(0, dtype=np.uint16)
    b = b""
    while len(b) < 2 * n_words:
        b += cps_to_str(run_codepoints(profile, max(n_words // 2, 64), rng)).encode("utf-16-le")
    cut = b[: 2 * n_words].decode("utf-16-le", errors="ignore").encode("utf-16-le")
    pad = np.frombuffer(_ascii_pad(rng, n_words - len(cut) // 2), dtype=np.uint8).astype("<u2")
    return np.concatenate([np.frombuffer(cut, dtype="<u2"), pad]).astype(np.uint16)


def config_buffer(profile: str, direction: int, n_bytes: int, config: int = 2) -> np.ndarray:
    """Input for one (config, profile, direction): uint8 for UTF-8, uint16 for UTF-16."""
    rng = rng_for(0, config, PROFILE_IDS[profile], direction)
    if direction == DIR_8TO16:
        return utf8_buffer(profile, n_bytes, rng)
    return utf16_buffer(profile, n_bytes // 2, rng)


def config1_buffer() -> np.ndarray:
    """The 64 KiB all-valid mixed UTF-8 buffer, seed 0."""
    return utf8_buffer("mixed4", 65536, rng_for(0))


# ---------------------------------------------------------------- error injection

UTF8_KINDS = ("stray", "overlong2", "overlong3", "overlong4", "surrogate", "too_large",
              "bad_byte", "truncated")
UTF16_KINDS = ("unpaired_high", "lone_low")


def utf8_error_item(kind: str, rng: np.random.Generator) -> bytes:
    """Byte sequence of one injected UTF-8 error (it is invalid at its first byte
    when placed at a character boundary and followed by a character start)."""
    def cont(lo=0x80, hi=0xBF):
        return int(rng.integers(lo, hi + 1))

    if kind == "stray":
        return bytes([cont()])
    if kind == "overlong2":
        return bytes([int(rng.integers(0xC0, 0xC2)), cont()])
    if kind == "overlong3":
        return bytes([0xE0, cont(0x80, 0x9F), cont()])
    if kind == "overlong4":
        return bytes([0xF0, cont(0x80, 0x8F), cont(), cont()])
    if kind == "surrogate":
        return bytes([0xED, cont(0xA0, 0xBF), cont()])
    if kind == "too_large":
        return bytes([0xF4, cont(0x90, 0xBF), cont(), cont()])
    if kind == "bad_byte":
        return bytes([int(rng.integers(0xF5, 0xF8)), cont(), cont(), cont()])
    if kind == "truncated":
        L = int(rng.integers(2, 5))
        lead = {2: int(rng.integers(0xC2, 0xE0)), 3: int(rng.integers(0xE1, 0xED)),
                4: int(rng.integers(0xF1, 0xF4))}[L]
        k = int(rng.integers(0, L - 1))  # fewer continuation bytes than needed
        return bytes([lead] + [cont() for _ in range(k)])
    raise ValueError(kind)


def utf16_error_item(kind: str, rng: np.random.Generator) -> List[int]:
    if kind == "unpaired_high":
        return [int(rng.integers(0xD800, 0xDC00))]
    if kind == "lone_low":
        return [int(rng.integers(0xDC00, 0xE000))]
    raise ValueError(kind)


def _utf8_units(cps: np.ndarray) -> np.ndarray:
    """Bytes per character of the drawn code points (their UTF-8 lengths), used only to
    decide which characters lie inside the buffer."""
    c = cps.astype(np.int64)
    return 1 + (c >= 0x80) + (c >= 0x800) + (c >= 0x10000)


def _error_slots(units: np.ndarray, n_units: int, n_err: int, rng: np.random.Generator) -> np.ndarray:
    """Indices of the characters an injection replaces: n_err drawn uniformly without
    replacement among the characters that end inside the buffer with room to spare for
    the items (at most 4 units each), ascending."""
    if n_err == 0:
        return np.zeros(0, np.int64)
    ends = np.cumsum(units)
    room = n_units - 4 * n_err
    m = int(np.searchsorted(ends, room, side="right")) if room > 0 else 0
    if m == 0:
        m = 1  # a buffer too short for the room: the first character, trimmed later
    return np.sort(rng.choice(m, size=min(n_err, m), replace=False))


@dataclass
class Injected:
    data: np.ndarray          # uint8 (UTF-8) or uint16 (UTF-16) input
    positions: np.ndarray     # offsets (input units) of the injected items, ascending
    kinds: List[str]


def inject_utf8(profile: str, n_bytes: int, rate: float, rng: np.random.Generator,
                kinds: Sequence[str] = UTF8_KINDS) -> Injected:
    """n_bytes of the profile with about round(rate * n_bytes) error items placed at
    character boundaries chosen uniformly, each followed by at least one whole
    character; the length stays n_bytes (ASCII padding at the end)."""
    bpc = _APPROX_BPC[profile][0]
    k = int(n_bytes / bpc * 1.05) + 64
    cps = draw_codepoints(profile, k, rng)
    n_err = max(1, int(round(rate * n_bytes))) if rate > 0 else 0
    at = _error_slots(_utf8_units(cps), n_bytes, n_err, rng)
    parts: List[bytes] = []
    pos: List[int] = []
    knd: List[str] = []
    off = 0
    prev = 0
    last_end = 0
    for a in at.tolist():
        if pos and a <= prev:
            continue  # keep a whole character between two items
        seg = cps_to_str(cps[prev:a]).encode("utf-8")
        kd = kinds[int(rng.integers(0, len(kinds)))]
        item = utf8_error_item(kd, rng)
        if off + len(seg) + len(item) > n_bytes:
            break
        parts.append(seg)
        off += len(seg)
        parts.append(item)
        pos.append(off)
        knd.append(kd)
        off += len(item)
        last_end = off
        prev = a + 1
    parts.append(cps_to_str(cps[prev:]).encode("utf-8"))
    b = b"".join(parts)
    if len(b) > n_bytes:
        tail = b[last_end:n_bytes].decode("utf-8", errors="ignore").encode("utf-8")
        b = b[:last_end] + tail
    b += _ascii_pad(rng, n_bytes - len(b))
    return Injected(np.frombuffer(b, dtype=np.uint8).copy(), np.array(pos, dtype=np.int64), knd)


def inject_utf16(profile: str, n_words: int, rate: float, rng: np.random.Generator,
                 kinds: Sequence[str] = UTF16_KINDS) -> Injected:
    """n_words of the profile with unpaired surrogates injected at character
    boundaries, each followed by at least one whole character."""
    bpc = _APPROX_BPC[profile][1]
    k = int(2 * n_words / bpc * 1.05) + 64
    cps = draw_codepoints(profile, k, rng)
    n_err = max(1, int(round(rate * n_words))) if rate > 0 else 0
    at = _error_slots(1 + (cps >= 0x10000).astype(np.int64), n_words, n_err, rng)
    parts: List[np.ndarray] = []
    pos: List[int] = []
    knd: List[str] = []
    off = 0
    prev = 0
    last_end = 0
    for a in at.tolist():
        if pos and a <= prev:
            continue
        seg = np.frombuffer(cps_to_str(cps[prev:a]).encode("utf-16-le"), dtype="<u2")
        kd = kinds[int(rng.integers(0, len(kinds)))]
        item = np.array(utf16_error_item(kd, rng), dtype="<u2")
        if off + seg.size + item.size > n_words:
            break
        parts.append(seg)
        off += seg.size
        parts.append(item)
        pos.append(off)
        knd.append(kd)
        off += item.size
        last_end = off
        prev = a + 1
    parts.append(np.frombuffer(cps_to_str(cps[prev:]).encode("utf-16-le"), dtype="<u2"))
    w = np.concatenate(parts).astype(np.uint16)
    if w.size > n_words:
        tail = w[last_end:n_words].astype("<u2").tobytes().decode("utf-16-le", errors="ignore")
        w = np.concatenate([w[:last_end], np.frombuffer(tail.encode("utf-16-le"), dtype="<u2")]).astype(np.uint16)
    if w.size < n_words:
        pad = rng.integers(0x20, 0x7F, size=n_words - w.size).astype(np.uint16)
        w = np.concatenate([w, pad])
    return Injected(w, np.array(pos, dtype=np.int64), knd)


# ---------------------------------------------------------------- batches and traces

@dataclass
class Batch:
    arena: np.ndarray        # uint8 input arena
    in_off: np.ndarray       # uint64 byte offsets into arena
    in_len: np.ndarray       # uint64 lengths in input units (bytes or words)
    direction: np.ndarray    # uint32, 0 = UTF-8 -> UTF-16LE, 1 = UTF-16LE -> UTF-8
    profile: np.ndarray      # uint8 profile id per string
    err_pos: np.ndarray      # int64 injected error offset (input units) or -1


def lognormal_lengths(rng: np.random.Generator, k: int, median: float, sigma: float,
                      lo: int, hi: int) -> np.ndarray:
    z = rng.standard_normal(k)
    L = np.exp(math.log(median) + sigma * z)
    return np.clip(np.rint(L), lo, hi).astype(np.int64)


def make_batch(n_strings: int, seed_key: Sequence[int] = (0, 4), median: float = 256.0,
               sigma: float = 2.0, lo: int = 8, hi: int = 4 << 20, err_frac: float = 0.005,
               align_utf8: int = 1) -> Batch:
    """Many independent strings of log-normal byte length, mixed profiles and
    directions, a fraction carrying one injected error.  UTF-8 strings start at
    arbitrary byte offsets (align_utf8 = 1); UTF-16 strings at even offsets."""
    rng = rng_for(*seed_key)
    lens = lognormal_lengths(rng, n_strings, median, sigma, lo, hi)
    dirs = rng.integers(0, 2, size=n_strings).astype(np.uint32)
    profs = rng.integers(0, len(SCRIPT_PROFILES), size=n_strings)
    has_err = rng.random(n_strings) < err_frac
    pieces: List[np.ndarray] = []
    in_off = np.zeros(n_strings, dtype=np.uint64)
    in_len = np.zeros(n_strings, dtype=np.uint64)
    err_pos = np.full(n_strings, -1, dtype=np.int64)
    off = 0
    for i in range(n_strings):
        prof = SCRIPT_PROFILES[int(profs[i])]
        L = int(lens[i])
        srng = rng_for(*seed_key, 1, i)
        if dirs[i] == DIR_8TO16:
            pad = int(srng.integers(0, 16)) if align_utf8 == 1 else 0
            if has_err[i]:
                inj = inject_utf8(prof, L, 1.0 / max(L, 1), srng)
                data = inj.data
                err_pos[i] = int(inj.positions[0]) if inj.positions.size else -1
            else:
                data = utf8_buffer(prof, L, srng)
            raw = data.view(np.uint8)
            in_len[i] = raw.size
        else:
            pad = 2 * int(srng.integers(0, 8))
            nw = L // 2
            if has_err[i] and nw > 0:
                inj = inject_utf16(prof, nw, 1.0 / max(nw, 1), srng)
                data = inj.data
                err_pos[i] = int(inj.positions[0]) if inj.positions.size else -1
            else:
                data = utf16_buffer(prof, nw, srng)
            raw = data.astype("<u2").view(np.uint8)
            in_len[i] = data.size
            if off % 2:
                pieces.append(np.zeros(1, dtype=np.uint8))
                off += 1
        if pad:
            pieces.append(np.zeros(pad, dtype=np.uint8))
            off += pad
        in_off[i] = off
        pieces.append(raw)
        off += raw.size
    pieces.append(np.zeros(64, dtype=np.uint8))
    arena = np.concatenate(pieces)
    return Batch(arena, in_off, in_len, dirs, profs.astype(np.uint8), err_pos)


def batch_output_layout(b: Batch, gap: int = 16):
    """Output slots of a batch with room for every string's worst case (n words for
    UTF-8 -> UTF-16LE, 3n bytes for UTF-16LE -> UTF-8), laid out back to back with
    `gap` bytes between slots, UTF-16 slots at even offsets.  Returns (caps in output
    units, out_off in bytes, total output bytes)."""
    caps = np.where(b.direction == 0, b.in_len, 3 * b.in_len).astype(np.uint64)
    sizes = np.where(b.direction == 0, 2 * caps, caps).astype(np.uint64)
    out_off = np.concatenate([[0], np.cumsum(sizes + gap)[:-1]]).astype(np.uint64)
    out_off += out_off % 2
    total = int(out_off[-1] + sizes[-1] + 64) if len(out_off) else 64
    return caps, out_off, total


@dataclass
class Trace:
    arrival_s: np.ndarray     # float64 arrival times, ascending
    size_bytes: np.ndarray    # int64 request input sizes
    direction: np.ndarray     # uint32
    profile: np.ndarray       # uint8


def poisson_trace(rate_per_s: float, duration_s: float, seed_key: Sequence[int] = (0, 5),
                  median: float = 1024.0, sigma: float = 2.5, lo: int = 8,
                  hi: int = 16 << 20) -> Trace:
    rng = rng_for(*seed_key, int(rate_per_s))
    k = rng.poisson(rate_per_s * duration_s)
    t = np.sort(rng.uniform(0.0, duration_s, size=k))
    sizes = lognormal_lengths(rng, k, median, sigma, lo, hi)
    dirs = rng.integers(0, 2, size=k).astype(np.uint32)
    profs = rng.integers(0, len(SCRIPT_PROFILES), size=k).astype(np.uint8)
    return Trace(t, sizes, dirs, profs)


def tile_edge_cases(tile_sizes: Sequence[int], n_bytes: int, rng: np.random.Generator,
                    direction: int) -> List[Tuple[np.ndarray, Optional[int]]]:
    """Inputs with a truncated sequence / unpaired high surrogate ending exactly at
    k*T - 1 for each tile size T, plus negative controls (valid characters straddling
    k*T).  Returns (data, injected_offset or None)."""
    cases: List[Tuple[np.ndarray, Optional[int]]] = []
    for T in tile_sizes:
        if direction == DIR_8TO16:
            base = utf8_buffer("mixed4", n_bytes, rng)
            k = max(1, (n_bytes // T) // 2)
            edge = k * T
            if edge >= n_bytes:
                continue
            b = bytearray(base.tobytes())
            # make b[edge-1] a lead byte of a 3-byte form with no continuations after it
            # by rebuilding the region around the edge from whole characters
            left = bytes(b[: edge - 1]).decode("utf-8", errors="ignore").encode("utf-8")
            left += b"A" * (edge - 1 - len(left))
            item = bytes([0xE2])
            right = b"B" + bytes(b[edge + 1:]).decode("utf-8", errors="ignore").encode("utf-8")
            data = (left + item + right)[:n_bytes]
            data += b"C" * (n_bytes - len(data))
            cases.append((np.frombuffer(data, dtype=np.uint8).copy(), edge - 1))
            # negative control: a 4-byte character straddling the edge
            ctrl = (left[:-2] if len(left) >= 2 else left) + b"\xf0\x9d\x92\xaa"
            ctrl += bytes(b[len(ctrl):]).decode("utf-8", errors="ignore").encode("utf-8")
            ctrl = ctrl[:n_bytes].decode("utf-8", errors="ignore").encode("utf-8")
            ctrl += b"D" * (n_bytes - len(ctrl))
            cases.append((np.frombuffer(ctrl, dtype=np.uint8).copy(), None))
        else:
            nw = n_bytes // 2
            base = utf16_buffer("emoji", nw, rng)
            Tw = T // 2
            k = max(1, (nw // Tw) // 2)
            edge = k * Tw
            if edge >= nw:
                continue
            w = base.copy()
            # a lone high surrogate at edge-1 followed by a non-surrogate
            if 0xDC00 <= w[edge - 1] < 0xE000:
                pass
            if 0xD800 <= w[edge - 2] < 0xDC00:
                w[edge - 2] = 0x41
            w[edge - 1] = 0xD83D
            w[edge] = 0x42
            if edge + 1 < nw and 0xDC00 <= w[edge + 1] < 0xE000:
                w[edge + 1] = 0x43
            cases.append((w, edge - 1))
            c = base.copy()
            if 0xD800 <= c[edge - 2] < 0xDC00:
                c[edge - 2] = 0x41
            if edge + 1 < nw and 0xDC00 <= c[edge + 1] < 0xE000:
                c[edge + 1] = 0x43
            c[edge - 1] = 0xD83D
            c[edge] = 0xDE00
            cases.append((c, None))
    return cases


def stream_cuts(n_units: int, rng: np.random.Generator, max_chunk: int, min_chunk: int = 0) -> List[int]:
    """Chunk boundaries [0, c1, ..., n] of a stream cut at arbitrary unit offsets: chunk
    lengths uniform in [min_chunk, max_chunk] (empty chunks included when min_chunk = 0)."""
    cuts = [0]
    while cuts[-1] < n_units:
        cuts.append(min(n_units, cuts[-1] + int(rng.integers(min_chunk, max_chunk + 1))))
    return cuts


def utf32_buffer(profile: str, n_units: int, rng: np.random.Generator) -> np.ndarray:
    """n_units i.i.d. code points of the profile as a UTF-32 buffer (uint32)."""
    return draw_codepoints(profile, n_units, rng)


def inject_utf32(units: np.ndarray, rate: float, rng: np.random.Generator) -> Tuple[np.ndarray, List[int]]:
    """A copy of a UTF-32 buffer with units replaced at the given rate (at least one) by
    values that are not characters: surrogates, the first value past U+10FFFF, random
    larger values.  Returns (buffer, sorted positions)."""
    out = np.array(units, dtype=np.uint32, copy=True)
    k = max(1, int(rng.binomial(out.size, rate)))
    pos = np.unique(rng.integers(0, out.size, size=k))
    bad = np.concatenate([rng.integers(0xD800, 0xE000, size=pos.size), np.full(pos.size, 0x110000),
                          rng.integers(0x110000, 1 << 32, size=pos.size)]).astype(np.uint32)
    out[pos] = rng.choice(bad, size=pos.size)
    return out, pos.tolist()
