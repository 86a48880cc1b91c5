"""CF cache files on the host: names, round trip and refusal of damaged
files (no GPU).  The on-disk model of the CFCache plugin (AWP framework
section) must hand back exactly the bytes it was given, and never a table
other than the one asked for."""

import os

import numpy as np
import pytest

from paper_2508_17187_amd import cfcache as C

SPEC = dict(terms=3, oversample=20, ps_support=7, n_w=32, w_max=4.8e5, h_min=8, h_max=32,
            n_fg=1, fg_hz=np.array([3.0e9]), dish_m=25.0, screen_m=0, storage=1)
GRID = (2048, 2048, 4, 1, 9.696273622190722e-07, 9.696273622190722e-07)


def test_key_is_deterministic_and_exact():
    k = C.cf_key(GRID, SPEC)
    assert k == C.cf_key(list(GRID), dict(SPEC, fg_hz=[3.0e9]))
    assert k == C.cf_key(dict(zip(("nx", "ny", "npol", "nplane", "cell_l", "cell_m"), GRID)), SPEC)
    # every field that shapes the table changes the name, down to one ulp
    for f in ("terms", "oversample", "ps_support", "n_w", "h_min", "h_max", "screen_m", "storage"):
        assert C.cf_key(GRID, dict(SPEC, **{f: SPEC[f] + 1})) != k, f
    for f in ("w_max", "dish_m"):
        assert C.cf_key(GRID, dict(SPEC, **{f: np.nextafter(SPEC[f], np.inf)})) != k, f
    assert C.cf_key(GRID, dict(SPEC, fg_hz=np.array([np.nextafter(3.0e9, 0)]))) != k
    assert C.cf_key(GRID, dict(SPEC, n_fg=2, fg_hz=np.array([3.0e9, 3.5e9]))) != k
    for i in range(6):
        g = list(GRID)
        g[i] = g[i] + 1 if i < 4 else np.nextafter(g[i], 1.0)
        assert C.cf_key(g, SPEC) != k, i


def _write(tmp_path, blob, name="t.lrcf"):
    hdr = dict(C.describe(GRID, SPEC), key=C.cf_key(GRID, SPEC), nbytes=int(blob.size))
    p = os.path.join(str(tmp_path), name)
    C.write_table(p, hdr, [blob[:blob.size // 3], blob[blob.size // 3:]])
    return p, hdr


def _read(p, chunk=4093, verify=True):
    h, off = C.read_header(p)
    out = np.zeros(h["nbytes"], np.uint8)

    def sink(v, s):
        out[s:s + len(v)] = v

    C.read_blob(p, off, h["nbytes"], sink, verify=verify, chunk=chunk)
    return h, out


@pytest.mark.parametrize("n", [0, 1, 4093, 100003])
def test_round_trip(tmp_path, n):
    blob = np.random.default_rng(n).integers(0, 256, n, dtype=np.uint8)
    p, hdr = _write(tmp_path, blob)
    h, out = _read(p)
    assert h == hdr
    assert np.array_equal(out, blob)
    assert os.path.getsize(p) == 16 + len(C.json.dumps(hdr, sort_keys=True).encode()) + n + 32


def test_damaged_files_are_refused(tmp_path):
    blob = np.random.default_rng(1).integers(0, 256, 50000, dtype=np.uint8)
    p, _ = _write(tmp_path, blob)
    raw = bytearray(open(p, "rb").read())
    # one flipped bit in the blob: the checksum catches it
    bad = bytearray(raw)
    bad[-100] ^= 1
    open(p, "wb").write(bad)
    with pytest.raises(C.BadTable):
        _read(p)
    _read(p, verify=False)            # without verification the bytes are read as they are
    # wrong magic, truncated file, garbage header
    for mutate in (lambda b: b"XXXX" + b[4:], lambda b: b[:-1], lambda b: b[:20],
                   lambda b: b[:16] + b"{" * 8 + b[24:]):
        open(p, "wb").write(bytes(mutate(bytes(raw))))
        with pytest.raises(C.BadTable):
            _read(p)


def test_failed_write_leaves_no_file(tmp_path):
    blob = np.zeros(10, np.uint8)
    hdr = dict(C.describe(GRID, SPEC), key="k", nbytes=11)      # wrong size
    p = os.path.join(str(tmp_path), "k.lrcf")
    with pytest.raises(ValueError):
        C.write_table(p, hdr, [blob])
    assert os.listdir(str(tmp_path)) == []
