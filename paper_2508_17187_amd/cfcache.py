"""CF cache: the CFCache plugin of the AWP framework (section on the AWP
framework; the CF configuration table).

CF tables stay in device memory between uses (in-memory model) and, given a
directory, also on disk between runs (persistent model).  A table is named by
everything its bytes depend on: the CF specification (terms, oversampling,
supports, w-planes, frequency groups, dish and screen size, storage type) and
the grid geometry.  The cache is filled the three ways the paper's cache can
be configured: `precompute` a list of tables up front, `get` on demand, or
both, so that a precomputed cache grows with use.  Every table built while a
directory is set is written there, and a later cache over the same directory
loads it instead of building it.

On-disk format (one file per table, `<key>.lrcf`; read with plain file I/O,
nothing in it is executed):

    8 bytes   magic  b"LRCF" 0x00 0x01 0x00 0x00
    8 bytes   little-endian length H of the header
    H bytes   UTF-8 JSON header: key, grid, spec (floats as hex strings, so
              they round-trip exactly), nbytes
    nbytes    the CF blob exactly as lr_cf_build wrote it (it is flat and
              relocatable: lr_cf_attach wraps it again)
    32 bytes  SHA-256 of the blob

A file whose magic, header, size or checksum does not match is not used: the
table is rebuilt and the file rewritten (counted in stats["bad_files"]).

When a byte budget is given, the least recently used tables leave device
memory once the resident total exceeds it (the one just requested stays).
"""

import collections
import hashlib
import json
import os
import struct
import tempfile

import numpy as np

MAGIC = b"LRCF\x00\x01\x00\x00"
SUFFIX = ".lrcf"
CHUNK = 64 << 20          # host staging per transfer step


class BadTable(Exception):
    """A cache file that cannot be used for the requested table."""


_GRID_FIELDS = ("nx", "ny", "npol", "nplane", "cell_l", "cell_m")
_SPEC_FIELDS = ("terms", "oversample", "ps_support", "n_w", "w_max", "h_min", "h_max",
                "n_fg", "dish_m", "screen_m", "storage")


def _exact(v):
    """JSON-safe exact form of an int or float."""
    if isinstance(v, (float, np.floating)):
        return float(v).hex()
    return int(v)


def describe(grid, spec):
    """Canonical description of a table: grid fields (a GridSpec or any
    object with nx, ny, npol, nplane, cell_l, cell_m) and spec fields (the
    dict lr_cf_build takes, fg_hz included)."""
    if isinstance(grid, (tuple, list)):
        grid = dict(zip(_GRID_FIELDS, grid))
    get = grid.get if isinstance(grid, dict) else (lambda f: getattr(grid, f))
    g = {f: _exact(get(f)) for f in _GRID_FIELDS}
    s = {f: _exact(spec[f]) for f in _SPEC_FIELDS}
    s["fg_hz"] = [float(x).hex() for x in np.asarray(spec["fg_hz"], np.float64).ravel()]
    if spec.get("pol_beam", 0):
        # a polarised beam (scalar-beam tables keep the names they had)
        for f in ("pol_beam", "beam_ellipticity", "beam_leakage"):
            s[f] = _exact(spec[f])
    return {"grid": g, "spec": s}


def cf_key(grid, spec):
    """Name of a table: SHA-256 of its canonical description."""
    d = json.dumps(describe(grid, spec), sort_keys=True, separators=(",", ":"))
    return hashlib.sha256(d.encode()).hexdigest()[:40]


# ---- files (host only) -------------------------------------------------------

def write_table(path, header, chunks):
    """Write a cache file from an iterable of byte chunks (the blob, in
    order), atomically: a partial file never carries the final name."""
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    h = json.dumps(header, sort_keys=True).encode()
    sha = hashlib.sha256()
    n = 0
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    try:
        with os.fdopen(fd, "wb") as f:
            f.write(MAGIC)
            f.write(struct.pack("<Q", len(h)))
            f.write(h)
            for c in chunks:
                mv = memoryview(c).cast("B")
                sha.update(mv)
                f.write(mv)
                n += len(mv)
            f.write(sha.digest())
        if n != header["nbytes"]:
            raise ValueError("blob has %d bytes, header says %d" % (n, header["nbytes"]))
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise


def read_header(path):
    """(header dict, byte offset of the blob); BadTable if the file is not a
    well-formed cache file."""
    try:
        with open(path, "rb") as f:
            if f.read(8) != MAGIC:
                raise BadTable("%s: not a CF cache file" % path)
            raw = f.read(8)
            if len(raw) != 8:
                raise BadTable("%s: truncated header" % path)
            (hl,) = struct.unpack("<Q", raw)
            if hl > (1 << 24):
                raise BadTable("%s: header length %d" % (path, hl))
            hb = f.read(hl)
            if len(hb) != hl:
                raise BadTable("%s: truncated header" % path)
            header = json.loads(hb.decode())
        size = os.path.getsize(path)
    except (OSError, ValueError, UnicodeDecodeError) as e:
        raise BadTable("%s: %s" % (path, e))
    off = 16 + hl
    if not isinstance(header, dict) or "nbytes" not in header:
        raise BadTable("%s: header without nbytes" % path)
    if size != off + int(header["nbytes"]) + 32:
        raise BadTable("%s: %d bytes on disk, expected %d" % (path, size,
                                                            off + int(header["nbytes"]) + 32))
    return header, off


def read_blob(path, offset, nbytes, sink, verify=True, chunk=CHUNK, staging=None):
    """Stream the blob to `sink(view, start)` in chunks of at most `chunk`
    bytes (views of `staging`, a uint8 numpy array, when given) and check
    its SHA-256 against the trailer (verify=True)."""
    sha = hashlib.sha256() if verify else None
    buf = staging if staging is not None else np.empty(min(chunk, max(nbytes, 1)), np.uint8)
    with open(path, "rb") as f:
        f.seek(offset)
        done = 0
        while done < nbytes:
            n = min(len(buf), nbytes - done)
            view = buf[:n]
            got = f.readinto(memoryview(view))
            if got != n:
                raise BadTable("%s: truncated blob" % path)
            if sha is not None:
                sha.update(memoryview(view))
            sink(view, done)
            done += n
        trailer = f.read(32)
    if len(trailer) != 32:
        raise BadTable("%s: missing checksum" % path)
    if sha is not None and sha.digest() != trailer:
        raise BadTable("%s: checksum mismatch" % path)


# ---- the cache ---------------------------------------------------------------

class CFCache:
    """In-memory (device) and optional on-disk cache of CF tables.

    directory   where tables are persisted (None: memory only)
    budget      bytes of resident tables before least recently used ones
                leave device memory (None: no limit)
    verify      check the SHA-256 of files read from disk
    """

    def __init__(self, directory=None, device="cuda", budget=None, verify=True):
        self.directory = directory
        self.device = device
        self.budget = budget
        self.verify = verify
        self.mem = collections.OrderedDict()      # key -> CF, LRU order
        self.resident = 0
        self.stats = dict(hits=0, loads=0, builds=0, saves=0, evictions=0, bad_files=0)

    def path(self, key):
        return os.path.join(self.directory, key + SUFFIX)

    def __contains__(self, key):
        return key in self.mem

    def get(self, grid, spec, stream=None):
        """The table for (grid, spec): resident, else loaded from disk, else
        built (and then written to disk when a directory is set)."""
        key = cf_key(grid, spec)
        cf = self.mem.get(key)
        if cf is not None:
            self.mem.move_to_end(key)
            self.stats["hits"] += 1
            return cf
        if self.directory and os.path.exists(self.path(key)):
            try:
                cf = self._load(key, grid, spec, stream)
                self.stats["loads"] += 1
            except (BadTable, OSError):
                self.stats["bad_files"] += 1
                cf = None
        if cf is None:
            cf = self._build(grid, spec, stream)
            self.stats["builds"] += 1
            if self.directory:
                self.save(cf, key)
        self._insert(key, cf)
        return cf

    def precompute(self, items, stream=None):
        """Fill the cache with every (grid, spec) of `items` up front."""
        return [self.get(g, s, stream=stream) for g, s in items]

    def evict(self, key):
        cf = self.mem.pop(key, None)
        if cf is not None:
            self.resident -= cf.nbytes
            self.stats["evictions"] += 1

    # -- internals
    def _insert(self, key, cf):
        self.mem[key] = cf
        self.resident += cf.nbytes
        if self.budget is not None:
            while self.resident > self.budget and len(self.mem) > 1:
                old = next(iter(self.mem))
                if old == key:
                    break
                self.evict(old)

    def _build(self, grid, spec, stream):
        from . import lr
        return lr.lr_cf_build(grid, dict(spec), device=self.device, stream=stream)

    def save(self, cf, key=None):
        """Write a resident table to the directory (device -> pinned host ->
        file, in chunks)."""
        import torch
        key = key or cf_key(cf.grid, self._spec_of(cf))
        header = dict(describe(cf.grid, self._spec_of(cf)), key=key, nbytes=int(cf.nbytes))
        torch.cuda.synchronize()
        staging = torch.empty(min(CHUNK, cf.nbytes), dtype=torch.uint8, pin_memory=True)

        def chunks():
            for s in range(0, cf.nbytes, CHUNK):
                n = min(CHUNK, cf.nbytes - s)
                staging[:n].copy_(cf.blob[s:s + n])
                yield staging[:n].numpy()

        write_table(self.path(key), header, chunks())
        self.stats["saves"] += 1

    def _load(self, key, grid, spec, stream):
        import torch
        from . import lr
        header, off = read_header(self.path(key))
        want = describe(grid, spec)
        if header.get("key") != key or header.get("grid") != want["grid"] or \
                header.get("spec") != want["spec"]:
            raise BadTable("%s: describes another table" % self.path(key))
        nbytes = int(header["nbytes"])
        blob = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        staging = torch.empty(min(CHUNK, max(nbytes, 1)), dtype=torch.uint8, pin_memory=True)

        def sink(view, start):
            blob[start:start + len(view)].copy_(staging[:len(view)])

        read_blob(self.path(key), off, nbytes, sink, verify=self.verify,
                  staging=staging.numpy())
        cf = lr.CF(grid, dict(spec), device=self.device, stream=stream, blob=blob)
        if cf.nbytes != nbytes:
            raise BadTable("%s: %d bytes for a table of %d" % (self.path(key), nbytes, cf.nbytes))
        return cf

    @staticmethod
    def _spec_of(cf):
        s = {f: getattr(cf.spec, f) for f in _SPEC_FIELDS}
        s["fg_hz"] = cf.fg
        return s
