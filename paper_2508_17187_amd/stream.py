"""Gridding and degridding of observations larger than one call, in row
chunks streamed from pinned host memory.

Every chunk is one lr_grid (accumulating into the same grid and sums of
weights) or lr_degrid call with a plan of its own.  Two device input buffers
alternate: the copy of chunk i + 1 runs on a copy stream while chunk i is
planned and gridded on the compute stream.  Gridding a sum of chunks equals
gridding their union, because the gridding sum runs over independent
samples (the partition additivity of Eq. IMAGE-MOD), so the chunk size
changes only the order of FP32 additions.
"""

import numpy as np
import torch

from . import lr


class ChunkStreamer:
    """uvw, vis and weight are host tensors [nrow, ...] in pinned memory
    (torch pin_memory); freq_hz, chan_plane, chan_fg are host arrays.
    chunk_rows rows travel per chunk."""

    def __init__(self, cf, precision, uvw, freq_hz, chan_plane=None, chan_fg=None,
                 weight=None, chunk_rows=390625, device="cuda"):
        self.cf, self.p, self.dev = cf, precision, device
        self.uvw_h, self.weight_h = uvw, weight
        self.freq = np.asarray(freq_hz, np.float64)
        self.chan_plane, self.chan_fg = chan_plane, chan_fg
        self.nrow = int(uvw.shape[0])
        self.chunk = int(min(chunk_rows, self.nrow))
        self.cdt = torch.complex128 if precision == lr.LR_F64 else torch.complex64
        self.rdt = torch.float64 if precision == lr.LR_F64 else torch.float32
        for t in (uvw, weight):
            if t is not None and not t.is_pinned():
                raise ValueError("host arrays must be in pinned memory")
        self.copy = torch.cuda.Stream(device=device)
        nchan, npol = weight.shape[1], weight.shape[2]
        self.bufs = [dict(uvw=torch.empty((self.chunk, 3), dtype=torch.float64, device=device),
                          vis=torch.empty((self.chunk, nchan, npol), dtype=self.cdt,
                                          device=device),
                          weight=torch.empty((self.chunk, nchan, npol), dtype=self.rdt,
                                             device=device),
                          done=torch.cuda.Event(), ready=torch.cuda.Event())
                     for _ in range(2)]
        v = self._vis(self.bufs[0], self.chunk)
        self.plan_buf = torch.empty(lr.plan_bytes(cf, v), dtype=torch.uint8, device=device)
        self.work = None

    def chunks(self):
        return [(r, min(r + self.chunk, self.nrow)) for r in range(0, self.nrow, self.chunk)]

    def _vis(self, b, n, with_vis=True):
        return lr.Vis(b["uvw"][:n], self.freq, self.chan_plane, self.chan_fg,
                      vis=b["vis"][:n] if with_vis else None, weight=b["weight"][:n])

    def _load(self, i, r0, r1, vis_h):
        b = self.bufs[i % 2]
        n = r1 - r0
        with torch.cuda.stream(self.copy):
            # the compute stream has finished with this buffer
            self.copy.wait_event(b["done"])
            b["uvw"][:n].copy_(self.uvw_h[r0:r1], non_blocking=True)
            b["weight"][:n].copy_(self.weight_h[r0:r1], non_blocking=True)
            if vis_h is not None:
                b["vis"][:n].copy_(vis_h[r0:r1], non_blocking=True)
            b["ready"].record(self.copy)
        return b

    def grid(self, vis_h, grid, sumwt=None, counters=None):
        """grid += G(all rows); sumwt and counters accumulate too."""
        cur = torch.cuda.current_stream(self.dev)
        ch = self.chunks()
        for b in self.bufs:
            b["done"].record(cur)
        nxt = self._load(0, *ch[0], vis_h)
        for i, (r0, r1) in enumerate(ch):
            b = nxt
            cur.wait_event(b["ready"])
            if i + 1 < len(ch):
                nxt = self._load(i + 1, *ch[i + 1], vis_h)
            v = self._vis(b, r1 - r0)
            v.plan = lr.Plan(self.cf, v, stream=cur, buf=self.plan_buf)
            self.work = lr.lr_grid(self.cf, v, self.p, grid, sumwt=sumwt, counters=counters,
                                   work=self.work, stream=cur)
            b["done"].record(cur)
        return grid

    def degrid(self, grid, vis_out_h):
        """vis_out_h (pinned host) = D(grid) for all rows."""
        cur = torch.cuda.current_stream(self.dev)
        ch = self.chunks()
        for b in self.bufs:
            b["done"].record(cur)
        nxt = self._load(0, *ch[0], None)
        for i, (r0, r1) in enumerate(ch):
            b = nxt
            cur.wait_event(b["ready"])
            if i + 1 < len(ch):
                nxt = self._load(i + 1, *ch[i + 1], None)
            v = self._vis(b, r1 - r0)
            v.plan = lr.Plan(self.cf, v, stream=cur, buf=self.plan_buf)
            self.work = lr.lr_degrid(self.cf, v, self.p, grid, work=self.work, stream=cur)
            vis_out_h[r0:r1].copy_(b["vis"][:r1 - r0], non_blocking=True)
            b["done"].record(cur)
        cur.synchronize()
        return vis_out_h
