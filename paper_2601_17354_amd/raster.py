"""Per-view rasterizer: owns the device buffers and sequences the C ABI calls.

forward:  pgs_project -> pgs_bin_sort -> pgs_render_fwd (optionally recording
          the replay trace S = {id, C_in, alpha} and count(u))
backward: pgs_render_bwd (trace replay, or recompute-T) -> pgs_project_bwd

Buffers are allocated with PyTorch once and reused; the pair capacity and the
replay trace grow when the device flags report an overflow (the caller
runs `forward_checked`, which synchronises once to read the flags).
"""

from __future__ import annotations

import math

import torch

from . import binding as B
from ._lib import GRAD2D_STRIDE, PGS_FLAG_CACHE_OVERFLOW, PGS_FLAG_PAIR_OVERFLOW, PROJ_STRIDE


def param_rows(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


MAX_ENTRIES = (1 << 32) - 1


# Words per replay-trace entry: 3 = C_in (alpha recomputed by the backward
# from the staged splat, same bits), 4 = (C_in, alpha) as the paper's cache
# stores it.  The lean layout moves a quarter fewer trace bytes.
TRACE_WORDS = 3


def new_trace(pair_capacity: int, nw: int, n_tiles: int, pixels: int, entries: int, device,
              words: int = TRACE_WORDS) -> dict:
    """Replay-trace buffers (layout of pgs_replay): masks per pair slot and
    wave, per-wave step counters and entry offsets, the entry counter,
    `entries` entries of `words` floats and per-pixel counts."""
    entries = max(1, min(int(entries), MAX_ENTRIES))
    return dict(
        mask=torch.empty((nw, max(pair_capacity, 1)), dtype=torch.int64, device=device),
        steps=torch.empty((n_tiles, nw), dtype=torch.int32, device=device),
        base=torch.empty((n_tiles, nw), dtype=torch.int32, device=device),
        used=torch.zeros(1, dtype=torch.int64, device=device),
        entry=torch.empty((entries, words), dtype=torch.float32, device=device),
        count=torch.empty(pixels, dtype=torch.int32, device=device),
        entry_capacity=entries, pair_capacity=int(pair_capacity),
    )


class Rasterizer:
    def __init__(self, n: int, sh_degree: int, width: int, height: int, tile=(16, 16),
                 cached: bool = True, capacity: int | None = None,
                 device="cuda", ordered: bool = True, entries: int | None = None,
                 trace_words: int = TRACE_WORDS):
        self.n = int(n)
        self.sh_degree = int(sh_degree)
        self.W, self.H = int(width), int(height)
        self.tw, self.th = tile
        self.TX = (self.W + self.tw - 1) // self.tw
        self.TY = (self.H + self.th - 1) // self.th
        self.n_tiles = self.TX * self.TY
        self.cached = cached
        self.trace_words = int(trace_words)
        self.device = torch.device(device)
        d = self.device
        n = max(self.n, 1)
        self.proj = torch.empty((n, PROJ_STRIDE), dtype=torch.float32, device=d)
        self.radius = torch.empty(n, dtype=torch.int32, device=d)
        self.rect = torch.empty((2, n), dtype=torch.int32, device=d)
        self.touched = torch.empty(n, dtype=torch.int32, device=d)
        self.ranges = torch.empty((2, self.n_tiles), dtype=torch.int32, device=d)
        self.num_pairs = torch.zeros(1, dtype=torch.int32, device=d)
        self.flags = torch.zeros(1, dtype=torch.int32, device=d)
        self.image = torch.empty((3, self.H, self.W), dtype=torch.float32, device=d)
        self.t_final = torch.empty((self.H, self.W), dtype=torch.float32, device=d)
        self.n_contrib = torch.empty((self.H, self.W), dtype=torch.int32, device=d)
        self.grad2d = torch.zeros((n, GRAD2D_STRIDE), dtype=torch.float32, device=d)
        # Heavy-first launch order of the tiles (scheduling only), used by the
        # backward and by the forward without a trace.  The forward that
        # records the trace launches in natural tile order instead (see
        # fwd_order).
        self.tile_order = torch.empty(self.n_tiles, dtype=torch.int32, device=d) if ordered else None
        self.capacity = 0
        self.trace = None
        self.nw = self.tw * self.th // 64
        self.entry_capacity = int(entries) if entries is not None else max(1 << 20, 32 * self.W * self.H)
        self._alloc_pairs(capacity if capacity is not None else max(1024, 4 * self.n))
        # Work of each compositing launch, for measurement: when a list, every
        # forward and backward appends its pair count P, trace entries E and
        # pixels (reading them synchronises, so it is off by default).
        self.work_log = None
        self.log_tag = None       # recorded with each entry (e.g. the camera index)
        self.log_phase = None     # and this label (e.g. the part of a measurement)

    # -- buffers ---------------------------------------------------------
    def _alloc_pairs(self, capacity: int, entries: int | None = None):
        """Pair buffers, sort workspace and (cached mode) the replay trace:
        masks per pair slot and `entries` trace entries (default: keep)."""
        capacity = int(capacity)
        if entries is not None:
            self.entry_capacity = min(int(entries), MAX_ENTRIES)
        d = self.device
        self.capacity = capacity
        self.keys = self.values = self.workspace = self.trace = None
        self.keys = torch.empty(max(capacity, 1), dtype=torch.int64, device=d)
        self.values = torch.empty(max(capacity, 1), dtype=torch.int32, device=d)
        ws = B.pgs_bin_sort_workspace(self.n, capacity)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=d)
        if self.cached:
            self.trace = new_trace(capacity, self.nw, self.n_tiles, self.H * self.W, self.entry_capacity, d,
                                   self.trace_words)

    def reserve(self, pair_factor: float = 2.0):
        """Enlarge the pair capacity and the trace entries ahead of training,
        whose Gaussians grow and touch more tiles over time."""
        self._alloc_pairs(int(self.capacity * pair_factor), int(self.entry_capacity * pair_factor))

    def trace_bytes(self) -> int:
        if self.trace is None:
            return 0
        return sum(v.numel() * v.element_size() for v in self.trace.values() if isinstance(v, torch.Tensor))

    # -- passes ----------------------------------------------------------
    def forward(self, params: torch.Tensor, cam: dict, bg=(0.0, 0.0, 0.0)):
        """Enqueue projection, binning/sort and compositing for one view."""
        n = self.n
        B.pgs_project(params, n, self.sh_degree, cam, self.tw, self.th, self.proj, self.radius,
                      self.rect, self.touched)
        self.bin_sort()
        B.pgs_render_fwd(self.W, self.H, self.tw, self.th, self.proj, n, self.values, self.ranges,
                         0, bg, self.image, self.t_final, self.n_contrib,
                         self.trace if self.cached else None, self.flags, self.fwd_order)
        self.log_work("render_fwd")
        return self.image

    def work(self) -> dict:
        """Pair count P, trace entries E (0 without a trace), pixels and
        whether the buffers held the pass (no overflow flag) of the last
        forward (synchronises)."""
        P = min(int(self.num_pairs.item()), self.capacity)
        E = int(self.trace["used"].item()) if self.cached else 0
        return dict(P=P, E=E, pixels=self.W * self.H, ok=int(self.flags.item()) == 0)

    def log_work(self, kernel: str):
        if self.work_log is not None:
            w = self.work()
            w.update(kernel=kernel, cached=self.cached, tag=self.log_tag, phase=self.log_phase)
            self.work_log.append(w)

    @property
    def fwd_order(self):
        """Launch order of the forward.  With the trace, natural tile order:
        tiles that run together then write neighbouring mask runs and read
        neighbouring pair ranges and splats, and the write-bound entry pass
        measured 6% faster than heavy-first; without the trace (compute
        bound) heavy-first avoids a tail of long tiles and is faster."""
        return None if self.cached else self.tile_order

    def bin_sort(self):
        B.pgs_bin_sort(self.n, self.proj, self.rect, self.touched, self.TX, self.n_tiles, 0,
                       self.capacity, self.keys, self.values, self.ranges, self.num_pairs,
                       self.flags, self.workspace)
        if self.tile_order is not None:
            B.pgs_tile_order(self.ranges, self.n_tiles, 0, self.n_tiles, self.tile_order)

    def read_flags(self) -> int:
        return B.pgs_check_flags(self.flags)[1]

    def forward_checked(self, params, cam, bg=(0.0, 0.0, 0.0), max_retries=8, headroom=1.25):
        """forward(), then grow the pair capacity / trace depth and rerun while
        the device reports an overflow.  Synchronises once per attempt."""
        for _ in range(max_retries + 1):
            self.flags.zero_()
            self.forward(params, cam, bg)
            f = self.read_flags()
            if f == 0:
                return self.image
            if f & (PGS_FLAG_PAIR_OVERFLOW | PGS_FLAG_CACHE_OVERFLOW):
                need = int(self.num_pairs.item())
                cap = self.capacity
                if need > cap:
                    cap = int(math.ceil(need * headroom)) + 1024
                ents = self.entry_capacity
                used = int(self.trace["used"].item()) if self.trace is not None else 0
                if used > ents:
                    ents = int(math.ceil(used * headroom)) + 4096
                self._alloc_pairs(cap, ents)
        raise RuntimeError("rasterizer buffers kept overflowing")

    def backward(self, params, cam, dl_dimage, grads, bg=(0.0, 0.0, 0.0), zero_grad2d=True):
        """Enqueue the compositing backward and the projection backward;
        `grads` ([F][n]) is accumulated into."""
        if zero_grad2d:
            self.grad2d.zero_()
        B.pgs_render_bwd(self.W, self.H, self.tw, self.th, self.proj, self.n, self.values,
                         self.ranges, 0, bg, self.t_final, self.n_contrib,
                         self.trace if self.cached else None, dl_dimage, self.grad2d, self.tile_order)
        self.log_work("render_bwd")
        B.pgs_project_bwd(params, self.n, self.sh_degree, cam, self.radius, self.grad2d, grads)
        return grads
