"""Batched multi-view training step, captured as a HIP graph.

Several views of uneven resolution advance one step together:
projection of every view in one pass over the Gaussians (pgs_project_views)
-> one bin/sort over all views
(pgs_bin_sort_views) -> heavy-first order of all tiles (pgs_tile_order) ->
one persistent compositing launch over every (view, tile) (pgs_render_fwd_views;
with the trace in natural tile order)
-> loss per view -> one persistent backward launch (pgs_render_bwd_views) ->
projection backward of every view in one pass into the canonical gradient
(pgs_project_bwd_views) -> Adam with the
step counter on the device (pgs_adam_step_dev).  Nothing in a step reads
back to the host, so the whole step can be captured once (pgs_graph_begin /
pgs_graph_end record the launches on the capture stream) and replayed with
pgs_graph_launch; buffers are allocated beforehand and the overflow flags
are read between replays (pgs_check_flags).  Tile shape, LDS batch size and the persistent grid
are parameters, chosen by `autotune`.
"""

from __future__ import annotations

import math

import torch

from . import binding as B
from ._lib import GRAD2D_STRIDE, PGS_FLAG_CACHE_OVERFLOW, PGS_FLAG_PAIR_OVERFLOW, PROJ_STRIDE
from .raster import MAX_ENTRIES, TRACE_WORDS, new_trace, param_rows
from .train import BETA1, BETA2, EPS, learning_rates


class BatchedStep:
    def __init__(self, params: torch.Tensor, sh_degree: int, cams: list, targets: list, tile=(16, 16),
                 batch: int = 256, blocks: int = 0, cached: bool = True, lam: float = 0.2, extent: float = 1.0,
                 capacity: int | None = None, bg=(0.0, 0.0, 0.0), ordered: bool = True,
                 entries: int | None = None, trace_words: int = TRACE_WORDS):
        self.params = params.contiguous()
        self.sh_degree = int(sh_degree)
        self.F, self.n = self.params.shape
        assert self.F == param_rows(self.sh_degree)
        d = self.device = self.params.device
        self.views = B.ViewBatch(cams, tile, batch, blocks)
        self.cams = list(cams)
        self.V = len(cams)
        self.cached, self.lam, self.bg = cached, lam, tuple(float(x) for x in bg)
        self.trace_words = int(trace_words)
        n, V = self.n, self.V
        self.tw, self.th = self.views.tile_w, self.views.tile_h
        self.nt = self.views.n_tiles
        self.npx = self.views.n_pixels
        self.proj = torch.empty((V, n, PROJ_STRIDE), dtype=torch.float32, device=d)
        self.radius = torch.empty((V, n), dtype=torch.int32, device=d)
        self.rect = torch.empty((V, 2, n), dtype=torch.int32, device=d)
        self.touched = torch.empty((V, n), dtype=torch.int32, device=d)
        self.ranges = torch.empty((2, self.nt), dtype=torch.int32, device=d)
        self.order = torch.empty(self.nt, dtype=torch.int32, device=d) if ordered else None
        self.queue = torch.zeros(4, dtype=torch.int32, device=d)
        self.num_pairs = torch.zeros(1, dtype=torch.int32, device=d)
        self.flags = torch.zeros(1, dtype=torch.int32, device=d)
        self.image = torch.empty(3 * self.npx, dtype=torch.float32, device=d)
        self.t_final = torch.empty(self.npx, dtype=torch.float32, device=d)
        self.n_contrib = torch.empty(self.npx, dtype=torch.int32, device=d)
        self.dl = torch.zeros(3 * self.npx, dtype=torch.float32, device=d)
        self.target = torch.empty(3 * self.npx, dtype=torch.float32, device=d)
        for v, t in enumerate(targets):
            self.view_slice(self.target, v).copy_(t.reshape(3, self.cams[v]["height"], self.cams[v]["width"]))
        self.grad2d = torch.zeros((V, n, GRAD2D_STRIDE), dtype=torch.float32, device=d)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.adam_state = torch.zeros(4, dtype=torch.int32, device=d)
        self.lr = learning_rates(self.sh_degree, extent)
        self.losses = torch.zeros(V, dtype=torch.float32, device=d)
        ws = max(B.pgs_loss_workspace(c["width"], c["height"]) for c in self.cams)
        self.loss_ws = torch.empty(ws, dtype=torch.uint8, device=d)
        self.capacity = 0
        self.graph = None
        self.events = None       # list: HIP events recorded after each stage (eager steps only)
        self.entry_capacity = int(entries) if entries is not None else max(1 << 20, 32 * self.npx)
        self._alloc_pairs(capacity if capacity is not None else max(4096, 4 * n * V))

    # -- layout ----------------------------------------------------------
    def view_slice(self, buf: torch.Tensor, v: int, channels: int = 3) -> torch.Tensor:
        p0, p1 = self.views.pixel_offsets[v], self.views.pixel_offsets[v + 1]
        W, H = self.cams[v]["width"], self.cams[v]["height"]
        if channels == 3:
            return buf[3 * p0:3 * p1].view(3, H, W)
        return buf[p0:p1].view(H, W)

    def _alloc_pairs(self, capacity: int, entries: int | None = None):
        capacity = int(capacity)
        if entries is not None:
            self.entry_capacity = min(int(entries), MAX_ENTRIES)
        d = self.device
        self.release_graph()
        self.keys = self.values = self.workspace = self.trace = None
        self.capacity = capacity
        self.keys = torch.empty(max(capacity, 1), dtype=torch.int64, device=d)
        self.values = torch.empty(max(capacity, 1), dtype=torch.int32, device=d)
        self.workspace = torch.empty(B.pgs_bin_sort_workspace(self.n * self.V, capacity), dtype=torch.uint8,
                                     device=d)
        if self.cached:
            self.trace = new_trace(capacity, self.tw * self.th // 64, self.nt, self.npx, self.entry_capacity, d,
                                   self.trace_words)

    def memory_bytes(self) -> int:
        tot = 0
        for t in list(vars(self).values()) + (list(self.trace.values()) if self.trace else []):
            if isinstance(t, torch.Tensor):
                tot += t.numel() * t.element_size()
        return tot

    # -- the step ----------------------------------------------------------
    def _mark(self, name):
        if self.events is not None:
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            self.events.append((name, ev))

    def forward(self):
        n = self.n
        self._mark("start")
        B.pgs_project_views(self.views, self.params, n, self.sh_degree, self.proj, self.radius, self.rect,
                            self.touched)
        self._mark("project_views")
        B.pgs_bin_sort_views(self.views, n, self.proj, self.rect, self.touched, self.capacity, self.keys,
                             self.values, self.ranges, self.num_pairs, self.flags, self.workspace)
        if self.order is not None:
            B.pgs_tile_order(self.ranges, self.nt, 0, self.nt, self.order)
        self._mark("bin_sort_views")
        # the forward that records the trace takes the tiles in natural order
        # (neighbouring pair ranges and mask runs together), the others
        # heavy-first, as in the single-view rasterizer
        B.pgs_render_fwd_views(self.views, self.proj, n, self.values, self.ranges, self.bg, self.image,
                               self.t_final, self.n_contrib, self.trace if self.cached else None, self.flags,
                               None if self.cached else self.order, self.queue)
        self._mark("render_fwd")

    def backward_from(self, dl=None):
        """Render and projection backward from dL/dimage (default: self.dl);
        accumulates into self.grads (the caller zeroes it)."""
        n = self.n
        self.grad2d.zero_()
        self._mark("zero")
        B.pgs_render_bwd_views(self.views, self.proj, n, self.values, self.ranges, self.bg, self.t_final,
                               self.n_contrib, self.trace if self.cached else None,
                               self.dl if dl is None else dl, self.grad2d, self.order, self.queue)
        self._mark("render_bwd")
        B.pgs_project_bwd_views(self.views, self.params, n, self.sh_degree, self.radius, self.grad2d, self.grads)
        self._mark("project_bwd_views")

    def step(self):
        """One full training step over every view (no host synchronisation)."""
        self.forward()
        for v, cam in enumerate(self.cams):
            B.pgs_loss_l1_dssim(self.view_slice(self.image, v), self.view_slice(self.target, v), cam["width"],
                                cam["height"], self.lam, self.losses[v:v + 1], self.view_slice(self.dl, v),
                                self.loss_ws)
        self._mark("loss")
        self.grads.zero_()
        self.backward_from()
        B.pgs_adam_step_dev(self.params, self.grads, self.m, self.v, self.F, self.n, self.lr, self.adam_state,
                            BETA1, BETA2, EPS)
        self._mark("adam")

    # -- overflow protocol -------------------------------------------------
    def read_flags(self) -> int:
        return B.pgs_check_flags(self.flags)[1]

    def prepare(self, max_retries=8, headroom=1.5):
        """Forward until the pair buffers fit (synchronises); drops any graph."""
        for _ in range(max_retries + 1):
            self.flags.zero_()
            self.forward()
            if self.read_flags() & (PGS_FLAG_PAIR_OVERFLOW | PGS_FLAG_CACHE_OVERFLOW) == 0:
                return
            need = int(self.num_pairs.item())
            cap = self.capacity if need <= self.capacity else int(math.ceil(need * headroom)) + 4096
            used = int(self.trace["used"].item()) if self.trace is not None else 0
            ents = self.entry_capacity if used <= self.entry_capacity else int(math.ceil(used * headroom)) + 4096
            self._alloc_pairs(cap, ents)
        raise RuntimeError("batched step buffers kept overflowing")

    # -- optimiser state -----------------------------------------------------
    def snapshot(self):
        """Copies of the parameters, Adam moments and step counter."""
        return [t.clone() for t in (self.params, self.m, self.v, self.adam_state)]

    def restore(self, snap):
        """Puts a snapshot back in place (same buffers, so a captured graph
        keeps working)."""
        for dst, src in zip((self.params, self.m, self.v, self.adam_state), snap):
            dst.copy_(src)

    # -- graph -------------------------------------------------------------
    def capture(self):
        """Records one step as a graph through the library's graph calls
        (pgs_graph_begin / pgs_graph_end) on a side stream, after a warm-up
        step there, which advances the Adam state like any step.  The step
        allocates nothing, so the recorded nodes are kernels only."""
        self.release_graph()
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self.step()
            B.pgs_graph_begin(s)
            try:
                self.step()
            finally:
                g = B.pgs_graph_end(s)
        torch.cuda.current_stream(self.device).wait_stream(s)
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        B.pgs_graph_launch(self.graph)

    def release_graph(self):
        if self.graph is not None:
            torch.cuda.synchronize(self.device)
            B.pgs_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.release_graph()
        except Exception:
            pass

    def stats(self) -> dict:
        return dict(views=self.V, gaussians=self.n, pixels=self.npx, tiles=self.nt,
                    pairs=int(self.num_pairs.item()), tile=f"{self.tw}x{self.th}", batch=self.views.batch,
                    trace_gb=round(sum(t.numel() * t.element_size() for t in self.trace.values()
                                       if isinstance(t, torch.Tensor)) / 1e9, 3) if self.trace else 0.0)


# Eight view sizes from 640x480 to 1920x1440: 9,733,632 pixels, 38,092
# tiles of 16x16 in total.
MIXED_SIZES = ((640, 480), (800, 600), (960, 720), (1024, 768), (1280, 960), (1440, 1080), (1600, 1200),
               (1920, 1440))


def mixed_views(n_views=8, radius=4.5, sizes=MIXED_SIZES):
    """Ring cameras of uneven resolution (one size per view, cycled)."""
    import synth
    return [synth.ring_cameras(n_views, *sizes[i % len(sizes)], radius=radius)[i] for i in range(n_views)]


def time_steps(step_fn, steps: int, warmup: int) -> float:
    """Average ms per call of step_fn with HIP events on the current stream."""
    for _ in range(warmup):
        step_fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step_fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps

