"""Serving novel views of the global model with continuous batching.

After training only the global Gaussians z are kept and rendered (Sec. 3.2:
the local copies are dropped and the global model synthesises novel views).
This server renders z for a stream of requests at mixed resolutions:

  - requests wait in a queue in arrival order;
  - a batch is formed from the waiting requests whenever one of the
    in-flight slots is free, as many as the slot's preallocated HBM arena
    admits (records, pixels and tile pairs are budgeted per request from a
    per-resolution calibration);
  - each batch is one frame (one render job per request) and goes through
    gs_project -> gs_bin_sort -> gs_render_fwd on the slot's own HIP
    stream, so batches admitted while others are still on the GPU overlap
    with them on the device;
  - each request's image is copied into its own pinned host buffer on the
    same stream; the request completes when that copy has landed.

A request renders the same bits alone or in any batch: jobs share no
records, tiles or pixels.  Every slot's device arena is sized up front from
the HBM budget, and pinned output buffers are recycled through a pool, so
the serving loop allocates nothing large (only each batch's small job table
is uploaded).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import gs


@dataclass
class Request:
    rid: int
    cam: object
    arrival: float
    started: float = None
    done: float = None
    image: torch.Tensor = None        # pinned host [3][H][W] FP32
    tries: int = 0                    # launches that overflowed the pair budget

    @property
    def pixels(self):
        return self.cam.width * self.cam.height


class Arena:
    """Device buffers of one in-flight batch, carved per frame."""

    def __init__(self, n_gauss, max_jobs, max_pixels, max_tiles, capacity, device):
        self.n_gauss, self.max_jobs = n_gauss, max_jobs
        self.max_pixels, self.max_tiles, self.capacity = max_pixels, max_tiles, capacity
        R = n_gauss * max_jobs
        self.rec = torch.empty(R * gs.REC_WORDS, dtype=torch.float32, device=device)
        self.meta = torch.empty(R * gs.META_WORDS, dtype=torch.int32, device=device)
        self.pair_off = torch.empty(R, dtype=torch.int32, device=device)
        self.ranges = torch.empty(max_tiles * 2, dtype=torch.int32, device=device)
        self.tile_order = torch.empty(max_tiles + 4, dtype=torch.int32, device=device)
        self.counters = torch.zeros(gs.N_COUNTERS, dtype=torch.int32, device=device)
        self.rgb = torch.empty(max_pixels * 3, dtype=torch.float32, device=device)
        self.T = torch.empty(max_pixels, dtype=torch.float32, device=device)
        self.ncontrib = torch.empty(max_pixels, dtype=torch.int32, device=device)
        self._alloc_pairs(capacity)
        self.counters_host = torch.zeros(gs.N_COUNTERS, dtype=torch.int32).pin_memory()
        self.f64 = False
        self.frame = None

    def _alloc_pairs(self, capacity):
        self.capacity = int(capacity)
        self.vals = torch.empty(self.capacity, dtype=torch.int32, device=self.rec.device)
        nb = gs.lib.gs_bin_sort_workspace_size(self.n_gauss * self.max_jobs, self.capacity, self.max_tiles)
        self.bin_ws = torch.empty(nb, dtype=torch.uint8, device=self.rec.device)

    def grow_pairs(self, capacity):
        """Reallocate the pair buffers for a larger capacity (only while the
        slot is idle: its last batch has completed)."""
        if capacity > self.capacity:
            self._alloc_pairs(capacity)

    def nbytes(self):
        return sum(t.numel() * t.element_size() for t in (self.rec, self.meta, self.pair_off, self.ranges,
                                                           self.tile_order, self.rgb, self.T, self.ncontrib,
                                                           self.vals, self.bin_ws))

    @staticmethod
    def bytes_for(n_gauss, max_jobs, max_pixels, max_tiles, capacity):
        """nbytes() of an arena of these sizes, without allocating it."""
        R = n_gauss * max_jobs
        return (R * (gs.REC_WORDS * 4 + gs.META_WORDS * 4 + 4) + max_tiles * 8 + (max_tiles + 4) * 4
                + max_pixels * 20 + capacity * 4 + int(gs.lib.gs_bin_sort_workspace_size(R, capacity, max_tiles)))

    @property
    def bins(self) -> gs.GsBins:
        return gs.GsBins(self.vals.data_ptr(), self.ranges.data_ptr(), self.pair_off.data_ptr(),
                         self.counters.data_ptr(), self.capacity, self.tile_order.data_ptr())


class Slot:
    def __init__(self, arena: Arena):
        self.arena = arena
        self.stream = torch.cuda.Stream()      # default priority
        self.event = None
        self.batch = None
        self.frame = None


class RenderServer:
    MAX_TRIES = 4      # overflowing launches of one request before the server gives up

    def __init__(self, params: torch.Tensor, cfg: gs.GsRasterCfg, hbm_budget: float = 32e9, n_slots: int = 3,
                 max_batch: int = 16, resolutions=None, pair_headroom: float = 1.5, spatial_order: bool = True):
        """params: global model [A][G] resident on the GPU.  The HBM budget
        (bytes, transient buffers only) is split over n_slots arenas.
        spatial_order: serve a copy of the model stored in Z-order of the
        means (gs_spatial_order), so that what a view sees forms long runs
        in memory; images are the same except between Gaussians of equal
        depth bits."""
        self.perm = None
        if spatial_order:
            self.perm = torch.from_numpy(gs.spatial_order(params)).to(params.device)
            params = params.index_select(1, self.perm).contiguous()
        self.params, self.cfg = params, cfg
        self.device = params.device
        self.G = params.shape[1]
        self.resolutions = list(resolutions or [(1920, 1080)])
        self.pairs_per_px = self._calibrate_pairs(pair_headroom)
        max_px = max(w * h for w, h in self.resolutions)
        tw, th = cfg.tile_w, cfg.tile_h
        max_tiles_view = max(((w + tw - 1) // tw) * ((h + th - 1) // th) for w, h in self.resolutions)
        slot_budget = hbm_budget / n_slots
        # the largest batch whose arena fits one slot's share (at least one view)
        cap_of = lambda b: int(self.pairs_per_px * max_px * b) + 4096  # noqa: E731
        b = max(1, int(max_batch))
        while b > 1 and Arena.bytes_for(self.G, b, max_px * b, max_tiles_view * b, cap_of(b)) > slot_budget:
            b -= 1
        self.max_batch = b
        cap = cap_of(b)
        self.slots = [Slot(Arena(self.G, self.max_batch, max_px * self.max_batch, max_tiles_view * self.max_batch,
                                 cap, self.device)) for _ in range(n_slots)]
        self.queue = []
        self.finished = []
        self.retries = 0
        self.largest_batch = 0        # most requests in one launched batch
        self.most_in_flight = 0       # most slots holding a batch at one time
        self.pool = {}
        # pre-fill the pinned pool for requests in flight (it grows on demand)
        for w, h in self.resolutions:
            for _ in range(min(8, n_slots * self.max_batch)):
                self.pool.setdefault((w, h), []).append(
                    torch.empty((3, h, w), dtype=torch.float32).pin_memory())

    # -- sizing ---------------------------------------------------------
    def _calibrate_pairs(self, headroom):
        """Tile pairs per pixel at each served resolution (one render each,
        on a ring view), with headroom."""
        from .scenes import look_at
        worst = 0.0
        for w, h in self.resolutions:
            cam = look_at([40.0, 10.0, 0.0], [0, 0, 0], w, h)
            f = gs.Frame([cam], [gs.JobSpec(0, 0, self.G, 1.0)], self.cfg, self.device)
            buf = gs.rasterize(self.params, f, self.cfg, capacity=4 * w * h)
            worst = max(worst, gs.read_counters(buf)["pairs"] / (w * h))
            del buf
        torch.cuda.synchronize()
        return worst * headroom

    # -- serving --------------------------------------------------------
    def _pinned(self, cam):
        key = (cam.width, cam.height)
        pool = self.pool.setdefault(key, [])
        if pool:
            return pool.pop()
        return torch.empty((3, cam.height, cam.width), dtype=torch.float32).pin_memory()

    def release(self, r: Request):
        """Return a finished request's pinned buffer to the pool."""
        if r.image is not None:
            self.pool.setdefault((r.cam.width, r.cam.height), []).append(r.image)
            r.image = None

    def submit(self, rid, cam, arrival):
        r = Request(rid, cam, arrival)
        self.queue.append(r)
        return r

    def _launch(self, slot: Slot, batch, now):
        a = slot.arena
        cams = [r.cam for r in batch]
        jobs = [gs.JobSpec(i, 0, self.G, 1.0) for i in range(len(batch))]
        with torch.cuda.stream(slot.stream):
            f = gs.Frame(cams, jobs, self.cfg, self.device)
            a.frame = f
            a.counters.zero_()
            gs.project(self.params, f, self.cfg, a)
            gs.bin_sort(f, self.cfg, a)
            gs.render_fwd(f, self.cfg, a)
            for i, r in enumerate(batch):
                r.image = self._pinned(r.cam)
                r.image.copy_(f.image(a.rgb, i), non_blocking=True)
            a.counters_host.copy_(a.counters, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        for r in batch:
            r.started = now
        slot.batch, slot.event, slot.frame = batch, ev, f
        self.largest_batch = max(self.largest_batch, len(batch))
        self.most_in_flight = max(self.most_in_flight, sum(s.batch is not None for s in self.slots))

    def _admit(self, slot: Slot):
        """Greedy admission of waiting requests into the slot's arena.  A
        request whose pair estimate alone exceeds the arena (the estimate
        grows after an overflow) gets the arena's pair buffers grown for it
        and is launched alone."""
        a = slot.arena
        batch, px = [], 0
        for r in self.queue:
            if len(batch) >= self.max_batch or px + r.pixels > a.max_pixels:
                break
            if self.pairs_per_px * (px + r.pixels) > a.capacity:
                if batch:
                    break
                a.grow_pairs(int(self.pairs_per_px * r.pixels) + 4096)
                batch.append(r)
                break
            batch.append(r)
            px += r.pixels
        del self.queue[:len(batch)]
        return batch

    def poll(self, now):
        """Retire finished batches, then fill free slots from the queue."""
        for s in self.slots:
            if s.batch is not None and s.event.query():
                st = int(s.arena.counters_host[gs.CTR_STATUS].item())
                if st & gs.GS_STATUS_PAIR_OVERFLOW:
                    # more pairs than budgeted: raise the pairs-per-pixel
                    # estimate to what this batch needed, so that admission
                    # makes the batch smaller (or grows the arena for a
                    # single request), and put the batch back in front
                    self.retries += 1
                    need = int(s.arena.counters_host[gs.CTR_PAIRS].item()) & 0xFFFFFFFF
                    px = sum(r.pixels for r in s.batch)
                    self.pairs_per_px = max(self.pairs_per_px, 1.1 * need / px)
                    for r in s.batch:
                        self.release(r)
                        r.tries += 1
                        if r.tries > self.MAX_TRIES:
                            raise RuntimeError(f"request {r.rid} overflowed its pair budget {r.tries} times "
                                               f"({need} pairs needed)")
                    self.queue[:0] = s.batch
                else:
                    t = time.perf_counter()
                    for r in s.batch:
                        r.done = t
                    self.finished.extend(s.batch)
                s.batch, s.event = None, None
        for s in self.slots:
            if s.batch is None and self.queue:
                batch = self._admit(s)
                if batch:
                    self._launch(s, batch, now)

    def idle(self):
        return not self.queue and all(s.batch is None for s in self.slots)

    def run_open_loop(self, cams, arrivals, warmup=0.0, keep=()):
        """Serve requests arriving at the given times (seconds from start).
        Returns latency / throughput statistics over requests arriving after
        ``warmup``; the images of request ids in ``keep`` are kept (copied out
        of the pinned pool), all others are released when done."""
        keep = set(keep)
        self.kept = {}
        t0 = time.perf_counter()
        nxt = 0
        reqs = []
        n_done = 0
        while nxt < len(arrivals) or not self.idle():
            now = time.perf_counter() - t0
            while nxt < len(arrivals) and arrivals[nxt] <= now:
                r = self.submit(nxt, cams[nxt], t0 + arrivals[nxt])
                reqs.append(r)
                nxt += 1
            self.poll(now)
            for r in self.finished[n_done:]:
                if r.rid in keep:
                    self.kept[r.rid] = r.image.clone()
                self.release(r)
            n_done = len(self.finished)
            if self.idle() and nxt < len(arrivals):
                time.sleep(max(0.0, min(1e-3, arrivals[nxt] - (time.perf_counter() - t0))))
        t_end = time.perf_counter()
        meas = [r for r in reqs if r.arrival - t0 >= warmup]
        lat = np.array([(r.done - r.arrival) * 1e3 for r in meas])
        span = max(r.done for r in meas) - min(r.arrival for r in meas)
        px = sum(r.pixels for r in meas)
        return {"requests": len(meas), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "frames_per_s": len(meas) / span, "mpx_per_s": px / span / 1e6,
                "wall_s": t_end - t0, "retries": self.retries, "max_batch": self.max_batch,
                "slots": len(self.slots), "largest_batch": self.largest_batch,
                "most_in_flight": self.most_in_flight}, reqs

    def render_alone(self, cam):
        """Render one view by itself (reference for the batching check)."""
        f = gs.Frame([cam], [gs.JobSpec(0, 0, self.G, 1.0)], self.cfg, self.device)
        buf = gs.rasterize(self.params, f, self.cfg, capacity=int(self.pairs_per_px * cam.width * cam.height) + 4096)
        return f.image(buf.rgb, 0).cpu()
