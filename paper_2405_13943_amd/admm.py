"""Batched K-block ADMM training on one GPU (Alg. 2, Eq. 8a-c).

The K blocks the paper spreads over compute nodes live together in one
GPU's HBM: the local copies of all blocks form one parameter store
(block k owns the contiguous range [off_k, off_k + n_k)), and every stage of
a local step is one launch over all blocks (one render job per block).
Every ``intv`` steps (after the local step, including t = 0, as Alg. 2
writes it) the consensus step averages the copies of each global Gaussian
over the blocks that hold it (``gs_consensus``); the duals start at zero.
With an ``AdaptivePenalty`` the per-group rho follows the primal and dual
residuals of each consensus (Sec. 3.3, ``gs_penalty_update``), the scaled
duals are rescaled with it (``gs_dual_rescale``), and the adjustment stops
after a fixed iteration.

Everything here is orchestration: device buffers come from torch, every
arithmetic step runs in libgs.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np
import torch

from . import gs

DEFAULT_LR = (1.6e-4, 1e-3, 5e-3, 2.5e-3, 5e-2)    # mean, rotation, scale, SH, opacity


@dataclass(frozen=True)
class AdaptivePenalty:
    """Residual balancing of Sec. 3.3: mu > 1 and the factors tau_inc,
    tau_dec (the paper leaves their values open; these are the usual ones of
    the scheme it adopts), applied at every consensus before iteration
    ``until`` (2000 in the paper's experiments)."""
    mu: float = 10.0
    tau_inc: float = 2.0
    tau_dec: float = 2.0
    until: int = 2000


def holder_csr(local_gid, n_global, local_index=None):
    """Holder CSR of the global ids: for each global id, the local indices of
    its copies in ascending block order (blocks are laid out in order).
    ``local_index[k]`` gives the store column of each of block k's copies
    (default: blocks back to back without padding)."""
    gid = np.concatenate(local_gid)
    if local_index is None:
        cols = np.arange(len(gid), dtype=np.int64)
    else:
        cols = np.concatenate(local_index)
    order = np.argsort(gid, kind="stable")          # stable: ascending block within a gid
    counts = np.bincount(gid, minlength=n_global)
    ptr = np.zeros(n_global + 1, np.int64)
    np.cumsum(counts, out=ptr[1:])
    return ptr, cols[order].astype(np.int64)


def split_cameras(boxes, cams, scale=1.4, ground_axes=(0, 2)):
    """Per block, the views whose centres its cell box, scaled by ``scale``,
    covers in the ground plane (Sec. 3.2: views are split with the points)."""
    centres = np.stack([-np.asarray(c.R, np.float64).T @ np.asarray(c.t, np.float64) for c in cams])
    groups = gs.split_group(boxes, scale, centres, ground_axes)
    return [[cams[i] for i in g] for g in groups]


def holder_order(local_gid, n_global, within=None):
    """Numbering of the global ids grouped by holder set: ids held by the
    same blocks become consecutive, groups ordered by (first holder, number
    of holders, holder set), inside a group by ``within`` (a rank per
    original id; default the original order), ids held by no block last.
    Returns (perm, inv): new id j is original id perm[j]; original id i
    becomes inv[i].

    With every block's copies stored in this order, the copies of one
    holder group are consecutive columns in each of its blocks, so the
    consensus streams dense lines: no wavefront mixes single-held and shared
    ids, and the duals of single-held ids (which never change) are never
    written between shared ones."""
    K = len(local_gid)
    if K > 63:
        raise ValueError("holder_order supports up to 63 blocks")
    mask = np.zeros(n_global, np.uint64)
    for k, g in enumerate(local_gid):
        mask[np.asarray(g, np.int64)] |= np.uint64(1 << k)
    count = np.zeros(n_global, np.int64)
    first = np.full(n_global, K, np.int64)
    for k in range(K - 1, -1, -1):
        bit = (mask >> np.uint64(k)) & np.uint64(1)
        count += bit.astype(np.int64)
        first[bit.astype(bool)] = k
    inner = np.arange(n_global) if within is None else np.asarray(within, np.int64)
    perm = np.lexsort((inner, mask, count, first)).astype(np.int64)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(n_global, dtype=np.int64)
    return perm, inv


@dataclass
class BlockModel:
    """Local copies of K blocks in one store plus the global model."""
    sh_degree: int
    z: torch.Tensor                   # [A][G] global model
    x: torch.Tensor                   # [A][L] local copies, blocks back to back
    offsets: list                     # block k's slot: [offsets[k], offsets[k+1]), 64-column aligned
    holder_ptr: torch.Tensor          # [G+1] int64
    holder_idx: torch.Tensor          # [H] int64 local indices
    local_gid: list = field(default_factory=list)   # per block: global ids (store numbering) of its columns
    ends: list = None                 # block k's copies: [offsets[k], ends[k])
    perm: np.ndarray = None           # store id j is the caller's global id perm[j] (None: identity)

    @classmethod
    def from_global(cls, params_global: np.ndarray, local_gid, device="cuda", align=64, group_holders=True,
                    spatial_strands=0):
        """Local copies of each block start on a multiple of ``align``
        columns (16-byte aligned slices for per-block streaming); the padding
        columns belong to no block and no holder set.  With
        ``group_holders`` the global ids are renumbered by holder set
        (``holder_order``) and each block's copies stored in that order;
        ``global_params`` returns z in the caller's order.  With
        ``spatial_strands`` > 0 the ids inside a holder group follow the
        Z-order of their means in 16-Gaussian chunks dealt over that many
        strands (``gs.spatial_order``; a storage layout)."""
        A, G = params_global.shape
        deg = gs.sh_degree_of(A)
        perm = None
        if group_holders:
            within = None
            if spatial_strands > 0:
                order = gs.spatial_order(params_global[0:3], chunk=16, strands=int(spatial_strands))
                within = np.empty(G, np.int64)
                within[order] = np.arange(G, dtype=np.int64)
            perm, inv = holder_order(local_gid, G, within)
            params_global = params_global[:, perm]
            local_gid = [np.sort(inv[np.asarray(g, np.int64)]) for g in local_gid]
        z = torch.from_numpy(np.ascontiguousarray(params_global)).to(device)
        offs, col_gid, base = [], [], 0
        for g in local_gid:
            offs.append(base)
            n = len(g)
            pad = (-n) % align
            col_gid.append(np.asarray(g, np.int64))
            if pad:
                col_gid.append(np.full(pad, int(g[0]) if n else 0, np.int64))
            base += n + pad
        offs.append(base)
        x = z.index_select(1, torch.from_numpy(np.concatenate(col_gid)).to(device)).contiguous()
        local_index = [np.arange(offs[k], offs[k] + len(local_gid[k]), dtype=np.int64) for k in range(len(local_gid))]
        ptr, idx = holder_csr(local_gid, G, local_index)
        ends = [offs[k] + len(local_gid[k]) for k in range(len(local_gid))]
        return cls(deg, z, x, offs[:-1] + [offs[-1]], torch.from_numpy(ptr).to(device),
                   torch.from_numpy(idx).to(device), [np.asarray(g) for g in local_gid], ends, perm)

    @classmethod
    def from_split(cls, params_global: np.ndarray, K: int, scale=1.4, ground_axes=(0, 2), device="cuda", align=64,
                   spatial_strands=0):
        """K blocks from the scene itself (Alg. 1 on the Gaussian means, then
        the overlap grouping with factor ``scale``; the paper uses 1.4):
        returns (model, cell boxes [K][6], per-block global ids in the
        caller's numbering)."""
        pts = np.ascontiguousarray(params_global[0:3].T, dtype=np.float64)
        boxes, _ = gs.split_scene(pts, K, ground_axes)
        groups = gs.split_group(boxes, scale, pts)
        return (cls.from_global(params_global, groups, device=device, align=align, spatial_strands=spatial_strands),
                boxes, groups)

    @property
    def K(self):
        return len(self.offsets) - 1

    def global_params(self) -> torch.Tensor:
        """The global model z with columns in the caller's global-id order."""
        if self.perm is None:
            return self.z
        out = torch.empty_like(self.z)
        out[:, torch.from_numpy(self.perm).to(self.z.device)] = self.z
        return out

    def block(self, k):
        """Store columns of block k's copies."""
        end = self.ends[k] if self.ends is not None else self.offsets[k + 1]
        return self.offsets[k], end


class AdmmTrainer:
    """One view per block per step, all K blocks in one launch per stage."""

    def __init__(self, model: BlockModel, cams, targets, cfg: gs.GsRasterCfg, lr=DEFAULT_LR, rho=(1e-3,) * 5,
                 intv=100, relax=1.0, beta1=0.9, beta2=0.999, eps=1e-8, capacity=None, mask=None, fused=True,
                 adaptive: AdaptivePenalty | None = None, lambda_ssim=0.0):
        """cams[k]: list of cameras of block k; targets[k][v]: device tensor
        [3*H*W] (or a callable (k, v) -> tensor) for block k, view v.
        fused: backward and optimiser in one call (gs_render_bwd_adam, the
        gradient never stored); else gs_render_bwd into a gradient buffer,
        then gs_adam_admm.  relax: over-relaxation alpha of the consensus
        (1: none; the paper uses 1.5-1.8).  adaptive: residual-balancing
        penalty (one host read of the residual sums per consensus while it
        is active).  lambda_ssim: weight of the D-SSIM term of Eq. 3 (0: the
        L1 term alone, fused into the backward)."""
        self.model, self.cfg = model, cfg
        self.lr, self.rho, self.intv, self.relax = tuple(lr), tuple(rho), int(intv), float(relax)
        self.beta1, self.beta2, self.eps = beta1, beta2, eps
        self.mask = mask
        x = model.x
        self.m = torch.zeros_like(x)
        self.v = torch.zeros_like(x)
        self.u = torch.zeros_like(x)
        # w = z - u with u = 0: the consensus target of every local copy
        self.w = x.clone()
        self.fused = fused
        self.g = None
        self.t = 0
        self.cams = cams
        self.targets = targets
        self.n_views = min(len(c) for c in cams)
        self._frames = {}
        self.buf = None
        self.capacity = capacity
        self.loss = torch.zeros(model.K, device=x.device)
        self.adaptive = adaptive
        self.lambda_ssim = float(lambda_ssim)
        self._dl = self._ssim_ws = None
        self.resid = torch.zeros(10, device=x.device)
        self.redone = 0          # local steps redone after pair-capacity overflows
        self.history = []        # (t, residual sums, rho after the update) per adaptive consensus

    # -- frames ----------------------------------------------------------
    def frame(self, views):
        """Frame with one job per block, block k rendering views[k]."""
        key = tuple(views)
        if key not in self._frames:
            cams, jobs = [], []
            for k, v in enumerate(views):
                a, b = self.model.block(k)
                cams.append(self.cams[k][v])
                jobs.append(gs.JobSpec(k, a, b, 1.0))
            self._frames[key] = gs.Frame(cams, jobs, self.cfg, self.model.x.device)
        return self._frames[key]

    def views_at(self, t):
        return [t % self.n_views] * self.model.K

    def target_buffer(self, views):
        parts = []
        for k, v in enumerate(views):
            tg = self.targets(k, v) if callable(self.targets) else self.targets[k][v]
            parts.append(tg.reshape(-1))
        return torch.cat(parts) if len(parts) > 1 else parts[0]

    # -- steps -----------------------------------------------------------
    def _buffers(self, f):
        if self.buf is None or self.buf.frame.n_records != f.n_records or self.buf.frame.n_pixels != f.n_pixels \
                or self.buf.frame.n_tiles != f.n_tiles:
            cap = self.capacity or max(1 << 20, 4 * f.n_records)
            self.buf = gs.Buffers(f, cap, self.model.x.dtype, self.model.x.device)
        self.buf.frame = f
        return self.buf

    def local_step(self, views=None, target=None):
        """One x-update step (Eq. 8a) for every block at once."""
        views = self.views_at(self.t) if views is None else views
        f = self.frame(views)
        buf = self._buffers(f)
        x = self.model.x
        gs.project(x, f, self.cfg, buf)
        gs.bin_sort(f, self.cfg, buf)
        gs.render_fwd(f, self.cfg, buf)
        tgt = self.target_buffer(views) if target is None else target
        self.loss.zero_()
        acfg = gs.adam_cfg(self.lr, self.rho, self.t + 1, self.beta1, self.beta2, self.eps)
        mode, gin, loss = gs.LOSS_L1, tgt, self.loss
        if self.lambda_ssim > 0:
            n = 3 * f.n_pixels
            if self._dl is None or self._dl.numel() < n:
                self._dl = torch.empty(n, device=x.device)
                self._ssim_ws = torch.empty(int(gs.lib.gs_ssim_workspace_size(f.n_pixels)), dtype=torch.uint8,
                                            device=x.device)
            gs.ssim_loss_grad(f, self.cfg, buf.rgb, tgt, self.lambda_ssim, grad_out=self._dl, loss_out=self.loss,
                              ws=self._ssim_ws)
            mode, gin, loss = gs.LOSS_EXTERNAL, self._dl, None
        if self.fused and f.jobs_disjoint:
            gs.render_bwd_adam(x, f, self.cfg, buf, self.m, self.v, self.w, self.mask, acfg, mode, gin, loss)
        else:
            if self.g is None:
                self.g = torch.empty_like(x)
            gs.render_bwd(x, f, self.cfg, buf, self.g, mode, gin, loss)
            gs.adam_admm(x, self.g, self.m, self.v, self.w, self.mask, acfg, status=buf)

    def consensus(self):
        """z = mean of holders' copies; u += x - z; w = z - u (Eq. 8b-c);
        then, while the adaptive penalty is active, the rho update and the
        matching rescale of the scaled duals (Sec. 3.3)."""
        self.resid.zero_()
        mdl = self.model
        gs.consensus(mdl.x, self.u, self.w, mdl.z, mdl.holder_ptr, mdl.holder_idx, self.relax, self.resid)
        ap = self.adaptive
        if ap is not None and self.t < ap.until:
            res = self.resid.cpu().tolist()
            rho, scale = gs.penalty_update(res, self.rho, ap.mu, ap.tau_inc, ap.tau_dec)
            if any(f != 1.0 for f in scale):
                gs.dual_rescale(self.u, self.w, mdl.z, mdl.holder_ptr, mdl.holder_idx, scale)
            self.rho = rho
            self.history.append((self.t, res, rho))

    def step(self):
        """Alg. 2: local step for all blocks, then consensus when t mod intv
        == 0.  Before a consensus reads x, the device counters are checked
        once and steps skipped after a pair-capacity overflow are redone, so
        a consensus never sees a block behind its step count."""
        self.local_step()
        if self.t % self.intv == 0:
            self.check()
            self.consensus()
        self.t += 1

    MAX_REGROW = 8

    def check(self):
        """Read the device counters once.  After a pair-capacity overflow the
        device skipped the optimiser update of the overflowing step and of
        every step after it (the status bit is sticky; counters[OVERFLOWED]
        counts them), so x, m and v are exactly as they were before the
        first of them.  Grow the pair buffers to what was needed, clear the
        status and redo those steps (their views follow from the step
        index).  Returns the number of steps redone."""
        redone = 0
        for _ in range(self.MAX_REGROW):
            c = gs.read_counters(self.buf)
            if c["status"] & gs.GS_STATUS_NONFINITE:
                raise FloatingPointError(f"non-finite parameter or optimiser state before step {self.t + 1}")
            if not c["status"] & gs.GS_STATUS_PAIR_OVERFLOW:
                return redone
            skipped = c["overflowed"]
            self.capacity = max(int(c["pairs"] * 1.3) + 4096, self.buf.capacity)
            self.buf.grow(self.capacity)
            self.buf.counters.zero_()
            t_now = self.t
            for t in range(t_now - skipped + 1, t_now + 1):
                self.t = t
                self.local_step()
                redone += 1
                self.redone += 1
            self.t = t_now
        raise RuntimeError("pair capacity still overflowing after growing the buffers")

    def calibrate(self, headroom=1.3):
        """Size the pair capacity from every view combination once (untimed)."""
        pmax = 0
        for v in range(self.n_views):
            views = [v] * self.model.K
            f = self.frame(views)
            buf = self._buffers(f)
            gs.rasterize(self.model.x, f, self.cfg, buf)
            pmax = max(pmax, gs.read_counters(buf)["pairs"])
        self.capacity = int(pmax * headroom) + 4096
        self.buf.grow(self.capacity)
        self.buf.counters.zero_()
        return pmax


# ---------------------------------------------------------------------------
# tile-shape autotuner

# (binning tile w, h, forward and backward compositing wavefronts per tile;
# -1: per tile from its list length)
TILES = ((16, 16, -1, -1), (32, 8, -1, -1), (16, 16, 2, 1), (16, 16, 2, -1), (16, 16, -1, 1), (32, 8, 2, 1),
         (16, 8, -1, -1), (8, 8, 1, 1))


def autotune_tile(run_step, key: str, cache_path=None, candidates=TILES, reps=5):
    """The fastest launch shape for ``run_step(tile)`` (one full training step
    with that tile shape) from libgs's tuner (gs_autotune: HIP-event timing
    of each candidate on the current stream, choices cached per workload key,
    in ``cache_path`` when given)."""
    if cache_path:
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
    gs.set_tune_cache(cache_path)
    best, _ = gs.autotune(key, candidates, run_step, reps)
    return tuple(best)


# ---------------------------------------------------------------------------
# blocks on concurrent streams

def contiguous_groups(sizes, n_groups):
    """Split blocks 0..K-1 into n_groups contiguous runs of similar total
    size (the largest run as small as possible; exhaustive over the cut
    points, K is small).  Returns [(k0, k1), ...]."""
    import itertools
    K = len(sizes)
    n_groups = max(1, min(int(n_groups), K))
    best, best_cost = None, None
    for cuts in itertools.combinations(range(1, K), n_groups - 1):
        edges = (0,) + cuts + (K,)
        cost = max(sum(sizes[a:b]) for a, b in zip(edges[:-1], edges[1:]))
        if best_cost is None or cost < best_cost:
            best, best_cost = edges, cost
    return [(a, b) for a, b in zip(best[:-1], best[1:])]


class StreamedAdmmTrainer:
    """Alg. 2 with the K blocks in contiguous groups, each group's local step
    on a HIP stream of its own (one launch per stage per group), so that one
    group's compositing (bound by vector ALU issue) and another group's
    streaming optimiser (bound by HBM) run on the device at the same time.
    The consensus runs on the calling stream after every group's stream has
    reached it; the groups' next steps wait for it.  The parameter store,
    optimiser state, duals and consensus targets are one set of tensors
    (each group works on its columns); results are those of AdmmTrainer."""

    def __init__(self, model: BlockModel, cams, targets, cfg: gs.GsRasterCfg, groups=2, capacity=None, **kw):
        self.model = model
        self.full = AdmmTrainer(model, cams, targets, cfg, capacity=capacity, **kw)
        sizes = [model.block(k)[1] - model.block(k)[0] for k in range(model.K)]
        self.parts = contiguous_groups(sizes, groups)
        self.subs = []
        for k0, k1 in self.parts:
            lo, hi = model.offsets[k0], model.offsets[k1]
            ends = model.ends if model.ends is not None else model.offsets[1:]
            sub_model = BlockModel(model.sh_degree, model.z, model.x[:, lo:hi],
                                   [o - lo for o in model.offsets[k0:k1 + 1]], model.holder_ptr, model.holder_idx,
                                   model.local_gid[k0:k1], [e - lo for e in ends[k0:k1]], model.perm)
            if callable(targets):
                tg = (lambda f, a: (lambda k, v: f(k + a, v)))(targets, k0)
            else:
                tg = targets[k0:k1]
            sub = AdmmTrainer(sub_model, cams[k0:k1], tg, cfg, capacity=capacity, **kw)
            # the group's columns of the shared state
            sub.m, sub.v = self.full.m[:, lo:hi], self.full.v[:, lo:hi]
            sub.u, sub.w = self.full.u[:, lo:hi], self.full.w[:, lo:hi]
            if sub.mask is not None:
                sub.mask = self.full.mask[lo:hi]
            sub.stream = torch.cuda.Stream(device=model.x.device)
            self.subs.append(sub)
        self.intv = self.full.intv
        self.t = 0

    @property
    def cfg(self):
        return self.full.cfg

    @property
    def capacity(self):
        return max(s.capacity or 0 for s in self.subs)

    def calibrate(self, headroom=1.3):
        pm = []
        for s in self.subs:
            with torch.cuda.stream(s.stream):
                pm.append(s.calibrate(headroom))
        torch.cuda.synchronize()
        return max(pm)

    def local_step(self):
        ev = torch.cuda.Event()
        ev.record()
        for s in self.subs:
            s.stream.wait_event(ev)
            s.t = self.t
            s.rho = self.full.rho
            with torch.cuda.stream(s.stream):
                s.local_step()

    def join(self):
        """The calling stream waits for every group's queued work."""
        cur = torch.cuda.current_stream()
        for s in self.subs:
            ev = torch.cuda.Event()
            ev.record(s.stream)
            cur.wait_event(ev)

    def consensus(self):
        self.join()
        self.full.t = self.t
        self.full.consensus()

    def check(self):
        redone = 0
        for s in self.subs:
            with torch.cuda.stream(s.stream):
                s.t = self.t
                redone += s.check()
        return redone

    def step(self):
        self.local_step()
        if self.t % self.intv == 0:
            self.check()
            self.consensus()
        self.t += 1

    def synchronize(self):
        self.join()

    @property
    def bufs(self):
        return [s.buf for s in self.subs]

    @property
    def resid(self):
        return self.full.resid

    @property
    def history(self):
        return self.full.history
