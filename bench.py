"""Benchmark: training steps/s of the per-block rasterizer step at scale.

Workload (one block): 500k Gaussians, SH degree 3, 64 ring cameras at
1600x1066 on a 40 m ring at 10 m height; one view per step (view = step mod
64); L1 loss against a seeded U(0,1) target; Adam with the ADMM penalty
(rho = 1e-3 on every group, dense).  A step is

    gs_project -> gs_bin_sort -> gs_render_fwd -> gs_render_bwd -> gs_adam_admm

with all inputs resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-serve] [--no-blocks4]

The default line also carries a serving leg (``serve``): the 6M-Gaussian
global model under Poisson requests at 200 req/s over mixed resolutions,
p50/p99 latency and frames/s, and 50 sampled requests rendered again alone
(bit-equal to their images from the mix); and a short K = 4 block leg
(``blocks4``): the batched step against the four blocks stepped one after
another, with the images-equal check.  ``--workload blocks4`` instead prints the
batched K = 4 block line (batched against sequential per-block steps) and
``--workload serve`` the serving leg alone.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
# VALU operations per (pixel, Gaussian) evaluation up to each pixel's
# termination, and per visible Gaussian, that bound the compositing and
# projection kernels from below (an exp counted as 4)
FWD_OPS = 25
BWD_OPS = 70
PROJ_OPS = 150
PROJ_BWD_OPS = 400
ADAM_OPS = 15            # per parameter
ORDER_STRANDS = 1024     # strands of the default training storage order (see setup)
LR = (1.6e-4, 1e-3, 5e-3, 2.5e-3, 5e-2)       # mean, rotation, scale, SH, opacity
RHO = (1e-3,) * 5


# sources each measured kernel's code comes from: its translation unit and the
# device headers it includes; of the public header only the type and constant
# definitions count (declarations of other entry points do not change a kernel)
KERNEL_SOURCES = {
    "k_project_bwd_adam": ("project.hip", "adam.hpp", "gs_device.hpp"),
    "k_render_bwd": ("render.hip", "gs_device.hpp"),
    "k_consensus": ("optim.hip", "adam.hpp", "gs_device.hpp"),
    "k_adam_admm": ("optim.hip", "adam.hpp", "gs_device.hpp"),
    "k_ssim_fwd": ("ssim.hip", "gs_device.hpp"),
    "k_ssim_bwd": ("ssim.hip", "gs_device.hpp"),
}


def _header_definitions():
    """The typedefs (structs, enums) and #defines of include/gs.h, in order."""
    import re
    with open(os.path.join(ROOT, "include", "gs.h")) as fh:
        text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
    defs = re.findall(r"typedef\s+(?:struct|enum)\s*\{.*?\}\s*\w+\s*;", text, flags=re.S)
    defs += re.findall(r"^#define\s+GS_\w+.*$", text, flags=re.M)
    return "\n".join(" ".join(d.split()) for d in defs)


def kernel_sources_sha256(kernel):
    """Fingerprint of the sources a kernel's code comes from."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2405_13943_amd", "csrc")
    for f in KERNEL_SOURCES[kernel]:
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    h.update(_header_definitions().encode())
    return h.hexdigest()


def measured_traffic(kernel, workload=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE / WRITE_SIZE scaled by a copy of known size), or None
    when the kernel's sources have changed since those counters were taken,
    or when `workload` is given and the counters were taken on another."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(kernel)
    if not rec or rec.get("kernel_sources_sha256") != kernel_sources_sha256(kernel):
        return None
    if workload is not None and rec.get("workload") != workload:
        return None
    return int(rec["traffic_bytes_per_launch"])


def train_workload_label(order):
    """Name of the default training workload in the traffic records."""
    return ("plain single block, 500k Gaussians SH3, 1600x1066, 16x16 tiles, wavefronts per tile from list length "
            f"(forward and backward), storage order {order}")


def _counter_per_dispatch(csv_dir, kernel, counter):
    """Mean value of a rocprofv3 counter over a kernel's dispatches (KiB)."""
    import csv
    import glob
    vals = []
    for path in glob.glob(os.path.join(csv_dir, "*counter_collection.csv")):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                name = r["Kernel_Name"].replace("(anonymous namespace)::", "")
                if r["Counter_Name"] == counter and (kernel is None or f"gs::{kernel}<" in name
                                                     or f"gs::{kernel}(" in name):
                    vals.append(float(r["Counter_Value"]))
    return sum(vals) / len(vals) if vals else None


def record_traffic(kernel, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, workload, commands):
    """Write the kernel's measured HBM bytes per launch into
    profiles/hbm_traffic.json: FETCH_SIZE and WRITE_SIZE (KiB per dispatch,
    one rocprofv3 --pmc run each) scaled so that the copy probe of 1 GiB
    reads and writes exactly 1 GiB."""
    import csv
    import glob

    def copy_value(d, counter):
        best = 0.0
        for path in glob.glob(os.path.join(d, "*counter_collection.csv")):
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]:
                        best = max(best, float(r["Counter_Value"]))
        if best <= 0:
            raise SystemExit(f"no copy-probe {counter} under {d}")
        return best

    gib_kib = float(1 << 20)
    f_scale = round(gib_kib / copy_value(copy_fetch_dir, "FETCH_SIZE"), 2)
    w_scale = round(gib_kib / copy_value(copy_write_dir, "WRITE_SIZE"), 2)
    fk = _counter_per_dispatch(fetch_dir, kernel, "FETCH_SIZE")
    wk = _counter_per_dispatch(write_dir, kernel, "WRITE_SIZE")
    if fk is None or wk is None:
        log(f"[record-traffic] no samples of {kernel}; left as it was")
        return
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    data[kernel] = {
        "workload": workload,
        "kernel_sources_sha256": kernel_sources_sha256(kernel),
        "fetch_size_kib_per_launch": round(fk, 1),
        "write_size_kib_per_launch": round(wk, 1),
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "traffic_bytes_per_launch": int(1024 * (fk * f_scale + wk * w_scale)),
        "copy_probe": f"1 GiB device copy: FETCH_SIZE x{f_scale}, WRITE_SIZE x{w_scale}",
        "commands": commands,
    }
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1)
    print(json.dumps(data[kernel]), flush=True)



def log(msg):
    print(msg, file=sys.stderr, flush=True)


def setup(n, n_cams, width, height, tile, order="generator"):
    import torch
    from paper_2405_13943_amd import gs, scenes
    scene = scenes.config2(n=n, n_cams=n_cams, width=width, height=height)
    if order != "generator":
        # storage layout only (the same Gaussians): Z-order of the means, by
        # default in 16-Gaussian chunks (one 64-byte line of a plane) dealt
        # over ORDER_STRANDS strands, so that a view's culled Gaussians leave
        # whole lines unread while each optimiser workgroup still mixes seen
        # and unseen Gaussians
        strands = ORDER_STRANDS if order == "z-strands" else 1
        perm = gs.spatial_order(scene.params[0:3], chunk=16, strands=strands)
        scene.params = np.ascontiguousarray(scene.params[:, perm])
    cfg = gs.raster_cfg(tile)
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(scene.params).to(dev)
    st = dict(x=x, m=torch.zeros_like(x), v=torch.zeros_like(x), w=x.clone(), g=torch.empty_like(x))
    frames = [gs.Frame(scene.cams, [gs.JobSpec(v, 0, n, 1.0)], cfg) for v in range(n_cams)]
    targets = [torch.from_numpy(t).reshape(-1).to(dev) for t in scenes.config2_targets(scene, range(n_cams))]
    return scene, cfg, st, frames, targets


def calibrate_capacity(gs, st, frames, cfg, headroom=1.3):
    """Largest pair count over the views (host reads; untimed)."""
    buf = gs.Buffers(frames[0], 1 << 22)
    pmax = 0
    for f in frames:
        gs.rasterize(st["x"], f, cfg, buf)
        pmax = max(pmax, gs.read_counters(buf)["pairs"])
    buf.grow(int(pmax * headroom) + 4096)
    return buf, pmax


class StageTimer:
    """HIP events around each call on the launch stream."""

    def __init__(self, torch, names):
        self.torch, self.names = torch, names
        self.ev = {k: [] for k in names}

    def mark(self, name):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.torch.cuda.current_stream())
        self.ev[name].append(e)

    def totals_ms(self):
        out = {}
        for a, b in zip(self.names[:-1], self.names[1:]):
            out[a] = sum(s.elapsed_time(e) for s, e in zip(self.ev[a], self.ev[b]))
        return out


def run_gpu(args):
    import torch
    from paper_2405_13943_amd import gs
    torch.cuda.set_device(0)
    t0 = time.time()
    scene, cfg, st, frames, targets = setup(args.n, args.cams, args.width, args.height,
                                            (args.tile, args.tile, args.fwd_waves, args.bwd_waves), args.order)
    A, N = st["x"].shape
    log(f"[bench] setup {time.time() - t0:.1f}s: N={N} A={A} views={len(frames)} {args.width}x{args.height}")
    buf, pmax = calibrate_capacity(gs, st, frames, cfg)
    log(f"[bench] max pairs over views {pmax}, capacity {buf.capacity}")
    loss = torch.zeros(1, device="cuda")
    buf.counters.zero_()
    lam = args.ssim
    if lam > 0:
        # Eq. 3 with the D-SSIM term: dL/dC from gs_ssim_loss_grad, then the
        # backward takes it as an external gradient
        dl = torch.empty(3 * max(f.n_pixels for f in frames), device="cuda")
        ssim_ws = torch.empty(int(gs.lib.gs_ssim_workspace_size(max(f.n_pixels for f in frames))),
                              dtype=torch.uint8, device="cuda")

    if args.unfused:
        names = ["project", "bin_sort", "render_fwd", "render_bwd", "adam_admm", "end"]
    else:
        names = ["project", "bin_sort", "render_fwd", "render_bwd_adam", "end"]
    if lam > 0:
        names.insert(3, "ssim")

    def step(t, timer=None):
        f = frames[t % len(frames)]
        mark = timer.mark if timer else (lambda _n: None)
        mark("project")
        gs.project(st["x"], f, cfg, buf)
        mark("bin_sort")
        gs.bin_sort(f, cfg, buf)
        mark("render_fwd")
        gs.render_fwd(f, cfg, buf)
        acfg = gs.adam_cfg(LR, RHO, t + 1)
        mode, gin = gs.LOSS_L1, targets[t % len(frames)]
        if lam > 0:
            mark("ssim")
            gs.ssim_loss_grad(f, cfg, buf.rgb, gin, lam, grad_out=dl, loss_out=loss, ws=ssim_ws)
            mode, gin = gs.LOSS_EXTERNAL, dl
        if args.unfused:
            mark("render_bwd")
            gs.render_bwd(st["x"], f, cfg, buf, st["g"], mode, gin, loss)
            mark("adam_admm")
            gs.adam_admm(st["x"], st["g"], st["m"], st["v"], st["w"], None, acfg)
        else:
            mark("render_bwd_adam")
            gs.render_bwd_adam(st["x"], f, cfg, buf, st["m"], st["v"], st["w"], None, acfg, mode, gin, loss)
        mark("end")

    for t in range(args.warmup):
        step(t)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps done")

    # timed region: HIP events bracket the whole loop; inside it the library
    # times the launches of the kernels the rooflines are taken on, with its
    # own HIP events on the launch stream (fused calls hold several kernels),
    # on every PROFILE_STRIDE-th step: each event pair costs the stream a few
    # microseconds, and a stride coprime to the 64 views samples a different
    # view each time.
    # The per-stage split comes from a further untimed run of steps with
    # events between the calls (--inline-stage-timing puts those events in
    # the timed loop instead; each event costs the stream a few microseconds).
    timer = StageTimer(torch, names)
    kernels = ["k_render_bwd", "k_adam_admm" if args.unfused else "k_project_bwd_adam"]
    if lam > 0:
        kernels += ["k_ssim_fwd", "k_ssim_bwd"]
    gs.profile_set(kernels)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    stride = max(1, args.profile_stride)
    e0.record()
    for t in range(args.warmup, args.warmup + args.steps):
        i = t - args.warmup
        gs.profile_enable(i % stride == 0)
        step(t, timer if args.inline_stage_timing else None)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    gs.profile_enable(True)
    kern, kern_n = {}, {}
    for k in kernels:
        tot, n = gs.profile_get(k)
        kern[k] = tot / max(n, 1)
        kern_n[k] = n
    gs.profile_set(None)
    n_stage = args.steps
    if not args.inline_stage_timing:
        n_stage = min(args.steps, 64)
        t0 = args.warmup + args.steps
        for t in range(t0, t0 + n_stage):
            step(t, timer)
        torch.cuda.synchronize()
    # work of the timed views, counted after the timed region on the final
    # parameters: (pixel, Gaussian) contributions and tile pairs per view
    kept = pairs = visible = 0
    nv = min(args.steps, len(frames))
    for t in range(args.warmup, args.warmup + nv):
        f = frames[t % len(frames)]
        gs.project(st["x"], f, cfg, buf)
        gs.bin_sort(f, cfg, buf)
        kept += gs.render_fwd_stats(f, cfg, buf)
        c = gs.read_counters(buf)
        pairs += c["pairs"]
        visible += c["visible"]
    kept, pairs, visible = kept / nv, pairs / nv, visible / nv
    status = gs.read_counters(buf)["status"]
    if status & gs.GS_STATUS_PAIR_OVERFLOW:
        raise SystemExit("pair capacity overflowed during the timed steps; rerun with more headroom")
    log(f"[bench] timed {args.steps} steps: {ms:.2f} ms")
    stage = {k: v / n_stage for k, v in timer.totals_ms().items()}
    log("[bench] per-stage ms: " + ", ".join(f"{k} {v:.4f}" for k, v in stage.items()))

    log("[bench] per-launch kernel ms: " + ", ".join(f"{k} {v:.4f}" for k, v in kern.items()))
    # HBM roofline of the streaming optimiser kernel.  Algorithmic bytes per
    # Gaussian: the two-call path reads x, g, m, v, w and writes x, m, v
    # (8 planes of 4 B); the fused kernel reads x, m, v, w and writes x, m, v
    # (7 planes) plus, per Gaussian, its meta word (16 B), pair offset (4 B)
    # and the nine FP32 partials of each of its tile pairs (36 B per pair).
    if args.unfused:
        opt_kernel, opt_bytes = "k_adam_admm", 32 * A * N
    else:
        opt_kernel, opt_bytes = "k_project_bwd_adam", 28 * A * N + 20 * N + 36 * pairs
    opt_ms = kern[opt_kernel]
    # ALU roofline of the compositing backward: BWD_OPS VALU operations per
    # (pixel, Gaussian) contribution (alpha recomputed, transmittance, colour
    # behind, dL/dalpha, colour and moment accumulations)
    bwd_flops = BWD_OPS * kept
    ssim = None
    if lam > 0:
        # algorithmic bytes of the two SSIM passes per colour value: the
        # forward reads image and target and writes three derivative maps
        # (20 B), the backward reads the maps, image and target and writes
        # dL/dC (24 B)
        px = 3 * args.width * args.height
        ssim_ms = kern["k_ssim_fwd"] + kern["k_ssim_bwd"]
        ssim = {"bound": "hbm", "kernel": "k_ssim_fwd + k_ssim_bwd", "achieved": round(44 * px / (ssim_ms * 1e-3) / 1e9, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(44 * px / (ssim_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "bytes": 44 * px, "ms": round(ssim_ms, 5), "lambda": lam}
        tf, tb = measured_traffic("k_ssim_fwd"), measured_traffic("k_ssim_bwd")
        ssim["traffic"] = tf + tb if tf is not None and tb is not None else None
    return dict(ms_per_step=ms / args.steps, steps=args.steps, stage_ms=stage, kernel_ms=kern, kernel_n=kern_n,
                opt_kernel=opt_kernel,
                ssim=ssim,
                opt_bytes=opt_bytes, opt_gbs=opt_bytes / (opt_ms * 1e-3) / 1e9, pairs_max=pmax, pairs=pairs,
                kept=kept, visible=visible, hw=args.width * args.height, bwd_flops=bwd_flops, bwd_tflops=bwd_flops / (kern["k_render_bwd"] * 1e-3) / 1e12, N=N, A=A,
                scene=scene)


def step_roofline(N, A, V, P, E, HW, ms_per_step, fused=True):
    """Roofline of the whole training step: T_roof = sum over its kernels of
    max(algorithmic HBM bytes / 8 TB/s, VALU operations / 157.3 TFLOP/s),
    against the measured time per step.  Per kernel (V visible records, P
    tile pairs, E (pixel, Gaussian) evaluations up to termination, HW
    pixels):
      project       12 N + 4 (A - 3) V + 52 V bytes      PROJ_OPS V
      pair emission 8 V + 12 P
      tile sort     24 P (one read and one write of the pairs)
      ranges        8 P
      forward       40 P + 20 HW                         FWD_OPS E
      backward      76 P + 44 HW (records, partials)     BWD_OPS E
      projection backward + Adam/ADMM, fused: x, m, v, w read and x, m, v
      written (28 A N), meta and pair offset (20 N), nine partials per pair
      (36 P)                                             PROJ_BWD_OPS V + ADAM_OPS A N
    The two-call form counts the projection backward (4 A V + 36 V + 4 A N)
    and the optimiser (32 A N: the gradient is written and read back)
    separately."""
    bw, alu = HBM_PEAK_GBS * 1e9, FP32_VECTOR_PEAK_TFLOPS * 1e12
    rows = {
        "project": (12 * N + 4 * (A - 3) * V + 52 * V, PROJ_OPS * V),
        "emit": (8 * V + 12 * P, 0.0),
        "sort": (24 * P, 0.0),
        "ranges": (8 * P, 0.0),
        "render_fwd": (40 * P + 20 * HW, FWD_OPS * E),
        "render_bwd": (76 * P + 44 * HW, BWD_OPS * E),
    }
    if fused:
        rows["project_bwd_adam"] = (28 * A * N + 20 * N + 36 * P, PROJ_BWD_OPS * V + ADAM_OPS * A * N)
    else:
        rows["project_bwd"] = (4 * A * V + 36 * V + 4 * A * N, PROJ_BWD_OPS * V)
        rows["adam_admm"] = (32 * A * N, ADAM_OPS * A * N)
    t = {k: max(b / bw, o / alu) for k, (b, o) in rows.items()}
    t_roof = sum(t.values())
    return {"t_roof_ms": round(t_roof * 1e3, 5), "t_measured_ms": round(ms_per_step, 5),
            "frac": round(t_roof * 1e3 / ms_per_step, 4),
            "per_kernel_roof_us": {k: round(v * 1e6, 2) for k, v in t.items()},
            "bytes": int(sum(b for b, _ in rows.values())), "valu_ops": float(sum(o for _, o in rows.values())),
            "counts": {"N": int(N), "A": int(A), "V": round(V), "P": round(P), "E": round(E), "HW": int(HW)}}


def run_serve(args):
    """Serving the global model: 6M Gaussians SH3 resident, Poisson requests at
    ``--rate`` req/s over mixed resolutions, continuous batching; latency is
    arrival -> image landed in pinned host memory."""
    import torch
    from paper_2405_13943_amd import gs, scenes, serve
    t0 = time.time()
    scene = scenes.config5(args.serve_n)
    params = torch.from_numpy(scene.params).to("cuda")
    del scene
    cfg = gs.raster_cfg((args.tile, args.tile, args.fwd_waves, args.bwd_waves))
    srv = serve.RenderServer(params, cfg, hbm_budget=args.serve_hbm * 1e9, n_slots=args.serve_slots,
                             max_batch=args.serve_max_batch, resolutions=scenes.SERVE_RESOLUTIONS)
    log(f"[serve] setup {time.time() - t0:.1f}s: N={params.shape[1]}, max_batch {srv.max_batch}, "
        f"{len(srv.slots)} slots x {srv.slots[0].arena.nbytes() / 1e9:.2f} GB, pairs/px {srv.pairs_per_px:.2f}")
    # warm-up burst (first launches, pinned pool), not measured
    wcams = scenes.serve_requests(24, 55)
    srv.run_open_loop(wcams, np.zeros(len(wcams)))
    torch.cuda.synchronize()
    # open loop at the offered rate; the first seconds are not counted
    warm = args.serve_warmup
    arr = scenes.poisson_arrivals(args.rate, args.serve_seconds + warm, 5005)
    cams = scenes.serve_requests(len(arr), 5006)
    # a seeded sample of the measured requests keeps its image: each is
    # rendered again alone afterwards and must match bit for bit
    measured = np.nonzero(np.asarray(arr) >= warm)[0]
    sample = np.random.default_rng(5008).choice(measured, min(50, len(measured)), replace=False)
    stats, _ = srv.run_open_loop(cams, arr, warmup=warm, keep=[int(i) for i in sample])
    log(f"[serve] open loop {args.rate:.0f} req/s: {stats}")
    n_equal, max_diff = 0, 0.0
    for rid in sample:
        alone = srv.render_alone(cams[int(rid)])
        mixed = srv.kept[int(rid)]
        n_equal += int(torch.equal(alone, mixed))
        max_diff = max(max_diff, float((alone - mixed).abs().max()))
    log(f"[serve] {n_equal} of {len(sample)} sampled requests equal alone and mixed (max diff {max_diff:.3g})")
    # saturation: a burst of requests all arriving at t = 0
    nb = int(args.rate * 2)
    bcams = scenes.serve_requests(nb, 5007)
    sat, _ = srv.run_open_loop(bcams, np.zeros(nb))
    log(f"[serve] burst of {nb}: {sat}")
    out = {"workload": f"global model {params.shape[1] // 1_000_000}M Gaussians SH3, Poisson {args.rate:.0f} req/s "
                       f"over {args.serve_seconds:.0f}s, resolutions uniform over "
                       + ", ".join(f"{w}x{h}" for w, h in scenes.SERVE_RESOLUTIONS),
           "requests": stats["requests"], "p50_ms": round(stats["p50_ms"], 3), "p99_ms": round(stats["p99_ms"], 3),
           "frames_per_s": round(stats["frames_per_s"], 1), "mpx_per_s": round(stats["mpx_per_s"], 1),
           "retries": stats["retries"], "max_batch": srv.max_batch, "slots": len(srv.slots),
           "saturated_frames_per_s": round(sat["frames_per_s"], 1), "saturated_mpx_per_s": round(sat["mpx_per_s"], 1),
           "saturated_p50_ms": round(sat["p50_ms"], 2), "warmup_s": warm,
           "largest_batch": stats["largest_batch"], "most_in_flight": stats["most_in_flight"],
           "sampled_alone_equal": f"{n_equal}/{len(sample)}", "sampled_max_abs_diff": max_diff}
    del srv, params
    torch.cuda.empty_cache()
    return out


KERNELS = ("k_project", "k_fill_u32", "k_scan_reduce", "k_scan_apply", "k_emit", "k_rs_hist", "k_rs_colscan",
           "k_rs_scatter", "k_ranges", "k_tile_sort", "k_tile_sort_long", "k_tile_plan", "k_render_fwd",
           "k_render_bwd", "k_project_bwd_rec", "k_zero_uncovered", "k_project_bwd_adam", "k_adam_uncovered", "k_adam_admm", "k_consensus")


def kernel_breakdown(gs, torch, fn, steps):
    """Per-kernel device time per step (ms) of ``steps`` calls of fn, from the
    library's own HIP events (run outside the timed region)."""
    gs.profile_set("*")
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    out = {}
    for k in KERNELS:
        ms, n = gs.profile_get(k)
        if n:
            out[k] = round(ms / steps, 4)
    gs.profile_set(None)
    return out


def consensus_roofline(model, tr, c_ms, kernels):
    """HBM roofline of the consensus kernel: algorithmic bytes (each held
    local copy's x and u read and w written, u written for Gaussians with
    several holders, z read and written per held global id, the holder CSR
    read once) over its mean launch duration (HIP events around each launch).
    ``call_ms`` is the whole trainer call: with the adaptive penalty it adds
    the host read of the residual sums and the dual rescale."""
    ptr = model.holder_ptr.cpu().numpy()
    cnt = np.diff(ptr)
    A = model.x.shape[0]
    copies = int(cnt.sum())
    multi = int(cnt[cnt > 1].sum())
    g_held = int((cnt > 0).sum())
    # the trainer always asks for the residual sums, so the previous z is read
    planes = 4 * A * (3 * copies + multi + 2 * g_held)
    nbytes = planes + 8 * (len(ptr) + copies)
    k_ms, k_n = kernels["k_consensus"]
    if not c_ms or not k_n:
        return None
    ms = k_ms / k_n
    gbs = nbytes / (ms * 1e-3) / 1e9
    r_ms, r_n = kernels["k_dual_rescale"]
    return {"bound": "hbm", "kernel": "k_consensus", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
            "frac": round(gbs / 8000.0, 4), "bytes": nbytes, "ms": round(ms, 4),
            "call_ms": round(float(np.mean(c_ms)), 4), "dual_rescale_ms": round(r_ms / r_n, 4) if r_n else None,
            "copies": copies, "multi_holder_copies": multi, "held_global": g_held}


def run_consensus(args):
    """The consensus step alone on the K = 4 block store (7.5M global
    Gaussians SH3, 8.25M local copies; global ids numbered by holder set):
    local copies drawn around the global model, then ``--block-steps``
    rounds of gs_consensus with the residual sums (over-relaxation
    ``--relax``), each followed by the penalty update and, when rho moves,
    gs_dual_rescale, as the trainer does before the freeze.  Timed with the
    library's HIP events per kernel."""
    import torch
    from paper_2405_13943_amd import admm, gs, scenes
    t0 = time.time()
    bs = scenes.block_scene(n_cams=1)
    model = admm.BlockModel.from_global(bs.params_global, bs.local_gid)
    del bs
    gen = torch.Generator(device="cuda").manual_seed(7)
    noise = torch.randn(model.x.shape, generator=gen, device="cuda")
    model.x.add_(noise, alpha=1e-2)
    del noise
    u = torch.zeros_like(model.x)
    w = model.x.clone()
    resid = torch.zeros(10, device="cuda")
    rho = RHO
    log(f"[consensus] setup {time.time() - t0:.1f}s: store {tuple(model.x.shape)}, global {model.z.shape[1]}")
    calls = max(2, args.block_steps // 100)
    gs.profile_set(["k_consensus", "k_dual_rescale"])
    torch.cuda.synchronize()
    t1 = time.time()
    rescaled = 0
    for i in range(calls):
        resid.zero_()
        gs.consensus(model.x, u, w, model.z, model.holder_ptr, model.holder_idx, args.relax, resid)
        new, scale = gs.penalty_update(resid, rho)
        if any(f != 1.0 for f in scale):
            gs.dual_rescale(u, w, model.z, model.holder_ptr, model.holder_idx, scale)
            rescaled += 1
        rho = new
        model.x.lerp_(w, 0.5)                      # stand-in for the local steps between rounds
    torch.cuda.synchronize()
    wall = time.time() - t1
    kernels = {k: gs.profile_get(k) for k in ("k_consensus", "k_dual_rescale")}
    gs.profile_set(None)

    class _Tr:
        relax = args.relax
    cons = consensus_roofline(model, _Tr, [1.0], kernels)
    cons.pop("call_ms")
    cons["traffic"] = measured_traffic("k_consensus")
    return {"metric": "consensus rounds/s (z, u, w and residual sums over 8.25M local copies, SH3)",
            "value": kernels["k_consensus"][1] / (kernels["k_consensus"][0] * 1e-3), "unit": "rounds/s",
            "n_gpus": 1, "steps": calls, "warmup": 0, "ms_per_step": kernels["k_consensus"][0] / calls,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (seeded slab blocks, copies = global model + N(0, 0.01))",
            "config": {"workload": "K=4 block store, 7.5M global Gaussians SH3, 8.25M local copies, "
                                   f"relax {args.relax}, residual sums and penalty update every round"},
            "roofline": cons, "rescales": rescaled, "wall_s": round(wall, 3), "final_rho": list(rho)}


def run_split4(args):
    """K = 4 blocks made from the scene (Alg. 1 on 7.5M Gaussian means of uneven
    density, overlap factor ``--split-scale``; views grouped by the same
    boxes): split time and balance, then the batched trainer (adaptive
    penalty and over-relaxation as given, consensus every 100 steps), one view
    per block per step."""
    import torch
    from paper_2405_13943_amd import admm, gs, scenes
    t0 = time.time()
    si = scenes.split_input()
    log(f"[split4] scene {time.time() - t0:.1f}s")
    t1 = time.time()
    model, boxes, groups = admm.BlockModel.from_split(si.params_global, 4, scale=args.split_scale,
                                                      spatial_strands=args.block_strands)
    split_s = time.time() - t1
    cams = admm.split_cameras(boxes, si.cams, scale=args.split_scale)
    K = len(groups)
    sizes = [len(g) for g in groups]
    n_global = si.params_global.shape[1]
    log(f"[split4] split + store {split_s:.1f}s: local {sizes}, views {[len(c) for c in cams]}")
    dev = torch.device("cuda", 0)
    tg = {}

    def target(k, v):
        if (k, v) not in tg:
            c = cams[k][v]
            tg[(k, v)] = torch.from_numpy(scenes.rng(si.seed * 1000 + 100 * k + v).random(
                (3, c.height, c.width)).astype(np.float32)).reshape(-1).to(dev)
        return tg[(k, v)]
    n_views = min(len(c) for c in cams)
    for k in range(K):
        for v in range(n_views):
            target(k, v)
    del si
    tile = (args.tile, args.tile, args.fwd_waves, args.bwd_waves)
    adaptive = admm.AdaptivePenalty() if args.adaptive else None
    tr = admm.AdmmTrainer(model, cams, target, gs.raster_cfg(tile), lr=LR, rho=RHO, intv=100, relax=args.relax,
                          adaptive=adaptive)
    tr.calibrate()
    for _ in range(args.warmup):
        tr.step()
    cons = []
    gs.profile_set(["k_consensus", "k_dual_rescale"])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    steps = args.block_steps
    for _ in range(steps):
        tr.local_step()
        if tr.t % tr.intv == 0:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            tr.consensus()
            b.record()
            cons.append((a, b))
        tr.t += 1
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kernels = {k: gs.profile_get(k) for k in ("k_consensus", "k_dual_rescale")}
    gs.profile_set(None)
    if gs.read_counters(tr.buf)["status"] & gs.GS_STATUS_PAIR_OVERFLOW:
        raise SystemExit("pair capacity overflowed during the timed steps")
    c_ms = [a.elapsed_time(b) for a, b in cons]
    roof = consensus_roofline(model, tr, c_ms, kernels)
    return {"metric": "K-block ADMM train steps/s on Alg. 1 blocks (4 blocks, 1 view each, consensus/100)",
            "value": 1000.0 * steps / ms, "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
            "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic (7.5M Gaussians, 70% uniform + 30% cluster; 8x8 view lattice; U(0,1) "
                                    "targets)",
            "config": {"workload": f"Alg. 1 split of 7.5M Gaussians SH3 into 4 blocks, overlap scale "
                                   f"{args.split_scale}, 1600x1066, consensus every 100 steps",
                       "tile": "x".join(map(str, tile[:2])), "waves_per_tile_fwd_bwd": list(tile[2:]),
                       "relax": args.relax, "adaptive_penalty": bool(args.adaptive),
                       "block_strands": args.block_strands},
            "split_s": round(split_s, 2), "local_copies": sizes, "global": n_global,
            "shared_fraction": round(sum(sizes) / n_global - 1.0, 4),
            "balance_max_over_min": round(max(sizes) / min(sizes), 4),
            "views_per_block": [len(c) for c in cams], "consensus_ms": c_ms, "consensus_roofline": roof}


def run_blocks4(args):
    """K = 4 uneven blocks (0.8M/1.5M/2.2M/3.0M own Gaussians, 10% shared with
    a neighbour), 32 ring views per block at 1600x1066: the batched trainer
    (one launch per stage over all blocks, consensus every 100 steps) against
    the same four blocks stepped one after another as plain single-block
    steps.  Tile shape from the autotuner."""
    import torch
    from paper_2405_13943_amd import admm, gs, scenes
    t0 = time.time()
    bs = scenes.block_scene(n_cams=args.block_cams)
    K = len(bs.local_gid)
    dev = torch.device("cuda", 0)
    tg_cache = {}

    def target(k, v):
        if (k, v) not in tg_cache:
            c = bs.cams[k][v]
            tg_cache[(k, v)] = torch.from_numpy(
                scenes.rng(bs.seed * 1000 + 100 * k + v).random((3, c.height, c.width)).astype(np.float32)
            ).reshape(-1).to(dev)
        return tg_cache[(k, v)]

    # every block's targets on the device before anything is timed
    for k in range(K):
        for v in range(args.block_cams):
            target(k, v)
    model = admm.BlockModel.from_global(bs.params_global, bs.local_gid, spatial_strands=args.block_strands)
    log(f"[blocks4] setup {time.time() - t0:.1f}s: local {[len(g) for g in bs.local_gid]}, store "
        f"{tuple(model.x.shape)}, global {model.z.shape[1]}")
    x0 = model.x.clone()
    trainers = {}

    def trainer(tile):
        if tile not in trainers:
            tr = admm.AdmmTrainer(model, bs.cams, target, gs.raster_cfg(tile), lr=LR, rho=RHO, intv=100)
            tr.calibrate()
            trainers[tile] = tr
        return trainers[tile]

    def run(tile):
        tr = trainer(tile)
        tr.local_step()
        tr.t += 1

    tile = admm.autotune_tile(run, f"blocks4-{model.x.shape[1]}-1600x1066", args.tune_cache, reps=3) \
        if not args.no_tile_auto else (args.tile, args.tile, args.fwd_waves, args.bwd_waves)
    log(f"[blocks4] tile {'x'.join(map(str, tile))}")
    for t, tr in list(trainers.items()):
        if t != tile:
            del trainers[t]
    torch.cuda.empty_cache()
    # fresh state for the timed run
    model.x.copy_(x0)
    adaptive = admm.AdaptivePenalty() if args.adaptive else None
    if args.block_groups > 1:
        # contiguous groups of blocks, each on a stream of its own
        tr = admm.StreamedAdmmTrainer(model, bs.cams, target, gs.raster_cfg(tile), groups=args.block_groups, lr=LR,
                                      rho=RHO, intv=100, relax=args.relax, adaptive=adaptive)
        trainers.clear()
        tr.calibrate()
    else:
        tr = admm.AdmmTrainer(model, bs.cams, target, gs.raster_cfg(tile), lr=LR, rho=RHO, intv=100,
                              capacity=trainers[tile].capacity if tile in trainers else None, relax=args.relax,
                              adaptive=adaptive)
        trainers.clear()
        if tr.capacity is None:
            tr.calibrate()
        else:
            tr._buffers(tr.frame([0] * K))
    cfg = tr.cfg
    # sequential baseline: each block as its own plain single-block model
    seq = []
    for k in range(K):
        mk = admm.BlockModel.from_global(bs.params_global, [bs.local_gid[k]], spatial_strands=args.block_strands)
        tk = admm.AdmmTrainer(mk, [bs.cams[k]], (lambda kk: (lambda _k, v: target(kk, v)))(k), cfg, lr=LR, rho=RHO,
                              intv=1 << 30)
        tk.calibrate()
        seq.append(tk)
    # the batched frames render every block exactly as its own plain render
    batched = [tr] if args.block_groups <= 1 else tr.subs
    same = True
    for bt in batched:
        kb = bt.model.K
        f = bt.frame([0] * kb)
        gs.rasterize(bt.model.x, f, cfg, bt.buf)
        k0 = 0 if bt is tr else tr.parts[tr.subs.index(bt)][0]
        for k in range(kb):
            fk = seq[k0 + k].frame([0])
            gs.rasterize(seq[k0 + k].model.x, fk, cfg, seq[k0 + k].buf)
            same &= bool(torch.equal(f.image(bt.buf.rgb, k), fk.image(seq[k0 + k].buf.rgb, 0)))
    for b in batched + seq:
        b.buf.counters.zero_()
    log(f"[blocks4] batched images equal to per-block renders: {same}")

    def timed(fn, steps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    for _ in range(args.warmup):
        tr.step()
        for tk in seq:
            tk.local_step()
            tk.t += 1
    cons_ms = []

    def batched_step():
        tr.local_step()
        if tr.t % tr.intv == 0:
            if hasattr(tr, "join"):
                tr.join()          # the groups' queued steps are not the consensus's time
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            tr.consensus()
            b.record()
            cons_ms.append((a, b))
        tr.t += 1

    def seq_step():
        for tk in seq:
            tk.local_step()
            tk.t += 1

    steps = args.block_steps
    gs.profile_set(["k_consensus", "k_dual_rescale"])
    ms_b = timed(batched_step, steps)
    cons_kernels = {k: gs.profile_get(k) for k in ("k_consensus", "k_dual_rescale")}
    gs.profile_set(None)
    ms_s = timed(seq_step, steps)
    ok = all(not gs.read_counters(b.buf)["status"] & gs.GS_STATUS_PAIR_OVERFLOW for b in batched + seq)
    if not ok:
        raise SystemExit("pair capacity overflowed during the timed steps; rerun with more headroom")
    c_ms = [a.elapsed_time(b) for a, b in cons_ms]
    kb = kernel_breakdown(gs, torch, lambda: (tr.local_step(), setattr(tr, "t", tr.t + 1)), 5)
    ks = kernel_breakdown(gs, torch, seq_step, 5)
    log(f"[blocks4] batched kernels ms/step: {kb}")
    log(f"[blocks4] sequential kernels ms/step: {ks}")
    res = tr.resid.cpu().numpy().tolist()
    cons = consensus_roofline(model, tr, c_ms, cons_kernels)
    log(f"[blocks4] consensus: {cons}")
    out = {"metric": "K-block ADMM train steps/s (4 blocks, 1 view each, fwd+bwd+Adam/ADMM + consensus/100)",
           "value": 1000.0 * steps / ms_b, "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
           "ms_per_step": ms_b / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic (seeded slab blocks, ring cameras, U(0,1) targets)",
           "config": {"workload": "batched K=4 blocks 0.8M/1.5M/2.2M/3.0M own Gaussians SH3 + 10% shared copies "
                                  f"({model.x.shape[1]} local slots), {args.block_cams} ring views per block at "
                                  "1600x1066, consensus every 100 steps",
                      "tile": "x".join(map(str, tile[:2])), "waves_per_tile_fwd_bwd": list(tile[2:]),
                      "block_strands": args.block_strands, "stream_groups": args.block_groups,
                      "groups": [list(p) for p in tr.parts] if args.block_groups > 1 else [[0, K]]},
           "sequential_ms_per_step": ms_s / steps, "batched_speedup": ms_s / ms_b,
           "consensus_ms": c_ms, "consensus_calls": len(c_ms), "consensus_roofline": cons,
           "relax": args.relax, "adaptive_penalty": bool(args.adaptive), "images_equal_per_block": same,
           "kernel_ms_batched": kb, "kernel_ms_sequential": ks,
           "kernel_ms_note": "per-kernel sums over all launches of a step; with stream groups the groups' "
                             "launches overlap, so the batched sums exceed the step's elapsed time",
           "last_residuals": res}
    return out


def cpu_model():
    """Model name of the host CPU (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, budget_s=8.0):
    """The FP64 oracle on the host.  All threads: fwd + bwd of one 1600x1066
    view on a seeded pixel sample sized to about budget_s (extrapolated by
    pixel count) plus the Adam + ADMM oracle over all N: the step rate.  One
    thread: the same on 32 and 160 pixels.  And one full step of the parity
    scene (2,000 Gaussians, four 128x128 views, fwd + bwd + Adam/ADMM) on
    all threads."""
    import oracle
    from paper_2405_13943_amd import scenes
    lib = oracle.load_library()
    cam = scene.cams[0]
    target = scenes.config2_targets(scene, [0])[0]
    rng = np.random.default_rng(5)
    npx_total = cam.width * cam.height
    nthreads = lib.orc_num_threads()

    def fwd_bwd(npx):
        pix = rng.choice(npx_total, npx, replace=False)
        t = time.time()
        r = oracle.render(scene.params, cam, pixels=pix)
        tg = target.reshape(3, -1)[:, pix]
        dl = np.sign(r["rgb"] - tg) / (3 * npx_total)
        oracle.backward(scene.params, cam, dl, pixels=pix)
        return time.time() - t

    def view_seconds(budget):
        # per-call time = fixed projection cost + per-pixel cost: two probes
        # separate them, then the sample is sized to about `budget`
        t64 = fwd_bwd(64)
        t256 = fwd_bwd(256)
        per_px = max((t256 - t64) / 192.0, 1e-6)
        npx = int(min(npx_total, max(256, (budget - t64) / per_px)))
        t_px = fwd_bwd(npx)
        # the whole view: one fixed part plus every pixel at the sampled rate
        return t64 + (t_px - t64) * (npx_total - 64) / max(npx - 64, 1), npx, t_px

    x = scene.params
    t = time.time()
    oracle.adam_admm(x, np.zeros_like(x), np.zeros_like(x), np.zeros_like(x), x, LR, RHO, 1)
    t_adam = time.time() - t
    t_img, npx, t_px = view_seconds(budget_s)
    step_s = t_img + t_adam
    # one thread: two sample sizes give the fixed and the per-pixel cost
    lib.orc_set_threads(1)
    try:
        t_a = fwd_bwd(32)
        npx1 = 160
        t_px1 = fwd_bwd(npx1)
    finally:
        lib.orc_set_threads(nthreads)
    t_img1 = t_a + max(t_px1 - t_a, 0.0) * (npx_total - 32) / (npx1 - 32)
    # parity scene: a full step, every pixel of the four views
    c1 = scenes.config1()
    t = time.time()
    g = np.zeros_like(c1.params, dtype=np.float64)
    for v, c in enumerate(c1.cams):
        r = oracle.render(c1.params, c)
        dl = 0.25 * np.sign(r["rgb"] - c1.targets[v]) / r["rgb"].size
        g += oracle.backward(c1.params, c, dl)
    x1 = c1.params.astype(np.float64)
    oracle.adam_admm(x1, g, np.zeros_like(x1), np.zeros_like(x1), x1, LR, RHO, 1)
    t_c1 = time.time() - t
    return {"value": 1.0 / step_s, "unit": "steps/s", "cores": int(nthreads), "kind": "oracle",
            "sample": f"fwd+bwd on {npx} seeded pixels of one 1600x1066 view ({t_px:.1f}s, extrapolated to "
                      f"{npx_total} px: {t_img:.1f}s) + Adam/ADMM oracle over all {x.shape[1]} Gaussians "
                      f"({t_adam:.1f}s)",
            "cpu_model": cpu_model(),
            "single_thread": {"value": 1.0 / (t_img1 + t_adam), "unit": "steps/s", "cores": 1,
                              "sample": f"fwd+bwd on {npx1} seeded pixels ({t_px1:.1f}s, extrapolated: "
                                        f"{t_img1:.1f}s) + the same Adam/ADMM time (all threads)"},
            "parity_scene_step_s": round(t_c1, 3),
            "parity_scene": "2,000 Gaussians SH0, 4 x 128x128 views, fwd+bwd+Adam/ADMM, every pixel, all threads"}


def crop_subset(pr, x0, y0, size):
    """Gaussians whose conservative footprint (the alpha_min ellipse's
    bounding box from the oracle's projection, grown by 1% and 1 px) meets
    the crop [x0, x0 + size) x [y0, y0 + size): every other Gaussian has
    alpha < alpha_min at every crop pixel."""
    o, S, m = pr["opacity"], pr["cov2d"], pr["mean2d"]
    c = 2.0 * np.log(np.maximum(o * 255.0, 1.0))
    hx = np.sqrt(c * S[:, 0]) * 1.01 + 1.0
    hy = np.sqrt(c * S[:, 2]) * 1.01 + 1.0
    sel = pr["valid"] & (o * 255.0 >= 1.0) & (m[:, 0] + hx >= x0) & (m[:, 0] - hx <= x0 + size) \
        & (m[:, 1] + hy >= y0) & (m[:, 1] - hy <= y0 + size)
    return np.nonzero(sel)[0]


def run_oracle_timing(args):
    """The FP64 oracle on this host, all threads and one thread: a full step
    of the parity scene; fwd + bwd of the scale scene (500k, 1600x1066) and
    of the 2M-Gaussian 1920x1080 scene on four seeded crops each (all
    threads; one thread on a corner of the first crop), extrapolated by pixel
    count to the whole view and labelled so; the Adam/ADMM oracle over all
    500k Gaussians; the consensus oracle on a sample of the K = 4 store's
    global ids, extrapolated to all of them."""
    import oracle
    from paper_2405_13943_amd import admm, scenes
    lib = oracle.load_library()
    nth = lib.orc_num_threads()

    def at(n, fn):
        lib.orc_set_threads(n)
        try:
            t = time.time()
            fn()
            return time.time() - t
        finally:
            lib.orc_set_threads(nth)

    rows = []
    c1 = scenes.config1()

    def cfg1_step():
        g = np.zeros_like(c1.params, dtype=np.float64)
        for v, c in enumerate(c1.cams):
            r = oracle.render(c1.params, c)
            g += oracle.backward(c1.params, c, 0.25 * np.sign(r["rgb"] - c1.targets[v]) / r["rgb"].size)
        x1 = c1.params.astype(np.float64)
        oracle.adam_admm(x1, g, np.zeros_like(x1), np.zeros_like(x1), x1, LR, RHO, 1)
    rows.append({"what": "parity scene step (2,000 Gaussians SH0, 4 x 128x128, fwd+bwd+Adam/ADMM, every pixel)",
                 "all_threads_s": round(at(nth, cfg1_step), 3), "one_thread_s": round(at(1, cfg1_step), 3)})
    log(f"[oracle] {rows[-1]}")
    crop, crop1 = args.oracle_crop, max(8, args.oracle_crop // 4)
    for name, scene in (("scale scene, 500k Gaussians SH3, one 1600x1066 view", scenes.config2(n=500_000, n_cams=1)),
                        ("2M Gaussians SH3, one 1920x1080 view", scenes.config4b())):
        cam = scene.cams[0]
        W, H = cam.width, cam.height
        target = scenes.rng(4242).random((3, H, W)).astype(np.float32)
        t_proj = at(nth, lambda: oracle.project(scene.params, cam))
        pr = oracle.project(scene.params, cam)
        rng = np.random.default_rng(4343)
        crops = [(int(rng.integers(0, W - crop)), int(rng.integers(0, H - crop))) for _ in range(4)]
        per_px_all, per_px_one, n_sub = [], [], []
        for i, (x0, y0) in enumerate(crops):
            idx = crop_subset(pr, x0, y0, crop)
            sub = np.ascontiguousarray(scene.params[:, idx])
            ys, xs = np.mgrid[y0:y0 + crop, x0:x0 + crop]
            pix = (ys * W + xs).ravel()

            def fwd_bwd():
                r = oracle.render(sub, cam, pixels=pix)
                dl = np.sign(r["rgb"] - target.reshape(3, -1)[:, pix]) / (3 * W * H)
                oracle.backward(sub, cam, dl, pixels=pix)
            per_px_all.append(at(nth, fwd_bwd) / pix.size)
            n_sub.append(int(len(idx)))
            if i == 0:
                # one thread: the same Gaussians, the crop's top-left
                # crop1 x crop1 pixels
                ys1, xs1 = np.mgrid[y0:y0 + crop1, x0:x0 + crop1]
                pix1 = (ys1 * W + xs1).ravel()

                def fwd_bwd1():
                    r = oracle.render(sub, cam, pixels=pix1)
                    dl = np.sign(r["rgb"] - target.reshape(3, -1)[:, pix1]) / (3 * W * H)
                    oracle.backward(sub, cam, dl, pixels=pix1)
                per_px_one.append(at(1, fwd_bwd1) / pix1.size)
            log(f"[oracle] {name}: crop {i} at ({x0}, {y0}), {len(idx)} Gaussians reach it, "
                f"{per_px_all[-1] * 1e3:.3f} ms/px all threads")
        rows.append({"what": f"fwd+bwd, {name}, extrapolated from four {crop}x{crop} crops by pixel count",
                     "oracle_input": "per crop, the Gaussians whose footprint box meets it (the selection the "
                                     "crop parity tests give the oracle); the projection of all of them timed apart",
                     "gaussians_per_crop": n_sub,
                     "all_threads_s": round(t_proj + float(np.mean(per_px_all)) * W * H, 1),
                     "one_thread_s": round(t_proj * nth + per_px_one[0] * float(np.mean(per_px_all)) / per_px_all[0]
                                           * W * H, 1),
                     "projection_all_threads_s": round(t_proj, 2),
                     "ms_per_px_all_threads": [round(v * 1e3, 4) for v in per_px_all],
                     "ms_per_px_one_thread": round(per_px_one[0] * 1e3, 4),
                     "crops": crops,
                     "one_thread_from": f"the first crop's Gaussians on its {crop1}x{crop1} top-left pixels, "
                                        "scaled by the mean per-pixel time of the four crops over the first's; "
                                        "projection time scaled by the thread count"})
        log(f"[oracle] {rows[-1]}")
    x = scenes.config2(n=500_000, n_cams=1).params
    t = time.time()
    oracle.adam_admm(x, np.zeros_like(x), np.zeros_like(x), np.zeros_like(x), x, LR, RHO, 1)
    rows.append({"what": "Adam/ADMM oracle over all 500k Gaussians (NumPy)", "s": round(time.time() - t, 2)})
    bs = scenes.block_scene(n_cams=1)
    n_global = bs.params_global.shape[1]
    ptr, idx = admm.holder_csr(bs.local_gid, n_global)
    xl = bs.params_global[:, np.concatenate(bs.local_gid)].astype(np.float64)
    sample = 50_000
    sp = ptr[:sample + 1]
    t = time.time()
    oracle.consensus(xl, np.zeros_like(xl), sp, idx, sample)
    t_s = time.time() - t
    rows.append({"what": f"consensus oracle, {sample} of the K = 4 store's {n_global} global ids "
                         f"({len(idx)} copies), extrapolated to all of them",
                 "sample_s": round(t_s, 2), "extrapolated_s": round(t_s * n_global / sample, 1)})
    log(f"[oracle] {rows[-1]}")
    return {"workload": "oracle timing", "cpu_model": cpu_model(), "threads": int(nth), "rows": rows}


def copy_probe(nbytes=1 << 30, reps=5):
    """Plain device-to-device copy of known size (reads and writes nbytes
    each), used to scale the HBM byte counters of rocprofv3."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=500_000)
    ap.add_argument("--cams", type=int, default=64)
    ap.add_argument("--width", type=int, default=1600)
    ap.add_argument("--height", type=int, default=1066)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--fwd-waves", type=int, default=-1,
                    help="forward compositing wavefronts per tile: 1, 2, 4, or -1 per tile from its list length")
    ap.add_argument("--bwd-waves", type=int, default=-1,
                    help="backward compositing wavefronts per tile: 1, 2, 4, or -1 per tile from its list length")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--unfused", action="store_true", help="backward and optimiser as two calls (gradient in HBM)")
    ap.add_argument("--order", choices=("z-strands", "z", "generator"), default="z-strands",
                    help="storage order of the training scene's Gaussians (a layout: the scene is the same): Z-order "
                         "of the means in 16-Gaussian chunks over 1024 strands, plain Z-order, or as drawn")
    ap.add_argument("--profile-stride", type=int, default=9,
                    help="time the roofline kernels' launches on every n-th timed step (1: all)")
    ap.add_argument("--inline-stage-timing", action="store_true",
                    help="record the per-stage events inside the timed loop (adds their cost to the step time)")
    ap.add_argument("--workload", choices=("train", "blocks4", "serve", "consensus", "split4", "oracle"), default="train",
                    help="train: single block at scale (+ serve leg); blocks4: batched K=4 blocks; serve: serving "
                         "only; consensus: the consensus step alone on the K=4 block store; split4: K=4 blocks from "
                         "the scene by Alg. 1")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg of the train workload")
    ap.add_argument("--no-blocks4", action="store_true", help="skip the K = 4 block leg of the train workload")
    ap.add_argument("--blocks4-steps", type=int, default=100, help="timed steps of the K = 4 leg in the train line")
    ap.add_argument("--ssim", type=float, default=0.0,
                    help="train: weight lambda of the D-SSIM term of the loss (0: the L1 loss alone)")
    ap.add_argument("--serve-n", type=int, default=6_000_000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--serve-seconds", type=float, default=20.0)
    ap.add_argument("--serve-warmup", type=float, default=1.0, help="seconds of arrivals not counted (config: 5)")
    ap.add_argument("--serve-hbm", type=float, default=48.0, help="GB of transient serving buffers")
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--serve-max-batch", type=int, default=8)
    ap.add_argument("--block-cams", type=int, default=32)
    ap.add_argument("--block-steps", type=int, default=200)
    ap.add_argument("--block-groups", type=int, default=2,
                    help="blocks4: contiguous groups of blocks, each on its own stream between consensus rounds "
                         "(1: one launch per stage over all blocks)")
    ap.add_argument("--no-tile-auto", action="store_true", help="blocks4: use --tile instead of the autotuner")
    ap.add_argument("--relax", type=float, default=1.0, help="blocks4: over-relaxation alpha of the consensus")
    ap.add_argument("--adaptive", action="store_true", help="blocks4: residual-balancing penalty (until 2000)")
    ap.add_argument("--split-scale", type=float, default=1.4, help="split4: overlap scale factor of the blocks")
    ap.add_argument("--block-strands", type=int, default=1024,
                    help="blocks4/split4: inside each holder group, Z-order of the means in 16-Gaussian chunks over "
                         "this many strands (0: the drawn order); a storage layout")
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--oracle-crop", type=int, default=256, help="oracle: side of the timed crops")
    ap.add_argument("--copy-probe", action="store_true", help="only run a 1 GiB device copy (counter scaling)")
    ap.add_argument("--record-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="host only: write profiles/hbm_traffic.json for the measured kernels from rocprofv3 --pmc "
                         "output directories (the bench runs, then the copy probe's)")
    ap.add_argument("--traffic-kernels", default=None,
                    help="with --record-traffic: comma-separated kernels to record (default: every measured kernel "
                         "with samples)")
    ap.add_argument("--traffic-args", default="--steps 4 --warmup 2 --no-cpu-baseline --no-serve --no-blocks4",
                    help="with --record-traffic: the bench arguments the counter runs used")
    ap.add_argument("--traffic-workload", default=None,
                    help="workload name stored with recorded traffic (default: the training workload and --order)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.record_traffic:
        fd, wd, cfd, cwd = args.record_traffic
        cmds = [f"rocprofv3 --pmc FETCH_SIZE -f csv -d {fd} -o bench -- python bench.py {args.traffic_args}",
                f"rocprofv3 --pmc WRITE_SIZE -f csv -d {wd} -o bench -- python bench.py {args.traffic_args}",
                f"rocprofv3 --pmc FETCH_SIZE -f csv -d {cfd} -o copy -- python bench.py --copy-probe",
                f"rocprofv3 --pmc WRITE_SIZE -f csv -d {cwd} -o copy -- python bench.py --copy-probe"]
        for kernel in (args.traffic_kernels.split(",") if args.traffic_kernels else KERNEL_SOURCES):
            record_traffic(kernel, fd, wd, cfd, cwd, args.traffic_workload or train_workload_label(args.order), cmds)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the path holds all K blocks in one GPU's HBM and this build has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "oracle":
        print(json.dumps(run_oracle_timing(args)), flush=True)
        return
    if args.workload == "blocks4":
        print(json.dumps(run_blocks4(args)), flush=True)
        return
    if args.workload == "split4":
        print(json.dumps(run_split4(args)), flush=True)
        return
    if args.workload == "consensus":
        print(json.dumps(run_consensus(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps({"serve": run_serve(args)}), flush=True)
        return
    r = run_gpu(args)
    srv = None
    if not args.no_serve:
        srv = run_serve(args)
    b4 = None
    if not args.no_blocks4:
        # the K = 4 block leg, short: batched against the blocks one after another
        import copy
        a4 = copy.copy(args)
        a4.block_steps, a4.warmup = args.blocks4_steps, 5
        res = run_blocks4(a4)
        b4 = {k: res[k] for k in ("ms_per_step", "sequential_ms_per_step", "batched_speedup", "images_equal_per_block")}
        b4["workload"] = res["config"]["workload"]
        b4["steps"] = a4.block_steps
        b4["tile"] = res["config"]["tile"] + "/" + "/".join(map(str, res["config"]["waves_per_tile_fwd_bwd"]))
        b4["stream_groups"] = res["config"]["stream_groups"]
        b4["consensus_ms"] = [round(c, 3) for c in res["consensus_ms"]]
        import torch
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(r["scene"])
        log(f"[bench] cpu baseline {cpu['value']:.3e} steps/s on {cpu['cores']} threads")
    sps = 1000.0 / r["ms_per_step"]
    out = {
        "metric": "train steps/s (fwd+bwd+Adam, 500k Gs, 1600x1066)",
        "value": sps,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussians, ring cameras, U(0,1) targets)",
        "config": {"workload": f"single block, {r['N']} Gaussians SH3, {args.width}x{args.height}, "
                               f"{args.cams} ring views, one view per step, L1 + Adam/ADMM rho=1e-3",
                   "tile": f"{args.tile}x{args.tile}", "waves_per_tile_fwd_bwd": [args.fwd_waves, args.bwd_waves],
                   "max_pairs": r["pairs_max"], "storage_order": args.order},
        "stage_ms": {k: round(v, 5) for k, v in r["stage_ms"].items()},
        "kernel_ms": {k: round(v, 5) for k, v in r["kernel_ms"].items()},
        "kernel_ms_launches": r["kernel_n"],
        "kernel_ms_note": f"HIP events on the launch stream around every {args.profile_stride}-th timed step's "
                          "launch of each kernel",
        "roofline": {"bound": "alu", "kernel": "k_render_bwd", "achieved": round(r["bwd_tflops"], 3),
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(r["bwd_tflops"] / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": measured_traffic("k_render_bwd", train_workload_label(args.order)),
                     "work": f"{BWD_OPS} VALU ops x {r['kept']:.4g} (pixel, Gaussian) contributions per launch"},
        "roofline_step": step_roofline(r["N"], r["A"], r["visible"], r["pairs"], r["kept"], r["hw"],
                                       r["ms_per_step"], fused=not args.unfused),
        "roofline_stream": {"bound": "hbm", "kernel": r["opt_kernel"], "achieved": round(r["opt_gbs"], 1),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(r["opt_gbs"] / HBM_PEAK_GBS, 4),
                            "traffic": measured_traffic(r["opt_kernel"], train_workload_label(args.order)),
                            "bytes": int(r["opt_bytes"])},
        "cpu_baseline": cpu,
        "serve": srv,
        "blocks4": b4,
    }
    if r["ssim"] is not None:
        out["roofline_ssim"] = r["ssim"]
        out["config"]["workload"] = out["config"]["workload"].replace("L1 +", f"L1 + {r['ssim']['lambda']} D-SSIM +")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
