"""Central finite differences of L = sum(W * C) through the HIP forward, many
coordinates per launch (test helper).

Each perturbed copy of the Gaussians is a job of its own over a disjoint
Gaussian range, all viewed by the same camera: one rasterize call renders
the + and - copies of up to `batch` coordinates.  A coordinate whose
keep/stop decisions (contributor counts) change inside [-h, h] is reported
as flipped and left out."""
import numpy as np
import torch

from paper_2405_13943_amd import gs


def finite_differences(params, cam, W, coords, cfg, h=1e-6, batch=256):
    """params: [A][n] FP64 device planes; W: FP64 device [3*H*W]; coords:
    list of (plane, Gaussian).  Returns (fd, noise, flipped) as numpy arrays
    over coords: noise bounds the FP64 rounding of each difference (ten
    units of rounding of the changed terms, divided by 2h)."""
    A, n = params.shape
    HW = cam.width * cam.height
    base = gs.rasterize(params, gs.Frame([cam], [gs.JobSpec(0, 0, n, 1.0)], cfg), cfg)
    base_n = base.ncontrib[:HW].clone()
    B = min(batch, len(coords))
    frame = gs.Frame([cam], [gs.JobSpec(0, k * n, (k + 1) * n, 1.0) for k in range(2 * B)], cfg)
    buf = None
    fd, noise, flipped = [], [], []
    eps = np.finfo(np.float64).eps
    for c0 in range(0, len(coords), B):
        chunk = list(coords[c0:c0 + B])
        m = len(chunk)
        chunk += [chunk[0]] * (B - m)                  # pad a ragged last chunk
        rep = params.repeat(1, 2 * B).contiguous()
        a = torch.tensor([c[0] for c in chunk], dtype=torch.long, device=params.device)
        i = torch.tensor([c[1] for c in chunk], dtype=torch.long, device=params.device)
        k = torch.arange(B, device=params.device)
        rep[a, 2 * k * n + i] += h
        rep[a, (2 * k + 1) * n + i] -= h
        buf = gs.rasterize(rep, frame, cfg, buf)
        rgb = buf.rgb[:2 * B * 3 * HW].view(B, 2, 3 * HW)
        nc = buf.ncontrib[:2 * B * HW].view(B, 2, HW)
        dW = (rgb[:, 0] - rgb[:, 1]) * W[None]
        fd.append((dW.sum(1) / (2 * h)).cpu().numpy()[:m])
        mag = ((rgb[:, 0].abs() + rgb[:, 1].abs()) * W.abs()[None] * (rgb[:, 0] != rgb[:, 1])).sum(1)
        noise.append((10 * eps * mag / (2 * h)).cpu().numpy()[:m])
        flipped.append((nc != base_n[None, None]).any(2).any(1).cpu().numpy()[:m])
    return np.concatenate(fd), np.concatenate(noise), np.concatenate(flipped)
