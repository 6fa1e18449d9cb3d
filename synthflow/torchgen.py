"""The piecewise-planar window generator of `make_window` with its per-pixel
work in torch (FP64), on any device.

It draws the scene, the camera motion and the moving regions from the same
seeded numpy generator, in the same order, as `make_window`, and casts, projects
and perturbs on the device.  With `noise_rng="numpy"` the per-pixel noise comes
from that generator too, and the window equals `make_window`'s up to the
rounding of the device's arithmetic; with `noise_rng="torch"` (the default) it
comes from a torch generator seeded from the window seed, which keeps the
distribution and moves thousands of windows a minute through a GPU, for
training sets too large to generate on the host.  Planes scenes only (the
small and indoor generators); the driving scene stays on the host.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _cumulative, _planes_scene, camera_motion, resolve_spec, window_rng

__all__ = ["make_window_torch"]


def _planes_depth_t(spec, scene, Ms, rays):
    """z-depth in cameras Ms (a list of (R, t)) of the frame-0 planar surface,
    all cameras and planes at once: a ray keeps the nearest plane whose
    intersection lies in that plane's Voronoi cell of frame 0, else the
    backdrop Z = d_max.  Returns [len(Ms), H, W]."""
    dev = rays.device
    R = torch.as_tensor(np.stack([M[0] for M in Ms]), dtype=torch.float64, device=dev)       # [F, 3, 3]
    o = torch.as_tensor(np.stack([-M[0].T @ M[1] for M in Ms]), dtype=torch.float64, device=dev)  # [F, 3]
    n = torch.as_tensor(scene["planes"], dtype=torch.float64, device=dev)          # [P, 3]
    seeds = torch.as_tensor(scene["seeds"], dtype=torch.float64, device=dev)       # [P, 2]
    # d = rays R per camera, as elementwise sums (no batched GEMM)
    d = sum(rays[None, ..., i, None] * R[:, None, None, i, :] for i in range(3))  # [F, H, W, 3]
    den = d @ n.T                                                                  # [F, H, W, P]
    s = ((1.0 - o @ n.T)[:, None, None, :]) / den
    P = o[:, None, None, None, :] + s[..., None] * d[..., None, :]                # [F, H, W, P, 3]
    ok = (s > 0) & (P[..., 2] > 1e-6) & torch.isfinite(s)
    px = spec.fx * P[..., 0] / P[..., 2] + spec.cx
    py = spec.fy * P[..., 1] / P[..., 2] + spec.cy
    ok &= torch.isfinite(px) & torch.isfinite(py)
    px = torch.where(ok, px, torch.zeros_like(px))
    py = torch.where(ok, py, torch.zeros_like(py))
    dist = (px[..., None] - seeds[:, 0]) ** 2 + (py[..., None] - seeds[:, 1]) ** 2  # [F, H, W, P, P]
    cell = torch.argmin(dist, dim=-1)
    ok &= cell == torch.arange(n.shape[0], device=dev)
    best = torch.where(ok, s, torch.full_like(s, math.inf)).amin(dim=-1)
    sb = (spec.d_max - o[:, 2, None, None]) / d[..., 2]
    sb = torch.where((sb > 0) & torch.isfinite(sb), sb, torch.full_like(sb, 10.0 * spec.d_max))
    return torch.where(torch.isfinite(best), best, sb)


def make_window_torch(spec, seed=0, device="cpu", noise=True, outliers=True, T=None, H=None, W=None,
                      keep_focal=False, noise_rng="torch"):
    """One window as `make_window` returns it, flows and depth as torch tensors
    on `device` (flows float32 [T,H,W,2], depth float64 [H,W], outlier bool
    [T,H,W]); poses, K and spec as there."""
    spec = resolve_spec(spec, T, H, W, keep_focal)
    if spec.scene != "planes":
        raise ValueError("make_window_torch generates planes scenes only")
    if noise_rng not in ("torch", "numpy"):
        raise ValueError("noise_rng must be 'torch' or 'numpy'")
    rng = window_rng(seed)
    Tn, Hn, Wn = spec.T, spec.H, spec.W
    poses = camera_motion(spec, rng, seed)
    Ms = _cumulative(poses)
    dev = torch.device(device)
    ys, xs = torch.meshgrid(torch.arange(Hn, dtype=torch.float64, device=dev),
                            torch.arange(Wn, dtype=torch.float64, device=dev), indexing="ij")
    rays = torch.stack([(xs - spec.cx) / spec.fx, (ys - spec.cy) / spec.fy, torch.ones_like(xs)], dim=-1)
    scene = _planes_scene(spec, rng)

    # frame t-1's depth (ray casting from camera t-1), moved by T_t, projected:
    # the flow on frame t-1's grid, every frame at once
    Z = _planes_depth_t(spec, scene, Ms[:Tn], rays)                                # [T, H, W]
    depth0 = Z[0].clone()
    R = torch.as_tensor(np.stack([P[0] for P in poses]), dtype=torch.float64, device=dev)
    t = torch.as_tensor(np.stack([P[1] for P in poses]), dtype=torch.float64, device=dev)
    Pc = Z[..., None] * rays                                                       # camera t-1 coordinates
    Pn = sum(Pc[..., i, None] * R[:, None, None, :, i] for i in range(3)) + t[:, None, None, :]
    flows = torch.stack([spec.fx * Pn[..., 0] / Pn[..., 2] + spec.cx - xs,
                         spec.fy * Pn[..., 1] / Pn[..., 2] + spec.cy - ys], dim=-1)
    outlier = torch.zeros((Tn, Hn, Wn), dtype=torch.bool, device=dev)

    if outliers and spec.outlier_kind in ("rect", "disc"):
        # the median end-point magnitude over the window, the mean of the two
        # middle values for an even count (as numpy's median)
        mag = torch.linalg.vector_norm(flows, dim=-1).reshape(-1)
        srt = torch.sort(mag).values
        m = srt.numel()
        med = float(srt[m // 2]) if m % 2 else float(0.5 * (srt[m // 2 - 1] + srt[m // 2]))
        r = max(10.0, 2.0 * med)
        n_obj = 2 if spec.outlier_kind == "rect" else 4
        area = spec.outlier_frac * Hn * Wn / n_obj
        for _ in range(n_obj):
            vel = rng.uniform(-r, r, 2)
            velt = torch.as_tensor(vel, dtype=torch.float64, device=dev)
            if spec.outlier_kind == "rect":
                aspect = rng.uniform(0.5, 2.0)
                w = math.sqrt(area * aspect)
                h = area / w
                x0 = rng.uniform(0, max(Wn - w, 1))
                y0 = rng.uniform(0, max(Hn - h, 1))
                for ti in range(1, Tn + 1):
                    ox, oy = x0 + vel[0] * (ti - 1), y0 + vel[1] * (ti - 1)
                    msk = (xs >= ox) & (xs < ox + w) & (ys >= oy) & (ys < oy + h)
                    flows[ti - 1][msk] = velt
                    outlier[ti - 1] |= msk
            else:
                rad = math.sqrt(area / math.pi)
                cx0 = rng.uniform(rad, max(Wn - rad, rad + 1))
                cy0 = rng.uniform(rad, max(Hn - rad, rad + 1))
                for ti in range(1, Tn + 1):
                    ox, oy = cx0 + vel[0] * (ti - 1), cy0 + vel[1] * (ti - 1)
                    msk = (xs - ox) ** 2 + (ys - oy) ** 2 < rad * rad
                    flows[ti - 1][msk] = velt
                    outlier[ti - 1] |= msk

    if noise:
        if noise_rng == "numpy":
            # the window generator's draws, frame by frame in its order
            us, angs = [], []
            for _ in range(Tn):
                us.append(rng.uniform(1e-12, 1 - 1e-12, (Hn, Wn)))
                angs.append(rng.uniform(0, 2 * np.pi, (Hn, Wn)))
            u = torch.as_tensor(np.stack(us), device=dev)
            ang = torch.as_tensor(np.stack(angs), device=dev)
        else:
            gen = torch.Generator(device=dev)
            gen.manual_seed(int(seed) + 0x5EED0000)
            u = 1e-12 + (1 - 2e-12) * torch.rand((Tn, Hn, Wn), generator=gen, dtype=torch.float64, device=dev)
            ang = 2 * math.pi * torch.rand((Tn, Hn, Wn), generator=gen, dtype=torch.float64, device=dev)
        # log-logistic end-point magnitude by its inverse CDF, uniform angle
        alpha = spec.noise_c1 * torch.linalg.vector_norm(flows, dim=-1) + spec.noise_c0
        e = alpha * (u / (1 - u)) ** (1.0 / spec.noise_beta)
        flows = flows + torch.stack([e * torch.cos(ang), e * torch.sin(ang)], dim=-1)

    return {
        "flows": flows.to(torch.float32),
        "K": (float(spec.fx), float(spec.fy), float(spec.cx), float(spec.cy)),
        "poses": poses,
        "depth": depth0,
        "outlier": outlier,
        "spec": spec,
    }
