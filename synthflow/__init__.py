"""Seeded synthetic optical-flow windows.

This module only *makes inputs*: a rigid scene, a camera trajectory, the
ground-truth flow fields between consecutive frames, log-logistic end-point
noise and independently moving regions.  It holds none of the inference
arithmetic (no residual model, no EM, no pose solver) and is shared by the
tests, the benchmark and the oracle timing so that every side sees the same
bytes.

Conventions (matching the problem statement of the paper, Sec. 3):
  * pixel j = (x, y) with integer pixel centres, x in [0, W), y in [0, H);
  * flow X_t[y, x] = (u, v) maps pixel (x, y) of image I_{t-1} to
    (x + u, y + v) in image I_t, stored as float32 [T, H, W, 2];
  * relative pose T_t = (R_t, t_t) maps a point from camera t-1 to camera t:
    P_t = R_t P_{t-1} + t_t; camera 0 is the world frame.

Workload shapes follow the indoor (640x480) and driving (1242x375) settings
the paper evaluates on; no dataset content is used.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["WindowSpec", "SPECS", "make_window", "make_batch", "BATCH_SHAPES", "BATCH_GROUPS", "rot_axis_angle"]


@dataclass
class WindowSpec:
    name: str
    T: int
    H: int
    W: int
    fx: float
    fy: float
    cx: float
    cy: float
    scene: str                      # "planes" or "driving"
    n_planes: int = 4
    d_min: float = 2.0
    d_max: float = 20.0
    trans: float = 0.3              # metres per frame (planes scenes)
    rot_deg: float = 2.0            # max rotation per frame (planes scenes)
    noise_c1: float = 0.05          # EPE scale alpha = c1*|f| + c0
    noise_c0: float = 0.1
    noise_beta: float = 3.0         # EPE shape
    outlier_kind: str = "rect"      # "rect", "disc", "box", "none"
    outlier_frac: float = 0.08
    n_iters: int = 3
    n_groups: int = 256
    n_boxes: int = 30
    extra: dict = field(default_factory=dict)


SPECS = {
    # CPU-sized plain EM window
    "small": WindowSpec("small", T=5, H=120, W=160, fx=120, fy=120, cx=80, cy=60,
                        scene="planes", n_planes=4, d_min=2.0, d_max=20.0,
                        trans=0.3, rot_deg=2.0, noise_c1=0.05, noise_c0=0.1,
                        noise_beta=3.0, outlier_kind="rect", outlier_frac=0.08,
                        n_iters=3, n_groups=256),
    # indoor-shaped window
    "indoor": WindowSpec("indoor", T=6, H=480, W=640, fx=525, fy=525, cx=320, cy=240,
                         scene="planes", n_planes=12, d_min=0.5, d_max=6.0,
                         trans=0.05, rot_deg=3.0, noise_c1=0.04, noise_c0=0.15,
                         noise_beta=2.5, outlier_kind="disc", outlier_frac=0.10,
                         n_iters=4, n_groups=2048),
    # driving-shaped window
    "driving": WindowSpec("driving", T=8, H=375, W=1242, fx=718, fy=718, cx=607, cy=185,
                          scene="driving", d_min=3.0, d_max=80.0, trans=1.0,
                          rot_deg=1.5, noise_c1=0.03, noise_c0=0.2, noise_beta=2.2,
                          outlier_kind="box", outlier_frac=0.15, n_iters=4,
                          n_groups=4096, n_boxes=30),
}


def rot_axis_angle(axis, angle):
    """Rodrigues rotation matrix for a unit axis and an angle in radians."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    Kx = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * Kx + (1 - math.cos(angle)) * (Kx @ Kx)


def _unit_sphere(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _cumulative(poses):
    """World (camera 0) -> camera t transforms M_0..M_T from relative poses."""
    Ms = [(np.eye(3), np.zeros(3))]
    for R, t in poses:
        Rm, tm = Ms[-1]
        Ms.append((R @ Rm, R @ tm + t))
    return Ms


def _rays(spec, H, W):
    xs, ys = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    xn = (xs - spec.cx) / spec.fx
    yn = (ys - spec.cy) / spec.fy
    return xs, ys, np.stack([xn, yn, np.ones_like(xn)], axis=-1)


# --------------------------------------------------------------------------
# piecewise-planar scene (Voronoi cells of frame 0, one plane per cell)
# --------------------------------------------------------------------------
def _planes_scene(spec, rng):
    H, W = spec.H, spec.W
    seeds = np.stack([rng.uniform(0, W, spec.n_planes), rng.uniform(0, H, spec.n_planes)], axis=1)
    corners = np.array([[0, 0], [W - 1, 0], [0, H - 1], [W - 1, H - 1]], dtype=np.float64)
    cn = np.stack([(corners[:, 0] - spec.cx) / spec.fx, (corners[:, 1] - spec.cy) / spec.fy,
                   np.ones(4)], axis=1)
    planes = []
    for _ in range(spec.n_planes):
        for _attempt in range(1000):
            inv = 1.0 / rng.uniform(spec.d_min, spec.d_max, 3)
            # plane n . P = 1 with inverse depth affine in normalised coordinates
            n = np.linalg.solve(cn[:3], inv)
            inv4 = cn[3] @ n
            if 1.0 / spec.d_max <= inv4 <= 1.0 / spec.d_min:
                planes.append(n)
                break
        else:  # pragma: no cover - practically unreachable
            planes.append(np.array([0.0, 0.0, 1.0 / spec.d_max]))
    return {"seeds": seeds, "planes": np.array(planes)}


def _cell_of(scene, px, py):
    s = scene["seeds"]
    d = (px[..., None] - s[:, 0]) ** 2 + (py[..., None] - s[:, 1]) ** 2
    return np.argmin(d, axis=-1)


def _planes_depth(spec, scene, M, rays):
    """z-depth in camera (R,t)=M of the frame-0 planar surface (ray casting)."""
    R, t = M
    o = -R.T @ t                              # camera centre in world
    d = rays @ R                              # world direction with unit camera-z
    best = np.full(rays.shape[:2], np.inf)
    for k, n in enumerate(scene["planes"]):
        den = d @ n
        with np.errstate(divide="ignore", invalid="ignore"):
            s = (1.0 - n @ o) / den
        P = o + s[..., None] * d
        ok = (s > 0) & (P[..., 2] > 1e-6) & np.isfinite(s)
        with np.errstate(divide="ignore", invalid="ignore"):
            px = spec.fx * P[..., 0] / P[..., 2] + spec.cx
            py = spec.fy * P[..., 1] / P[..., 2] + spec.cy
        ok &= np.isfinite(px) & np.isfinite(py)
        cell = _cell_of(scene, np.where(ok, px, 0.0), np.where(ok, py, 0.0))
        ok &= cell == k
        best = np.where(ok & (s < best), s, best)
    # fronto-parallel backdrop Z = d_max in the world frame
    with np.errstate(divide="ignore", invalid="ignore"):
        sb = (spec.d_max - o[2]) / d[..., 2]
    sb = np.where((sb > 0) & np.isfinite(sb), sb, 10.0 * spec.d_max)
    return np.where(np.isfinite(best), best, sb)


# --------------------------------------------------------------------------
# driving scene: ground plane, axis-aligned boxes, backdrop
# --------------------------------------------------------------------------
def _driving_scene(spec, rng):
    boxes = []
    for _ in range(spec.n_boxes):
        size = rng.uniform(1.0, 4.0, 3)
        cxw = rng.uniform(-15.0, 15.0)
        czw = rng.uniform(3.0 + size[2] / 2, spec.d_max - size[2] / 2)
        lo = np.array([cxw - size[0] / 2, 1.6 - size[1], czw - size[2] / 2])
        hi = np.array([cxw + size[0] / 2, 1.6, czw + size[2] / 2])
        boxes.append((lo, hi))
    return {"boxes": boxes, "ground_y": 1.6, "moving": np.zeros(spec.n_boxes, bool),
            "vel": np.zeros((spec.n_boxes, 3))}


def _slab(o, d, lo, hi):
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t0 = (lo - o) * inv
        t1 = (hi - o) * inv
    tmin = np.nanmax(np.minimum(t0, t1), axis=-1)
    tmax = np.nanmin(np.maximum(t0, t1), axis=-1)
    hit = (tmax >= tmin) & (tmax > 0)
    ent = np.where(tmin > 0, tmin, np.inf)
    return np.where(hit, ent, np.inf)


def _driving_depth(spec, scene, M, rays, frame):
    """z-depth and hit-object id (-1 static background) in camera M at `frame`."""
    R, t = M
    o = -R.T @ t
    d = rays @ R
    best = np.full(rays.shape[:2], np.inf)
    obj = np.full(rays.shape[:2], -1, dtype=np.int64)
    with np.errstate(divide="ignore", invalid="ignore"):
        sg = (scene["ground_y"] - o[1]) / d[..., 1]
    sg = np.where((sg > 0) & np.isfinite(sg), sg, np.inf)
    best = np.minimum(best, sg)
    H, W = rays.shape[:2]
    for k, (lo, hi) in enumerate(scene["boxes"]):
        off = scene["vel"][k] * frame
        blo, bhi = lo + off, hi + off
        # pixels whose rays can meet the box: for a box wholly in front of the
        # camera, the bounding rectangle of its projected corners (plus a
        # margin); the test itself is the same elementwise slab test
        corners = np.array([[a, b, c] for a in (blo[0], bhi[0]) for b in (blo[1], bhi[1])
                            for c in (blo[2], bhi[2])])
        pc = corners @ R.T + t
        y0, y1, x0, x1 = 0, H, 0, W
        if np.all(pc[:, 2] > 1e-6):
            u, v = _project(spec, pc)
            x0, x1 = max(int(np.floor(u.min())) - 2, 0), min(int(np.ceil(u.max())) + 3, W)
            y0, y1 = max(int(np.floor(v.min())) - 2, 0), min(int(np.ceil(v.max())) + 3, H)
            if x0 >= x1 or y0 >= y1:
                continue
        s = _slab(o, d[y0:y1, x0:x1], blo, bhi)
        take = s < best[y0:y1, x0:x1]
        best[y0:y1, x0:x1] = np.where(take, s, best[y0:y1, x0:x1])
        obj[y0:y1, x0:x1] = np.where(take, k, obj[y0:y1, x0:x1])
    with np.errstate(divide="ignore", invalid="ignore"):
        sb = (spec.d_max - o[2]) / d[..., 2]
    sb = np.where((sb > 0) & np.isfinite(sb), sb, 10.0 * spec.d_max)
    take = sb < best
    best = np.where(take, sb, best)
    obj = np.where(take, -1, obj)
    return best, obj


# --------------------------------------------------------------------------
def _project(spec, P):
    return (spec.fx * P[..., 0] / P[..., 2] + spec.cx, spec.fy * P[..., 1] / P[..., 2] + spec.cy)


def _fisk_noise(rng, flow, c1, c0, beta):
    """End-point noise with log-logistic magnitude (inverse CDF) and uniform angle."""
    mag = np.linalg.norm(flow, axis=-1)
    alpha = c1 * mag + c0
    u = rng.uniform(1e-12, 1 - 1e-12, mag.shape)
    e = alpha * (u / (1 - u)) ** (1.0 / beta)
    ang = rng.uniform(0, 2 * np.pi, mag.shape)
    return np.stack([e * np.cos(ang), e * np.sin(ang)], axis=-1)


def resolve_spec(spec, T=None, H=None, W=None, keep_focal=False):
    """A copy of the spec (or the named one) with T/H/W overrides applied; a
    new size scales the intrinsics (keep_focal: only the principal point)."""
    if isinstance(spec, str):
        spec = SPECS[spec]
    spec = WindowSpec(**{**spec.__dict__})
    if T is not None:
        spec.T = T
    if H is not None or W is not None:
        sx = (W if W is not None else spec.W) / spec.W
        sy = (H if H is not None else spec.H) / spec.H
        spec.W = W if W is not None else spec.W
        spec.H = H if H is not None else spec.H
        if keep_focal:
            # centre crop: same focal length, so flow magnitudes stay realistic
            spec.cx *= sx
            spec.cy *= sy
        else:
            spec.fx *= sx
            spec.cx *= sx
            spec.fy *= sy
            spec.cy *= sy
    return spec


def window_rng(seed):
    """The generator of window `seed` (scene, motion, outliers and noise draws)."""
    return np.random.Generator(np.random.Philox(key=np.uint64(seed) + np.uint64(0x5EED0000)))


def camera_motion(spec, rng, seed=0, speed_range=None):
    """The T relative ground-truth poses (R, t) of a window, drawn from rng."""
    poses = []
    for _ in range(spec.T):
        if spec.scene == "driving":
            yaw = math.radians(rng.uniform(-spec.rot_deg, spec.rot_deg))
            R = rot_axis_angle([0.0, 1.0, 0.0], yaw)
            c = np.array([0.0, 0.0, spec.trans])          # camera moves forward
            t = -R @ c
        else:
            R = rot_axis_angle(_unit_sphere(rng), math.radians(rng.uniform(0.0, spec.rot_deg)))
            t = spec.trans * _unit_sphere(rng)
        poses.append((R, t))
    if speed_range is not None:
        srng = np.random.Generator(np.random.Philox(key=np.uint64(seed) + np.uint64(0x5BEED000)))
        poses = [(R, t * srng.uniform(*speed_range)) for R, t in poses]
    return poses


def make_window(spec, seed=0, noise=True, outliers=True, T=None, H=None, W=None, keep_focal=False,
                speed_range=None):
    """Generate one window.

    Returns a dict with
      flows     float32 [T,H,W,2]
      K         (fx, fy, cx, cy)
      poses     list of T (R 3x3, t 3) relative ground-truth poses
      depth     float64 [H,W] ground-truth z-depth of frame 0
      outlier   bool [T,H,W] independently-moving pixels on frame t-1's grid
      spec      the WindowSpec used (with T/H/W overrides applied)
    speed_range (lo, hi): each frame's translation is scaled by a factor drawn
    uniformly from [lo, hi] by a generator of its own (the default draws
    nothing and leaves every other stream unchanged).
    """
    spec = resolve_spec(spec, T, H, W, keep_focal)
    rng = window_rng(seed)
    Tn, Hn, Wn = spec.T, spec.H, spec.W
    poses = camera_motion(spec, rng, seed, speed_range)
    Ms = _cumulative(poses)

    xs, ys, rays = _rays(spec, Hn, Wn)
    scene = _planes_scene(spec, rng) if spec.scene == "planes" else _driving_scene(spec, rng)

    # ---- moving boxes (driving) are chosen on frame 0 before casting
    if spec.scene == "driving" and outliers and spec.outlier_kind == "box":
        _, obj0 = _driving_depth(spec, scene, Ms[0], rays, 0)
        covered = np.zeros((Hn, Wn), bool)
        order = rng.permutation(spec.n_boxes)
        for k in order:
            if covered.mean() >= spec.outlier_frac:
                break
            m = obj0 == k
            if not m.any():
                continue
            scene["moving"][k] = True
            ang = rng.uniform(0, 2 * np.pi)
            sp = rng.uniform(0.5, 2.0)
            scene["vel"][k] = np.array([sp * math.cos(ang), 0.0, sp * math.sin(ang)])
            covered |= m

    flows = np.zeros((Tn, Hn, Wn, 2), np.float64)
    outlier = np.zeros((Tn, Hn, Wn), bool)
    depth0 = None
    for ti in range(1, Tn + 1):
        Mprev = Ms[ti - 1]
        if spec.scene == "planes":
            Z = _planes_depth(spec, scene, Mprev, rays)
            obj = None
        else:
            Z, obj = _driving_depth(spec, scene, Mprev, rays, ti - 1)
        if ti == 1:
            depth0 = Z.copy()
        Pc = Z[..., None] * rays                       # camera t-1 coordinates
        R, t = poses[ti - 1]
        if obj is not None and scene["moving"].any():
            # moving boxes: displace the world point by the box velocity
            Rm, tm = Mprev
            Pw = (Pc - tm) @ Rm                         # world coordinates
            mv = (obj >= 0) & scene["moving"][np.clip(obj, 0, None)]
            Pw = Pw + np.where(mv[..., None], scene["vel"][np.clip(obj, 0, None)], 0.0)
            Rn, tn = Ms[ti]
            Pn = Pw @ Rn.T + tn
            outlier[ti - 1] = mv
        else:
            Pn = Pc @ R.T + t
        u1, v1 = _project(spec, Pn)
        flows[ti - 1, ..., 0] = u1 - xs
        flows[ti - 1, ..., 1] = v1 - ys

    # ---- image-space moving regions (rectangles / discs)
    if outliers and spec.outlier_kind in ("rect", "disc"):
        med = float(np.median(np.linalg.norm(flows, axis=-1)))
        r = max(10.0, 2.0 * med)
        n_obj = 2 if spec.outlier_kind == "rect" else 4
        area = spec.outlier_frac * Hn * Wn / n_obj
        for _ in range(n_obj):
            vel = rng.uniform(-r, r, 2)
            if spec.outlier_kind == "rect":
                aspect = rng.uniform(0.5, 2.0)
                w = math.sqrt(area * aspect)
                h = area / w
                x0 = rng.uniform(0, max(Wn - w, 1))
                y0 = rng.uniform(0, max(Hn - h, 1))
                for ti in range(1, Tn + 1):
                    ox, oy = x0 + vel[0] * (ti - 1), y0 + vel[1] * (ti - 1)
                    m = (xs >= ox) & (xs < ox + w) & (ys >= oy) & (ys < oy + h)
                    flows[ti - 1][m] = vel
                    outlier[ti - 1] |= m
            else:
                rad = math.sqrt(area / math.pi)
                cx0 = rng.uniform(rad, max(Wn - rad, rad + 1))
                cy0 = rng.uniform(rad, max(Hn - rad, rad + 1))
                for ti in range(1, Tn + 1):
                    ox, oy = cx0 + vel[0] * (ti - 1), cy0 + vel[1] * (ti - 1)
                    m = (xs - ox) ** 2 + (ys - oy) ** 2 < rad * rad
                    flows[ti - 1][m] = vel
                    outlier[ti - 1] |= m

    if noise:
        for ti in range(Tn):
            flows[ti] += _fisk_noise(rng, flows[ti], spec.noise_c1, spec.noise_c0, spec.noise_beta)

    return {
        "flows": flows.astype(np.float32),
        "K": (float(spec.fx), float(spec.fy), float(spec.cx), float(spec.cy)),
        "poses": poses,
        "depth": depth0,
        "outlier": outlier,
        "spec": spec,
    }


# shapes of a mixed batch: (generator, W, H); the 320x240 windows use the
# CPU-sized generator with its intrinsics scaled x2, 640x480 the indoor one,
# 1242x375 the driving one
BATCH_SHAPES = (("small", 320, 240), ("indoor", 640, 480), ("driving", 1242, 375))
# P3P groups per frame of a batch window, by shape
BATCH_GROUPS = {(320, 240): 1024, (640, 480): 2048, (1242, 375): 4096}


def _batch_item(args):
    name, sd, noise, outliers, T, H, W = args
    return make_window(name, sd, noise=noise, outliers=outliers, T=T, H=H, W=W)


def make_batch(n=32, seed=0, shapes=BATCH_SHAPES, T_range=(4, 8), noise=True, outliers=True, workers=1):
    """n independent windows, each with a shape drawn uniformly from `shapes`
    and T drawn uniformly from T_range (inclusive), generated as make_window
    does for that shape; window i uses seed (seed << 16) + i.  Returns a list of
    make_window dicts.  workers > 1 generates them in forked worker processes
    (call it before the process touches a GPU)."""
    rng = np.random.Generator(np.random.Philox(key=np.uint64(seed) + np.uint64(0xBA7C0000)))
    jobs = []
    for i in range(n):
        name, W, H = shapes[int(rng.integers(len(shapes)))]
        T = int(rng.integers(T_range[0], T_range[1] + 1))
        jobs.append((name, (seed << 16) + i, noise, outliers, T, H, W))
    if workers <= 1:
        return [_batch_item(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(workers, n)) as pool:
        return pool.map(_batch_item, jobs, chunksize=1)

