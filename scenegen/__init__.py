"""Seeded synthetic piecewise-planar multi-view scenes (input generator only).

This module produces the inputs that both the GPU path and the CPU oracle consume:
8-bit grey images, pinhole cameras (K, R, t with X_cam = R X_world + t), the depth
range handed to the solver, and ground truth (depth, normal, plane id) for the
reference view.  It is a plain ray caster; it holds none of the stereo method's
arithmetic (no matching cost, no homography warp, no search) and is shared by the
oracle tests, the GPU tests and the benchmark.

Scene recipe (the paper evaluates on ETH3D high-resolution scenes, which these stand
in for; every number below is this generator's own choice):

* The master camera (the reference view for single-reference scenes) sees a Voronoi
  partition of its image into ``n_planes`` cells from seeded sites; cell i carries
  plane i.  Plane normals are uniform on the cap within ``normal_max_deg`` of the
  master optical axis, the depth at the cell site is uniform in
  [site_depth_lo, site_depth_hi]; a normal is re-drawn until the plane's depth over
  its cell stays within [0.75 lo, 1.5 hi].
* The surface is the union of the plane pieces inside their cells' viewing cones.
  A ray of any camera is intersected with every plane; a hit is accepted iff it lies
  in front of the master camera and projects back into that plane's cell; the
  nearest accepted hit wins; rays with no accepted hit see a textured backdrop.
* Texture is band-limited value noise in plane coordinates (consistent across
  views): lattice values from an integer hash keyed by (seed, plane, octave, i, j),
  quintic fade, 4 octaves with halving amplitude, finest lattice spacing 3 px at the
  plane's farthest depth in the master view, mapped to [40, 215].  A seeded fraction
  of the planes is texture-less (constant intensity drawn from U[60, 200]).
* Rendering uses 2x2 supersampling, then i.i.d. Gaussian noise (Box-Muller on hash
  uniforms) with sigma = 2, round-half-even, clamp to [0, 255], uint8.
* Cameras: pinhole, f = 0.9 W, principal point ((W-1)/2, (H-1)/2).  Sources sit on
  a horizontal arc of ``arc_deg`` degrees around the look-at point at the median
  master depth, the reference in the middle; all look at that point.  A seeded
  global rigid transform is applied so that the world frame is not the reference
  camera frame.
* The depth range is [0.9 min GT, 1.1 max GT] over the reference view.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

M32 = 0xFFFFFFFF
_DT = torch.float64


# ----------------------------------------------------------------------------- hashing
def _hash32(x: torch.Tensor) -> torch.Tensor:
    """32-bit avalanche hash (xorshift-multiply finaliser) on int64 tensors."""
    x = x & M32
    x = x ^ (x >> 16)
    x = (x * 0x7FEB352D) & M32
    x = x ^ (x >> 15)
    x = (x * 0x846CA68B) & M32
    x = x ^ (x >> 16)
    return x


def _mix(*vals) -> torch.Tensor:
    h = None
    for v in vals:
        if not torch.is_tensor(v):
            v = torch.tensor(int(v), dtype=torch.int64)
        v = v.to(torch.int64) & M32
        h = _hash32(v ^ 0x9E3779B9) if h is None else _hash32(h ^ _hash32(v + 0x632BE5AB))
    return h


def _unit(h: torch.Tensor) -> torch.Tensor:
    """Hash -> uniform in [0, 1) with 24 bits."""
    return (h >> 8).to(_DT) * (1.0 / 16777216.0)


# ----------------------------------------------------------------------------- configs
@dataclass
class SceneConfig:
    width: int
    height: int
    n_src: int
    n_planes: int
    textureless_frac: float
    site_depth_lo: float
    site_depth_hi: float
    normal_max_deg: float = 50.0
    arc_deg: float = 15.0
    noise_sigma: float = 2.0
    n_textureless: Optional[int] = None  # exact count overrides the fraction


#: The benchmark workloads, by what they are.
CONFIGS = {
    # 1 ref + 4 sources, 160x120, 3 planes (one texture-less), depth 2-8 m
    "tiny": SceneConfig(160, 120, 4, 3, 0.0, 2.0, 8.0, n_textureless=1),
    # 1 ref + 9 sources, 1600x1066, 12 planes (30% texture-less), depth 2-8 m
    "mid": SceneConfig(1600, 1066, 9, 12, 0.30, 2.0, 8.0),
    # 1 ref + 10 sources, 3200x2130, 25 planes (35% texture-less), depth 1-20 m
    "highres": SceneConfig(3200, 2130, 10, 25, 0.35, 1.0, 20.0),
    # training scenes of the learned proposal: the high-resolution recipe at 1600x1066
    "proposal_train": SceneConfig(1600, 1066, 10, 25, 0.35, 1.0, 20.0),
}

#: window side, dilation, top-K, iterations per workload
SOLVER = {
    "tiny": dict(window=11, dilation=1, top_k=4, iters=3),
    "mid": dict(window=21, dilation=2, top_k=4, iters=8),
    "mid_dense": dict(window=21, dilation=1, top_k=4, iters=8),
    "highres": dict(window=31, dilation=3, top_k=5, iters=8),
    "proposal_train": dict(window=21, dilation=2, top_k=5, iters=8),
}

SCENE_SEEDS = {"tiny": 1, "mid": 2, "highres": 3, "batched": 4}
#: seeds of the proposal network's training scenes (disjoint from the workloads above)
PROPOSAL_TRAIN_SEEDS = range(100000, 102000)
PM_SEED = 0x5EED


@dataclass
class Camera:
    K: np.ndarray  # 3x3
    R: np.ndarray  # 3x3 world->cam
    t: np.ndarray  # 3
    width: int
    height: int


@dataclass
class Scene:
    images: List[np.ndarray]  # uint8 (H_i, W_i); index 0 = reference
    cams: List[Camera]
    depth_range: tuple  # (d_lo, d_hi) for the reference
    gt_depth: np.ndarray  # (H, W) float64, reference camera Z
    gt_normal: np.ndarray  # (H, W, 3) float64, reference camera frame, facing the camera
    gt_plane: np.ndarray  # (H, W) int32 plane id
    textured: np.ndarray  # (n_planes,) bool
    seed: int = 0
    meta: dict = field(default_factory=dict)

    # stacked camera arrays (n, 3, 3) / (n, 3) in float64
    @property
    def K(self):
        return np.stack([c.K for c in self.cams])

    @property
    def R(self):
        return np.stack([c.R for c in self.cams])

    @property
    def t(self):
        return np.stack([c.t for c in self.cams])


# ----------------------------------------------------------------------------- geometry helpers
def _apply3(M: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """M (3x3) applied to points X (..., 3), written out (no BLAS call per chunk)."""
    return torch.stack([M[0, 0] * X[..., 0] + M[0, 1] * X[..., 1] + M[0, 2] * X[..., 2],
                        M[1, 0] * X[..., 0] + M[1, 1] * X[..., 1] + M[1, 2] * X[..., 2],
                        M[2, 0] * X[..., 0] + M[2, 1] * X[..., 1] + M[2, 2] * X[..., 2]], -1)


def _intrinsics(w: int, h: int) -> np.ndarray:
    f = 0.9 * w
    return np.array([[f, 0.0, (w - 1) / 2.0], [0.0, f, (h - 1) / 2.0], [0.0, 0.0, 1.0]])


def _rot_y(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def _rot_x(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d],
    ])


class _World:
    """Planes, cells and textures, all expressed in the master camera frame."""

    def __init__(self, seed, K0, w0, h0, n_planes, n_textureless, lo, hi, normal_max_deg, device):
        self.seed = seed
        self.device = device
        self.K0 = torch.tensor(K0, dtype=_DT, device=device)
        self.K0inv = torch.linalg.inv(self.K0)
        self.w0, self.h0 = w0, h0
        rng = np.random.default_rng([seed, 0x51735])
        self.P = n_planes
        sites = np.stack([rng.uniform(0, w0 - 1, n_planes), rng.uniform(0, h0 - 1, n_planes)], 1)
        self.sites = torch.tensor(sites, dtype=_DT, device=device)
        # label map over an extended domain [-w0, 2w0) x [-h0, 2h0) at 1 px
        self.lx0, self.ly0 = -w0, -h0
        self.lw, self.lh = 3 * w0, 3 * h0
        self.label = self._label_map()
        # master-view pixel rays
        ys, xs = torch.meshgrid(torch.arange(h0, dtype=_DT, device=device),
                                torch.arange(w0, dtype=_DT, device=device), indexing="ij")
        lab0 = self.label[(ys - self.ly0).long(), (xs - self.lx0).long()]
        rays0 = self._rays(self.K0inv, xs, ys)  # (h0, w0, 3)
        cosmax = math.cos(math.radians(normal_max_deg))
        normals, points, zfar = [], [], []
        for i in range(n_planes):
            sx, sy = sites[i]
            d_site = rng.uniform(lo, hi)
            rs = self.K0inv @ torch.tensor([sx, sy, 1.0], dtype=_DT, device=device)
            X = d_site * rs
            mask = lab0 == i
            rr = rays0[mask]  # (m, 3)
            chosen = None
            for _ in range(200):
                ct = rng.uniform(cosmax, 1.0)
                st = math.sqrt(max(0.0, 1 - ct * ct))
                ps = rng.uniform(0, 2 * math.pi)
                n = torch.tensor([st * math.cos(ps), st * math.sin(ps), ct], dtype=_DT, device=device)
                n = -n  # face the master camera: n . r < 0
                if rr.shape[0] == 0:
                    chosen = n
                    break
                den = rr @ n
                if bool((den < 0).all()):
                    z = (n @ X) / den
                    if float(z.min()) >= 0.75 * lo and float(z.max()) <= 1.5 * hi:
                        chosen = n
                        break
            if chosen is None:
                chosen = torch.tensor([0.0, 0.0, -1.0], dtype=_DT, device=device)
            normals.append(chosen)
            points.append(X)
            if rr.shape[0]:
                zfar.append(float(((chosen @ X) / (rr @ chosen)).max()))
            else:
                zfar.append(float(X[2]))
        tl = set(rng.choice(n_planes, size=n_textureless, replace=False).tolist()) if n_textureless else set()
        self.textured = np.array([i not in tl for i in range(n_planes)] + [True])
        self.const_val = rng.uniform(60.0, 200.0, n_planes + 1)
        # backdrop: fronto-parallel plane beyond every piece (used only when no piece is hit)
        zmax_all = max(zfar)
        normals.append(torch.tensor([0.0, 0.0, -1.0], dtype=_DT, device=device))
        points.append(torch.tensor([0.0, 0.0, 1.2 * zmax_all], dtype=_DT, device=device))
        zfar.append(1.2 * zmax_all * 1.6)
        self.n = torch.stack(normals)  # (P+1, 3)
        self.X = torch.stack(points)  # (P+1, 3)
        self.offs = (self.n * self.X).sum(1)  # n . X = offs on plane
        # in-plane texture basis
        e1s, e2s = [], []
        for i in range(n_planes + 1):
            n = self.n[i]
            a = torch.tensor([0.0, 1.0, 0.0] if abs(float(n[1])) < 0.9 else [1.0, 0.0, 0.0], dtype=_DT, device=device)
            e1 = torch.linalg.cross(n, a)
            e1 = e1 / e1.norm()
            e2 = torch.linalg.cross(n, e1)
            e1s.append(e1)
            e2s.append(e2)
        self.e1 = torch.stack(e1s)
        self.e2 = torch.stack(e2s)
        f0 = float(K0[0][0])
        self.spacing = torch.tensor([3.0 * z / f0 for z in zfar], dtype=_DT, device=device)
        self.zfar = zfar

    def _label_map(self):
        d = self.device
        lab = torch.empty((self.lh, self.lw), dtype=torch.int16, device=d)
        xs = torch.arange(self.lw, dtype=_DT, device=d) + self.lx0
        step = max(1, int(4_000_000 // self.lw))
        for y0 in range(0, self.lh, step):
            ys = torch.arange(y0, min(self.lh, y0 + step), dtype=_DT, device=d) + self.ly0
            dx = xs[None, :, None] - self.sites[None, None, :, 0]
            dy = ys[:, None, None] - self.sites[None, None, :, 1]
            lab[y0:y0 + ys.shape[0]] = (dx * dx + dy * dy).argmin(-1).to(torch.int16)
        return lab

    @staticmethod
    def _rays(Kinv, xs, ys):
        return torch.stack([Kinv[0, 0] * xs + Kinv[0, 1] * ys + Kinv[0, 2],
                            Kinv[1, 0] * xs + Kinv[1, 1] * ys + Kinv[1, 2],
                            Kinv[2, 0] * xs + Kinv[2, 1] * ys + Kinv[2, 2]], -1)

    def lookup_label(self, X):
        """Cell id of master-frame points X (..., 3) by projecting into the master view."""
        p = _apply3(self.K0, X)
        px = p[..., 0] / p[..., 2]
        py = p[..., 1] / p[..., 2]
        ix = torch.nan_to_num(torch.round(px) - self.lx0, nan=0.0).clamp(0, self.lw - 1).long()
        iy = torch.nan_to_num(torch.round(py) - self.ly0, nan=0.0).clamp(0, self.lh - 1).long()
        return self.label[iy, ix].long()

    def trace(self, origin, dirs):
        """Nearest accepted hit per ray. origin (3,), dirs (m, 3) -> plane id (m,), hit (m, 3)."""
        m = dirs.shape[0]
        best_t = torch.full((m,), float("inf"), dtype=_DT, device=self.device)
        best_i = torch.full((m,), self.P, dtype=torch.long, device=self.device)
        for i in range(self.P):
            ni = self.n[i]
            den = dirs[:, 0] * ni[0] + dirs[:, 1] * ni[1] + dirs[:, 2] * ni[2]
            num = self.offs[i] - origin @ ni
            t = num / den
            hit = origin[None, :] + t[:, None] * dirs
            ok = (t > 1e-9) & (hit[:, 2] > 1e-9) & torch.isfinite(t)
            lab = self.lookup_label(torch.where(ok[:, None], hit, torch.ones_like(hit)))
            ok = ok & (lab == i) & (t < best_t)
            best_t = torch.where(ok, t, best_t)
            best_i = torch.where(ok, torch.full_like(best_i, i), best_i)
        # backdrop for rays with no accepted piece
        nb = self.n[self.P]
        tb = (self.offs[self.P] - origin @ nb) / (dirs[:, 0] * nb[0] + dirs[:, 1] * nb[1] + dirs[:, 2] * nb[2])
        none = best_i == self.P
        best_t = torch.where(none, tb, best_t)
        hit = origin[None, :] + best_t[:, None] * dirs
        return best_i, hit

    def shade(self, pid, hit):
        """Texture value in [40, 215] (or the plane's constant) at hit points."""
        rel = hit - self.X[pid]
        u = (rel * self.e1[pid]).sum(1)
        v = (rel * self.e2[pid]).sum(1)
        sp = self.spacing[pid]
        val = torch.zeros_like(u)
        amp_sum = 0.0
        for o in range(4):
            L = sp * float(2 ** (3 - o))
            amp = 0.5 ** o
            val = val + amp * self._value_noise(pid, o, u / L, v / L)
            amp_sum += amp
        val = val / amp_sum
        # stretch the (centre-heavy) octave sum to use the range
        val = ((val - 0.5) * 2.2 + 0.5).clamp(0.0, 1.0)
        tex = 40.0 + 175.0 * val
        textured = torch.tensor(self.textured, device=self.device)[pid]
        const = torch.tensor(self.const_val, dtype=_DT, device=self.device)[pid]
        return torch.where(textured, tex, const)

    def _value_noise(self, pid, octave, u, v):
        i0 = torch.floor(u)
        j0 = torch.floor(v)
        fu = u - i0
        fv = v - j0
        i0 = i0.long()
        j0 = j0.long()
        # _mix(seed, pid, octave, i, j) with the shared stages hashed once: the
        # (seed, pid, octave) prefix per plane, the i and j stages per lattice line
        planes = torch.arange(int(pid.max().item()) + 1 if pid.numel() else 1, device=pid.device)
        prefix = _mix(self.seed, planes, octave)[pid]
        hi = [_hash32(((i0 + di) & M32) + 0x632BE5AB) for di in (0, 1)]
        hj = [_hash32(((j0 + dj) & M32) + 0x632BE5AB) for dj in (0, 1)]
        row = [_hash32(prefix ^ h) for h in hi]

        def lat(di, dj):
            return _unit(_hash32(row[di] ^ hj[dj]))

        def fade(t):
            return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

        su, sv = fade(fu), fade(fv)
        top = lat(0, 0) + su * (lat(1, 0) - lat(0, 0))
        bot = lat(0, 1) + su * (lat(1, 1) - lat(0, 1))
        return top + sv * (bot - top)


def _render(world: _World, K, R_m, C_m, w, h, view_key, noise_sigma, seed, chunk_rows=None, want_depth=False):
    """Render one camera (pose in the master frame: X_cam = R_m (X - C_m)); optionally also
    the camera-Z depth of the surface seen through each pixel centre."""
    d = world.device
    Kinv = torch.linalg.inv(torch.tensor(K, dtype=_DT, device=d))
    Rt = torch.tensor(R_m, dtype=_DT, device=d).T
    C = torch.tensor(C_m, dtype=_DT, device=d)
    img = torch.empty((h, w), dtype=_DT, device=d)
    depth = torch.empty((h, w), dtype=_DT, device=d) if want_depth else None
    Rm = torch.tensor(R_m, dtype=_DT, device=d)
    if chunk_rows is None:
        budget = 16_000_000 if str(d).startswith("cuda") else 1_000_000
        chunk_rows = max(1, int(budget // (4 * w)))
    xs = torch.arange(w, dtype=_DT, device=d)
    offsets = ((-0.25, -0.25), (-0.25, 0.25), (0.25, -0.25), (0.25, 0.25))  # (oy, ox)
    for y0 in range(0, h, chunk_rows):
        y1 = min(h, y0 + chunk_rows)
        ys = torch.arange(y0, y1, dtype=_DT, device=d)
        # the four sub-pixel samples of every pixel of the chunk in one pass
        Y = torch.stack([torch.meshgrid(ys + oy, xs + ox, indexing="ij")[0] for oy, ox in offsets])
        X = torch.stack([torch.meshgrid(ys + oy, xs + ox, indexing="ij")[1] for oy, ox in offsets])
        dirs = _apply3(Rt, _World._rays(Kinv, X, Y).reshape(-1, 3))
        pid, hit = world.trace(C, dirs)
        sub = world.shade(pid, hit).reshape(4, y1 - y0, w)
        acc = torch.zeros((y1 - y0, w), dtype=_DT, device=d)
        for k in range(4):
            acc += sub[k]
        img[y0:y1] = acc * 0.25
        if want_depth:
            Y, X = torch.meshgrid(ys, xs, indexing="ij")
            dirs = _apply3(Rt, _World._rays(Kinv, X, Y).reshape(-1, 3))
            _, hit = world.trace(C, dirs)
            rel = hit - C[None, :]
            depth[y0:y1] = (rel[:, 0] * Rm[2, 0] + rel[:, 1] * Rm[2, 1] + rel[:, 2] * Rm[2, 2]).reshape(y1 - y0, w)
    # Gaussian noise from hash uniforms (Box-Muller), round half to even, clamp
    Y, X = torch.meshgrid(torch.arange(h, device=d, dtype=torch.int64),
                          torch.arange(w, device=d, dtype=torch.int64), indexing="ij")
    u1 = _unit(_mix(seed, view_key, 0x0A11CE, X, Y)) + (0.5 / 16777216.0)
    u2 = _unit(_mix(seed, view_key, 0x0B0B, X, Y))
    g = torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)
    img = img + noise_sigma * g
    img = torch.round(img).clamp(0, 255)  # torch.round is half-to-even
    out = img.to(torch.uint8).cpu().numpy()
    if want_depth:
        return out, depth.cpu().numpy()
    return out


def _ground_truth(world: _World):
    d = world.device
    h0, w0 = world.h0, world.w0
    ys, xs = torch.meshgrid(torch.arange(h0, dtype=_DT, device=d),
                            torch.arange(w0, dtype=_DT, device=d), indexing="ij")
    lab = world.label[(ys - world.ly0).long(), (xs - world.lx0).long()].long()
    r = _World._rays(world.K0inv, xs, ys)
    n = world.n[lab]
    z = world.offs[lab] / (r * n).sum(-1) * r[..., 2]
    return z.cpu().numpy(), n.cpu().numpy(), lab.to(torch.int32).cpu().numpy()


def _default_device(device):
    if device is not None:
        return device
    return "cuda" if torch.cuda.is_available() else "cpu"


def make_scene(seed: int, cfg: SceneConfig, device=None) -> Scene:
    """Render a reference view plus ``cfg.n_src`` sources on a horizontal arc."""
    device = _default_device(device)
    w, h = cfg.width, cfg.height
    K = _intrinsics(w, h)
    ntl = cfg.n_textureless if cfg.n_textureless is not None else int(round(cfg.textureless_frac * cfg.n_planes))
    world = _World(seed, K, w, h, cfg.n_planes, ntl, cfg.site_depth_lo, cfg.site_depth_hi,
                   cfg.normal_max_deg, device)
    gt_depth, gt_normal, gt_plane = _ground_truth(world)
    dmed = float(np.median(gt_depth))
    L = np.array([0.0, 0.0, dmed])
    n = cfg.n_src
    left, right = n - n // 2, n // 2
    half = math.radians(cfg.arc_deg) / 2.0
    angles = [0.0] + [-half * i / left for i in range(1, left + 1)] + [half * i / right for i in range(1, right + 1)]
    # global rigid transform: X_world = Q X_master + q
    rng = np.random.default_rng([seed, 0x6E0])
    Q = _random_rotation(rng)
    q = rng.uniform(-5, 5, 3)
    images, cams = [], []
    for vi, a in enumerate(angles):
        Rm = _rot_y(a).T
        Cm = L + _rot_y(a) @ np.array([0.0, 0.0, -dmed])
        images.append(_render(world, K, Rm, Cm, w, h, vi, cfg.noise_sigma, seed))
        Rw = Rm @ Q.T
        tw = -Rm @ (Q.T @ q + Cm)
        cams.append(Camera(K.copy(), Rw, tw, w, h))
    d_lo = 0.9 * float(gt_depth.min())
    d_hi = 1.1 * float(gt_depth.max())
    gt_normal_cam = gt_normal  # master frame == reference camera frame
    return Scene(images, cams, (d_lo, d_hi), gt_depth, gt_normal_cam, gt_plane,
                 world.textured[:-1].copy(), seed, meta=dict(angles=angles, n_textureless=ntl))


def crop_reference(scene: Scene, width: int, height: int) -> Scene:
    """A centred crop of the reference as a separate problem instance: the reference
    image is cropped and its principal point shifted; sources stay whole."""
    H, W = scene.images[0].shape
    x0 = (W - width) // 2
    y0 = (H - height) // 2
    c0 = scene.cams[0]
    K = c0.K.copy()
    K[0, 2] -= x0
    K[1, 2] -= y0
    cams = [Camera(K, c0.R.copy(), c0.t.copy(), width, height)] + scene.cams[1:]
    images = [np.ascontiguousarray(scene.images[0][y0:y0 + height, x0:x0 + width])] + scene.images[1:]
    return Scene(images, cams, scene.depth_range,
                 scene.gt_depth[y0:y0 + height, x0:x0 + width].copy(),
                 scene.gt_normal[y0:y0 + height, x0:x0 + width].copy(),
                 scene.gt_plane[y0:y0 + height, x0:x0 + width].copy(),
                 scene.textured, scene.seed, meta=dict(scene.meta, crop=(x0, y0, width, height)))


@dataclass
class MultiViewScene:
    """Many cameras around one scene; some of them are references with their own sources."""
    images: List[np.ndarray]
    cams: List[Camera]
    depth_ranges: np.ndarray  # (n, 2) per camera
    refs: List[int]
    sources: List[List[int]]
    windows: List[tuple]  # (window, dilation) per reference
    seed: int = 0
    gt_depths: dict = field(default_factory=dict)  # reference camera -> rendered depth (H, W)

    @property
    def K(self):
        return np.stack([c.K for c in self.cams])

    @property
    def R(self):
        return np.stack([c.R for c in self.cams])

    @property
    def t(self):
        return np.stack([c.t for c in self.cams])


#: reference size classes of the batched workload: (width, height, window, dilation)
BATCH_CLASSES = [(3200, 2130, 31, 3), (1600, 1066, 21, 2), (960, 640, 11, 1)]


def make_multiview_scene(seed: int = 4, grid=(5, 8), az_deg=20.0, el_deg=8.0, n_planes=30,
                         textureless_frac=0.3, refs_per_class=8, classes=None, other_size=(1600, 1066),
                         n_src_range=(6, 12), site_depth=(2.0, 12.0), device=None,
                         master_size=(1600, 1066)) -> MultiViewScene:
    """A grid of cameras (elevations x azimuths, all looking at the centre of the scene);
    `refs_per_class` references per size class, each with 6-12 nearest cameras as sources.
    Class windows keep 11x11 taps: 31x31 at dilation 3, 21x21 at 2, 11x11 at 1."""
    device = _default_device(device)
    classes = BATCH_CLASSES if classes is None else classes
    mw, mh = master_size
    K0 = _intrinsics(mw, mh)
    ntl = int(round(textureless_frac * n_planes))
    world = _World(seed, K0, mw, mh, n_planes, ntl, site_depth[0], site_depth[1], 50.0, device)
    gt0, _, _ = _ground_truth(world)
    dmed = float(np.median(gt0))
    L = np.array([0.0, 0.0, dmed])
    n_el, n_az = grid
    rng = np.random.default_rng([seed, 0xB47C])
    n_cams = n_el * n_az
    n_refs = refs_per_class * len(classes)
    order = rng.permutation(n_cams)
    ref_ids = sorted(order[:n_refs].tolist())
    sizes = {}
    windows = {}
    for k, cam in enumerate(ref_ids):
        cls = classes[k % len(classes)]
        sizes[cam] = (cls[0], cls[1])
        windows[cam] = (cls[2], cls[3])
    dirs = []
    for ei, el in enumerate(np.linspace(-el_deg, el_deg, n_el)):
        for ai, az in enumerate(np.linspace(-az_deg, az_deg, n_az)):
            dirs.append((math.radians(az), math.radians(el)))
    Q = _random_rotation(rng)
    q = rng.uniform(-5, 5, 3)
    images, cams, dranges, gts = [], [], [], {}
    for ci, (az, el) in enumerate(dirs):
        w, h = sizes.get(ci, other_size)
        K = _intrinsics(w, h)
        Rrot = _rot_y(az) @ _rot_x(el)           # camera axes in the master frame
        Rm = Rrot.T
        Cm = L + Rrot @ np.array([0.0, 0.0, -dmed])
        img, dep = _render(world, K, Rm, Cm, w, h, ci, 2.0, seed, want_depth=True)
        images.append(img)
        good = np.isfinite(dep) & (dep > 0)
        dranges.append((0.9 * float(dep[good].min()), 1.1 * float(dep[good].max())))
        if ci in sizes:
            gts[ci] = dep.astype(np.float32)
        cams.append(Camera(K, Rm @ Q.T, -Rm @ (Q.T @ q + Cm), w, h))
    # sources: the nearest cameras by viewing direction, 6-12 of them
    centers = np.array([[math.sin(az) * math.cos(el), math.sin(el), math.cos(az) * math.cos(el)] for az, el in dirs])
    sources, wins = [], []
    for cam in ref_ids:
        nsrc = int(rng.integers(n_src_range[0], n_src_range[1] + 1))
        ang = np.arccos(np.clip(centers @ centers[cam], -1, 1))
        ang[cam] = np.inf
        sources.append(np.argsort(ang, kind="stable")[:nsrc].tolist())
        wins.append(windows[cam])
    return MultiViewScene(images, cams, np.array(dranges), ref_ids, sources, wins, seed, gts)


def workload_scene(name: str, device=None, seed: Optional[int] = None) -> Scene:
    cfg = CONFIGS[name]
    return make_scene(SCENE_SEEDS[name] if seed is None else seed, cfg, device)


def tiny_config(width=64, height=48, n_src=2, n_planes=2, n_textureless=0, lo=2.0, hi=6.0) -> SceneConfig:
    """Small scenes for CPU tests (same recipe, smaller sizes)."""
    return SceneConfig(width, height, n_src, n_planes, 0.0, lo, hi, n_textureless=n_textureless)
