"""ctypes front end of the CPU oracle (``oracle.cpp``) — TEST INFRASTRUCTURE ONLY.

The oracle is the plain statement of the PatchMatch depth-map estimation step of the
paper (Sec. III-B, Sec. III-C, Eq. 4, Eq. 5, Algorithm 1 "depth map estimation").
Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may
import this package; the GPU library never does.

Each function here marshals arguments to ``oracle.cpp``, except ``phi_select``, which
subsamples the hypothesis maps, calls the exact MAP enumeration of ``oracle.cpp`` and
brings the decoded depth back to full size in plain Python loops.

``oracle.cpp`` is built twice from the same source: ``liboracle.so`` single-threaded and
``liboracle_omp.so`` with OpenMP over the pixels of one colour (bitwise the same results,
since pixels of one colour are independent within a half-sweep).  The functions taking
``threads`` use the OpenMP build when it is above 1.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")

CMAX = 2.0


def _compile(path: str, openmp: bool, verbose: bool) -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-mfma",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas"] + (["-fopenmp"] if openmp else []) + \
          ["-o", path + ".tmp", _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(path + ".tmp", path)
    return path


def build(verbose: bool = False) -> str:
    """Compile the oracle with g++ (no fast-math, no fp contraction): the single-threaded
    library and the OpenMP build of the same source."""
    _compile(_OMP_PATH, True, verbose)
    return _compile(_LIB_PATH, False, verbose)


class _Problem(C.Structure):
    _fields_ = [
        ("n_views", C.c_int32),
        ("width", C.POINTER(C.c_int32)),
        ("height", C.POINTER(C.c_int32)),
        ("images", C.POINTER(C.POINTER(C.c_float))),
        ("K", C.POINTER(C.c_double)),
        ("R", C.POINTER(C.c_double)),
        ("t", C.POINTER(C.c_double)),
        ("d_lo", C.c_double),
        ("d_hi", C.c_double),
        ("window", C.c_int32),
        ("dilation", C.c_int32),
        ("top_k", C.c_int32),
        ("bilateral", C.c_int32),
        ("sigma_s", C.c_double),
        ("sigma_c", C.c_double),
        ("eps_v", C.c_double),
        ("eps_c", C.c_double),
        ("seed", C.c_uint64),
        ("tap_radius", C.c_int32),
        ("lanes", C.c_int32),
    ]


_libs = {}


def default_threads() -> int:
    """The host threads this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def lib(threads: int = 1):
    """The single-threaded oracle, or (threads > 1) its OpenMP build set to that many threads."""
    omp = threads > 1
    path = _OMP_PATH if omp else _LIB_PATH
    if path not in _libs:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            _compile(path, omp, False)
        L = C.CDLL(path)
        P = C.POINTER(_Problem)
        dp = C.POINTER(C.c_double)
        fp = C.POINTER(C.c_float)
        ip = C.POINTER(C.c_int32)
        up = C.POINTER(C.c_uint32)
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = C.c_int
        L.oracle_philox4x32_10.argtypes = [up, up, up]
        L.oracle_patchmatch.argtypes = [P, C.c_int, C.c_int, fp, fp, fp]
        L.oracle_init.argtypes = [P, C.c_int, dp, dp]
        L.oracle_halfsweep.argtypes = [P, C.c_int, C.c_int, C.c_int, dp, dp, ip, C.c_int, C.c_int, C.c_int]
        L.oracle_eval_cost.argtypes = [P, C.c_int, dp, dp, dp, ip, ip, C.c_int]
        L.oracle_homography.argtypes = [P, C.c_int, dp, C.c_double, C.c_int, C.c_int, dp]
        L.oracle_bilinear.argtypes = [fp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int]
        L.oracle_bilinear.restype = C.c_double
        L.oracle_aggregate.argtypes = [dp, ip, C.c_int, C.c_int, C.c_double, C.c_int]
        L.oracle_aggregate.restype = C.c_double
        L.oracle_consistency.argtypes = [C.c_int, ip, ip, dp, dp, dp, C.POINTER(fp), C.POINTER(fp), C.c_int, ip,
                                         C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, fp, fp,
                                         C.POINTER(C.c_uint8)]
        L.oracle_phi_hypotheses.argtypes = [fp, C.c_int, C.c_int, fp]
        L.oracle_phi_hypotheses.restype = None
        L.oracle_phi_map_bruteforce.argtypes = [fp, fp, fp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                                C.c_double, ip]
        L.oracle_phi_map_bruteforce.restype = C.c_double
        L.oracle_phi_trws.argtypes = [fp, fp, fp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_int, ip, fp]
        L.oracle_phi_trws.restype = None
        L.oracle_phi_normals.argtypes = [fp, C.c_int, C.c_int, dp, fp]
        L.oracle_fuse.argtypes = [C.c_int, ip, ip, dp, dp, dp, C.POINTER(fp), C.c_double, fp, ip,
                                  C.POINTER(C.c_int64)]
        for f in ("oracle_patchmatch", "oracle_init", "oracle_halfsweep", "oracle_eval_cost", "oracle_homography",
                  "oracle_consistency", "oracle_phi_normals", "oracle_fuse"):
            getattr(L, f).restype = C.c_int
        _libs[path] = L
    L = _libs[path]
    if omp:
        L.oracle_set_threads(int(threads))
    return L


def threads_in_effect(threads: int) -> int:
    """How many threads a call with ``threads`` runs on (1 for the single-threaded build)."""
    return int(lib(threads).oracle_set_threads(int(threads) if threads > 1 else 0))


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Problem:
    """A reference view (index 0) plus sources, with cameras and solver parameters."""

    def __init__(self, images: Sequence[np.ndarray], K, R, t, depth_range, window: int, dilation: int,
                 top_k: int = 0, bilateral: bool = True, sigma_s: Optional[float] = None,
                 sigma_c: float = 12.0, eps_v: float = 1e-4, eps_c: float = 1e-4, seed: int = 0x5EED,
                 tap_radius: int = 0, lanes: int = 1):
        self.images = [np.ascontiguousarray(im, dtype=np.float32) for im in images]
        n = len(self.images)
        self.K = np.ascontiguousarray(np.asarray(K, dtype=np.float64).reshape(n, 9))
        self.R = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(n, 9))
        self.t = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(n, 3))
        self.w = np.array([im.shape[1] for im in self.images], dtype=np.int32)
        self.h = np.array([im.shape[0] for im in self.images], dtype=np.int32)
        self._imgptrs = (C.POINTER(C.c_float) * n)(*[_ptr(im, C.c_float) for im in self.images])
        if sigma_s is None:
            sigma_s = (window - 1) / 2.0
        self.window, self.dilation, self.top_k, self.tap_radius = window, dilation, top_k, tap_radius
        self.lanes = lanes
        self.s = _Problem(n, _ptr(self.w, C.c_int32), _ptr(self.h, C.c_int32), self._imgptrs,
                          _ptr(self.K, C.c_double), _ptr(self.R, C.c_double), _ptr(self.t, C.c_double),
                          float(depth_range[0]), float(depth_range[1]), window, dilation, top_k,
                          1 if bilateral else 0, float(sigma_s), float(sigma_c), float(eps_v), float(eps_c),
                          int(seed) & 0xFFFFFFFFFFFFFFFF, int(tap_radius), int(lanes))

    @property
    def W(self):
        return int(self.w[0])

    @property
    def H(self):
        return int(self.h[0])

    @property
    def n_src(self):
        return len(self.images) - 1

    @classmethod
    def from_scene(cls, scene, window, dilation, top_k=0, **kw):
        return cls(scene.images, scene.K, scene.R, scene.t, scene.depth_range, window, dilation, top_k, **kw)

    def radius(self):
        if self.tap_radius > 0:
            return (self.window - 1) // 2
        return self.dilation * ((self.window - 1) // (2 * self.dilation))

    def valid_mask(self):
        r = self.radius()
        m = np.zeros((self.H, self.W), dtype=bool)
        if self.H - 2 * r > 0 and self.W - 2 * r > 0:
            m[r:self.H - r, r:self.W - r] = True
        return m


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def patchmatch(pb: Problem, iters: int, fp64: bool = False, threads: int = 1):
    """Full run -> (depth (H,W), normal (H,W,3), cost (H,W)) float32."""
    H, W = pb.H, pb.W
    d = np.zeros((H, W), np.float32)
    n = np.zeros((H, W, 3), np.float32)
    c = np.zeros((H, W), np.float32)
    rc = lib(threads).oracle_patchmatch(C.byref(pb.s), iters, int(fp64), _ptr(d, C.c_float), _ptr(n, C.c_float),
                                 _ptr(c, C.c_float))
    if rc != 0:
        raise ValueError("oracle_patchmatch failed (singular reference K?)")
    return d, n, c


def init(pb: Problem, fp64: bool = False, threads: int = 1):
    planes = np.zeros((pb.H, pb.W, 4), np.float64)
    cost = np.zeros((pb.H, pb.W), np.float64)
    if lib(threads).oracle_init(C.byref(pb.s), int(fp64), _ptr(planes, C.c_double), _ptr(cost, C.c_double)) != 0:
        raise ValueError("oracle_init failed")
    return planes, cost


def halfsweep(pb: Problem, planes, cost, iteration: int, colour: int, fp64: bool = False, subset=None,
              propagate: bool = True, refine: bool = True, threads: int = 1):
    P = np.ascontiguousarray(planes, dtype=np.float64).copy()
    Cc = np.ascontiguousarray(cost, dtype=np.float64).copy()
    sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int32)
    rc = lib(threads).oracle_halfsweep(C.byref(pb.s), iteration, colour, int(fp64), _ptr(P, C.c_double),
                                _ptr(Cc, C.c_double), None if sub is None else _ptr(sub, C.c_int32),
                                0 if sub is None else len(sub), int(propagate), int(refine))
    if rc != 0:
        raise ValueError("oracle_halfsweep failed")
    return P, Cc


def eval_cost(pb: Problem, planes, fp64: bool = False, subset=None, threads: int = 1):
    """Cost of the given planes -> (cost (H,W), per_view (H,W,n_src), valid (H,W,n_src))."""
    P = np.ascontiguousarray(planes, dtype=np.float64)
    H, W, n = pb.H, pb.W, pb.n_src
    cost = np.full((H, W), CMAX, np.float64)
    pv = np.full((H, W, n), CMAX, np.float64)
    ok = np.zeros((H, W, n), np.int32)
    sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int32)
    rc = lib(threads).oracle_eval_cost(C.byref(pb.s), int(fp64), _ptr(P, C.c_double), _ptr(cost, C.c_double),
                                _ptr(pv, C.c_double), _ptr(ok, C.c_int32),
                                None if sub is None else _ptr(sub, C.c_int32), 0 if sub is None else len(sub))
    if rc != 0:
        raise ValueError("oracle_eval_cost failed")
    return cost, pv, ok.astype(bool)


def homography(pb: Problem, j: int, n, d: float, x: int, y: int):
    nn = np.ascontiguousarray(n, dtype=np.float64)
    Hm = np.zeros(9, np.float64)
    lib().oracle_homography(C.byref(pb.s), j, _ptr(nn, C.c_double), float(d), int(x), int(y), _ptr(Hm, C.c_double))
    return Hm.reshape(3, 3)


def bilinear(img, u: float, v: float, fp64: bool = True) -> float:
    im = np.ascontiguousarray(img, dtype=np.float32)
    return lib().oracle_bilinear(_ptr(im, C.c_float), im.shape[1], im.shape[0], float(u), float(v), int(fp64))


def aggregate(cj, valid, top_k: int = 0, eps_c: float = 1e-4, fp64: bool = True) -> float:
    c = np.ascontiguousarray(cj, dtype=np.float64)
    v = np.ascontiguousarray(valid, dtype=np.int32)
    return lib().oracle_aggregate(_ptr(c, C.c_double), _ptr(v, C.c_int32), len(c), top_k, eps_c, int(fp64))


def consistency(depths, normals, K, R, t, ref: int, nbrs, tau_d: float = 0.02, tau_n_deg: float = 30.0,
                tau_r: float = 1.0, min_consistent: int = 2):
    """Geometric-consistency filter of view ``ref`` (Sec. III-D).  depths / normals: dicts
    view -> (H, W) / (H, W, 3) float32 maps; K, R: (n, 3, 3), t: (n, 3) for all n views.
    -> (depth, normal, count) of the reference: kept values or zeros, consistent neighbours."""
    n = len(K)
    W = np.zeros(n, np.int32)
    H = np.zeros(n, np.int32)
    keep = []
    dptr = (C.POINTER(C.c_float) * n)()
    nptr = (C.POINTER(C.c_float) * n)()
    for v in range(n):
        if v in depths:
            d = np.ascontiguousarray(depths[v], dtype=np.float32)
            nm = np.ascontiguousarray(normals[v], dtype=np.float32)
            keep += [d, nm]
            H[v], W[v] = d.shape
            dptr[v] = _ptr(d, C.c_float)
            nptr[v] = _ptr(nm, C.c_float)
    Kd = np.ascontiguousarray(np.asarray(K, np.float64).reshape(n, 9))
    Rd = np.ascontiguousarray(np.asarray(R, np.float64).reshape(n, 9))
    td = np.ascontiguousarray(np.asarray(t, np.float64).reshape(n, 3))
    nb = np.ascontiguousarray(nbrs, dtype=np.int32)
    Hr, Wr = int(H[ref]), int(W[ref])
    # every output element is written by the oracle: NaN / 255 beforehand would show one that is not
    od = np.full((Hr, Wr), np.nan, np.float32)
    on = np.full((Hr, Wr, 3), np.nan, np.float32)
    oc = np.full((Hr, Wr), 255, np.uint8)
    rc = lib().oracle_consistency(n, _ptr(W, C.c_int32), _ptr(H, C.c_int32), _ptr(Kd, C.c_double),
                                  _ptr(Rd, C.c_double), _ptr(td, C.c_double), dptr, nptr, ref, _ptr(nb, C.c_int32),
                                  len(nb), tau_d, tau_n_deg, tau_r, min_consistent, _ptr(od, C.c_float),
                                  _ptr(on, C.c_float), _ptr(oc, C.c_uint8))
    if rc != 0:
        raise ValueError("oracle_consistency failed (bad view, neighbour or camera)")
    return od, on, oc


def fuse(depths, K, R, t, max_rel_dist: float = 0.01):
    """Depth-map fusion (Sec. III-F) of the maps in the order given.  depths: list of
    (H_i, W_i) float32 maps (<= 0: no depth); K, R: (n, 3, 3), t: (n, 3) of those maps'
    cameras.  -> (points (P, 3) float32, support (P,) int32, owner (P,) int64) over the
    concatenated pixels (P = sum of H_i W_i; map i at the offset of the earlier maps)."""
    n = len(depths)
    W = np.array([d.shape[1] for d in depths], np.int32)
    H = np.array([d.shape[0] for d in depths], np.int32)
    keep = [np.ascontiguousarray(d, dtype=np.float32) for d in depths]
    dptr = (C.POINTER(C.c_float) * n)(*[_ptr(d, C.c_float) for d in keep])
    Kd = np.ascontiguousarray(np.asarray(K, np.float64).reshape(n, 9))
    Rd = np.ascontiguousarray(np.asarray(R, np.float64).reshape(n, 9))
    td = np.ascontiguousarray(np.asarray(t, np.float64).reshape(n, 3))
    P = int((W.astype(np.int64) * H).sum())
    pts = np.zeros((P, 3), np.float32)
    sup = np.zeros(P, np.int32)
    own = np.zeros(P, np.int64)
    rc = lib().oracle_fuse(n, _ptr(W, C.c_int32), _ptr(H, C.c_int32), _ptr(Kd, C.c_double), _ptr(Rd, C.c_double),
                           _ptr(td, C.c_double), dptr, float(max_rel_dist), _ptr(pts, C.c_float),
                           _ptr(sup, C.c_int32), _ptr(own, C.c_int64))
    if rc != 0:
        raise ValueError("oracle_fuse failed (bad map or camera)")
    return pts, sup, own


def phi_hypotheses(depth):
    """Plane-hypothesis depths (Sec. III-E) of the pixels without depth: (H, W, 4), 0 = none."""
    d = np.ascontiguousarray(depth, dtype=np.float32)
    H, W = d.shape
    hyp = np.full((H, W, 4), np.nan, np.float32)  # every element is written
    lib().oracle_phi_hypotheses(_ptr(d, C.c_float), W, H, _ptr(hyp, C.c_float))
    return hyp


def phi_map_bruteforce(depth, hyp, cost, k1: float, k2: float, k3: float, cmax: float = CMAX):
    """Exact MAP labelling of the pairwise model of Sec. III-E on a tiny grid -> (labels (H, W), log potential)."""
    d = np.ascontiguousarray(depth, dtype=np.float32)
    h = np.ascontiguousarray(hyp, dtype=np.float32)
    c = np.ascontiguousarray(cost, dtype=np.float32)
    H, W = d.shape
    lab = np.zeros((H, W), np.int32)
    e = lib().oracle_phi_map_bruteforce(_ptr(d, C.c_float), _ptr(h, C.c_float), _ptr(c, C.c_float), W, H, k1, k2, k3,
                                        cmax, _ptr(lab, C.c_int32))
    return lab, e


def phi_normals(depth, K):
    """Normals of Eq. 10 from a depth map (H, W) and intrinsics K -> (H, W, 3), 0 where undefined."""
    d = np.ascontiguousarray(depth, dtype=np.float32)
    Kd = np.ascontiguousarray(np.asarray(K, np.float64).reshape(9))
    H, W = d.shape
    n = np.full((H, W, 3), np.nan, np.float32)  # every element is written
    if lib().oracle_phi_normals(_ptr(d, C.c_float), W, H, _ptr(Kd, C.c_double), _ptr(n, C.c_float)) != 0:
        raise ValueError("singular K")
    return n


def phi_trws(depth, hyp, cost, k1: float = 1.0, k2: float = 0.1, k3: float = 2.0, cmax: float = CMAX,
             iterations: int = 8):
    """Sequential TRW decoding of the pairwise model of Sec. III-E (the paper's decoder)
    -> (labels (H, W) int32, -1 = fixed or no state; depth (H, W) float32, 0 = no state)."""
    d = np.ascontiguousarray(depth, dtype=np.float32)
    h = np.ascontiguousarray(hyp, dtype=np.float32)
    c = np.ascontiguousarray(cost, dtype=np.float32)
    H, W = d.shape
    lab = np.zeros((H, W), np.int32)
    val = np.full((H, W), np.nan, np.float32)  # every element is written
    lib().oracle_phi_trws(_ptr(d, C.c_float), _ptr(h, C.c_float), _ptr(c, C.c_float), W, H, k1, k2, k3, cmax,
                          int(iterations), _ptr(lab, C.c_int32), _ptr(val, C.c_float))
    return lab, val


def phi_select(depth, hyp, cost, k1: float = 1.0, k2: float = 0.1, k3: float = 2.0, cmax: float = CMAX,
               iterations=None):
    """Selection step of Sec. III-E: the hypothesis maps (H, W, 4) are subsampled to half
    size (node (X, Y) <- pixel (2X, 2Y)), the graph model is decoded (iterations None: the
    exact MAP by enumeration, for tiny maps; else that many TRW iterations), the decoded
    depth is brought back to full size (pixel (x, y) <- node (x // 2, y // 2)) as the
    reference map, and each pixel without depth takes its hypothesis closest to the
    reference (lowest k on ties; none without hypothesis or reference).  -> depth (H, W)
    float32."""
    d = np.asarray(depth, np.float32)
    h = np.asarray(hyp, np.float32)
    c = np.asarray(cost, np.float32)
    d2, h2, c2 = d[::2, ::2], h[::2, ::2], c[::2, ::2]
    if iterations is None:
        lab, _ = phi_map_bruteforce(d2, h2, c2, k1, k2, k3, cmax)
        fixed = d2 > 0
        picked = np.take_along_axis(h2, np.maximum(lab, 0)[..., None], 2)[..., 0]
        dec = np.where(fixed, d2, np.where(lab >= 0, picked, 0.0)).astype(np.float32)
    else:
        _, dec = phi_trws(d2, h2, c2, k1, k2, k3, cmax, iterations)
    H, W = d.shape
    ref = dec[np.arange(H)[:, None] // 2, np.arange(W)[None, :] // 2].astype(np.float64)
    # distance of each hypothesis to the reference; a missing hypothesis never wins
    dist = np.where(h > 0, np.abs(h.astype(np.float64) - ref[..., None]), np.inf)
    k = np.argmin(dist, axis=2)  # the first of equal distances: lowest k
    best = np.take_along_axis(h, k[..., None], 2)[..., 0]
    usable = (ref > 0) & np.isfinite(np.take_along_axis(dist, k[..., None], 2)[..., 0])
    out = np.where(d > 0, d, np.where(usable, best, 0.0)).astype(np.float32)
    return out
