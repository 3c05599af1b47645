"""Python binding of the MI355X PatchMatch multi-view stereo library (``libphimvs.so``).

Argument marshalling only: every step of the depth-map estimation runs in the HIP
kernels behind the C ABI declared in ``include/phimvs.h``.  Device buffers are torch
tensors on the context's GPU; work is issued on torch's current stream.  Importing
this package does not need a GPU, but creating a ``Context`` does, and a missing or
unbuilt library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphimvs.so")

PHIMVS_OK = 0
ERRORS = {-1: "PHIMVS_E_ARG", -2: "PHIMVS_E_STATE", -3: "PHIMVS_E_DEVICE", -4: "PHIMVS_E_OOM",
          -5: "PHIMVS_E_UNSUPPORTED"}
COST_MAX = 2.0
MAX_SOURCES = 12

#: every symbol the C ABI exports (include/phimvs.h)
EXPORTS = ("phimvs_default_params", "phimvs_create", "phimvs_destroy", "phimvs_last_error", "phimvs_set_stream",
           "phimvs_sync", "phimvs_set_views", "phimvs_patchmatch", "phimvs_prepare", "phimvs_init_planes",
           "phimvs_step", "phimvs_get_state", "phimvs_set_state", "phimvs_output", "phimvs_eval_cost",
           "phimvs_patchmatch_batch", "phimvs_set_tuning", "phimvs_get_tuning", "phimvs_autotune",
           "phimvs_diag_enable", "phimvs_diag_read", "phimvs_check_reciprocal",
           "phimvs_default_filter_params", "phimvs_filter", "phimvs_default_fuse_params", "phimvs_fuse",
           "phimvs_phi_hypotheses", "phimvs_phi_hypotheses_noalloc", "phimvs_phi_costs", "phimvs_default_phi_params",
           "phimvs_phi_select", "phimvs_phi_decode_host", "phimvs_phi_normals",
           # learned initial-plane proposal (include/phimvs_net.h)
           "phimvs_net_create", "phimvs_net_destroy", "phimvs_net_last_error", "phimvs_net_set_stream",
           "phimvs_net_param_count", "phimvs_net_set_params", "phimvs_net_get_params", "phimvs_net_forward",
           "phimvs_net_loss_grad", "phimvs_net_adam", "phimvs_net_inputs", "phimvs_net_propose",
           "phimvs_net_decode", "phimvs_net_targets", "phimvs_net_tensor", "phimvs_patchmatch_proposal")
DIAG_COUNT = 1
DIAG_TIME = 2


class PhimvsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Image(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("stride_bytes", C.c_int64), ("dtype", C.c_int32),
                ("data", C.c_void_p), ("on_device", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("top_k", C.c_int32), ("bilateral", C.c_int32), ("sigma_spatial_px", C.c_double),
                ("sigma_color", C.c_double), ("eps_var", C.c_double), ("eps_cost", C.c_double),
                ("seed", C.c_uint64), ("tap_radius", C.c_int32), ("lanes", C.c_int32),
                ("score_all", C.c_int32)]


class _Job(C.Structure):
    _fields_ = [("ref", C.c_int32), ("srcs", C.POINTER(C.c_int32)), ("n_srcs", C.c_int32), ("window", C.c_int32),
                ("dilation", C.c_int32), ("params", _Params), ("depth", C.c_void_p), ("normal", C.c_void_p),
                ("cost", C.c_void_p)]


class _Tuning(C.Structure):
    _fields_ = [("tile_rows", C.c_int32), ("persistent", C.c_int32), ("wgs_per_cu", C.c_int32),
                ("order_by_depth", C.c_int32), ("ms", C.c_double)]


class _DepthMap(C.Structure):
    _fields_ = [("view", C.c_int32), ("depth", C.c_void_p), ("normal", C.c_void_p)]


class _FilterParams(C.Structure):
    _fields_ = [("max_rel_depth", C.c_double), ("max_angle_deg", C.c_double), ("max_reproj_px", C.c_double),
                ("min_consistent", C.c_int32)]


@dataclass
class FilterParams:
    """Thresholds of the geometric-consistency filter (include/phimvs.h)."""
    max_rel_depth: float = 0.02
    max_angle_deg: float = 30.0
    max_reproj_px: float = 1.0
    min_consistent: int = 2


class _FuseParams(C.Structure):
    _fields_ = [("max_rel_dist", C.c_double)]


class _PhiParams(C.Structure):
    _fields_ = [("k1", C.c_double), ("k2", C.c_double), ("k3", C.c_double), ("iterations", C.c_int32)]


@dataclass
class PhiParams:
    """Potentials and decoder sweeps of plane hypothesis inference (include/phimvs.h)."""
    k1: float = 1.0
    k2: float = 0.1
    k3: float = 2.0
    iterations: int = 8

    def _c(self):
        return _PhiParams(self.k1, self.k2, self.k3, self.iterations)


@dataclass
class Tuning:
    tile_rows: int = 4
    persistent: bool = False
    wgs_per_cu: int = 0
    ms: float = 0.0
    order_by_depth: int = 0  # mask: 1 initialisation, 2 propagation, 4 refinement (True: all)


@dataclass
class Params:
    top_k: int = 0
    bilateral: bool = True
    sigma_spatial_px: float = 0.0  # <= 0: the window radius
    sigma_color: float = 12.0
    eps_var: float = 1e-4
    eps_cost: float = 1e-4
    seed: int = 0x5EED
    tap_radius: int = 0  # > 0: the window-resize scheme with this many taps per side
    lanes: int = 0  # 2..16: that many lanes share each pixel (split tap sums), for small references
    score_all: int = 0  # 0: leave out candidates that cannot win; 1: not those offered before; 2: none

    def _c(self) -> _Params:
        return _Params(int(self.top_k), 1 if self.bilateral else 0, float(self.sigma_spatial_px),
                       float(self.sigma_color), float(self.eps_var), float(self.eps_cost),
                       int(self.seed) & 0xFFFFFFFFFFFFFFFF, int(self.tap_radius), int(self.lanes),
                       int(self.score_all))


_lib = None


def lib():
    """Load libphimvs.so (built by ``paper_2104_06165_amd.build``); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2104_06165_amd.build` "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        vp, ip, fp, dp = C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_double)
        L.phimvs_default_params.argtypes = [C.POINTER(_Params)]
        L.phimvs_default_params.restype = None
        L.phimvs_create.argtypes = [C.POINTER(vp), ip, vp]
        L.phimvs_destroy.argtypes = [vp]
        L.phimvs_destroy.restype = None
        L.phimvs_last_error.argtypes = [vp]
        L.phimvs_last_error.restype = C.c_char_p
        L.phimvs_set_stream.argtypes = [vp, vp]
        L.phimvs_sync.argtypes = [vp]
        L.phimvs_set_views.argtypes = [vp, ip, C.POINTER(_Image), dp, dp, dp, dp]
        L.phimvs_patchmatch.argtypes = [vp, ip, C.POINTER(C.c_int), ip, ip, ip, ip, C.POINTER(_Params), fp, fp, fp, ip]
        L.phimvs_prepare.argtypes = [vp, ip, C.POINTER(C.c_int), ip, ip, ip, C.POINTER(_Params)]
        L.phimvs_init_planes.argtypes = [vp, fp, ip]
        L.phimvs_step.argtypes = [vp, ip, ip, ip, ip]
        L.phimvs_get_state.argtypes = [vp, fp, fp, ip]
        L.phimvs_set_state.argtypes = [vp, fp, fp, ip]
        L.phimvs_output.argtypes = [vp, fp, fp, fp, ip]
        L.phimvs_eval_cost.argtypes = [vp, fp, fp, fp, vp, ip]
        L.phimvs_patchmatch_batch.argtypes = [vp, ip, C.POINTER(_Job), ip, ip]
        L.phimvs_set_tuning.argtypes = [vp, C.POINTER(_Tuning)]
        L.phimvs_get_tuning.argtypes = [vp, C.POINTER(_Tuning)]
        L.phimvs_autotune.argtypes = [vp, ip, C.POINTER(_Job), ip, C.POINTER(_Tuning), C.POINTER(C.c_int)]
        L.phimvs_diag_enable.argtypes = [vp, ip]
        L.phimvs_diag_read.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_double)]
        L.phimvs_check_reciprocal.argtypes = [vp, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint64),
                                              C.POINTER(C.c_uint32)]
        L.phimvs_default_filter_params.argtypes = [C.POINTER(_FilterParams)]
        L.phimvs_default_filter_params.restype = None
        L.phimvs_filter.argtypes = [vp, ip, C.POINTER(_DepthMap), ip, C.POINTER(C.c_int32), ip,
                                    C.POINTER(_FilterParams), fp, fp, vp]
        L.phimvs_default_fuse_params.argtypes = [C.POINTER(_FuseParams)]
        L.phimvs_default_fuse_params.restype = None
        L.phimvs_fuse.argtypes = [vp, ip, C.POINTER(_DepthMap), C.POINTER(_FuseParams), fp, fp, fp]
        L.phimvs_phi_hypotheses.argtypes = [vp, ip, ip, fp, fp]
        L.phimvs_phi_hypotheses_noalloc.argtypes = [vp, ip, ip, fp, fp]
        L.phimvs_phi_costs.argtypes = [vp, fp, fp]
        L.phimvs_default_phi_params.argtypes = [C.POINTER(_PhiParams)]
        L.phimvs_default_phi_params.restype = None
        L.phimvs_phi_select.argtypes = [vp, ip, ip, fp, fp, fp, C.POINTER(_PhiParams), fp]
        L.phimvs_phi_decode_host.argtypes = [ip, ip, fp, fp, fp, C.c_double, C.c_double, C.c_double, C.c_double, ip,
                                             vp, vp]
        L.phimvs_phi_normals.argtypes = [vp, ip, fp, fp]
        L.phimvs_net_create.argtypes = [C.POINTER(vp), ip, vp]
        L.phimvs_net_destroy.argtypes = [vp]
        L.phimvs_net_destroy.restype = None
        L.phimvs_net_last_error.argtypes = [vp]
        L.phimvs_net_last_error.restype = C.c_char_p
        L.phimvs_net_set_stream.argtypes = [vp, vp]
        L.phimvs_net_param_count.argtypes = []
        L.phimvs_net_set_params.argtypes = [vp, fp, ip]
        L.phimvs_net_get_params.argtypes = [vp, fp, ip]
        L.phimvs_net_forward.argtypes = [vp, ip, ip, ip, fp, fp]
        L.phimvs_net_loss_grad.argtypes = [vp, ip, ip, ip, fp, fp, fp, fp, C.c_float, dp, fp]
        L.phimvs_net_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
        L.phimvs_net_tensor.argtypes = [vp, ip, ip, fp]
        L.phimvs_net_inputs.argtypes = [vp, vp, ip, C.POINTER(C.c_int), ip, fp]
        L.phimvs_net_propose.argtypes = [vp, vp, ip, C.POINTER(C.c_int), ip, fp]
        L.phimvs_net_decode.argtypes = [vp, vp, ip, fp, fp]
        L.phimvs_net_targets.argtypes = [vp, ip, ip, fp, fp, fp, C.c_float, fp, fp]
        L.phimvs_patchmatch_proposal.argtypes = [vp, ip, C.POINTER(C.c_int), ip, ip, ip, ip, C.POINTER(_Params),
                                                 fp, fp, fp, fp, ip]
        for name in EXPORTS:
            f = getattr(L, name)
            if name not in ("phimvs_default_params", "phimvs_destroy", "phimvs_last_error", "phimvs_net_destroy",
                            "phimvs_net_last_error", "phimvs_default_filter_params", "phimvs_default_phi_params",
                  "phimvs_default_fuse_params"):
                f.restype = C.c_int
        L.phimvs_net_param_count.restype = C.c_int64
        _lib = L
    return _lib


def default_params() -> Params:
    p = _Params()
    lib().phimvs_default_params(C.byref(p))
    return Params(p.top_k, bool(p.bilateral), p.sigma_spatial_px, p.sigma_color, p.eps_var, p.eps_cost, p.seed,
                  p.tap_radius, p.lanes, p.score_all)


def _dptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Context:
    """One library context on one GPU, issuing work on torch's current stream."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        torch.cuda.init()
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
        rc = lib().phimvs_create(C.byref(h), device, C.c_void_p(stream))
        if rc != PHIMVS_OK:
            raise PhimvsError(rc, "phimvs_create failed")
        self.h = h
        self.W = self.H = None
        self.n_src = None
        self.views = []

    def close(self):
        if getattr(self, "h", None):
            lib().phimvs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != PHIMVS_OK:
            raise PhimvsError(rc, lib().phimvs_last_error(self.h).decode())

    def _sync_stream(self):
        s = self.torch.cuda.current_stream(self.device).cuda_stream
        self._check(lib().phimvs_set_stream(self.h, C.c_void_p(s)))

    # ------------------------------------------------------------------ scene
    def set_views(self, images: Sequence, K, R, t, depth_ranges):
        """images: uint8 arrays (H, W) (numpy on the host, or torch on this device)."""
        self._sync_stream()
        n = len(images)
        ims = (_Image * n)()
        keep = []
        for i, im in enumerate(images):
            if isinstance(im, np.ndarray):
                a = np.ascontiguousarray(im, dtype=np.uint8)
                keep.append(a)
                ims[i] = _Image(a.shape[1], a.shape[0], 0, 0, a.ctypes.data, 0)
            else:
                a = im.contiguous()
                if a.dtype != self.torch.uint8:
                    raise TypeError("images must be uint8")
                keep.append(a)
                ims[i] = _Image(a.shape[1], a.shape[0], 0, 0, a.data_ptr(), 1)
        Kd = np.ascontiguousarray(np.asarray(K, dtype=np.float64).reshape(n, 9))
        Rd = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(n, 9))
        td = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(n, 3))
        dr = np.ascontiguousarray(np.asarray(depth_ranges, dtype=np.float64).reshape(n, 2))
        dp = C.POINTER(C.c_double)
        self._check(lib().phimvs_set_views(self.h, n, ims, Kd.ctypes.data_as(dp), Rd.ctypes.data_as(dp),
                                           td.ctypes.data_as(dp), dr.ctypes.data_as(dp)))
        self.views = [(int(a.shape[0]), int(a.shape[1])) for a in keep]

    def set_scene(self, scene):
        """Upload a ``scenegen.Scene`` (every view uses the scene's depth range)."""
        n = len(scene.images)
        self.set_views(scene.images, scene.K, scene.R, scene.t, np.tile(np.asarray(scene.depth_range), (n, 1)))

    # ------------------------------------------------------------------ full run
    def patchmatch(self, ref: int, srcs: Sequence[int], window: int, dilation: int, iters: int,
                   params: Optional[Params] = None, out=None):
        """-> (depth (H, W), normal (H, W, 3), cost (H, W)) float32 tensors on the device."""
        torch = self.torch
        self._sync_stream()
        # an out-of-range ref is the library's to reject (PHIMVS_E_ARG)
        H, W = self.views[ref] if 0 <= ref < len(self.views) else (1, 1)
        if out is None:
            out = (torch.empty((H, W), dtype=torch.float32, device=self.device),
                   torch.empty((H, W, 3), dtype=torch.float32, device=self.device),
                   torch.empty((H, W), dtype=torch.float32, device=self.device))
        sa = (C.c_int * len(srcs))(*srcs)
        p = (params or default_params())._c()
        self._check(lib().phimvs_patchmatch(self.h, ref, sa, len(srcs), window, dilation, iters, C.byref(p),
                                            out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), 1))
        return out

    def patchmatch_proposal(self, ref: int, srcs: Sequence[int], window: int, dilation: int, iters: int,
                            proposal, params: Optional[Params] = None, out=None):
        """``patchmatch`` with the random initialisation gated by proposal planes (H, W, 4) on the device."""
        torch = self.torch
        self._sync_stream()
        H, W = self.views[ref] if 0 <= ref < len(self.views) else (1, 1)
        if out is None:
            out = (torch.empty((H, W), dtype=torch.float32, device=self.device),
                   torch.empty((H, W, 3), dtype=torch.float32, device=self.device),
                   torch.empty((H, W), dtype=torch.float32, device=self.device))
        if proposal.dtype != torch.float32 or not proposal.is_contiguous() or proposal.numel() != H * W * 4:
            raise ValueError("proposal must be a contiguous float32 (H, W, 4) tensor")
        sa = (C.c_int * len(srcs))(*srcs)
        p = (params or default_params())._c()
        self._check(lib().phimvs_patchmatch_proposal(self.h, ref, sa, len(srcs), window, dilation, iters, C.byref(p),
                                                     proposal.data_ptr(), out[0].data_ptr(), out[1].data_ptr(),
                                                     out[2].data_ptr(), 1))
        return out

    # ------------------------------------------------------------------ consistency filter
    def filter(self, maps, ref_map: int, nbrs: Sequence[int], params: Optional[FilterParams] = None):
        """Geometric-consistency filter of maps[ref_map] against maps[nbrs].  maps: list of
        (view, depth (H, W), normal (H, W, 3)) device tensors.  -> (depth, normal, count)."""
        torch = self.torch
        self._sync_stream()
        arr = (_DepthMap * len(maps))()
        for i, (v, d, n) in enumerate(maps):
            if d.dtype != torch.float32 or n.dtype != torch.float32 or not d.is_contiguous() or not n.is_contiguous():
                raise ValueError("depth / normal maps must be contiguous float32 tensors")
            arr[i] = _DepthMap(int(v), d.data_ptr(), n.data_ptr())
        v0 = maps[ref_map][0] if 0 <= ref_map < len(maps) else -1
        H, W = self.views[v0] if 0 <= v0 < len(self.views) else (1, 1)
        od = torch.empty((H, W), dtype=torch.float32, device=self.device)
        on = torch.empty((H, W, 3), dtype=torch.float32, device=self.device)
        oc = torch.empty((H, W), dtype=torch.uint8, device=self.device)
        nb = (C.c_int32 * max(len(nbrs), 1))(*nbrs)
        fp_ = params or FilterParams()
        cp = _FilterParams(fp_.max_rel_depth, fp_.max_angle_deg, fp_.max_reproj_px, fp_.min_consistent)
        self._check(lib().phimvs_filter(self.h, len(maps), arr, ref_map, nb, len(nbrs), C.byref(cp), od.data_ptr(),
                                        on.data_ptr(), oc.data_ptr()))
        return od, on, oc

    # ------------------------------------------------------------------ depth-map fusion
    def fuse(self, maps, max_rel_dist: float = 0.01):
        """Depth-map fusion of the maps in the order given.  maps: list of (view, depth (H, W))
        device tensors.  -> (points (P, 3) float32, support (P,) int32, owner (P,) int64) over
        the concatenated pixels (map k after the pixels of maps 0..k-1)."""
        torch = self.torch
        self._sync_stream()
        arr = (_DepthMap * max(len(maps), 1))()
        P = 0
        for i, (v, d) in enumerate(maps):
            if d.dtype != torch.float32 or not d.is_contiguous():
                raise ValueError("depth maps must be contiguous float32 tensors")
            arr[i] = _DepthMap(int(v), d.data_ptr(), None)
            if 0 <= int(v) < len(self.views):
                H, W = self.views[int(v)]
                if d.shape != (H, W):
                    raise ValueError(f"map {i}: depth shape {tuple(d.shape)} is not the view's {(H, W)}")
                P += H * W
        pts = torch.empty((max(P, 1), 3), dtype=torch.float32, device=self.device)
        sup = torch.empty((max(P, 1),), dtype=torch.int32, device=self.device)
        own = torch.empty((max(P, 1),), dtype=torch.int64, device=self.device)
        cp = _FuseParams(float(max_rel_dist))
        self._check(lib().phimvs_fuse(self.h, len(maps), arr, C.byref(cp), pts.data_ptr(), sup.data_ptr(),
                                      own.data_ptr()))
        return pts[:P], sup[:P], own[:P]

    # ------------------------------------------------------------------ plane hypothesis inference
    def phi_hypotheses(self, depth):
        """Depth hypotheses (4, H, W) of the pixels of ``depth`` (H, W) without depth (0 = none)."""
        torch = self.torch
        self._sync_stream()
        d = depth.contiguous()
        H, W = d.shape
        hyp = torch.empty((4, H, W), dtype=torch.float32, device=self.device)
        self._check(lib().phimvs_phi_hypotheses(self.h, W, H, d.data_ptr(), hyp.data_ptr()))
        return hyp

    def phi_hypotheses_noalloc(self, depth, out):
        """The same hypotheses into the caller's (4, H, W) float32 tensor ``out``, through the
        entry point that allocates nothing (its scratch is a fixed device array)."""
        self._sync_stream()
        d = depth.contiguous()
        H, W = d.shape
        assert out.shape == (4, H, W) and out.dtype == self.torch.float32 and out.is_contiguous()
        self._check(lib().phimvs_phi_hypotheses_noalloc(self.h, W, H, d.data_ptr(), out.data_ptr()))
        return out

    def phi_costs(self, hyp):
        """Matching cost (4, H, W) of the hypotheses under the prepared problem."""
        torch = self.torch
        self._sync_stream()
        h = hyp.contiguous()
        cost = torch.empty_like(h)
        self._check(lib().phimvs_phi_costs(self.h, h.data_ptr(), cost.data_ptr()))
        return cost

    def phi_select(self, depth, hyp, cost, params: Optional["PhiParams"] = None):
        """One hypothesis per pixel without depth (graph model decoded on the host) -> depth (H, W)."""
        torch = self.torch
        self._sync_stream()
        d = depth.contiguous()
        H, W = d.shape
        out = torch.empty_like(d)
        p = (params or PhiParams())._c()
        self._check(lib().phimvs_phi_select(self.h, W, H, d.data_ptr(), hyp.contiguous().data_ptr(),
                                            cost.contiguous().data_ptr(), C.byref(p), out.data_ptr()))
        return out

    def phi_normals(self, view: int, depth):
        """Normals of Eq. 10 (H, W, 3) from a depth map of ``view``."""
        torch = self.torch
        self._sync_stream()
        d = depth.contiguous()
        H, W = d.shape
        n = torch.empty((H, W, 3), dtype=torch.float32, device=self.device)
        self._check(lib().phimvs_phi_normals(self.h, view, d.data_ptr(), n.data_ptr()))
        return n

    # ------------------------------------------------------------------ learned proposal
    def net_inputs(self, net: "Net", ref: int, srcs: Sequence[int]):
        """Network input (h, w, 5) of reference ``ref``; h, w = ceil(H/4), ceil(W/4)."""
        torch = self.torch
        self._sync_stream()
        net._sync_stream()
        H, W = self.views[ref] if 0 <= ref < len(self.views) else (4, 4)
        x = torch.empty(((H + 3) // 4, (W + 3) // 4, 5), dtype=torch.float32, device=self.device)
        sa = (C.c_int * len(srcs))(*srcs)
        self._check(lib().phimvs_net_inputs(self.h, net.h, ref, sa, len(srcs), x.data_ptr()))
        return x

    def net_decode(self, net: "Net", ref: int, output):
        torch = self.torch
        self._sync_stream()
        H, W = self.views[ref] if 0 <= ref < len(self.views) else (1, 1)
        if output.dtype != torch.float32 or not output.is_contiguous() or output.numel() != ((H + 3) // 4) * ((W + 3) // 4) * 4:
            raise ValueError("output must be a contiguous float32 (ceil(H/4), ceil(W/4), 4) tensor")
        planes = torch.empty((H, W, 4), dtype=torch.float32, device=self.device)
        self._check(lib().phimvs_net_decode(self.h, net.h, ref, output.data_ptr(), planes.data_ptr()))
        return planes

    def propose(self, net: "Net", ref: int, srcs: Sequence[int], out=None):
        """Proposal planes (H, W, 4) of reference ``ref`` from the network."""
        torch = self.torch
        self._sync_stream()
        H, W = self.views[ref] if 0 <= ref < len(self.views) else (1, 1)
        planes = out if out is not None else torch.empty((H, W, 4), dtype=torch.float32, device=self.device)
        sa = (C.c_int * len(srcs))(*srcs)
        self._check(lib().phimvs_net_propose(self.h, net.h, ref, sa, len(srcs), planes.data_ptr()))
        return planes

    # ------------------------------------------------------------------ step-wise
    def prepare(self, ref: int, srcs: Sequence[int], window: int, dilation: int, params: Optional[Params] = None):
        self._sync_stream()
        sa = (C.c_int * len(srcs))(*srcs)
        p = (params or default_params())._c()
        self._check(lib().phimvs_prepare(self.h, ref, sa, len(srcs), window, dilation, C.byref(p)))
        self.H, self.W = self.views[ref]  # ref validated by the library
        self.n_src = len(srcs)

    def init_planes(self, proposal=None):
        self._sync_stream()
        self._check(lib().phimvs_init_planes(self.h, _dptr(proposal), 1))

    def step(self, iteration: int, colour: int, propagate: bool = True, refine: bool = True):
        self._sync_stream()
        self._check(lib().phimvs_step(self.h, iteration, colour, int(propagate), int(refine)))

    def get_state(self):
        torch = self.torch
        self._sync_stream()
        planes = torch.empty((self.H, self.W, 4), dtype=torch.float32, device=self.device)
        cost = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        self._check(lib().phimvs_get_state(self.h, planes.data_ptr(), cost.data_ptr(), 1))
        return planes, cost

    def set_state(self, planes, cost):
        self._sync_stream()
        planes = planes.contiguous().float()
        cost = cost.contiguous().float()
        self._check(lib().phimvs_set_state(self.h, planes.data_ptr(), cost.data_ptr(), 1))
        self._keep = (planes, cost)

    def output(self):
        torch = self.torch
        self._sync_stream()
        d = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        n = torch.empty((self.H, self.W, 3), dtype=torch.float32, device=self.device)
        c = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        self._check(lib().phimvs_output(self.h, d.data_ptr(), n.data_ptr(), c.data_ptr(), 1))
        return d, n, c

    def eval_cost(self, planes, per_view: bool = False):
        """Cost of the given planes (H, W, 4) -> cost (H, W) [, per-view (H, W, n), valid (H, W, n)]."""
        torch = self.torch
        self._sync_stream()
        planes = planes.contiguous().float()
        cost = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        pv = vm = None
        if per_view:
            pv = torch.empty((self.H, self.W, self.n_src), dtype=torch.float32, device=self.device)
            vm = torch.empty((self.H, self.W, self.n_src), dtype=torch.uint8, device=self.device)
        self._check(lib().phimvs_eval_cost(self.h, planes.data_ptr(), cost.data_ptr(), _dptr(pv), _dptr(vm), 1))
        return (cost, pv, vm) if per_view else cost

    def sync(self):
        self._check(lib().phimvs_sync(self.h))

    # ------------------------------------------------------------------ batches
    def _jobs(self, jobs):
        """jobs: dicts with ref, srcs, window, dilation, params (optional), and device tensors
        depth / normal / cost (optional; allocated when missing)."""
        torch = self.torch
        arr = (_Job * len(jobs))()
        keep = []
        outs = []
        for i, j in enumerate(jobs):
            H, W = self.views[j["ref"]] if 0 <= j["ref"] < len(self.views) else (1, 1)
            d = j.get("depth")
            n = j.get("normal")
            c = j.get("cost")
            if d is None:
                d = torch.empty((H, W), dtype=torch.float32, device=self.device)
            if n is None:
                n = torch.empty((H, W, 3), dtype=torch.float32, device=self.device)
            if c is None:
                c = torch.empty((H, W), dtype=torch.float32, device=self.device)
            sa = (C.c_int32 * len(j["srcs"]))(*j["srcs"])
            keep.append(sa)
            p = (j.get("params") or default_params())._c()
            arr[i] = _Job(j["ref"], sa, len(j["srcs"]), j["window"], j["dilation"], p, d.data_ptr(), n.data_ptr(),
                          c.data_ptr())
            outs.append((d, n, c))
        return arr, keep, outs

    def patchmatch_batch(self, jobs, iters: int, use_graph: bool = True):
        """-> list of (depth, normal, cost) device tensors, one per job."""
        self._sync_stream()
        arr, keep, outs = self._jobs(jobs)
        self._check(lib().phimvs_patchmatch_batch(self.h, len(jobs), arr, iters, int(use_graph)))
        return outs

    def set_tuning(self, t: Tuning):
        self._check(lib().phimvs_set_tuning(self.h, C.byref(_Tuning(t.tile_rows, int(t.persistent), t.wgs_per_cu,
                                                                     (7 if t.order_by_depth is True else int(t.order_by_depth)), t.ms))))

    def get_tuning(self) -> Tuning:
        t = _Tuning()
        self._check(lib().phimvs_get_tuning(self.h, C.byref(t)))
        return Tuning(t.tile_rows, bool(t.persistent), t.wgs_per_cu, t.ms, int(t.order_by_depth))

    def autotune(self, jobs, iters: int = 1):
        """Time the built-in launch configurations on this batch; keep the fastest.
        -> (best Tuning, list of every Tuning with its time)."""
        self._sync_stream()
        arr, keep, outs = self._jobs(jobs)
        cap = 32
        res = (_Tuning * cap)()
        n = C.c_int(cap)
        self._check(lib().phimvs_autotune(self.h, len(jobs), arr, iters, res, C.byref(n)))
        allr = [Tuning(r.tile_rows, bool(r.persistent), r.wgs_per_cu, r.ms, int(r.order_by_depth))
                for r in res[:n.value]]
        return self.get_tuning(), allr

    def diag_enable(self, flags: int):
        self._sync_stream()
        self._check(lib().phimvs_diag_enable(self.h, flags))

    def diag_read(self):
        """-> (hypotheses scored, evaluate launches timed, their summed duration in ms)."""
        n, l, ms = C.c_uint64(), C.c_uint64(), C.c_double()
        self._check(lib().phimvs_diag_read(self.h, C.byref(n), C.byref(l), C.byref(ms)))
        return int(n.value), int(l.value), float(ms.value)

    def check_reciprocal(self, first_bits: int, count: int):
        m = C.c_uint64()
        e = C.c_uint32()
        self._check(lib().phimvs_check_reciprocal(self.h, first_bits, count, C.byref(m), C.byref(e)))
        return int(m.value), int(e.value)


class Net:
    """The learned initial-plane proposal network (include/phimvs_net.h) on one GPU,
    issuing work on torch's current stream."""

    IN, OUT, WIDTH, LAYERS = 5, 4, 32, 5
    #: (cin, cout) of each 3x3 convolution
    SHAPES = ((5, 32), (32, 32), (32, 32), (32, 32), (32, 4))

    def __init__(self, device: int = 0, params=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        torch.cuda.init()
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
        rc = lib().phimvs_net_create(C.byref(h), device, C.c_void_p(stream))
        if rc != PHIMVS_OK:
            raise PhimvsError(rc, "phimvs_net_create failed")
        self.h = h
        self.n_params = int(lib().phimvs_net_param_count())
        if params is not None:
            self.set_params(params)

    @staticmethod
    def param_count() -> int:
        return int(lib().phimvs_net_param_count())

    def close(self):
        if getattr(self, "h", None):
            lib().phimvs_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != PHIMVS_OK:
            raise PhimvsError(rc, lib().phimvs_net_last_error(self.h).decode())

    def _sync_stream(self):
        s = self.torch.cuda.current_stream(self.device).cuda_stream
        self._check(lib().phimvs_net_set_stream(self.h, C.c_void_p(s)))

    def set_params(self, params):
        """params: flat float32 vector (numpy or a device tensor) in the layout of phimvs_net.h."""
        self._sync_stream()
        if isinstance(params, np.ndarray):
            a = np.ascontiguousarray(params, dtype=np.float32)
            if a.size != self.n_params:
                raise ValueError(f"expected {self.n_params} parameters, got {a.size}")
            self._check(lib().phimvs_net_set_params(self.h, a.ctypes.data, 0))
        else:
            if params.dtype != self.torch.float32 or not params.is_contiguous() or params.numel() != self.n_params:
                raise ValueError("params must be a contiguous float32 tensor of param_count() values")
            self._check(lib().phimvs_net_set_params(self.h, params.data_ptr(), 1))

    def get_params(self) -> np.ndarray:
        self._sync_stream()
        a = np.empty(self.n_params, dtype=np.float32)
        self._check(lib().phimvs_net_get_params(self.h, a.ctypes.data, 0))
        return a

    def forward(self, x):
        """x: (B, h, w, 5) or (h, w, 5) float32 device tensor -> raw outputs (..., 4)."""
        torch = self.torch
        self._sync_stream()
        xb = x if x.dim() == 4 else x.unsqueeze(0)
        if xb.dtype != torch.float32 or xb.shape[-1] != self.IN:
            raise ValueError("input must be float32 with 5 channels")
        xb = xb.contiguous()
        B, h, w, _ = xb.shape
        out = torch.empty((B, h, w, self.OUT), dtype=torch.float32, device=self.device)
        self._check(lib().phimvs_net_forward(self.h, B, h, w, xb.data_ptr(), out.data_ptr()))
        self._last_shape = (B, h, w)
        return out if x.dim() == 4 else out[0]

    def loss_grad(self, x, target, mask, depth_range, normal_weight: float = 1.0, want_loss: bool = True,
                  want_grad: bool = False):
        """Loss and parameter gradient (kept for ``adam``) -> (loss or None, grad tensor or None)."""
        torch = self.torch
        self._sync_stream()
        B, h, w, _ = x.shape
        for t, shape in ((x, (B, h, w, 5)), (target, (B, h, w, 4)), (mask, (B, h, w)), (depth_range, (B, 2))):
            if t.dtype != torch.float32 or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"expected a contiguous float32 tensor of shape {shape}")
        loss = C.c_double(0.0)
        grad = torch.empty(self.n_params, dtype=torch.float32, device=self.device) if want_grad else None
        self._check(lib().phimvs_net_loss_grad(self.h, B, h, w, x.data_ptr(), target.data_ptr(), mask.data_ptr(),
                                               depth_range.data_ptr(), float(normal_weight),
                                               C.byref(loss) if want_loss else None, _dptr(grad)))
        self._last_shape = (B, h, w)
        return (loss.value if want_loss else None), grad

    def tensor(self, kind: int, layer: int):
        """A tensor the last pass stored (bfloat16 widened to float32), (B, h, w, C): kind 0
        the activation entering ``layer`` (0 = the input), kind 1 the loss gradient at the
        output of ``layer`` (the last layer's is the loss's own)."""
        torch = self.torch
        self._sync_stream()
        B, h, w = getattr(self, "_last_shape", (0, 0, 0))
        last = len(self.SHAPES) - 1
        C_ = (self.IN if layer == 0 else 32) if kind == 0 else (self.OUT if layer == last else 32)
        out = torch.empty((B, h, w, C_), dtype=torch.float32, device=self.device)
        self._check(lib().phimvs_net_tensor(self.h, kind, layer, out.data_ptr()))
        return out

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self._sync_stream()
        self._check(lib().phimvs_net_adam(self.h, lr, beta1, beta2, eps))

    def targets(self, depth, normal, cost, max_cost: float):
        """Training targets (h, w, 4) and mask (h, w) from a full-resolution result."""
        torch = self.torch
        self._sync_stream()
        H, W = depth.shape
        h, w = (H + 3) // 4, (W + 3) // 4
        tgt = torch.empty((h, w, 4), dtype=torch.float32, device=self.device)
        mask = torch.empty((h, w), dtype=torch.float32, device=self.device)
        self._check(lib().phimvs_net_targets(self.h, W, H, depth.contiguous().data_ptr(), normal.contiguous().data_ptr(),
                                             cost.contiguous().data_ptr(), float(max_cost), tgt.data_ptr(),
                                             mask.data_ptr()))
        return tgt, mask


def phi_decode_host(depth, hyp, cost, params: Optional[PhiParams] = None, cost_max: float = COST_MAX):
    """The host-side graph-model decoder of plane hypothesis inference on numpy arrays:
    depth (H, W), hyp / cost (4, H, W) -> (labels (H, W) int32, depth (H, W) float32)."""
    p = params or PhiParams()
    d = np.ascontiguousarray(depth, dtype=np.float32)
    h = np.ascontiguousarray(hyp, dtype=np.float32)
    c = np.ascontiguousarray(cost, dtype=np.float32)
    H, W = d.shape
    if h.shape != (4, H, W) or c.shape != (4, H, W):
        raise ValueError("hyp and cost must be (4, H, W)")
    lab = np.zeros((H, W), np.int32)
    out = np.zeros((H, W), np.float32)
    fp = C.POINTER(C.c_float)
    rc = lib().phimvs_phi_decode_host(W, H, d.ctypes.data_as(fp), h.ctypes.data_as(fp), c.ctypes.data_as(fp), p.k1,
                                      p.k2, p.k3, cost_max, p.iterations, lab.ctypes.data, out.ctypes.data)
    if rc != PHIMVS_OK:
        raise PhimvsError(rc, "invalid decoder arguments")
    return lab, out
