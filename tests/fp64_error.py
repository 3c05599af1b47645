"""The FP64 oracle's distance to an FP32 result, printed beside each parity check: cost
as an absolute difference, depth as a relative one (valid pixels only)."""
import sys

import numpy as np


def report(tag, gpu_cost=None, fp64_cost=None, mask=None, gpu_depth=None, fp64_depth=None):
    parts = []
    if gpu_cost is not None:
        g = np.asarray(gpu_cost, np.float64)
        o = np.asarray(fp64_cost, np.float64)
        e = np.abs(g - o) if mask is None else np.abs(g - o)[mask]
        if e.size:
            parts.append(f"cost |fp32 - fp64| max {e.max():.3e} mean {e.mean():.3e} "
                         f"99.9th pct {np.quantile(e, 0.999):.3e} within 1e-4 {np.mean(e <= 1e-4):.6f}")
    if gpu_depth is not None:
        g = np.asarray(gpu_depth, np.float64)
        o = np.asarray(fp64_depth, np.float64)
        if mask is not None:
            g, o = g[mask], o[mask]
        rel = np.abs(g - o) / np.maximum(np.abs(o), 1e-30)
        if rel.size:
            parts.append(f"depth |fp32 - fp64|/fp64 median {np.median(rel):.3e} max {rel.max():.3e} "
                         f"within 1e-3 {np.mean(rel <= 1e-3):.6f}")
    print(f"{tag} vs FP64 oracle: " + "; ".join(parts), flush=True)
    sys.stdout.flush()
