"""Void and plastic clusters of a solved grid (Sec. 3) through the C ABI.

``analyze(void_mask, plastic_mask)`` labels the periodic nearest-neighbour
clusters of the void-plastic phase on the device, joins plastic clusters
without a void to the cluster of their nearest void, and returns the
canonical labels with the counts behind the paper's indicators
(``indicators``).  Argument marshalling only.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import PmClusterIndicators, PmClusterStats, check, lib


def analyze(void_mask: torch.Tensor, plastic: torch.Tensor, stream=None):
    """(labels int32 (L, L) on the device, stats dict)."""
    L = int(void_mask.shape[0])
    dev = void_mask.device
    vm = void_mask.to(dtype=torch.uint8).contiguous()
    pm_ = plastic.to(device=dev, dtype=torch.uint8).contiguous()
    if tuple(vm.shape) != (L, L) or tuple(pm_.shape) != (L, L):
        raise ValueError("masks must be L x L")
    nws = lib().pm_cluster_workspace_bytes(L)
    if nws == 0:
        raise ValueError(f"L = {L} must be a power of two in [4, 8192]")
    ws = torch.empty(nws + 256, dtype=torch.uint8, device=dev)
    base = ws.data_ptr()
    ptr = base + (-base) % 256
    labels = torch.empty((L, L), dtype=torch.int32, device=dev)
    st = PmClusterStats()
    s = torch.cuda.current_stream(dev).cuda_stream if stream is None else stream
    check(lib().pm_clusters(L, vm.data_ptr(), pm_.data_ptr(), labels.data_ptr(), ptr, nws, ctypes.byref(st), s),
          "pm_clusters")
    stats = {k: getattr(st, k) for k, _ in st._fields_ if k != "pad"}
    stats["spans_x1"] = bool(stats["spans_x1"])
    stats["spans_x2"] = bool(stats["spans_x2"])
    return labels, stats


def indicators(stats, L, f=None):
    """Sec. 3 indicators v_p, f_p, v_max, i and n, computed by the library
    from the counts of ``analyze`` (f: the void fraction; None = realised)."""
    st = PmClusterStats()
    for k, _ in st._fields_:
        if k != "pad":
            setattr(st, k, int(stats[k]))
    out = PmClusterIndicators()
    check(lib().pm_cluster_indicators(ctypes.byref(st), int(L), -1.0 if f is None else float(f), ctypes.byref(out)),
          "pm_cluster_indicators")
    return {k: getattr(out, k) for k, _ in out._fields_}


def path_derivatives(x, y):
    """(dy/dx, d2y/dx2) of samples y at strictly increasing x (host arrays),
    three-point finite differences computed by the library."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    if x.shape != y.shape or x.ndim != 1:
        raise ValueError("x and y must be 1-D arrays of one length")
    dy = np.empty_like(x)
    d2y = np.empty_like(x)
    check(lib().pm_path_derivatives(len(x), x.ctypes.data, y.ctypes.data, dy.ctypes.data, d2y.ctypes.data),
          "pm_path_derivatives")
    return dy, d2y


def path_indicators(eps0, n, sigma0):
    """Sec. 3 indicators along a loading path: r = dn/d eps0 and
    -d2 sigma0 / d eps0^2 at each step."""
    r, _ = path_derivatives(eps0, n)
    _, s2 = path_derivatives(eps0, sigma0)
    return dict(r=r, minus_d2sigma0=-s2)
