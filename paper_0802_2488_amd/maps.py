"""Strain-map post-processing through the C ABI (argument marshalling only):
the CG2 five-point average (Sec. 2) and the measures of a strain map used to
compare the methods (Fig. 1: checkerboard index, sharpness, mean and maximum
equivalent strain on the matrix pixels)."""
from __future__ import annotations

import ctypes

import torch

from ._lib import PM_FP32, PM_FP64, PmStrainMapOut, check, lib


def _prec(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return PM_FP64
    if t.dtype == torch.float32:
        return PM_FP32
    raise ValueError("fields must be float32 or float64")


def five_point_average(planes: torch.Tensor, stream=None) -> torch.Tensor:
    """CG2: average of every plane over each pixel and its four neighbours."""
    x = planes.contiguous()
    n, L = x.shape[0], x.shape[-1]
    out = torch.empty_like(x)
    s = torch.cuda.current_stream(x.device).cuda_stream if stream is None else stream
    check(lib().pm_five_point_average(L, _prec(x), n, x.data_ptr(), out.data_ptr(), s), "pm_five_point_average")
    return out


def strain_map_metrics(eps: torch.Tensor, void_mask: torch.Tensor, stream=None) -> dict:
    """Measures of a (4, L, L) strain field on the matrix pixels of void_mask."""
    e = eps.contiguous()
    L = e.shape[-1]
    m = void_mask.to(device=e.device, dtype=torch.uint8).contiguous()
    n = lib().pm_strain_map_workspace_bytes(L)
    if n == 0:
        raise ValueError(f"L = {L} is not a supported size")
    ws = torch.empty(n // 8 + 1, dtype=torch.float64, device=e.device)
    out = PmStrainMapOut()
    s = torch.cuda.current_stream(e.device).cuda_stream if stream is None else stream
    check(lib().pm_strain_map_metrics(L, _prec(e), e.data_ptr(), m.data_ptr(), ws.data_ptr(), n, ctypes.byref(out),
                                      s), "pm_strain_map_metrics")
    return {k: getattr(out, k) for k, _ in out._fields_}
