"""Marshalling helpers: upload a synthetic workload (dict of numpy arrays) to
the device with torch and drive the C-ABI.  No solver arithmetic here."""
from __future__ import annotations

import numpy as np

from .fh import Context


def device_tensor(arr, dtype=None, device="cuda:0"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(arr))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


def setup_context(wl: dict, device: int = 0, ctx: Context | None = None,
                  Cref=None, bind_workspace: bool = True) -> Context:
    """Configure a context for workload `wl` (keys as synth.workload)."""
    import torch
    ctx = ctx or Context(device)
    dev = f"cuda:{device}"
    ctx.set_grid(wl["n"][: wl["dim"]], wl["problem"], wl["element"], wl.get("l"))
    if wl.get("phase") is not None:
        ph = device_tensor(wl["phase"].astype(np.uint8), device=dev)
        ctx.set_phases(ph, wl["mat"])
    else:
        k = device_tensor(wl["kfield"].astype(np.float64), device=dev)
        ctx.set_conductivity_field(k)
    ctx.set_reference(Cref)
    ctx.set_load(wl["loads"])
    if bind_workspace:
        nbytes = ctx.workspace_size()
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        ctx.bind_workspace(ws[off:off + nbytes])
    return ctx


def fluctuations(ctx: Context, device: int = 0):
    import torch
    out = []
    for j in range(ctx.nload):
        u = torch.empty(ctx.nd * ctx.N, dtype=torch.float64, device=f"cuda:{device}")
        ctx.get_fluctuation(j, u)
        out.append(u.cpu().numpy())
    return out
