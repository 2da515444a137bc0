"""Helpers for the GPU parity tests: seeded parents on host and device, layout
round trips through the library, and the oracle's expected results."""

from __future__ import annotations

import sys

import numpy as np

import oracle
from seeded_inputs import residues_np, residues_torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def parent_host(seed: int, p: int, N: int) -> np.ndarray:
    return residues_np(seed, p, N, N)


def parent_device(seed: int, p: int, N: int):
    torch = torch_cuda()
    return residues_torch(seed, p, N, N, device="cuda")


def host_of(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def device_of(a: np.ndarray):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def stream_handle() -> int:
    torch = torch_cuda()
    return torch.cuda.current_stream().cuda_stream


def to_mh(mh, ctx, cart_dev, N: int, T: int):
    """Morton-hybrid copy (device) of a Cartesian N x N device tensor."""
    torch = torch_cuda()
    out = torch.empty(N * N, dtype=torch.int32, device="cuda")
    mh.check(mh.mh_layout_from_cartesian(ctx, out.data_ptr(), cart_dev.data_ptr(),
                                         cart_dev.stride(0), N, T, stream_handle()), "from")
    return out


def to_cart(mh, ctx, mh_dev, N: int, T: int):
    torch = torch_cuda()
    out = torch.empty((N, N), dtype=torch.int32, device="cuda")
    mh.check(mh.mh_layout_to_cartesian(ctx, out.data_ptr(), N, mh_dev.data_ptr(), N, T,
                                       stream_handle()), "to")
    return out


def expected_view(C, A, B, p, rc, cc, ra, ca, rb, cb, m, k, n):
    """Oracle: whole C parent after C[rc.., cc..] += A[ra.., ca..] B[rb.., cb..] mod p."""
    want = C.copy()
    oracle.matmul_modp_view(want, A, B, p, rc, cc, ra, ca, rb, cb, m, k, n)
    return want
