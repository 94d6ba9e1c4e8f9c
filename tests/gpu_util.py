"""Helpers for the GPU tests: column-major device tensors and host copies."""
import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def torch_cuda():
    import torch

    return torch


def to_dev(a, ld=None, dtype=None):
    """Column-major (Fortran) numpy array -> column-major CUDA tensor view with
    leading dimension ld >= rows. Padding rows hold NaN so stray reads show."""
    import torch

    a = np.asarray(a)
    if a.ndim == 1:
        a = a.reshape(-1, 1, order="F")
    m, n = a.shape
    ld = m if ld is None else ld
    dt = dtype or (torch.float64 if a.dtype == np.float64 else torch.float32)
    buf = torch.full((max(n, 1), max(ld, 1)), float("nan"), dtype=dt)
    buf[:n, :m] = torch.from_numpy(np.ascontiguousarray(a.T)).to(dt)
    return buf.cuda().T[:m, :n]


def to_host(t):
    """Column-major CUDA tensor view -> Fortran-order numpy array."""
    return np.asfortranarray(t.T.contiguous().cpu().numpy().T)


def ipiv_dev(k):
    import torch

    return torch.zeros(max(k, 1), dtype=torch.int32, device="cuda")


def rel_fro(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
