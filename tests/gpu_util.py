"""Helpers shared by the GPU tests: host <-> device copies of uint64 arrays."""

import numpy as np


def banner(msg):
    """Names the case before its GPU work starts."""
    print("[case] " + msg, flush=True)


def torch_mod():
    import torch
    return torch


def to_dev(a: np.ndarray, device="cuda:0"):
    torch = torch_mod()
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device).view(torch.uint64)


def to_host(t) -> np.ndarray:
    torch = torch_mod()
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def level_offsets(n_rows: int):
    offs, sizes, off, n = [], [], 0, n_rows
    while True:
        offs.append(off)
        sizes.append(n)
        off += n
        if n == 1:
            break
        n = (n + 1) // 2
    return offs, sizes


def rows_from_colmajor(flat: np.ndarray, n_rows: int, n_cols: int, rows) -> np.ndarray:
    """The selected rows (as a column-major [n_cols][len(rows)] block) of a column-major matrix."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.arange(n_cols, dtype=np.int64)
    return flat[(cols[:, None] * n_rows + rows[None, :])].reshape(-1)
