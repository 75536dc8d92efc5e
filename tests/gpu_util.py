"""Helpers shared by the GPU tests (host <-> device column-major transfers)."""
import numpy as np

U64 = 2.0 ** -53


def gamma(k: int) -> float:
    """Standard bound constant k*u / (1 - k*u) for a length-k dot product."""
    return k * U64 / (1.0 - k * U64)


def to_dev(a: np.ndarray, ld: int | None = None, offset: int = 0):
    """Column-major FP64 device copy of a host matrix, optional padded ld and
    an element offset into the allocation (to exercise unaligned bases)."""
    import torch
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    ld = max(ld or m, 1)
    buf = torch.zeros(n * ld + offset + 8, dtype=torch.float64, device="cuda")
    view = buf[offset:offset + n * ld].view(n, ld).t()[:m, :]
    view.copy_(torch.from_numpy(np.ascontiguousarray(a)).cuda())
    return view


def to_host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return np.asfortranarray(t.detach().cpu().numpy())
