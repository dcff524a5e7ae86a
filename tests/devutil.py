"""Device-array helpers shared by the GPU tests (plain torch marshalling)."""
import numpy as np


def to_dev(X, dtype=None):
    """A host array as an (n, ncols) column-major CUDA tensor."""
    import torch
    X = np.asarray(X)
    if X.ndim == 1:
        X = X.reshape(-1, 1)
    t = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda")
    if dtype is not None:
        t = t.to(dtype)
    return t.t()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def dense_of(hm, H, n):
    """The dense matrix an H-matrix applies (original order), column by column."""
    I = hm.colmajor(n, n)
    I.zero_()
    I.diagonal().fill_(1.0)
    Y = hm.colmajor(n, n)
    H.matvec(I, Y, order=hm.HM_ORDER_ORIGINAL)
    return to_host(Y)
