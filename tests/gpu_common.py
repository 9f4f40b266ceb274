"""Helpers shared by the GPU tests (error metrics, parameter upload)."""
import numpy as np

TOL_C64 = 1e-5      # complex64 path vs the complex128 oracle
TOL_BF16X3 = 1e-3   # split-BF16 wide nodes


def rel_err(z, ref, floor):
    """|z - ref| / max(|ref|, floor): the floor is 2^(-n/2) for amplitudes
    (their RMS size) and 1 for Pauli expectations and energies, so values
    near zero do not inflate the error."""
    return abs(complex(z) - complex(ref)) / max(abs(complex(ref)), floor)


def grad_err(g, ref):
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1.0)


def device_params(params, batch=None):
    import torch
    p = np.ascontiguousarray(np.asarray(params, np.float32))
    if batch is not None:
        p = p.reshape(batch, -1)
    return torch.from_numpy(p).to("cuda").contiguous()
