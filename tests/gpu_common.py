"""Helpers shared by the GPU tests (error metrics, parameter upload)."""
import numpy as np

TOL_C64 = 1e-5      # complex64 path vs the complex128 oracle
TOL_BF16X3 = 1e-3   # split-BF16 wide nodes


def rel_err(z, ref, floor):
    """|z - ref| / max(|ref|, floor): the floor is 2^(-n/2) for amplitudes
    (their RMS size) and 1 for Pauli expectations and energies, so values
    near zero do not inflate the error."""
    return abs(complex(z) - complex(ref)) / max(abs(complex(ref)), floor)


def true_rel_err(z, ref):
    """|z - ref| / |ref| with no floor (reported beside rel_err where the
    reference value is far below its floor)."""
    return abs(complex(z) - complex(ref)) / abs(complex(ref))


def grad_err(g, ref):
    """||g - ref||_2 / max(||ref||_2, 1) over the whole gradient vector."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1.0)


def grad_max_abs(g, ref):
    """Largest error of a single gradient component, max_i |g_i - ref_i|
    (one wrong slot cannot hide in the norm of the others)."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(g - ref))) if g.size else 0.0


def assert_grad(g, ref, tol, what=""):
    """Both gradient metrics within tol: the norm ratio and the largest
    component error (absolute: the components here are O(1))."""
    e2, em = grad_err(g, ref), grad_max_abs(g, ref)
    assert e2 < tol and em < tol, f"{what} grad_err {e2:.3e} max_abs {em:.3e} tol {tol:.0e}"


def device_params(params, batch=None):
    import torch
    p = np.ascontiguousarray(np.asarray(params, np.float32))
    if batch is not None:
        p = p.reshape(batch, -1)
    return torch.from_numpy(p).to("cuda").contiguous()
