"""Helpers for the GPU tests: move seeded numpy inputs to the device, run the
library through its C ABI, bring results back, and compare with the oracle."""
import os
import sys

import numpy as np

TOL = {"f64": 1e-12, "f32": 5e-6}  # relative L2 bound vs the FP64 oracle


def say(msg: str) -> None:
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    sys.stdout.write("[gpu] %s\n" % msg)
    sys.stdout.flush()


def torch_mod():
    import torch
    return torch


def dev_real(x: np.ndarray, dtype: str):
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32 if dtype == "f32" else np.float64))
    return t.to("cuda")


def dev_cplx(X: np.ndarray, dtype: str):
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(X, dtype=np.complex64 if dtype == "f32" else np.complex128))
    return t.to("cuda")


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def rounded(x: np.ndarray, dtype: str) -> np.ndarray:
    """The values the GPU sees, as FP64 / complex128 for the oracle."""
    if np.iscomplexobj(x):
        return x.astype(np.complex64).astype(np.complex128) if dtype == "f32" else x.astype(np.complex128)
    return x.astype(np.float32).astype(np.float64) if dtype == "f32" else x.astype(np.float64)


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def oracle_threads() -> int:
    return int(os.environ.get("FFT3D_ORACLE_THREADS", "0"))
