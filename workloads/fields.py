"""Seeded synthetic inputs for the 3D r2c/c2r path.

This module only draws random numbers and builds spectra.  It holds no code of
the GPU library and none of the oracle: the tests, the smoke check and the
benchmark all take their inputs from here, so both sides see the same values.

The paper's workloads are 1024^3 and 2048^3 turbulence fields (Sec. 3) and it
publishes no dataset; these generators stand in for a pseudo-spectral solver's
fields:

* ``uniform``: i.i.d. uniform[-1, 1] values in FP64, C order.
* ``k53_spectrum``: a random-phase half spectrum n0 x n1 x (n2/2+1) whose shell
  energy follows k^(-5/3): |X(k)| = |k|^(-11/6) for 0 < |k| <= kmax
  (4 pi k^2 |X|^2 ~ k^(-5/3)), zero elsewhere; kmax = floor(min(n)/3) (the
  two-thirds dealiasing cutoff); phases uniform on [0, 2 pi) drawn over the
  half spectrum in C order; the k2 = 0 plane made Hermitian by overwriting
  each bin whose mirror (-k0, -k1) comes first in C order with the mirror's
  conjugate.  Wavenumbers are signed: index i of an axis of length n stands
  for i if i < n/2 and i - n otherwise.
* ``k53_field``: that spectrum synthesised to real space with numpy's own
  pocketfft (``numpy.fft.irfftn``, a third-party routine that is neither the
  oracle nor the GPU library), then scaled to unit RMS.  The mean is zero
  because the DC bin is.
* ``velocity_spectrum`` / ``velocity_field``: three components,
  u(k) = |k|^(-11/6) (e^{i p1} e1 + e^{i p2} e2) / sqrt(2) with e1, e2 unit
  vectors orthogonal to k (solenoidal, k . u = 0), the same cutoff and
  Hermitian rule; all three components share one scale factor so that the
  mean of |u|^2 / 3 is 1 (separate factors would break k . u = 0).
* FP32 inputs are the FP64 values rounded to nearest (``as_dtype``).
"""
from __future__ import annotations

import math

import numpy as np


def uniform(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=tuple(shape))


def signed_wavenumbers(n: int) -> np.ndarray:
    """Index i -> i for i < n/2, i - n otherwise (integers)."""
    i = np.arange(n, dtype=np.int64)
    return np.where(i < (n + 1) // 2, i, i - n)


def default_kmax(shape) -> int:
    return int(min(shape)) // 3


def _kgrid(shape):
    n0, n1, n2 = shape
    h = n2 // 2 + 1
    k0 = signed_wavenumbers(n0).astype(np.float64)[:, None, None]
    k1 = signed_wavenumbers(n1).astype(np.float64)[None, :, None]
    k2 = np.arange(h, dtype=np.float64)[None, None, :]
    return k0, k1, k2


def _hermitian_k2_zero(X: np.ndarray) -> None:
    """In place: on the k2 = 0 plane (and k2 = n2/2 for even n2, passed in as
    a separate view by the caller) make X[-k0,-k1] = conj(X[k0,k1]).  The bin
    of each mirror pair that comes later in C order is overwritten; bins that
    are their own mirror are made real."""
    n0, n1 = X.shape
    i0 = np.arange(n0)[:, None]
    i1 = np.arange(n1)[None, :]
    m0 = (-i0) % n0
    m1 = (-i1) % n1
    flat = i0 * n1 + i1
    mflat = m0 * n1 + m1
    later = flat > mflat
    src = X[m0, m1]
    X[later] = np.conj(src[later])
    self_mirror = flat == mflat
    X[self_mirror] = X[self_mirror].real


def k53_spectrum(shape, seed: int, kmax: int | None = None) -> np.ndarray:
    n0, n1, n2 = shape
    if kmax is None:
        kmax = default_kmax(shape)
    rng = np.random.default_rng(seed)
    h = n2 // 2 + 1
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(n0, n1, h))
    k0, k1, k2 = _kgrid(shape)
    kk = np.sqrt(k0 * k0 + k1 * k1 + k2 * k2)
    with np.errstate(divide="ignore"):
        amp = np.where((kk > 0) & (kk <= kmax), kk ** (-11.0 / 6.0), 0.0)
    X = amp * np.exp(1j * phase)
    del phase, amp, kk
    _hermitian_k2_zero(X[:, :, 0])
    if n2 % 2 == 0:
        _hermitian_k2_zero(X[:, :, n2 // 2])
    return X


def _synth(X: np.ndarray, shape) -> np.ndarray:
    # numpy's pocketfft, unnormalised inverse: y = sum_k ... e^{+2 pi i k.j/n}
    return np.fft.irfftn(X, s=tuple(shape), axes=(0, 1, 2), norm="forward")


def k53_field(shape, seed: int, kmax: int | None = None) -> np.ndarray:
    x = _synth(k53_spectrum(shape, seed, kmax), shape)
    rms = np.sqrt(np.mean(x * x))
    if rms > 0:
        x /= rms
    return x


def velocity_spectrum(shape, seed: int, kmax: int | None = None) -> np.ndarray:
    """Returns a (3, n0, n1, n2/2+1) complex array: the three components."""
    n0, n1, n2 = shape
    if kmax is None:
        kmax = default_kmax(shape)
    rng = np.random.default_rng(seed)
    h = n2 // 2 + 1
    p1 = rng.uniform(0.0, 2.0 * np.pi, size=(n0, n1, h))
    p2 = rng.uniform(0.0, 2.0 * np.pi, size=(n0, n1, h))
    k0, k1, k2 = _kgrid(shape)
    K = np.stack(np.broadcast_arrays(k0, k1, k2))  # (3, n0, n1, h)
    kk = np.sqrt(np.sum(K * K, axis=0))
    # e1 = k x a / |k x a| with a = z-hat, or x-hat where k is parallel to z-hat
    a = np.zeros_like(K)
    par = (K[0] == 0) & (K[1] == 0)
    a[2] = np.where(par, 0.0, 1.0)
    a[0] = np.where(par, 1.0, 0.0)
    e1 = np.cross(K, a, axis=0)
    n_e1 = np.sqrt(np.sum(e1 * e1, axis=0))
    e1 /= np.where(n_e1 > 0, n_e1, 1.0)
    e2 = np.cross(K, e1, axis=0)
    e2 /= np.where(kk > 0, kk, 1.0)
    with np.errstate(divide="ignore"):
        amp = np.where((kk > 0) & (kk <= kmax), kk ** (-11.0 / 6.0), 0.0)
    U = amp * (np.exp(1j * p1) * e1 + np.exp(1j * p2) * e2) / np.sqrt(2.0)
    for c in range(3):
        _hermitian_k2_zero(U[c, :, :, 0])
        if n2 % 2 == 0:
            _hermitian_k2_zero(U[c, :, :, n2 // 2])
    return U


def velocity_field(shape, seed: int, kmax: int | None = None) -> np.ndarray:
    """Returns (3, n0, n1, n2) real components with mean(|u|^2)/3 = 1."""
    U = velocity_spectrum(shape, seed, kmax)
    u = np.stack([_synth(U[c], shape) for c in range(3)])
    rms = np.sqrt(np.mean(u * u))
    if rms > 0:
        u /= rms
    return u


def as_dtype(x: np.ndarray, dtype: str) -> np.ndarray:
    """'f64' -> float64 / complex128 unchanged; 'f32' -> rounded to nearest."""
    if dtype == "f64":
        return np.ascontiguousarray(x, dtype=np.complex128 if np.iscomplexobj(x) else np.float64)
    if dtype == "f32":
        return np.ascontiguousarray(x, dtype=np.complex64 if np.iscomplexobj(x) else np.float32)
    raise ValueError("dtype must be 'f32' or 'f64'")


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2 over all stored scalars (re and im)."""
    a = np.asarray(a)
    b = np.asarray(b)
    num = np.linalg.norm((a.astype(np.complex128) - b.astype(np.complex128)).ravel())
    den = np.linalg.norm(b.astype(np.complex128).ravel())
    return float(num / den) if den > 0 else float(num)


# ---- workload recipes (sizes and mixes; no transform arithmetic) ----

BATCH_SHAPES = ((32, 32, 32), (48, 48, 48), (64, 64, 64), (96, 96, 96), (128, 128, 128), (192, 192, 96))


def batch_mix(count: int = 64, seed: int = 4):
    """The mixed batch: `count` fields, shapes i.i.d. uniform over
    BATCH_SHAPES, dtype FP32 or FP64 with probability 1/2 each.  Returns a list
    of (shape, dtype); field i takes its values from uniform(shape, 1000 + i)."""
    rng = np.random.default_rng(seed)
    si = rng.integers(0, len(BATCH_SHAPES), size=count)
    di = rng.integers(0, 2, size=count)
    return [(BATCH_SHAPES[int(a)], "f64" if int(b) else "f32") for a, b in zip(si, di)]


SERVE_SHAPES = ((64, 64, 64), (128, 128, 128), (256, 256, 256), (256, 256, 128), (512, 512, 512))
SERVE_LARGE = (1024, 1024, 1024)


def serve_mix(count: int, rate: float, seed: int = 5, p_large: float = 0.02, p_f64: float = 0.2):
    """The served stream: `count` requests with Poisson arrivals of mean rate
    `rate` per second.  Each: shape uniform over SERVE_SHAPES, or SERVE_LARGE
    (always FP32) with probability p_large; FP64 with probability p_f64
    otherwise; r2c or c2r with probability 1/2; three components.  Returns
    (arrival times in s from 0, list of (shape, dtype, direction) with
    direction 0 = r2c, 1 = c2r)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    reqs = []
    for _ in range(count):
        if rng.random() < p_large:
            shape, dt = SERVE_LARGE, "f32"
        else:
            shape = SERVE_SHAPES[int(rng.integers(len(SERVE_SHAPES)))]
            dt = "f64" if rng.random() < p_f64 else "f32"
        reqs.append((shape, dt, int(rng.integers(2))))
    return t, reqs


def velocity_pool_torch(shape, seed: int, dtype: str, device="cuda", kmax: int | None = None, slab: int = 32):
    """GPU version of velocity_spectrum / velocity_field for the large fields of
    the served workload (numpy takes minutes at 512^3 and more): the same
    construction -- amplitude |k|^(-11/6) for 0 < |k| <= kmax, random phases
    on the two unit vectors orthogonal to k -- with torch's seeded generator
    (so not the same values as the numpy version), built in slabs of `slab`
    k0 planes, synthesised with torch.fft.irfftn (rocFFT, a third-party
    routine), all three components scaled so that mean(|u|^2)/3 = 1.  The
    k2 = 0 and n2/2 planes are left as drawn (c2r reads them as defined for
    any half spectrum).  Returns (real (3, n0, n1, n2), spectrum (3, n0, n1,
    n2/2+1)) in the dtype ('f32' or 'f64'): the spectrum is the synthesised
    one, scaled like the field, so that c2r of it is N times the field."""
    import torch
    n0, n1, n2 = shape
    h = n2 // 2 + 1
    if kmax is None:
        kmax = default_kmax(shape)
    rdt, cdt = (torch.float32, torch.complex64) if dtype == "f32" else (torch.float64, torch.complex128)
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def signed(n):
        i = torch.arange(n, device=device, dtype=rdt)
        return torch.where(i < n / 2, i, i - n)

    k1 = signed(n1).view(1, n1, 1)
    k2 = torch.arange(h, device=device, dtype=rdt).view(1, 1, h)
    U = torch.empty((3, n0, n1, h), dtype=cdt, device=device)
    for a in range(0, n0, slab):
        b = min(n0, a + slab)
        k0 = signed(n0)[a:b].view(b - a, 1, 1)
        K0, K1, K2 = torch.broadcast_tensors(k0, k1, k2)
        kk = torch.sqrt(K0 * K0 + K1 * K1 + K2 * K2)
        par = (K0 == 0) & (K1 == 0)
        # e1 = k x a / |k x a|, a = z-hat (x-hat where k is parallel to z-hat)
        az = torch.where(par, 0.0, 1.0).to(rdt)
        ax = 1.0 - az
        e1 = torch.stack((K1 * az, ax * K2 - K0 * az, -K1 * ax))
        ne = torch.sqrt((e1 * e1).sum(0))
        e1 = e1 / torch.where(ne > 0, ne, torch.ones_like(ne))
        e2 = torch.stack((K1 * e1[2] - K2 * e1[1], K2 * e1[0] - K0 * e1[2], K0 * e1[1] - K1 * e1[0]))
        e2 = e2 / torch.where(kk > 0, kk, torch.ones_like(kk))
        amp = torch.where((kk > 0) & (kk <= kmax), kk.clamp(min=1.0) ** (-11.0 / 6.0), torch.zeros_like(kk))
        p1 = torch.rand(kk.shape, generator=g, device=device, dtype=rdt) * (2 * math.pi)
        p2 = torch.rand(kk.shape, generator=g, device=device, dtype=rdt) * (2 * math.pi)
        w1 = torch.polar(amp / math.sqrt(2.0), p1)
        w2 = torch.polar(amp / math.sqrt(2.0), p2)
        U[:, a:b] = w1 * e1 + w2 * e2
        del K0, K1, K2, kk, par, az, ax, e1, ne, e2, amp, p1, p2, w1, w2
    u = torch.empty((3, n0, n1, n2), dtype=rdt, device=device)
    for c in range(3):
        u[c] = torch.fft.irfftn(U[c], s=(n0, n1, n2))
    ms = float((u.double() ** 2).mean()) if u.numel() < (1 << 28) else float(
        sum(float((u[c].double() ** 2).mean()) for c in range(3)) / 3)
    scale = 1.0 / math.sqrt(ms) if ms > 0 else 1.0
    u *= scale
    U *= scale
    return u, U
