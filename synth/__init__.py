"""Seeded synthetic inputs shaped like the paper's workloads.

The paper's datasets (a DNS of a premixed hydrogen/ammonia/nitrogen flame and a
channel-flow lambda_2 field, Sec. 6) are not available, so every input here is
generated from a seed.  This module holds no arithmetic of the method itself:
it draws fields, isovalues, saliency weights, extra variables, histogram edges
and initial sites, which both the GPU library and the CPU oracle consume as
inputs.

Workloads (all arrays are C-order [nz, ny, nx], linear index x + nx*(y + ny*z)):

* ``blobs``   64^3 sum of 8 isotropic Gaussians plus N(0, 0.01^2) noise,
  4 isovalues at the 0.2/0.4/0.6/0.8 quantiles, uniform weight, one site per
  512 voxels of each component, 10 updates, 3 statistics variables
  (the field and two N(0,1) fields), 16-bin histograms, no covariance.
* ``fourier`` 256^3 turbulence-like field: 512 Fourier modes with |k| uniform
  in [1, 64] cycles per domain, isotropic directions, random phases and
  amplitudes |k|^(-5/6) (so E(k) ~ k^(-5/3)), normalised to [0, 1]; 8
  isovalues at quantiles i/9; weight = |grad f| quantised to uint16; one site
  per 4096 weight-scaled voxels; 20 updates; 8 variables of the same spectrum,
  32-bin histograms and the full 8x8 covariance.
* ``flame``   1024x512x512 combustion-shaped sheet (mixture fraction Z,
  temperature T, 16 species), 10 isovalues of Z, weight = |grad T|.

Wave vectors are rounded to integers (cycles per box edge) so that a field is
one inverse FFT of a sparse spectrum; the field is then periodic on its box.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field

import numpy as np

try:  # multi-threaded FFT when scipy is present
    import scipy.fft as _fft

    def _ifftn(spec):
        return _fft.ifftn(spec, workers=-1, overwrite_x=True)
except Exception:  # pragma: no cover
    def _ifftn(spec):
        return np.fft.ifftn(spec)


# --------------------------------------------------------------------------
# fields
def blobs_field(shape=(64, 64, 64), seed: int = 1, n_blobs: int = 8, noise: float = 0.01) -> np.ndarray:
    """Sum of isotropic Gaussians A exp(-|x-c|^2 / (2 sigma^2)) plus white noise.

    Centres uniform in the box, sigma ~ U[4, 10] voxels, A ~ U[0.5, 1],
    noise N(0, noise^2); evaluated at integer voxel coordinates, float32."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    c = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * np.array([nx, ny, nz], dtype=np.float64)
    sig = rng.uniform(4.0, 10.0, size=n_blobs)
    amp = rng.uniform(0.5, 1.0, size=n_blobs)
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    f = np.zeros(shape, dtype=np.float64)
    for i in range(n_blobs):
        r2 = (x - c[i, 0]) ** 2 + (y - c[i, 1]) ** 2 + (z - c[i, 2]) ** 2
        f += amp[i] * np.exp(-r2 / (2.0 * sig[i] ** 2))
    f += rng.normal(0.0, noise, size=shape)
    return f.astype(np.float32)


def fourier_field(shape, seed: int, n_modes: int = 512, kmin: float = 1.0, kmax: float = 64.0,
                  L: float | None = None, normalise: bool = True) -> np.ndarray:
    """Sum of random Fourier modes a cos(2 pi kappa.x + phi), E(k) ~ k^(-5/3).

    |k| ~ U[kmin, kmax] in cycles per ``L`` (default: the longest edge), the
    direction is uniform on the sphere, phi ~ U[0, 2 pi) and a = |k|^(-5/6).
    Each component of k is rescaled to cycles per box edge and rounded to an
    integer (kappa), so the field is the real part of one inverse FFT of a
    sparse spectrum and is periodic on its box.  Float32, normalised to [0, 1]
    unless ``normalise`` is False."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = (int(s) for s in shape)
    L = float(max(shape)) if L is None else float(L)
    kmag = rng.uniform(kmin, kmax, size=n_modes)
    d = rng.normal(size=(n_modes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    kv = kmag[:, None] * d  # cycles per L, order (x, y, z)
    kint = np.rint(kv * (np.array([nx, ny, nz], dtype=np.float64) / L)).astype(np.int64)
    amp = kmag ** (-5.0 / 6.0)
    n = nz * ny * nx
    big = n > (1 << 25)
    spec = np.zeros((nz, ny, nx), dtype=np.complex64 if big else np.complex128)
    np.add.at(spec, (kint[:, 2] % nz, kint[:, 1] % ny, kint[:, 0] % nx), amp * np.exp(1j * phase))
    f = _ifftn(spec).real * float(n)
    del spec
    if normalise:
        lo, hi = f.min(), f.max()
        f = (f - lo) / (hi - lo) if hi > lo else np.zeros_like(f)
    return f.astype(np.float32)


# --------------------------------------------------------------------------
# derived inputs
def quantile_isovalues(f: np.ndarray, qs) -> np.ndarray:
    """Isovalues at the given quantiles of f (linear interpolation, float64),
    cast to float32 and nudged upward where the cast makes them non-increasing."""
    v = np.quantile(f.astype(np.float64).ravel(), np.asarray(qs, dtype=np.float64), method="linear")
    iso = v.astype(np.float32)
    for i in range(1, len(iso)):
        if not iso[i - 1] < iso[i]:
            iso[i] = np.nextafter(iso[i - 1], np.float32(np.inf))
    return iso


def gradient_weight(f: np.ndarray) -> np.ndarray:
    """Saliency weight max(1, round(65535 |grad f| / max |grad f|)) as uint16."""
    f64 = f.astype(np.float64)
    mag2 = np.zeros(f.shape, dtype=np.float64)
    for axis in range(f.ndim):
        if f.shape[axis] >= 2:          # an axis of length 1 has no gradient
            mag2 += np.gradient(f64, axis=axis) ** 2
    mag = np.sqrt(mag2)
    gmax = mag.max()
    if gmax <= 0:
        return np.ones(f.shape, dtype=np.uint16)
    w = np.rint(65535.0 * mag / gmax)
    return np.clip(w, 1, 65535).astype(np.uint16)


def histogram_edges(variables: np.ndarray, n_bins: int) -> np.ndarray:
    """Per-variable edges linspace(min, max, B+1) in float64, cast to float32."""
    m = variables.shape[0]
    flat = variables.reshape(m, -1)
    e = np.empty((m, n_bins + 1), dtype=np.float32)
    for j in range(m):
        lo, hi = float(flat[j].min()), float(flat[j].max())
        e[j] = np.linspace(lo, hi, n_bins + 1).astype(np.float32)
    return e


def seed_sites(comp: np.ndarray, n_comp: int, weights: np.ndarray | None, rho: float, seed: int) -> np.ndarray:
    """Initial sites: n_c = max(ceil(sum_C w / (rho * mean_V w)), 1) per component
    (uniform weight: max(ceil(|C| / rho), 1)), drawn without replacement with
    probability proportional to w (uniform when ``weights`` is None).

    Draws use exponential keys E_v / w_v (the n_c smallest win), one draw per
    voxel in linear order from numpy PCG64 ``default_rng(seed)``.  Site ids are
    ordered by (component id, draw order).  Returned as uint32 linear indices."""
    c = np.ascontiguousarray(comp, dtype=np.uint32).ravel()
    n = c.size
    rng = np.random.default_rng(seed)
    if weights is None:
        w = np.ones(n, dtype=np.float64)
    else:
        w = np.ascontiguousarray(weights).ravel().astype(np.float64)
    mass = np.bincount(c, weights=w, minlength=n_comp)
    size = np.bincount(c, minlength=n_comp)
    mean_w = w.mean()
    nc = np.maximum(np.ceil(mass / (rho * mean_w) - 1e-9), 1).astype(np.int64)
    # a component cannot hold more distinct sites than voxels with positive weight
    posw = np.bincount(c, weights=(w > 0).astype(np.float64), minlength=n_comp).astype(np.int64)
    nc = np.minimum(nc, np.maximum(posw, 1))
    nc = np.minimum(nc, size)
    e = rng.exponential(size=n)
    with np.errstate(divide="ignore"):
        key = np.where(w > 0, e / np.where(w > 0, w, 1.0), np.inf)
    order = np.lexsort((key, c))            # by component, then key
    start = np.concatenate([[0], np.cumsum(size)[:-1]])
    take = np.concatenate([order[start[k]:start[k] + nc[k]] for k in range(n_comp)]) if n_comp else \
        np.zeros(0, dtype=np.int64)
    return take.astype(np.uint32)


# --------------------------------------------------------------------------
# workloads
@dataclass
class Workload:
    name: str
    field: np.ndarray                 # float32 [nz, ny, nx]
    iso: np.ndarray                   # float32 [K]
    weights: np.ndarray | None        # uint16 [nz, ny, nx] or None (uniform)
    variables: np.ndarray             # float32 [m, nz, ny, nx]
    edges: np.ndarray | None          # float32 [m, B+1]
    iters: int
    rho: float
    seed: int
    cov: bool
    meta: dict = dc_field(default_factory=dict)

    @property
    def shape(self):
        return self.field.shape

    @property
    def n_bands(self):
        return len(self.iso) + 1


def blobs_workload(shape=(64, 64, 64), seed: int = 1, iters: int = 10) -> Workload:
    """The 64^3 Gaussian-blob workload (uniform weight, 3 variables, 16 bins)."""
    f = blobs_field(shape, seed)
    iso = quantile_isovalues(f, [0.2, 0.4, 0.6, 0.8])
    rng = np.random.default_rng(seed + 100)
    extra = rng.normal(0.0, 1.0, size=(2,) + tuple(shape)).astype(np.float32)
    variables = np.concatenate([f[None], extra], axis=0)
    edges = histogram_edges(variables, 16)
    return Workload("blobs", f, iso, None, variables, edges, iters, 512.0, seed, False,
                    {"n_blobs": 8, "noise_sigma": 0.01})


def fourier_workload(shape=(256, 256, 256), seed: int = 2, iters: int = 20, n_iso: int = 8,
                     n_vars: int = 8, n_bins: int = 32, rho: float = 4096.0, n_modes: int = 512) -> Workload:
    """The turbulence-like Fourier workload (|grad f| weight, m vars, B bins, covariance)."""
    f = fourier_field(shape, seed, n_modes=n_modes)
    iso = quantile_isovalues(f, [(i + 1) / (n_iso + 1) for i in range(n_iso)])
    w = gradient_weight(f)
    variables = np.stack([fourier_field(shape, 1000 * seed + 1 + j, n_modes=n_modes) for j in range(n_vars)])
    edges = histogram_edges(variables, n_bins)
    return Workload("fourier", f, iso, w, variables, edges, iters, rho, seed, True, {"n_modes": n_modes})


def workload_sites(wl: Workload, comp: np.ndarray, n_comp: int) -> np.ndarray:
    """Initial sites for a workload from its component labels (seed 7919 * seed + 1)."""
    return seed_sites(comp, n_comp, wl.weights, wl.rho, 7919 * wl.seed + 1)
