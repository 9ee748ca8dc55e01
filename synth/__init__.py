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
  temperature T, 16 species), 10 isovalues of Z, weight = |grad T|, 30
  updates, 18 variables with 32-bin histograms and the full covariance; its
  sites come from ``flame_sites`` (independent draws, no global sort).

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


def _modes_separable(shape, seed: int, n_modes: int, kmin: float, kmax: float, L: float) -> np.ndarray:
    """The mode sum of ``fourier_field`` (same draws, integer wave vectors
    kappa) evaluated separably: for each distinct kappa_z a (y, x) plane
    P = sum of a e^{i phi} e^{2 pi i (ky y / ny + kx x / nx)} over its modes,
    then f[z] = Re sum_kz e^{2 pi i kz z / nz} P_kz as two real matrix
    products.  Float32, not normalised."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = (int(v) for v in shape)
    kmag = rng.uniform(kmin, kmax, size=n_modes)
    d = rng.normal(size=(n_modes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    kv = kmag[:, None] * d
    kint = np.rint(kv * (np.array([nx, ny, nz], dtype=np.float64) / L)).astype(np.int64)
    amp = kmag ** (-5.0 / 6.0)
    kzs = np.unique(kint[:, 2])
    P = np.zeros((len(kzs), ny, nx), dtype=np.complex64)
    ey = lambda k: np.exp(2j * math.pi * k * np.arange(ny) / ny).astype(np.complex64)
    ex = lambda k: np.exp(2j * math.pi * k * np.arange(nx) / nx).astype(np.complex64)
    for m in range(n_modes):
        j = int(np.searchsorted(kzs, kint[m, 2]))
        c = np.complex64(amp[m] * np.exp(1j * phase[m]))
        P[j] += np.outer(c * ey(kint[m, 1]), ex(kint[m, 0]))
    E = np.exp(2j * math.pi * np.outer(np.arange(nz), kzs) / nz).astype(np.complex64)
    Pf = P.reshape(len(kzs), ny * nx)
    c = np.ascontiguousarray  # contiguous real and imaginary parts: BLAS products
    f = c(E.real) @ c(Pf.real)
    f -= c(E.imag) @ c(Pf.imag)
    return f.reshape(nz, ny, nx)


def flame_fields(shape=(512, 512, 1024), seed: int = 4, n_species: int = 16, n_modes: int = 512):
    """Combustion-shaped fields on a box (nz, ny, nx): a thin wrinkled flame
    sheet across y.  s = (y/(ny-1) - 1/2) + 0.05 n with n the mode sum of
    ``fourier_field`` (512 modes, |k| in [1, 64] cycles per 512 voxels)
    rescaled to [-1, 1]; mixture fraction Z = (1 + tanh(s / 0.02)) / 2;
    temperature T = 300 + 1700 exp(-((Z - 0.3) / 0.1)^2); species
    Y_i = exp(-((Z - z_i) / w_i)^2) + 0.02 g_i with z_i = (i - 1/2) / n_species,
    w_i cycling 0.05, 0.1, 0.15, 0.2 (exponents clamped at -80), and g_i one
    N(0, 1) float32 field (numpy
    PCG64 ``default_rng(seed + 100)``) rolled by 7919 (i + 1) voxels in linear
    order.  Returns float32 [2 + n_species, nz, ny, nx] = (Z, T, Y_1, ...)."""
    nz, ny, nx = (int(v) for v in shape)
    s = _modes_separable(shape, seed, n_modes, 1.0, 64.0, 512.0)
    lo, hi = float(s.min()), float(s.max())
    s -= np.float32(lo)
    s *= np.float32(2.0 * 0.05 / (hi - lo)) if hi > lo else np.float32(0.0)
    s -= np.float32(0.05)
    s += (np.arange(ny, dtype=np.float32) / np.float32(max(ny - 1, 1)) - np.float32(0.5))[None, :, None]
    out = np.empty((2 + n_species,) + (nz, ny, nx), dtype=np.float32)
    Z = out[0]
    s /= np.float32(0.02)
    np.tanh(s, out=Z)
    del s
    Z += 1.0
    Z *= 0.5
    t = out[1]
    np.subtract(Z, np.float32(0.3), out=t)
    t /= np.float32(0.1)
    np.square(t, out=t)
    np.negative(t, out=t)
    np.exp(t, out=t)
    t *= 1700.0
    t += 300.0
    widths = (0.05, 0.1, 0.15, 0.2)
    g = np.random.default_rng(seed + 100).standard_normal(size=Z.size, dtype=np.float32)
    g *= np.float32(0.02)
    rolled = np.empty_like(g)
    n = g.size
    for i in range(n_species):
        zi = np.float32((i + 0.5) / n_species)
        wi = np.float32(widths[i % 4])
        y = out[2 + i]
        np.subtract(Z, zi, out=y)
        y /= wi
        np.square(y, out=y)
        np.negative(y, out=y)
        np.maximum(y, np.float32(-80.0), out=y)  # no subnormal results (< 2e-35 change)
        np.exp(y, out=y)
        k = (7919 * (i + 1)) % n  # rolled = np.roll(g, k), without a new array
        rolled[k:] = g[:n - k]
        rolled[:k] = g[n - k:]
        y += rolled.reshape(Z.shape)
    return out


def flame_sites(comp: np.ndarray, n_comp: int, weights: np.ndarray, rho: float, seed: int) -> np.ndarray:
    """Initial sites for large volumes: every voxel is drawn independently with
    probability min(1, w_v / (rho * mean w)) (uniform numbers from numpy PCG64
    ``default_rng(seed)``, one per voxel in linear order), and a component
    that drew no voxel gets its first voxel.  Ids ordered by (component,
    linear index).  uint32 linear indices."""
    c = np.ascontiguousarray(comp, dtype=np.uint32).ravel()
    w = np.ascontiguousarray(weights).ravel()
    rng = np.random.default_rng(seed)
    p = w.astype(np.float32) / np.float32(rho * float(w.mean(dtype=np.float64)))
    u = rng.random(size=c.size, dtype=np.float32)
    pick = np.flatnonzero((u < p) & (c != 0xFFFFFFFF))
    del u, p
    have = np.zeros(n_comp, dtype=bool)
    have[c[pick]] = True
    miss = np.flatnonzero(~have)
    if len(miss):
        # first voxel of each component without a site
        first = np.full(n_comp, np.iinfo(np.int64).max, dtype=np.int64)
        lab = np.flatnonzero(c != 0xFFFFFFFF)
        np.minimum.at(first, c[lab], lab)
        pick = np.concatenate([pick, first[miss]])
    order = np.lexsort((pick, c[pick]))
    return pick[order].astype(np.uint32)


def flame_workload(shape=(512, 512, 1024), seed: int = 4, iters: int = 30, n_bins: int = 32,
                   rho: float = 4096.0) -> Workload:
    """The combustion-shaped workload: 1024 x 512 x 512 (nx, ny, nz), 10
    isovalues of Z at 0.05 .. 0.95, weight = |grad T| as uint16, 18 variables
    (Z, T, 16 species) with 32-bin histograms and the full 18 x 18 covariance,
    30 updates, one site per 4096 weight-scaled voxels."""
    v = flame_fields(shape, seed)
    iso = np.array([0.05 + 0.1 * i for i in range(10)], dtype=np.float32)
    w = gradient_weight(v[1])
    edges = histogram_edges(v, n_bins)
    return Workload("flame", v[0], iso, w, v, edges, iters, rho, seed, True, {"n_species": 16})


def batch_specs(n_jobs: int = 64, seed: int = 3):
    """The uneven batch: per job (shape, seed, isovalue count).  Long edge
    e from {32, 48, ..., 192}; a cube, or by coin a 2:1:1 box with the long
    axis random; 3..10 isovalues; job seeds 3000 + j."""
    rng = np.random.default_rng(seed)
    specs = []
    for j in range(n_jobs):
        e = int(rng.choice(np.arange(32, 193, 16)))
        if rng.random() < 0.5:
            shape = (e, e, e)
        else:
            sh = [e // 2, e // 2, e // 2]
            sh[int(rng.integers(0, 3))] = e
            shape = tuple(sh)
        specs.append((shape, 3000 + j, int(rng.integers(3, 11))))
    return specs


def fourier_job(shape, seed: int, n_iso: int, n_vars: int = 8, n_bins: int = 32, n_modes: int = 128):
    """Host arrays of one batch or serving job: a Fourier field, isovalues at
    quantiles, |grad| weights, n_vars Fourier variables (seeds 1000 seed + 1 + j)
    and their histogram edges."""
    f = fourier_field(shape, seed, n_modes=n_modes)
    iso = quantile_isovalues(f, [(i + 1) / (n_iso + 1) for i in range(n_iso)])
    w = gradient_weight(f)
    x = np.stack([fourier_field(shape, 1000 * seed + 1 + j, n_modes=n_modes) for j in range(n_vars)])
    return f, iso, w, np.ascontiguousarray(x), histogram_edges(x, n_bins)
