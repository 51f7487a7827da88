"""Seeded synthetic fp32 fields shaped like the paper's evaluation data.

The paper evaluates on SDRBench fields (HACC 1D, CESM-ATM 2D, Hurricane 3D,
Nyx 3D; table of datasets in Sec. 4.1).  Those files are not available here,
so these generators stand in for them with the same shapes, value ranges and
smoothness character.  They hold no part of the compression method: both the
oracle-side tests and the GPU path consume the arrays they return.

All generators draw from ``numpy.random.default_rng(seed)`` (PCG64) in float64
and cast to float32 at the end, so a (generator, shape, seed) triple names one
exact array on every machine.
"""
from __future__ import annotations

import numpy as np

# Workload shapes (slowest -> fastest axis).
C1_SHAPE = (1800, 3600)          # CESM-ATM-like 2D climate field
C2_SHAPE = (100, 500, 500)       # Hurricane-ISABEL-like 3D field
C3_N = 280_953_867               # HACC-like 1D particle coordinate array


def fourier2d(shape=C1_SHAPE, seed: int = 1, modes: int = 64, noise: float = 1e-3) -> np.ndarray:
    """Sum of ``modes`` random Fourier modes with amplitude |k|^-2 plus
    N(0, noise) white noise.  Integer wavenumbers kx in [0, 32],
    ky in [-32, 32], |k| >= 1, phases uniform in [0, 2 pi)."""
    ny, nx = shape
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < modes:
        kx = int(rng.integers(0, 33))
        ky = int(rng.integers(-32, 33))
        if kx * kx + ky * ky >= 1:
            ks.append((ky, kx))
    k = np.array(ks, dtype=np.float64)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=modes)
    amp = (k[:, 0] ** 2 + k[:, 1] ** 2) ** -1.0
    iy = np.arange(ny, dtype=np.float64)[:, None]
    ix = np.arange(nx, dtype=np.float64)[:, None]
    ay = 2.0 * np.pi * iy * (k[:, 0] / ny)[None, :] + phase[None, :]   # (ny, modes)
    ax = 2.0 * np.pi * ix * (k[:, 1] / nx)[None, :]                    # (nx, modes)
    # cos(a + b) = cos a cos b - sin a sin b, summed over modes as two products
    field = (np.cos(ay) * amp) @ np.cos(ax).T - (np.sin(ay) * amp) @ np.sin(ax).T
    field += rng.normal(0.0, noise, size=shape)
    return field.astype(np.float32)


def grf(shape, seed: int, slope: float = -11.0 / 3.0, workers: int = 0) -> np.ndarray:
    """Unit-variance Gaussian random field with power spectrum P(|k|) ~ |k|^slope
    (default: Kolmogorov E(k) ~ k^-5/3, i.e. P ~ k^-11/3 in 3D), by FFT
    filtering of white noise.  float64 result.  ``workers`` > 0 takes the
    transforms from scipy.fft with that many threads (same definition, other
    rounding: a different array than the default)."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    if workers > 0:
        import scipy.fft as sfft
        spec = sfft.rfftn(white, workers=workers)
    else:
        spec = np.fft.rfftn(white)
    freqs = [np.fft.fftfreq(n) for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    k2 = np.zeros(spec.shape, dtype=np.float64)
    for ax, f in enumerate(freqs):
        sh = [1] * len(shape)
        sh[ax] = f.size
        k2 = k2 + (f.reshape(sh) * shape[ax]) ** 2
    k2.flat[0] = 1.0
    filt = k2 ** (slope / 4.0)       # sqrt(P) = |k|^(slope/2) = (k^2)^(slope/4)
    filt.flat[0] = 0.0               # zero mean
    spec *= filt
    if workers > 0:
        field = sfft.irfftn(spec, s=shape, axes=list(range(len(shape))), workers=workers)
    else:
        field = np.fft.irfftn(spec, s=shape, axes=list(range(len(shape))))
    sd = field.std()
    if sd > 0:
        field /= sd
    return field


def hurricane3d(shape=C2_SHAPE, seed: int = 2, vmax: float = 10.0, core: float = 25.0) -> np.ndarray:
    """Kolmogorov GRF plus a Lamb-Oseen vortex speed profile
    v(r) = V (r_c / r)(1 - exp(-r^2 / r_c^2)) centred in the (y, x) plane,
    tapered linearly with height."""
    nz, ny, nx = shape
    g = grf(shape, seed)
    yy = np.arange(ny, dtype=np.float64)[:, None] - ny / 2.0
    xx = np.arange(nx, dtype=np.float64)[None, :] - nx / 2.0
    r = np.sqrt(yy * yy + xx * xx)
    r = np.where(r == 0.0, 1e-12, r)
    v = vmax * (core / r) * (1.0 - np.exp(-(r * r) / (core * core)))
    taper = 1.0 - np.arange(nz, dtype=np.float64) / (2.0 * nz)
    g += taper[:, None, None] * v[None, :, :]
    return g.astype(np.float32)


def particles1d(n: int = C3_N, seed: int = 3, box: float = 256.0, jitter: float = 0.05,
                shuffle_block: int = 4096, chunk: int = 1 << 24) -> np.ndarray:
    """Sorted uniform positions in [0, box) plus N(0, jitter) noise, cut into
    blocks of ``shuffle_block`` elements whose order is permuted (particle
    arrays stored in spatially sorted tiles visited in random order).

    Sorted uniforms are drawn as normalised cumulative sums of n + 1
    exponential spacings (two passes over the same seeded stream), which
    avoids sorting n values."""
    def spacings():
        rng = np.random.default_rng(seed)
        done = 0
        while done < n:
            m = min(chunk, n - done)
            yield rng.standard_exponential(m)
            done += m

    total = 0.0
    for s in spacings():
        total += float(s.sum())
    total += float(np.random.default_rng(seed + 1).standard_exponential())
    out = np.empty(n, dtype=np.float32)
    jit = np.random.default_rng(seed + 2)
    acc = 0.0
    done = 0
    for s in spacings():
        c = np.cumsum(s) + acc
        acc = float(c[-1])
        pos = c * (box / total) + jit.normal(0.0, jitter, size=s.size)
        out[done:done + s.size] = pos.astype(np.float32)
        done += s.size
    if shuffle_block and n > shuffle_block:
        nblk = (n + shuffle_block - 1) // shuffle_block
        perm = np.random.default_rng(seed + 3).permutation(nblk)
        starts = perm * shuffle_block
        lens = np.minimum(shuffle_block, n - starts)
        res = np.empty_like(out)
        o = 0
        for s0, ln in zip(starts.tolist(), lens.tolist()):
            res[o:o + ln] = out[s0:s0 + ln]
            o += ln
        out = res
    return out


def workload(name: str, scale: float = 1.0) -> np.ndarray:
    """Named workload arrays: 'c1' (2D 1800x3600), 'c2' (3D 100x500x500),
    'c3' (1D 280,953,867).  ``scale`` < 1 shrinks every axis (for tests)."""
    def sc(shape):
        return tuple(max(1, int(round(s * scale))) for s in shape)
    if name == "c1":
        return fourier2d(sc(C1_SHAPE))
    if name == "c2":
        return hurricane3d(sc(C2_SHAPE))
    if name == "c3":
        return particles1d(sc((C3_N,))[0])
    raise KeyError(name)


C4_FIELDS = 64
C4_EDGES = (64, 512)
C4_EBS = (1e-2, 1e-3, 1e-4)


def _wrap_take(a: np.ndarray, axis: int, start: int, n: int) -> np.ndarray:
    """Elements start .. start + n - 1 of ``a`` along ``axis``, wrapping around."""
    size = a.shape[axis]
    start %= size
    if start + n <= size:
        return np.take(a, range(start, start + n), axis=axis) if n < size else a
    head = [slice(None)] * a.ndim
    tail = [slice(None)] * a.ndim
    head[axis] = slice(start, size)
    tail[axis] = slice(0, start + n - size)
    return np.concatenate([a[tuple(head)], a[tuple(tail)]], axis=axis)


class BatchWorkload:
    """Uneven 3D fields for batched compression (Nyx-like mixed fields):
    field 0 is a 512^3 log-normal density exp(2 g - 2) of a unit-variance
    Kolmogorov GRF g (sigma = 2: heavy upper tail); fields 1.. have edges
    drawn uniformly from [64, 512] and are boxes cut (with periodic wrap, at
    seeded offsets) from one 512^3 Kolmogorov GRF, each with its own seeded
    offset and scale.  Each field has a value-range-relative eb drawn from
    {1e-2, 1e-3, 1e-4}.  ``scale`` < 1 shrinks every edge (tests)."""

    def __init__(self, n: int = C4_FIELDS, seed: int = 4, scale: float = 1.0, workers: int = 8):
        rng = np.random.default_rng(seed)
        self.seed = seed
        self.scale = scale
        lo, hi = C4_EDGES
        def sc(e):
            return max(1, int(round(e * scale)))
        self.pool_edge = sc(512)
        self.shapes = [(sc(512),) * 3]
        for _ in range(1, n):
            self.shapes.append(tuple(sc(int(e)) for e in rng.integers(lo, hi + 1, size=3)))
        self.ebs = [float(e) for e in rng.choice(np.array(C4_EBS), size=n)]
        self.offsets = [tuple(int(o) for o in rng.integers(0, self.pool_edge, size=3)) for _ in range(n)]
        self.affine = [(float(a), float(b)) for a, b in zip(rng.normal(0.0, 10.0, n), rng.uniform(0.5, 4.0, n))]
        self._pool = None
        self.workers = workers

    def __len__(self):
        return len(self.shapes)

    def field(self, i: int) -> np.ndarray:
        if i == 0:
            g = grf(self.shapes[0], self.seed + 1000, workers=self.workers)
            return np.exp(2.0 * g - 2.0).astype(np.float32)
        if self._pool is None:
            self._pool = grf((self.pool_edge,) * 3, self.seed + 2000, workers=self.workers).astype(np.float32)
        box = self._pool
        for ax, (n, o) in enumerate(zip(self.shapes[i], self.offsets[i])):
            box = _wrap_take(box, ax, o, n)
        a, b = self.affine[i]
        return (box * np.float32(b) + np.float32(a)).astype(np.float32)

    def elements(self) -> int:
        return int(sum(int(np.prod(s)) for s in self.shapes))


C5_RATES = (50, 100, 200, 500, 1000, 2000)
C5_RATES_SATURATION = (5000, 10000, 20000)   # past the configured range, until the server saturates


class ServeWorkload:
    """Request pool and Poisson request streams for serving: ``pool`` fields,
    a third each 1D (n log-uniform in [1e5, 1e8]), 2D (edges log-uniform in
    [64, 3600]) and 3D (edges log-uniform in [32, 256]), cut at seeded offsets
    from one Kolmogorov GRF per dimensionality (1D of 2^27 points, 2D 3600^2,
    3D 256^3; spectra k^-5/3, k^-8/3, k^-11/3).  ``scale`` < 1 shrinks the
    size ranges (tests)."""

    def __init__(self, pool: int = 48, seed: int = 5, scale: float = 1.0, workers: int = 8):
        rng = np.random.default_rng(seed)
        self.seed = seed
        self.workers = workers
        def lu(lo, hi):
            return float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        s = scale
        self.src_shape = {1: (max(1024, int((1 << 27) * s)),), 2: (max(64, int(3600 * s)),) * 2,
                          3: (max(32, int(256 * s)),) * 3}
        self.shapes = []
        for k in range(pool):
            nd = 1 + k % 3
            if nd == 1:
                sh = (max(1, int(lu(1e5 * s, 1e8 * s))),)
            elif nd == 2:
                sh = tuple(max(1, int(lu(64 * s, 3600 * s))) for _ in range(2))
            else:
                sh = tuple(max(1, int(lu(32 * s, 256 * s))) for _ in range(3))
            self.shapes.append(tuple(min(a, b) for a, b in zip(sh, self.src_shape[nd])))
        self.offsets = [tuple(int(o) for o in rng.integers(0, 1 << 30, size=len(sh))) for sh in self.shapes]
        self._src = {}

    def __len__(self):
        return len(self.shapes)

    def field(self, i: int) -> np.ndarray:
        sh = self.shapes[i]
        nd = len(sh)
        if nd not in self._src:
            slope = {1: -5.0 / 3.0, 2: -8.0 / 3.0, 3: -11.0 / 3.0}[nd]
            self._src[nd] = grf(self.src_shape[nd], self.seed + 100 * nd, slope=slope,
                                workers=self.workers).astype(np.float32)
        box = self._src[nd]
        for ax, (n, o) in enumerate(zip(sh, self.offsets[i])):
            box = _wrap_take(box, ax, o, n)
        return np.ascontiguousarray(box)

    def release_sources(self):
        self._src = {}

    def requests(self, rate: float, n: int, seed: int):
        """n requests arriving as a Poisson process of the given rate: arrays
        of arrival times (s), kinds (0 compress, 1 decompress), pool indices
        and value-range-relative error bounds (log-uniform in [1e-5, 1e-2])."""
        rng = np.random.default_rng([self.seed, int(rate), seed])
        t = np.cumsum(rng.exponential(1.0 / rate, size=n))
        kind = rng.integers(0, 2, size=n)
        idx = rng.integers(0, len(self.shapes), size=n)
        eb = np.exp(rng.uniform(np.log(1e-5), np.log(1e-2), size=n))
        return t, kind, idx, eb
