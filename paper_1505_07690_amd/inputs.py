"""Seeded synthetic inputs shared by the oracle-side and the GPU-side tests.

This module holds no arithmetic of the transform itself: it only draws test
volumes and orientation sets.

* ``tubes``: crossing-tube volumes standing in for the elongated, crossing and
  noisy structures the paper processes (Sec. 4.1, Figs. 6-7: artificial crossing
  data with Gaussian noise; vessel data).  The datasets behind those figures are
  not available, so these seeded volumes replace them.
* ``icosahedral_orientations``: orientation sets from the icosahedron and its
  midpoint tessellations (Sec. 2.1: the sphere is sampled with platonic solids,
  refined by tessellation), in the standard orientation whose vertices are the
  cyclic permutations of (0, +-1, +-phi).  The sets are antipodally closed.
* ``bandlimited``: white noise low-passed to a ball in the DFT grid, the class
  of inputs for which the discrete reconstruction of Eq. (8) is exact.
"""
from __future__ import annotations

import numpy as np

__all__ = ["tubes", "tubes_device", "icosahedral_orientations", "platonic_orientations", "bandlimited", "CONFIGS",
           "config_volume",
           "serving_stream", "SERVING_SHAPES"]


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def _tube_params(shape, n_tubes, sigma, n_cross_pairs, rng):
    nz, ny, nx = (int(s) for s in shape)
    ext = np.array([nx, ny, nz], dtype=np.float64)
    dirs, cents = [], []
    t = 0
    for _ in range(n_cross_pairs):
        q = rng.uniform(0.3, 0.7, 3) * ext
        ua = _unit(rng.standard_normal(3))
        ub = _unit(rng.standard_normal(3))
        delta = rng.uniform(0.0, 4.0)
        w = np.cross(ua, ub)
        w = w / np.linalg.norm(w)
        dirs += [ua, ub]
        cents += [q, q + delta * w]
        t += 2
    for _ in range(n_tubes - t):
        dirs.append(_unit(rng.standard_normal(3)))
        cents.append(rng.uniform(0.25, 0.75, 3) * ext)
    if np.isscalar(sigma):
        sig = np.full(n_tubes, float(sigma))
    else:
        sig = rng.uniform(sigma[0], sigma[1], n_tubes)
    return dirs, cents, sig


def tubes(shape, n_tubes, sigma, noise, n_cross_pairs=0, seed=0):
    """Sum of straight tubes with Gaussian cross-section plus white noise.

    shape: (Nz, Ny, Nx); voxel centres sit at integer coordinates; the
    returned array is float32 [Nz][Ny][Nx] (x fastest).
    sigma: a float (every tube) or a (lo, hi) range drawn uniformly per tube.
    The first ``2 * n_cross_pairs`` tubes come in forced crossing pairs whose
    axes pass within 4 voxels of each other.

    Draw order (PCG64 via numpy.random.default_rng(seed)): for every tube in
    turn, pairs first: [pair: q (3), u_a (3), u_b (3), delta (1)] or
    [single: u (3), c (3)]; then all sigmas (n_tubes, if a range); then the
    noise field.
    """
    nz, ny, nx = (int(s) for s in shape)
    rng = np.random.default_rng(seed)
    dirs, cents, sig = _tube_params(shape, n_tubes, sigma, n_cross_pairs, rng)
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    f = np.zeros((nz, ny, nx), dtype=np.float64)
    for u, c, s in zip(dirs, cents, sig):
        dx, dy, dz = x - c[0], y - c[1], z - c[2]
        along = dx * u[0] + dy * u[1] + dz * u[2]
        d2 = dx * dx + dy * dy + dz * dz - along * along
        f += np.exp(-np.maximum(d2, 0.0) / (2.0 * s * s))
    f += noise * rng.standard_normal((nz, ny, nx))
    return f.astype(np.float32)


def tubes_device(shape, n_tubes, sigma, noise, n_cross_pairs=0, seed=0, device="cuda"):
    """The same tube geometry as ``tubes`` (same parameter draws), evaluated
    in float32 with torch on `device`; the noise comes from a torch generator
    seeded with `seed`, so the values differ from ``tubes`` by the noise
    field and float32 rounding.  For request streams whose volumes are made
    on the device."""
    import torch
    nz, ny, nx = (int(s) for s in shape)
    rng = np.random.default_rng(seed)
    dirs, cents, sig = _tube_params(shape, n_tubes, sigma, n_cross_pairs, rng)
    z = torch.arange(nz, dtype=torch.float32, device=device)[:, None, None]
    y = torch.arange(ny, dtype=torch.float32, device=device)[None, :, None]
    x = torch.arange(nx, dtype=torch.float32, device=device)[None, None, :]
    f = torch.zeros((nz, ny, nx), dtype=torch.float32, device=device)
    for u, c, s in zip(dirs, cents, sig):
        dx, dy, dz = x - float(c[0]), y - float(c[1]), z - float(c[2])
        along = dx * float(u[0]) + dy * float(u[1]) + dz * float(u[2])
        d2 = (dx * dx + dy * dy + dz * dz - along * along).clamp_min_(0.0)
        f += torch.exp(d2 * (-0.5 / float(s * s)))
    g = torch.Generator(device=device).manual_seed(int(seed))
    f += noise * torch.randn((nz, ny, nx), generator=g, device=device, dtype=torch.float32)
    return f


def serving_stream(n_requests=1000, rate=50.0, seed=4):
    """Poisson request stream: exponential gaps of mean 1/rate seconds; per
    request a shape from SERVING_SHAPES, N_o from {42, 162} and L from
    {16, 24} drawn independently and uniformly, and a volume seed.  Returns
    a list of (t_arrival_s, shape, n_orients, L, volume_seed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate)
        shape = SERVING_SHAPES[int(rng.integers(len(SERVING_SHAPES)))]
        n = (42, 162)[int(rng.integers(2))]
        L = (16, 24)[int(rng.integers(2))]
        out.append((t, shape, n, L, int(rng.integers(2 ** 31))))
    return out


def _icosahedron():
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-p, p):
            v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(v, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # faces: triples of mutually nearest vertices (edge length is the minimum distance)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    emin = d[d > 1e-9].min()
    adj = np.abs(d - emin) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    return v, faces


def icosahedral_orientations(level):
    """Icosahedron vertices (level 0: 12), subdivided `level` times by edge
    midpoints projected to the sphere (42, 162, ...).  float64 [N_o][3] as
    (x, y, z) unit vectors."""
    v, faces = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        index = {}
        new_faces = []
        pts = list(verts)

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in index:
                m = _unit(np.add(pts[a], pts[b]))
                index[key] = len(pts)
                pts.append(tuple(m))
            return index[key]

        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        verts, faces = pts, new_faces
    return np.array(verts, dtype=np.float64)


def platonic_orientations(name):
    """Vertex directions of a platonic solid (Sec. 2.1 samples the sphere with
    them): "tetrahedron" (4, not antipodally closed), "octahedron" (6),
    "cube" (8), "dodecahedron" (20), "icosahedron" (12).  float64 [N][3]."""
    p = (1.0 + 5.0 ** 0.5) / 2.0
    if name == "tetrahedron":
        v = [(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]
    elif name == "octahedron":
        v = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    elif name == "cube":
        v = [(a, b, c) for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)]
    elif name == "dodecahedron":
        v = [(a, b, c) for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)]
        for a in (-1, 1):
            for b in (-1, 1):
                v += [(0, a / p, b * p), (a / p, b * p, 0), (a * p, 0, b / p)]
    elif name == "icosahedron":
        return icosahedral_orientations(0)
    else:
        raise ValueError(name)
    v = np.array(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def bandlimited(shape, frac, seed=0, batch=None, dtype=np.float32):
    """White noise restricted to the DFT frequencies with |omega| <= frac*pi
    (omega_d = 2*pi*k_d/N_d with k_d in [-N_d/2, N_d/2)), no Nyquist plane,
    real output (float32 unless `dtype` says otherwise; rounding to float32
    leaves out-of-band noise at the 1e-8 level).  numpy.fft is used only to
    produce the input."""
    rng = np.random.default_rng(seed)
    shp = tuple(int(s) for s in shape)
    full = shp if batch is None else (batch,) + shp
    w = rng.standard_normal(full)
    W = np.fft.fftn(w, axes=(-3, -2, -1))
    om2 = np.zeros(shp)
    nyq = np.zeros(shp, dtype=bool)
    for ax, n in enumerate(shp):
        k = np.arange(n)
        kt = np.where(k < (n + 1) // 2, k, k - n)
        sh = [1, 1, 1]
        sh[ax] = n
        om2 = om2 + ((2 * np.pi * kt / n) ** 2).reshape(sh)
        if n % 2 == 0:
            nyq = nyq | (k == n // 2).reshape(sh)
    keep = (om2 <= (frac * np.pi) ** 2) & ~nyq
    W = W * keep
    out = np.real(np.fft.ifftn(W, axes=(-3, -2, -1)))
    out /= max(np.sqrt(np.mean(out ** 2)), 1e-30)
    return out.astype(dtype)


def s_theta_for(n_orients):
    """Angular window width scaled with the orientation spacing: 0.7 at 42
    orientations (the setting of Fig. 6), scaled by sqrt(42/N_o)."""
    return 0.7 * (42.0 / n_orients) ** 0.5


# The five workloads: crossing-tube volume recipe, orientation level and order L.
CONFIGS = {
    "A": dict(shape=(32, 32, 32), tubes=3, sigma=1.5, noise=0.1, pairs=0, seed=0, level=0, L=8),
    "B": dict(shape=(128, 128, 128), tubes=12, sigma=(1.0, 3.0), noise=0.2, pairs=5, seed=1, level=1, L=16),
    "C": dict(shape=(256, 256, 256), tubes=40, sigma=(1.0, 4.0), noise=0.3, pairs=0, seed=2, level=2, L=24),
}


# Request shapes (z, y, x) of the serving workload.
SERVING_SHAPES = [(64, 64, 64), (96, 80, 64), (128, 128, 128), (160, 128, 128), (256, 256, 256)]


def config_volume(name):
    c = CONFIGS[name]
    return tubes(c["shape"], c["tubes"], c["sigma"], c["noise"], c["pairs"], c["seed"])
