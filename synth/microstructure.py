"""Seeded synthetic microstructures and material tables.

Grid arrays are C-ordered with x fastest: shape (nz, ny, nx) in 3D and
(ny, nx) in 2D, so the flat index of voxel (x, y, z) is x + nx*(y + ny*z).
A voxel (pixel) carries the index of its lowest corner node.

Geometry rules (stated readings, the paper gives no generator):
  * a voxel belongs to an inclusion when its centre lies within periodic
    distance <= r of the inclusion centre;
  * spheres are placed by random sequential addition, non-overlapping in the
    continuum (periodic centre distance >= r_i + r_j), until the voxel
    fraction reaches the target (or the attempt budget runs out; the achieved
    fraction is returned either way);
  * 2D circles may overlap;
  * random numbers come from numpy's PCG64 generator seeded with the given
    integer.
"""
from __future__ import annotations

import math

import numpy as np

# Mandel ordering of the symmetric strain in 3D: 11, 22, 33, 23, 13, 12;
# in 2D: 11, 22, 12.


def isotropic_mandel(E: float, nu: float, dim: int = 3) -> np.ndarray:
    """Isotropic stiffness in Mandel notation (plane strain in 2D).

    lam = E nu / ((1+nu)(1-2nu)), mu = E / (2(1+nu));
    C = lam * (1 on the normal block) + 2 mu * identity.
    """
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    dm = 6 if dim == 3 else 3
    C = np.zeros((dm, dm))
    C[:dim, :dim] = lam
    C += 2.0 * mu * np.eye(dm)
    return C


def isotropic_conductivity(k: float, dim: int = 3) -> np.ndarray:
    return k * np.eye(dim)


def _periodic_delta(a: np.ndarray, c: float, n: int) -> np.ndarray:
    return (a - c + 0.5 * n) % n - 0.5 * n


def _paint_ball(phase, centre, r, value):
    """Set voxels whose centre lies within periodic distance r of centre."""
    dim = phase.ndim
    shape_xyz = phase.shape[::-1]
    idx = []
    for ax in range(dim):
        n = shape_xyz[ax]
        lo = int(math.floor(centre[ax] - r - 1))
        hi = int(math.ceil(centre[ax] + r + 1))
        rng = np.arange(lo, hi + 1)
        if rng.size > n:
            rng = np.arange(n)
        idx.append(np.unique(rng % n))
    # distances along each axis, broadcast to the box
    d2 = 0.0
    grids = np.meshgrid(*idx, indexing="ij")  # x, y(, z)
    for ax in range(dim):
        d = _periodic_delta(grids[ax] + 0.5, centre[ax], shape_xyz[ax])
        d2 = d2 + d * d
    inside = d2 <= r * r
    sel = tuple(g[inside] for g in grids[::-1])  # numpy order z, y, x
    before = np.count_nonzero(phase[sel] == value)
    phase[sel] = value
    return int(inside.sum()) - before


def spheres(n: int, r_range=(6.0, 12.0), vf: float = 0.3, seed: int = 0,
            max_attempts: int = 200000):
    """Random sequential addition of non-overlapping spheres in an n^3 box.

    Returns (phase uint8 (n, n, n), achieved voxel fraction, list of
    (cx, cy, cz, r)).
    """
    rng = np.random.default_rng(seed)
    phase = np.zeros((n, n, n), dtype=np.uint8)
    centres = np.zeros((0, 3))
    radii = np.zeros((0,))
    count = 0
    target = vf * n ** 3
    attempts = 0
    while count < target and attempts < max_attempts:
        attempts += 1
        r = rng.uniform(r_range[0], r_range[1])
        c = rng.uniform(0.0, n, size=3)
        if radii.size:
            d = _periodic_delta(centres, c, n)
            dist = np.sqrt((d * d).sum(axis=1))
            if np.any(dist < radii + r):
                continue
        centres = np.vstack([centres, c])
        radii = np.append(radii, r)
        count += _paint_ball(phase, c, r, 1)
    spheres_list = [tuple(c) + (r,) for c, r in zip(centres, radii)]
    return phase, count / n ** 3, spheres_list


def circles2d(n: int = 32, count: int = 8, r_range=(3.0, 6.0), seed: int = 0):
    """`count` possibly overlapping circles in an n x n periodic pixel grid."""
    rng = np.random.default_rng(seed)
    phase = np.zeros((n, n), dtype=np.uint8)
    for _ in range(count):
        r = rng.uniform(r_range[0], r_range[1])
        c = rng.uniform(0.0, n, size=2)
        _paint_ball(phase, c, r, 1)
    return phase


def laminate(shape_xyz, axis: int, layers) -> np.ndarray:
    """Phase grid of layers normal to `axis` (0 = x, 1 = y, 2 = z).

    `layers` gives the phase of every grid plane along `axis` (length
    shape_xyz[axis]); interfaces therefore lie on voxel faces.
    """
    dim = len(shape_xyz)
    layers = np.asarray(layers, dtype=np.uint8)
    assert layers.size == shape_xyz[axis]
    shp = [1] * dim
    shp[dim - 1 - axis] = shape_xyz[axis]
    return np.broadcast_to(layers.reshape(shp), tuple(shape_xyz[::-1])).copy()


def gaussian_random_field(n: int, ell: float, sigma: float, seed: int = 0,
                          dim: int = 3) -> np.ndarray:
    """Periodic Gaussian random field with squared-exponential correlation.

    White noise is filtered in Fourier space with the square root of the
    spectral density of sigma^2 exp(-r^2 / (2 ell^2)); the result is shifted
    to zero mean and rescaled to sample standard deviation sigma.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n,) * dim)
    k = 2.0 * np.pi * np.fft.fftfreq(n)
    kk = np.meshgrid(*([k] * dim), indexing="ij")
    k2 = sum(g * g for g in kk)
    filt = np.exp(-0.25 * ell * ell * k2)  # sqrt of exp(-ell^2 k^2 / 2)
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    g -= g.mean()
    g *= sigma / g.std()
    return g


def conductivity_grf(n: int = 256, ell: float = 8.0, sigma: float = 1.5,
                     contrast: float = 1e3, seed: int = 0, dim: int = 3):
    """k = exp(g) with g clipped to +-ln(contrast)/2, so max/min <= contrast."""
    g = gaussian_random_field(n, ell, sigma, seed, dim)
    c = 0.5 * math.log(contrast)
    return np.exp(np.clip(g, -c, c))


def _unit_loads(dm: int) -> np.ndarray:
    return np.eye(dm)


def workload(name: str, seed: int = 0, n: int | None = None) -> dict:
    """Named seeded workloads.

    Returned dict keys: dim, n (nx, ny, nz), problem ('scalar'|'elastic'),
    element ('hex8'|'quad4'|'tri2'), phase (uint8 grid) and mat
    (nphase x dm x dm) -- or kfield (float64 grid) for a per-voxel scalar
    conductivity --, loads (nload x dm), eta, and metadata.

    * 'conductivity2d_tri'  : 2D scalar, 32^2 pixels, two P1 triangles per
      pixel, 8 circles r~U[3,6], k=10 inside / 1 outside, load (1, 0).
    * 'elastic3d_spheres'   : 3D elasticity, 128^3 voxels, trilinear hex with
      8 Gauss points, spheres r~U[6,12] (scaled by n/128 for other n, floor
      2), voxel fraction 0.3, E_incl/E_matrix = 100, nu = 0.3, 6 unit loads.
    * 'conduction3d_grf'    : 3D scalar, 256^3, k = exp(GRF), ell = 8,
      sigma = 1.5, contrast <= 1e3, 3 unit gradients.
    """
    if name == "conductivity2d_tri":
        n = n or 32
        phase = circles2d(n, 8, (3.0, 6.0), seed)
        mat = np.stack([isotropic_conductivity(1.0, 2),
                        isotropic_conductivity(10.0, 2)])
        return dict(name=name, dim=2, n=(n, n, 1), problem="scalar",
                    element="tri2", phase=phase, mat=mat,
                    loads=np.array([[1.0, 0.0]]), eta=1e-10)
    if name == "elastic3d_spheres":
        n = n or 128
        s = n / 128.0
        rr = (max(2.0, 6.0 * s), max(2.0, 12.0 * s))
        phase, vf, _ = spheres(n, rr, 0.3, seed)
        mat = np.stack([isotropic_mandel(1.0, 0.3), isotropic_mandel(100.0, 0.3)])
        return dict(name=name, dim=3, n=(n, n, n), problem="elastic",
                    element="hex8", phase=phase, mat=mat, loads=_unit_loads(6),
                    eta=1e-10, vf=vf, r_range=rr)
    if name == "conduction3d_grf":
        n = n or 256
        k = conductivity_grf(n, 8.0 * n / 256.0, 1.5, 1e3, seed)
        return dict(name=name, dim=3, n=(n, n, n), problem="scalar",
                    element="hex8", kfield=k, loads=_unit_loads(3), eta=1e-8)
    raise KeyError(name)


def batch_workload(count: int = 96, seed0: int = 1000,
                   sizes=(32, 48, 64, 96), fixed_n: int | None = None,
                   max_attempts: int = 20000):
    """Batched elasticity microstructures.

    For microstructure i (seed seed0 + i): n ~ U{sizes} (or fixed_n),
    voxel fraction ~ U[0.1, 0.4], stiffness contrast ~ U[10, 1000] (linear
    uniform), nu = 0.3, spheres with radii U[6,12] * n/128 (floor 2).
    Random sequential addition stops after `max_attempts` rejected or
    accepted draws; the achieved fraction is returned as 'vf' (near the
    jamming limit it can stay below the drawn target 'vf_target').
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(fixed_n) if fixed_n else int(rng.choice(np.asarray(sizes)))
        vf = float(rng.uniform(0.1, 0.4))
        contrast = float(rng.uniform(10.0, 1000.0))
        s = n / 128.0
        rr = (max(2.0, 6.0 * s), max(2.0, 12.0 * s))
        phase, got, _ = spheres(n, rr, vf, seed0 + i + 7919, max_attempts)
        mat = np.stack([isotropic_mandel(1.0, 0.3),
                        isotropic_mandel(contrast, 0.3)])
        out.append(dict(name="elastic3d_spheres_batch", dim=3, n=(n, n, n),
                        problem="elastic", element="hex8", phase=phase,
                        mat=mat, loads=_unit_loads(6), eta=1e-6, vf=got,
                        vf_target=vf, contrast=contrast, seed=seed0 + i))
    return out


def batch_workload_parallel(count: int = 96, seed0: int = 1000,
                            sizes=(32, 48, 64, 96), fixed_n: int | None = None,
                            max_attempts: int = 20000, workers: int = 8):
    """The microstructures of batch_workload(count, seed0, ...), generated in
    `workers` fresh processes (each one is drawn from its own seed, so the
    result is identical to the serial call)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    if workers <= 1 or count <= 1:
        return batch_workload(count, seed0, sizes, fixed_n, max_attempts)
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(batch_workload, 1, seed0 + i, sizes, fixed_n, max_attempts)
                for i in range(count)]
        return [f.result()[0] for f in futs]
