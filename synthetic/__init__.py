"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module generates inputs only: random-ellipsoid phantoms, the (phi, theta)
angle sets of the radial sampling pattern, the unit line directions of the
polar-to-Cartesian map (Section 2.1.1, eq 2.1), and the workload recipes.  It
contains none of the transform's arithmetic: no Fourier sums, no kernels, no
deapodization, no interpolation.  The CPU oracle and the HIP library both take
these arrays as their inputs.

Phantom recipe (the paper's Shepp-Logan slices and clinical images are not
available; random ellipsoids stand in for them):
  * voxel centre u_n = (n - N/2) * (2/N) in [-1, 1) per axis;
  * an ellipsoid is density * 1{ || D^-1 R^T (u - c) || <= 1 };
  * centre uniform in the ball of radius 0.6, semi-axes U[0.05, 0.3] each,
    rotation Haar-uniform, density U[0.1, 1]; overlapping ellipsoids add;
  * optional i.i.d. Gaussian noise per voxel.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------
# Random ellipsoid phantoms
# ----------------------------------------------------------------------------
@dataclass
class Ellipsoid:
    center: np.ndarray      # (3,) in normalised coordinates [-1, 1)
    axes: np.ndarray        # (3,) semi-axes
    rot: np.ndarray         # (3, 3) rotation, columns are the ellipsoid axes
    density: float


def haar_rotation(rng: np.random.Generator) -> np.ndarray:
    """Haar-uniform rotation from the QR factorisation of a Gaussian matrix."""
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def random_ellipsoids(rng: np.random.Generator, count: int) -> list[Ellipsoid]:
    out = []
    for _ in range(count):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        c = 0.6 * rng.uniform() ** (1.0 / 3.0) * v
        axes = rng.uniform(0.05, 0.3, size=3)
        rot = haar_rotation(rng)
        dens = float(rng.uniform(0.1, 1.0))
        out.append(Ellipsoid(c, axes, rot, dens))
    return out


def voxel_coords(N: int) -> np.ndarray:
    return (np.arange(N, dtype=np.float64) - N // 2) * (2.0 / N)


def voxelize(ells: list[Ellipsoid], N: int) -> np.ndarray:
    """Point-sampled indicator ellipsoids on the N^3 voxel grid (float64).

    Each ellipsoid is evaluated only inside the box that holds its
    circumscribed ball (radius = largest semi-axis); outside it the indicator
    is zero, so the result equals evaluating it everywhere."""
    u = voxel_coords(N)
    vol = np.zeros((N, N, N), dtype=np.float64)
    for e in ells:
        r = float(np.max(e.axes))
        sl = []
        for d in range(3):
            lo = int(np.floor((e.center[d] - r) * N / 2 + N // 2)) - 1
            hi = int(np.ceil((e.center[d] + r) * N / 2 + N // 2)) + 2
            sl.append(slice(max(lo, 0), min(hi, N)))
        if any(s.start >= s.stop for s in sl):
            continue
        U0, U1, U2 = np.meshgrid(u[sl[0]], u[sl[1]], u[sl[2]], indexing="ij")
        d = np.stack([U0, U1, U2], axis=-1) - e.center
        loc = d @ e.rot  # coordinates along the ellipsoid axes
        q = np.sum((loc / e.axes) ** 2, axis=-1)
        vol[sl[0], sl[1], sl[2]] += e.density * (q <= 1.0)
    return vol


def ellipsoid_phantom(N: int, count: int, seed: int, noise_sigma: float = 0.0,
                      perturb: bool = False) -> np.ndarray:
    """Sum of `count` random ellipsoids, seeded; float64 (N, N, N)."""
    rng = np.random.default_rng(seed)
    ells = random_ellipsoids(rng, count)
    if perturb:
        prng = np.random.default_rng(seed + 7919)
        for e in ells:
            e.density *= float(prng.uniform(0.9, 1.1))
            e.center = e.center + prng.normal(0.0, 0.01, size=3)
    vol = voxelize(ells, N)
    if noise_sigma > 0.0:
        vol = vol + rng.normal(0.0, noise_sigma, size=vol.shape)
    return vol


def gaussian_blob(N: int, center_vox: np.ndarray, cov_vox: np.ndarray,
                  amp: float = 1.0) -> np.ndarray:
    """Sampled Gaussian amp*exp(-0.5 (m-c)^T C^-1 (m-c)) with m = n - N/2 (voxels)."""
    m = np.arange(N, dtype=np.float64) - N // 2
    M0, M1, M2 = np.meshgrid(m, m, m, indexing="ij")
    d = np.stack([M0, M1, M2], axis=-1) - center_vox
    ci = np.linalg.inv(cov_vox)
    q = np.einsum("...i,ij,...j->...", d, ci, d)
    return amp * np.exp(-0.5 * q)


# ----------------------------------------------------------------------------
# Radial sampling pattern
# ----------------------------------------------------------------------------
def azimuths(n_phi: int) -> np.ndarray:
    """phi_a = 2 pi a / N_phi, a = 0..N_phi-1."""
    return np.arange(n_phi, dtype=np.float64) * (TWO_PI / n_phi)


def polar_angles(n_theta: int, margin: float = 0.2) -> np.ndarray:
    """theta_b = margin + b (pi - 2 margin)/(N_theta - 1), inclusive ends."""
    if n_theta == 1:
        return np.array([math.pi / 2])
    return margin + np.arange(n_theta, dtype=np.float64) * ((math.pi - 2 * margin) / (n_theta - 1))


def line_directions(phi: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Unit directions of the radial lines, eq 2.1 with rho = 1.

    Lines are ordered [a][b] (azimuth outer, polar inner); returns (L, 3) float64
    with components (sin th cos ph, sin th sin ph, cos th) pairing with volume
    axes (0, 1, 2).
    """
    ph = np.repeat(np.asarray(phi, dtype=np.float64), len(theta))
    th = np.tile(np.asarray(theta, dtype=np.float64), len(phi))
    st = np.sin(th)
    return np.stack([st * np.cos(ph), st * np.sin(ph), np.cos(th)], axis=1)


def radial_grid(n_r: int) -> np.ndarray:
    """r_c = (c - N_r/2) * (2 pi / N_r), c = 0..N_r-1: samples of [-pi, pi)."""
    return (np.arange(n_r, dtype=np.float64) - (n_r // 2)) * (TWO_PI / n_r)


def radial_points(dirs: np.ndarray, n_r: int) -> np.ndarray:
    """omega[l*N_r + c] = r_c * nhat_l, (L*N_r, 3) float64, lines contiguous."""
    r = radial_grid(n_r)
    return (r[None, :, None] * dirs[:, None, :]).reshape(-1, 3)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    N: int
    K: int
    J: int
    n_phi: int
    n_theta: int
    n_r: int
    n_ell: int
    seed: int
    noise: float = 0.0
    batch: int = 1
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_lines(self) -> int:
        return self.n_phi * self.n_theta

    @property
    def M(self) -> int:
        return self.n_lines * self.n_r

    def directions(self) -> np.ndarray:
        return line_directions(azimuths(self.n_phi), polar_angles(self.n_theta))

    def volume(self, item: int = 0, perturb: bool = False) -> np.ndarray:
        return ellipsoid_phantom(self.N, self.n_ell, self.seed + item, self.noise,
                                 perturb=perturb)


WORKLOADS = {
    # plain forward NUFFT in float64 at a small size; checked against the NUDFT
    "c1": Workload("c1", N=32, K=64, J=4, n_phi=32, n_theta=16, n_r=64, n_ell=8, seed=1000),
    # forward + adjoint, complex64, derivative-Radon radial stage
    "c2": Workload("c2", N=128, K=256, J=6, n_phi=180, n_theta=90, n_r=256, n_ell=20, seed=2000),
    # precision comparison at 256^3 (the benchmark workload)
    "c3": Workload("c3", N=256, K=512, J=6, n_phi=360, n_theta=180, n_r=512, n_ell=40,
                   seed=3000, noise=0.01),
    # differentiation, batch 4 at 128^3
    "c4": Workload("c4", N=128, K=256, J=6, n_phi=180, n_theta=90, n_r=256, n_ell=20,
                   seed=4000, batch=4),
}


def batch_workload(count: int = 64, seed: int = 5000, sizes=(48, 64, 96, 128, 160)):
    """Uneven batch: volume b gets N from `sizes`, 10-30 ellipsoids, even
    N_phi in [60, 240], N_theta = N_phi/2, N_r = 2N, K = 2N, J = 6."""
    items = []
    for b in range(count):
        rng = np.random.default_rng(seed + b)
        N = int(rng.choice(sizes))
        n_ell = int(rng.integers(10, 31))
        n_phi = int(rng.integers(30, 121)) * 2
        items.append(Workload(f"c5[{b}]", N=N, K=2 * N, J=6, n_phi=n_phi,
                              n_theta=n_phi // 2, n_r=2 * N, n_ell=n_ell, seed=seed + b))
    return items


def complex_noise(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
