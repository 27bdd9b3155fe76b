"""Seeded synthetic inputs: initial fields and the workload definitions.

This module holds no lattice-Boltzmann arithmetic.  It builds the initial
condition of Sec. 4 of Cartalade, Younsi & Plapp (arXiv:1602.07483): diffuse
spherical nuclei phi = tanh((R - d)/(sqrt(2) W0)) in an undercooled melt with
constant U0 and theta0, optionally with seeded uniform noise on U.  The same
arrays feed the GPU library and the FP64 oracle.

Noise: u = SplitMix64(seed, linear node index) mapped to a double in [0, 1),
the published SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014).
"""
from dataclasses import dataclass, field, asdict
from typing import List, Sequence, Tuple

import numpy as np

NOFLUX = 0
SYMMETRY = 1

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(seed: int, index: np.ndarray) -> np.ndarray:
    """SplitMix64 output for state seed + (index+1) * golden gamma."""
    with np.errstate(over="ignore"):
        z = (np.uint64(seed) + (index.astype(np.uint64) + np.uint64(1))
             * np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """n doubles in [0, 1) from the top 53 bits of SplitMix64."""
    z = splitmix64(seed, np.arange(n, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def sphere_field(shape: Tuple[int, int, int], centres: Sequence[Sequence[float]],
                 radius: float, W0: float = 1.0, dx: float = 1.0) -> np.ndarray:
    """phi0 = max over seeds of tanh((R - d)/(sqrt(2) W0)), d the distance to
    the seed centre; centres and R in node-index (lattice) units; shape is
    (nz, ny, nx).  Each seed is evaluated on its bounding box only: beyond
    (R - d) dx / (sqrt(2) W0) < -30 the double tanh is exactly -1."""
    nz, ny, nx = shape
    phi = np.full(shape, -1.0)
    reach = radius + 30.0 * np.sqrt(2.0) * W0 / dx + 1.0
    for c in centres:
        lo = [max(0, int(np.floor(c[a] - reach))) for a in range(3)]
        hi = [min(n, int(np.ceil(c[a] + reach)) + 1) for a, n in enumerate((nx, ny, nz))]
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        z, y, x = np.meshgrid(np.arange(lo[2], hi[2], dtype=np.float64),
                              np.arange(lo[1], hi[1], dtype=np.float64),
                              np.arange(lo[0], hi[0], dtype=np.float64), indexing="ij")
        d = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        box = phi[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        np.maximum(box, np.tanh((radius - d) * dx / (np.sqrt(2.0) * W0)), out=box)
    return phi


@dataclass
class Problem:
    """One domain: grid, walls, model parameters and initial condition."""
    name: str
    nx: int
    ny: int
    nz: int
    lattice: int = 19
    walls: Tuple[int, ...] = (NOFLUX,) * 6          # -x,+x,-y,+y,-z,+z
    dx: float = 1.0
    dt: float = 1.0
    W0: float = 1.0
    tau0: float = 1.0
    lam: float = 3.2
    Mcinf: float = 1.0
    k: float = 0.15
    D: float = 2.0
    kappa: float = 20.0
    aniso: int = 0
    eps: float = 0.05
    delta: float = 0.0
    vel: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # advective velocity of theta
    # initial condition
    centres: List[Tuple[float, float, float]] = field(default_factory=list)
    radius: float = 5.0
    U0: float = -0.55
    theta0: float = -0.55
    noise_amp: float = 0.0
    noise_seed: int = 0
    steps: int = 100
    reduce_every: int = 0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def nodes(self):
        return self.nx * self.ny * self.nz

    def centre(self):
        """Reference point of the tip measurement (first seed)."""
        return tuple(self.centres[0]) if self.centres else (0.0, 0.0, 0.0)

    def model_kwargs(self):
        d = asdict(self)
        keys = ("lattice", "walls", "dx", "dt", "W0", "tau0", "lam", "Mcinf", "k", "D",
                "kappa", "aniso", "eps", "delta", "vel")
        return {kk: d[kk] for kk in keys}

    def initial_fields(self):
        """(phi0, U0, theta0) as float64 arrays of shape (nz, ny, nx)."""
        phi = sphere_field(self.shape, self.centres, self.radius, self.W0, self.dx)
        U = np.full(self.shape, self.U0)
        if self.noise_amp:
            u = uniform01(self.noise_seed, self.nodes).reshape(self.shape)
            U = U + self.noise_amp * (2.0 * u - 1.0)
        th = np.full(self.shape, self.theta0)
        return phi, U, th


# --------------------------------------------------------------------------
# Workloads.  Units W0 = tau0 = 1 with dx = W0 (one node per interface width).
# Parameters the workload statements leave open are fixed here and listed in
# the design notes: Mc_inf = 1, D = 2, lambda = 3.2 (the paper's alloy
# benchmark, Sec. 4.2), kappa = 10 D, theta0 = -Delta.  The time step is the
# paper's 3D ratio dt/tau0 = 0.15 (Sec. 4.1): dt = tau0 makes the explicit
# reaction term unstable wherever a_s < 1 (amplification 1 - 2 dt/(tau0 a_s^2)
# < -1) and D = 2 per unit time step makes the U scheme unstable.
# --------------------------------------------------------------------------
DT = 0.15
CORNER = (-0.5, -0.5, -0.5)
SEED_FACES = (SYMMETRY, NOFLUX, SYMMETRY, NOFLUX, SYMMETRY, NOFLUX)


def workload_small(steps: int = 300, n: int = 32) -> Problem:
    """32^3 D3Q19, sphere R=5 at the corner, symmetry walls on the seed faces,
    no-flux elsewhere, U noise 1e-3 (seed 1)."""
    return Problem("corner-%d" % n, n, n, n, 19, SEED_FACES, dt=DT, eps=0.05,
                   k=0.15, U0=-0.55, theta0=-0.55, centres=[CORNER], radius=5.0,
                   noise_amp=1e-3, noise_seed=1, steps=steps, reduce_every=10)


def workload_octant(n: int = 128, steps: int = 5000) -> Problem:
    """n^3 D3Q19 octant dendrite, R=8 at the corner, walls and noise as the
    small case, kappa/D = 10."""
    return Problem("octant-%d" % n, n, n, n, 19, SEED_FACES, dt=DT, eps=0.05,
                   k=0.15, U0=-0.55, theta0=-0.55, centres=[CORNER], radius=8.0,
                   noise_amp=1e-3, noise_seed=2, steps=steps, reduce_every=100)


def workload_centred(n: int = 256, steps: int = 10000) -> Problem:
    """n^3 D3Q19, centred seed R=10, all walls no-flux, Delta=0.6, no noise."""
    c = (n - 1) / 2.0
    return Problem("centred-%d" % n, n, n, n, 19, (NOFLUX,) * 6, dt=DT, eps=0.05,
                   k=0.15, U0=-0.6, theta0=-0.6, centres=[(c, c, c)], radius=10.0,
                   steps=steps, reduce_every=100)


def workload_centred_octant(n: int = 256, steps: int = 10000) -> Problem:
    """The octant x, y, z >= n/2 of workload_centred(n): an (n/2)^3 domain with
    mirror walls on the three faces through the seed centre (which sits on
    the half link between nodes n/2-1 and n/2) and the original no-flux walls
    on the far faces.  A run of it equals that octant of the full run, and
    its reductions give the full domain's tip position and solid fraction
    (sums scale by 8)."""
    m = n // 2
    return Problem("centred-%d-octant" % n, m, m, m, 19, SEED_FACES, dt=DT, eps=0.05,
                   k=0.15, U0=-0.6, theta0=-0.6, centres=[CORNER], radius=10.0,
                   steps=steps, reduce_every=100)


def workload_interior(lattice: int = 19) -> Problem:
    """136 x 40 x 24 with a seed R = 8 in the middle and a second one at a
    mirror corner, walls of both kinds, U noise 1e-3 (seed 7): with the
    default launches of both step kernels (tiles of 32 x 8, 64 x 4, 32 x 4 or
    64 x 8 nodes) some tiles have no node on an x or y face, so the growing
    interface crosses tiles on the wall-free path that large domains run."""
    walls = (SYMMETRY, NOFLUX, SYMMETRY, NOFLUX, NOFLUX, SYMMETRY)
    return Problem("interior", 136, 40, 24, lattice, walls, dt=DT if lattice == 19 else 0.11, eps=0.05,
                   centres=[(67.5, 19.5, 11.5), (-0.5, -0.5, 23.5)], radius=8.0, U0=-0.55,
                   theta0=-0.55, noise_amp=1e-3, noise_seed=7)


def workload_thermal2d(n: int = 500, steps: int = 37500, dx: float = 0.4) -> Problem:
    """Pure-substance thermal dendrite of Sec. 4.1 (anisotropic case) as a
    one-node-thick D3Q19 slab (mirror walls in z, which reduce D3Q19 to D2Q9):
    quadrant of n^2 nodes, dx/W0 = 0.4, dt/tau0 = 0.008, kappa = 4,
    lambda = 6.3826 (zero kinetic coefficient), eps = 0.05, Delta = 0.55,
    seed radius 10 dx at the mirror corner.  The solute field is decoupled
    (M c_inf = 0); its diffusivity only has to keep its scheme stable.
    37 500 steps reach T = t/tau0 = 300.

    Another dx refines the grid under diffusive scaling, dt = 0.008 (dx/0.4)^2
    (every relaxation time unchanged), with the seed radius kept at 4 W0:
    n nodes then span n dx W0 and T = steps dt."""
    walls = (SYMMETRY, NOFLUX, SYMMETRY, NOFLUX, SYMMETRY, SYMMETRY)
    dt = 0.008 * (dx / 0.4) ** 2
    return Problem("thermal2d-%d" % n if dx == 0.4 else "thermal2d-%d-dx%g" % (n, dx), n, n, 1, 19, walls,
                   dx=dx, dt=dt, W0=1.0, tau0=1.0, lam=6.3826, Mcinf=0.0, k=0.15, D=1.0, kappa=4.0,
                   eps=0.05, centres=[(-0.5, -0.5, 0.0)], radius=4.0 / dx, U0=0.0, theta0=-0.55,
                   steps=steps, reduce_every=500)


ENSEMBLE_DT = {15: 0.11, 19: DT}


def workload_ensemble(count: int = 64, seed: int = 4, steps: int = 2000) -> List[Problem]:
    """Batch of independent cubic domains: edge L_j uniform in {32..96},
    eps_j uniform in [0.02, 0.07], Delta_j uniform in [0.45, 0.65] (draws from
    SplitMix64 with the given seed), k = 0.15, centred seed R = 8, all walls
    no-flux, U noise 1e-3 with seed j.  The first half uses D3Q15, the second
    D3Q19.  Time step: dt/tau0 = 0.15 on D3Q19.  The D3Q15 scheme with the
    coupled U equation stays finite and within |phi| <= 1 + 1e-3 for all 32
    of its domains over 2000 steps only near dt/tau0 = 0.11 (at 0.12 and at
    0.06-0.08 some domains diverge), which its half uses.  Domains with eps > 1/15 have a negative cubic
    stiffness 1 - 15 eps along <100> and are ill-posed (sharp corners)."""
    u = uniform01(seed, 3 * count).reshape(count, 3)
    out = []
    for j in range(count):
        L = 32 + int(u[j, 0] * 65.0)
        eps = float(0.02 + 0.05 * u[j, 1])
        delta = float(0.45 + 0.20 * u[j, 2])
        c = (L - 1) / 2.0
        lat = 15 if j < count // 2 else 19
        out.append(Problem("ens-%02d" % j, L, L, L, lat, (NOFLUX,) * 6,
                           dt=ENSEMBLE_DT[lat], eps=eps, k=0.15, U0=-delta, theta0=-delta,
                           centres=[(c, c, c)], radius=8.0, noise_amp=1e-3, noise_seed=j,
                           steps=steps, reduce_every=0))
    return out


def seed_centres(count: int, lo: float, hi: float, min_sep: float, seed: int):
    """Seed centres uniform in [lo, hi]^3 with pairwise distance >= min_sep,
    by rejection sampling of SplitMix64 draws (three per candidate)."""
    centres = []
    k = 0
    while len(centres) < count:
        u = uniform01(seed, 3 * (k + 1))[3 * k:3 * k + 3]
        k += 1
        c = tuple(float(lo + (hi - lo) * v) for v in u)
        if all(sum((a - b) ** 2 for a, b in zip(c, o)) >= min_sep ** 2 for o in centres):
            centres.append(c)
        if k > 100000:
            raise RuntimeError("cannot place %d seeds" % count)
    return centres


def workload_multiseed(n: int = 512, aniso: int = 0, steps: int = 20000) -> Problem:
    """n^3 D3Q19, 8 nuclei of radius 6 at SplitMix64 positions (seed 5) in
    [n/16, n - 1 - n/16]^3 with pairwise separation >= n/8, all walls no-flux,
    Delta = 0.55, k = 0.15.  aniso 0: cubic a_s with eps = 0.05; aniso 1: the
    K41/K61 function of Sec. 4.3 with eps = 0, delta = -0.02."""
    m = n // 16
    centres = seed_centres(8, float(m), float(n - 1 - m), n / 8.0, 5)
    eps, delta = (0.05, 0.0) if aniso == 0 else (0.0, -0.02)
    return Problem("multiseed-%d-%s" % (n, "cubic" if aniso == 0 else "k41k61"), n, n, n, 19,
                   (NOFLUX,) * 6, dt=DT, aniso=aniso, eps=eps, delta=delta, k=0.15,
                   U0=-0.55, theta0=-0.55, centres=centres, radius=6.0, steps=steps,
                   reduce_every=500)
