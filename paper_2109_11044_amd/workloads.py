"""Seeded synthetic workloads: grids, observation locations and parameter
draws shaped like the paper's experiments (Section 3.3, Table 3, the
Ridgecrest application of Section 4).

This module only draws inputs; it holds none of the method's arithmetic and
is shared by the tests, the benchmark and (through the tests) the oracle.

Location generators (numpy ``default_rng``):
  * uniform   -- iid uniform on [0, 1]^2 (Table 3 uses uniform locations).
  * clustered -- 70 % from 5 equal-weight isotropic Gaussian clusters with
    sd 0.05 and centres uniform on [0.1, 0.9]^2 (draws outside [0, 1]^2 are
    redrawn), 30 % uniform; a stand-in for seismic-station networks, which
    are dense near population centres.
Grids are m x m on the unit square with both edges included (spacing
1 / (m - 1)).
"""

from dataclasses import dataclass, field

import numpy as np

SEED_LOCATIONS = 1
SEED_VALUES = 0
SEED_REALIZATIONS = 2
SEED_EVENTS = 3
SEED_WEIGHTS = 4


def uniform_locations(n, seed=SEED_LOCATIONS):
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(n, 2))


def clustered_locations(n, seed=SEED_LOCATIONS, nclusters=5, sd=0.05,
                        frac_uniform=0.3):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.1, 0.9, size=(nclusters, 2))
    nu = int(round(frac_uniform * n))
    nc = n - nu
    lab = rng.integers(0, nclusters, size=nc)
    pts = centres[lab] + sd * rng.normal(size=(nc, 2))
    bad = np.any((pts < 0) | (pts > 1), axis=1)
    while bad.any():
        pts[bad] = centres[lab[bad]] + sd * rng.normal(size=(int(bad.sum()), 2))
        bad = np.any((pts < 0) | (pts > 1), axis=1)
    out = np.vstack([pts, rng.uniform(0.0, 1.0, size=(nu, 2))])
    return out[rng.permutation(n)]


def locations(kind, n, seed=SEED_LOCATIONS):
    return uniform_locations(n, seed) if kind == "uniform" else \
        clustered_locations(n, seed)


def iid_values(n, variance, seed=SEED_VALUES):
    """Observed values with the model's marginal variance but no spatial
    correlation; throughput does not depend on the values."""
    return np.sqrt(variance) * np.random.default_rng(seed).normal(size=n)


@dataclass
class Workload:
    """One conditional-simulation problem on an m x m unit-square grid."""
    name: str
    m: int
    nu: float
    sigma2: float
    range: float
    n: int
    locs: str
    k: int
    tau2: float
    nreal: int
    torus: int = 0                  # 0: choose by the ladder
    batch: int = 0                  # realizations per simulate/condition call
    aniso_ratio: float = 1.0
    aniso_angle: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def dx(self):
        return 1.0 / (self.m - 1)

    def obs_xy(self):
        return locations(self.locs, self.n, self.extra.get("loc_seed", SEED_LOCATIONS))


# Small exact case: exponential, 64^2 grid, 200 uniform points, 4x4 windows.
C1 = Workload("c1_exp64_n200_k16", m=64, nu=0.5, sigma2=1.0, range=0.1,
              n=200, locs="uniform", k=16, tau2=0.05, nreal=10, torus=128)
# Matern nu = 1 on 256^2 with 1000 uniform points, 6x6 windows.
C2 = Workload("c2_matern1_256_n1000_k36", m=256, nu=1.0, sigma2=1.0,
              range=0.15, n=1000, locs="uniform", k=36, tau2=0.1, nreal=100)
# Differentiation-sized problem (used here as a parity case).
C4 = Workload("c4_matern1_512_n2000cl", m=512, nu=1.0, sigma2=1.0, range=0.1,
              n=2000, locs="clustered", k=36, tau2=0.05, nreal=200)
# ShakeMap scale.
C5 = Workload("c5_exp2048_n20000cl_k36", m=2048, nu=0.5, sigma2=1.0,
              range=0.02, n=20000, locs="clustered", k=36, tau2=0.02,
              nreal=1000, batch=64)
# Headline throughput workload: 1024^2 grid, 5000 clustered stations.
DM = Workload("exp1024_n5000cl_k36_R1000", m=1024, nu=0.5, sigma2=1.0,
              range=0.02, n=5000, locs="clustered", k=36, tau2=0.02,
              nreal=1000, batch=1000)

# Nearest-neighbour Kriging at the same grid: fine grid, sparse stations
# (the setting Section 2.2 suits), 2 x 2 neighbourhoods.
NN = Workload("nn_exp1024_n500cl_k4_R1000", m=1024, nu=0.5, sigma2=1.0,
              range=0.02, n=500, locs="clustered", k=4, tau2=0.02,
              nreal=1000, batch=1000)


def event_table(nevents=64, seed=SEED_EVENTS):
    """Uneven batched events: grids from {128, 256, 512}^2, Matern
    nu in {1/2, 3/2}, range U[0.05, 0.3] along a random angle, anisotropy
    ratio U[1, 3], nugget U[0.02, 0.1], 100-3000 clustered points, 6x6
    windows, 200 realizations each."""
    rng = np.random.default_rng(seed)
    out = []
    for e in range(nevents):
        m = int(rng.choice([128, 256, 512]))
        out.append(Workload(
            f"event{e}", m=m, nu=float(rng.choice([0.5, 1.5])), sigma2=1.0,
            range=float(rng.uniform(0.05, 0.3)),
            n=int(rng.integers(100, 3001)), locs="clustered", k=36,
            tau2=float(rng.uniform(0.02, 0.1)), nreal=200,
            aniso_ratio=float(rng.uniform(1.0, 3.0)),
            aniso_angle=float(rng.uniform(0.0, np.pi)),
            extra=dict(loc_seed=1000 + e)))
    return out


def event_inputs(table, values_seed=2000):
    """Per-event inputs of a batch built from ``event_table``: station
    coordinates and iid observed values (seed values_seed + e), as plain
    dicts of parameters and arrays."""
    out = []
    for e, wl in enumerate(table):
        out.append(dict(nu=wl.nu, sigma2=wl.sigma2, range=wl.range,
                        aniso_ratio=wl.aniso_ratio, aniso_angle=wl.aniso_angle,
                        m=wl.m, obs_xy=wl.obs_xy(),
                        z=iid_values(wl.n, wl.sigma2 + wl.tau2, seed=values_seed + e),
                        nugget=wl.tau2, k=wl.k, nreal=wl.nreal, event_id=e))
    return out


# Accuracy study of Section 3.3: [0, 60]^2 domain with a 61 x 61 grid (unit
# spacing), 35 observations uniform on the domain, sigma^2 = 1, nuggets
# tau = 0.1, 0.2, 0.3, smoothness nu = 1/2 and 3/2, and ranges at which the
# correlation falls to 5 % at 20, 45 and 70 units: 18 cases, each over many
# random configurations, with local-Kriging windows n_p = 1..4.
STUDY_GRID = (61, 61, 0.0, 0.0, 1.0, 1.0)
STUDY_NOBS = 35
STUDY_TAUS = (0.1, 0.2, 0.3)
STUDY_NUS = (0.5, 1.5)
STUDY_DISTANCES = (20.0, 45.0, 70.0)
STUDY_NP = (1, 2, 3, 4)


def study_grid(pad=0):
    """The study grid, optionally widened by ``pad`` grid units on every side
    (Section 2.1: the grid is extended by at least n_p units so that every
    observation's window lies inside it); the original 61 x 61 nodes are
    rows and columns pad .. pad + 60 of the widened grid."""
    m1, m2, x0, y0, dx, dy = STUDY_GRID
    return (m1 + 2 * pad, m2 + 2 * pad, x0 - pad * dx, y0 - pad * dy, dx, dy)


def _root_five_percent_matern32():
    """t > 0 with (1 + t) exp(-t) = 0.05 (bisection; the left side falls
    monotonically from 1)."""
    lo, hi = 1.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (1.0 + mid) * np.exp(-mid) > 0.05:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def study_range(nu, distance):
    """Range theta at which the Matern correlation (argument sqrt(2 nu) d /
    theta) is 5 % at the given distance: d / ln 20 for nu = 1/2, sqrt(3) d / t
    with (1 + t) e^{-t} = 0.05 for nu = 3/2."""
    if nu == 0.5:
        return distance / np.log(20.0)
    if nu == 1.5:
        return np.sqrt(3.0) * distance / _root_five_percent_matern32()
    raise ValueError("the study uses nu = 1/2 and 3/2")


def study_cases():
    """The 18 cases (nu, distance, theta, tau) in the order nu, distance, tau."""
    return [dict(nu=nu, distance=d, theta=study_range(nu, d), tau=tau)
            for nu in STUDY_NUS for d in STUDY_DISTANCES for tau in STUDY_TAUS]


def study_locations(config, n=STUDY_NOBS):
    """Configuration ``config``: n points uniform on [0, 60]^2 (seed 1000 + config)."""
    return np.random.default_rng(1000 + config).uniform(0.0, 60.0, size=(n, 2))
