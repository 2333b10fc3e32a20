"""The five synthetic workloads of the IETI-DP hot path, plus small helpers.

The paper's own experiments use a 27-patch cube with a manufactured solution
and METIS partitions (Section 4); the partitions and data are not published,
so these seeded workloads of the same kind (multi-patch cubes and a
motor-like ring, uneven multi-patch subdomains, piecewise-constant
reluctivity) stand in for them.

Names:

* ``cube8``       2x2x2 patches, one subdomain per patch, p=2, 4 elements per
                  patch and direction, nu=1, manufactured polynomial A in the
                  spline space (J = curl curl A).
* ``cube64``      4x4x4 patches, p=3, 8 elements, 16 uneven subdomains (1-8
                  patches) from the seeded greedy partitioner, nu in {1, 1e-3}
                  with P(1e-3)=0.3, J = curl of a random trigonometric field.
* ``cube256``     8x8x4 patches, p=2, 6 elements, 64 subdomains (1-8 patches),
                  nu log-uniform in [1e-3, 1], random trigonometric J.
* ``ring576``     NURBS annulus, 48 azimuthal x 3 radial x 4 axial patches,
                  p=2, 5 elements, 48 azimuthal sectors as subdomains; iron
                  (nu=1e-3), air gap and coil (nu=1), azimuthal coil current.
* ``stream256``   256 independent small cubes (see :func:`stream_problem`).
"""
from __future__ import annotations

import numpy as np

from . import sources
from .partition import greedy_partition
from .problem import GEOM_ANNULUS, GEOM_BOX, Problem

MASTER_SEEDS = {"cube8": 1001, "cube64": 1002, "cube256": 1003, "ring576": 1004, "stream256": 1005}


def config_names():
    return list(MASTER_SEEDS)


def box_problem(P, degree, n_el, patch_to_sub, nu, source, name="box", exact_A=None, exact_B=None,
                extent=(0.0, 1.0, 0.0, 1.0, 0.0, 1.0), seed=0, meta=None):
    return Problem(
        name=name,
        geom_kind=GEOM_BOX,
        patches=tuple(P),
        periodic=(0, 0, 0),
        geom_params=np.array(extent, dtype=np.float64),
        degree=degree,
        n_el=n_el,
        patch_to_sub=np.asarray(patch_to_sub, dtype=np.int32),
        nu=np.asarray(nu, dtype=np.float64),
        source=source,
        exact_A=exact_A,
        exact_B=exact_B,
        seed=seed,
        meta=meta or {},
    )


def cube8(degree=2, n_el=4):
    P = (2, 2, 2)
    part = np.arange(8, dtype=np.int32)
    return box_problem(P, degree, n_el, part, np.ones(8), sources.poly_J, name="cube8",
                       exact_A=sources.poly_A, exact_B=sources.poly_B, seed=MASTER_SEEDS["cube8"])


def cube64(degree=3, n_el=8):
    seed = MASTER_SEEDS["cube64"]
    rng = np.random.default_rng(seed)
    P = (4, 4, 4)
    part, attempts = greedy_partition(P, 16, seed=int(rng.integers(2**31)))
    nu = np.where(rng.random(64) < 0.3, 1e-3, 1.0)
    src = sources.TrigCurlSource(int(rng.integers(2**31)))
    return box_problem(P, degree, n_el, part, nu, src, name="cube64", seed=seed,
                       meta={"partition_attempts": attempts})


def cube256(degree=2, n_el=6):
    seed = MASTER_SEEDS["cube256"]
    rng = np.random.default_rng(seed)
    P = (8, 8, 4)
    part, attempts = greedy_partition(P, 64, seed=int(rng.integers(2**31)))
    nu = 10.0 ** rng.uniform(-3.0, 0.0, size=256)
    src = sources.TrigCurlSource(int(rng.integers(2**31)))
    return box_problem(P, degree, n_el, part, nu, src, name="cube256", seed=seed,
                       meta={"partition_attempts": attempts})


RING_RADII = (1.00, 1.25, 1.50, 1.75)


RING_TRAIN = 512
RING_HELD_OUT = 64


def ring_sample_seed(i):
    """Seed of ring sample i: i < 512 training draws, 512 <= i < 576 held out."""
    return MASTER_SEEDS["ring576"] * 1000 + int(i)


def ring_coefficients(sample=None, n_theta=48):
    """Per-patch reluctivity and per-axial-ring coil current of the annulus:
    iron (1e-3) in the inner radial layer, air gap and coil (1) outside;
    ``sample`` = None gives the nominal values, an integer seed a draw with
    both multiplied by U(0.7, 1.3) (reluctivity per patch, current per ring)."""
    P = (n_theta, 3, 4)
    n = int(np.prod(P))
    radial = (np.arange(n) // P[0]) % P[1]
    nu = np.where(radial == 0, 1e-3, 1.0)
    ring_current = np.ones(P[2])
    if sample is not None:
        rng = np.random.default_rng(sample)
        nu = nu * rng.uniform(0.7, 1.3, size=n)
        ring_current = rng.uniform(0.7, 1.3, size=P[2])
    return nu, ring_current


def ring_load_scale(ring_current, n_theta=48):
    """Per-patch load factor of a coil-current draw: the current of the
    patch's axial ring (the source is zero outside the coil layer)."""
    P = (n_theta, 3, 4)
    axial = np.arange(int(np.prod(P))) // (P[0] * P[1])
    return np.asarray(ring_current, dtype=np.float64)[axial]


def ring576(degree=2, n_el=5, sample=None, n_theta=48):
    """Motor-like annulus.  ``sample`` selects a seeded perturbation draw:
    None = nominal, else the integer seed of a +-30% draw of the per-patch
    reluctivity and the per-axial-ring coil current."""
    P = (n_theta, 3, 4)
    n = int(np.prod(P))
    theta = np.arange(n) % P[0]
    nu, ring_current = ring_coefficients(sample, n_theta)
    z_edges = np.linspace(0.0, 1.0, P[2] + 1)
    src = sources.CoilSource(RING_RADII[2], RING_RADII[3], z_edges, ring_current)
    part = theta.astype(np.int32)
    return Problem(
        name="ring576",
        geom_kind=GEOM_ANNULUS,
        patches=P,
        periodic=(1, 0, 0),
        geom_params=np.array([0.0, 1.0, *RING_RADII], dtype=np.float64),
        degree=degree,
        n_el=n_el,
        patch_to_sub=part,
        nu=nu,
        source=src,
        seed=MASTER_SEEDS["ring576"] if sample is None else int(sample),
        meta={"ring_current": ring_current.tolist(), "nu_features": nu.tolist()},
    )


def stream_problem(i):
    """Problem i of the 256-problem stream: 2^a x 2^b x 2^c patches with
    a,b,c in {1,2,3}, p in {2,3}, 4-6 elements, nu in [1e-3, 1]."""
    seed = MASTER_SEEDS["stream256"] * 1000 + int(i)
    rng = np.random.default_rng(seed)
    P = tuple(int(2 ** rng.integers(1, 4)) for _ in range(3))
    degree = int(rng.integers(2, 4))
    n_el = int(rng.integers(4, 7))
    n = int(np.prod(P))
    part, attempts = greedy_partition(P, None, seed=int(rng.integers(2**31)))
    nu = 10.0 ** rng.uniform(-3.0, 0.0, size=n)
    src = sources.TrigCurlSource(int(rng.integers(2**31)))
    return box_problem(P, degree, n_el, part, nu, src, name=f"stream256[{i}]", seed=seed,
                       meta={"partition_attempts": attempts})


def paper_cube(degree=2, n_el=2, n_sub=3, seed=None):
    """The paper's experiment domain (Section 4): (0,3)^3 in 3x3x3 unit
    patches, nu = 1, the closed-form A_ana with its tangential trace as
    Dirichlet data, and an admissible seeded partition into n_sub
    subdomains (greedy region growing in place of METIS)."""
    P = (3, 3, 3)
    seed = MASTER_SEEDS["cube8"] * 1000 + 27 * 100 + int(n_sub) if seed is None else int(seed)
    part, attempts = greedy_partition(P, int(n_sub), seed=seed, smin=1, smax=27)
    prob = box_problem(P, degree, n_el, part, np.ones(27), sources.paper_J, name=f"paper_cube[{n_sub}]",
                       exact_A=sources.paper_A, exact_B=sources.paper_B, extent=(0.0, 3.0, 0.0, 3.0, 0.0, 3.0),
                       seed=seed, meta={"partition_attempts": attempts})
    prob.dirichlet_A = sources.paper_A
    return prob


def make_config(name, **kw):
    if name == "cube8":
        return cube8(**kw)
    if name == "cube64":
        return cube64(**kw)
    if name == "cube256":
        return cube256(**kw)
    if name == "ring576":
        return ring576(**kw)
    if name == "paper_cube":
        return paper_cube(**kw)
    if name == "stream256":
        return [stream_problem(i) for i in range(kw.get("count", 256))]
    raise KeyError(name)


def small_cube(P=(2, 2, 2), part=None, degree=2, n_el=2, nu=None, source="sine", seed=7):
    """Small cubes for tests.  ``part`` defaults to one subdomain per patch."""
    n = int(np.prod(P))
    if part is None:
        part = np.arange(n, dtype=np.int32)
    if nu is None:
        nu = np.ones(n)
    if source == "sine":
        src, A, B = sources.sine_J, sources.sine_A, sources.sine_B
    elif source == "poly":
        src, A, B = sources.poly_J, sources.poly_A, sources.poly_B
    else:
        src, A, B = sources.TrigCurlSource(seed), None, None
    return box_problem(P, degree, n_el, part, nu, src, name=f"small{P}", exact_A=A, exact_B=B, seed=seed)
