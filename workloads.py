"""Seeded synthetic suspensions: the inputs that both the HIP path and the
oracle consume.

This module only draws random particle configurations and states particle
properties (shape, single-body drag mobility, external force and torque). It
performs none of the collision-resolution arithmetic: no distances, no contact
Jacobian, no mobility products, no solve. Every random number comes from a
NumPy PCG64 stream seeded with ``SEED_BASE + workload number`` (batched
instance ``k`` adds ``k``), so a given workload is the same array on every
machine.

Workload shapes follow the paper's test problems: sphere suspensions at a given
volume fraction (section 6.3 uses N = 1000 spheres), and spherocylinder
suspensions at a density that gives a chosen mean number of close pairs per rod
(sections 1 and 8 describe the method for any convex shape, spherocylinders in
particular). Positions are uniform in a periodic cube with overlaps allowed, so
the solve starts from a strongly violated configuration.

Mobility convention. The paper treats the mobility as any SPD operator
(section 2). Here each particle carries its own dry (no hydrodynamic coupling)
6x6 block ``diag(A, B)`` with ``A = a_par p p^T + a_perp (I - p p^T)`` and
``B = b_par p p^T + b_perp (I - p p^T)``, stored as ``mob[k] = (a_par, a_perp,
b_par, b_perp)``. Spheres use the single-sphere Stokes values quoted in
section 6.1.1 (1/(6 pi mu a) and 1/(8 pi mu a^3)); rods use leading-order
slender-body drag with log(L/D) and no end corrections (a chosen convention:
the paper defers rod mobility to other work).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 19090662300

# spherocylinder geometry of the rod workloads: segment length 1, diameter 0.05
ROD_LENGTH = 1.0
ROD_DIAMETER = 0.05
ROD_DELTA = 0.015          # 30% of the sum of the radii of two rods
SPHERE_RADIUS = 0.5
SPHERE_DELTA = 0.1         # close-pair threshold of the 1000-sphere workload
MU = 1.0


@dataclasses.dataclass
class Suspension:
    """One periodic suspension; every array is float64, particle-major."""
    name: str
    pos: np.ndarray        # [N,3] centres, inside [lo, lo+L)
    axis: np.ndarray       # [N,3] unit axis (arbitrary unit vector for spheres)
    radius: np.ndarray     # [N]
    half_len: np.ndarray   # [N] half segment length, 0 for spheres
    mob: np.ndarray        # [N,4] a_par, a_perp, b_par, b_perp
    f_ext: np.ndarray      # [N,6] external force and torque
    box: np.ndarray        # [3] periodic box side
    delta: float           # close-pair threshold on the minimum separation
    dt: float              # time step
    tol: float = 1e-6      # absolute tolerance on ||min(gamma, g)||_2
    lo: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    periodic: int = 1
    walls: int = 0         # non-periodic boxes: bit 2a (2a+1) = wall at the lower
                           # (upper) face of axis a
    hydro_radius: np.ndarray | None = None   # [N] radii of a hydrodynamic mobility
                                              # (None: the collision radius)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def interaction_range(self) -> float:
        """Largest centre distance at which a pair can still be close."""
        return 2.0 * float(np.max(self.radius + self.half_len)) + self.delta

    def subset(self, idx) -> "Suspension":
        idx = np.asarray(idx)
        return dataclasses.replace(
            self, pos=self.pos[idx].copy(), axis=self.axis[idx].copy(),
            radius=self.radius[idx].copy(), half_len=self.half_len[idx].copy(),
            mob=self.mob[idx].copy(), f_ext=self.f_ext[idx].copy(),
            hydro_radius=None if self.hydro_radius is None else self.hydro_radius[idx].copy())


# ---------------------------------------------------------------- properties

def sphere_mobility(radius, mu=MU):
    """Single-sphere Stokes translational and rotational mobilities."""
    radius = np.asarray(radius, dtype=np.float64)
    mt = 1.0 / (6.0 * math.pi * mu * radius)
    mr = 1.0 / (8.0 * math.pi * mu * radius ** 3)
    return np.stack([mt, mt, mr, mr], axis=-1)


def rod_mobility(length=ROD_LENGTH, diameter=ROD_DIAMETER, mu=MU):
    """Leading-order slender-body mobilities (a_par, a_perp, b_par, b_perp)."""
    lg = math.log(length / diameter)
    zeta_par = 2.0 * math.pi * mu * length / lg
    zeta_perp = 2.0 * zeta_par
    zeta_rot_perp = math.pi * mu * length ** 3 / (3.0 * lg)
    zeta_rot_par = math.pi * mu * diameter ** 2 * length
    return np.array([1.0 / zeta_par, 1.0 / zeta_perp,
                     1.0 / zeta_rot_par, 1.0 / zeta_rot_perp])


def sphere_volume(radius):
    return 4.0 / 3.0 * math.pi * radius ** 3


def spherocylinder_volume(length=ROD_LENGTH, diameter=ROD_DIAMETER):
    r = 0.5 * diameter
    return math.pi * r * r * length + 4.0 / 3.0 * math.pi * r ** 3


def rod_density_for_pairs(pairs_per_rod, length=ROD_LENGTH,
                          diameter=ROD_DIAMETER, delta=ROD_DELTA):
    """Number density at which a rod has ``pairs_per_rod`` close neighbours on
    average, from the isotropic excluded volume of spherocylinders of
    effective diameter D + delta (Onsager)."""
    de = diameter + delta
    vex = (4.0 / 3.0 * math.pi * de ** 3 + 2.0 * math.pi * de ** 2 * length
           + 0.5 * math.pi * de * length ** 2)
    return pairs_per_rod / vex


# ---------------------------------------------------------------- sampling

def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _isotropic_axes(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _watson_axes(rng, n, kappa):
    """Axes with density proportional to exp(kappa (e_z . p)^2): cos(theta)
    by rejection from uniform on [-1, 1] with acceptance exp(kappa (t^2 - 1)),
    azimuth uniform."""
    out = np.empty(n)
    filled = 0
    while filled < n:
        m = max(1024, 2 * (n - filled))
        t = rng.uniform(-1.0, 1.0, m)
        u = rng.uniform(0.0, 1.0, m)
        keep = t[u < np.exp(kappa * (t * t - 1.0))]
        take = min(keep.size, n - filled)
        out[filled:filled + take] = keep[:take]
        filled += take
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    st = np.sqrt(np.maximum(0.0, 1.0 - out * out))
    return np.stack([st * np.cos(ph), st * np.sin(ph), out], axis=1)


def spheres(n, phi, seed, radius=SPHERE_RADIUS, delta=SPHERE_DELTA, dt=1e-3,
            tol=1e-6, name=None):
    """``n`` spheres of one radius, uniform centres in a periodic cube whose
    side gives volume fraction ``phi``; Gaussian force/torque, sigma 1."""
    rng = _rng(seed)
    side = (n * sphere_volume(radius) / phi) ** (1.0 / 3.0)
    box = np.full(3, side)
    pos = rng.uniform(0.0, side, (n, 3))
    axis = _isotropic_axes(rng, n)
    f_ext = rng.standard_normal((n, 6))
    rad = np.full(n, float(radius))
    return Suspension(name or f"spheres_n{n}_phi{phi:g}", pos, axis, rad,
                      np.zeros(n), sphere_mobility(rad), f_ext, box, delta,
                      dt, tol)


def sphere_cluster(n, seed, phi=0.2, a=1.0, collision_scale=1.05, force=1.0, mu=MU,
                   tol=1e-6, squeeze=0.0, name=None):
    """The dense sedimenting cluster of the paper's section 6.3: ``n`` spheres
    of hydrodynamic radius ``a`` in a ball whose hydrodynamic volume
    fraction is ``phi``, placed by random sequential addition without
    overlap of their collision spheres (radius ``collision_scale * a``);
    the same force ``-force e_z`` on each, no torque; unbounded fluid (a
    non-periodic box that only sizes the search grid); delta = 30% of the
    sum of two collision radii and dt = 0.05 mu a^2 / force. ``squeeze`` > 0
    adds an inward radial force of that many times ``force`` (a compressed
    cluster, with many active contacts)."""
    rng = _rng(seed)
    rc = collision_scale * a
    R = a * (n / phi) ** (1.0 / 3.0)
    cell = 2.0 * rc
    grid = {}
    pos = np.empty((n, 3))
    k = 0
    while k < n:
        x = rng.uniform(-R, R, 3)
        if x @ x > (R - rc) ** 2:
            continue
        key = tuple(np.floor(x / cell).astype(int))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for m in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        d = pos[m] - x
                        if d @ d < cell * cell:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        pos[k] = x
        grid.setdefault(key, []).append(k)
        k += 1
    f_ext = np.zeros((n, 6))
    f_ext[:, 2] = -force
    if squeeze:
        rn = np.linalg.norm(pos, axis=1, keepdims=True)
        f_ext[:, :3] -= squeeze * force * pos / np.maximum(rn, 1e-300)
    hyd = np.full(n, float(a))
    delta = 0.3 * 2.0 * rc
    margin = 2.0 * rc + delta
    lo = np.full(3, -R - margin)
    return Suspension(name or f"cluster_n{n}", pos, _isotropic_axes(rng, n), np.full(n, rc),
                      np.zeros(n), sphere_mobility(hyd, mu), f_ext,
                      np.full(3, 2.0 * (R + margin)), delta, 0.05 * mu * a * a / force, tol,
                      lo=lo, periodic=0, hydro_radius=hyd)


def rods(n, seed, density=None, phi=None, pairs_per_rod=6.0, kappa=None,
         length=ROD_LENGTH, diameter=ROD_DIAMETER, delta=ROD_DELTA, dt=1e-4,
         tol=1e-6, min_side=None, name=None):
    """``n`` spherocylinders (segment ``length``, ``diameter``) with uniform
    centres in a periodic cube and isotropic (or Watson ``kappa``) axes.
    Density: ``density`` if given, else from volume fraction ``phi``, else
    from ``pairs_per_rod``. ``min_side`` lowers the density if needed so that
    the box is at least that wide."""
    rng = _rng(seed)
    if density is None:
        if phi is not None:
            density = phi / spherocylinder_volume(length, diameter)
        else:
            density = rod_density_for_pairs(pairs_per_rod, length, diameter,
                                            delta)
    side = (n / density) ** (1.0 / 3.0)
    if min_side is not None and side < min_side:
        side = float(min_side)
    box = np.full(3, side)
    pos = rng.uniform(0.0, side, (n, 3))
    axis = _isotropic_axes(rng, n) if kappa is None else _watson_axes(rng, n, kappa)
    f_ext = rng.standard_normal((n, 6))
    mob = np.tile(rod_mobility(length, diameter), (n, 1))
    return Suspension(name or f"rods_n{n}", pos, axis,
                      np.full(n, 0.5 * diameter), np.full(n, 0.5 * length),
                      mob, f_ext, box, delta, dt, tol)


def rods_and_spheres(n_rods, n_spheres, seed, kappa=5.0,
                     sphere_radius=0.05, delta=ROD_DELTA, dt=1e-4, tol=1e-6,
                     name=None):
    """Rods at the 6-pairs-per-rod density (Watson-biased axes) plus small
    spheres, all in one periodic cube sized by the rod density."""
    rng = _rng(seed)
    density = rod_density_for_pairs(6.0)
    side = (n_rods / density) ** (1.0 / 3.0)
    n = n_rods + n_spheres
    pos = rng.uniform(0.0, side, (n, 3))
    axis = np.concatenate([_watson_axes(rng, n_rods, kappa),
                           _isotropic_axes(rng, n_spheres)])
    f_ext = rng.standard_normal((n, 6))
    radius = np.concatenate([np.full(n_rods, 0.5 * ROD_DIAMETER),
                             np.full(n_spheres, float(sphere_radius))])
    half_len = np.concatenate([np.full(n_rods, 0.5 * ROD_LENGTH),
                               np.zeros(n_spheres)])
    mob = np.concatenate([np.tile(rod_mobility(), (n_rods, 1)),
                          sphere_mobility(np.full(n_spheres, sphere_radius))])
    return Suspension(name or f"rods{n_rods}_spheres{n_spheres}", pos, axis,
                      radius, half_len, mob, f_ext, np.full(3, side), delta,
                      dt, tol)


# ---------------------------------------------------------------- workloads

WORKLOADS = {
    1: "1000 spheres R=0.5, volume fraction 0.3, delta 0.1, dt 1e-3",
    2: "100000 spherocylinders L=1 D=0.05, ~6 close pairs per rod, delta 0.015, dt 1e-4",
    3: "1000000 Watson(kappa=5) spherocylinders + 100000 spheres D=0.1, dt 1e-4",
    4: "workload 2 with loss 1/2 ||D gamma||^2 for the adjoint",
    5: "512 independent sphere/rod suspensions, N log-uniform in [200, 20000]",
}


def workload(k, scale=1.0):
    """Workload ``k`` (1-4). ``scale`` < 1 shrinks the particle count at the
    same density (for quick tests); the seed is unchanged."""
    seed = SEED_BASE + k
    if k == 1:
        return spheres(max(2, int(round(1000 * scale))), 0.3, seed,
                       name="spheres1000")
    if k in (2, 4):
        return rods(max(2, int(round(100000 * scale))), seed,
                    name="rods100k" if k == 2 else "rods100k_adjoint")
    if k == 3:
        return rods_and_spheres(max(1, int(round(1000000 * scale))),
                                max(1, int(round(100000 * scale))), seed,
                                name="rods1M_spheres100k")
    raise ValueError(f"no single-suspension workload {k}")


def batched_instances(count=512, seed=None, n_min=200, n_max=20000,
                      phi_lo=0.1, phi_hi=0.4):
    """Independent suspensions of uneven size: N log-uniform in
    [n_min, n_max], a density parameter phi uniform in [phi_lo, phi_hi],
    sphere or rod with probability 1/2. Spheres take phi as their volume
    fraction. For rods phi sets the contact density instead: 15 phi close
    pairs per rod (6 at phi = 0.4, as the 100k-rod suspension), because
    uniformly placed rods of aspect ratio 20 at a volume fraction above
    about 0.2 have more contacts than 6 N rigid-body degrees of freedom, an
    over-constrained LCP with a singular M. Rod boxes are widened to at
    least twice the interaction range (lowering the density to fit); returns
    the list of suspensions and the indices of the widened instances."""
    base = SEED_BASE + 5 if seed is None else seed
    meta = _rng(base)
    ns = np.rint(np.exp(meta.uniform(math.log(n_min), math.log(n_max), count))).astype(int)
    phis = meta.uniform(phi_lo, phi_hi, count)
    kinds = meta.uniform(0.0, 1.0, count) < 0.5
    out, widened = [], []
    rod_range = 2.0 * (0.5 * ROD_DIAMETER + 0.5 * ROD_LENGTH) + ROD_DELTA
    for k in range(count):
        if kinds[k]:
            s = spheres(int(ns[k]), float(phis[k]), base + 1 + k,
                        name=f"inst{k}_spheres")
        else:
            s = rods(int(ns[k]), base + 1 + k, pairs_per_rod=15.0 * float(phis[k]),
                     min_side=2.0 * rod_range, name=f"inst{k}_rods")
            if abs(s.box[0] - 2.0 * rod_range) < 1e-12:
                widened.append(k)
        out.append(s)
    return out, widened
