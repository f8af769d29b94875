"""Seeded synthetic inputs for the known-object prediction path.

This module produces *inputs only*: a Chebyshev-tabulated perturber
ephemeris (a stand-in for a planetary SPK kernel), Cartesian states of
massless small bodies, and telescope frames (time, observer position and
the inward great-circle normals of each rectangular field of view).
Both the GPU path and the CPU oracle consume what it writes; it performs
none of the prediction arithmetic itself (no Chebyshev evaluation, no
force model, no integration, no universal-variable propagation, no light
time, no membership test).

Where an input needs orbital geometry (placing bodies on orbits, aiming
frames), it uses the textbook elliptic-elements construction: mean
anomaly -> eccentric anomaly by Newton on Kepler's equation -> perifocal
coordinates -> ecliptic rotation.  That builds *inputs*; it is not the
propagation method under test.

Units: au, TDB days, au/day.  Frame: ecliptic J2000, origin at the solar
system barycentre.  Time zero is the J2000 epoch label.

The synthetic configurations restate the workload sizes of the paper's
two survey simulations (Sect. 2) with generated stand-ins: the real
ZTF/WISE metadata, the MPC catalogue and DE440 are not used.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Constants (public values).
# --------------------------------------------------------------------------
AU_KM = 149597870.7
C_AU_PER_DAY = 299792.458 * 86400.0 / AU_KM          # 173.144632674...
OBLIQUITY_J2000_RAD = math.radians(84381.448 / 3600.0)

# GM in au^3/day^2 (DE440 values for the Sun and the planetary systems).
GM_SUN = 2.9591220828411956e-04
_PLANETS = [
    # name, GM, a[au], e, I[deg], L[deg], long.peri[deg], node[deg]
    # J2000 mean elements (Standish, "Keplerian elements for approximate
    # positions of the major planets", table 1).
    ("mercury", 4.9125001948893182e-11, 0.38709927, 0.20563593, 7.00497902, 252.25032350, 77.45779628, 48.33076593),
    ("venus",   7.2434523326441187e-10, 0.72333566, 0.00677672, 3.39467605, 181.97909950, 131.60246718, 76.67984255),
    ("earth",   8.9970116036316091e-10, 1.00000261, 0.01671123, -0.00001531, 100.46457166, 102.93768193, 0.0),
    ("mars",    9.5495488297258119e-11, 1.52371034, 0.09339410, 1.84969142, -4.55343205, -23.94362959, 49.55953891),
    ("jupiter", 2.8253458252257917e-07, 5.20288700, 0.04838624, 1.30439695, 34.39644051, 14.72847983, 100.47390909),
    ("saturn",  8.4597059933762903e-08, 9.53667594, 0.05386179, 2.48599187, 49.95424423, 92.59887831, 113.66242448),
    ("uranus",  1.2920265649682399e-08, 19.18916464, 0.04725744, 0.77263783, 313.23810451, 170.95427630, 74.01692503),
    ("neptune", 1.5243573478851939e-08, 30.06992276, 0.00859048, 1.77004347, -55.12002969, 44.96476227, 131.78422574),
]
PLANET_NAMES = [p[0] for p in _PLANETS]
# Extra perturbers: the largest main-belt asteroids on fixed ellipses, with
# rounded published GM values and rounded osculating elements (stand-ins
# for their ephemerides, same columns as above; L and long.peri in deg).
_ASTEROIDS = [
    ("ceres",      1.3962e-13, 2.7675, 0.0758, 10.594, 153.9 + 95.0, 153.9, 80.3),
    ("vesta",      3.8548e-14, 2.3615, 0.0887, 7.140, 255.0 + 20.0, 255.0, 103.8),
    ("pallas",     3.0471e-14, 2.7720, 0.2305, 34.840, 123.1 + 40.0, 123.1, 173.1),
    ("hygiea",     1.2542e-14, 3.1421, 0.1125, 3.832, 235.5 + 200.0, 235.5, 283.2),
    ("interamnia", 5.8e-15, 3.0560, 0.1550, 17.310, 15.7 + 100.0, 15.7, 280.3),
    ("eunomia",    4.7e-15, 2.6440, 0.1870, 11.750, 31.5 + 300.0, 31.5, 292.9),
    ("juno",       4.0e-15, 2.6690, 0.2570, 12.990, 57.9 + 250.0, 57.9, 169.8),
]
ASTEROID_NAMES = [p[0] for p in _ASTEROIDS]
# Bodies that carry the first post-Newtonian correction (Sun, Jupiter, Earth).
GR_BODIES = ("sun", "jupiter", "earth")

# The Moon as a registered mass: the "earth" row above is the Earth-Moon
# barycentre; with the Moon, the Earth and the Moon (DE440 GM values) sit
# on either side of it, the Moon's geocentric orbit a mean ellipse whose
# node regresses and perigee advances uniformly (rounded published mean
# elements at J2000, ecliptic; angles in degrees, rates in degrees/day).
GM_EARTH = 8.8876924467071033e-10
GM_MOON = 1.0931894624024351e-11
_MOON_ORBIT = dict(a=384400.0 / 149597870.7, e=0.0549, I=5.145,
                   L0=218.3164477, Ldot=13.17639648, peri0=83.3532465, peridot=0.1114040,
                   node0=125.0445479, nodedot=-0.0529539)

# Oblateness of the bodies that carry the App. A.3 term: J2, equatorial
# radius (km) and the pole's right ascension and declination (deg,
# equatorial J2000), rounded published values (IAU rotation elements;
# helioseismic solar J2; Juno gravity field).
_J2_BODIES = {
    "sun": (2.2e-7, 696000.0, 286.13, 63.87),
    "jupiter": (1.4696514e-2, 71492.0, 268.056595, 64.495303),
}
AU_KM = 149597870.7

SEG_DAYS = 8.0
CHEB_DEGREE = 12


# --------------------------------------------------------------------------
# Elliptic elements -> Cartesian (input construction only).
# --------------------------------------------------------------------------
def _solve_kepler_E(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    M = np.mod(M, 2.0 * np.pi)
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    small = False
    for _ in range(60):
        f = E - e * np.sin(E) - M
        fp = 1.0 - e * np.cos(E)
        dE = f / fp
        E = E - dE
        if small:            # one Newton step past |dE| < 1e-12 reaches round-off
            break
        small = E.size == 0 or np.max(np.abs(dE)) < 1e-12
    return E


def elements_to_state(a, e, inc, node, peri, M, mu):
    """Elliptic elements (radians) -> heliocentric ecliptic state [..., 6]."""
    a = np.asarray(a, float); e = np.asarray(e, float)
    E = _solve_kepler_E(np.asarray(M, float), e)
    cE, sE = np.cos(E), np.sin(E)
    b = np.sqrt(1.0 - e * e)
    r = a * (1.0 - e * cE)
    xp = a * (cE - e)
    yp = a * b * sE
    k = np.sqrt(mu * a) / r
    vxp = -k * sE
    vyp = k * b * cE
    cO, sO = np.cos(node), np.sin(node)
    ci, si = np.cos(inc), np.sin(inc)
    cw, sw = np.cos(peri), np.sin(peri)
    # Columns of the perifocal -> ecliptic rotation R3(-node) R1(-inc) R3(-peri).
    Px = cO * cw - sO * sw * ci
    Py = sO * cw + cO * sw * ci
    Pz = sw * si
    Qx = -cO * sw - sO * cw * ci
    Qy = -sO * sw + cO * cw * ci
    Qz = cw * si
    out = np.empty(np.broadcast(a, M).shape + (6,))
    out[..., 0] = xp * Px + yp * Qx
    out[..., 1] = xp * Py + yp * Qy
    out[..., 2] = xp * Pz + yp * Qz
    out[..., 3] = vxp * Px + vyp * Qx
    out[..., 4] = vxp * Py + vyp * Qy
    out[..., 5] = vxp * Pz + vyp * Qz
    return out


@dataclasses.dataclass
class PlanetModel:
    """Sun plus planets on fixed heliocentric ellipses (an analytic stand-in
    for a planetary ephemeris), optionally the Moon about the Earth."""
    names: List[str]
    gm: np.ndarray          # [n_body] (index 0 = Sun) registered masses
    el: np.ndarray          # [n_planet, 6]: a, e, I, node, peri, M0 (radians)
    n: np.ndarray           # mean motions [rad/day]
    msys: np.ndarray        # [n_planet] mass of each ellipse's system (Earth + Moon for "earth")
    moon: bool = False      # last body: the Moon; the "earth" ellipse carries their barycentre

    @staticmethod
    def make(planets: Optional[List[str]] = None, moon: Optional[bool] = None) -> "PlanetModel":
        """The planets (all eight by default) and, by default when the
        Earth is among them, the Moon (the default registered masses of
        Sect. 3.2)."""
        planets = PLANET_NAMES if planets is None else list(planets)
        moon = ("earth" in planets) if moon is None else bool(moon)
        if moon and "earth" not in planets:
            raise ValueError("the Moon needs the Earth")
        order = PLANET_NAMES + ASTEROID_NAMES
        rows = [p for p in _PLANETS + _ASTEROIDS if p[0] in planets]
        rows.sort(key=lambda p: order.index(p[0]))
        msys = np.array([p[1] for p in rows])
        el = []
        for p in rows:
            a, e, I, L, varpi, node = p[2:]
            el.append([a, e, math.radians(I), math.radians(node),
                       math.radians(varpi - node), math.radians(L - varpi)])
        el = np.array(el).reshape(-1, 6)
        n = np.sqrt((GM_SUN + msys) / el[:, 0] ** 3)
        names = ["sun"] + [p[0] for p in rows]
        gm = np.concatenate([[GM_SUN], msys])
        if moon:
            gm[names.index("earth")] = GM_EARTH
            gm = np.concatenate([gm, [GM_MOON]])
            names = names + ["moon"]
        return PlanetModel(names, gm, el, n, msys, moon)

    def helio(self, t: np.ndarray) -> np.ndarray:
        """Heliocentric states [..., n_planet, 6] of the ellipses (the
        Earth-Moon barycentre for "earth") at times t [...]."""
        t = np.asarray(t, float)
        M = self.el[:, 5] + self.n * t[..., None]
        mu = GM_SUN + self.msys
        return elements_to_state(self.el[:, 0], self.el[:, 1], self.el[:, 2],
                                 self.el[:, 3], self.el[:, 4], M, mu)

    def moon_geo(self, t: np.ndarray) -> np.ndarray:
        """Geocentric state [..., 6] of the Moon at times t [...]: the
        position on the mean ellipse and its exact time derivative
        (motion in mean anomaly plus the turning node and perigee)."""
        t = np.asarray(t, float)
        o = _MOON_ORBIT
        mu = GM_EARTH + GM_MOON
        node = np.radians(o["node0"] + o["nodedot"] * t)
        varpi = np.radians(o["peri0"] + o["peridot"] * t)
        M = np.radians(o["L0"] + o["Ldot"] * t) - varpi
        st = elements_to_state(o["a"], o["e"], math.radians(o["I"]), node, varpi - node, M, mu)
        r, vk = st[..., :3], st[..., 3:]
        n_kep = math.sqrt(mu / o["a"] ** 3)
        Mdot = math.radians(o["Ldot"] - o["peridot"])
        Odot = math.radians(o["nodedot"])
        wdot = math.radians(o["peridot"] - o["nodedot"])
        h = np.cross(r, vk)
        h /= np.linalg.norm(h, axis=-1, keepdims=True)
        zr = np.stack([-r[..., 1], r[..., 0], np.zeros_like(r[..., 0])], axis=-1)     # z x r
        v = vk * (Mdot / n_kep) + Odot * zr + wdot * np.cross(h, r)
        return np.concatenate([r, v], axis=-1)

    def bary(self, t: np.ndarray) -> np.ndarray:
        """Barycentric states [..., n_body, 6]; body 0 is the Sun."""
        h = self.helio(t)
        m = self.msys / (GM_SUN + self.msys.sum())
        sun = -(m[:, None] * h).sum(axis=-2)
        out = np.concatenate([sun[..., None, :], sun[..., None, :] + h], axis=-2)
        if self.moon:
            ie = self.names.index("earth")
            g = self.moon_geo(t)
            emb = out[..., ie, :].copy()
            out[..., ie, :] = emb - (GM_MOON / (GM_EARTH + GM_MOON)) * g
            out = np.concatenate([out, (emb + (GM_EARTH / (GM_EARTH + GM_MOON)) * g)[..., None, :]], axis=-2)
        return out

    def sun(self, t):
        return self.bary(t)[..., 0, :]


# --------------------------------------------------------------------------
# Chebyshev tables.
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Ephemeris:
    """Chebyshev-tabulated perturber positions.

    coef[body][seg][xyz][k] gives the position of `body` inside segment
    `seg` (covering [t_start + seg*seg_days, t_start + (seg+1)*seg_days])
    as sum_k coef[k] T_k(tau), tau = 2 (t - t_seg)/seg_days - 1.
    """
    coef: np.ndarray
    gm: np.ndarray
    flags: np.ndarray       # uint32, bit0 = first post-Newtonian term
    t_start: float
    seg_days: float
    names: List[str]
    j2: Optional[np.ndarray] = None   # [n_body, 5]: J2, radius (au), unit pole; J2 = 0: no term (App. A.3)

    @property
    def n_body(self): return self.coef.shape[0]
    @property
    def n_seg(self): return self.coef.shape[1]
    @property
    def degree(self): return self.coef.shape[3] - 1
    @property
    def t_end(self): return self.t_start + self.n_seg * self.seg_days


def cheb_fit_nodes(degree: int) -> np.ndarray:
    """Chebyshev-Gauss nodes (roots of T_{degree+1}) on [-1, 1]."""
    m = degree + 1
    return np.cos(np.pi * (np.arange(m) + 0.5) / m)


def cheb_fit_matrix(degree: int) -> np.ndarray:
    """Discrete Chebyshev transform: coef = W @ f(nodes)."""
    m = degree + 1
    x = cheb_fit_nodes(degree)
    T = np.cos(np.outer(np.arange(m), np.arccos(x)))   # T[k, j] = T_k(x_j)
    W = (2.0 / m) * T
    W[0] *= 0.5
    return W


def j2_rows(names: List[str]) -> Optional[np.ndarray]:
    """[n_body, 5] J2 rows (J2, radius au, unit pole in the ecliptic
    integration frame) of the bodies in _J2_BODIES, zero rows for the
    others; None when no body has one."""
    rows = np.zeros((len(names), 5))
    for i, nm in enumerate(names):
        if nm in _J2_BODIES:
            j2, r_km, ra, dec = _J2_BODIES[nm]
            ra, dec = math.radians(ra), math.radians(dec)
            pole_eq = np.array([math.cos(dec) * math.cos(ra), math.cos(dec) * math.sin(ra), math.sin(dec)])
            rows[i] = [j2, r_km / AU_KM, *equatorial_to_ecliptic(pole_eq)]
    return rows if rows[:, 0].any() else None


def make_ephemeris(model: PlanetModel, t_start: float, n_seg: int,
                   seg_days: float = SEG_DAYS, degree: int = CHEB_DEGREE,
                   gr: bool = True, j2: bool = True) -> Ephemeris:
    """Tabulate `model` as Chebyshev segments by interpolation at the
    Chebyshev-Gauss nodes of every segment; the Sun and Jupiter get their
    J2 term (App. A.3) unless j2 is False."""
    x = cheb_fit_nodes(degree)
    W = cheb_fit_matrix(degree)
    seg0 = t_start + seg_days * np.arange(n_seg)
    tn = seg0[:, None] + 0.5 * seg_days * (x[None, :] + 1.0)     # [seg, node]
    st = model.bary(tn)                                           # [seg, node, body, 6]
    pos = st[..., :3]                                             # [seg, node, body, 3]
    coef = np.einsum("kj,sjbc->bsck", W, pos)                     # [body, seg, 3, deg+1]
    flags = np.array([1 if (gr and nm in GR_BODIES) else 0 for nm in model.names],
                     dtype=np.uint32)
    return Ephemeris(np.ascontiguousarray(coef), model.gm.copy(), flags,
                     float(t_start), float(seg_days), list(model.names),
                     j2_rows(list(model.names)) if j2 else None)


def sun_only_ephemeris(t_start: float, n_seg: int, gr: bool = False,
                       seg_days: float = SEG_DAYS, degree: int = CHEB_DEGREE,
                       j2: Optional[Tuple[float, float, Sequence[float]]] = None) -> Ephemeris:
    """A single perturber (the Sun) fixed at the origin; j2 = (J2, radius
    in au, pole) gives it the oblateness term of App. A.3."""
    coef = np.zeros((1, n_seg, 3, degree + 1))
    row = None
    if j2 is not None:
        pole = np.asarray(j2[2], float)
        row = np.array([[float(j2[0]), float(j2[1]), *(pole / np.linalg.norm(pole))]])
    return Ephemeris(coef, np.array([GM_SUN]), np.array([1 if gr else 0], np.uint32),
                     float(t_start), float(seg_days), ["sun"], row)


def polynomial_ephemeris(rng: np.random.Generator, n_body: int, t_start: float,
                         n_seg: int, seg_days: float = SEG_DAYS,
                         degree: int = CHEB_DEGREE) -> Ephemeris:
    """Random coefficient tables (for evaluator tests)."""
    coef = rng.normal(size=(n_body, n_seg, 3, degree + 1))
    gm = np.full(n_body, 1e-9)
    return Ephemeris(coef, gm, np.zeros(n_body, np.uint32), float(t_start),
                     float(seg_days), [f"b{i}" for i in range(n_body)])


# --------------------------------------------------------------------------
# Small bodies.
# --------------------------------------------------------------------------
def _rayleigh_truncated(rng, sigma, n, upper):
    out = rng.rayleigh(sigma, n)
    bad = out >= upper
    while bad.any():
        out[bad] = rng.rayleigh(sigma, bad.sum())
        bad = out >= upper
    return out


def main_belt_elements(rng: np.random.Generator, n: int) -> np.ndarray:
    """a ~ U(2.1, 3.3) au; e ~ Rayleigh(0.1) resampled until e < 0.4;
    i ~ Rayleigh(8 deg); node, peri, M ~ U(0, 2 pi)."""
    a = rng.uniform(2.1, 3.3, n)
    e = _rayleigh_truncated(rng, 0.1, n, 0.4)
    inc = rng.rayleigh(math.radians(8.0), n)
    ang = rng.uniform(0.0, 2.0 * np.pi, (3, n))
    return np.stack([a, e, inc, ang[0], ang[1], ang[2]], axis=1)


def neo_elements(rng: np.random.Generator, n: int) -> np.ndarray:
    """a ~ U(0.8, 2.0) au; e ~ U(0.1, 0.7); i ~ Rayleigh(8 deg)."""
    a = rng.uniform(0.8, 2.0, n)
    e = rng.uniform(0.1, 0.7, n)
    inc = rng.rayleigh(math.radians(8.0), n)
    ang = rng.uniform(0.0, 2.0 * np.pi, (3, n))
    return np.stack([a, e, inc, ang[0], ang[1], ang[2]], axis=1)


def bodies_from_elements(model: PlanetModel, el: np.ndarray, epoch: float) -> np.ndarray:
    """Barycentric states [n, 6] at `epoch` from heliocentric elements."""
    st = elements_to_state(el[:, 0], el[:, 1], el[:, 2], el[:, 3], el[:, 4], el[:, 5], GM_SUN)
    return st + model.sun(np.array(epoch))[None, :]


def hg_params(rng: np.random.Generator, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Absolute magnitude H and slope G of n bodies for the H-G magnitude
    system: H uniform in [8, 20] (numbered main-belt range), G normal
    around the customary 0.15 (sigma 0.08) clipped to [-0.1, 0.6]."""
    H = rng.uniform(8.0, 20.0, n)
    G = np.clip(rng.normal(0.15, 0.08, n), -0.1, 0.6)
    return H, G


def make_population(rng, model, n, neo_frac, epoch):
    n_neo = int(round(n * neo_frac))
    el = np.concatenate([main_belt_elements(rng, n - n_neo), neo_elements(rng, n_neo)])
    is_neo = np.zeros(n, bool); is_neo[n - n_neo:] = True
    perm = rng.permutation(n)
    el, is_neo = el[perm], is_neo[perm]
    return bodies_from_elements(model, el, epoch), el, is_neo


# --------------------------------------------------------------------------
# Frames.
# --------------------------------------------------------------------------
def tangent_basis(center: np.ndarray):
    """Local east/north unit vectors at ecliptic directions `center` [...,3]."""
    z = np.array([0.0, 0.0, 1.0])
    east = np.cross(z, center)
    nrm = np.linalg.norm(east, axis=-1, keepdims=True)
    polar = nrm[..., 0] < 1e-12
    east = np.where(polar[..., None], np.array([0.0, 1.0, 0.0]), east / np.where(nrm > 0, nrm, 1))
    north = np.cross(center, east)
    return east, north


def rect_normals(center, u, w, half_u, half_w):
    """Inward great-circle normals [..., 4, 3] of the gnomonic rectangle
    |d.u/d.c| < tan(half_u), |d.w/d.c| < tan(half_w)."""
    su, cu = np.sin(half_u)[..., None], np.cos(half_u)[..., None]
    sw, cw = np.sin(half_w)[..., None], np.cos(half_w)[..., None]
    n = np.stack([su * center - cu * u, su * center + cu * u,
                  sw * center - cw * w, sw * center + cw * w], axis=-2)
    return n


@dataclasses.dataclass
class Frames:
    """Frames with per-sub-frame geometry; center .. half_w may be None for
    large footprint sets, where only the normals are kept."""
    t: np.ndarray          # [F]
    obs: np.ndarray        # [F, 3] barycentric observer position
    center: np.ndarray     # [F, S, 3] sub-frame centres
    u: np.ndarray          # [F, S, 3]
    w: np.ndarray          # [F, S, 3]
    half_u: np.ndarray     # [F, S] radians
    half_w: np.ndarray     # [F, S]
    normals: np.ndarray    # [F, S, 4, 3]

    @property
    def n_frames(self): return self.t.shape[0]
    @property
    def n_sub(self): return self.normals.shape[1]

    def subset(self, idx):
        idx = np.asarray(idx)
        g = lambda a: None if a is None else a[idx]
        return Frames(self.t[idx], self.obs[idx], g(self.center), g(self.u), g(self.w),
                      g(self.half_u), g(self.half_w), self.normals[idx])

    @staticmethod
    def concat(parts):
        def cat(name):
            arrs = [getattr(p, name) for p in parts]
            return None if any(a is None for a in arrs) else np.concatenate(arrs)
        return Frames(*[cat(f.name) for f in dataclasses.fields(Frames)])


def _frames_from_pointing(t, obs, center, roll, half_u, half_w):
    east, north = tangent_basis(center)
    cr, sr = np.cos(roll)[..., None], np.sin(roll)[..., None]
    u = cr * east + sr * north
    w = -sr * east + cr * north
    half_u = np.broadcast_to(half_u, center.shape[:-1]).astype(float)
    half_w = np.broadcast_to(half_w, center.shape[:-1]).astype(float)
    return Frames(t, obs, center[:, None], u[:, None], w[:, None],
                  half_u[:, None], half_w[:, None],
                  rect_normals(center, u, w, half_u, half_w)[:, None])


def circular_observer(model: PlanetModel, t: np.ndarray, phase0: float = 0.0) -> np.ndarray:
    """Barycentric position of an observer on a 1 au circular heliocentric
    orbit in the ecliptic."""
    n = math.sqrt(GM_SUN)
    th = phase0 + n * t
    helio = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], axis=-1)
    return helio + model.sun(t)[..., :3]


def frames_tiny(rng, model, n_frames, t0, span, width_deg, max_lat_deg=20.0):
    """Square frames pointed uniformly (in solid angle) within +-max_lat of
    the ecliptic, exposure times uniform over [t0, t0+span], roll 0."""
    t = np.sort(rng.uniform(t0, t0 + span, n_frames))
    lon = rng.uniform(0.0, 2.0 * np.pi, n_frames)
    slat = rng.uniform(-math.sin(math.radians(max_lat_deg)), math.sin(math.radians(max_lat_deg)), n_frames)
    clat = np.sqrt(1.0 - slat ** 2)
    center = np.stack([clat * np.cos(lon), clat * np.sin(lon), slat], axis=1)
    obs = circular_observer(model, t)
    h = math.radians(width_deg / 2.0)
    return _frames_from_pointing(t, obs, center, np.zeros(n_frames), h, h)


def frames_survey(rng, model, n_frames, t0, span, width_deg=0.78, seq_len=12,
                  cadence_s=11.0, step_deg=0.7, offset_km=7000.0,
                  offset_period_min=97.1, max_lat_deg=40.0):
    """Space-survey frames: observer on a 1 au circle plus a circular
    terminator offset orbit; sequences of `seq_len` exposures `cadence_s`
    apart, stepping `step_deg` along the 90-degree-elongation great circle,
    each frame rolled so that its first axis is the scan direction."""
    n_seq = -(-n_frames // seq_len)
    # one telescope: sequences start at jittered times but never overlap,
    # so the exposure list is chronological
    gap = (span - 1.0 / 24.0) / n_seq
    busy = min(1.0, (seq_len - 1) * cadence_s / 86400.0 / gap)
    t_seq = t0 + (np.arange(n_seq) + rng.uniform(0, 1, n_seq) * (1.0 - busy)) * gap
    j = np.arange(seq_len)
    t = (t_seq[:, None] + j[None, :] * cadence_s / 86400.0).reshape(-1)[:n_frames]
    n = math.sqrt(GM_SUN)
    th = n * t
    rhat = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], axis=-1)
    along = np.stack([-np.sin(th), np.cos(th), np.zeros_like(th)], axis=-1)
    zhat = np.broadcast_to(np.array([0.0, 0.0, 1.0]), rhat.shape)
    phi = 2.0 * np.pi * t / (offset_period_min / 1440.0)
    R = offset_km / AU_KM
    obs = model.sun(t)[..., :3] + rhat + R * (np.cos(phi)[:, None] * zhat + np.sin(phi)[:, None] * along)
    # start angle on the elongation-90 circle: d(psi) = cos psi along + sin psi z
    side = rng.integers(0, 2, n_seq) * np.pi
    psi0 = rng.uniform(-math.radians(max_lat_deg), math.radians(max_lat_deg), n_seq)
    psi = ((psi0[:, None] + j[None, :] * math.radians(step_deg)).reshape(-1)[:n_frames]
           + np.repeat(side, seq_len)[:n_frames])
    cp, sp = np.cos(psi)[:, None], np.sin(psi)[:, None]
    center = cp * along + sp * zhat
    u = -sp * along + cp * zhat                   # scan direction
    w = np.cross(center, u)
    h = math.radians(width_deg / 2.0)
    hu = np.full(n_frames, h); hw = np.full(n_frames, h)
    return Frames(t, obs, center[:, None], u[:, None], w[:, None], hu[:, None], hw[:, None],
                  rect_normals(center, u, w, hu, hw)[:, None])


def frames_targeted(rng, model, states_el, t0, span, n_frames, width_deg=1.5,
                    straddle_frac=0.5):
    """Frames aimed at the analytic two-body direction of randomly chosen
    bodies (from their elements), half of them offset so that the body
    lies near an edge.  Used to obtain many (object, frame) pairs in
    small parity cases."""
    el = states_el
    idx = rng.integers(0, el.shape[0], n_frames)
    t = np.sort(rng.uniform(t0, t0 + span, n_frames))
    M = el[idx, 5] + np.sqrt(GM_SUN / el[idx, 0] ** 3) * (t - t0)
    helio = elements_to_state(el[idx, 0], el[idx, 1], el[idx, 2], el[idx, 3], el[idx, 4], M, GM_SUN)
    obs = circular_observer(model, t)
    pos = helio[:, :3] + model.sun(t)[:, :3]
    d = pos - obs
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    h = math.radians(width_deg / 2.0)
    east, north = tangent_basis(d)
    off = np.zeros((n_frames, 2))
    k = rng.uniform(0, 1, n_frames) < straddle_frac
    # put the body near an edge: shift the centre by about one half-width
    off[k, 0] = rng.choice([-1, 1], k.sum()) * h * rng.uniform(0.9, 1.1, k.sum())
    off[k, 1] = rng.uniform(-0.5, 0.5, k.sum()) * h
    center = d + off[:, :1] * east + off[:, 1:] * north
    center /= np.linalg.norm(center, axis=1, keepdims=True)
    roll = rng.uniform(0, 2 * np.pi, n_frames)
    return _frames_from_pointing(t, obs, center, roll, h, h)


R_EARTH_AU = 6378.137 / AU_KM


def equatorial_to_ecliptic(v: np.ndarray) -> np.ndarray:
    ce, se = math.cos(OBLIQUITY_J2000_RAD), math.sin(OBLIQUITY_J2000_RAD)
    out = np.empty_like(v)
    out[..., 0] = v[..., 0]
    out[..., 1] = ce * v[..., 1] + se * v[..., 2]
    out[..., 2] = -se * v[..., 1] + ce * v[..., 2]
    return out


def ground_sites(t: np.ndarray, lon: np.ndarray, lat: float) -> np.ndarray:
    """Equatorial unit vectors of sites at east longitude `lon` and latitude
    `lat` (radians) at times t, the Earth turning by the Earth Rotation
    Angle (time scales not distinguished)."""
    era = 2.0 * np.pi * (0.7790572732640 + 1.00273781191135448 * t)
    a = era + lon
    return np.stack([math.cos(lat) * np.cos(a), math.cos(lat) * np.sin(a), np.full_like(a, math.sin(lat))], -1)


def frames_ground(rng, model, n_frames, t0, span, n_sites=6, lat_deg=33.0, exposure_s=30.0, night_h=8.0,
                  foot_u_deg=7.0, foot_w_deg=7.3, grid=8, sub_deg=0.87, min_alt_deg=30.0,
                  keep_geometry=False, chunk=65536):
    """Ground-survey footprints: n_sites sites at latitude lat_deg, spread
    evenly in longitude, each exposing every exposure_s seconds through an
    8 h block centred on local midnight; each exposure points uniformly in
    solid angle above min_alt_deg and is a foot_u x foot_w degree footprint
    made of grid x grid square sub-frames of sub_deg degrees on the
    footprint's gnomonic plane.  The first n_frames exposures in time order
    are kept.  Only the normals of the sub-frames are stored unless
    keep_geometry is set."""
    lons = 2.0 * np.pi * np.arange(n_sites) / n_sites
    per_night = int(round(night_h * 3600.0 / exposure_s))
    n_days = int(math.ceil(span)) + 1
    ts, ls = [], []
    for s_i, lon in enumerate(lons):
        # local midnight: t = n + 1/2 - lon / 2 pi (J2000 at noon)
        mid = np.arange(-1, n_days + 1) + 0.5 - lon / (2.0 * np.pi)
        tt = (mid[:, None] + ((np.arange(per_night) + 0.5) * exposure_s / 86400.0 - night_h / 48.0)[None, :]).ravel()
        tt = tt[(tt >= t0) & (tt < t0 + span)]
        ts.append(tt)
        ls.append(np.full(tt.size, lon))
    t = np.concatenate(ts)
    lon = np.concatenate(ls)
    order = np.argsort(t, kind="stable")[:n_frames]
    t, lon = t[order], lon[order]
    F = t.size
    lat = math.radians(lat_deg)
    zen_eq = ground_sites(t, lon, lat)
    ie = PLANET_NAMES.index("earth") + 1
    earth = model.bary(t)[:, ie, :3]
    obs = earth + R_EARTH_AU * equatorial_to_ecliptic(zen_eq)
    # pointing: altitude with uniform sin, azimuth uniform
    salt = rng.uniform(math.sin(math.radians(min_alt_deg)), 1.0, F)
    calt = np.sqrt(1.0 - salt * salt)
    az = rng.uniform(0.0, 2.0 * np.pi, F)
    east_eq = np.stack([-zen_eq[:, 1], zen_eq[:, 0], np.zeros(F)], -1)
    east_eq /= np.linalg.norm(east_eq, axis=-1, keepdims=True)
    north_eq = np.cross(zen_eq, east_eq)
    d_eq = salt[:, None] * zen_eq + calt[:, None] * (np.cos(az)[:, None] * north_eq + np.sin(az)[:, None] * east_eq)
    center = equatorial_to_ecliptic(d_eq)
    center /= np.linalg.norm(center, axis=-1, keepdims=True)
    fu, fw = tangent_basis(center)
    S = grid * grid
    h = math.radians(sub_deg / 2.0)
    xi = np.tan(math.radians(foot_u_deg) / grid) * (np.arange(grid) - (grid - 1) / 2.0)
    eta = np.tan(math.radians(foot_w_deg) / grid) * (np.arange(grid) - (grid - 1) / 2.0)
    gx, gy = np.meshgrid(xi, eta, indexing="ij")
    gx, gy = gx.ravel(), gy.ravel()
    normals = np.empty((F, S, 4, 3))
    geo = None
    if keep_geometry:
        geo = [np.empty((F, S, 3)), np.empty((F, S, 3)), np.empty((F, S, 3))]
    def fill(a):
        b = min(F, a + chunk)
        c = center[a:b, None, :] + gx[None, :, None] * fu[a:b, None, :] + gy[None, :, None] * fw[a:b, None, :]
        c /= np.linalg.norm(c, axis=-1, keepdims=True)
        u = fu[a:b, None, :] - np.sum(fu[a:b, None, :] * c, -1, keepdims=True) * c
        u /= np.linalg.norm(u, axis=-1, keepdims=True)
        w = np.cross(c, u)
        hh = np.full(c.shape[:-1], h)
        normals[a:b] = rect_normals(c, u, w, hh, hh)
        if keep_geometry:
            geo[0][a:b], geo[1][a:b], geo[2][a:b] = c, u, w

    # disjoint slices, numpy releases the GIL: fill them on a few threads
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(fill, range(0, F, chunk)))
    if keep_geometry:
        hu = np.full((F, S), h)
        return Frames(t, obs, geo[0], geo[1], geo[2], hu, hu.copy(), normals)
    return Frames(t, obs, None, None, None, None, None, normals)


def footprint_case(seed: int = 3, n_obj: int = 750_000, n_frames: int = 2_000_000, span: float = 365.25,
                   neo_frac: float = 0.05, keep_geometry: bool = False) -> PropagationCase:
    """750,000 bodies (main belt plus 5% NEO-like), all 8 planets, one
    year, 2,000,000 ground footprints of 7 x 7.3 degrees in 8 x 8
    sub-frames of 0.87 degrees from six sites at latitude 33 degrees."""
    rng = np.random.default_rng(seed)
    model = PlanetModel.make()
    n_seg = int(math.ceil((span + 24.0) / SEG_DAYS))
    eph = make_ephemeris(model, -8.0, n_seg)
    x0, el, is_neo = make_population(rng, model, n_obj, neo_frac, 0.0)
    fr = frames_ground(rng, model, n_frames, 0.0, span, keep_geometry=keep_geometry) if n_frames else None
    return PropagationCase("footprint", eph, model, x0, el, is_neo, 0.0, span, fr, seed)


def ecliptic_to_equatorial(v: np.ndarray) -> np.ndarray:
    ce, se = math.cos(OBLIQUITY_J2000_RAD), math.sin(OBLIQUITY_J2000_RAD)
    out = np.empty_like(v)
    out[..., 0] = v[..., 0]
    out[..., 1] = ce * v[..., 1] - se * v[..., 2]
    out[..., 2] = se * v[..., 1] + ce * v[..., 2]
    return out


# --------------------------------------------------------------------------
# Configurations (sizes of the five workloads; `scale` shrinks counts).
# --------------------------------------------------------------------------
@dataclasses.dataclass
class PropagationCase:
    name: str
    ephem: Ephemeris
    model: PlanetModel
    x0: np.ndarray           # [N, 6]
    elements: np.ndarray     # [N, 6] heliocentric elements at t0
    is_neo: np.ndarray
    t0: float
    span: float
    frames: Optional[Frames]
    seed: int


def tiny_case(seed: int = 1, n_obj: int = 1000, n_frames: int = 100, span: float = 30.0,
              n_targeted: int = 0) -> PropagationCase:
    """1,000 main-belt bodies, Sun + Jupiter + Saturn as 8-day degree-12
    Chebyshev segments, 30 days, 100 frames of 1.5 deg x 1.5 deg from a
    1 au circular observer pointed within +-20 deg of the ecliptic."""
    rng = np.random.default_rng(seed)
    model = PlanetModel.make(["jupiter", "saturn"])
    n_seg = int(math.ceil((span + 24.0) / SEG_DAYS))
    eph = make_ephemeris(model, -8.0, n_seg)
    el = main_belt_elements(rng, n_obj)
    x0 = bodies_from_elements(model, el, 0.0)
    fr = frames_tiny(rng, model, n_frames, 0.0, span, 1.5)
    if n_targeted:
        fr = Frames.concat([fr, frames_targeted(rng, model, el, 0.0, span, n_targeted)])
        order = np.argsort(fr.t, kind="stable")
        fr = fr.subset(order)
    return PropagationCase("tiny", eph, model, x0, el, np.zeros(n_obj, bool), 0.0, span, fr, seed)


def survey_case(seed: int = 2, n_obj: int = 100_000, n_frames: int = 500_000,
                span: float = 365.25, neo_frac: float = 0.05) -> PropagationCase:
    """100,000 bodies (95% main belt, 5% NEO-like), all 8 planets, one year,
    500,000 frames of 0.78 deg from a space observer on a 1 au orbit plus
    a 7,000 km offset orbit, in 11 s sequences of 12 along great circles."""
    rng = np.random.default_rng(seed)
    model = PlanetModel.make()
    n_seg = int(math.ceil((span + 24.0) / SEG_DAYS))
    eph = make_ephemeris(model, -8.0, n_seg)
    x0, el, is_neo = make_population(rng, model, n_obj, neo_frac, 0.0)
    fr = frames_survey(rng, model, n_frames, 0.0, span) if n_frames else None
    return PropagationCase("survey", eph, model, x0, el, is_neo, 0.0, span, fr, seed)


@dataclasses.dataclass
class GradientCase:
    ephem: Ephemeris
    x_true: np.ndarray       # [N, 6]
    x0: np.ndarray           # [N, 6] perturbed start
    t0: float
    t_obs: np.ndarray        # [N, K]
    obs_pos: np.ndarray      # [N, K, 3]
    radec_obs: np.ndarray    # [N, K, 2] equatorial RA/Dec (radians)
    arc: float


def gradient_case(seed: int = 4, n_obj: int = 100_000, k_obs: int = 20, arc: float = 60.0,
                  neo_frac: float = 0.05, noise_arcsec: float = 0.1) -> GradientCase:
    """Bodies with a 60-day arc of 20 observations each from a 1 au
    observer.  The observed RA/Dec are the analytic two-body directions of
    the generating elements plus Gaussian noise; the start state is the
    generating state plus N(0, 1e-6 au), N(0, 1e-8 au/day)."""
    rng = np.random.default_rng(seed)
    model = PlanetModel.make()
    eph = make_ephemeris(model, -8.0, int(math.ceil((arc + 24.0) / SEG_DAYS)))
    x_true, el, _ = make_population(rng, model, n_obj, neo_frac, 0.0)
    t_obs = np.sort(rng.uniform(0.0, arc, (n_obj, k_obs)), axis=1)
    obs = circular_observer(model, t_obs)
    M = el[:, None, 5] + np.sqrt(GM_SUN / el[:, None, 0] ** 3) * t_obs
    helio = elements_to_state(el[:, None, 0], el[:, None, 1], el[:, None, 2],
                              el[:, None, 3], el[:, None, 4], M, GM_SUN)
    pos = helio[..., :3] + model.sun(t_obs)[..., :3]
    d = ecliptic_to_equatorial(pos - obs)
    ra = np.arctan2(d[..., 1], d[..., 0]) % (2 * np.pi)
    dec = np.arcsin(d[..., 2] / np.linalg.norm(d, axis=-1))
    sig = math.radians(noise_arcsec / 3600.0)
    dec_o = dec + rng.normal(0, sig, dec.shape)
    ra_o = (ra + rng.normal(0, sig, ra.shape) / np.cos(dec)) % (2 * np.pi)
    x0 = x_true.copy()
    x0[:, :3] += rng.normal(0, 1e-6, (n_obj, 3))
    x0[:, 3:] += rng.normal(0, 1e-8, (n_obj, 3))
    return GradientCase(eph, x_true, x0, 0.0, t_obs, obs, np.stack([ra_o, dec_o], -1), arc)


@dataclasses.dataclass
class JobSpec:
    n_obj: np.ndarray        # [J]
    span: np.ndarray         # [J] days
    n_frames: np.ndarray     # [J]


def batched_job_specs(seed: int = 5, n_jobs: int = 4096, max_obj: int = 20_000,
                      max_span: float = 3652.5, max_frames: int = 5000) -> JobSpec:
    """Log-uniform object counts [1, 20000], spans [1 d, 10 yr] and frame
    counts [1, 5000]."""
    rng = np.random.default_rng(seed)
    lu = lambda lo, hi: np.exp(rng.uniform(math.log(lo), math.log(hi), n_jobs))
    return JobSpec(np.maximum(1, np.round(lu(1, max_obj))).astype(np.int64),
                   lu(1.0, max_span),
                   np.maximum(1, np.round(lu(1, max_frames))).astype(np.int64))


def batched_jobs(seed: int = 5, n_jobs: int = 4096, max_obj: int = 20_000, max_span: float = 3652.5,
                 max_frames: int = 5000, neo_frac: float = 0.05, width_deg: float = 1.5,
                 targeted_frac: float = 0.5, max_t0: float = 16.0):
    """Independent propagation + field-of-view jobs of uneven size: for
    each job, log-uniform body count, span and frame count (as in
    batched_job_specs), a start epoch uniform in [0, max_t0]; bodies drawn
    as in survey_case (main belt plus NEO-like); frames as in tiny_case
    over the job's span, a fraction of them aimed at the job's own bodies.
    Returns (ephemeris covering every job, [(x0 [n, 6], t0, Frames)])."""
    spec = batched_job_specs(seed, n_jobs, max_obj, max_span, max_frames)
    rng = np.random.default_rng(seed + 1000)
    model = PlanetModel.make()
    t0s = np.round(rng.uniform(0.0, max_t0, n_jobs), 3)
    end = float((t0s + spec.span).max())
    eph = make_ephemeris(model, -8.0, int(math.ceil((end + 24.0) / SEG_DAYS)))
    jobs = []
    for k in range(n_jobs):
        n = int(spec.n_obj[k])
        t0 = float(t0s[k])
        span = float(spec.span[k])
        n_neo = int(rng.binomial(n, neo_frac))
        el = np.concatenate([main_belt_elements(rng, n - n_neo), neo_elements(rng, n_neo)])
        x0 = bodies_from_elements(model, el, t0)
        nf = int(spec.n_frames[k])
        n_tg = int(round(targeted_frac * nf))
        parts = []
        if nf - n_tg:
            parts.append(frames_tiny(rng, model, nf - n_tg, t0, span, width_deg))
        if n_tg:
            parts.append(frames_targeted(rng, model, el, t0, span, n_tg, width_deg))
        fr = Frames.concat(parts) if len(parts) > 1 else parts[0]
        fr = fr.subset(np.argsort(fr.t, kind="stable"))
        jobs.append((x0, t0, fr))
    return eph, jobs
