"""Seeded synthetic workloads for the Fisher/SNR path.

This module only *draws* inputs: event parameters, detector sites and
frequency-grid descriptors, with the shapes and distributions of the
compact-binary catalogues the method is run on.  It contains none of the
method's arithmetic (no waveform, no antenna pattern, no PSD evaluation);
both the GPU path and the CPU oracle read the same arrays from it.

Parameter order (the Fisher row order, with aligned spins given as
chi1z/chi2z and the two tidal deformabilities last):

    0 Mc [Msun, detector frame]   1 eta            2 dL [Gpc]
    3 theta [rad]                 4 phi [rad]      5 iota [rad]
    6 psi [rad]                   7 tcoal [GMST days; Fisher column per s]
    8 Phicoal [rad]               9 chi1z          10 chi2z
    11 Lambda1                    12 Lambda2

Units follow the paper's parameter table (sec. 2.1, Table 1).  The sky
angles are theta = pi/2 - dec and phi = RA.  Masses are ordered m1 >= m2,
so chi1z and Lambda1 belong to the heavier body.

Grid lengths of the BNS catalogue are set by the total mass, i.e. by the
cut frequency that scales as 1/M: n_e = 2000 + floor(18000 u_e) with
u_e = ln(4.4 Msun / M_e) / ln 2 for M_e in [2.2, 4.4] Msun.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

NPAR_MAX = 13
PAR_NAMES = ("Mc", "eta", "dL", "theta", "phi", "iota", "psi", "tcoal",
             "Phicoal", "chi1z", "chi2z", "Lambda1", "Lambda2")
PAR = {n: i for i, n in enumerate(PAR_NAMES)}

SHAPE_L = 0
SHAPE_T = 1

PSD_ANALYTIC, PSD_TABLE, ASD_TABLE = 0, 1, 2

FLAG_EARTH_ROT = 1
FLAG_TIDAL = 2
FLAG_ECCENTRIC = 8

DEG = math.pi / 180.0

# Detector sites of the paper's Table 2 (lat, lon, gamma in degrees; zeta; shape).
SITES = {
    "H1": (46.5, -119.4, 171.0, 90.0, SHAPE_L),
    "L1": (30.6, -90.8, 242.7, 90.0, SHAPE_L),
    "Virgo": (43.6, 10.5, 115.6, 90.0, SHAPE_L),
    "KAGRA": (36.4, 137.3, 15.4, 90.0, SHAPE_L),
    "LIGOI": (19.6, 77.0, 287.4, 90.0, SHAPE_L),
    "ETS": (40.5, 9.4, 0.0, 60.0, SHAPE_T),
    "ETMR": (50.7, 5.9, 0.0, 60.0, SHAPE_T),
    "CE1Id": (43.8, -112.8, -45.0, 90.0, SHAPE_L),
    "CE2NM": (33.2, -106.5, -105.0, 90.0, SHAPE_L),
    "CE2NSW": (-34.0, 145.0, 0.0, 90.0, SHAPE_L),
}

SEEDS = {"bbh100": 2207069100, "bns1e4": 2207069101, "mixed1e4": 2207069103,
         "catalog1e6": 2207069104}


@dataclass
class Site:
    """One detector site in radians. A triangle (shape T) is three
    co-located 60-degree interferometers; gamma is its first arm's angle
    from local East, for an L it is the arm bisector's angle."""
    lat: float
    lon: float
    gamma: float
    zeta: float
    shape: int
    S0: float = 1e-49      # analytic PSD scale [1/Hz]; the scale of a sampled curve
    f0: float = 215.0      # analytic PSD knee [Hz]
    psd_kind: int = PSD_ANALYTIC     # or PSD_TABLE / ASD_TABLE: a sampled noise curve
    psd_f: np.ndarray | None = None  # float64 [m], increasing [Hz] (sampled curves)
    psd_S: np.ndarray | None = None  # float64 [m], the PSD [1/Hz] or ASD [1/sqrt(Hz)] there

    @property
    def n_ifo(self) -> int:
        return 3 if self.shape == SHAPE_T else 1

    def with_curve(self, f, S, asd=False, scale=1.0) -> "Site":
        """The same site with a sampled noise curve (the paper's psd_path
        file, with is_ASD): frequencies f and values S, scaled by `scale`."""
        import dataclasses
        return dataclasses.replace(self, S0=float(scale), psd_kind=ASD_TABLE if asd else PSD_TABLE,
                                   psd_f=np.ascontiguousarray(f, dtype=np.float64),
                                   psd_S=np.ascontiguousarray(S, dtype=np.float64))


@dataclass
class Workload:
    name: str
    par: np.ndarray              # float64 [13][N]
    sites: list
    fmin: np.ndarray             # float64 [N]
    npts: np.ndarray             # int32 [N]
    fmax: np.ndarray | None      # float64 [N] or None: grid ends at each event's cut frequency
    flags: int
    npar: int                    # 11 (no tides) or 13
    tc_s: np.ndarray | None = None
    meta: dict = field(default_factory=dict)
    active: np.ndarray | None = None   # uint8 [n_ifo][N] or None: interferometers on (duty factor)
    par_mask: np.ndarray | None = None  # uint32 [N] or None: each event's Fisher rows (bit r: row r)
    grid_f: np.ndarray | None = None    # float64 [sum npts] or None: explicit grids, event e's
                                        # frequencies at its exclusive prefix sum of npts
    ecc: np.ndarray | None = None       # float64 [N] or None: e0 (with FLAG_ECCENTRIC)
    f_ref_ecc: np.ndarray | None = None  # float64 [N] or None: reference frequency of e0
                                         # (None: each grid's first frequency)

    @property
    def n(self) -> int:
        return self.par.shape[1]

    @property
    def n_ifo(self) -> int:
        return sum(s.n_ifo for s in self.sites)

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx)
        return Workload(self.name + "[sub]", np.ascontiguousarray(self.par[:, idx]),
                        list(self.sites), self.fmin[idx].copy(), self.npts[idx].copy(),
                        None if self.fmax is None else self.fmax[idx].copy(),
                        self.flags, self.npar,
                        None if self.tc_s is None else self.tc_s[idx].copy(),
                        {k: (v[idx] if isinstance(v, np.ndarray) and v.shape[:1] == (self.n,) else v)
                         for k, v in self.meta.items()},
                        None if self.active is None else np.ascontiguousarray(self.active[:, idx]),
                        None if self.par_mask is None else self.par_mask[idx].copy(),
                        None if self.grid_f is None else np.concatenate(
                            [self.event_grid(int(e)) for e in idx]),
                        None if self.ecc is None else self.ecc[idx].copy(),
                        None if self.f_ref_ecc is None else self.f_ref_ecc[idx].copy())

    def with_duty_factor(self, duty, seed: int) -> "Workload":
        """A copy whose interferometers are each on for an event with
        probability duty (a number, or one per site; a triangle's three
        interferometers are drawn separately): uniform draws of a seeded
        PCG64, interferometer by interferometer, compared with the factor."""
        w = self.subset(np.arange(self.n))
        w.name = self.name + f"[duty {duty}]"
        per_site = np.broadcast_to(np.asarray(duty, dtype=np.float64), (len(self.sites),))
        fac = np.concatenate([np.full(s.n_ifo, per_site[i]) for i, s in enumerate(self.sites)])
        rng = np.random.default_rng(seed)
        u = rng.random((len(fac), self.n))
        w.active = (u < fac[:, None]).astype(np.uint8)
        return w

    def with_par_masks(self) -> "Workload":
        """A copy in which each event's Fisher matrix has the parameters of
        its kind (meta["kind"]): black-hole pairs without deformabilities (11
        rows), neutron-star pairs with both (13), NS-BH pairs with the
        neutron star's Lambda2 only (12; m1 >= m2, so body 2 is the star)."""
        w = self.subset(np.arange(self.n))
        w.name = self.name + "[par masks]"
        w.par_mask = population_masks(self.meta["kind"], self.npar)
        return w

    def with_eccentricity(self, e0, f_ref=None) -> "Workload":
        """A copy with orbital eccentricities e0 [N] (or one value for all),
        given at the reference frequencies f_ref [N] (None: each grid's first
        frequency); the Fisher matrices gain e0 as their last row."""
        w = self.subset(np.arange(self.n))
        w.name = self.name + "[eccentric]"
        w.ecc = np.broadcast_to(np.asarray(e0, dtype=np.float64), (self.n,)).copy()
        w.f_ref_ecc = None if f_ref is None else np.broadcast_to(
            np.asarray(f_ref, dtype=np.float64), (self.n,)).copy()
        if not self.flags & FLAG_ECCENTRIC:
            w.flags = self.flags | FLAG_ECCENTRIC
            w.npar = self.npar + 1
        return w

    def grid_offsets(self) -> np.ndarray:
        """int64 [N]: first column of each event's explicit grid in grid_f."""
        return np.concatenate([[0], np.cumsum(self.npts, dtype=np.int64)[:-1]])

    def event_grid(self, e: int) -> np.ndarray:
        o = int(self.grid_offsets()[e])
        return self.grid_f[o:o + int(self.npts[e])]

    def with_grid_f(self, freqs) -> "Workload":
        """A copy on explicit grids: freqs is a list of N increasing float64
        arrays (event e's frequencies, at least two each); npts follows."""
        w = self.subset(np.arange(self.n))
        w.name = self.name + "[explicit grids]"
        fs = [np.ascontiguousarray(f, dtype=np.float64) for f in freqs]
        assert len(fs) == self.n and all(len(f) >= 2 for f in fs)
        w.npts = np.array([len(f) for f in fs], dtype=np.int32)
        w.grid_f = np.concatenate(fs)
        return w

    def with_npts(self, n: int) -> "Workload":
        w = self.subset(np.arange(self.n))
        w.npts = np.full(self.n, n, dtype=np.int32)
        w.grid_f = None
        return w

    def site_array(self) -> np.ndarray:
        """[n_site][7] = lat, lon, gamma, zeta, shape, S0, f0."""
        return np.array([[s.lat, s.lon, s.gamma, s.zeta, float(s.shape), s.S0, s.f0]
                         for s in self.sites], dtype=np.float64).reshape(-1, 7)


def site(name: str, S0: float = 1e-49, f0: float = 215.0) -> Site:
    lat, lon, gam, zeta, shape = SITES[name]
    return Site(lat * DEG, lon * DEG, gam * DEG, zeta * DEG, shape, S0, f0)


def _masses_to_mc_eta(m1, m2):
    m = m1 + m2
    eta = m1 * m2 / (m * m)
    mc = m * eta ** 0.6
    return mc, eta


def _isotropic(rng, n, par):
    par[3] = np.arccos(rng.uniform(-1.0, 1.0, n))
    par[4] = rng.uniform(0.0, 2 * np.pi, n)
    par[5] = np.arccos(rng.uniform(-1.0, 1.0, n))
    par[6] = rng.uniform(0.0, np.pi, n)
    par[7] = rng.uniform(0.0, 1.0, n)
    par[8] = rng.uniform(0.0, 2 * np.pi, n)


def _random_sites(rng, shapes):
    out = []
    for shape in shapes:
        lat = float(np.arcsin(rng.uniform(-1.0, 1.0)))
        lon = float(rng.uniform(-np.pi, np.pi))
        gam = float(rng.uniform(0.0, np.pi))
        s0 = float(10.0 ** rng.uniform(-51.0, -49.0))
        f0 = float(rng.uniform(100.0, 300.0))
        zeta = np.pi / 3 if shape == SHAPE_T else np.pi / 2
        out.append(Site(lat, lon, gam, zeta, shape, s0, f0))
    return out


def bbh100(n: int = 100, npts: int = 1000, seed: int = SEEDS["bbh100"]) -> Workload:
    """100 BBH events, one L-shaped detector at the H1 site, no Earth
    rotation, analytic PSD with S0 = 1e-49 /Hz and a 215 Hz knee, 1000
    log-spaced points from 10 Hz to the cut frequency, 11 parameters."""
    rng = np.random.default_rng(seed)
    par = np.zeros((NPAR_MAX, n))
    par[0] = rng.uniform(5.0, 40.0, n)
    par[1] = rng.uniform(0.1, 0.25, n)
    par[2] = rng.uniform(100.0, 3000.0, n) / 1000.0
    _isotropic(rng, n, par)
    par[9] = rng.uniform(-0.5, 0.5, n)
    par[10] = rng.uniform(-0.5, 0.5, n)
    return Workload("bbh100", par, [site("H1")], np.full(n, 10.0),
                    np.full(n, npts, dtype=np.int32), None, 0, 11)


def bns_masses(rng, n):
    m = rng.uniform(1.1, 2.2, (2, n))
    m1 = np.maximum(m[0], m[1])
    m2 = np.minimum(m[0], m[1])
    return m1, m2


def bns1e4(n: int = 10000, seed: int = SEEDS["bns1e4"], nmin: int = 2000,
           nspan: int = 18000) -> Workload:
    """10^4 BNS events on a 3G-like network: one triangle (three 60-degree
    interferometers) and two L-shaped sites at seeded positions, each with
    its own analytic PSD scale and knee; Earth rotation on; tidal terms on
    (13 parameters); grids from 2 Hz to the cut frequency with 2000-20000
    log-spaced points set by the total mass."""
    rng = np.random.default_rng(seed)
    par = np.zeros((NPAR_MAX, n))
    m1, m2 = bns_masses(rng, n)
    par[0], par[1] = _masses_to_mc_eta(m1, m2)
    par[2] = rng.uniform(50.0, 2000.0, n) / 1000.0
    _isotropic(rng, n, par)
    par[9] = rng.uniform(-0.05, 0.05, n)
    par[10] = rng.uniform(-0.05, 0.05, n)
    par[11] = rng.uniform(0.0, 2000.0, n)
    par[12] = rng.uniform(0.0, 2000.0, n)
    sites = _random_sites(rng, [SHAPE_T, SHAPE_L, SHAPE_L])
    mtot = m1 + m2
    u = np.clip(np.log(4.4 / mtot) / np.log(2.0), 0.0, 1.0)
    npts = (nmin + np.floor(nspan * u)).astype(np.int32)
    return Workload("bns1e4", par, sites, np.full(n, 2.0), npts, None,
                    FLAG_EARTH_ROT | FLAG_TIDAL, 13, meta={"m1": m1, "m2": m2})


def _population(rng, n, fractions, bbh_mc):
    """Masses, spins, deformabilities and distances of a mixed BBH / BNS /
    NSBH population (kind 0 / 1 / 2 drawn with the given fractions)."""
    kind = rng.choice(3, n, p=np.asarray(fractions, dtype=np.float64) / np.sum(fractions))
    par = np.zeros((NPAR_MAX, n))
    m1, m2 = np.zeros(n), np.zeros(n)
    b = kind == 0
    mc = rng.uniform(bbh_mc[0], bbh_mc[1], n)
    eta = rng.uniform(0.1, 0.25, n)
    mt = mc * eta ** -0.6
    d = np.sqrt(np.maximum(1.0 - 4.0 * eta, 0.0))
    m1[b], m2[b] = 0.5 * mt[b] * (1 + d[b]), 0.5 * mt[b] * (1 - d[b])
    ns = kind == 1
    bm1, bm2 = bns_masses(rng, n)
    m1[ns], m2[ns] = bm1[ns], bm2[ns]
    nb = kind == 2
    m1[nb], m2[nb] = rng.uniform(5.0, 20.0, n)[nb], rng.uniform(1.2, 2.0, n)[nb]
    par[0], par[1] = _masses_to_mc_eta(m1, m2)
    par[1] = np.minimum(par[1], 0.25)
    par[2] = np.where(kind == 1, rng.uniform(50.0, 2000.0, n), rng.uniform(100.0, 3000.0, n)) / 1000.0
    _isotropic(rng, n, par)
    big = rng.uniform(-0.5, 0.5, (2, n))
    small = rng.uniform(-0.05, 0.05, (2, n))
    par[9] = np.where(kind == 1, small[0], big[0])
    par[10] = np.where(kind == 0, big[1], small[1])
    lam = rng.uniform(0.0, 2000.0, (2, n))
    par[11] = np.where(kind == 1, lam[0], 0.0)
    par[12] = np.where(kind == 0, 0.0, lam[1])
    return par, kind, m1 + m2


MASK_BBH = (1 << 11) - 1                  # rows Mc ... chi2z
MASK_BNS = (1 << 13) - 1                  # and Lambda1, Lambda2
MASK_NSBH = MASK_BBH | (1 << 12)          # and Lambda2 only


def population_masks(kind, npar: int = 13) -> np.ndarray:
    """uint32 [N] Fisher-row sets of a population's kinds (0 BBH, 1 BNS,
    2 NSBH), restricted to npar rows."""
    kind = np.asarray(kind)
    m = np.select([kind == 0, kind == 1, kind == 2], [MASK_BBH, MASK_BNS, MASK_NSBH], MASK_BNS)
    return (m & ((1 << npar) - 1)).astype(np.uint32)


def _grid_lengths(mtot, nmin, nmax, m_lo, m_hi):
    """n = nmin + floor((nmax - nmin) u), u = ln(m_hi / M) / ln(m_hi / m_lo)
    clipped to [0, 1]: lighter systems, whose grids from the same fmin reach
    higher cut frequencies, get more points."""
    u = np.clip(np.log(m_hi / mtot) / np.log(m_hi / m_lo), 0.0, 1.0)
    return (nmin + np.floor((nmax - nmin) * u)).astype(np.int32)


# Grid lengths of the mixed populations: the heaviest system of the
# catalogue (Mc = 60 Msun at eta = 0.1, f_cut = 18.41 Hz) gets 500 points and
# the lightest neutron-star pair (2.2 Msun, f_cut = 1998.72 Hz) 20000.
M_GRID_HI = 60.0 * 0.1 ** -0.6
M_GRID_LO = 2.2


def mixed1e4(n: int = 10000, seed: int = SEEDS["mixed1e4"]) -> Workload:
    """10^4 events, 60% BBH (Mc 5-40 Msun, eta 0.1-0.25, spins up to 0.5;
    11 Fisher rows: no deformabilities) and 40% BNS (as the BNS catalogue,
    13 rows), on five L-shaped sites at seeded positions and orientations
    with their own analytic PSDs; Earth rotation and tidal terms on; grids
    from 2 Hz to the cut frequency with 500-20000 points set by the total
    mass as in the 10^6-event catalogue.  The detector-gradient workload."""
    rng = np.random.default_rng(seed)
    par, kind, mtot = _population(rng, n, (0.6, 0.4, 0.0), (5.0, 40.0))
    sites = _random_sites(rng, [SHAPE_L] * 5)
    npts = _grid_lengths(mtot, 500, 20000, M_GRID_LO, M_GRID_HI)
    return Workload("mixed1e4", par, sites, np.full(n, 2.0), npts, None,
                    FLAG_EARTH_ROT | FLAG_TIDAL, 13, meta={"kind": kind},
                    par_mask=population_masks(kind))


def catalog1e6(n: int = 1000000, seed: int = SEEDS["catalog1e6"]) -> Workload:
    """10^6 events: 60% BBH (Mc 5-60 Msun; 11 Fisher rows), 35% BNS (m
    1.1-2.2 Msun; 13 rows), 5% NSBH (m1 5-20, m2 1.2-2 Msun, Lambda1 = 0;
    12 rows, the black hole's deformability left out) on the BNS catalogue's
    network (the triangle and the two L sites of bns1e4), Earth rotation and
    tides on; grids from 2 Hz with 500-20000 points,
    n = 500 + floor(19500 u), u = ln(f_cut / 18.41 Hz) / ln(1998.72 / 18.41).
    The batched-catalogue workload (total points exceed 2^31)."""
    rng = np.random.default_rng(seed)
    par, kind, mtot = _population(rng, n, (0.60, 0.35, 0.05), (5.0, 60.0))
    sites = list(bns1e4().sites)
    npts = _grid_lengths(mtot, 500, 20000, M_GRID_LO, M_GRID_HI)
    return Workload("catalog1e6", par, sites, np.full(n, 2.0), npts, None,
                    FLAG_EARTH_ROT | FLAG_TIDAL, 13, meta={"kind": kind},
                    par_mask=population_masks(kind))


WORKLOADS = {"bbh100": bbh100, "bns1e4": bns1e4, "mixed1e4": mixed1e4, "catalog1e6": catalog1e6}
