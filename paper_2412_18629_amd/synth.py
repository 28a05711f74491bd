"""Seeded synthetic particle sets shaped like the paper's N-body snapshots.

The paper (Parallelization section) runs the halo finder on cosmological
N-body snapshots; none are available here, so this module builds stand-ins
with the same structure: a periodic box holding a uniform background plus
NFW haloes whose particle counts follow a power-law mass function, each host
carrying 0-3 NFW subhaloes (optionally nested several levels deep) that move
with a bulk velocity relative to their host.

This module holds only input generation; it contains none of the halo
finder's arithmetic and is shared by the oracle-side and the GPU-side tests.
All random draws come from one ``torch.Generator`` seeded per call, so the
arrays are a deterministic function of (config, seed, device).  The same
arrays are always handed to both the oracle and the HIP path.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import torch

# Gravitational constant in Mpc (km/s)^2 / Msun, critical density in
# (Msun/h) / (Mpc/h)^3, matter density parameter used for the particle mass.
G_MPC_KMS2_MSUN = 4.30091e-9
RHO_CRIT = 2.775e11
OMEGA_M = 0.3


@dataclass(frozen=True)
class SynthConfig:
    """Parameters of one synthetic workload."""

    name: str
    n: int                    # total particle count
    box: float                # periodic box side, Mpc/h
    bg_frac: float            # fraction of particles in the uniform background
    n_hosts: int              # number of host haloes
    m_lo: float               # host mass range (particles) of the power law
    m_hi: float
    slope: float = -1.9       # dn/dM ~ M^slope
    conc: tuple = (8.0, 12.0) # NFW concentration range
    n_sub_max: int = 3        # 0..n_sub_max subhaloes per (sub)halo
    sub_frac: tuple = (0.05, 0.15)   # subhalo mass / parent mass
    sub_offset: tuple = (0.3, 0.8)   # subhalo offset / parent r_vir
    sub_bulk: float = 200.0   # subhalo bulk speed relative to parent, km/s
    sub_depth: int = 1        # nesting depth of subhaloes
    sigma_bg: float = 50.0    # 1D velocity dispersion of the background
    host_bulk_sigma: float = 100.0  # 1D dispersion of host bulk velocities
    b: float = 0.28           # FoF linking parameter (fraction of mean spacing)
    f: float = 0.7            # phase-space linked fraction
    min_group: int = 10
    min_sub: int = 10

    @property
    def mean_spacing(self) -> float:
        side = round(self.n ** (1.0 / 3.0))
        cbrt = float(side) if side ** 3 == self.n else self.n ** (1.0 / 3.0)
        return self.box / cbrt

    @property
    def link_len(self) -> float:
        """b times the mean interparticle spacing, computed in fp64 and
        rounded once to fp32."""
        import numpy as np
        return float(np.float32(self.b * self.mean_spacing))


# The five workloads: a 32^3 CPU-checkable box, the 256^3 box, the 512^3 box
# (the headline size), and the 1024^3 single-process share with three levels
# of nested substructure.
CONFIGS = {
    "c32": SynthConfig("c32", 32 ** 3, 20.0, 0.30, 40, 50.0, 3000.0),
    "c256": SynthConfig("c256", 256 ** 3, 160.0, 0.30, 20000, 20.0, 2.0e5),
    "c512": SynthConfig("c512", 512 ** 3, 320.0, 0.10, 150000, 20.0, 2.0e6),
    "c1024": SynthConfig("c1024", 1024 ** 3, 640.0, 0.10, 1200000, 20.0, 1.0e7,
                         sub_depth=3),
}


def scaled(cfg: SynthConfig, n: int, name: str | None = None) -> SynthConfig:
    """Same generator at a different particle count and constant mean density.

    The box side scales as n^(1/3) and the host count as n; the mass range is
    kept.  Used for parity cases between the named workload sizes.
    """
    r = n / cfg.n
    d = asdict(cfg)
    d.update(name=name or f"{cfg.name}_n{n}", n=n, box=cfg.box * r ** (1.0 / 3.0),
             n_hosts=max(1, int(round(cfg.n_hosts * r))))
    return SynthConfig(**d)


def _uniform(g, shape, lo, hi, device):
    return lo + (hi - lo) * torch.rand(shape, generator=g, dtype=torch.float64, device=device)


def _unit_vectors(g, m, device):
    v = torch.randn((m, 3), generator=g, dtype=torch.float64, device=device)
    return v / v.norm(dim=1, keepdim=True).clamp_min(1e-300)


def _nfw_mu(x):
    return torch.log1p(x) - x / (1.0 + x)


def _nfw_radius(u, conc):
    """Solve mu(x)/mu(c) = u for x in [0, c] by bisection (fp64)."""
    target = u * _nfw_mu(conc)
    lo = torch.zeros_like(u)
    hi = conc.clone()
    for _ in range(48):
        mid = 0.5 * (lo + hi)
        below = _nfw_mu(mid) < target
        lo = torch.where(below, mid, lo)
        hi = torch.where(below, hi, mid)
    return 0.5 * (lo + hi)


def _power_law(g, m, lo, hi, slope, device):
    """Inverse-CDF draws from dn/dM ~ M^slope on [lo, hi]."""
    u = _uniform(g, (m,), 0.0, 1.0, device)
    e = slope + 1.0
    return (lo ** e + u * (hi ** e - lo ** e)) ** (1.0 / e)


def build_halo_catalog(cfg: SynthConfig, g, device):
    """Hosts and nested subhaloes: masses (particles), centres, bulk velocities.

    Mass budget reading: the stated host count, slope and mass range fix the
    shape of the mass function, but their expected total is well below the
    stated halo fraction of the box; all host masses are therefore multiplied
    by one common factor so that the haloes hold exactly (1 - bg_frac) * n
    particles.  Subhalo masses are carved out of their parent.
    """
    n_halo_target = int(round(cfg.n * (1.0 - cfg.bg_frac)))
    m_host = _power_law(g, cfg.n_hosts, cfg.m_lo, cfg.m_hi, cfg.slope, device)
    m_host = m_host * (n_halo_target / m_host.sum())
    centres = _uniform(g, (cfg.n_hosts, 3), 0.0, cfg.box, device)
    bulk = torch.randn((cfg.n_hosts, 3), generator=g, dtype=torch.float64,
                       device=device) * cfg.host_bulk_sigma
    level = torch.zeros(cfg.n_hosts, dtype=torch.int64, device=device)
    masses, cents, bulks, levels = [m_host], [centres], [bulk], [level]
    parent_m, parent_c, parent_v = m_host, centres, bulk
    remaining = [m_host.clone()]
    for depth in range(1, cfg.sub_depth + 1):
        npar = parent_m.numel()
        nsub = torch.randint(0, cfg.n_sub_max + 1, (npar,), generator=g, device=device)
        idx = torch.repeat_interleave(torch.arange(npar, device=device), nsub)
        m = idx.numel()
        frac = _uniform(g, (m,), cfg.sub_frac[0], cfg.sub_frac[1], device)
        sub_m = parent_m[idx] * frac
        rv_par = _rvir(parent_m[idx], cfg)
        off = _unit_vectors(g, m, device) * (_uniform(g, (m,), cfg.sub_offset[0],
                                                      cfg.sub_offset[1], device) * rv_par)[:, None]
        sub_c = parent_c[idx] + off
        sub_v = parent_v[idx] + _unit_vectors(g, m, device) * cfg.sub_bulk
        # carve the subhalo mass out of its parent
        carved = torch.zeros_like(parent_m).index_add_(0, idx, sub_m)
        remaining[-1] = remaining[-1] - carved
        masses.append(sub_m); cents.append(sub_c); bulks.append(sub_v)
        levels.append(torch.full((m,), depth, dtype=torch.int64, device=device))
        remaining.append(sub_m.clone())
        parent_m, parent_c, parent_v = sub_m, sub_c, sub_v
    own = torch.cat(remaining)           # particles each object owns itself
    total = torch.cat(masses)            # virial mass of each object (sets r_vir, sigma)
    return dict(own=own, mass=total, centre=torch.cat(cents), bulk=torch.cat(bulks),
                level=torch.cat(levels))


def _rvir(m, cfg: SynthConfig):
    nbar = cfg.n / cfg.box ** 3
    return (m / (4.0 / 3.0 * math.pi * 200.0 * nbar)) ** (1.0 / 3.0)


def _sigma1d(m, cfg: SynthConfig):
    lbar = cfg.box / cfg.n ** (1.0 / 3.0)
    m_p = OMEGA_M * RHO_CRIT * lbar ** 3
    vvir2 = G_MPC_KMS2_MSUN * m * m_p / _rvir(m, cfg)
    return torch.sqrt(vvir2 / 2.0)


def _integer_counts(own, total):
    """Round per-object particle counts so they sum to exactly ``total``."""
    fl = torch.floor(own.clamp_min(0.0))
    short = int(total - int(fl.sum().item()))
    if short > 0:
        frac = own - fl
        order = torch.argsort(frac, descending=True)
        add = torch.zeros_like(fl)
        add[order[:short]] = 1.0
        fl = fl + add
    elif short < 0:
        order = torch.argsort(fl, descending=True)
        sub = torch.zeros_like(fl)
        sub[order[: -short]] = 1.0
        fl = fl - sub
    return fl.to(torch.int64)


# Boxes above this many particles draw their halo particles in chunks of
# CHUNK particles (fp32 output written as it goes) so the fp64 intermediates
# stay bounded; smaller boxes draw everything at once.  The draw order differs
# between the two paths, so each is its own deterministic workload.
CHUNKED_ABOVE = 1 << 28
CHUNK = 1 << 25


def _halo_particles_chunked(cfg, g, device, cat, counts, n_bg):
    n_obj = counts.numel()
    m = int(counts.sum().item())
    conc_obj = _uniform(g, (n_obj,), cfg.conc[0], cfg.conc[1], device)
    first = torch.cumsum(counts, 0) - counts          # first particle of each object
    pos32 = torch.empty((cfg.n, 3), dtype=torch.float32, device=device)
    vel32 = torch.empty((cfg.n, 3), dtype=torch.float32, device=device)
    for p0 in range(0, m, CHUNK):
        p1 = min(p0 + CHUNK, m)
        ids = torch.arange(p0, p1, device=device)
        obj = torch.searchsorted(first, ids, right=True) - 1
        mass = cat["mass"][obj]
        conc = conc_obj[obj]
        rv = _rvir(mass, cfg)
        x = _nfw_radius(_uniform(g, (p1 - p0,), 0.0, 1.0, device), conc)
        r = x * (rv / conc)
        pos = cat["centre"][obj] + _unit_vectors(g, p1 - p0, device) * r[:, None]
        pos32[p0:p1] = torch.remainder(pos, cfg.box).to(torch.float32)
        sig = _sigma1d(mass, cfg)
        vel = cat["bulk"][obj] + torch.randn((p1 - p0, 3), generator=g, dtype=torch.float64,
                                             device=device) * sig[:, None]
        vel32[p0:p1] = vel.to(torch.float32)
        del ids, obj, mass, conc, rv, x, r, pos, sig, vel
    for b0 in range(0, n_bg, CHUNK):
        b1 = min(b0 + CHUNK, n_bg)
        bpos = _uniform(g, (b1 - b0, 3), 0.0, cfg.box, device)
        pos32[m + b0:m + b1] = torch.remainder(bpos, cfg.box).to(torch.float32)
        bvel = torch.randn((b1 - b0, 3), generator=g, dtype=torch.float64,
                           device=device) * cfg.sigma_bg
        vel32[m + b0:m + b1] = bvel.to(torch.float32)
    return pos32, vel32, m


def generate(cfg: SynthConfig | str, seed: int = 0, device="cpu", return_meta=False):
    """Generate (x, y, z, vx, vy, vz) as fp32 tensors on ``device``.

    Positions lie in [0, box); velocities are in km/s.  Particle order is a
    random permutation, as in a shuffled snapshot.
    """
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    device = torch.device(device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    cat = build_halo_catalog(cfg, g, device)
    n_halo_target = int(round(cfg.n * (1.0 - cfg.bg_frac)))
    counts = _integer_counts(cat["own"], n_halo_target)
    n_bg = cfg.n - n_halo_target
    n_obj = counts.numel()
    if cfg.n > CHUNKED_ABOVE:
        pos32, vel32, m = _halo_particles_chunked(cfg, g, device, cat, counts, n_bg)
    else:
        obj = torch.repeat_interleave(torch.arange(n_obj, device=device), counts)
        m = obj.numel()
        mass = cat["mass"][obj]
        conc = _uniform(g, (n_obj,), cfg.conc[0], cfg.conc[1], device)[obj]
        rv = _rvir(mass, cfg)
        x = _nfw_radius(_uniform(g, (m,), 0.0, 1.0, device), conc)
        r = x * (rv / conc)
        pos = cat["centre"][obj] + _unit_vectors(g, m, device) * r[:, None]
        sig = _sigma1d(mass, cfg)
        vel = cat["bulk"][obj] + torch.randn((m, 3), generator=g, dtype=torch.float64,
                                             device=device) * sig[:, None]
        del mass, conc, rv, x, r, sig
        bpos = _uniform(g, (n_bg, 3), 0.0, cfg.box, device)
        bvel = torch.randn((n_bg, 3), generator=g, dtype=torch.float64,
                           device=device) * cfg.sigma_bg
        pos = torch.cat([pos, bpos])
        vel = torch.cat([vel, bvel])
        del bpos, bvel
        pos = torch.remainder(pos, cfg.box)
        pos32 = pos.to(torch.float32)
        del pos
        vel32 = vel.to(torch.float32)
        del vel
    box32 = torch.tensor(cfg.box, dtype=torch.float32, device=device)
    pos32 = torch.where(pos32 >= box32, torch.zeros_like(pos32), pos32)
    perm = torch.randperm(cfg.n, generator=g, device=device)
    pos32 = pos32[perm]
    vel32 = vel32[perm]
    out = tuple(t.contiguous() for t in (pos32[:, 0], pos32[:, 1], pos32[:, 2],
                                         vel32[:, 0], vel32[:, 1], vel32[:, 2]))
    if return_meta:
        meta = dict(config=cfg.name, n=cfg.n, box=cfg.box, seed=seed,
                    n_background=n_bg, n_objects=n_obj, n_hosts=cfg.n_hosts,
                    host_mass_min=float(counts[: cfg.n_hosts].min().item()) if cfg.n_hosts else 0,
                    host_mass_max=float(counts[: cfg.n_hosts].max().item()) if cfg.n_hosts else 0,
                    halo_fraction=float(m / cfg.n),
                    link_len=cfg.link_len)
        return out, meta
    return out


def random_uniform(n, box, seed=0, vel_sigma=100.0, device="cpu"):
    """Uniform positions in [0, box) and Gaussian velocities (test inputs)."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    pos = torch.rand((n, 3), generator=g, dtype=torch.float64, device=device) * box
    pos32 = pos.to(torch.float32)
    pos32 = torch.where(pos32 >= box, torch.zeros_like(pos32), pos32)
    vel = (torch.randn((n, 3), generator=g, dtype=torch.float64, device=device)
           * vel_sigma).to(torch.float32)
    return tuple(t.contiguous() for t in (pos32[:, 0], pos32[:, 1], pos32[:, 2],
                                         vel[:, 0], vel[:, 1], vel[:, 2]))
