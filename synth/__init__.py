"""Seeded synthetic inputs for the VESIS hot path.

This module only *draws* inputs: atom positions and per-atom parameters,
grid sizes and model constants.  It holds none of the method's arithmetic
(no densities, no energies, no flips) and is the only code shared by the
HIP path, the CPU oracle, the tests and the benchmark.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), used as a
counter-based stream: output k of stream ``seed`` is the SplitMix64 mix of
``seed + (k + 1) * 0x9E3779B97F4A7C15``.  Uniform doubles are
``(z >> 11) * 2**-53``.  Only +, -, *, / and sqrt (all correctly rounded in
IEEE-754) touch the drawn numbers, so every platform produces the same bits.

Units are nm, kJ/mol and elementary charges unless a workload says
otherwise.  The model constants follow the paper's parameter table
(Table "Model parameters": rho_w = 0.0333 per cubic angstrom, gamma_0 =
0.174, eps_m = 1, eps_w = 80); the surface tension is taken as 0.174
kJ/mol per square angstrom, i.e. 17.4 kJ mol^-1 nm^-2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_TWO53 = 1.0 / 9007199254740992.0

# Coulomb constant 1/(4 pi eps0) in kJ mol^-1 nm e^-2 (CODATA-derived value
# used by common MD packages).
COULOMB_K_NM_KJMOL = 138.935458
# k_B T at 298 K in kJ/mol, for the paper-units (angstrom, k_B T) workloads.
KBT_298_KJMOL = 0.0083144626 * 298.0


class SplitMix64:
    """Counter-based SplitMix64 stream (see module docstring)."""

    def __init__(self, seed: int):
        self.seed = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        self.count = 0

    def u64(self, m: int) -> np.ndarray:
        k = np.arange(self.count + 1, self.count + 1 + m, dtype=np.uint64)
        self.count += m
        with np.errstate(over="ignore"):
            z = self.seed + k * _GOLDEN
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        return z

    def uniform(self, m: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        u = (self.u64(m) >> np.uint64(11)).astype(np.float64) * _TWO53
        return lo + (hi - lo) * u


@dataclass
class Params:
    """Model constants (one consistent unit system)."""

    rho_w: float = 33.3            # solvent number density
    gamma0: float = 17.4           # surface tension
    eps_m: float = 1.0             # solute relative permittivity
    eps_w: float = 80.0            # solvent relative permittivity
    coulomb_k: float = COULOMB_K_NM_KJMOL   # 1/(4 pi eps0)
    rho_s: float = 3.0             # kernel radius delta over cell size h
    r2_min: float = 1.0e-6         # floor on squared atom-cell distance
    far_nf: int = 32               # far-field face nodes per axis
    far_ntau: int = 16             # far-field radial nodes


def paper_units_params() -> Params:
    """Constants in the paper's own units (angstrom, k_B T at 298 K)."""
    return Params(rho_w=0.0333, gamma0=0.174, eps_m=1.0, eps_w=80.0,
                  coulomb_k=COULOMB_K_NM_KJMOL * 10.0 / KBT_298_KJMOL,
                  rho_s=3.0, r2_min=1.0e-4)


@dataclass
class Workload:
    name: str
    n: int
    h: float
    center: np.ndarray
    xyz: np.ndarray
    q: np.ndarray
    sigma: np.ndarray
    eps: np.ndarray
    params: Params
    init_mode: str = "tight"       # "loose" or "tight"
    init_param: float = 1.0        # loose: sphere radius; tight: d_i = param * sigma_i
    precision: int = 32
    bonds: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    bond_r0: np.ndarray = field(default_factory=lambda: np.zeros(0))
    bond_k: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def natoms(self) -> int:
        return int(self.xyz.shape[0])


def _unit_vectors(rng: SplitMix64, m: int) -> np.ndarray:
    """m directions, uniform on the sphere, by rejection in the cube."""
    out = []
    while len(out) < m:
        v = rng.uniform(6 * m, -1.0, 1.0).reshape(-1, 3)
        r2 = (v * v).sum(axis=1)
        ok = (r2 > 1e-4) & (r2 <= 1.0)
        v = v[ok] / np.sqrt(r2[ok])[:, None]
        out.extend(v)
    return np.asarray(out[:m])


_WALK = None


def _walk_lib():
    """The compiled walk (synth/walk.c), or None if it has not been built."""
    global _WALK
    if _WALK is None:
        import ctypes as C
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwalk.so")
        _WALK = False
        if os.path.exists(path):
            lib = C.CDLL(path)
            lib.synth_globule.argtypes = [C.c_int64, C.c_uint64, C.c_double, C.c_double,
                                          C.c_double, C.c_double, C.c_int, C.c_int, C.c_void_p]
            lib.synth_globule.restype = C.c_int
            _WALK = lib
    return _WALK or None


def globule(natoms: int, seed: int, bond: float = 0.15, min_sep: float = 0.30,
            min_sep2: float = 0.24, density: float = 35.0, trials: int = 200,
            backtrack: int = 10, compiled: bool = True) -> np.ndarray:
    """Seeded self-avoiding chain confined to a sphere ("protein-like globule").

    Uses the compiled walk of synth/walk.c when it has been built (the same
    draws and decisions, bit for bit; a CPU test checks this), else the
    Python walk below.
    """
    lib = _walk_lib() if compiled else None
    if lib is not None:
        pos = np.zeros((natoms, 3))
        rc = lib.synth_globule(natoms, seed & 0xFFFFFFFFFFFFFFFF, bond, min_sep, min_sep2,
                               density, trials, backtrack, pos.ctypes.data)
        if rc != 0:
            raise RuntimeError("globule walk did not finish")
        return pos - pos.mean(axis=0)
    return _globule_py(natoms, seed, bond, min_sep, min_sep2, density, trials, backtrack)


def _globule_py(natoms: int, seed: int, bond: float, min_sep: float, min_sep2: float,
                density: float, trials: int, backtrack: int) -> np.ndarray:
    """Seeded self-avoiding chain confined to a sphere ("protein-like globule").

    Consecutive atoms sit ``bond`` apart; atoms two apart keep ``min_sep2``,
    all others ``min_sep``.  The chain stays within a sphere holding
    ``density`` atoms per unit volume.  A step that finds no valid direction
    among ``trials`` draws discards the last ``backtrack`` atoms.
    """
    rng = SplitMix64(seed)
    rconf = (3.0 * natoms / (4.0 * math.pi * density)) ** (1.0 / 3.0)
    pos = np.zeros((natoms, 3))
    binw = min_sep
    bins: dict[tuple, list] = {}

    def key(p):
        return (int(math.floor(p[0] / binw)), int(math.floor(p[1] / binw)),
                int(math.floor(p[2] / binw)))

    def add(i):
        bins.setdefault(key(pos[i]), []).append(i)

    def remove(i):
        bins[key(pos[i])].remove(i)

    add(0)
    i = 1
    guard = 0
    ms2, ms22 = min_sep * min_sep, min_sep2 * min_sep2
    while i < natoms:
        guard += 1
        if guard > 200 * natoms:
            raise RuntimeError("globule walk did not finish")
        cands = pos[i - 1] + bond * _unit_vectors(rng, trials)
        placed = False
        for c in cands:
            if c @ c > rconf * rconf:
                continue
            kx, ky, kz = key(c)
            ok = True
            for ax in (kx - 1, kx, kx + 1):
                for ay in (ky - 1, ky, ky + 1):
                    for az in (kz - 1, kz, kz + 1):
                        for j in bins.get((ax, ay, az), ()):
                            if j >= i - 1:
                                continue
                            d = c - pos[j]
                            lim = ms22 if j == i - 2 else ms2
                            if d @ d < lim:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                pos[i] = c
                add(i)
                i += 1
                placed = True
                break
        if not placed:
            back = min(backtrack, i - 1)
            for j in range(i - 1, i - 1 - back, -1):
                remove(j)
            i -= back
    return pos - pos.mean(axis=0)


def atom_params(natoms: int, seed: int):
    """Per-atom sigma ~ U[0.30,0.40], eps ~ U[0.1,0.6], q ~ U[-0.4,0.4] (neutralised)."""
    rng = SplitMix64(seed ^ 0x5EED5EED)
    u = rng.uniform(3 * natoms).reshape(natoms, 3)
    sigma = 0.30 + 0.10 * u[:, 0]
    eps = 0.1 + 0.5 * u[:, 1]
    q = -0.4 + 0.8 * u[:, 2]
    q = q - q.mean()
    return sigma, eps, q


def chain_bonds(natoms: int, offset: int = 0, r0: float = 0.15, k: float = 1.0e5):
    ij = np.stack([np.arange(natoms - 1), np.arange(1, natoms)], axis=1) + offset
    return ij.astype(np.int32), np.full(natoms - 1, r0), np.full(natoms - 1, k)


@dataclass
class Topology:
    """Solute-solute terms beyond the bonds (Eq. "Gss"): bending triplets
    (i, j, k; vertex j) with theta0 (rad) and B (kJ mol^-1 rad^-2), torsion
    quadruples with C_0..C_6 (kJ/mol) and phases psi_0..psi_6 (0 or pi), and
    the non-bonded pairs: every pair not listed in ``exclusions``, with
    per-atom LJ parameters sigma_ss, eps_ss (None = the atoms' own)."""
    angles: np.ndarray
    theta0: np.ndarray
    k_angle: np.ndarray
    torsions: np.ndarray
    c: np.ndarray
    psi: np.ndarray
    nonbonded: bool = True
    sigma_ss: np.ndarray | None = None
    eps_ss: np.ndarray | None = None
    exclusions: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))


def chain_topology(chains, seed: int, nonbonded: bool = True, exclude: int = 2) -> Topology:
    """Bending triplets (i, i+1, i+2) and torsion quadruples (i .. i+3) along
    each chain (first atom, atom count) of ``chains``; theta0 ~ U[1.8, 2.0]
    rad, B ~ U[300, 500], C_0 ~ U[0, 1], C_1..C_3 ~ U[0, 1.5], C_4..C_6 ~
    U[0, 0.5]; psi_n = 0 for odd n and pi for even n (so that positive C_n
    have their minimum in the trans position).  Pairs at most ``exclude``
    bonds apart along a chain are excluded from the non-bonded terms."""
    rng = SplitMix64(seed ^ 0x70B010)
    ang, tor, exc = [], [], []
    for first, count in chains:
        idx = np.arange(first, first + count, dtype=np.int32)
        if count >= 3:
            ang.append(np.stack([idx[:-2], idx[1:-1], idx[2:]], axis=1))
        if count >= 4:
            tor.append(np.stack([idx[:-3], idx[1:-2], idx[2:-1], idx[3:]], axis=1))
        for d in range(1, exclude + 1):
            if count > d:
                exc.append(np.stack([idx[:-d], idx[d:]], axis=1))
    angles = np.concatenate(ang) if ang else np.zeros((0, 3), np.int32)
    torsions = np.concatenate(tor) if tor else np.zeros((0, 4), np.int32)
    na, nt = len(angles), len(torsions)
    u = rng.uniform(2 * na).reshape(na, 2) if na else np.zeros((0, 2))
    theta0 = 1.8 + 0.2 * u[:, 0]
    k_angle = 300.0 + 200.0 * u[:, 1]
    scale = np.array([1.0, 1.5, 1.5, 1.5, 0.5, 0.5, 0.5])
    c = (rng.uniform(7 * nt).reshape(nt, 7) * scale) if nt else np.zeros((0, 7))
    psi = np.tile(np.array([math.pi if n % 2 == 0 else 0.0 for n in range(7)]), (nt, 1))
    excl = np.concatenate(exc).astype(np.int32) if exc else np.zeros((0, 2), np.int32)
    return Topology(angles=angles.astype(np.int32), theta0=theta0, k_angle=k_angle,
                    torsions=torsions.astype(np.int32), c=c, psi=psi, nonbonded=nonbonded,
                    exclusions=excl)


# ---------------------------------------------------------------- workloads

def single_atom(n: int = 64) -> Workload:
    """One uncharged LJ atom (sigma 0.35 nm, eps 0.65 kJ/mol) at the centre of
    the box [-1.5, 1.5]^3 nm; loose initial sphere of radius 1.2 nm; FP64."""
    return Workload(name=f"single_atom_{n}", n=n, h=3.0 / n, center=np.zeros(3),
                    xyz=np.zeros((1, 3)), q=np.zeros(1), sigma=np.array([0.35]),
                    eps=np.array([0.65]), params=Params(), init_mode="loose",
                    init_param=1.2, precision=64)


def chain_1000(n: int = 128, h: float = 0.05, init_mode: str = "tight") -> Workload:
    """1,000-atom seeded globule on a 128^3 grid, spacing 0.05 nm (box 6.4 nm)."""
    xyz = globule(1000, seed=2000)
    sigma, eps, q = atom_params(1000, seed=2000)
    ij, r0, k = chain_bonds(1000)
    return Workload(name=f"chain1000_{n}", n=n, h=h, center=np.zeros(3), xyz=xyz,
                    q=q, sigma=sigma, eps=eps, params=Params(), init_mode=init_mode,
                    init_param=1.0 if init_mode == "tight" else 2.6, bonds=ij,
                    bond_r0=r0, bond_k=k)


def two_globules(n: int = 256, h: float = 0.05, natoms_each: int = 5000,
                 gap: float = 1.5) -> Workload:
    """Two seeded globules whose bounding spheres are ``gap`` apart, placed
    along the box diagonal, on an n^3 grid of spacing h (256^3, 0.05 nm:
    12.8 nm box, 10,000 atoms)."""
    a = globule(natoms_each, seed=3000)
    b = globule(natoms_each, seed=3001)
    ra = float(np.sqrt((a * a).sum(1)).max())
    rb = float(np.sqrt((b * b).sum(1)).max())
    s = (ra + rb + gap) / 2.0
    u = np.ones(3) / math.sqrt(3.0)
    xyz = np.concatenate([a - s * u, b + s * u])
    sa, ea, qa = atom_params(natoms_each, seed=3000)
    sb, eb, qb = atom_params(natoms_each, seed=3001)
    ij1, r01, k1 = chain_bonds(natoms_each)
    ij2, r02, k2 = chain_bonds(natoms_each, offset=natoms_each)
    return Workload(name=f"two_globules_{natoms_each}x2_{n}", n=n, h=h,
                    center=np.zeros(3), xyz=xyz, q=np.concatenate([qa, qb]),
                    sigma=np.concatenate([sa, sb]), eps=np.concatenate([ea, eb]),
                    params=Params(), init_mode="tight", init_param=1.0,
                    bonds=np.concatenate([ij1, ij2]), bond_r0=np.concatenate([r01, r02]),
                    bond_k=np.concatenate([k1, k2]))


def batch_conformations(count: int = 64, h: float = 0.05, seed0: int = 4000):
    """Molecules with atom counts log-uniform in [200, 3000] and cubic grids
    between 64^3 and 160^3 (multiples of 16) sized to the molecule."""
    rng = SplitMix64(seed0)
    u = rng.uniform(count)
    out = []
    for m in range(count):
        na = int(round(math.exp(math.log(200.0) + u[m] * (math.log(3000.0) - math.log(200.0)))))
        xyz = globule(na, seed=seed0 + 1 + m)
        sigma, eps, q = atom_params(na, seed=seed0 + 1 + m)
        rb = float(np.sqrt((xyz * xyz).sum(1)).max())
        nm = 16 * math.ceil(2.0 * (rb + 0.6) / (16 * h))
        nm = max(64, min(160, nm))
        out.append(Workload(name=f"batch{m}", n=nm, h=h, center=np.zeros(3), xyz=xyz,
                            q=q, sigma=sigma, eps=eps, params=Params()))
    return out


def random_small(n: int, natoms: int, seed: int, h: float = 0.05, charged: bool = True,
                 spread: float | None = None) -> Workload:
    """Small random molecule for parity tests: atoms uniform in a ball well
    inside the box, the usual parameter distributions."""
    rng = SplitMix64(seed)
    L = n * h / 2.0
    rad = spread if spread is not None else 0.45 * L
    pts = []
    while len(pts) < natoms:
        v = rng.uniform(3, -1.0, 1.0)
        if v @ v <= 1.0:
            pts.append(v * rad)
    xyz = np.asarray(pts)
    sigma, eps, q = atom_params(natoms, seed)
    if not charged:
        q = np.zeros(natoms)
    return Workload(name=f"random{natoms}_{n}_s{seed}", n=n, h=h, center=np.zeros(3),
                    xyz=xyz, q=q, sigma=sigma, eps=eps, params=Params())


def conv_weights(specs, head_channels: int, seed: int = 0):
    """He-uniform weights for 3x3x3 convolutions, drawn from the SplitMix64
    stream: {name: (w (27, cout, cin) float32, zero bias)} for each
    (name, cin, cout) in specs, plus "head": (w (head_channels,), zero bias)."""
    rng = SplitMix64(seed)
    out = {}
    for name, cin, cout in specs:
        a = math.sqrt(6.0 / (27 * cin))
        w = rng.uniform(27 * cout * cin, -a, a).astype(np.float32).reshape(27, cout, cin)
        out[name] = (w, np.zeros(cout, np.float32))
    a = math.sqrt(6.0 / head_channels)
    out["head"] = (rng.uniform(head_channels, -a, a).astype(np.float32), np.zeros(1, np.float32))
    return out


def warm_start_set(count: int, n: int = 128, h: float = 0.05, seed0: int = 5000):
    """Molecules for the learned warm start: globules with atom counts
    log-uniform in [300, 1500] on an n^3 grid of spacing h (the 1,000-atom
    chain workload's generator and grid)."""
    rng = SplitMix64(seed0)
    u = rng.uniform(count)
    out = []
    for m in range(count):
        na = int(round(math.exp(math.log(300.0) + u[m] * (math.log(1500.0) - math.log(300.0)))))
        xyz = globule(na, seed=seed0 + 1 + m)
        sigma, eps, q = atom_params(na, seed=seed0 + 1 + m)
        out.append(Workload(name=f"warm{m}", n=n, h=h, center=np.zeros(3), xyz=xyz, q=q,
                            sigma=sigma, eps=eps, params=Params()))
    return out
