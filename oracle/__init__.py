"""ctypes binding of the FP64 VESIS oracle (oracle/vesis_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke``
and by the benchmark's CPU-baseline leg, never by the product package.
It shares no code with the HIP path; both take their inputs from ``synth``.

Labels are int8 arrays of length n^3 in the order i + n (j + n k) (x fastest),
-1 for solute and +1 for solvent.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

_D = C.c_double
_I32 = C.c_int32
_I64 = C.c_int64
_P = C.c_void_p


class _Sys(C.Structure):
    _fields_ = [("n", _I32), ("far_nf", _I32), ("far_ntau", _I32), ("pad0", _I32),
                ("center", _D * 3), ("h", _D), ("na", _I64),
                ("xyz", _P), ("q", _P), ("sigma", _P), ("eps", _P),
                ("rho_w", _D), ("gamma0", _D), ("eps_m", _D), ("eps_w", _D),
                ("coulomb_k", _D), ("rho_s", _D), ("r2_min", _D), ("ss", _P)]


class _SS(C.Structure):
    _fields_ = [("nang", _I64), ("ang", _P), ("theta0", _P), ("kang", _P),
                ("ntor", _I64), ("tor", _P), ("tc", _P), ("tpsi", _P),
                ("nonbonded", _I32), ("pad", _I32), ("sigma_ss", _P), ("eps_ss", _P),
                ("nexcl", _I64), ("excl", _P)]


class SoluteTerms:
    """Solute-solute terms of Eq. "Gss" beyond bonds: bending triplets
    (i, j, k; vertex j), torsion quadruples with C_0..C_6 and psi_0..psi_6,
    and the non-bonded LJ + Coulomb pairs (all pairs minus `exclusions`)."""

    def __init__(self, angles=None, theta0=None, k_angle=None, torsions=None, c=None, psi=None,
                 nonbonded=False, sigma_ss=None, eps_ss=None, exclusions=None):
        def arr(a, shape, dt):
            return np.ascontiguousarray(np.zeros(shape) if a is None else a, dtype=dt).reshape(shape)
        na = 0 if angles is None else len(angles)
        nt = 0 if torsions is None else len(torsions)
        ne = 0 if exclusions is None else len(exclusions)
        self.angles = arr(angles, (na, 3), np.int32)
        self.theta0 = arr(theta0, (na,), np.float64)
        self.k_angle = arr(k_angle, (na,), np.float64)
        self.torsions = arr(torsions, (nt, 4), np.int32)
        self.c = arr(c, (nt, 7), np.float64)
        self.psi = arr(psi, (nt, 7), np.float64)
        self.nonbonded = bool(nonbonded)
        self.sigma_ss = None if sigma_ss is None else np.ascontiguousarray(sigma_ss, np.float64)
        self.eps_ss = None if eps_ss is None else np.ascontiguousarray(eps_ss, np.float64)
        self.exclusions = arr(exclusions, (ne, 2), np.int32)

    def struct(self, sigma, eps) -> _SS:
        t = _SS()
        t.nang, t.ang = len(self.angles), self.angles.ctypes.data
        t.theta0, t.kang = self.theta0.ctypes.data, self.k_angle.ctypes.data
        t.ntor, t.tor = len(self.torsions), self.torsions.ctypes.data
        t.tc, t.tpsi = self.c.ctypes.data, self.psi.ctypes.data
        t.nonbonded = int(self.nonbonded)
        self._sig = self.sigma_ss if self.sigma_ss is not None else sigma
        self._eps = self.eps_ss if self.eps_ss is not None else eps
        t.sigma_ss, t.eps_ss = self._sig.ctypes.data, self._eps.ctypes.data
        t.nexcl, t.excl = len(self.exclusions), self.exclusions.ctypes.data
        return t


class Mobility(C.Structure):
    """State of the adaptive-mobility descent (M, alpha, dt, ...)."""
    _fields_ = [("M", _D), ("alpha", _D), ("dt", _D), ("dG_frac", _D), ("M_min", _D),
                ("G_old", _D), ("N_cnt", _I32), ("N_cnt_max", _I32), ("k", _I32),
                ("max_retries", _I32)]


class StepInfo(C.Structure):
    _fields_ = [("accepted", _I32), ("retries", _I32), ("G_old", _D), ("G_new", _D),
                ("max_grad", _D), ("omega", _D)]


class RelaxOpts(C.Structure):
    _fields_ = [("max_iters", _I32), ("persist", _I32), ("max_sweeps", _I32), ("pad", _I32),
                ("tol_grad", _D), ("tol_energy", _D)]


class RelaxReport(C.Structure):
    _fields_ = [("iters", _I32), ("stop_reason", _I32), ("sweeps", _I32), ("retries", _I32),
                ("G_final", _D), ("max_grad", _D), ("dG_abs", _D), ("dG_rel", _D)]


ENERGY_KEYS = ("geom", "vdw_in", "vdw_far", "elec_in", "elec_far", "bond", "bend", "torsion",
               "vdw_ss", "elec_ss", "total")


def default_mobility(dt: float = 0.1) -> Mobility:
    return Mobility(M=1.0, alpha=2.0 ** -0.5, dt=dt, dG_frac=0.05, M_min=1e-12, G_old=0.0,
                    N_cnt=0, N_cnt_max=5, k=0, max_retries=200)


def set_threads(n: int):
    """Threads of the oracle's OpenMP loops (timing only)."""
    lib().orc_set_threads(int(n))


def lib():
    global _LIB
    if _LIB is None:
        # a test that plants a mistake in a copy of the oracle points this at
        # the mutated build
        path = os.environ.get("VESIS_ORACLE_LIB")
        if path is None:
            path = _build.LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
                _build.build()
        L = C.CDLL(path)
        sp = C.POINTER(_Sys)
        L.orc_C0.restype = _D
        L.orc_surface_prefactor.restype = _D
        L.orc_surface_prefactor.argtypes = [sp]
        L.orc_cfa_prefactor.restype = _D
        L.orc_cfa_prefactor.argtypes = [sp]
        L.orc_cell_center.argtypes = [sp, _I64, _P]
        L.orc_density_point.argtypes = [sp, _P, _P, _P, _P]
        L.orc_density_points.argtypes = [sp, _I64, _P, _P, _P, _P]
        L.orc_density_grid.argtypes = [sp, _P, _P, _P]
        L.orc_gauss_legendre.argtypes = [C.c_int, _P, _P]
        L.orc_far_nodes.argtypes = [sp, _P, _P]
        L.orc_far_nodes.restype = _I64
        L.orc_far_field.argtypes = [sp, _P]
        L.orc_geom_energy.argtypes = [sp, _P]
        L.orc_geom_energy.restype = _D
        L.orc_energy.argtypes = [sp, _P, _P, _P, _P, _P]
        L.orc_bond_energy.argtypes = [_I64, _P, _P, _P, _P]
        L.orc_bond_energy.restype = _D
        L.orc_ss_energy.argtypes = [sp, _P]
        L.orc_ss_gradient.argtypes = [sp, _P]
        L.orc_delta_e.argtypes = [sp, _P, _P, _I64]
        L.orc_delta_e.restype = _D
        L.orc_in_band.argtypes = [sp, _P, _I64]
        L.orc_in_band.restype = C.c_int
        L.orc_colours.argtypes = [sp]
        L.orc_colours.restype = C.c_int
        L.orc_colour_of.argtypes = [sp, _I64]
        L.orc_colour_of.restype = C.c_int
        L.orc_colour_pass.argtypes = [sp, _P, _P, C.c_int, _D, _P, _P, _P, _P, _I64, _P]
        L.orc_colour_pass.restype = _I64
        L.orc_band_size.argtypes = [sp, _P]
        L.orc_band_size.restype = _I64
        L.orc_minimize_colour.argtypes = [sp, _P, _P, C.c_int, _D, _P, _P, _P, _I64]
        L.orc_minimize_colour.restype = C.c_int
        L.orc_minimize_heap.argtypes = [sp, _P, _P, _I64, _P]
        L.orc_minimize_heap.restype = C.c_int
        L.orc_init_loose.argtypes = [sp, _D, _P]
        L.orc_init_tight.argtypes = [sp, _P, _P]
        L.orc_forces.argtypes = [sp, _P, _I64, _P, _P, _P, _P]
        L.orc_forces_subset.argtypes = [sp, _P, _P, _I64, _P, _I64, _P, _P, _P, _P]
        L.orc_total_energy.argtypes = [sp, _P, _I64, _P, _P, _P, _P]
        L.orc_total_energy.restype = _D
        L.orc_atom_step.argtypes = [sp, _P, _P, _P, _I64, _P, _P, _P, C.POINTER(Mobility),
                                    C.POINTER(StepInfo)]
        L.orc_atom_step.restype = C.c_int
        L.orc_relax.argtypes = [sp, _P, _P, _P, _I64, _P, _P, _P, C.POINTER(RelaxOpts),
                                C.POINTER(Mobility), C.POINTER(RelaxReport)]
        L.orc_relax.restype = C.c_int
        _LIB = L
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def C0() -> float:
    return lib().orc_C0()


def gauss_legendre(m: int):
    x = np.zeros(m)
    w = np.zeros(m)
    lib().orc_gauss_legendre(m, _ptr(x), _ptr(w))
    return x, w


class System:
    """One molecule on one grid, in the oracle's terms."""

    def __init__(self, n, h, center, xyz, q, sigma, eps, params, bonds=None, bond_r0=None,
                 bond_k=None, ss: SoluteTerms | None = None):
        self.n = int(n)
        self.h = float(h)
        self.center = np.ascontiguousarray(center, dtype=np.float64)
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        self.q = np.ascontiguousarray(q, dtype=np.float64)
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        self.eps = np.ascontiguousarray(eps, dtype=np.float64)
        self.params = params
        nb = 0 if bonds is None else len(bonds)
        self.bonds = np.ascontiguousarray(
            bonds if bonds is not None else np.zeros((0, 2)), dtype=np.int32).reshape(-1, 2)
        self.bond_r0 = np.ascontiguousarray(bond_r0 if nb else np.zeros(0), dtype=np.float64)
        self.bond_k = np.ascontiguousarray(bond_k if nb else np.zeros(0), dtype=np.float64)
        self.ss = ss
        self._rebuild()

    @classmethod
    def from_workload(cls, w, with_bonds: bool = False, ss: SoluteTerms | None = None):
        return cls(w.n, w.h, w.center, w.xyz, w.q, w.sigma, w.eps, w.params,
                   w.bonds if with_bonds else None, w.bond_r0 if with_bonds else None,
                   w.bond_k if with_bonds else None, ss)

    def _rebuild(self):
        p = self.params
        s = _Sys()
        s.n = self.n
        s.far_nf = int(p.far_nf)
        s.far_ntau = int(p.far_ntau)
        for d in range(3):
            s.center[d] = float(self.center[d])
        s.h = self.h
        s.na = self.xyz.shape[0]
        s.xyz = self.xyz.ctypes.data
        s.q = self.q.ctypes.data
        s.sigma = self.sigma.ctypes.data
        s.eps = self.eps.ctypes.data
        s.rho_w, s.gamma0, s.eps_m, s.eps_w = p.rho_w, p.gamma0, p.eps_m, p.eps_w
        s.coulomb_k, s.rho_s, s.r2_min = p.coulomb_k, p.rho_s, p.r2_min
        if self.ss is not None:
            self._ss = self.ss.struct(self.sigma, self.eps)
            s.ss = C.addressof(self._ss)
        self._s = s

    def with_positions(self, xyz):
        return System(self.n, self.h, self.center, xyz, self.q, self.sigma, self.eps,
                      self.params, self.bonds if len(self.bonds) else None, self.bond_r0,
                      self.bond_k, self.ss)

    @property
    def ncell(self) -> int:
        return self.n ** 3

    @property
    def sref(self):
        return C.byref(self._s)

    # ------------------------------------------------------------ queries
    def surface_prefactor(self) -> float:
        return lib().orc_surface_prefactor(self.sref)

    def cfa_prefactor(self) -> float:
        return lib().orc_cfa_prefactor(self.sref)

    def cell_center(self, idx: int) -> np.ndarray:
        x = np.zeros(3)
        lib().orc_cell_center(self.sref, int(idx), _ptr(x))
        return x

    def density_grid(self, efield: bool = False):
        m = self.ncell
        ulj = np.zeros(m)
        ucfa = np.zeros(m)
        e = np.zeros((m, 3)) if efield else None
        lib().orc_density_grid(self.sref, _ptr(ulj), _ptr(ucfa), _ptr(e) if efield else None)
        return (ulj, ucfa, e) if efield else (ulj, ucfa)

    def density_points(self, pts, efield: bool = False):
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        m = pts.shape[0]
        ulj = np.zeros(m)
        ucfa = np.zeros(m)
        e = np.zeros((m, 3)) if efield else None
        lib().orc_density_points(self.sref, m, _ptr(pts), _ptr(ulj), _ptr(ucfa),
                                 _ptr(e) if efield else None)
        return (ulj, ucfa, e) if efield else (ulj, ucfa)

    def far_nodes(self):
        m = 6 * self.params.far_nf ** 2 * self.params.far_ntau
        pts = np.zeros((m, 3))
        w = np.zeros(m)
        lib().orc_far_nodes(self.sref, _ptr(pts), _ptr(w))
        return pts, w

    def far_field(self):
        out = np.zeros(2)
        lib().orc_far_field(self.sref, _ptr(out))
        return float(out[0]), float(out[1])

    def geom_energy(self, phi) -> float:
        phi = np.ascontiguousarray(phi, dtype=np.int8)
        return lib().orc_geom_energy(self.sref, _ptr(phi))

    def energy(self, phi, ulj, ucfa, far):
        phi = np.ascontiguousarray(phi, dtype=np.int8)
        out = np.zeros(6)
        farr = np.asarray(far, dtype=np.float64)
        lib().orc_energy(self.sref, _ptr(phi), _ptr(np.ascontiguousarray(ulj)),
                         _ptr(np.ascontiguousarray(ucfa)), _ptr(farr), _ptr(out))
        return dict(geom=out[0], vdw_in=out[1], vdw_far=out[2], elec_in=out[3],
                    elec_far=out[4], total=out[5])

    def bond_energy(self, xyz=None) -> float:
        xyz = np.ascontiguousarray(self.xyz if xyz is None else xyz, dtype=np.float64)
        return lib().orc_bond_energy(len(self.bonds), _ptr(self.bonds), _ptr(self.bond_r0),
                                     _ptr(self.bond_k), _ptr(xyz))

    def delta_e(self, phi, u, j) -> float:
        return lib().orc_delta_e(self.sref, _ptr(phi), _ptr(u), int(j))

    def in_band(self, phi, j) -> bool:
        return bool(lib().orc_in_band(self.sref, _ptr(phi), int(j)))

    def band_size(self, phi) -> int:
        return lib().orc_band_size(self.sref, _ptr(np.ascontiguousarray(phi, np.int8)))

    def colours(self) -> int:
        return lib().orc_colours(self.sref)

    def colour_pass(self, phi, u, colour, tie_tol: float = 0.0):
        """In place on phi.  Returns (flips, candidates, sum of flipped dE)."""
        nc = np.zeros(1, np.int64)
        ds = np.zeros(1)
        nt = np.zeros(1, np.int64)
        f = lib().orc_colour_pass(self.sref, _ptr(phi), _ptr(u), int(colour), float(tie_tol),
                                  _ptr(nc), _ptr(ds), None, None, 0, _ptr(nt))
        return int(f), int(nc[0]), float(ds[0])

    def minimize_colour(self, phi, u, max_sweeps: int = 10000, tie_tol: float = 0.0,
                        tie_cap: int = 4096):
        """In place on phi.  Returns (status, stats dict, tie cells, tie dE)."""
        stats = np.zeros(6, np.int64)
        tl = np.zeros(tie_cap, np.int64)
        td = np.zeros(tie_cap)
        rc = lib().orc_minimize_colour(self.sref, _ptr(phi), _ptr(u), int(max_sweeps),
                                       float(tie_tol), _ptr(stats), _ptr(tl), _ptr(td), tie_cap)
        st = dict(sweeps=int(stats[0]), flips=int(stats[1]), converged=int(stats[2]),
                  ties=int(stats[3]), band=int(stats[4]), candidates=int(stats[5]))
        k = min(st["ties"], tie_cap)
        return rc, st, tl[:k].copy(), td[:k].copy()

    def minimize_heap(self, phi, u, max_flips: int = 1 << 40):
        stats = np.zeros(3, np.int64)
        rc = lib().orc_minimize_heap(self.sref, _ptr(phi), _ptr(u), int(max_flips), _ptr(stats))
        return rc, dict(flips=int(stats[0]), converged=int(stats[1]), band=int(stats[2]))

    def init_loose(self, R0: float) -> np.ndarray:
        phi = np.zeros(self.ncell, np.int8)
        lib().orc_init_loose(self.sref, float(R0), _ptr(phi))
        return phi

    def init_tight(self, d=None) -> np.ndarray:
        d = np.ascontiguousarray(self.sigma if d is None else d, dtype=np.float64)
        phi = np.zeros(self.ncell, np.int8)
        lib().orc_init_tight(self.sref, _ptr(d), _ptr(phi))
        return phi

    def forces(self, phi) -> np.ndarray:
        phi = np.ascontiguousarray(phi, dtype=np.int8)
        f = np.zeros((self.xyz.shape[0], 3))
        lib().orc_forces(self.sref, _ptr(phi), len(self.bonds), _ptr(self.bonds),
                         _ptr(self.bond_r0), _ptr(self.bond_k), _ptr(f))
        return f

    def forces_subset(self, phi, efield, sel) -> np.ndarray:
        """Forces on atoms `sel` given the grid field E (ncell x 3)."""
        phi = np.ascontiguousarray(phi, dtype=np.int8)
        e = np.ascontiguousarray(efield, dtype=np.float64)
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        f = np.zeros((len(sel), 3))
        lib().orc_forces_subset(self.sref, _ptr(phi), _ptr(e), len(sel), _ptr(sel),
                                len(self.bonds), _ptr(self.bonds), _ptr(self.bond_r0),
                                _ptr(self.bond_k), _ptr(f))
        return f

    def total_energy(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.int8)
        comps = np.zeros(11)
        lib().orc_total_energy(self.sref, _ptr(phi), len(self.bonds), _ptr(self.bonds),
                               _ptr(self.bond_r0), _ptr(self.bond_k), _ptr(comps))
        return dict(zip(ENERGY_KEYS, (float(v) for v in comps)))

    def ss_energy(self) -> dict:
        """Bending, torsion, solute-solute LJ and Coulomb energies."""
        out = np.zeros(4)
        lib().orc_ss_energy(self.sref, _ptr(out))
        return dict(bend=out[0], torsion=out[1], vdw_ss=out[2], elec_ss=out[3])

    def ss_gradient(self) -> np.ndarray:
        """Gradient (na x 3) of the bending, torsion and non-bonded terms."""
        g = np.zeros((self.xyz.shape[0], 3))
        lib().orc_ss_gradient(self.sref, _ptr(g))
        return g

    def atom_step(self, xyz, phi, mobility: Mobility, movable=None):
        """One adaptive-mobility step; xyz (na x 3) is updated in place."""
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        phi = np.ascontiguousarray(phi, dtype=np.int8)
        mv = None if movable is None else np.ascontiguousarray(movable, dtype=np.uint8)
        info = StepInfo()
        rc = lib().orc_atom_step(self.sref, _ptr(xyz), _ptr(phi),
                                 None if mv is None else _ptr(mv), len(self.bonds),
                                 _ptr(self.bonds), _ptr(self.bond_r0), _ptr(self.bond_k),
                                 C.byref(mobility), C.byref(info))
        return rc, xyz, info

    def relax(self, xyz, phi, opts: RelaxOpts, mobility: Mobility, movable=None):
        """Steps 2-5 of the algorithm; xyz and phi are updated in place."""
        mv = None if movable is None else np.ascontiguousarray(movable, dtype=np.uint8)
        rep = RelaxReport()
        rc = lib().orc_relax(self.sref, _ptr(xyz), _ptr(phi), None if mv is None else _ptr(mv),
                             len(self.bonds), _ptr(self.bonds), _ptr(self.bond_r0),
                             _ptr(self.bond_k), C.byref(opts), C.byref(mobility), C.byref(rep))
        return rc, rep
