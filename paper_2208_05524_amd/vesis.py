"""Python binding of libvesis (the MI355X VESIS hot path).

Argument marshalling only.  PyTorch provides the device workspace (one uint8
tensor) and the stream (the current torch stream of the device); every step
of the method runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (EnergyParts, MinStats, Mobility, Params, RelaxOpts, RelaxReport, StepInfo,
                   VesisError)

KERNEL_KINDS = {"density": 0, "far_field": 1, "init": 2, "flip": 3, "energy": 4, "force": 5,
                "other": 6, "solute": 7}


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def default_mobility(dt: float = 0.1) -> Mobility:
    """M = 1, alpha = 1/sqrt 2, N_cnt* = 5, delta G* = 5 % (the paper's choices)."""
    return Mobility(M=1.0, alpha=2.0 ** -0.5, dt=dt, dG_frac=0.05, M_min=1e-12, G_old=0.0,
                    N_cnt=0, N_cnt_max=5, k=0, max_retries=200)


class Context:
    """One molecule on one grid on one GPU."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        self._torch = torch
        self.lib = _lib.load()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        rc = self.lib.vesis_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise VesisError(rc, "vesis_create failed")
        self.h = h
        self.workspace = None
        self.n = 0
        self.natoms = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.vesis_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(0,)):
        if rc not in allow:
            msg = self.lib.vesis_last_error(self.h)
            raise VesisError(rc, msg.decode() if msg else "")
        return rc

    # ------------------------------------------------------------ set-up
    def set_params(self, p, precision: int = 32):
        prm = Params(rho_w=p.rho_w, gamma0=p.gamma0, eps_m=p.eps_m, eps_w=p.eps_w,
                     coulomb_k=p.coulomb_k, rho_s=p.rho_s, r2_min=p.r2_min, far_nf=p.far_nf,
                     far_ntau=p.far_ntau, precision=precision, reserved=0)
        self._check(self.lib.vesis_set_params(self.h, C.byref(prm)))

    def set_grid(self, n: int, center, h: float):
        c = _f64(center, (3,))
        self._check(self.lib.vesis_set_grid(self.h, int(n), _ptr(c), float(h)))
        self.n = int(n)

    def set_atoms(self, xyz, q, sigma, eps, movable=None):
        xyz = _f64(xyz, (-1, 3))
        na = xyz.shape[0]
        mv = None if movable is None else np.ascontiguousarray(movable, dtype=np.uint8)
        self._check(self.lib.vesis_set_atoms(self.h, na, _ptr(xyz), _ptr(_f64(q)),
                                             _ptr(_f64(sigma)), _ptr(_f64(eps)), _ptr(mv)))
        self.natoms = na

    def set_bonds(self, ij, r0, k):
        ij = np.ascontiguousarray(ij, dtype=np.int32).reshape(-1, 2)
        self._check(self.lib.vesis_set_bonds(self.h, ij.shape[0], _ptr(ij), _ptr(_f64(r0)),
                                             _ptr(_f64(k))))

    def set_angles(self, ijk, theta0, k):
        ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
        self._check(self.lib.vesis_set_angles(self.h, ijk.shape[0], _ptr(ijk),
                                              _ptr(_f64(theta0)), _ptr(_f64(k))))

    def set_torsions(self, ijkl, c, psi):
        ijkl = np.ascontiguousarray(ijkl, dtype=np.int32).reshape(-1, 4)
        self._check(self.lib.vesis_set_torsions(self.h, ijkl.shape[0], _ptr(ijkl),
                                                _ptr(_f64(c, (-1, 7))), _ptr(_f64(psi, (-1, 7)))))

    def set_nonbonded(self, enable=True, sigma_ss=None, eps_ss=None, exclusions=None):
        ex = np.ascontiguousarray(np.zeros((0, 2)) if exclusions is None else exclusions,
                                  dtype=np.int32).reshape(-1, 2)
        self._check(self.lib.vesis_set_nonbonded(
            self.h, int(bool(enable)), None if sigma_ss is None else _ptr(_f64(sigma_ss)),
            None if eps_ss is None else _ptr(_f64(eps_ss)), ex.shape[0], _ptr(ex)))

    def set_topology(self, top):
        """Bending, torsion and non-bonded terms of a ``synth.Topology``.
        Call before allocate_workspace (or allocate again afterwards)."""
        self.set_angles(top.angles, top.theta0, top.k_angle)
        self.set_torsions(top.torsions, top.c, top.psi)
        self.set_nonbonded(top.nonbonded, top.sigma_ss, top.eps_ss, top.exclusions)

    def set_positions(self, xyz):
        """Host array (n x 3) or a CUDA float64 tensor of n x 3 (device copy)."""
        t = self._torch
        if isinstance(xyz, t.Tensor):
            assert xyz.is_cuda and xyz.dtype == t.float64 and xyz.is_contiguous()
            self._check(self.lib.vesis_set_positions(self.h, C.c_void_p(xyz.data_ptr()), 1))
        else:
            a = _f64(xyz, (-1, 3))
            self._check(self.lib.vesis_set_positions(self.h, _ptr(a), 0))

    def positions(self) -> np.ndarray:
        out = np.zeros((self.natoms, 3))
        self._check(self.lib.vesis_get_positions(self.h, _ptr(out)))
        return out

    def workspace_size(self) -> int:
        n = C.c_size_t()
        self._check(self.lib.vesis_workspace_size(self.h, C.byref(n)))
        return int(n.value)

    def allocate_workspace(self):
        t = self._torch
        nbytes = self.workspace_size()
        self.workspace = t.empty(nbytes + 256, dtype=t.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self._check(self.lib.vesis_set_workspace(self.h, C.c_void_p(aligned), nbytes))
        return nbytes

    def setup(self, w, precision=None, with_bonds: bool = False, topology=None):
        """Params, grid, atoms (bonds, other solute-solute terms of a
        ``synth.Topology``) of a ``synth.Workload``, then workspace."""
        self.set_params(w.params, precision if precision is not None else w.precision)
        self.set_grid(w.n, w.center, w.h)
        self.set_atoms(w.xyz, w.q, w.sigma, w.eps)
        if with_bonds and len(w.bonds):
            self.set_bonds(w.bonds, w.bond_r0, w.bond_k)
        if topology is not None:
            self.set_topology(topology)
        self.allocate_workspace()
        return self

    # ------------------------------------------------------------ operations
    def init_labels(self, mode: str, param: float = 1.0, user=None):
        m = {"loose": 0, "tight": 1, "user": 2}[mode]
        u = None if user is None else np.ascontiguousarray(user, dtype=np.int8)
        self._check(self.lib.vesis_init_labels(self.h, m, float(param), _ptr(u)))

    def init_labels_logits(self, logits):
        """Labels from a CUDA float32 tensor of n^3 logits (solute where > 0)."""
        t = self._torch
        assert logits.is_cuda and logits.dtype == t.float32 and logits.numel() == self.n ** 3
        self._check(self.lib.vesis_init_labels_logits(self.h, C.c_void_p(logits.data_ptr())))

    def minimize(self, max_sweeps: int = 20000):
        st = MinStats()
        rc = self._check(self.lib.vesis_minimize_interface(self.h, int(max_sweeps), C.byref(st)),
                         allow=(0, 1))
        return rc, dict(sweeps=st.sweeps, converged=st.converged, flips=st.flips,
                        band=st.band_cells, near_ties=st.near_ties,
                        fp64_recomputes=st.fp64_recomputes)

    def minimize_heap(self, max_flips: int = 1 << 40):
        """The serial min-heap flipping schedule (host heap, device density)."""
        st = MinStats()
        rc = self._check(self.lib.vesis_minimize_heap(self.h, int(max_flips), C.byref(st)),
                         allow=(0, 1))
        return rc, dict(converged=st.converged, flips=st.flips, band=st.band_cells,
                        near_ties=st.near_ties, fp64_recomputes=st.fp64_recomputes)

    def energy(self) -> dict:
        e = EnergyParts()
        self._check(self.lib.vesis_energy(self.h, C.byref(e)))
        return {k: getattr(e, k) for k, _ in EnergyParts._fields_}

    def forces(self) -> np.ndarray:
        f = np.zeros((self.natoms, 3))
        self._check(self.lib.vesis_forces(self.h, _ptr(f)))
        return f

    def atom_step(self, mobility: Mobility):
        info = StepInfo()
        rc = self._check(self.lib.vesis_atom_step(self.h, C.byref(mobility), C.byref(info)),
                         allow=(0, 1))
        return rc, info

    def relax(self, mobility: Mobility, max_iters: int = 3000, persist: int = 100,
              max_sweeps: int = 20000, tol_grad: float = 1e-4, tol_energy: float = 1e-5):
        """Steps 2-5 of the paper's algorithm (interface and atoms alternately)."""
        opts = RelaxOpts(max_iters=max_iters, persist=persist, max_sweeps=max_sweeps, reserved=0,
                         tol_grad=tol_grad, tol_energy=tol_energy)
        rep = RelaxReport()
        rc = self._check(self.lib.vesis_relax(self.h, C.byref(opts), C.byref(mobility),
                                              C.byref(rep)), allow=(0, 1))
        return rc, rep

    def labels(self) -> np.ndarray:
        out = np.zeros(self.n ** 3, np.int8)
        self._check(self.lib.vesis_get_labels(self.h, _ptr(out)))
        return out

    def density(self, with_bound: bool = False):
        m = self.n ** 3
        a = np.zeros(m)
        b = np.zeros(m)
        c = np.zeros(m) if with_bound else None
        self._check(self.lib.vesis_get_density(self.h, _ptr(a), _ptr(b), _ptr(c)))
        return (a, b, c) if with_bound else (a, b)

    def profile(self, enable: bool = True):
        self._check(self.lib.vesis_profile(self.h, 1 if enable else 0))

    def profile_read(self, kind: str):
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.lib.vesis_profile_read(self.h, KERNEL_KINDS[kind], C.byref(ms),
                                                C.byref(n)))
        return ms.value, n.value


class Batch:
    """Several contexts (one molecule each) relaxed together: one density
    launch and one launch per colour pass for the whole batch.  The batch's
    tables live in one more torch uint8 device tensor."""

    def __init__(self, contexts):
        if not contexts:
            raise ValueError("empty batch")
        self.contexts = list(contexts)
        self.lib = self.contexts[0].lib
        self._torch = self.contexts[0]._torch
        m = len(self.contexts)
        self._arr = (C.c_void_p * m)(*[c.h for c in self.contexts])
        n = C.c_size_t()
        rc = self.lib.vesis_batch_workspace_size(self._arr, m, C.byref(n))
        self._check(rc)
        t = self._torch
        self.nbytes = int(n.value)
        self.workspace = t.empty(self.nbytes + 256, dtype=t.uint8,
                                 device=self.contexts[0].device)
        self._ptr = (self.workspace.data_ptr() + 255) & ~255
        self.variant = 0

    def _check(self, rc, allow=(0,)):
        if rc not in allow:
            msg = self.lib.vesis_last_error(self.contexts[0].h)
            raise VesisError(rc, msg.decode() if msg else "")
        return rc

    DENSITY_VARIANTS = 3
    FLIP_VARIANTS = 2

    def tune(self):
        """Time the density tilings and (when every molecule has labels) the
        colour-pass variants on this batch and keep the fastest of each:
        returns (variant, ms), ms = the density tilings' times then one
        sweep's time per colour-pass variant (-1: not timed)."""
        best = C.c_int32()
        nv = self.DENSITY_VARIANTS + self.FLIP_VARIANTS
        ms = (C.c_double * nv)()
        self._check(self.lib.vesis_batch_tune(self._arr, len(self.contexts),
                                              C.c_void_p(self._ptr), self.nbytes,
                                              C.byref(best), ms))
        self.variant = int(best.value)
        return self.variant, [ms[k] for k in range(nv)]

    def minimize(self, max_sweeps: int = 20000, variant=None, graph: bool = True):
        m = len(self.contexts)
        st = (MinStats * m)()
        v = self.variant if variant is None else int(variant)
        flags = 0 if graph else 1
        rc = self._check(self.lib.vesis_minimize_batch(self._arr, m, C.c_void_p(self._ptr),
                                                       self.nbytes, int(max_sweeps), v, flags,
                                                       st),
                         allow=(0, 1))
        return rc, [dict(sweeps=s.sweeps, converged=s.converged, flips=s.flips,
                         band=s.band_cells, near_ties=s.near_ties,
                         fp64_recomputes=s.fp64_recomputes) for s in st]
