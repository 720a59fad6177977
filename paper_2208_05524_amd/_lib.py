"""ctypes declarations of the C ABI in include/vesis.h.

Argument marshalling only: every step of the hot path runs in libvesis.so.
Loading fails loudly when the library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvesis.so")

VESIS_OK = 0
VESIS_NOT_CONVERGED = 1
STATUS_NAMES = {0: "VESIS_OK", 1: "VESIS_NOT_CONVERGED", -1: "VESIS_E_ARG", -2: "VESIS_E_STATE",
                -3: "VESIS_E_OUT_OF_BOX", -4: "VESIS_E_NONFINITE", -5: "VESIS_E_NO_DEVICE",
                -6: "VESIS_E_DEVICE", -7: "VESIS_E_WORKSPACE"}

EXPORTS = ["vesis_create", "vesis_destroy", "vesis_last_error", "vesis_set_params",
           "vesis_set_grid", "vesis_set_atoms", "vesis_set_positions", "vesis_get_positions",
           "vesis_set_bonds", "vesis_set_angles", "vesis_set_torsions", "vesis_set_nonbonded",
           "vesis_workspace_size", "vesis_set_workspace", "vesis_init_labels",
           "vesis_init_labels_logits",
           "vesis_minimize_interface", "vesis_minimize_heap", "vesis_energy", "vesis_forces", "vesis_atom_step",
           "vesis_relax", "vesis_batch_workspace_size", "vesis_batch_tune", "vesis_minimize_batch",
           "vesis_get_labels", "vesis_get_density", "vesis_profile", "vesis_profile_read"]


class Params(C.Structure):
    _fields_ = [("rho_w", C.c_double), ("gamma0", C.c_double), ("eps_m", C.c_double),
                ("eps_w", C.c_double), ("coulomb_k", C.c_double), ("rho_s", C.c_double),
                ("r2_min", C.c_double), ("far_nf", C.c_int32), ("far_ntau", C.c_int32),
                ("precision", C.c_int32), ("reserved", C.c_int32)]


class EnergyParts(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("geom", "vdw_in", "vdw_far", "elec_in", "elec_far", "bond", "bend", "torsion",
                 "vdw_ss", "elec_ss", "total")]


class MinStats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("converged", C.c_int32), ("flips", C.c_int64),
                ("band_cells", C.c_int64), ("near_ties", C.c_int64),
                ("fp64_recomputes", C.c_int64)]


class Mobility(C.Structure):
    _fields_ = [("M", C.c_double), ("alpha", C.c_double), ("dt", C.c_double),
                ("dG_frac", C.c_double), ("M_min", C.c_double), ("G_old", C.c_double),
                ("N_cnt", C.c_int32), ("N_cnt_max", C.c_int32), ("k", C.c_int32),
                ("max_retries", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("accepted", C.c_int32), ("retries", C.c_int32), ("G_old", C.c_double),
                ("G_new", C.c_double), ("max_grad", C.c_double), ("omega", C.c_double)]


class RelaxOpts(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("persist", C.c_int32), ("max_sweeps", C.c_int32),
                ("reserved", C.c_int32), ("tol_grad", C.c_double), ("tol_energy", C.c_double)]


class RelaxReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("stop_reason", C.c_int32), ("sweeps", C.c_int32),
                ("retries", C.c_int32), ("G_final", C.c_double), ("max_grad", C.c_double),
                ("dG_abs", C.c_double), ("dG_rel", C.c_double)]


_lib = None


class VesisError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load():
    """Load libvesis.so (built by ``python -m paper_2208_05524_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2208_05524_amd.build` (no fallback exists)")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    st = C.c_int
    L.vesis_create.argtypes = [I32, P, C.POINTER(P)]
    L.vesis_create.restype = st
    L.vesis_destroy.argtypes = [P]
    L.vesis_destroy.restype = None
    L.vesis_last_error.argtypes = [P]
    L.vesis_last_error.restype = C.c_char_p
    L.vesis_set_params.argtypes = [P, C.POINTER(Params)]
    L.vesis_set_grid.argtypes = [P, I32, P, D]
    L.vesis_set_atoms.argtypes = [P, I64, P, P, P, P, P]
    L.vesis_set_positions.argtypes = [P, P, I32]
    L.vesis_get_positions.argtypes = [P, P]
    L.vesis_set_bonds.argtypes = [P, I64, P, P, P]
    L.vesis_set_angles.argtypes = [P, I64, P, P, P]
    L.vesis_set_torsions.argtypes = [P, I64, P, P, P]
    L.vesis_set_nonbonded.argtypes = [P, C.c_int32, P, P, I64, P]
    L.vesis_workspace_size.argtypes = [P, C.POINTER(C.c_size_t)]
    L.vesis_set_workspace.argtypes = [P, P, C.c_size_t]
    L.vesis_init_labels.argtypes = [P, I32, D, P]
    L.vesis_minimize_interface.argtypes = [P, I32, C.POINTER(MinStats)]
    L.vesis_minimize_heap.argtypes = [P, I64, C.POINTER(MinStats)]
    L.vesis_energy.argtypes = [P, C.POINTER(EnergyParts)]
    L.vesis_forces.argtypes = [P, P]
    L.vesis_atom_step.argtypes = [P, C.POINTER(Mobility), C.POINTER(StepInfo)]
    L.vesis_relax.argtypes = [P, C.POINTER(RelaxOpts), C.POINTER(Mobility), C.POINTER(RelaxReport)]
    L.vesis_init_labels_logits.argtypes = [P, P]
    PP = C.POINTER(C.c_void_p)
    L.vesis_batch_workspace_size.argtypes = [PP, C.c_int32, C.POINTER(C.c_size_t)]
    L.vesis_batch_tune.argtypes = [PP, C.c_int32, P, C.c_size_t, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_double)]
    L.vesis_minimize_batch.argtypes = [PP, C.c_int32, P, C.c_size_t, C.c_int32, C.c_int32,
                                       C.c_int32, C.POINTER(MinStats)]
    L.vesis_get_labels.argtypes = [P, P]
    L.vesis_get_density.argtypes = [P, P, P, P]
    L.vesis_profile.argtypes = [P, I32]
    L.vesis_profile_read.argtypes = [P, I32, C.POINTER(D), C.POINTER(I64)]
    for name in EXPORTS:
        if name not in ("vesis_destroy", "vesis_last_error"):
            getattr(L, name).restype = st
    _lib = L
    return L
