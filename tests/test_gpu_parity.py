"""GPU path (through the C ABI) against the FP64 oracle, element by element.

Bars: labels bit-exact wherever the oracle's flip decisions clear
1e-9 |G|; energies within 1e-6 |G|; per-cell FP32 densities inside the
kernel's own error bound; forces within 1e-4 per atom (relative to
max(|F_n|, 1e-3 max |F|)); FP64-mode densities within 1e-11.
"""
import dataclasses

import numpy as np
import pytest

import synth
from helpers import (check_labels, energies_close, force_close, gpu_context, log,
                     oracle_system,
                     ragged_small)

pytestmark = pytest.mark.gpu


def _oracle_state(w, phi0=None, mode="tight", param=1.0, max_sweeps=100000):
    s = oracle_system(w)
    ulj, ucfa = s.density_grid()
    far = s.far_field()
    if phi0 is not None:
        phi = phi0.copy()
    elif mode == "tight":
        phi = s.init_tight(param * np.asarray(w.sigma))
    else:
        phi = s.init_loose(param)
    e0 = s.energy(phi, ulj, ucfa, far)["total"]
    tie_tol = 1e-9 * abs(e0)
    rc, st, ties, tde = s.minimize_colour(phi, ulj + ucfa, max_sweeps=max_sweeps, tie_tol=tie_tol)
    e = s.energy(phi, ulj, ucfa, far)
    return s, phi, st, ties, e, (ulj, ucfa, far)


def _oracle_relax_from(w, phi0):
    """The oracle's colour schedule from labels phi0; every decision is
    logged and those within 1e-9 |G| of the final G are counted (a start
    with solvent inside atoms has an enormous G0, so the window is taken
    against where the relaxation ends).  Returns (labels, stats, near-tie cells,
    energy parts)."""
    import oracle
    s = oracle.System.from_workload(w)
    ulj, ucfa = s.density_grid()
    far = s.far_field()
    phi = phi0.copy()
    _, ost, tl, tde = s.minimize_colour(phi, ulj + ucfa, tie_tol=np.inf, tie_cap=1 << 22)
    assert ost["ties"] <= 1 << 22
    oe = s.energy(phi, ulj, ucfa, far)
    near = tl[np.abs(tde) <= 1e-9 * abs(oe["total"])]
    return phi, ost, near, oe


def _check_relax_from(w, phi0, label):
    ctx = gpu_context(w)
    ctx.init_labels("user", user=phi0)
    rc, gst = ctx.minimize()
    ophi, ost, near, oe = _oracle_relax_from(w, phi0)
    log(label, "gpu", gst, "oracle", ost, "decisions inside 1e-9 |G|:", len(near))
    assert rc == 0 and gst["converged"] == 1
    check_labels(ctx.labels(), ophi, near, gst, ost, what=label)
    assert not energies_close(ctx.energy(), oe, 1e-6)
    return gst


# ------------------------------------------------------------------ density

@pytest.mark.parametrize("n,natoms,seed", [(40, 300, 5), (37, 257, 6), (32, 1, 7)])
def test_fp32_density_within_its_error_bound(n, natoms, seed):
    w = ragged_small(seed=seed, n=n, natoms=natoms)
    log("density fp32", n, natoms, seed)
    ctx = gpu_context(w, precision=32)
    ulj, ucfa, bound = ctx.density(with_bound=True)
    oulj, oucfa = oracle_system(w).density_grid()
    err = np.abs((ulj + ucfa) - (oulj + oucfa))
    ratio = err / np.where(np.isfinite(bound), bound, np.inf)
    log("max err/bound", float(ratio.max()), "median rel err",
        float(np.median(err / (np.abs(oulj + oucfa) + 1e-30))))
    assert np.all(err <= bound)
    # cells whose nearest atom is closer than the guard distance carry an
    # infinite bound (always decided in FP64); elsewhere the FP32 sum keeps
    # ~6 digits of each part
    fin = np.isfinite(bound)
    assert fin.mean() > 0.9
    for g, o in ((ulj, oulj), (ucfa, oucfa)):
        if not np.abs(o).max() > 0:           # e.g. no charge: the CFA part is zero
            assert not np.abs(g).max() > 0
            continue
        rel = np.abs(g - o)[fin] / (np.abs(o)[fin] + 1e-12 * np.abs(o).max())
        assert np.quantile(rel, 0.99) < 1e-5


def test_fp64_density_matches():
    w = ragged_small(seed=8, n=37, natoms=300)
    ctx = gpu_context(w, precision=64)
    ulj, ucfa = ctx.density()
    oulj, oucfa = oracle_system(w).density_grid()
    np.testing.assert_allclose(ulj, oulj, rtol=1e-11, atol=1e-11 * np.abs(oulj).max())
    np.testing.assert_allclose(ucfa, oucfa, rtol=1e-11, atol=1e-11 * np.abs(oucfa).max())


# ------------------------------------------------------------------ labels

@pytest.mark.parametrize("mode,param", [("loose", 0.9), ("tight", 1.0), ("tight", 0.8)])
def test_initial_labels_bit_exact(mode, param):
    w = ragged_small(seed=9, n=37, natoms=200)
    ctx = gpu_context(w)
    ctx.init_labels(mode, param)
    s = oracle_system(w)
    ref = s.init_tight(param * w.sigma) if mode == "tight" else s.init_loose(param)
    assert np.array_equal(ctx.labels(), ref)


def test_user_labels_round_trip_and_energy():
    w = ragged_small(seed=10, n=33, natoms=120)
    rng = np.random.default_rng(1)
    phi = np.where(rng.random(w.n ** 3) < 0.4, -1, 1).astype(np.int8)
    ctx = gpu_context(w)
    ctx.init_labels("user", user=phi)
    assert np.array_equal(ctx.labels(), phi)
    s = oracle_system(w)
    ulj, ucfa = s.density_grid()
    ref = s.energy(phi, ulj, ucfa, s.far_field())
    got = ctx.energy()
    # integer shell counts on the GPU vs the oracle's sequential FP64 sum of
    # ~10^6 kernel values: only the oracle's rounding differs
    assert got["geom"] == pytest.approx(ref["geom"], rel=1e-10)
    assert not energies_close(got, ref, 1e-6)


# ------------------------------------------------------------- minimisation

def _compare_minimisation(w, mode, param, precision):
    ctx = gpu_context(w, precision=precision)
    ctx.init_labels(mode, param)
    rc, gst = ctx.minimize()
    glab = ctx.labels()
    ge = ctx.energy()
    s, ophi, ost, ties, oe, _ = _oracle_state(w, mode=mode, param=param)
    log(w.name, mode, "gpu", gst, "oracle", ost, "ties", len(ties))
    assert rc == 0 and gst["converged"] == 1
    check_labels(glab, ophi, ties, gst, ost, what=f"{w.name} {mode}")
    bad = energies_close(ge, oe, 1e-6)
    assert not bad, bad
    return ctx, glab, ge


@pytest.mark.parametrize("mode,param", [("tight", 1.0), ("loose", 0.95)])
def test_minimize_bit_exact_ragged(mode, param):
    w = ragged_small(seed=11, n=40, natoms=300)
    _compare_minimisation(w, mode, param, 32)


@pytest.mark.parametrize("rho_s,mode,param", [(2.0, "tight", 1.0), (1.5, "loose", 0.95)])
def test_minimize_colour_period_two(rho_s, mode, param):
    """Kernel radius rho_s <= 2: colour period p = 2 (8 colours, 16 cells of a
    colour per 32-cell word), on a grid ragged against the words."""
    w = ragged_small(seed=13, n=37, natoms=257)
    w = dataclasses.replace(w, params=dataclasses.replace(w.params, rho_s=rho_s))
    _compare_minimisation(w, mode, param, 32)


@pytest.mark.parametrize("rho_s", [3.0, 2.0])
def test_minimize_from_random_labels(rho_s):
    """Random labels (40 % solute) put almost every cell in the band, so a
    workgroup's lanes hold far more candidates than it has threads and the
    shared candidate list takes many rounds; labels, sweeps, flips and band
    size must still equal the oracle's colour schedule."""
    w = ragged_small(seed=14, n=40, natoms=200)
    w = dataclasses.replace(w, params=dataclasses.replace(w.params, rho_s=rho_s))
    rng = synth.SplitMix64(1400 + int(rho_s))
    phi0 = np.where(rng.uniform(w.n ** 3) < 0.4, -1, 1).astype(np.int8)
    _check_relax_from(w, phi0, f"random start {rho_s}")


@pytest.mark.parametrize("start", ["all_solvent", "all_solute", "one_solute_cell"])
def test_minimize_degenerate_labels(start):
    """Degenerate starts: every cell solvent (empty band: one sweep, no
    flip), every cell solute (the band is the box's boundary shell, as cells
    outside count as solvent) and a single solute cell off the atoms; each
    relaxes exactly as the oracle's colour schedule does."""
    w = ragged_small(seed=15, n=35, natoms=60)
    n = w.n
    phi0 = np.ones(n ** 3, np.int8)
    if start == "all_solute":
        phi0[:] = -1
    elif start == "one_solute_cell":
        phi0[3 + n * (4 + n * 5)] = -1
    gst = _check_relax_from(w, phi0, start)
    if start == "all_solvent":
        assert (gst["sweeps"], gst["flips"], gst["band"]) == (1, 0, 0)


def test_minimize_fp64_single_atom_64():
    """One LJ atom at the centre of [-1.5, 1.5]^3 nm, 64^3, FP64, loose sphere
    R0 = 1.2 nm."""
    w = synth.single_atom(64)
    _compare_minimisation(w, "loose", 1.2, 64)


@pytest.mark.parametrize("mode,param", [("loose", 6.0), ("tight", 1.0)])
def test_minimize_dry_and_wet_two_atoms(mode, param):
    """Two LJ atoms 8 A apart in the paper's units ((-8, 8)^3 A, 64^3, FP64):
    the loose start ends in one dry region holding both atoms, the tight
    start in two wet spheres; both bit-exact against the oracle."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "two_atom_tables.json")))
    m = g["model"]
    w = synth.Workload(name="two_atoms_8A", n=64, h=16.0 / 64, center=np.zeros(3),
                       xyz=np.asarray(g["r0_8"]["final_positions"], float).reshape(-1, 3),
                       q=np.zeros(2), sigma=np.full(2, m["sigma"]), eps=np.full(2, m["eps"]),
                       params=synth.paper_units_params(), precision=64)
    _compare_minimisation(w, mode, param, 64)


def test_minimize_chain1000_128():
    """1,000-atom globule, 128^3 grid at 0.05 nm, tight start, FP32 densities."""
    w = synth.chain_1000()
    _compare_minimisation(w, "tight", 1.0, 32)


def test_minimize_is_deterministic_and_resumable():
    w = ragged_small(seed=12, n=40, natoms=300)
    a = gpu_context(w)
    a.init_labels("tight", 1.0)
    a.minimize()
    la, ea = a.labels(), a.energy()
    b = gpu_context(w)
    b.init_labels("tight", 1.0)
    rc, st = b.minimize(max_sweeps=2)
    assert rc == 1 and st["sweeps"] == 2 and st["converged"] == 0
    rc, st = b.minimize()
    assert rc == 0
    assert np.array_equal(b.labels(), la)
    assert b.energy() == ea


# ------------------------------------------------------------------ forces

def _small_bonded(seed=13):
    w = synth.random_small(24, 30, seed, h=0.07)
    ij = np.array([[i, i + 1] for i in range(0, 29, 2)], np.int32)
    w.bonds, w.bond_r0, w.bond_k = ij, np.full(len(ij), 0.2), np.full(len(ij), 500.0)
    return w


@pytest.mark.parametrize("precision", [32, 64])
def test_forces_match_oracle(precision):
    w = _small_bonded()
    s = oracle_system(w, with_bonds=True)
    phi = s.init_tight()
    ctx = gpu_context(w, precision=precision, with_bonds=True)
    ctx.init_labels("user", user=phi)
    fg = ctx.forces()
    fo = s.forces(phi)
    ok, rel = force_close(fg, fo, 1e-4 if precision == 32 else 1e-9)
    log("force max rel err", float(rel.max()))
    assert ok.all()
    e = ctx.energy()
    ref = s.total_energy(phi)
    assert e["bond"] == pytest.approx(ref["bond"], rel=1e-12)
    assert e["total"] == pytest.approx(ref["total"], rel=1e-6)


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("n,h,pattern", [(37, 0.06, "random"), (37, 0.06, "checker"),
                                         (37, 0.06, "solute"), (12, 0.12, "random")])
def test_forces_label_patterns_match_oracle(precision, n, h, pattern):
    """The force sum over label fields that exercise its staging of x-rows
    of 16 cells, on a 37^3 grid whose last chunk along each axis is
    partial (and a 12^3 grid, one partial chunk): outside the tight
    start's solute core, random labels (rows
    mixing solute and solvent cells in every chunk) or alternating ones
    along x (every kept row half solute); or every cell solute (no row
    kept: the far field only).  The core keeps solvent cells off the atom
    centres, where the LJ gradient is astronomically large; no bonds, so
    the comparison is of the solvent forces alone."""
    w = synth.random_small(n, 40, 23, h=h)
    s = oracle_system(w)
    core = s.init_tight() == -1
    if pattern == "random":
        out = np.where(np.random.default_rng(29).random(n ** 3) < 0.5, 1, -1)
    elif pattern == "checker":
        out = np.where(np.arange(n ** 3) % n % 2 == 0, 1, -1)   # x fastest
    else:
        out = np.full(n ** 3, -1)
    phi = np.where(core, -1, out).astype(np.int8)
    ctx = gpu_context(w, precision=precision)
    ctx.init_labels("user", user=phi)
    fg = ctx.forces()
    fo = s.forces(phi)
    ok, rel = force_close(fg, fo, 1e-4 if precision == 32 else 1e-9)
    log("labels", pattern, "precision", precision, "solvent cells", int((phi == 1).sum()),
        "force max rel err", float(rel.max()), "max |F|", float(np.abs(fo).max()))
    assert ok.all()


def test_atom_step_matches_oracle():
    w = _small_bonded(seed=14)
    s = oracle_system(w, with_bonds=True)
    phi = s.init_tight()
    ctx = gpu_context(w, with_bonds=True)
    ctx.init_labels("user", user=phi)
    import oracle
    from paper_2208_05524_amd import default_mobility
    mo = oracle.default_mobility(0.1)
    mg = default_mobility(0.1)
    xo = w.xyz.copy()
    for step in range(3):
        rc_o, xo, io = s.atom_step(xo, phi, mo)
        rc_g, ig = ctx.atom_step(mg)
        xg = ctx.positions()
        log("step", step, rc_o, rc_g, io.accepted, ig.accepted, io.retries, ig.retries,
            io.G_new, ig.G_new)
        assert rc_o == rc_g and io.accepted == ig.accepted and io.retries == ig.retries
        assert ig.G_new == pytest.approx(io.G_new, rel=1e-6)
        np.testing.assert_allclose(xg, xo, rtol=0, atol=1e-6)
        assert mg.M == mo.M and mg.N_cnt == mo.N_cnt


# ------------------------------------------------------------- error paths

def test_error_statuses():
    from paper_2208_05524_amd import VesisError
    w = ragged_small(seed=15, n=24, natoms=10)
    ctx = gpu_context(w)
    with pytest.raises(VesisError) as e:
        ctx.minimize()
    assert e.value.status == -2                      # labels not initialised
    bad = w.xyz.copy()
    bad[0, 0] = 100.0
    with pytest.raises(VesisError) as e:
        ctx.set_positions(bad)
    assert e.value.status == -3                      # outside the box
    bad[0, 0] = np.nan
    with pytest.raises(VesisError) as e:
        ctx.set_positions(bad)
    assert e.value.status == -4                      # non-finite
    p = dataclasses.replace(w.params, rho_s=3.5)
    with pytest.raises(VesisError) as e:
        ctx.set_params(p)
    assert e.value.status == -1                      # kernel radius out of range
    with pytest.raises(VesisError) as e:
        ctx.init_labels("user", user=np.zeros(w.n ** 3, np.int8))
    assert e.value.status == -1                      # labels must be +-1
    import ctypes
    lib = ctx.lib
    assert lib.vesis_set_workspace(ctx.h, ctypes.c_void_p(ctx.workspace.data_ptr() + 256 - (ctx.workspace.data_ptr() % 256)), 16) == -7
