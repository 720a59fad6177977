"""Parity at the benchmark's full size: two seeded 5,000-atom globules 1.5 nm
apart on 256^3 cells of 0.05 nm, in the launch configuration bench.py times
(FP32 densities, tight start, chain bonds).

The oracle computes the whole grid here (density with field, initial
labels, colour minimisation, energy) on the host cores, and forces on 64
seeded atoms.  Every cell's density must lie inside the kernel's certified
bound; labels, sweep and flip counts must match exactly, except at cells
whose oracle decision fell inside 1e-9 |G|; energies within 1e-6 |G|;
forces within 1e-4.
A last test checks the FP64 force adjoint at this size against
Richardson-extrapolated central differences of the energy.
"""
import time

import numpy as np
import pytest

import synth
from helpers import check_labels, energies_close, force_close, gpu_context, log, oracle_system

pytestmark = pytest.mark.gpu


def _sample_atoms(natoms, seed, count=64):
    """count distinct atoms in the order the generator draws them (so the
    sample spans both globules and every atom workgroup of the adjoint)."""
    v = (synth.SplitMix64(seed).uniform(4 * count) * natoms).astype(np.int64)
    first = np.unique(v, return_index=True)[1]
    sel = v[np.sort(first)][:count]
    assert len(sel) == count
    return sel


@pytest.fixture(scope="module")
def full():
    t0 = time.time()
    w = synth.two_globules()
    log("full size: workload", w.name, w.natoms, w.n)
    ctx = gpu_context(w, precision=32, with_bonds=True)
    ctx.init_labels("tight", 1.0)
    g_init = ctx.labels()
    rc, gst = ctx.minimize()
    out = dict(w=w, rc=rc, gst=gst, g_init=g_init, g_lab=ctx.labels(), g_e=ctx.energy(),
               g_f=ctx.forces())
    out["g_ulj"], out["g_ucfa"], out["g_bound"] = ctx.density(with_bound=True)
    ctx.close()
    log("gpu done", gst, f"{time.time() - t0:.1f}s")
    s = oracle_system(w, with_bonds=True)
    oulj, oucfa, oe = s.density_grid(efield=True)
    log("oracle density done", f"{time.time() - t0:.1f}s")
    far = s.far_field()
    phi = s.init_tight()
    out["o_init"] = phi.copy()
    e0 = s.energy(phi, oulj, oucfa, far)["total"]
    rc_o, ost, ties, _ = s.minimize_colour(phi, oulj + oucfa, tie_tol=1e-9 * abs(e0))
    log("oracle minimisation done", ost, "ties", len(ties), f"{time.time() - t0:.1f}s")
    e = s.energy(phi, oulj, oucfa, far)
    e["bond"] = s.bond_energy()
    e["total"] += e["bond"]
    sel = _sample_atoms(w.natoms, 3064)
    log("sampled atoms span", int(sel.min()), "to", int(sel.max()))
    out.update(s=s, o_ulj=oulj, o_ucfa=oucfa, o_lab=phi, o_st=ost, o_ties=ties, o_e=e, sel=sel,
               o_f=s.forces_subset(phi, oe, sel))
    log("oracle forces done", f"{time.time() - t0:.1f}s")
    return out


def test_full_size_initial_labels(full):
    assert np.array_equal(full["g_init"], full["o_init"])


def test_full_size_density_inside_bound_everywhere(full):
    err = np.abs((full["g_ulj"] + full["g_ucfa"]) - (full["o_ulj"] + full["o_ucfa"]))
    b = full["g_bound"]
    fin = np.isfinite(b)
    ratio = err / b
    worst = int(np.argmax(ratio))
    x = full["s"].cell_center(worst)
    dmin = float(np.sqrt(((full["w"].xyz - x) ** 2).sum(1)).min())
    log("cells with a bound:", fin.mean(), "max err/bound", float(ratio[worst]),
        "at cell", worst, "nearest atom", dmin, "nm")
    assert np.all(err <= b)


def test_full_size_labels_and_energy(full):
    gst, ost = full["gst"], full["o_st"]
    log("gpu", gst, "oracle", ost)
    assert full["rc"] == 0 and gst["converged"] == 1 and ost["converged"] == 1
    assert full["o_st"]["ties"] == len(full["o_ties"])  # every near tie logged
    check_labels(full["g_lab"], full["o_lab"], full["o_ties"], gst, ost, what="full size")
    bad = energies_close(full["g_e"], full["o_e"], 1e-6, keys=("geom", "vdw_in", "vdw_far",
                                                             "elec_in", "elec_far", "bond",
                                                             "total"))
    log("energy gpu", full["g_e"], "oracle", full["o_e"])
    assert not bad, bad


def test_full_size_forces_on_sampled_atoms(full):
    fg = full["g_f"][full["sel"]]
    ok, rel = force_close(fg, full["o_f"], 1e-4)
    log("force max rel err", float(rel.max()))
    assert ok.all()


@pytest.mark.parametrize("chunk", range(4))
def test_full_size_forces_match_central_differences_fp64(chunk):
    """The force adjoint at the benchmark's full size against central
    differences of the energy at fixed labels, with FP64 densities, on 64
    seeded atoms (16 per chunk, drawn across both globules) x 3 directions;
    1e-4 relative, as for the oracle comparison.

    At this size the central difference with step h = 1e-4 nm still carries
    its O(h^2) truncation error (up to ~5e-3 relative here: the difference
    moves by 4x per doubling of h), so the differences at h and h/2 are
    combined by Richardson extrapolation, (4 D(h/2) - D(h)) / 3, which
    cancels the h^2 term."""
    import time

    w = synth.two_globules()
    ctx = gpu_context(w, precision=64, with_bonds=True)
    ctx.init_labels("tight", 1.0)
    t0 = time.time()
    f = ctx.forces()
    sel = _sample_atoms(w.natoms, 3065)[16 * chunk:16 * (chunk + 1)]
    hfd = 1e-4

    def central(a, d, step):
        xp = w.xyz.copy()
        xp[a, d] += step
        ctx.set_positions(xp)
        ep = ctx.energy()["total"]
        xm = w.xyz.copy()
        xm[a, d] -= step
        ctx.set_positions(xm)
        em = ctx.energy()["total"]
        return -(ep - em) / (2 * step)

    fd = np.zeros((len(sel), 3))
    plain = np.zeros((len(sel), 3))
    for k, a in enumerate(sel):
        for d in range(3):
            d1, d2 = central(a, d, hfd), central(a, d, hfd / 2)
            plain[k, d] = d1
            fd[k, d] = (4.0 * d2 - d1) / 3.0
    ctx.set_positions(w.xyz)
    ok, rel = force_close(f[sel], fd, 1e-4)
    _, rel_plain = force_close(f[sel], plain, 1e-4)
    log("full-size FD (FP64):", len(sel), "atoms, max rel err", float(rel.max()),
        "(plain h = 1e-4 difference:", float(rel_plain.max()), ")", f"{time.time() - t0:.1f}s")
    assert ok.all()
