"""The largest grid the library accepts: 1024^3 cells (the near-tie cache
holds 2^31 FP64 entries; the force adjoint's chunk groups no longer fit the
second launch dimension at four chunks each, so each group takes five), with
a small molecule of 12 atoms at 0.01 nm.

The GPU relaxes the interface from the tight start; the oracle, given the
GPU's labels, computes the band size, the energy and the forces on sampled
atoms at the same size (about a minute of host work and 60 GB of host
memory).  Bars as at the benchmark's size: energies within 1e-6 |G|, forces
within 1e-4.
"""
import time

import numpy as np
import pytest

import synth
from helpers import energies_close, force_close, gpu_context, log, oracle_system

pytestmark = pytest.mark.gpu


def test_largest_grid():
    import torch

    w = synth.random_small(1024, 12, seed=91, h=0.01)
    t0 = time.time()
    ctx = gpu_context(w, precision=32)
    ctx.init_labels("tight", 1.0)
    rc, st = ctx.minimize()
    e = ctx.energy()
    f = ctx.forces()
    lab = ctx.labels()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    log("1024^3:", st, "G", e["total"], f"{time.time() - t0:.1f}s")
    assert rc == 0 and st["converged"] == 1 and st["flips"] > 0
    s = oracle_system(w)
    assert st["band"] == s.band_size(lab)
    ulj, ucfa, ef = s.density_grid(efield=True)
    log("oracle density done", f"{time.time() - t0:.1f}s")
    ref = s.energy(lab, ulj, ucfa, s.far_field())
    del ulj, ucfa
    bad = energies_close(e, ref, 1e-6)
    log("energy rel err", {k: (e[k] - ref[k]) / abs(ref["total"]) for k in ref})
    assert not bad, bad
    sel = np.array([0, 5, 11])
    fo = s.forces_subset(lab, ef, sel)
    ok, rel = force_close(f[sel], fo, 1e-4)
    log("force max rel err", float(rel.max()), f"{time.time() - t0:.1f}s")
    assert ok.all()
