"""The serial min-heap flipping schedule through the C ABI against the
oracle's heap schedule (same process: key (Delta E, cell index), flip the
smallest negative, re-evaluate the flip's neighbourhood).

In FP64 storage the keys agree to rounding, so labels, flip counts and band
size must be identical.  In FP32 storage the decisions are the colour
passes' (stored U unless inside the cell's bound, then FP64), so the end
state must be a local minimum of the oracle's FP64 energy: no band cell with
Delta E below -1e-12 of its terms' size.
"""
import dataclasses

import numpy as np
import pytest

from helpers import energies_close, gpu_context, log, oracle_system, ragged_small

pytestmark = pytest.mark.gpu


def _oracle_heap(w, phi0, max_flips=1 << 40):
    s = oracle_system(w)
    ulj, ucfa = s.density_grid()
    phi = phi0.copy()
    rc, st = s.minimize_heap(phi, ulj + ucfa, max_flips=max_flips)
    return s, phi, rc, st, (ulj, ucfa)


def _start(w, mode):
    s = oracle_system(w)
    if mode == "tight":
        return s.init_tight(np.asarray(w.sigma))
    return s.init_loose(0.4 * w.n * w.h)


@pytest.mark.parametrize("mode", ["tight", "loose"])
def test_heap_fp64_equals_the_oracle_heap(mode):
    w = ragged_small(seed=16, n=30, natoms=80)
    phi0 = _start(w, mode)
    log("heap fp64", mode, w.n, len(w.sigma))
    ctx = gpu_context(w, precision=64)
    ctx.init_labels("user", user=phi0)
    rc, gst = ctx.minimize_heap()
    s, ophi, orc, ost, (ulj, ucfa) = _oracle_heap(w, phi0)
    log("gpu", gst, "oracle", ost)
    assert rc == 0 and orc == 0 and gst["converged"] == 1
    assert np.array_equal(ctx.labels(), ophi)
    assert (gst["flips"], gst["band"]) == (ost["flips"], ost["band"])
    oe = s.energy(ophi, ulj, ucfa, s.far_field())
    bad = energies_close(ctx.energy(), oe, 1e-9)
    assert not bad, bad


def test_heap_stops_at_max_flips_and_resumes():
    w = ragged_small(seed=17, n=28, natoms=60)
    phi0 = _start(w, "loose")
    ctx = gpu_context(w, precision=64)
    ctx.init_labels("user", user=phi0)
    rc, st = ctx.minimize_heap(max_flips=7)
    _, ophi7, orc, ost = _oracle_heap(w, phi0, max_flips=7)[:4]
    assert rc == 1 and orc == 1 and st["flips"] == 7 and st["converged"] == 0
    assert np.array_equal(ctx.labels(), ophi7)
    # the heap order is a function of the labels alone, so resuming from
    # the 7-flip state ends where one uninterrupted run ends
    rc, st2 = ctx.minimize_heap()
    _, ophi, _, ost = _oracle_heap(w, phi0)[:4]
    assert rc == 0 and st2["flips"] + 7 == ost["flips"]
    assert np.array_equal(ctx.labels(), ophi)


def test_heap_fp32_ends_in_a_local_minimum():
    w = ragged_small(seed=18, n=34, natoms=120)
    phi0 = _start(w, "loose")
    ctx = gpu_context(w, precision=32)
    ctx.init_labels("user", user=phi0)
    rc, gst = ctx.minimize_heap()
    glab = ctx.labels()
    s, ophi, orc, ost, (ulj, ucfa) = _oracle_heap(w, phi0)
    u = ulj + ucfa
    h3 = w.h ** 3
    worst = 0.0
    for c in range(w.n ** 3):
        if not s.in_band(glab, c):
            continue
        de = s.delta_e(glab, u, c)
        worst = min(worst, de / (abs(h3 * u[c]) + 1e-30))
    diff = int(np.count_nonzero(glab != ophi))
    log("heap fp32", gst, "oracle", ost, "labels differing from the oracle heap:", diff,
        "most negative band Delta E / h^3|U|:", worst)
    assert rc == 0 and gst["converged"] == 1
    assert worst >= -1e-12
    assert gst["band"] == s.band_size(glab)
    # the energy the device reports is the oracle's energy of those labels
    bad = energies_close(ctx.energy(), s.energy(glab, ulj, ucfa, s.far_field()), 1e-6)
    assert not bad, bad


def test_heap_degenerate_starts():
    """Every cell solvent: an empty band, nothing to do.  Every cell solute:
    the band is the box's boundary shell (outside counts as solvent) and the
    heap schedule relaxes it as the oracle's does."""
    w = ragged_small(seed=19, n=24, natoms=30)
    n = w.n
    ctx = gpu_context(w, precision=64)
    ctx.init_labels("user", user=np.ones(n ** 3, np.int8))
    rc, st = ctx.minimize_heap()
    assert rc == 0 and (st["flips"], st["band"]) == (0, 0)
    assert np.all(ctx.labels() == 1)
    phi0 = -np.ones(n ** 3, np.int8)
    ctx.init_labels("user", user=phi0)
    rc, st = ctx.minimize_heap()
    _, ophi, orc, ost = _oracle_heap(w, phi0)[:4]
    log("all solute", st, ost)
    assert rc == 0 and st["flips"] == ost["flips"]
    assert np.array_equal(ctx.labels(), ophi)


def test_heap_colour_period_two_fp32():
    """Kernel radius rho_s = 2 (a smaller support, fewer stencil shells) in
    FP32 storage, loose start: a local minimum of the oracle's FP64 energy
    (the labels' difference from the oracle heap's is logged)."""
    w = ragged_small(seed=20, n=29, natoms=70)
    w = dataclasses.replace(w, params=dataclasses.replace(w.params, rho_s=2.0))
    phi0 = _start(w, "loose")
    ctx = gpu_context(w, precision=32)
    ctx.init_labels("user", user=phi0)
    rc, gst = ctx.minimize_heap()
    glab = ctx.labels()
    s, ophi, orc, ost, (ulj, ucfa) = _oracle_heap(w, phi0)
    u = ulj + ucfa
    band = [c for c in range(w.n ** 3) if s.in_band(glab, c)]
    worst = min((s.delta_e(glab, u, c) / (abs(w.h ** 3 * u[c]) + 1e-30) for c in band),
                default=0.0)
    log("heap rho_s 2", gst, "oracle", ost, "differing", int(np.count_nonzero(glab != ophi)),
        "worst", worst)
    assert rc == 0 and gst["converged"] == 1
    assert worst >= -1e-12
    assert gst["band"] == len(band)


def test_heap_argument_errors():
    from paper_2208_05524_amd import VesisError
    w = ragged_small(seed=21, n=20, natoms=10)
    ctx = gpu_context(w)
    with pytest.raises(VesisError) as e:
        ctx.minimize_heap()
    assert e.value.status == -2                      # labels not initialised
    ctx.init_labels("tight", 1.0)
    with pytest.raises(VesisError) as e:
        ctx.minimize_heap(max_flips=-1)
    assert e.value.status == -1                      # negative flip budget
    rc, st = ctx.minimize_heap(max_flips=0)
    assert st["flips"] == 0 and rc in (0, 1)
