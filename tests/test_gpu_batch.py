"""Batched interface relaxation (many molecules per launch) on the GPU.

Each molecule of a batch must end exactly where the oracle's colour
schedule takes it, and where a single-molecule call takes it: same labels,
same sweep, flip and band counts, and energies within 1e-6.
"""
import dataclasses

import numpy as np
import pytest

import synth
from helpers import check_labels, energies_close, gpu_context, log, oracle_system

pytestmark = pytest.mark.gpu


def _molecules():
    # uneven grids (ragged against the 16 x 8 x 4 bricks and 32-cell words)
    # and atom counts
    spec = [(24, 20, 41), (40, 150, 42), (33, 60, 43), (48, 300, 44), (36, 90, 45)]
    return [synth.random_small(n, na, seed, h=0.06) for n, na, seed in spec]


@pytest.mark.parametrize("variant", [0, 1])
def test_batch_matches_oracle_and_single_contexts(variant):
    _check_batch(_molecules(), variant)


def test_batch_colour_period_two():
    """The same with rho_s = 2 (colour period 2, 8 colours per sweep)."""
    ws = [dataclasses.replace(w, params=dataclasses.replace(w.params, rho_s=2.0))
          for w in _molecules()]
    _check_batch(ws, 0)


def test_batch_of_one_and_mixed_far_nodes():
    """A batch of one molecule, and a batch whose molecules have different
    far-field node counts (far_nf 32, 20 and 8; ntau 16, 12 and 4): every
    result equals the single-molecule path's."""
    ws = _molecules()
    _check_batch(ws[:1], 0)
    mixed = []
    for w, (nf, nt) in zip(ws[1:4], [(32, 16), (20, 12), (8, 4)]):
        mixed.append(dataclasses.replace(w, params=dataclasses.replace(w.params, far_nf=nf,
                                                                      far_ntau=nt)))
    _check_batch(mixed, 0)


def test_batch_recomputes_only_the_molecules_that_moved():
    """After a batched relaxation, one molecule's atoms move: the next batch
    call recomputes the density and far field of that molecule alone (the
    others keep theirs) and ends where a fresh single context ends, bit for
    bit; the others keep their labels and energies."""
    from paper_2208_05524_amd import Batch
    ws = _molecules()[:3]
    ctxs = [gpu_context(w) for w in ws]
    for c in ctxs:
        c.init_labels("tight", 1.0)
    b = Batch(ctxs)
    assert b.minimize()[0] == 0
    before = [(c.labels(), c.energy()) for c in ctxs]
    moved = ws[1].xyz + np.array([0.013, -0.007, 0.011])
    ctxs[1].set_positions(moved)
    ctxs[1].init_labels("tight", 1.0)
    rc, st = b.minimize()
    assert rc == 0
    for i in (0, 2):
        assert np.array_equal(ctxs[i].labels(), before[i][0])
        assert ctxs[i].energy() == before[i][1]
    w1 = dataclasses.replace(ws[1], xyz=moved)
    single = gpu_context(w1)
    single.init_labels("tight", 1.0)
    _, sst = single.minimize()
    assert np.array_equal(single.labels(), ctxs[1].labels())
    assert (sst["sweeps"], sst["flips"], sst["band"]) == (st[1]["sweeps"], st[1]["flips"],
                                                          st[1]["band"])
    e, es = ctxs[1].energy(), single.energy()
    for k in ("vdw_in", "elec_in", "vdw_far", "elec_far", "geom", "total"):
        assert e[k] == es[k], k


def _check_batch(ws, variant):
    from paper_2208_05524_amd import Batch
    ctxs = [gpu_context(w) for w in ws]
    for c in ctxs:
        c.init_labels("tight", 1.0)
    b = Batch(ctxs)
    rc, stats = b.minimize(variant=variant)
    assert rc == 0
    for w, c, st in zip(ws, ctxs, stats):
        s = oracle_system(w)
        ulj, ucfa = s.density_grid()
        far = s.far_field()
        phi = s.init_tight()
        e0 = s.energy(phi, ulj, ucfa, far)["total"]
        _, ost, ties, _ = s.minimize_colour(phi, ulj + ucfa, tie_tol=1e-9 * abs(e0))
        lab = c.labels()
        log(w.name, "batch", st, "oracle", ost, "ties", len(ties))
        assert ost["ties"] == len(ties)
        check_labels(lab, phi, ties, st, ost, what=f"{w.name} batch")
        e = c.energy()
        ref = s.energy(phi, ulj, ucfa, far)
        bad = energies_close(e, ref, 1e-6)
        log("energy rel err", {k: (e[k] - ref[k]) / abs(ref["total"]) for k in ref})
        assert not bad, bad
        # the single-molecule path from the same start
        single = gpu_context(w)
        single.init_labels("tight", 1.0)
        _, sst = single.minimize()
        assert np.array_equal(single.labels(), lab)
        assert (sst["sweeps"], sst["flips"], sst["band"]) == (st["sweeps"], st["flips"],
                                                              st["band"])
        # the batched far field computes what the single-molecule launches
        # compute, in the same order: bit for bit; so does the batched
        # density in variant 0, whose bricks (16 x 8 x 4) are the single
        # kernel's (variant 1's 16 x 8 x 2 bricks split atoms into near and
        # far differently, so its volume terms differ by FP32 rounding)
        es = single.energy()
        exact = ("vdw_far", "elec_far", "geom")
        if variant == 0:
            exact += ("vdw_in", "elec_in", "total")
        for k in exact:
            assert e[k] == es[k], (k, e[k], es[k])


def test_batch_resumes_after_max_sweeps():
    from paper_2208_05524_amd import Batch
    ws = _molecules()
    one = [gpu_context(w) for w in ws]
    two = [gpu_context(w) for w in ws]
    for c in one + two:
        c.init_labels("tight", 1.0)
    _, s1 = Batch(one).minimize()
    b2 = Batch(two)
    rc, part = b2.minimize(max_sweeps=2)
    assert rc == 1 and any(st["converged"] == 0 for st in part)
    rc, rest = b2.minimize()
    assert rc == 0
    for c1, c2 in zip(one, two):
        assert np.array_equal(c1.labels(), c2.labels())


def test_batch_tune_and_errors():
    from paper_2208_05524_amd import Batch, VesisError
    ws = _molecules()[:3]
    ctxs = [gpu_context(w) for w in ws]
    for c in ctxs:
        c.init_labels("tight", 1.0)
    b = Batch(ctxs)
    before = [c.labels() for c in ctxs]
    best, ms = b.tune()
    log("tune", best, ms)
    assert 0 <= best < Batch.DENSITY_VARIANTS * Batch.FLIP_VARIANTS and all(t > 0 for t in ms)
    # the colour-pass timing ran from the labels and put them back
    assert all(np.array_equal(a, c.labels()) for a, c in zip(before, ctxs))
    rc, _ = b.minimize()
    assert rc == 0
    # FP64 members are refused
    c64 = gpu_context(ws[0], precision=64)
    c64.init_labels("tight", 1.0)
    with pytest.raises(VesisError) as e:
        Batch([ctxs[0], c64]).minimize()
    assert e.value.status == -1
    # a context twice
    with pytest.raises(VesisError) as e:
        Batch([ctxs[0], ctxs[0]]).minimize()
    assert e.value.status == -1
    # labels missing
    fresh = gpu_context(ws[1])
    with pytest.raises(VesisError) as e:
        Batch([ctxs[0], fresh]).minimize()
    assert e.value.status == -2


def test_full_batch_64_molecules_matches_single():
    """The 64-molecule batch (atom counts log-uniform in [200, 3000], grids
    64^3 to 160^3 at 0.05 nm): every molecule's labels and counts equal the
    single-molecule result, and the energies agree to 1e-6."""
    import time

    import torch

    from paper_2208_05524_amd import Batch
    ws = synth.batch_conformations()
    single = [gpu_context(w) for w in ws]
    batch = [gpu_context(w) for w in ws]
    for c in single + batch:
        c.init_labels("tight", 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sst = [c.minimize()[1] for c in single]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b = Batch(batch)
    rc, bst = b.minimize()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"64 molecules: one at a time {1e3 * (t1 - t0):.1f} ms, batched {1e3 * (t2 - t1):.1f} ms")
    assert rc == 0
    for cs, cb, a, bb in zip(single, batch, sst, bst):
        assert np.array_equal(cs.labels(), cb.labels())
        assert (a["sweeps"], a["flips"], a["band"]) == (bb["sweeps"], bb["flips"], bb["band"])
        es, eb = cs.energy(), cb.energy()
        assert abs(es["total"] - eb["total"]) <= 1e-6 * abs(es["total"])


def test_batch_graph_replays_match_eager():
    """The captured group of sweeps, replayed several times per call with the
    host's reads and synchronisations between replays, ends where direct
    launches end; twice in a row."""
    from paper_2208_05524_amd import Batch
    ws = _molecules()
    eager = [gpu_context(w) for w in ws]
    graph = [gpu_context(w) for w in ws]
    be, bg = Batch(eager), Batch(graph)
    for rep in range(2):
        # a loose sphere filling most of the box needs many sweeps (two or
        # more replays of the 8-sweep group); then a tight start
        for w, c in zip(ws + ws, eager + graph):
            if rep == 0:
                c.init_labels("loose", 0.45 * w.n * w.h)
            else:
                c.init_labels("tight", 1.0)
        rc_e, se = be.minimize(graph=False)
        rc_g, sg = bg.minimize(graph=True)
        log("rep", rep, "sweeps", [s["sweeps"] for s in sg])
        assert rc_e == rc_g == 0
        if rep == 0:
            assert max(s["sweeps"] for s in sg) > 8  # two replays or more
        for ce, cg, a, b in zip(eager, graph, se, sg):
            assert np.array_equal(ce.labels(), cg.labels())
            assert a == b


def test_full_batch_64_molecules_matches_oracle():
    """The 64-molecule batch against the oracle's colour schedule, molecule by
    molecule: labels (differences only at cells whose oracle decision fell
    inside 1e-9 |G|), sweep, flip and band counts, and every energy part
    within 1e-6 |G|.  Covers the large uneven shapes (up to 160^3 cells and
    3,000 atoms) that the small-molecule batch tests do not reach; the
    oracle's densities take about a minute on the host cores."""
    import time

    from paper_2208_05524_amd import Batch
    ws = synth.batch_conformations()
    ctxs = [gpu_context(w) for w in ws]
    for c in ctxs:
        c.init_labels("tight", 1.0)
    rc, bst = Batch(ctxs).minimize()
    assert rc == 0
    got = [(c.labels(), c.energy()) for c in ctxs]
    for c in ctxs:
        c.close()
    t0 = time.time()
    worst = 0.0
    for w, st, (lab, e) in zip(ws, bst, got):
        s = oracle_system(w)
        ulj, ucfa = s.density_grid()
        far = s.far_field()
        phi = s.init_tight()
        e0 = s.energy(phi, ulj, ucfa, far)["total"]
        _, ost, ties, _ = s.minimize_colour(phi, ulj + ucfa, tie_tol=1e-9 * abs(e0))
        assert ost["ties"] == len(ties)
        ref = s.energy(phi, ulj, ucfa, far)
        rel = max(abs(e[k] - ref[k]) for k in ("geom", "vdw_in", "vdw_far", "elec_in",
                                               "elec_far", "total")) / abs(ref["total"])
        worst = max(worst, rel)
        log(f"{w.name} n={w.n} atoms={w.natoms} sweeps {st['sweeps']}/{ost['sweeps']} "
            f"max |dE|/|G| {rel:.2e} ties {len(ties)} ({time.time() - t0:.0f}s)")
        check_labels(lab, phi, ties, st, ost, what=w.name)
        bad = energies_close(e, ref, 1e-6)
        assert not bad, (w.name, bad)
    log("64 molecules: largest energy difference / |G|", worst)


def test_every_batch_variant_reaches_the_single_molecule_result():
    """Each density tiling and colour-pass register variant the tuner picks
    among ends in the single-molecule path's labels, sweep, flip and band
    counts (decisions are exact whatever the FP32 rounding), with energies
    within 1e-6 |G|; twice in a row per variant, the second call replaying
    the graph kept from the first."""
    from paper_2208_05524_amd import Batch
    ws = _molecules()
    single = []
    for w in ws:
        c = gpu_context(w)
        c.init_labels("tight", 1.0)
        _, st = c.minimize()
        single.append((c.labels(), st, c.energy()))
    ctxs = [gpu_context(w) for w in ws]
    b = Batch(ctxs)
    for v in range(Batch.DENSITY_VARIANTS * Batch.FLIP_VARIANTS):
        for rep in range(2):
            for c, w in zip(ctxs, ws):
                c.set_positions(w.xyz)
                c.init_labels("tight", 1.0)
            rc, st = b.minimize(variant=v)
            assert rc == 0
            for c, (lab, sst, es), bst in zip(ctxs, single, st):
                assert np.array_equal(c.labels(), lab), (v, rep)
                assert (sst["sweeps"], sst["flips"], sst["band"]) == \
                    (bst["sweeps"], bst["flips"], bst["band"]), (v, rep)
                e = c.energy()
                assert abs(e["total"] - es["total"]) <= 1e-6 * abs(es["total"]), (v, rep)
        log("variant", v, "ok")
