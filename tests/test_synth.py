"""The seeded input generators: determinism and the stated geometry."""
import numpy as np
import pytest

import synth


def test_splitmix_reference_values():
    # SplitMix64 reference outputs for seed 0 (the published algorithm)
    z = synth.SplitMix64(0).u64(3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_generators_are_deterministic():
    a = synth.chain_1000()
    b = synth.chain_1000()
    assert np.array_equal(a.xyz, b.xyz) and np.array_equal(a.q, b.q)


def test_globule_geometry():
    x = synth.globule(400, seed=17)
    d1 = np.linalg.norm(x[1:] - x[:-1], axis=1)
    np.testing.assert_allclose(d1, 0.15, rtol=1e-12)
    d2 = np.linalg.norm(x[2:] - x[:-2], axis=1)
    assert d2.min() >= 0.24 - 1e-12
    dd = np.linalg.norm(x[:, None] - x[None], axis=-1)
    i, j = np.triu_indices(len(x), 3)
    assert dd[i, j].min() >= 0.30 - 1e-12


def test_atom_parameter_ranges_and_neutrality():
    s, e, q = synth.atom_params(1000, seed=5)
    assert s.min() >= 0.30 and s.max() <= 0.40
    assert e.min() >= 0.1 and e.max() <= 0.6
    assert abs(q.sum()) < 1e-12


def test_two_globules_fit_the_box():
    w = synth.two_globules()
    L = w.n * w.h / 2
    assert np.abs(w.xyz).max() + 0.4 + 3 * w.h < L


@pytest.mark.parametrize("natoms,seed", [(300, 1), (1000, 2000), (2500, 4017)])
def test_compiled_walk_matches_python_walk(natoms, seed):
    """The compiled globule walk reproduces the Python walk bit for bit."""
    if synth._walk_lib() is None:
        pytest.skip("synth/libwalk.so not built")
    a = synth.globule(natoms, seed, compiled=False)
    b = synth.globule(natoms, seed, compiled=True)
    assert np.array_equal(a, b)
