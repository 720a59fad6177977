"""Pins of the oracle's solute-solute terms (Eq. "Gss" beyond bonds: bending,
torsion, non-bonded LJ and Coulomb) and of their gradients (Appendix, "Force
calculations of molecular mechanical interactions").

Energies are checked on geometries built with a known angle or distance,
where the term reduces to its defining formula at that angle; gradients
against central differences of the energy and against the invariances of
an internal potential (zero net force and zero net torque).  CPU only.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _rotation(seed):
    """A seeded proper rotation (QR of a Gaussian-free uniform matrix)."""
    u = synth.SplitMix64(seed).uniform(9, -1.0, 1.0).reshape(3, 3)
    q, r = np.linalg.qr(u)
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _system(xyz, ss, q=None, sigma=None, eps=None, params=None):
    xyz = np.asarray(xyz, float).reshape(-1, 3)
    n = len(xyz)
    return oracle.System(32, 0.1, np.zeros(3), xyz,
                         np.zeros(n) if q is None else np.asarray(q, float),
                         np.full(n, 0.35) if sigma is None else np.asarray(sigma, float),
                         np.full(n, 0.4) if eps is None else np.asarray(eps, float),
                         params or synth.Params(), ss=ss)


def _place(pts, seed):
    """Rotate and translate a small geometry by a seeded rigid motion."""
    return np.asarray(pts, float) @ _rotation(seed).T + np.array([0.31, -0.17, 0.23])


def test_bend_energy_closed_form():
    """Vertex j, arms of lengths 0.15 and 0.21 nm at an angle theta built
    into the coordinates: the term is (1/2) B (theta - theta0)^2."""
    total, pts, ang = 0.0, [], []
    B, th0 = 410.0, 1.91
    for m, th in enumerate([0.4, 1.2, 1.91, 2.5, 3.0]):
        base = 3 * m
        arm_i = 0.15 * np.array([1.0, 0.0, 0.0])
        arm_k = 0.21 * np.array([math.cos(th), math.sin(th), 0.0])
        local = np.array([arm_i, [0.0, 0.0, 0.0], arm_k]) + np.array([0.0, 0.0, 0.5 * m])
        pts.extend(local)
        ang.append([base, base + 1, base + 2])
        total += 0.5 * B * (th - th0) ** 2
    ss = oracle.SoluteTerms(angles=ang, theta0=[th0] * len(ang), k_angle=[B] * len(ang))
    s = _system(_place(pts, 11), ss)
    assert s.ss_energy()["bend"] == pytest.approx(total, rel=1e-12)


def _dihedral_points(alpha):
    """i, j, k, l with the j-k axis along x, i displaced along +y and l along
    (0, cos alpha, sin alpha): the planes (i, j, k) and (j, k, l) meet at the
    angle alpha (alpha = 0 cis, alpha = pi trans)."""
    return np.array([[-0.05, 0.14, 0.0], [0.0, 0.0, 0.0], [0.15, 0.0, 0.0],
                     [0.22, 0.13 * math.cos(alpha), 0.13 * math.sin(alpha)]])


@pytest.mark.parametrize("alpha", [0.2, 1.0, math.pi / 2, 2.4, 3.0, 4.0, 5.5])
def test_torsion_energy_closed_form(alpha):
    """The torsion term at a built dihedral angle alpha equals
    sum_n C_n [1 + cos(n tau - psi_n)] with tau = alpha folded into [0, pi]
    (the angle between two planes); psi_n = 0 for odd n, pi for even n."""
    c = synth.SplitMix64(91).uniform(7, 0.1, 2.0)
    psi = np.array([math.pi if n % 2 == 0 else 0.0 for n in range(7)])
    tau = alpha if alpha <= math.pi else 2 * math.pi - alpha
    ref = sum(c[n] * (1.0 + math.cos(n * tau - psi[n])) for n in range(7))
    ss = oracle.SoluteTerms(torsions=[[0, 1, 2, 3]], c=c[None, :], psi=psi[None, :])
    s = _system(_place(_dihedral_points(alpha), 12), ss)
    assert s.ss_energy()["torsion"] == pytest.approx(ref, rel=1e-12)


def test_torsion_trans_is_the_minimum_of_a_positive_odd_term():
    """With only C_1 > 0 and psi_1 = 0 the term is 0 in trans and 2 C_1 in cis."""
    c = np.zeros((1, 7))
    c[0, 1] = 1.7
    ss = oracle.SoluteTerms(torsions=[[0, 1, 2, 3]], c=c, psi=np.zeros((1, 7)))
    trans = _system(_dihedral_points(math.pi), ss).ss_energy()["torsion"]
    cis = _system(_dihedral_points(0.0), ss).ss_energy()["torsion"]
    assert abs(trans) < 1e-12 and cis == pytest.approx(3.4, rel=1e-12)


def test_nonbonded_pair_closed_forms():
    """Two atoms with different sigma and eps at r = 2^(1/6) sigma_ij sit at
    the LJ minimum -eps_ij, with sigma_ij = (sigma_1 + sigma_2)/2 and
    eps_ij = sqrt(eps_1 eps_2); their Coulomb energy is k Q_1 Q_2/(eps_w r)."""
    s1, s2, e1, e2, q1, q2 = 0.31, 0.39, 0.2, 0.55, 0.3, -0.25
    sij, eij = 0.5 * (s1 + s2), math.sqrt(e1 * e2)
    r = 2.0 ** (1.0 / 6.0) * sij
    p = synth.Params()
    ss = oracle.SoluteTerms(nonbonded=True, sigma_ss=[s1, s2], eps_ss=[e1, e2])
    s = _system(_place([[0, 0, 0], [r, 0, 0]], 13), ss, q=[q1, q2])
    e = s.ss_energy()
    assert e["vdw_ss"] == pytest.approx(-eij, rel=1e-12)
    assert e["elec_ss"] == pytest.approx(p.coulomb_k * q1 * q2 / (p.eps_w * r), rel=1e-12)


def test_exclusions_remove_exactly_the_listed_pairs():
    """Four atoms with pairs (0,1) and (2,3) excluded: the non-bonded sums
    equal those of the other four pairs, each evaluated as a two-atom system."""
    xyz = synth.random_small(16, 4, seed=71, spread=0.5).xyz
    q = np.array([0.3, -0.2, 0.15, -0.25])
    sig = np.array([0.30, 0.34, 0.37, 0.40])
    eps = np.array([0.2, 0.3, 0.45, 0.6])
    ss = oracle.SoluteTerms(nonbonded=True, sigma_ss=sig, eps_ss=eps,
                            exclusions=[[1, 0], [2, 3]])
    e = _system(xyz, ss, q=q).ss_energy()
    lj = el = 0.0
    for i, j in [(0, 2), (0, 3), (1, 2), (1, 3)]:
        pair = oracle.SoluteTerms(nonbonded=True, sigma_ss=sig[[i, j]], eps_ss=eps[[i, j]])
        ep = _system(xyz[[i, j]], pair, q=q[[i, j]]).ss_energy()
        lj += ep["vdw_ss"]
        el += ep["elec_ss"]
    assert e["vdw_ss"] == pytest.approx(lj, rel=1e-12)
    assert e["elec_ss"] == pytest.approx(el, rel=1e-12)


def _chain(natoms=12, seed=81):
    w = synth.random_small(32, natoms, seed=seed, spread=0.6)
    xyz = synth.globule(natoms, seed=seed) * 1.6
    top = synth.chain_topology([(0, natoms)], seed=seed, exclude=2)
    ss = oracle.SoluteTerms(top.angles, top.theta0, top.k_angle, top.torsions, top.c, top.psi,
                            True, None, None, top.exclusions)
    return w, xyz, ss


def test_ss_forces_match_central_differences():
    """Gradient of the bending, torsion and non-bonded terms of a 12-atom
    chain against central differences of their energy (step 1e-5 nm)."""
    w, xyz, ss = _chain()
    s = _system(xyz, ss, q=w.q, sigma=w.sigma, eps=w.eps)
    g = s.ss_gradient()
    hfd = 1e-5
    fd = np.zeros_like(g)
    for a in range(len(xyz)):
        for d in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[a, d] += hfd
            xm[a, d] -= hfd
            ep = sum(_system(xp, ss, q=w.q, sigma=w.sigma, eps=w.eps).ss_energy().values())
            em = sum(_system(xm, ss, q=w.q, sigma=w.sigma, eps=w.eps).ss_energy().values())
            fd[a, d] = (ep - em) / (2 * hfd)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7 * np.abs(g).max())


def test_ss_forces_are_internal():
    """An energy of relative positions only: the gradients sum to zero and
    exert no net torque, term by term."""
    w, xyz, ss_all = _chain(16, seed=82)
    for part in ("bend", "torsion", "pairs"):
        ss = oracle.SoluteTerms(
            angles=ss_all.angles if part == "bend" else None,
            theta0=ss_all.theta0 if part == "bend" else None,
            k_angle=ss_all.k_angle if part == "bend" else None,
            torsions=ss_all.torsions if part == "torsion" else None,
            c=ss_all.c if part == "torsion" else None,
            psi=ss_all.psi if part == "torsion" else None,
            nonbonded=part == "pairs", exclusions=ss_all.exclusions)
        g = _system(xyz, ss, q=w.q, sigma=w.sigma, eps=w.eps).ss_gradient()
        scale = np.abs(g).max() * np.abs(xyz).max()
        assert np.abs(g.sum(0)).max() <= 1e-12 * np.abs(g).max() * len(g), part
        assert np.abs(np.cross(xyz, g).sum(0)).max() <= 1e-12 * scale * len(g), part


def test_total_forces_include_the_solute_terms():
    """orc_forces with solute-solute terms against central differences of
    the total energy (solvent, far field, bonds and Eq. "Gss" terms)."""
    natoms = 6
    xyz = synth.globule(natoms, seed=83) * 1.5
    w = synth.random_small(16, natoms, seed=83, h=0.07)
    top = synth.chain_topology([(0, natoms)], seed=83, exclude=1)
    ss = oracle.SoluteTerms(top.angles, top.theta0, top.k_angle, top.torsions, top.c, top.psi,
                            True, None, None, top.exclusions)
    bonds, r0, kb = synth.chain_bonds(natoms)
    s = oracle.System(w.n, w.h, w.center, xyz, w.q, w.sigma, w.eps, w.params, bonds, r0,
                      kb * 1e-2, ss)
    phi = s.init_tight()
    f = s.forces(phi)
    e = s.total_energy(phi)
    assert e["total"] == pytest.approx(
        sum(v for k, v in e.items() if k != "total"), rel=1e-13)
    hfd = 1e-5
    fd = np.zeros_like(f)
    for a in range(natoms):
        for d in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[a, d] += hfd
            xm[a, d] -= hfd
            ep = s.with_positions(xp).total_energy(phi)["total"]
            em = s.with_positions(xm).total_energy(phi)["total"]
            fd[a, d] = -(ep - em) / (2 * hfd)
    np.testing.assert_allclose(f, fd, rtol=1e-5, atol=1e-6 * np.abs(f).max())
