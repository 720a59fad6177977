"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks one part of the oracle against something other than the
oracle's own formula: a closed form, an independent numerical integral, a
brute-force recomputation by a different route, an invariance, or a number
the paper prints.  All run on the CPU.
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.optimize import minimize_scalar
from scipy.special import eval_legendre

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _sys(n, h, xyz, q, sigma, eps, params=None, center=(0.0, 0.0, 0.0)):
    return oracle.System(n, h, np.asarray(center, float), np.asarray(xyz, float).reshape(-1, 3),
                         np.asarray(q, float), np.asarray(sigma, float), np.asarray(eps, float),
                         params or synth.Params())


# ------------------------------------------------------------------ constants

def test_C0_matches_its_defining_integral():
    """C0 (area formula) = 1 / int_0^1 int_{B, y3>s} K dy ds, integrated here
    through spherical-cap areas: the part of the sphere |y| = r above y3 = s
    has area 2 pi r (r - s)."""
    inner = lambda s: integrate.quad(
        lambda r: math.sin(math.pi * r) ** 2 * 2 * math.pi * r * (r - s), s, 1.0,
        epsabs=0, epsrel=1e-13)[0]
    total = integrate.quad(inner, 0.0, 1.0, epsabs=0, epsrel=1e-13)[0]
    assert oracle.C0() == pytest.approx(1.0 / total, rel=1e-11)


def test_gauss_legendre_matches_library_rule():
    for m in (2, 5, 16, 32, 64):
        x, w = oracle.gauss_legendre(m)
        xr, wr = np.polynomial.legendre.leggauss(m)
        order = np.argsort(x)
        np.testing.assert_allclose(x[order], xr, atol=1e-14)
        np.testing.assert_allclose(w[order], wr, atol=1e-14)


# ------------------------------------------------------------ surface energy

@pytest.mark.parametrize("rho_s", [1.5, 2.5, 3.0])
@pytest.mark.parametrize("m", [4, 7])
def test_geom_energy_of_a_cube_matches_pair_count(rho_s, m):
    """A solute cube of m^3 cells: the number of (solute j, solvent j+o)
    pairs for offset o is m^3 - prod_i (m - |o_i|), so the surface energy is
    c sum_o K(|o|/rho_s) (m^3 - prod (m - |o_i|)) with c = gamma0 C0 h^6/delta^4."""
    n, h = 16, 0.05
    params = dataclasses.replace(synth.Params(), rho_s=rho_s)
    s = _sys(n, h, [[0, 0, 0]], [0], [0.3], [0.5], params)
    phi = np.ones((n, n, n), np.int8)
    lo = (n - m) // 2
    phi[lo:lo + m, lo:lo + m, lo:lo + m] = -1
    R = math.ceil(rho_s)
    total = 0.0
    for dz in range(-R, R + 1):
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                r = math.sqrt(dx * dx + dy * dy + dz * dz)
                if r == 0 or r >= rho_s:
                    continue
                pairs = m ** 3 - (m - abs(dx)) * (m - abs(dy)) * (m - abs(dz))
                total += math.sin(math.pi * r / rho_s) ** 2 * pairs
    c = params.gamma0 * oracle.C0() * h ** 6 / (rho_s * h) ** 4
    assert s.geom_energy(phi.ravel()) == pytest.approx(c * total, rel=1e-12)


def test_surface_prefactor_is_area_normalised():
    """The discrete surface energy of a sphere approaches gamma0 * 4 pi R^2:
    digitised sphere of radius 0.32 nm at h = 3/64 nm, rho_s = 3."""
    s = _sys(64, 3.0 / 64, [[0, 0, 0]], [0], [0.35], [0.65])
    R = 0.3195045
    phi = s.init_loose(R)
    geom = s.geom_energy(phi)
    assert geom == pytest.approx(4 * math.pi * 17.4 * R * R, rel=0.02)


# ----------------------------------------------------------- density + far field

def _g_sphere(R, sigma, eps, gamma0, rho_w):
    """Closed form G(R) = 4 pi gamma0 R^2 + rho_w int_{|x|>R} U_LJ, for one
    atom at the centre of a spherical solute of radius R."""
    x = sigma / R
    return (4 * math.pi * gamma0 * R * R,
            16 * math.pi * rho_w * eps * sigma ** 3 * (x ** 9 / 9 - x ** 3 / 3))


def test_lj_sphere_energy_closed_form():
    """Single uncharged LJ atom (sigma 0.35 nm, eps 0.65 kJ/mol) at the centre,
    labels = digitised sphere of radius R*: the vdW energy (in-box midpoint
    sum + far field) approaches the closed form, first order in h."""
    R = 0.3195045
    _, vdw_exact = _g_sphere(R, 0.35, 0.65, 17.4, 33.3)
    errs = []
    for n in (32, 64):
        s = _sys(n, 3.0 / n, [[0, 0, 0]], [0], [0.35], [0.65])
        ulj, ucfa = s.density_grid()
        far = s.far_field()
        e = s.energy(s.init_loose(R), ulj, ucfa, far)
        errs.append(abs(e["vdw_in"] + e["vdw_far"] - vdw_exact) / abs(vdw_exact))
    assert errs[1] < 2e-3
    assert errs[1] < errs[0]


def test_born_energy_closed_form():
    """One charge Q at the centre of a spherical solute of radius R: the CFA
    energy is the Born energy (Q^2/(8 pi eps0 R))(1/eps_w - 1/eps_m)."""
    R, Q = 0.4, 1.0
    p = synth.Params()
    born = p.coulomb_k * Q * Q / (2 * R) * (1 / p.eps_w - 1 / p.eps_m)
    s = _sys(96, 3.0 / 96, [[0, 0, 0]], [Q], [0.35], [0.0])
    ulj, ucfa = s.density_grid()
    far = s.far_field()
    e = s.energy(s.init_loose(R), ulj, ucfa, far)
    assert e["elec_in"] + e["elec_far"] == pytest.approx(born, rel=2e-3)


def test_two_charge_cfa_exterior_of_ball_closed_form():
    """Two opposite charges inside a ball of radius R: outside the ball
    E = -grad psi with psi = sum_i Q_i/|x - a_i|, and
    int_{|x|>R} |E|^2 = 4 pi sum_ij Q_i Q_j sum_l (l+1)/(2l+1) (a_i a_j)^l
    P_l(cos angle_ij) / R^(2l+1) (Legendre addition theorem).  A CFA that
    summed |E_i|^2 per atom instead of |sum E_i|^2 would miss the cross terms
    and fail by far more than the tolerance."""
    R = 0.6
    a = np.array([[0.12, 0.0, 0.0], [-0.10, 0.07, 0.0]])
    Q = np.array([1.0, -1.0])
    p = synth.Params()
    ccfa = p.coulomb_k / (8 * math.pi) * (1 / p.eps_w - 1 / p.eps_m)
    total = 0.0
    for i in range(2):
        for j in range(2):
            ai, aj = np.linalg.norm(a[i]), np.linalg.norm(a[j])
            cosg = a[i] @ a[j] / (ai * aj)
            for l in range(80):
                total += Q[i] * Q[j] * (l + 1) / (2 * l + 1) * (ai * aj) ** l * \
                    eval_legendre(l, cosg) / R ** (2 * l + 1)
    exact = ccfa * 4 * math.pi * total
    errs = []
    for n in (48, 96):
        s = _sys(n, 3.0 / n, a, Q, [0.3, 0.3], [0.0, 0.0])
        ulj, ucfa = s.density_grid()
        far = s.far_field()
        e = s.energy(s.init_loose(R), ulj, ucfa, far)
        errs.append(abs(e["elec_in"] + e["elec_far"] - exact) / abs(exact))
    # digitisation error of the ball, first order in h (1.6 %, 0.6 %)
    assert errs[1] < 0.01
    assert errs[1] < 0.6 * errs[0]


def _face_integral(radial, L):
    """int over directions of radial(rho(w)) where rho(w) is the distance
    from the box centre to the cube surface along w; gnomonic coordinates on
    one face, times 6 (cube symmetry of the integrand required)."""
    f = lambda v, u: radial(L * math.sqrt(1 + u * u + v * v)) / (1 + u * u + v * v) ** 1.5
    return 6 * integrate.dblquad(f, -1, 1, -1, 1, epsabs=0, epsrel=1e-11)[0]


def test_far_field_centred_atom_independent_integral():
    """Far field of one atom at the box centre: the radial integrals have
    closed forms, int_rho^inf U_LJ r^2 dr = 4 eps (sigma^12/(9 rho^9) -
    sigma^6/(3 rho^3)) and int_rho^inf Q^2 r^-2 dr = Q^2/rho; the angular
    integral is done adaptively in gnomonic coordinates."""
    sig, eps, Q, L = 0.35, 0.65, 0.7, 1.5
    p = synth.Params()
    ccfa = p.coulomb_k / (8 * math.pi) * (1 / p.eps_w - 1 / p.eps_m)
    lj = p.rho_w * _face_integral(
        lambda r: 4 * eps * (sig ** 12 / (9 * r ** 9) - sig ** 6 / (3 * r ** 3)), L)
    cfa = ccfa * _face_integral(lambda r: Q * Q / r, L)
    s = _sys(64, 2 * L / 64, [[0, 0, 0]], [Q], [sig], [eps])
    far_lj, far_cfa = s.far_field()
    assert far_lj == pytest.approx(lj, rel=1e-9)
    assert far_cfa == pytest.approx(cfa, rel=1e-9)
    # the value quoted for the single-atom workload
    assert far_lj == pytest.approx(-0.11833344, rel=1e-7)


def _shell_exterior(nexp, a, Rb):
    """int_{|x|>Rb} |x - a|^-nexp dV for 0 < |a| < Rb, from the sphere average
    of |x - a|^-n over |x| = rho, ((rho-a)^(2-n) - (rho+a)^(2-n)) / (2 rho a (n-2)),
    integrated in rho with 4 pi rho^2 (substituting s = rho -+ a)."""
    m = nexp - 2
    if m == 2:
        val = math.log((Rb + a) / (Rb - a)) + a / (Rb - a) + a / (Rb + a)
    else:
        first = -((Rb - a) ** (2 - m) / (2 - m) + a * (Rb - a) ** (1 - m) / (1 - m))
        second = -((Rb + a) ** (2 - m) / (2 - m) - a * (Rb + a) ** (1 - m) / (1 - m))
        val = first - second
    return 4 * math.pi / (2 * a * m) * val


def test_far_field_off_centre_atom_independent_integral():
    """Far field of one off-centre charged LJ atom: the exterior of the
    circumscribed ball in closed form (sphere averages), plus the region
    between the cube and that ball by adaptive cubature."""
    sig, eps, Q, L = 0.33, 0.4, -0.6, 1.5
    apos = np.array([0.31, -0.22, 0.17])
    a = float(np.linalg.norm(apos))
    Rb = L * math.sqrt(3.0)
    p = synth.Params()
    ccfa = p.coulomb_k / (8 * math.pi) * (1 / p.eps_w - 1 / p.eps_m)

    def dens(x):
        d = x - apos
        r2 = d @ d
        sr6 = (sig * sig / r2) ** 3
        return p.rho_w * 4 * eps * (sr6 * sr6 - sr6) + ccfa * Q * Q / (r2 * r2)

    outer = p.rho_w * 4 * eps * (sig ** 12 * _shell_exterior(12, a, Rb) -
                                 sig ** 6 * _shell_exterior(6, a, Rb)) + \
        ccfa * Q * Q * _shell_exterior(4, a, Rb)
    inner = 0.0
    for axis in range(3):
        for sgn in (1.0, -1.0):
            def f(r, v, u, axis=axis, sgn=sgn):
                w = np.empty(3)
                w[axis] = sgn
                w[(axis + 1) % 3] = u
                w[(axis + 2) % 3] = v
                nrm = math.sqrt(1 + u * u + v * v)
                w /= nrm
                return dens(r * w) * r * r / nrm ** 3
            inner += integrate.tplquad(
                f, -1, 1, -1, 1, lambda u, v: L * math.sqrt(1 + u * u + v * v),
                lambda u, v: Rb, epsabs=1e-13, epsrel=1e-10)[0]
    s = _sys(64, 2 * L / 64, [apos], [Q], [sig], [eps])
    far_lj, far_cfa = s.far_field()
    assert far_lj + far_cfa == pytest.approx(outer + inner, rel=1e-7)


def test_far_field_converged_in_quadrature_order():
    w = synth.random_small(32, 12, seed=11)
    s = oracle.System.from_workload(w)
    base = np.array(s.far_field())
    w2 = dataclasses.replace(w.params, far_nf=64, far_ntau=32)
    s2 = oracle.System(w.n, w.h, w.center, w.xyz, w.q, w.sigma, w.eps, w2)
    fine = np.array(s2.far_field())
    np.testing.assert_allclose(base, fine, rtol=1e-9)


# ------------------------------------------------------------------ flips

def _tiny_case(seed=3, n=10):
    rng = np.random.default_rng(seed)
    h = 0.1
    xyz = rng.uniform(-0.25, 0.25, size=(4, 3))
    q = np.array([0.3, -0.2, 0.25, -0.35])
    s = _sys(n, h, xyz, q, rng.uniform(0.3, 0.4, 4), rng.uniform(0.1, 0.6, 4))
    phi = np.where(rng.random(n ** 3) < 0.5, -1, 1).astype(np.int8)
    return s, phi


def test_delta_e_equals_energy_difference_of_a_flip():
    """Eqs. dGj1/dGj2 against the change of the full discrete energy,
    recomputed from scratch, for every cell of a random label field."""
    s, phi = _tiny_case()
    ulj, ucfa = s.density_grid()
    u = ulj + ucfa
    far = s.far_field()
    e0 = s.energy(phi, ulj, ucfa, far)["total"]
    scale = abs(e0) + s.h ** 3 * np.abs(u).sum() + s.geom_energy(-np.ones_like(phi))
    for j in range(s.ncell):
        phi2 = phi.copy()
        phi2[j] = -phi2[j]
        de = s.energy(phi2, ulj, ucfa, far)["total"] - e0
        assert s.delta_e(phi, u, j) == pytest.approx(de, abs=1e-12 * scale)


def test_band_is_face_neighbour_disagreement():
    s, phi = _tiny_case(seed=5)
    n = s.n
    g = np.pad(phi.reshape(n, n, n), 1, constant_values=1)
    c = g[1:-1, 1:-1, 1:-1]
    band = np.zeros_like(c, bool)
    for ax in range(3):
        for sh in (-1, 1):
            band |= np.roll(g, sh, axis=ax)[1:-1, 1:-1, 1:-1] != c
    got = np.array([s.in_band(phi, j) for j in range(s.ncell)])
    assert np.array_equal(got, band.ravel())


def test_colour_pass_energy_change_is_sum_of_flip_changes():
    """Cells of one colour lie outside each other's kernel support, so a
    pass changes the energy by exactly the sum of its flips' Delta E, and
    that sum is negative."""
    s, phi = _tiny_case(seed=7, n=12)
    ulj, ucfa = s.density_grid()
    u = ulj + ucfa
    far = s.far_field()
    for sweep in range(3):
        for c in range(s.colours()):
            e0 = s.energy(phi, ulj, ucfa, far)["total"]
            flips, ncand, dsum = s.colour_pass(phi, u, c)
            e1 = s.energy(phi, ulj, ucfa, far)["total"]
            assert e1 - e0 == pytest.approx(dsum, abs=1e-11 * (abs(e0) + 1))
            assert dsum <= 0.0


def test_minimised_labels_are_a_local_minimum():
    """At convergence no band cell can lower the energy by flipping (checked
    by recomputing the full energy), and the energy never rose."""
    w = synth.random_small(14, 5, seed=21, h=0.06)
    s = oracle.System.from_workload(w)
    ulj, ucfa = s.density_grid()
    u = ulj + ucfa
    far = s.far_field()
    phi = s.init_tight()
    e_init = s.energy(phi, ulj, ucfa, far)["total"]
    rc, st, _, _ = s.minimize_colour(phi, u)
    assert rc == 0 and st["converged"] == 1
    e_fin = s.energy(phi, ulj, ucfa, far)["total"]
    assert e_fin <= e_init
    for j in range(s.ncell):
        if not s.in_band(phi, j):
            continue
        phi2 = phi.copy()
        phi2[j] = -phi2[j]
        assert s.energy(phi2, ulj, ucfa, far)["total"] >= e_fin - 1e-12 * abs(e_fin)


@pytest.mark.parametrize("rho_s,n", [(3.0, 40), (3.0, 31), (2.0, 33)])
def test_colour_pass_lists_every_band_cell_of_its_colour(rho_s, n):
    """From random labels, where nearly every cell is in the band, each colour
    pass's candidates are exactly the band cells of that colour, counted here
    with numpy from the definitions (a face neighbour with the other label,
    cells outside the box solvent; colour (x mod p, y mod p, z mod p)), also
    on grids that p = ceil(rho_s) does not divide, where one colour holds
    ceil(n / p)^3 cells."""
    rng = np.random.default_rng(31)
    params = dataclasses.replace(synth.Params(), rho_s=rho_s)
    s = _sys(n, 0.1, rng.uniform(-0.3, 0.3, size=(3, 3)), [0.2, -0.1, -0.1],
             [0.35, 0.3, 0.4], [0.3, 0.4, 0.5], params)
    phi = np.where(rng.random(n ** 3) < 0.4, -1, 1).astype(np.int8)
    u = np.zeros(n ** 3)
    g = np.pad(phi.reshape(n, n, n), 1, constant_values=1)  # [z, y, x], solvent outside
    c = g[1:-1, 1:-1, 1:-1]
    band = np.zeros_like(c, dtype=bool)
    for ax in range(3):
        for sh in (-1, 1):
            band |= np.roll(g, sh, axis=ax)[1:-1, 1:-1, 1:-1] != c
    p = math.ceil(rho_s)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    colour = x % p + p * (y % p) + p * p * (z % p)
    assert s.colours() == p ** 3
    for col in range(p ** 3):
        _, ncand, _ = s.colour_pass(phi.copy(), u, col)
        assert ncand == int((band & (colour == col)).sum()), col


def test_colour_pass_equals_a_serial_pass_in_reverse_order():
    """A colour pass (every band cell of one colour evaluated on the labels at
    the start of the pass, those with Delta E < 0 flipped) equals visiting the
    same candidates one at a time, here in reverse index order, each judged on
    the labels the earlier flips left: cells of one colour lie outside each
    other's kernel support and face neighbourhood, so a flip leaves every
    other candidate's Delta E unchanged (bit for bit) and lowers the energy by
    its own Delta E."""
    s, phi = _tiny_case(seed=9, n=12)
    ulj, ucfa = s.density_grid()
    u = ulj + ucfa
    far = s.far_field()
    L = oracle.lib()
    for c in range(s.colours()):
        ref = phi.copy()
        s.colour_pass(ref, u, c)
        ser = phi.copy()
        cand = [j for j in range(s.ncell) if L.orc_colour_of(s.sref, j) == c and s.in_band(phi, j)]
        for j in reversed(cand):
            d0 = s.delta_e(phi, u, j)
            d = s.delta_e(ser, u, j)
            assert d == d0
            if d < 0:
                e0 = s.energy(ser, ulj, ucfa, far)["total"]
                ser[j] = -ser[j]
                e1 = s.energy(ser, ulj, ucfa, far)["total"]
                assert e1 < e0
                assert e1 - e0 == pytest.approx(d, abs=1e-11 * (abs(e0) + 1))
        assert np.array_equal(ser, ref)
        phi = ref


def test_loose_and_tight_starts_agree_for_a_convex_solute():
    """One atom: the relaxation from a loose sphere and from the tight
    surface (Sec. "Initial surfaces") ends in the same labels."""
    w = synth.single_atom(40)
    s = oracle.System.from_workload(w)
    ulj, ucfa = s.density_grid()
    u = ulj + ucfa
    a = s.init_loose(1.2)
    b = s.init_tight()
    s.minimize_colour(a, u)
    s.minimize_colour(b, u)
    assert np.array_equal(a, b)


def test_loose_start_keeps_a_dry_region_between_separated_atoms():
    """Two LJ atoms 8 A apart (the paper's r0 = 8 A state, its units): from a
    loose sphere enclosing both the relaxation stops in one solute region
    holding both atoms (a dry state), from the tight surface in two separate
    spheres (wet) -- the dependence on the initial surface the paper reports
    for its two plates and the two domains of BphC.  Here the dry state is
    the higher local minimum."""
    from scipy import ndimage
    g = _golden()
    m = g["model"]
    s = _sys(64, 16.0 / 64, g["r0_8"]["final_positions"], [0, 0], [m["sigma"]] * 2,
             [m["eps"]] * 2, synth.paper_units_params())
    ulj, ucfa = s.density_grid()
    u = ulj + ucfa
    far = s.far_field()
    dry = s.init_loose(6.0)
    wet = s.init_tight()
    s.minimize_colour(dry, u)
    s.minimize_colour(wet, u)
    n = s.n
    ndry = ndimage.label(dry.reshape(n, n, n) == -1)[1]
    nwet = ndimage.label(wet.reshape(n, n, n) == -1)[1]
    assert (ndry, nwet) == (1, 2)
    assert s.energy(dry, ulj, ucfa, far)["total"] > s.energy(wet, ulj, ucfa, far)["total"]


def test_heap_and_colour_schedules_agree_on_single_atom():
    w = synth.single_atom(48)
    s = oracle.System.from_workload(w)
    ulj, ucfa = s.density_grid()
    u = ulj + ucfa
    a = s.init_loose(1.2)
    b = a.copy()
    s.minimize_colour(a, u)
    rc, st = s.minimize_heap(b, u, max_flips=s.ncell)
    assert rc == 0
    assert np.array_equal(a, b)


def test_single_atom_minimum_near_closed_form():
    """Single LJ atom, 64^3, loose sphere R0 = 1.2 nm: the minimised discrete
    free energy lies within 1 % of the closed-form minimum
    min_R [4 pi gamma0 R^2 + 16 pi rho_w eps sigma^3 (x^9/9 - x^3/3)]."""
    res = minimize_scalar(lambda R: sum(_g_sphere(R, 0.35, 0.65, 17.4, 33.3)),
                          bounds=(0.2, 0.6), method="bounded", options={"xatol": 1e-10})
    w = synth.single_atom(64)
    s = oracle.System.from_workload(w)
    ulj, ucfa = s.density_grid()
    far = s.far_field()
    phi = s.init_loose(1.2)
    s.minimize_colour(phi, ulj + ucfa)
    e = s.energy(phi, ulj, ucfa, far)
    assert res.fun == pytest.approx(13.654430, rel=1e-6)
    assert e["total"] == pytest.approx(res.fun, rel=0.01)


def _golden():
    with open(os.path.join(HERE, "golden", "two_atom_tables.json")) as f:
        return json.load(f)


def test_paper_two_atom_energy_matches_closed_form():
    """Table for r0 = 8 A prints G = 33.93 k_B T for two separated atoms.
    With the paper's constants (Table "Model parameters") two isolated LJ
    spheres give 2 min_R G(R); agreement pins the reading of the units
    (gamma0 in k_B T/A^2, rho_w in A^-3, the 4 eps LJ convention)."""
    g = _golden()
    m = g["model"]
    res = minimize_scalar(
        lambda R: sum(_g_sphere(R, m["sigma"], m["eps"], m["gamma0"], m["rho_w"])),
        bounds=(2.0, 6.0), method="bounded", options={"xatol": 1e-10})
    assert 2 * res.fun == pytest.approx(g["r0_8"]["free_energy"], rel=1e-3)


def test_paper_two_atom_energy_oracle():
    """The oracle's discrete minimum for the r0 = 8 A two-atom state (atoms
    fixed at +-4 A, box (-8, 8)^3 A, 64^3 cells, tight start) lies within 3 %
    of the printed 33.93 k_B T (grid and kernel radius of the paper's run are
    not stated, so only this discretisation-level agreement is asserted)."""
    g = _golden()
    m = g["model"]
    s = _sys(64, 16.0 / 64, g["r0_8"]["final_positions"], [0, 0], [m["sigma"]] * 2,
             [m["eps"]] * 2, synth.paper_units_params())
    ulj, ucfa = s.density_grid()
    far = s.far_field()
    phi = s.init_tight()
    s.minimize_colour(phi, ulj + ucfa)
    e = s.energy(phi, ulj, ucfa, far)
    assert e["total"] == pytest.approx(g["r0_8"]["free_energy"], rel=0.03)


# ------------------------------------------------------------- invariances

def test_integer_cell_translation_invariance():
    w = synth.random_small(16, 6, seed=31, h=0.06)
    s = oracle.System.from_workload(w)
    shift = np.array([2, -1, 3]) * w.h
    t = oracle.System(w.n, w.h, w.center + shift, w.xyz + shift, w.q, w.sigma, w.eps, w.params)
    phi = s.init_tight()
    phit = t.init_tight()
    assert np.array_equal(phi, phit)
    a = s.density_grid()
    b = t.density_grid()
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=1e-11, atol=1e-9 * np.abs(x).max())
    ea = s.energy(phi, *a, s.far_field())["total"]
    eb = t.energy(phit, *b, t.far_field())["total"]
    assert ea == pytest.approx(eb, rel=1e-11)


def _cube_maps():
    """A few of the 48 signed axis permutations (rotations and reflections)."""
    return [((0, 1, 2), (1, 1, 1)), ((1, 0, 2), (1, -1, 1)), ((2, 0, 1), (1, 1, 1)),
            ((0, 2, 1), (-1, 1, -1)), ((1, 2, 0), (-1, -1, 1)), ((0, 1, 2), (-1, -1, -1))]


def test_cube_symmetry_invariance_of_energy_and_forces():
    w = synth.random_small(16, 6, seed=41, h=0.06)
    s = oracle.System.from_workload(w)
    phi = s.init_tight()
    e0 = s.total_energy(phi)["total"]
    f0 = s.forces(phi)
    n = w.n
    for perm, sgn in _cube_maps():
        M = np.zeros((3, 3))
        for i in range(3):
            M[i, perm[i]] = sgn[i]
        xyz = w.xyz @ M.T
        t = oracle.System(n, w.h, w.center, xyz, w.q, w.sigma, w.eps, w.params)
        # label of new cell x' = M x is the old label at x = M^T x'
        g = phi.reshape(n, n, n).transpose(2, 1, 0)          # g[i, j, k]
        gn = np.empty_like(g)
        idx = np.indices((n, n, n)).reshape(3, -1)          # new (i, j, k)
        centred = 2 * idx - (n - 1)                           # 2 * offset from centre
        old = (M.T.astype(np.int64) @ centred + (n - 1)) // 2
        gn[tuple(idx)] = g[tuple(old)]
        phin = np.ascontiguousarray(gn.transpose(2, 1, 0)).ravel()
        assert t.total_energy(phin)["total"] == pytest.approx(e0, rel=1e-11)
        np.testing.assert_allclose(t.forces(phin), f0 @ M.T, rtol=1e-8,
                                   atol=1e-9 * np.abs(f0).max())


def test_rotation_leaves_density_pointwise_invariant():
    w = synth.random_small(16, 8, seed=51, h=0.06)
    s = oracle.System.from_workload(w)
    rng = np.random.default_rng(0)
    A = rng.normal(size=(3, 3))
    Qm, _ = np.linalg.qr(A)
    t = oracle.System(w.n, w.h, w.center, w.xyz @ Qm.T, w.q, w.sigma, w.eps, w.params)
    pts = rng.uniform(-0.5, 0.5, size=(200, 3))
    a = s.density_points(pts, efield=True)
    b = t.density_points(pts @ Qm.T, efield=True)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-10)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-10)
    np.testing.assert_allclose(a[2] @ Qm.T, b[2], rtol=1e-9, atol=1e-9)


def test_tight_start_of_centred_atom_is_the_loose_sphere():
    s = _sys(32, 0.05, [[0, 0, 0]], [0], [0.37], [0.5])
    assert np.array_equal(s.init_tight(np.array([0.37])), s.init_loose(0.37))


# --------------------------------------------------------------- forces

def test_forces_match_central_differences():
    """Forces at fixed labels against central differences of the full
    discrete energy (in-box sum, far field and harmonic bonds), step 1e-4 nm."""
    w = synth.random_small(16, 5, seed=61, h=0.07)
    bonds = np.array([[0, 1], [1, 2], [3, 4]], np.int32)
    s = oracle.System(w.n, w.h, w.center, w.xyz, w.q, w.sigma, w.eps, w.params, bonds,
                      np.array([0.15, 0.2, 0.3]), np.array([1e3, 5e2, 2e3]))
    phi = s.init_tight()
    f = s.forces(phi)
    hfd = 1e-4
    fd = np.zeros_like(f)
    for a in range(w.natoms):
        for d in range(3):
            xp = w.xyz.copy()
            xp[a, d] += hfd
            xm = w.xyz.copy()
            xm[a, d] -= hfd
            ep = s.with_positions(xp).total_energy(phi)["total"]
            em = s.with_positions(xm).total_energy(phi)["total"]
            fd[a, d] = -(ep - em) / (2 * hfd)
    np.testing.assert_allclose(f, fd, rtol=1e-5, atol=1e-6 * np.abs(f).max())


def test_forces_subset_equals_the_rows_of_the_full_forces():
    """The per-atom force sum used on large grids (field given per cell, its
    own far-field, bond and solute-solute loops) equals the rows of the full
    force sum, itself pinned by central differences, to 1e-12 relative.  A
    charged, bonded chain with bending, torsion and non-bonded terms; the
    sample lists atoms out of order and holds both chain ends and interior
    atoms, so each atom is the first and the second atom of some bond."""
    natoms = 8
    xyz = synth.globule(natoms, seed=84) * 1.5
    w = synth.random_small(16, natoms, seed=84, h=0.07)
    top = synth.chain_topology([(0, natoms)], seed=84, exclude=1)
    ss = oracle.SoluteTerms(top.angles, top.theta0, top.k_angle, top.torsions, top.c, top.psi,
                            True, None, None, top.exclusions)
    bonds, r0, kb = synth.chain_bonds(natoms)
    s = oracle.System(w.n, w.h, w.center, xyz, w.q, w.sigma, w.eps, w.params, bonds, r0,
                      kb * 1e-2, ss)
    phi = s.init_tight()
    assert 0 < np.count_nonzero(phi == -1) < phi.size
    f = s.forces(phi)
    _, _, e = s.density_grid(efield=True)
    sel = np.array([natoms - 1, 3, 0, 5, 1])
    fs = s.forces_subset(phi, e, sel)
    scale = np.linalg.norm(f, axis=1).max()
    assert np.abs(fs - f[sel]).max() <= 1e-12 * scale, np.abs(fs - f[sel]).max() / scale


# ------------------------------------------------------------ atom step

def test_adaptive_mobility_relaxes_a_bond_to_its_rest_length():
    """Two atoms with the solvent switched off (rho_w = 0, no charge): the
    adaptive-mobility descent drives the bond to r0."""
    p = dataclasses.replace(synth.Params(), rho_w=0.0)
    xyz = np.array([[-0.25, 0.0, 0.0], [0.25, 0.0, 0.0]])
    s = oracle.System(16, 0.1, np.zeros(3), xyz, [0, 0], [0.3, 0.3], [0.5, 0.5], p,
                      np.array([[0, 1]], np.int32), np.array([0.3]), np.array([1e3]))
    phi = s.init_tight()
    mob = oracle.default_mobility(dt=0.1)
    x = xyz.copy()
    for _ in range(200):
        rc, x, info = s.atom_step(x, phi, mob)
        if rc != 0:
            break
    assert np.linalg.norm(x[0] - x[1]) == pytest.approx(0.3, abs=1e-6)


def test_adaptive_mobility_shrinks_after_an_overshoot():
    """A step far too long raises the energy by more than 5 %: the trial is
    rejected, M shrinks by alpha = 1/sqrt 2 and N_cnt resets (Step 3.4)."""
    p = dataclasses.replace(synth.Params(), rho_w=0.0)
    xyz = np.array([[-0.16, 0.0, 0.0], [0.16, 0.0, 0.0]])
    s = oracle.System(16, 0.1, np.zeros(3), xyz, [0, 0], [0.3, 0.3], [0.5, 0.5], p,
                      np.array([[0, 1]], np.int32), np.array([0.3]), np.array([1e3]))
    phi = s.init_tight()
    mob = oracle.default_mobility(dt=0.1)
    mob.M = 8.0
    mob.N_cnt = 3
    rc, x, info = s.atom_step(xyz.copy(), phi, mob)
    assert rc == 0 and info.accepted == 1
    assert info.retries >= 1
    assert mob.M == pytest.approx(8.0 * (2 ** -0.5) ** info.retries)
    assert mob.N_cnt == 1
    assert info.G_new <= info.G_old + 0.05 * abs(info.G_old)


# ------------------------------------------------------- full alternation

@pytest.mark.parametrize("case", ["r0_8", "r0_3"])
def test_paper_two_atom_relaxation_reaches_printed_state(case):
    """Steps 2-5 of the algorithm on the paper's two-atom molecule (Tables
    for experiments 1.1 and 1.2): starting 14 A apart, the alternation of
    interface sweeps and adaptive-mobility atom steps ends with the bond at
    the printed length, the atoms placed symmetrically about the box centre
    as printed, and G within 3 % of the printed free energy (the paper's
    grid is not stated; here 48^3 cells over (-8, 8)^3 A)."""
    g = _golden()
    m = g["model"]
    r0 = g[case]["bond_length"]
    xyz = np.array([[7.0, 0.0, 0.0], [-7.0, 0.0, 0.0]])
    s = oracle.System(48, 16.0 / 48, np.zeros(3), xyz, [0, 0], [m["sigma"]] * 2, [m["eps"]] * 2,
                      synth.paper_units_params(), np.array([[0, 1]], np.int32),
                      np.array([r0]), np.array([m["bond_A"]]))
    phi = s.init_tight()
    x = xyz.copy()
    opts = oracle.RelaxOpts(max_iters=3000, persist=100, max_sweeps=10000, pad=0,
                            tol_grad=1e-4, tol_energy=1e-5)
    rc, rep = s.relax(x, phi, opts, oracle.default_mobility(dt=1.0))
    assert rc == 0 and rep.stop_reason in (1, 2)
    assert np.linalg.norm(x[0] - x[1]) == pytest.approx(r0, abs=0.02)
    np.testing.assert_allclose(x, g[case]["final_positions"], atol=0.05)
    assert rep.G_final == pytest.approx(g[case]["free_energy"], rel=0.03)
