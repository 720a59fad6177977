/*
 * VESIS oracle: a plain, slow, FP64 CPU implementation of the VESIS hot path
 * (arXiv 2208.05524, "Sec. Numerical Methods" and the Appendix).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header, table or constant generator with
 * the HIP path.  Every function below states the passage of the paper it
 * writes out.  Loops are the definitions themselves: no blocking, no fusion,
 * no reordering beyond what the definition states.  OpenMP is used only
 * across independent cells or atoms; every sum is an FP64 sum in a fixed
 * order (index order, or per z-plane and then the planes in order).
 *
 * Readings of the paper taken here (the paper is silent or garbled at these
 * points):
 *   - the kernel radius is parameterised as rho_s = delta / h (the paper's
 *     delta = lambda sqrt(h) never fixes lambda); the support is the open
 *     ball |x_k - x_j| < delta (K vanishes on its boundary);
 *   - the surface kernel is evaluated at (x_j - x_k)/delta, as in the
 *     continuous area formula, and the flip energy uses h^3 U(x_j), the
 *     midpoint-rule weight of the discrete energy;
 *   - cells outside the box count as solvent (+1) and never flip;
 *   - r^2 = |x - r_i|^2 is floored at r2_min so a cell centre sitting on an
 *     atom stays finite;
 *   - the far-field integral over R^3 minus the box uses the face-cone
 *     parameterisation p = c + (y - c)/tau (y on a face, tau in (0,1]) with
 *     Gauss-Legendre rules in (u, v, tau);
 *   - the flip schedule compared bit for bit with the GPU is the colour
 *     schedule (orc_minimize_colour); the paper's min-heap descent is kept as
 *     orc_minimize_heap and compared by energy only;
 *   - forces are minus the exact gradient of the discrete energy at fixed
 *     labels (in-box midpoint sum + far-field quadrature + bonds + the
 *     solute-solute terms);
 *   - solute-solute LJ pairs mix by sigma_ij = (sigma_i + sigma_j)/2 and
 *     eps_ij = sqrt(eps_i eps_j); the non-bonded pairs are all pairs not on
 *     an explicit exclusion list; the torsion angle is unsigned, tau in
 *     [0, pi], and psi_n is 0 or pi (the Appendix's gradient assumes this);
 *   - the adaptive-mobility step follows Step 3.3-3.4 of the algorithm with
 *     delta G* = dG_frac * |G_old|.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int32_t n;          /* cells per box edge */
    int32_t far_nf;     /* Gauss-Legendre nodes per face axis (far field) */
    int32_t far_ntau;   /* Gauss-Legendre nodes in tau (far field) */
    int32_t pad0;
    double center[3];   /* box centre c; the box is (c - L, c + L)^3 */
    double h;           /* cell edge; L = n h / 2 */
    int64_t na;         /* number of atoms */
    const double* xyz;  /* na x 3 atom positions */
    const double* q;    /* partial charges Q_i */
    const double* sigma;/* solute-water LJ sigma_i */
    const double* eps;  /* solute-water LJ epsilon_i */
    double rho_w;       /* solvent number density */
    double gamma0;      /* surface tension */
    double eps_m;       /* solute relative permittivity */
    double eps_w;       /* solvent relative permittivity */
    double coulomb_k;   /* 1 / (4 pi eps0) */
    double rho_s;       /* delta / h */
    double r2_min;      /* floor on |x - r_i|^2 */
    const struct orc_ss* ss; /* solute-solute terms beyond bonds, or NULL */
} orc_sys;

/* Solute-solute terms of Eq. "Gss" beyond the bonds (which are passed to the
 * energy and force calls directly):
 *   bending   sum over triplets (i, j, k) of (1/2) B (theta_ijk - theta0)^2,
 *             theta_ijk the angle at j between r_i - r_j and r_k - r_j;
 *   torsion   sum over quadruples (i, j, k, l) of
 *             sum_{n=0..6} C_n [1 + cos(n tau - psi_n)], tau in [0, pi] the
 *             angle between the planes (i, j, k) and (j, k, l);
 *   LJ, Coulomb over the pairs i < j not listed in excl:
 *             4 eps_ij [(sigma_ij/r)^12 - (sigma_ij/r)^6] with
 *             sigma_ij = (sigma_i + sigma_j)/2, eps_ij = sqrt(eps_i eps_j),
 *             and coulomb_k Q_i Q_j / (eps_w r). */
typedef struct orc_ss {
    int64_t nang;
    const int32_t* ang;     /* nang x 3: i, j (vertex), k */
    const double* theta0;   /* equilibrium angle, radians */
    const double* kang;     /* B */
    int64_t ntor;
    const int32_t* tor;     /* ntor x 4: i, j, k, l */
    const double* tc;       /* ntor x 7: C_0 .. C_6 */
    const double* tpsi;     /* ntor x 7: psi_0 .. psi_6, each 0 or pi */
    int32_t nonbonded;      /* nonzero: include the LJ and Coulomb pair terms */
    int32_t pad;
    const double* sigma_ss; /* per-atom solute-solute LJ sigma */
    const double* eps_ss;   /* per-atom solute-solute LJ epsilon */
    int64_t nexcl;
    const int32_t* excl;    /* nexcl x 2 excluded pairs (any order) */
} orc_ss;

/* ------------------------------------------------------------- constants */

/* C0 of the area formula (Sec. "Approximation of the surface energy"):
 * C0^-1 = int_0^1 int_{B(0,1), y3 > s} K(y) dy ds.  Exchanging the order of
 * integration, int_0^1 [y3 > s] ds = y3, so C0^-1 = int_{B, y3>0} K(y) y3 dy
 * = pi int_0^1 r^3 sin^2(pi r) dr = (pi^2 - 3) / (8 pi). */
double orc_C0(void) { return 8.0 * M_PI / (M_PI * M_PI - 3.0); }

/* The kernel K(x) = sin^2(pi |x|) for |x| <= 1, else 0 (same section). */
static double kernel_K(double r) {
    if (r > 1.0) return 0.0;
    double s = sin(M_PI * r);
    return s * s;
}

/* Prefactor of the discrete surface energy, gamma0 C0 h^4 / lambda^4 with
 * delta = lambda sqrt(h), i.e. gamma0 C0 h^6 / delta^4 (Eq. "4flip"). */
double orc_surface_prefactor(const orc_sys* s) {
    double delta = s->rho_s * s->h;
    return s->gamma0 * orc_C0() * pow(s->h, 6) / pow(delta, 4);
}

/* CFA prefactor 1/(32 pi^2 eps0) (1/eps_w - 1/eps_m), Eq. "G_VISM";
 * 1/(32 pi^2 eps0) = (1/(4 pi eps0)) / (8 pi). */
double orc_cfa_prefactor(const orc_sys* s) {
    return s->coulomb_k / (8.0 * M_PI) * (1.0 / s->eps_w - 1.0 / s->eps_m);
}

/* ------------------------------------------------------------------ grid */

/* Cell-centred uniform grid of the box (Sec. "A Binary Level-Set Method"):
 * cell (i,j,k) has centre c - L + (i + 1/2, j + 1/2, k + 1/2) h, linear index
 * i + n (j + n k). */
void orc_cell_center(const orc_sys* s, int64_t idx, double x[3]) {
    int64_t n = s->n;
    int64_t i = idx % n, j = (idx / n) % n, k = idx / (n * n);
    double L = 0.5 * (double)n * s->h;
    x[0] = s->center[0] - L + ((double)i + 0.5) * s->h;
    x[1] = s->center[1] - L + ((double)j + 0.5) * s->h;
    x[2] = s->center[2] - L + ((double)k + 0.5) * s->h;
}

/* Label of cell (i,j,k); cells outside the box are solvent (+1). */
static int label_at(const orc_sys* s, const int8_t* phi, int64_t i, int64_t j, int64_t k) {
    int64_t n = s->n;
    if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) return 1;
    return phi[i + n * (j + n * k)];
}

/* --------------------------------------------------------------- density */

/* Energy density U(x) of Eq. "Ur": rho_w sum_i U_LJ^(i)(|x - r_i|) plus the
 * CFA term, with U_LJ(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6]
 * (Eq. "eq:LJpotential") and the field E(x) = sum_i Q_i (x - r_i)/|x - r_i|^3.
 * Returns the LJ part, the CFA part and E. */
void orc_density_point(const orc_sys* s, const double x[3], double* u_lj, double* u_cfa,
                       double e[3]) {
    double lj = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    for (int64_t i = 0; i < s->na; ++i) {
        double dx = x[0] - s->xyz[3 * i + 0];
        double dy = x[1] - s->xyz[3 * i + 1];
        double dz = x[2] - s->xyz[3 * i + 2];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < s->r2_min) r2 = s->r2_min;
        double r = sqrt(r2);
        double sr = s->sigma[i] / r;
        double sr6 = sr * sr * sr * sr * sr * sr;
        lj += 4.0 * s->eps[i] * (sr6 * sr6 - sr6);
        double f = s->q[i] / (r2 * r);
        ex += f * dx;
        ey += f * dy;
        ez += f * dz;
    }
    *u_lj = s->rho_w * lj;
    *u_cfa = orc_cfa_prefactor(s) * (ex * ex + ey * ey + ez * ez);
    if (e) { e[0] = ex; e[1] = ey; e[2] = ez; }
}

void orc_density_points(const orc_sys* s, int64_t np, const double* pts, double* u_lj,
                        double* u_cfa, double* e) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < np; ++p)
        orc_density_point(s, pts + 3 * p, u_lj + p, u_cfa + p, e ? e + 3 * p : NULL);
}

void orc_density_grid(const orc_sys* s, double* u_lj, double* u_cfa, double* e) {
    int64_t ncell = (int64_t)s->n * s->n * s->n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = 0; c < ncell; ++c) {
        double x[3];
        orc_cell_center(s, c, x);
        orc_density_point(s, x, u_lj + c, u_cfa + c, e ? e + 3 * c : NULL);
    }
}

/* ------------------------------------------------------------- far field */

/* Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on the
 * three-term Legendre recurrence). */
void orc_gauss_legendre(int m, double* x, double* w) {
    for (int i = 0; i < m; ++i) {
        double z = cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= m; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= m; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = m * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Quadrature nodes for int_{R^3 \ box} f dV (last term of Eq. "4flip").
 * Every point outside the box is p = c + (y - c)/tau with y on one face and
 * tau in (0, 1); for the face x = c_x + L, y = c + (L, u, v) and
 * dV = L tau^-4 du dv dtau.  Gauss-Legendre in u, v on [-L, L] (far_nf nodes)
 * and in tau on (0, 1) (far_ntau nodes).  Writes 6 nf^2 ntau points and
 * weights; returns the count. */
int64_t orc_far_nodes(const orc_sys* s, double* pts, double* wts) {
    int nf = s->far_nf, nt = s->far_ntau;
    double* gx = malloc(sizeof(double) * nf);
    double* gw = malloc(sizeof(double) * nf);
    double* tx = malloc(sizeof(double) * nt);
    double* tw = malloc(sizeof(double) * nt);
    orc_gauss_legendre(nf, gx, gw);
    orc_gauss_legendre(nt, tx, tw);
    double L = 0.5 * (double)s->n * s->h;
    int64_t m = 0;
    for (int face = 0; face < 6; ++face) {
        int axis = face / 2;
        double sgn = (face % 2 == 0) ? 1.0 : -1.0;
        int a1 = (axis + 1) % 3, a2 = (axis + 2) % 3;
        for (int it = 0; it < nt; ++it) {
            double tau = 0.5 * (tx[it] + 1.0);
            double wt = 0.5 * tw[it];
            for (int iv = 0; iv < nf; ++iv) {
                for (int iu = 0; iu < nf; ++iu) {
                    double y[3];
                    y[axis] = sgn * L;
                    y[a1] = L * gx[iu];
                    y[a2] = L * gx[iv];
                    for (int d = 0; d < 3; ++d) pts[3 * m + d] = s->center[d] + y[d] / tau;
                    wts[m] = (L * gw[iu]) * (L * gw[iv]) * wt * L / (tau * tau * tau * tau);
                    ++m;
                }
            }
        }
    }
    free(gx); free(gw); free(tx); free(tw);
    return m;
}

/* F_far = int_{R^3 \ box} U dV, split into its LJ and CFA parts. */
void orc_far_field(const orc_sys* s, double out[2]) {
    int64_t m = 6LL * s->far_nf * s->far_nf * s->far_ntau;
    double* pts = malloc(sizeof(double) * 3 * m);
    double* w = malloc(sizeof(double) * m);
    double* ulj = malloc(sizeof(double) * m);
    double* ucfa = malloc(sizeof(double) * m);
    orc_far_nodes(s, pts, w);
    orc_density_points(s, m, pts, ulj, ucfa, NULL);
    double a = 0.0, b = 0.0;
    for (int64_t p = 0; p < m; ++p) {
        a += w[p] * ulj[p];
        b += w[p] * ucfa[p];
    }
    out[0] = a;
    out[1] = b;
    free(pts); free(w); free(ulj); free(ucfa);
}

/* ---------------------------------------------------------------- energy */

/* Discrete surface energy, first term of Eq. "4flip":
 * gamma0 C0 h^4/lambda^4 sum_{x_j in solute} sum_{x_k in solvent,
 * |x_k - x_j| < delta} K((x_j - x_k)/delta). */
double orc_geom_energy(const orc_sys* s, const int8_t* phi) {
    int64_t n = s->n;
    double h = s->h, delta = s->rho_s * s->h;
    int R = (int)ceil(s->rho_s);
    /* one sequential partial sum per z-plane (planes in parallel), then the
     * planes in order: a fixed summation order */
    double* plane = calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n; ++k) {
        double sum = 0.0;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) {
                if (phi[i + n * (j + n * k)] != -1) continue;
                for (int dz = -R; dz <= R; ++dz)
                    for (int dy = -R; dy <= R; ++dy)
                        for (int dx = -R; dx <= R; ++dx) {
                            double d = h * sqrt((double)(dx * dx + dy * dy + dz * dz));
                            if (d == 0.0 || !(d < delta)) continue;
                            if (label_at(s, phi, i + dx, j + dy, k + dz) == 1)
                                sum += kernel_K(d / delta);
                        }
            }
        plane[k] = sum;
    }
    double sum = 0.0;
    for (int64_t k = 0; k < n; ++k) sum += plane[k];
    free(plane);
    return orc_surface_prefactor(s) * sum;
}

/* Discrete VISM energy of Eq. "4flip" with its parts reported separately
 * (the paper's tables list surface, vdW and CFA energies):
 * out = {geom, vdw_in, vdw_far, elec_in, elec_far, total}.
 * In-box integrals use the midpoint rule h^3 sum_{x_j in solvent} U(x_j). */
void orc_energy(const orc_sys* s, const int8_t* phi, const double* u_lj, const double* u_cfa,
                const double far[2], double out[6]) {
    int64_t ncell = (int64_t)s->n * s->n * s->n;
    double h3 = s->h * s->h * s->h;
    double a = 0.0, b = 0.0;
    for (int64_t c = 0; c < ncell; ++c) {
        if (phi[c] != 1) continue;
        a += u_lj[c];
        b += u_cfa[c];
    }
    out[0] = orc_geom_energy(s, phi);
    out[1] = h3 * a;
    out[2] = far[0];
    out[3] = h3 * b;
    out[4] = far[1];
    out[5] = out[0] + out[1] + out[2] + out[3] + out[4];
}

/* Harmonic bond energy, first term of Eq. "Gss": sum (1/2) A_ij (r_ij - r0_ij)^2. */
double orc_bond_energy(int64_t nb, const int32_t* ij, const double* r0, const double* kb,
                       const double* xyz) {
    double e = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        const double* p = xyz + 3 * ij[2 * b];
        const double* q = xyz + 3 * ij[2 * b + 1];
        double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        e += 0.5 * kb[b] * (r - r0[b]) * (r - r0[b]);
    }
    return e;
}

/* ------------------------------------------------- solute-solute terms */

static void sub3(const double* a, const double* b, double* o) {
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Bending angle theta_ijk at vertex j (second term of Eq. "Gss"). */
static double bend_angle(const double* ri, const double* rj, const double* rk) {
    double qji[3], qjk[3];
    sub3(ri, rj, qji);
    sub3(rk, rj, qjk);
    double c = dot3(qji, qjk) / (sqrt(dot3(qji, qji)) * sqrt(dot3(qjk, qjk)));
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    return acos(c);
}

/* cos tau of quadruple (i, j, k, l): Lambda = u.v / (|u| |v|), u = q1 x q2,
 * v = q2 x q3 with q1 = r_j - r_i, q2 = r_k - r_j, q3 = r_l - r_k (Appendix,
 * "Force calculations of molecular mechanical interactions"). */
static double torsion_cos(const double* ri, const double* rj, const double* rk, const double* rl) {
    double q1[3], q2[3], q3[3], u[3], v[3];
    sub3(rj, ri, q1);
    sub3(rk, rj, q2);
    sub3(rl, rk, q3);
    cross3(q1, q2, u);
    cross3(q2, q3, v);
    double c = dot3(u, v) / (sqrt(dot3(u, u)) * sqrt(dot3(v, v)));
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    return c;
}

/* Sum over triplets of (1/2) B (theta - theta0)^2. */
double orc_bend_energy(const orc_ss* t, const double* xyz) {
    double e = 0.0;
    for (int64_t a = 0; a < t->nang; ++a) {
        const int32_t* id = t->ang + 3 * a;
        double th = bend_angle(xyz + 3 * id[0], xyz + 3 * id[1], xyz + 3 * id[2]);
        e += 0.5 * t->kang[a] * (th - t->theta0[a]) * (th - t->theta0[a]);
    }
    return e;
}

/* Sum over quadruples of sum_n C_n [1 + cos(n tau - psi_n)], tau = acos Lambda. */
double orc_torsion_energy(const orc_ss* t, const double* xyz) {
    double e = 0.0;
    for (int64_t a = 0; a < t->ntor; ++a) {
        const int32_t* id = t->tor + 4 * a;
        double tau = acos(torsion_cos(xyz + 3 * id[0], xyz + 3 * id[1], xyz + 3 * id[2],
                                      xyz + 3 * id[3]));
        for (int n = 0; n <= 6; ++n)
            e += t->tc[7 * a + n] * (1.0 + cos(n * tau - t->tpsi[7 * a + n]));
    }
    return e;
}

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* Sorted keys min(i,j) * na + max(i,j) of the excluded pairs. */
static int64_t* exclusion_keys(const orc_ss* t, int64_t na) {
    int64_t* k = malloc(sizeof(int64_t) * (size_t)(t->nexcl > 0 ? t->nexcl : 1));
    for (int64_t e = 0; e < t->nexcl; ++e) {
        int64_t i = t->excl[2 * e], j = t->excl[2 * e + 1];
        k[e] = (i < j ? i : j) * na + (i < j ? j : i);
    }
    qsort(k, (size_t)t->nexcl, sizeof(int64_t), cmp_i64);
    return k;
}

static int excluded(const int64_t* keys, int64_t nkeys, int64_t na, int64_t i, int64_t j) {
    int64_t key = (i < j ? i : j) * na + (i < j ? j : i);
    return bsearch(&key, keys, (size_t)nkeys, sizeof(int64_t), cmp_i64) != NULL;
}

/* LJ (u[0]) and Coulomb (u[1]) energy of one non-bonded pair, and
 * dU/dr / r of their sum (the last two terms of Eq. "Gss"). */
static void pair_terms(const orc_sys* s, int64_t i, int64_t j, double r2, double* u, double* du) {
    const orc_ss* t = s->ss;
    double sg = 0.5 * (t->sigma_ss[i] + t->sigma_ss[j]);
    double ep = sqrt(t->eps_ss[i] * t->eps_ss[j]);
    double r = sqrt(r2);
    double sr6 = pow(sg / r, 6.0);
    double kq = s->coulomb_k * s->q[i] * s->q[j] / s->eps_w;
    u[0] = 4.0 * ep * (sr6 * sr6 - sr6);
    u[1] = kq / r;
    /* d/dr of 4 eps (sr^12 - sr^6) = 4 eps (-12 sr^12 + 6 sr^6) / r */
    *du = (4.0 * ep * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r - kq / r2) / r;
}

/* LJ (out[0]) and Coulomb (out[1]) sums over non-excluded pairs i < j; the
 * row sums of each i are added in index order. */
void orc_nonbonded_energy(const orc_sys* s, double* out) {
    const orc_ss* t = s->ss;
    out[0] = out[1] = 0.0;
    if (!t || !t->nonbonded) return;
    int64_t na = s->na;
    int64_t* keys = exclusion_keys(t, na);
    double* row = calloc((size_t)(2 * na), sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < na; ++i) {
        for (int64_t j = i + 1; j < na; ++j) {
            if (excluded(keys, t->nexcl, na, i, j)) continue;
            double d[3], u[2], du;
            sub3(s->xyz + 3 * i, s->xyz + 3 * j, d);
            pair_terms(s, i, j, dot3(d, d), u, &du);
            row[2 * i] += u[0];
            row[2 * i + 1] += u[1];
        }
    }
    for (int64_t i = 0; i < na; ++i) {
        out[0] += row[2 * i];
        out[1] += row[2 * i + 1];
    }
    free(row);
    free(keys);
}

/* g (na x 3) += grad of the bending, torsion and non-bonded terms, as the
 * Appendix writes them: for the bend, B (theta - theta0) grad theta with
 *   grad_i theta = (cos theta q_ji / q_ji^2 - q_jk / (q_ji q_jk)) / sin theta,
 *   grad_k theta = (cos theta q_jk / q_jk^2 - q_ji / (q_ji q_jk)) / sin theta,
 *   grad_j theta = -(grad_i theta + grad_k theta)
 * (the printed grad_k carries q_ji where the derivative has q_jk; the
 * printed grad_j equals the sum form used here); for the torsion,
 *   dW/dLambda grad Lambda with dW/dLambda the polynomial in Lambda of the
 *   Appendix (psi_n in {0, pi}) and grad Lambda from grad_{q1,q2,q3} Lambda;
 * for the pairs, U'(r) (r_i - r_j)/r on i and its negative on j. */
void orc_ss_gradient(const orc_sys* s, double* g) {
    const orc_ss* t = s->ss;
    if (!t) return;
    const double* x = s->xyz;
    for (int64_t a = 0; a < t->nang; ++a) {
        const int32_t* id = t->ang + 3 * a;
        double qji[3], qjk[3];
        sub3(x + 3 * id[0], x + 3 * id[1], qji);
        sub3(x + 3 * id[2], x + 3 * id[1], qjk);
        double lji = sqrt(dot3(qji, qji)), ljk = sqrt(dot3(qjk, qjk));
        double th = bend_angle(x + 3 * id[0], x + 3 * id[1], x + 3 * id[2]);
        double c = cos(th), sn = sin(th);
        double pre = t->kang[a] * (th - t->theta0[a]) / sn;
        for (int d = 0; d < 3; ++d) {
            double gi = pre * (c * qji[d] / (lji * lji) - qjk[d] / (lji * ljk));
            double gk = pre * (c * qjk[d] / (ljk * ljk) - qji[d] / (lji * ljk));
            g[3 * id[0] + d] += gi;
            g[3 * id[2] + d] += gk;
            g[3 * id[1] + d] -= gi + gk;
        }
    }
    for (int64_t a = 0; a < t->ntor; ++a) {
        const int32_t* id = t->tor + 4 * a;
        double q1[3], q2[3], q3[3], u[3], v[3];
        sub3(x + 3 * id[1], x + 3 * id[0], q1);
        sub3(x + 3 * id[2], x + 3 * id[1], q2);
        sub3(x + 3 * id[3], x + 3 * id[2], q3);
        cross3(q1, q2, u);
        cross3(q2, q3, v);
        double uu = dot3(u, u), vv = dot3(v, v), uv = dot3(u, v);
        double nu = sqrt(uu), nv = sqrt(vv);
        double L = uv / (nu * nv);
        double cp[7];
        for (int n = 0; n <= 6; ++n) cp[n] = t->tc[7 * a + n] * cos(t->tpsi[7 * a + n]);
        double dW = (cp[1] - 3.0 * cp[3] + 5.0 * cp[5]) +
                    L * (4.0 * cp[2] - 16.0 * cp[4] + 36.0 * cp[6]) +
                    L * L * (12.0 * cp[3] - 60.0 * cp[5]) +
                    L * L * L * (32.0 * cp[4] - 192.0 * cp[6]) + L * L * L * L * (80.0 * cp[5]) +
                    L * L * L * L * L * (192.0 * cp[6]);
        double q2v[3], q2u[3], q1v[3], q1u[3], q3u[3], q3v[3];
        cross3(q2, v, q2v);
        cross3(q2, u, q2u);
        cross3(q1, v, q1v);
        cross3(q1, u, q1u);
        cross3(q3, u, q3u);
        cross3(q3, v, q3v);
        double uuu = uu * nu * nv, vvv = nu * vv * nv;
        for (int d = 0; d < 3; ++d) {
            double g1 = (q2v[d] * uu - uv * q2u[d]) / uuu;
            double g2 = (-q1v[d] * uu + uv * q1u[d]) / uuu + (q3u[d] * vv - uv * q3v[d]) / vvv;
            double g3 = (-q2u[d] * vv + uv * q2v[d]) / vvv;
            g[3 * id[0] + d] += dW * (-g1);
            g[3 * id[1] + d] += dW * (g1 - g2);
            g[3 * id[2] + d] += dW * (g2 - g3);
            g[3 * id[3] + d] += dW * g3;
        }
    }
    if (t->nonbonded) {
        int64_t na = s->na;
        int64_t* keys = exclusion_keys(t, na);
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < na; ++i) {
            double gi[3] = {0.0, 0.0, 0.0};
            for (int64_t j = 0; j < na; ++j) {
                if (j == i || excluded(keys, t->nexcl, na, i, j)) continue;
                double d[3], u[2], du;
                sub3(x + 3 * i, x + 3 * j, d);
                pair_terms(s, i, j, dot3(d, d), u, &du);
                for (int k = 0; k < 3; ++k) gi[k] += du * d[k];
            }
            for (int k = 0; k < 3; ++k) g[3 * i + k] += gi[k];
        }
        free(keys);
    }
}

/* Energies of the terms above: out = {bend, torsion, LJ, Coulomb}. */
void orc_ss_energy(const orc_sys* s, double* out) {
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (!s->ss) return;
    out[0] = orc_bend_energy(s->ss, s->xyz);
    out[1] = orc_torsion_energy(s->ss, s->xyz);
    orc_nonbonded_energy(s, out + 2);
}

/* ---------------------------------------------------------------- flips */

/* Energy change of flipping cell j, Eqs. "dGj1" (phi_j = -1) and "dGj2"
 * (phi_j = +1).  u holds U = U_LJ + U_CFA per cell. */
double orc_delta_e(const orc_sys* s, const int8_t* phi, const double* u, int64_t j) {
    int64_t n = s->n;
    int64_t i0 = j % n, j0 = (j / n) % n, k0 = j / (n * n);
    double h = s->h, delta = s->rho_s * s->h, h3 = h * h * h;
    int R = (int)ceil(s->rho_s);
    double sum_m = 0.0, sum_w = 0.0;
    for (int dz = -R; dz <= R; ++dz)
        for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx) {
                double d = h * sqrt((double)(dx * dx + dy * dy + dz * dz));
                if (d == 0.0 || !(d < delta)) continue;
                double kv = kernel_K(d / delta);
                if (label_at(s, phi, i0 + dx, j0 + dy, k0 + dz) == -1)
                    sum_m += kv;
                else
                    sum_w += kv;
            }
    double pref = orc_surface_prefactor(s);
    if (phi[j] == -1) return pref * sum_m - pref * sum_w + h3 * u[j];
    return pref * sum_w - pref * sum_m - h3 * u[j];
}

/* A cell "immediately next to the interface": one of its six face
 * neighbours carries the other label (outside the box counts as +1). */
int orc_in_band(const orc_sys* s, const int8_t* phi, int64_t j) {
    int64_t n = s->n;
    int64_t i = j % n, jj = (j / n) % n, k = j / (n * n);
    int me = phi[j];
    return label_at(s, phi, i - 1, jj, k) != me || label_at(s, phi, i + 1, jj, k) != me ||
           label_at(s, phi, i, jj - 1, k) != me || label_at(s, phi, i, jj + 1, k) != me ||
           label_at(s, phi, i, jj, k - 1) != me || label_at(s, phi, i, jj, k + 1) != me;
}

int orc_colours(const orc_sys* s) {
    int p = (int)ceil(s->rho_s);
    return p * p * p;
}

/* Colour (i mod p) + p (j mod p) + p^2 (k mod p) with p = ceil(rho_s): two
 * cells of one colour differ by a multiple of p >= delta/h along some axis,
 * so neither lies in the other's kernel support and their flips do not
 * interact. */
int orc_colour_of(const orc_sys* s, int64_t idx) {
    int64_t n = s->n;
    int p = (int)ceil(s->rho_s);
    int64_t i = idx % n, j = (idx / n) % n, k = idx / (n * n);
    return (int)(i % p + p * (j % p) + p * p * (k % p));
}

/* One colour pass: the band cells of colour c, with Delta E evaluated on
 * the labels at the start of the pass; every candidate with Delta E < 0
 * flips.  Returns the number of flips; *de_sum gets the sum of their
 * Delta E.  Candidates with |Delta E| <= tie_tol are appended to tie_log
 * (cell index) / tie_de (value) while *ntie < tie_cap. */
int64_t orc_colour_pass(const orc_sys* s, int8_t* phi, const double* u, int colour,
                        double tie_tol, int64_t* ncand_out, double* de_sum, int64_t* tie_log,
                        double* tie_de, int64_t tie_cap, int64_t* ntie) {
    int64_t n = s->n;
    int p = (int)ceil(s->rho_s);
    int64_t cap = ((n + p - 1) / p) * ((n + p - 1) / p) * ((n + p - 1) / p), nc = 0;
    /* cap: the cells of one colour, ceil(n / p) along each axis at most */
    int64_t* cand = malloc(sizeof(int64_t) * (size_t)cap);
    /* the cells of colour c are i = c mod p, j = (c / p) mod p, k = c / p^2,
     * each stepping by p */
    for (int64_t k = colour / (p * p); k < n; k += p)
        for (int64_t j = (colour / p) % p; j < n; j += p)
            for (int64_t i = colour % p; i < n; i += p) {
                int64_t c = i + n * (j + n * k);
                if (!orc_in_band(s, phi, c)) continue;
                cand[nc++] = c;
            }
    double* de = malloc(sizeof(double) * (size_t)(nc + 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nc; ++t) de[t] = orc_delta_e(s, phi, u, cand[t]);
    int64_t flips = 0;
    double sum = 0.0;
    for (int64_t t = 0; t < nc; ++t) {
        if (fabs(de[t]) <= tie_tol && *ntie < tie_cap) {
            if (tie_log) tie_log[*ntie] = cand[t];
            if (tie_de) tie_de[*ntie] = de[t];
            ++*ntie;
        }
        if (de[t] < 0.0) {
            phi[cand[t]] = (int8_t)(-phi[cand[t]]);
            sum += de[t];
            ++flips;
        }
    }
    if (ncand_out) *ncand_out = nc;
    if (de_sum) *de_sum = sum;
    free(cand);
    free(de);
    return flips;
}

int64_t orc_band_size(const orc_sys* s, const int8_t* phi) {
    int64_t ncell = (int64_t)s->n * s->n * s->n, m = 0;
    for (int64_t c = 0; c < ncell; ++c) m += orc_in_band(s, phi, c);
    return m;
}

/* Colour-schedule descent: sweeps of all colour passes in order 0..p^3-1
 * until a sweep flips nothing (converged) or max_sweeps sweeps ran.
 * stats = {sweeps, flips, converged, ties_logged, final_band, candidates}.
 * Returns 0 if converged, 1 otherwise. */
int orc_minimize_colour(const orc_sys* s, int8_t* phi, const double* u, int max_sweeps,
                        double tie_tol, int64_t* stats, int64_t* tie_log, double* tie_de,
                        int64_t tie_cap) {
    int ncol = orc_colours(s);
    int64_t flips = 0, ntie = 0, ncand = 0;
    int converged = 0, sweeps = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        int64_t f = 0;
        for (int c = 0; c < ncol; ++c) {
            int64_t nc = 0;
            f += orc_colour_pass(s, phi, u, c, tie_tol, &nc, NULL, tie_log, tie_de, tie_cap,
                                 &ntie);
            ncand += nc;
        }
        flips += f;
        sweeps = sw + 1;
        if (f == 0) {
            converged = 1;
            break;
        }
    }
    if (stats) {
        stats[0] = sweeps;
        stats[1] = flips;
        stats[2] = converged;
        stats[3] = ntie;
        stats[4] = orc_band_size(s, phi);
        stats[5] = ncand;
    }
    return converged ? 0 : 1;
}

/* --------------------------------------------------------------- min-heap */

typedef struct { double key; int64_t idx; int64_t ver; } heap_item;
typedef struct { heap_item* a; int64_t n, cap; } heap_t;

static int heap_less(const heap_item* x, const heap_item* y) {
    if (x->key != y->key) return x->key < y->key;
    return x->idx < y->idx;
}
static void heap_push(heap_t* h, heap_item it) {
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->a = realloc(h->a, sizeof(heap_item) * (size_t)h->cap);
    }
    int64_t i = h->n++;
    h->a[i] = it;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!heap_less(&h->a[i], &h->a[p])) break;
        heap_item t = h->a[i]; h->a[i] = h->a[p]; h->a[p] = t;
        i = p;
    }
}
static heap_item heap_pop(heap_t* h) {
    heap_item top = h->a[0];
    h->a[0] = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && heap_less(&h->a[l], &h->a[m])) m = l;
        if (r < h->n && heap_less(&h->a[r], &h->a[m])) m = r;
        if (m == i) break;
        heap_item t = h->a[i]; h->a[i] = h->a[m]; h->a[m] = t;
        i = m;
    }
    return top;
}

/* The paper's flipping process (Step 2.1-2.3): Delta E of every band cell
 * goes into a min-heap; while the smallest Delta E is negative, flip that
 * cell, recompute Delta E for the cells whose value or band membership the
 * flip changed (its kernel neighbourhood), and continue.  Stale entries are
 * dropped lazily by a per-cell version number; ties in Delta E break by cell
 * index.  stats = {flips, converged, final_band}.  Returns 0 if it reached a
 * state with every band Delta E >= 0 within max_flips flips. */
int orc_minimize_heap(const orc_sys* s, int8_t* phi, const double* u, int64_t max_flips,
                      int64_t* stats) {
    int64_t n = s->n, ncell = n * n * n;
    int R = (int)ceil(s->rho_s);
    int64_t* ver = calloc((size_t)ncell, sizeof(int64_t));
    heap_t hp = {0};
    for (int64_t c = 0; c < ncell; ++c)
        if (orc_in_band(s, phi, c)) heap_push(&hp, (heap_item){orc_delta_e(s, phi, u, c), c, 0});
    int64_t flips = 0;
    int converged = 0;
    while (hp.n > 0) {
        heap_item it = heap_pop(&hp);
        if (it.ver != ver[it.idx]) continue;
        if (it.key >= 0.0) { converged = 1; break; }
        if (flips == max_flips) break;
        phi[it.idx] = (int8_t)(-phi[it.idx]);
        ++flips;
        int64_t i0 = it.idx % n, j0 = (it.idx / n) % n, k0 = it.idx / (n * n);
        for (int dz = -R; dz <= R; ++dz)
            for (int dy = -R; dy <= R; ++dy)
                for (int dx = -R; dx <= R; ++dx) {
                    int64_t i = i0 + dx, j = j0 + dy, k = k0 + dz;
                    if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) continue;
                    int64_t c = i + n * (j + n * k);
                    ++ver[c];
                    if (orc_in_band(s, phi, c))
                        heap_push(&hp, (heap_item){orc_delta_e(s, phi, u, c), c, ver[c]});
                }
    }
    if (hp.n == 0) converged = 1;
    if (stats) {
        stats[0] = flips;
        stats[1] = converged;
        stats[2] = orc_band_size(s, phi);
    }
    free(ver);
    free(hp.a);
    return converged ? 0 : 1;
}

/* ---------------------------------------------------------- initial labels */

/* Loose initial surface: a sphere of radius R0 about the box centre
 * (Sec. "Initial surfaces"); a cell is solute iff |x - c| <= R0. */
void orc_init_loose(const orc_sys* s, double R0, int8_t* phi) {
    int64_t ncell = (int64_t)s->n * s->n * s->n;
    for (int64_t c = 0; c < ncell; ++c) {
        double x[3];
        orc_cell_center(s, c, x);
        double dx = x[0] - s->center[0], dy = x[1] - s->center[1], dz = x[2] - s->center[2];
        phi[c] = (sqrt(dx * dx + dy * dy + dz * dz) <= R0) ? -1 : 1;
    }
}

/* Tight initial surface: the sign of varphi(r) = min_i (|r - r_i| - d_i) at
 * each cell centre, solute where varphi <= 0 (same section). */
void orc_init_tight(const orc_sys* s, const double* d, int8_t* phi) {
    int64_t ncell = (int64_t)s->n * s->n * s->n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = 0; c < ncell; ++c) {
        double x[3];
        orc_cell_center(s, c, x);
        double vmin = INFINITY;
        for (int64_t i = 0; i < s->na; ++i) {
            double dx = x[0] - s->xyz[3 * i], dy = x[1] - s->xyz[3 * i + 1],
                   dz = x[2] - s->xyz[3 * i + 2];
            /* |dx| > d_i already gives |x - r_i| - d_i > 0: such an atom
             * cannot make the minimum non-positive, so only the sign of the
             * minimum (all that the label uses) is computed exactly */
            if (fabs(dx) > d[i]) continue;
            double v = sqrt(dx * dx + dy * dy + dz * dz) - d[i];
            if (v < vmin) vmin = v;
        }
        phi[c] = (vmin <= 0.0) ? -1 : 1;
    }
}

/* ---------------------------------------------------------------- forces */

/* Gradient of U(x) with respect to atom position r_n, given the total
 * field E(x).  d = x - r_n, r^2 floored at r2_min (where the floor is active
 * the LJ part is constant and E_n = Q_n d / r_min^3).
 *   grad_{r_n} rho_w U_LJ = rho_w (24 eps_n / r^2)(2 (sigma/r)^12 - (sigma/r)^6) d
 *   grad_{r_n} Ccfa |E|^2 = 2 Ccfa (dE/dr_n)^T E,
 *     dE/dr_n = -Q_n (I/r^3 - 3 d d^T / r^5). */
static void grad_u_atom(const orc_sys* s, int64_t nidx, const double x[3], const double e[3],
                        double ccfa, double g[3]) {
    double dx = x[0] - s->xyz[3 * nidx], dy = x[1] - s->xyz[3 * nidx + 1],
           dz = x[2] - s->xyz[3 * nidx + 2];
    double r2 = dx * dx + dy * dy + dz * dz;
    double qn = s->q[nidx];
    if (r2 < s->r2_min) {
        double r3 = s->r2_min * sqrt(s->r2_min);
        g[0] = 2.0 * ccfa * (-qn * e[0] / r3);
        g[1] = 2.0 * ccfa * (-qn * e[1] / r3);
        g[2] = 2.0 * ccfa * (-qn * e[2] / r3);
        return;
    }
    double r = sqrt(r2);
    double sr = s->sigma[nidx] / r;
    double sr6 = sr * sr * sr * sr * sr * sr;
    double clj = s->rho_w * 24.0 * s->eps[nidx] / r2 * (2.0 * sr6 * sr6 - sr6);
    double r3 = r2 * r, r5 = r3 * r2;
    double ed = e[0] * dx + e[1] * dy + e[2] * dz;
    double gx = -qn * (e[0] / r3 - 3.0 * ed * dx / r5);
    double gy = -qn * (e[1] / r3 - 3.0 * ed * dy / r5);
    double gz = -qn * (e[2] / r3 - 3.0 * ed * dz / r5);
    g[0] = clj * dx + 2.0 * ccfa * gx;
    g[1] = clj * dy + 2.0 * ccfa * gy;
    g[2] = clj * dz + 2.0 * ccfa * gz;
}

/* Forces F_n = -grad_{r_n} G at fixed labels, G = the discrete energy of
 * Eq. "4flip" (in-box midpoint sum over solvent cells + far-field quadrature)
 * plus the harmonic bonds.  This is the solvent part and the bond part of
 * the Appendix gradient, taken as the exact derivative of the discrete
 * energy.  f is na x 3. */
void orc_forces(const orc_sys* s, const int8_t* phi, int64_t nb, const int32_t* ij,
                const double* r0, const double* kb, double* f) {
    int64_t ncell = (int64_t)s->n * s->n * s->n;
    double h3 = s->h * s->h * s->h, ccfa = orc_cfa_prefactor(s);
    int64_t nsolv = 0;
    for (int64_t c = 0; c < ncell; ++c) nsolv += (phi[c] == 1);
    int64_t nfar = 6LL * s->far_nf * s->far_nf * s->far_ntau;
    int64_t m = nsolv + nfar;
    double* pts = malloc(sizeof(double) * 3 * (size_t)m);
    double* w = malloc(sizeof(double) * (size_t)m);
    double* e = malloc(sizeof(double) * 3 * (size_t)m);
    double* tmp = malloc(sizeof(double) * 2 * (size_t)m);
    int64_t t = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        if (phi[c] != 1) continue;
        orc_cell_center(s, c, pts + 3 * t);
        w[t] = h3;
        ++t;
    }
    orc_far_nodes(s, pts + 3 * nsolv, w + nsolv);
    orc_density_points(s, m, pts, tmp, tmp + m, e);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < s->na; ++a) {
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int64_t p = 0; p < m; ++p) {
            double g[3];
            grad_u_atom(s, a, pts + 3 * p, e + 3 * p, ccfa, g);
            gx += w[p] * g[0];
            gy += w[p] * g[1];
            gz += w[p] * g[2];
        }
        f[3 * a + 0] = -gx;
        f[3 * a + 1] = -gy;
        f[3 * a + 2] = -gz;
    }
    for (int64_t b = 0; b < nb; ++b) {
        int64_t i = ij[2 * b], j = ij[2 * b + 1];
        double dx = s->xyz[3 * i] - s->xyz[3 * j], dy = s->xyz[3 * i + 1] - s->xyz[3 * j + 1],
               dz = s->xyz[3 * i + 2] - s->xyz[3 * j + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double c = kb[b] * (r - r0[b]) / r;
        f[3 * i + 0] -= c * dx; f[3 * i + 1] -= c * dy; f[3 * i + 2] -= c * dz;
        f[3 * j + 0] += c * dx; f[3 * j + 1] += c * dy; f[3 * j + 2] += c * dz;
    }
    if (s->ss) {
        double* g = calloc((size_t)(3 * s->na), sizeof(double));
        orc_ss_gradient(s, g);
        for (int64_t k = 0; k < 3 * s->na; ++k) f[k] -= g[k];
        free(g);
    }
    free(pts); free(w); free(e); free(tmp);
}

/* Forces on the atoms listed in sel (nsel of them) at fixed labels, given
 * the field E on every grid cell (ncell x 3, e.g. from orc_density_grid):
 * the same sum as orc_forces restricted to those atoms, for large grids where
 * only a sample of atoms is checked.  f is nsel x 3. */
void orc_forces_subset(const orc_sys* s, const int8_t* phi, const double* efield, int64_t nsel,
                       const int64_t* sel, int64_t nb, const int32_t* ij, const double* r0,
                       const double* kb, double* f) {
    int64_t ncell = (int64_t)s->n * s->n * s->n;
    double h3 = s->h * s->h * s->h, ccfa = orc_cfa_prefactor(s);
    int64_t nfar = 6LL * s->far_nf * s->far_nf * s->far_ntau;
    double* fpts = malloc(sizeof(double) * 3 * (size_t)nfar);
    double* fw = malloc(sizeof(double) * (size_t)nfar);
    double* fe = malloc(sizeof(double) * 3 * (size_t)nfar);
    double* tmp = malloc(sizeof(double) * 2 * (size_t)nfar);
    orc_far_nodes(s, fpts, fw);
    orc_density_points(s, nfar, fpts, tmp, tmp + nfar, fe);
    double* gss = calloc((size_t)(3 * s->na), sizeof(double));
    orc_ss_gradient(s, gss);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nsel; ++t) {
        int64_t a = sel[t];
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int64_t c = 0; c < ncell; ++c) {
            if (phi[c] != 1) continue;
            double x[3], g[3];
            orc_cell_center(s, c, x);
            grad_u_atom(s, a, x, efield + 3 * c, ccfa, g);
            gx += h3 * g[0];
            gy += h3 * g[1];
            gz += h3 * g[2];
        }
        for (int64_t p = 0; p < nfar; ++p) {
            double g[3];
            grad_u_atom(s, a, fpts + 3 * p, fe + 3 * p, ccfa, g);
            gx += fw[p] * g[0];
            gy += fw[p] * g[1];
            gz += fw[p] * g[2];
        }
        for (int64_t b = 0; b < nb; ++b) {
            int64_t i = ij[2 * b], j = ij[2 * b + 1];
            if (i != a && j != a) continue;
            double dx = s->xyz[3 * i] - s->xyz[3 * j], dy = s->xyz[3 * i + 1] - s->xyz[3 * j + 1],
                   dz = s->xyz[3 * i + 2] - s->xyz[3 * j + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double c = kb[b] * (r - r0[b]) / r * (i == a ? 1.0 : -1.0);
            gx += c * dx; gy += c * dy; gz += c * dz;
        }
        f[3 * t + 0] = -gx - gss[3 * a];
        f[3 * t + 1] = -gy - gss[3 * a + 1];
        f[3 * t + 2] = -gz - gss[3 * a + 2];
    }
    free(fpts); free(fw); free(fe); free(tmp); free(gss);
}

/* Total free energy at fixed labels: discrete VISM energy + bonds + the
 * solute-solute terms of s->ss.  comps (optional) = {geom, vdw_in, vdw_far,
 * elec_in, elec_far, bond, bend, torsion, vdw_ss, elec_ss, total}. */
double orc_total_energy(const orc_sys* s, const int8_t* phi, int64_t nb, const int32_t* ij,
                        const double* r0, const double* kb, double* comps) {
    int64_t ncell = (int64_t)s->n * s->n * s->n;
    double* ulj = malloc(sizeof(double) * (size_t)ncell);
    double* ucfa = malloc(sizeof(double) * (size_t)ncell);
    double far[2], e[6];
    orc_density_grid(s, ulj, ucfa, NULL);
    orc_far_field(s, far);
    orc_energy(s, phi, ulj, ucfa, far, e);
    double eb = orc_bond_energy(nb, ij, r0, kb, s->xyz);
    double ess[4];
    orc_ss_energy(s, ess);
    double total = e[5] + eb + ess[0] + ess[1] + ess[2] + ess[3];
    if (comps) {
        for (int i = 0; i < 5; ++i) comps[i] = e[i];
        comps[5] = eb;
        for (int i = 0; i < 4; ++i) comps[6 + i] = ess[i];
        comps[10] = total;
    }
    free(ulj);
    free(ucfa);
    return total;
}

/* ------------------------------------------------------- adaptive mobility */

typedef struct {
    double M;          /* adjustable mobility factor (starts at 1) */
    double alpha;      /* shrink factor (1/sqrt 2) */
    double dt;         /* time step */
    double dG_frac;    /* delta G* = dG_frac |G_old| (5 %) */
    double M_min;      /* give up below this M */
    double G_old;      /* energy at the accepted positions (output) */
    int32_t N_cnt;     /* consecutive steps with the same M */
    int32_t N_cnt_max; /* N_cnt* (5) */
    int32_t k;         /* accepted steps so far */
    int32_t max_retries;
} orc_mobility;

typedef struct {
    int32_t accepted;
    int32_t retries;
    double G_old;
    double G_new;
    double max_grad;
    double omega;
} orc_step_info;

/* One adaptive-mobility gradient-descent step (Sec. "Adaptive-Mobility
 * Gradient Descent", Eq. "eq:adjustmml", Steps 3.1-3.4): with labels fixed,
 * take grad G at R, omega = 1/max |dG/dr_{m,k}| over moving atoms, trial
 * R' = R - dt omega M grad G; reject (and shrink M by alpha, reset N_cnt)
 * iff dG > dG* or (N_cnt >= N_cnt* and 0 < dG <= dG*), otherwise accept and
 * increment N_cnt.  A rejected trial retries from R with the same gradient.
 * xyz (na x 3) is updated in place on acceptance.  Returns 0 when a step was
 * accepted, 1 when M fell below M_min or the retries ran out, 2 when the
 * gradient is zero. */
int orc_atom_step(const orc_sys* s0, double* xyz, const int8_t* phi, const uint8_t* movable,
                  int64_t nb, const int32_t* ij, const double* r0, const double* kb,
                  orc_mobility* st, orc_step_info* info) {
    orc_sys s = *s0;
    int64_t na = s.na;
    s.xyz = xyz;
    double* f = malloc(sizeof(double) * 3 * (size_t)na);
    double* trial = malloc(sizeof(double) * 3 * (size_t)na);
    double G_old = orc_total_energy(&s, phi, nb, ij, r0, kb, NULL);
    orc_forces(&s, phi, nb, ij, r0, kb, f);
    double gmax = 0.0;
    for (int64_t a = 0; a < na; ++a) {
        if (movable && !movable[a]) continue;
        for (int d = 0; d < 3; ++d)
            if (fabs(f[3 * a + d]) > gmax) gmax = fabs(f[3 * a + d]);
    }
    info->accepted = 0;
    info->retries = 0;
    info->G_old = G_old;
    info->G_new = G_old;
    info->max_grad = gmax;
    info->omega = 0.0;
    if (gmax == 0.0) {
        st->G_old = G_old;
        free(f); free(trial);
        return 2;
    }
    double omega = 1.0 / gmax;
    info->omega = omega;
    int rc = 1;
    for (;;) {
        /* grad G = -f */
        for (int64_t a = 0; a < na; ++a)
            for (int d = 0; d < 3; ++d) {
                double g = -f[3 * a + d];
                trial[3 * a + d] =
                    (movable && !movable[a]) ? xyz[3 * a + d] : xyz[3 * a + d] - st->dt * omega * st->M * g;
            }
        s.xyz = trial;
        double G_new = orc_total_energy(&s, phi, nb, ij, r0, kb, NULL);
        double dG = G_new - G_old;
        double dGs = st->dG_frac * fabs(G_old);
        int reject = (dG > dGs) || (st->N_cnt >= st->N_cnt_max && dG > 0.0 && dG <= dGs);
        info->G_new = G_new;
        if (!reject) {
            memcpy(xyz, trial, sizeof(double) * 3 * (size_t)na);
            st->N_cnt += 1;
            st->k += 1;
            st->G_old = G_new;
            info->accepted = 1;
            rc = 0;
            break;
        }
        st->M *= st->alpha;
        st->N_cnt = 0;
        info->retries += 1;
        if (st->M < st->M_min || info->retries > st->max_retries) {
            st->G_old = G_old;
            rc = 1;
            break;
        }
    }
    free(f);
    free(trial);
    return rc;
}

/* ------------------------------------------------------ full alternation */

typedef struct {
    int32_t max_iters;   /* k_max (3000 in the paper) */
    int32_t persist;     /* consecutive small energy changes needed (100) */
    int32_t max_sweeps;  /* colour sweeps allowed per interface relaxation */
    int32_t pad;
    double tol_grad;     /* Tol1: stop when every |dG/dr| < tol_grad (1e-4) */
    double tol_energy;   /* Tol2: small relative or absolute change (1e-5) */
} orc_relax_opts;

typedef struct {
    int32_t iters;       /* outer iterations run */
    int32_t stop_reason; /* 1 gradient, 2 energy change, 3 max_iters, 4 mobility */
    int32_t sweeps;      /* colour sweeps over all iterations */
    int32_t retries;     /* rejected trial steps over all iterations */
    double G_final;
    double max_grad;
    double dG_abs;
    double dG_rel;
} orc_relax_report;

/* The paper's algorithm, Steps 2-5: alternate the interface relaxation at
 * fixed atoms (colour sweeps to a local minimum) with one adaptive-mobility
 * atom step at the fixed interface; stop when every gradient component of
 * the moving atoms is below tol_grad (Step 3.2), when the relative or the
 * absolute change of G between iterations stays below tol_energy for
 * `persist` iterations in a row (Step 5), after max_iters iterations, or
 * when the mobility cannot find an acceptable step.  xyz and phi are
 * updated in place; st carries the mobility state across iterations. */
int orc_relax(const orc_sys* s0, double* xyz, int8_t* phi, const uint8_t* movable, int64_t nb,
              const int32_t* ij, const double* r0, const double* kb, const orc_relax_opts* o,
              orc_mobility* st, orc_relax_report* rep) {
    orc_sys s = *s0;
    s.xyz = xyz;
    int64_t ncell = (int64_t)s.n * s.n * s.n, na = s.na;
    double* ulj = malloc(sizeof(double) * (size_t)ncell);
    double* ucfa = malloc(sizeof(double) * (size_t)ncell);
    double* u = malloc(sizeof(double) * (size_t)ncell);
    double* f = malloc(sizeof(double) * 3 * (size_t)na);
    int calm = 0, reason = 3;
    double G_prev = NAN;
    memset(rep, 0, sizeof(*rep));
    int k;
    for (k = 0; k < o->max_iters; ++k) {
        rep->iters = k + 1;
        /* Step 2: interface at fixed atoms */
        int64_t stats[6];
        orc_density_grid(&s, ulj, ucfa, NULL);
        for (int64_t c = 0; c < ncell; ++c) u[c] = ulj[c] + ucfa[c];
        orc_minimize_colour(&s, phi, u, o->max_sweeps, 0.0, stats, NULL, NULL, 0);
        rep->sweeps += (int32_t)stats[0];
        /* Step 3.1-3.2: gradient test */
        orc_forces(&s, phi, nb, ij, r0, kb, f);
        double gmax = 0.0;
        for (int64_t a = 0; a < na; ++a) {
            if (movable && !movable[a]) continue;
            for (int d = 0; d < 3; ++d)
                if (fabs(f[3 * a + d]) > gmax) gmax = fabs(f[3 * a + d]);
        }
        rep->max_grad = gmax;
        if (gmax < o->tol_grad) {
            rep->G_final = orc_total_energy(&s, phi, nb, ij, r0, kb, NULL);
            reason = 1;
            break;
        }
        /* Step 3.3-3.4: one accepted step */
        orc_step_info info;
        int rc = orc_atom_step(&s, xyz, phi, movable, nb, ij, r0, kb, st, &info);
        rep->retries += info.retries;
        if (rc != 0) {
            rep->G_final = info.G_old;
            reason = 4;
            break;
        }
        /* Steps 4-5: change of G between iterations */
        double G = info.G_new;
        rep->G_final = G;
        if (!isnan(G_prev)) {
            rep->dG_abs = fabs(G - G_prev);
            rep->dG_rel = rep->dG_abs / fabs(G_prev);
            if (rep->dG_rel < o->tol_energy || rep->dG_abs < o->tol_energy)
                ++calm;
            else
                calm = 0;
            if (calm >= o->persist) {
                reason = 2;
                break;
            }
        }
        G_prev = G;
    }
    rep->stop_reason = reason;
    free(ulj); free(ucfa); free(u); free(f);
    return reason == 3 ? 1 : 0;
}

/* Threads of the OpenMP loops (measurement only: no result depends on it,
 * every parallel loop writing disjoint entries). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
