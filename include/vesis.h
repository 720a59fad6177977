/*
 * vesis.h - C ABI of the MI355X (gfx950) VESIS hot path.
 *
 * The operations follow the statement of the problem in arXiv 2208.05524:
 * solute atoms with positions r_i, charges Q_i and solute-water LJ
 * parameters (sigma_i, eps_i) sit in the box Omega = (c - L, c + L)^3
 * (Sec. "A Binary Level-Set Method"), which carries a uniform grid of n^3
 * cells of edge h = 2L/n.  A binary level set phi labels every cell solute
 * (-1) or solvent (+1).  The discrete free energy is Eq. "4flip": the kernel
 * surface energy, h^3 times the energy density U (Eq. "Ur": rho_w-weighted
 * LJ plus the Coulomb-field approximation) summed over solvent cells, and
 * the integral of U over R^3 outside the box.  The interface is relaxed by
 * flipping band cells whose energy change (Eqs. "dGj1", "dGj2") is negative;
 * atoms move by adaptive-mobility gradient descent (Eq. "eq:moveatoms",
 * Eq. "eq:adjustmml" and Steps 3.1-3.4 of the algorithm).
 *
 * Conventions for every call:
 *  - Pointers named in the argument lists are host pointers unless stated.
 *    Host inputs are copied before the call returns; the library never keeps
 *    a caller pointer.  Arrays of atoms are row-major (atom, xyz), FP64.
 *  - Cell (i, j, k) has centre c - L + (i + 1/2, j + 1/2, k + 1/2) h and
 *    linear index i + n (j + n k) (x fastest).  Labels are int8: -1 solute,
 *    +1 solvent.  Cells outside the box count as solvent and never flip.
 *  - All device work runs on the stream given to vesis_create, in order.
 *    Calls that return host data synchronise that stream before returning.
 *  - Device memory: one caller-provided workspace (vesis_workspace_size /
 *    vesis_set_workspace); the library allocates no device memory itself.
 *  - Every call returns a vesis_status; negative values are errors and the
 *    per-context message is available from vesis_last_error.  After an error
 *    the context stays usable; device state may be partly updated only for
 *    VESIS_E_DEVICE.
 *  - Call order: vesis_set_params, vesis_set_grid, vesis_set_atoms,
 *    vesis_set_workspace, vesis_init_labels; a call made before its inputs
 *    exist returns VESIS_E_STATE.  Changing the grid or the atom count
 *    invalidates the workspace and the labels; changing the precision
 *    invalidates the workspace (its per-cell arrays change size).
 *  - One host thread per context at a time; separate contexts are independent.
 */
#ifndef VESIS_H
#define VESIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vesis_ctx vesis_ctx;

typedef enum {
    VESIS_OK = 0,
    VESIS_NOT_CONVERGED = 1,   /* minimisation stopped at max_sweeps; state valid, resumable */
    VESIS_E_ARG = -1,          /* bad argument (null pointer, size, range) */
    VESIS_E_STATE = -2,        /* call made before its inputs were set */
    VESIS_E_OUT_OF_BOX = -3,   /* an atom lies outside the box */
    VESIS_E_NONFINITE = -4,    /* NaN or Inf in an input */
    VESIS_E_NO_DEVICE = -5,    /* no usable gfx950 device */
    VESIS_E_DEVICE = -6,       /* HIP runtime error */
    VESIS_E_WORKSPACE = -7     /* workspace missing or too small */
} vesis_status;

/* Model constants, in one consistent unit system (e.g. nm, kJ/mol, e).
 * rho_w, gamma0, eps_m, eps_w: Table "Model parameters" of the paper;
 * coulomb_k = 1/(4 pi eps0) so the CFA prefactor 1/(32 pi^2 eps0)(1/eps_w -
 * 1/eps_m) of Eq. "G_VISM" equals coulomb_k/(8 pi)(1/eps_w - 1/eps_m);
 * rho_s = delta/h, the kernel radius in cells (1 < rho_s <= 3; the paper
 * writes delta = lambda sqrt(h)); r2_min floors |x - r_i|^2 (> 0);
 * far_nf, far_ntau: Gauss-Legendre orders of the far-field quadrature over
 * R^3 outside the box (per face axis and radially, 1..128);
 * precision: 32 (FP32 density sums, FP64 totals and FP64 near-tie
 * decisions) or 64 (FP64 density throughout). */
typedef struct {
    double rho_w;
    double gamma0;
    double eps_m;
    double eps_w;
    double coulomb_k;
    double rho_s;
    double r2_min;
    int32_t far_nf;
    int32_t far_ntau;
    int32_t precision;
    int32_t reserved;
} vesis_params;

/* Energy parts of Eq. "4flip" plus the solute-solute terms of Eq. "Gss":
 * geom = surface energy, *_in = h^3 sum over solvent cells, *_far = integral
 * over R^3 outside the box; bond, bend (bending), torsion, vdw_ss and
 * elec_ss (non-bonded LJ and Coulomb) are 0 when not set; total = their
 * sum. */
typedef struct {
    double geom, vdw_in, vdw_far, elec_in, elec_far, bond, bend, torsion, vdw_ss, elec_ss, total;
} vesis_energy_parts;

/* Interface minimisation report.  sweeps counts colour sweeps run, the last
 * one (flipping nothing) included when converged; near_ties counts flip
 * candidates whose FP32 energy change fell inside its error bound and were
 * decided in FP64; fp64_recomputes counts cells whose density was recomputed
 * in FP64 for that (each at most once per atom configuration). */
typedef struct {
    int32_t sweeps;
    int32_t converged;
    int64_t flips;
    int64_t band_cells;
    int64_t near_ties;
    int64_t fp64_recomputes;
} vesis_min_stats;

/* State of the adaptive-mobility descent (Sec. "Adaptive-Mobility Gradient
 * Descent"): M (starts at 1), alpha (1/sqrt 2), dt, dG_frac (delta G* =
 * dG_frac |G_old|, 0.05), M_min (give up below), G_old (energy at the
 * accepted positions, written by the step), N_cnt (consecutive steps with
 * the same M), N_cnt_max (N_cnt*, 5), k (accepted steps), max_retries. */
typedef struct {
    double M, alpha, dt, dG_frac, M_min, G_old;
    int32_t N_cnt, N_cnt_max, k, max_retries;
} vesis_mobility;

typedef struct {
    int32_t accepted, retries;
    double G_old, G_new, max_grad, omega;
} vesis_step_info;

/* Create a context on HIP device `device`, issuing all work on `stream`
 * (a hipStream_t; NULL = the null stream).  Returns VESIS_E_NO_DEVICE when
 * the device does not exist or is not gfx950.  *out is NULL on error. */
vesis_status vesis_create(int32_t device, void* stream, vesis_ctx** out);

/* Destroy a context (NULL is a no-op).  Does not free the workspace, which
 * belongs to the caller. */
void vesis_destroy(vesis_ctx* ctx);

/* Message of the last error on this context ("" if none).  The string lives
 * until the next call on the context. */
const char* vesis_last_error(const vesis_ctx* ctx);

/* Set the model constants (see vesis_params).  Invalidates densities. */
vesis_status vesis_set_params(vesis_ctx* ctx, const vesis_params* p);

/* Set the cubic box and grid: n cells per edge (4 <= n <= 1024), centre
 * c = center[0..2], cell edge h > 0 (Sec. "A Binary Level-Set Method").
 * Invalidates the workspace and labels. */
vesis_status vesis_set_grid(vesis_ctx* ctx, int32_t n, const double center[3], double h);

/* Set the solute atoms: n >= 1 atoms, xyz (n x 3), charges q, LJ sigma > 0
 * and eps >= 0 (Eq. "eq:LJpotential"); movable (n bytes, nonzero = moves in
 * vesis_atom_step) may be NULL (all move).  Every atom must lie inside the
 * box (VESIS_E_OUT_OF_BOX).  A new atom count invalidates the workspace. */
vesis_status vesis_set_atoms(vesis_ctx* ctx, int64_t n, const double* xyz, const double* q,
                             const double* sigma, const double* eps, const uint8_t* movable);

/* Replace the atom positions (n x 3, same count).  on_device != 0 means xyz
 * is a device pointer (copied device to device on the context stream). */
vesis_status vesis_set_positions(vesis_ctx* ctx, const double* xyz, int32_t on_device);

/* Copy the current atom positions (n x 3) to host memory. */
vesis_status vesis_get_positions(vesis_ctx* ctx, double* xyz);

/* Harmonic bonds of Eq. "Gss", (1/2) k (r_ij - r0)^2: nb bonds, ij (nb x 2
 * atom indices), rest lengths r0 and constants k.  nb = 0 removes bonds.
 * Must be called after vesis_set_atoms; takes effect at the next
 * vesis_set_workspace if the bond count grew. */
vesis_status vesis_set_bonds(vesis_ctx* ctx, int64_t nb, const int32_t* ij, const double* r0,
                             const double* k);

/* Bending terms of Eq. "Gss", (1/2) B (theta_ijk - theta0)^2 with theta_ijk
 * the angle at atom j between r_i - r_j and r_k - r_j: nang triplets ijk
 * (nang x 3 atom indices, three different atoms), theta0 in [0, pi] (rad)
 * and B = k.  The gradient is that of the Appendix; sin theta is floored at
 * 1e-12 for collinear atoms.  nang = 0 removes them.  Like vesis_set_bonds,
 * more terms than the workspace was planned for require vesis_set_workspace
 * again (VESIS_E_WORKSPACE until then). */
vesis_status vesis_set_angles(vesis_ctx* ctx, int64_t nang, const int32_t* ijk,
                              const double* theta0, const double* k);

/* Torsion terms of Eq. "Gss", sum_{n=0..6} C_n [1 + cos(n tau - psi_n)] per
 * quadruple ijkl (ntor x 4 atom indices, four different atoms), tau in
 * [0, pi] the angle between the planes (r_i, r_j, r_k) and (r_j, r_k, r_l)
 * (Appendix: cos tau = u.v/(|u||v|), u = (r_j - r_i) x (r_k - r_j),
 * v = (r_k - r_j) x (r_l - r_k)); c and psi are ntor x 7 (n = 0..6), every
 * psi_n 0 or pi (the Appendix's gradient assumes so; VESIS_E_ARG
 * otherwise).  ntor = 0 removes them. */
vesis_status vesis_set_torsions(vesis_ctx* ctx, int64_t ntor, const int32_t* ijkl,
                                const double* c, const double* psi);

/* Non-bonded solute-solute terms of Eq. "Gss" over every pair of atoms not
 * listed in excl (nexcl x 2 atom indices, any order, duplicates allowed):
 * 4 eps_ij [(sigma_ij/r)^12 - (sigma_ij/r)^6] with sigma_ij = (sigma_i +
 * sigma_j)/2, eps_ij = sqrt(eps_i eps_j) from sigma_ss, eps_ss (n values
 * each; NULL = the atoms' sigma and eps of vesis_set_atoms), plus
 * coulomb_k Q_i Q_j / (eps_w r).  enable = 0 turns them off.  Coincident
 * non-excluded atoms give a non-finite energy. */
vesis_status vesis_set_nonbonded(vesis_ctx* ctx, int32_t enable, const double* sigma_ss,
                                 const double* eps_ss, int64_t nexcl, const int32_t* excl);

/* Bytes of device workspace needed for the current grid, atoms, bonds and
 * solute-solute terms. */
vesis_status vesis_workspace_size(vesis_ctx* ctx, size_t* bytes);

/* Hand the context a device buffer of `bytes` bytes (256-byte aligned),
 * owned by the caller and kept alive while the context uses it.
 * VESIS_E_WORKSPACE when smaller than vesis_workspace_size. */
vesis_status vesis_set_workspace(vesis_ctx* ctx, void* device_ptr, size_t bytes);

/* Initial labels (Sec. "Initial surfaces").  mode 0: loose sphere, solute
 * iff |x - c| <= param (param > 0); mode 1: tight surface, solute iff
 * min_i (|x - r_i| - param * sigma_i) <= 0 (param > 0); mode 2: the caller's
 * labels `user` (n^3 int8, each -1 or +1). */
vesis_status vesis_init_labels(vesis_ctx* ctx, int32_t mode, double param, const int8_t* user);

/* Relax the interface at fixed atoms (Step 2 of the algorithm): colour
 * sweeps over the band (cells with a face neighbour of the other label),
 * each sweep visiting the p^3 colours (i mod p) + p (j mod p) + p^2 (k mod p),
 * p = ceil(rho_s), in order; within a colour every band cell whose energy
 * change is negative flips (cells of one colour do not interact).  Stops
 * after a sweep with no flip (VESIS_OK) or after max_sweeps sweeps
 * (VESIS_NOT_CONVERGED; calling again resumes).  With p = 3 the three
 * colours that share their rows run in one launch, with the result of the
 * sequence.  Recomputes the density first if the atoms moved.  out may be
 * NULL. */
vesis_status vesis_minimize_interface(vesis_ctx* ctx, int32_t max_sweeps, vesis_min_stats* out);

/* Relax the interface at fixed atoms by the paper's serial flipping process
 * (Sec. "Flipping grid cells", Steps 2.1-2.3 of the algorithm): the energy
 * change of every band cell goes into a min-heap keyed by (Delta E, cell
 * index); while the smallest key is negative that one cell flips and the
 * cells whose Delta E or band membership the flip changed (those within two
 * cells along each axis) are re-evaluated and pushed, stale entries being
 * dropped.  The density (computed on the device, recomputed if the atoms
 * moved) is read back once; the heap and the flips run on the host, one flip
 * at a time, and the final labels are written back to the device.  Each
 * Delta E is decided as the colour passes decide it: from the stored U,
 * unless it lies within the cell's error bound, then from U recomputed in
 * FP64 on the device (once per cell).  A different schedule from
 * vesis_minimize_interface, so it may end in a different local minimum; for
 * checking and small grids, not for speed.  Stops with every band Delta E
 * >= 0 (VESIS_OK) or after max_flips flips (VESIS_NOT_CONVERGED).  out (may
 * be NULL) gets sweeps = 0, flips, converged, band_cells (after), near_ties
 * and fp64_recomputes. */
vesis_status vesis_minimize_heap(vesis_ctx* ctx, int64_t max_flips, vesis_min_stats* out);

/* Discrete free energy of the current labels and atoms (Eq. "4flip" plus
 * the solute-solute terms that are set). */
vesis_status vesis_energy(vesis_ctx* ctx, vesis_energy_parts* out);

/* Forces F_n = -grad_{r_n} G at fixed labels (solvent and far-field terms of
 * the Appendix gradient, taken as the exact derivative of the discrete
 * energy, plus the solute-solute terms that are set), written to f_out
 * (n x 3 host array). */
vesis_status vesis_forces(vesis_ctx* ctx, double* f_out);

/* One adaptive-mobility step at fixed labels (Steps 3.1-3.4): gradient at
 * the current positions, omega = 1 / max |dG/dr| over movable atoms, trial
 * R' = R - dt omega M grad G, rejected (M *= alpha, N_cnt = 0, retry from R)
 * iff dG > dG* or (N_cnt >= N_cnt_max and 0 < dG <= dG*) with
 * dG* = dG_frac |G_old|; otherwise accepted (N_cnt += 1).  Returns VESIS_OK
 * on acceptance, VESIS_NOT_CONVERGED when M fell below M_min or the retries
 * ran out (positions unchanged) or the gradient is zero. */
vesis_status vesis_atom_step(vesis_ctx* ctx, vesis_mobility* state, vesis_step_info* out);

/* Labels from per-cell logits on the device (n^3 FP32, x fastest, e.g. the
 * output of the learned warm start of vesis_nn.h): solute (-1) where the
 * logit is positive, solvent elsewhere.  A start for
 * vesis_minimize_interface like the loose and tight spheres of Sec.
 * "Initial surfaces"; the relaxation from it is the paper's Step 2. */
vesis_status vesis_init_labels_logits(vesis_ctx* ctx, const float* logits);

/* Options of the full alternation (Steps 1-5 of the algorithm): max_iters
 * (k_max, 3000 in the paper), persist (consecutive iterations with a small
 * energy change needed to stop, 100), max_sweeps (colour sweeps allowed per
 * interface relaxation), tol_grad (Tol1: stop once every gradient component
 * of the movable atoms is below it, 1e-4), tol_energy (Tol2: an iteration is
 * "small" when the relative or the absolute change of G is below it, 1e-5). */
typedef struct {
    int32_t max_iters, persist, max_sweeps, reserved;
    double tol_grad, tol_energy;
} vesis_relax_opts;

/* stop_reason: 1 gradient below tol_grad, 2 energy change small for
 * `persist` iterations, 3 max_iters reached, 4 no acceptable step (mobility
 * below M_min or retries exhausted). */
typedef struct {
    int32_t iters, stop_reason, sweeps, retries;
    double G_final, max_grad, dG_abs, dG_rel;
} vesis_relax_report;

/* The paper's alternating minimisation (Sec. "Numerical Algorithm", Steps
 * 2-5): each iteration relaxes the interface at fixed atoms
 * (vesis_minimize_interface), tests the gradient (Step 3.2), takes one
 * adaptive-mobility step at the fixed interface (vesis_atom_step, Steps
 * 3.3-3.4) and tests the change of G against the previous iteration (Steps
 * 4-5).  Labels and positions are updated in place; `state` carries the
 * mobility across iterations (and across calls).  Returns VESIS_OK when a
 * stopping rule fired, VESIS_NOT_CONVERGED when max_iters ran out. */
vesis_status vesis_relax(vesis_ctx* ctx, const vesis_relax_opts* opts, vesis_mobility* state,
                         vesis_relax_report* out);

/* ---- Batches of molecules -------------------------------------------------
 * Many contexts (one molecule each, own grid and atoms, set up as above, all
 * with FP32 densities, one device, one stream and one colour period) are
 * relaxed together: one density launch covers every molecule's cells and each
 * colour pass is one launch over every unconverged molecule's label words.
 * Per molecule the result is the one vesis_minimize_interface gives: the
 * same passes in the same order (the paper's Step 2, batched), and the far
 * field of all molecules is evaluated together with the same result as one
 * at a time.  The calls need a device buffer for the batch's own tables
 * (descriptors, block maps): vesis_batch_workspace_size gives its size; it
 * must be 256-byte aligned.  The first context of a batch keeps a pinned
 * host buffer for staging those tables (host memory, grown as needed, freed
 * by vesis_destroy), so that no call waits for a copy to finish.  Contexts
 * must not be used concurrently with a batch call. */
vesis_status vesis_batch_workspace_size(vesis_ctx* const* ctxs, int32_t m, size_t* bytes);

/* Autotune the batch's launch shapes.  Times each density tiling d (0: two
 * cells per lane on 16x8x4 bricks; 1: one cell per lane on 16x8x2 bricks;
 * 2: four cells per lane on 16x8x8 bricks) on the batch, and, when every
 * molecule has labels, the first four sweeps of colour passes with each
 * colour-pass variant f from the current labels, which are put back
 * afterwards: with colour period 3, f = 0 runs the three colours that share
 * their rows in one launch and f = 1 one launch per colour; with period 2
 * both launch one colour at a time, and only f = 0 is timed.
 * *best = d + 3 f of the fastest of each (f = 0 when not timed), the value
 * vesis_minimize_batch takes as `variant`; ms (may be NULL, 5 entries)
 * receives the density times (ms[d]) and the sweep times (ms[3 + f], -1
 * when not timed).  Every variant computes the same labels; the density
 * tilings round differently in FP32.  Leaves the densities marked stale. */
vesis_status vesis_batch_tune(vesis_ctx* const* ctxs, int32_t m, void* batch_ws, size_t bytes,
                              int32_t* best, double* ms);

/* Relax the interfaces of m molecules (Step 2 for each), recomputing the
 * density of those whose atoms changed; variant = d + 3 f selects the
 * density tiling d and the colour-pass variant f (see vesis_batch_tune).
 * Sweeps run in groups of 8; a full group is captured once as a HIP graph
 * (on a private stream; kept by the first context for later calls with the
 * same batch workspace, molecule count, pass grid, colour period and f) and
 * replayed on the context stream, unless flags holds VESIS_BATCH_EAGER.
 * While many molecules are still relaxing, the next group is queued before
 * the host reads the current one's flip counts. 
 * out (m entries, may be NULL) receives each molecule's statistics.
 * Returns VESIS_OK when every molecule converged within max_sweeps,
 * VESIS_NOT_CONVERGED otherwise (the others keep their state and a new call
 * resumes them). */
#define VESIS_BATCH_EAGER 1 /* flags: launch every pass directly instead of replaying a graph */
vesis_status vesis_minimize_batch(vesis_ctx* const* ctxs, int32_t m, void* batch_ws, size_t bytes,
                                  int32_t max_sweeps, int32_t variant, int32_t flags,
                                  vesis_min_stats* out);

/* Copy the labels (n^3 int8, -1/+1) to host memory. */
vesis_status vesis_get_labels(vesis_ctx* ctx, int8_t* out);

/* Copy the per-cell density parts U_LJ and U_CFA (n^3 values each, x
 * fastest, written as FP64) and, if bound != NULL, the per-cell bound on
 * |U_stored - U_exact| used for near-tie decisions (n^3).  The library
 * stores them in the precision of the density sums: with precision 32 as
 * FP32 (widened here; the bound includes that storage rounding), with
 * precision 64 as FP64. */
vesis_status vesis_get_density(vesis_ctx* ctx, double* u_lj, double* u_cfa, double* bound);

/* Kernel timing for measurement: enable != 0 records HIP events around
 * every launch of each kernel kind on the context stream. */
vesis_status vesis_profile(vesis_ctx* ctx, int32_t enable);

/* Accumulated device time (ms) and launch count of kernel kind `kind`
 * since profiling was enabled: 0 density (grid), 1 far-field density,
 * 2 initial labels, 3 flip passes, 4 energy reductions, 5 force adjoint,
 * 6 other, 7 solute-solute terms.  Synchronises the stream. */
vesis_status vesis_profile_read(vesis_ctx* ctx, int32_t kind, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* VESIS_H */
