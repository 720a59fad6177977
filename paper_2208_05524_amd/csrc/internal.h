// Internal types shared by the HIP translation units of libvesis.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vesis {

// Cell grid and bit-packed label layout.
//
// Labels are one bit per cell, 1 = solvent (+1), 0 = solute (-1).  Every
// x-row (fixed y, z) is `W` 32-bit words: word 0 is a padding word for
// x in [-32, 0), words 1..nwin hold x in [0, n) (bits past n are padding),
// word W-1 pads x >= 32 nwin.  Rows exist for y, z in [-2, n + 2); rows and
// padding bits outside the box are all 1 (solvent) and never change, so a
// 5x5x5 neighbourhood of any cell needs no bounds checks.
struct Grid {
    int n;        // cells per edge
    int nwin;     // in-box words per row, ceil(n / 32)
    int W;        // words per row, nwin + 2
    int rdim;     // rows per edge including halo, n + 4
    double h;     // cell edge
    double x0, y0, z0;  // centre of cell (0, 0, 0)
    double cx, cy, cz;  // box centre
    double L;     // half edge

    __host__ __device__ int64_t ncell() const { return (int64_t)n * n * n; }
    __host__ __device__ int64_t nwords() const { return (int64_t)W * rdim * rdim; }
    // index of the word holding bit x of row (y, z); x may be in [-32, 32 nwin + 32)
    __host__ __device__ int64_t row(int y, int z) const {
        return ((int64_t)(z + 2) * rdim + (y + 2)) * W;
    }
};

// Surface-term constants: weight w[s] of squared offset s = 1..8
// (w[s] = K(sqrt(s)/rho_s) inside the support, 0 outside), the prefactor
// c = gamma0 C0 h^6 / delta^4, and the colour period p = ceil(rho_s).
struct Stencil {
    double w[9];
    double c;
    int p;
};

// Atom arrays on the device.
struct Atoms {
    int64_t n;
    const double4* pos;   // x, y, z, 0
    const double4* prm64; // sigma^2, 4 rho_w eps, Q, sigma
    const float4* prm32;  // 4 rho_w eps sigma^6, 4 rho_w eps sigma^12, Q, |Q|
};

struct Physics {
    double ccfa;     // CFA prefactor
    double r2min;    // floor on r^2
    double rho_w;
    double h3;       // cell volume
};

// Per-cell outputs of the density kernel, ncell values each (x fastest), in
// the precision of the density sums: float with FP32 sums (f32 != 0), double
// with FP64 sums.  bound bounds |U_stored - U_exact| in U units, where
// U_stored = U_LJ + U_CFA as stored (for float storage it includes the
// rounding of both to float, and is itself rounded up).
struct CellFields {
    void* ulj;
    void* ucfa;
    void* ex;
    void* ey;
    void* ez;
    void* bound;
    int f32;
};

// Value c of a per-cell array stored as float (f32 != 0) or double.
__host__ __device__ inline double cell_value(const void* a, int f32, int64_t c) {
    return f32 ? (double)static_cast<const float*>(a)[c] : static_cast<const double*>(a)[c];
}

enum KernelKind {
    K_DENSITY = 0, K_FAR = 1, K_INIT = 2, K_FLIP = 3, K_ENERGY = 4, K_FORCE = 5, K_OTHER = 6,
    K_SOLUTE = 7, K_NKINDS = 8
};

// One molecule of a batch, in device memory: what the batched density and
// flip-pass kernels need.  brick0 / slot0: the molecule's first brick and
// first flip-pass slot in the batch's launch order.
struct MolDesc {
    Grid g;
    Stencil sc;
    Atoms a;
    Physics ph;
    CellFields f;
    uint32_t* bits;
    int* stamp;
    double* u64cache;
    int* sweep_flips;
    int64_t* counters;
    int64_t brick0;
    int64_t slot0;
};

// Launch wrappers (one per translation unit; all asynchronous on `st`).
hipError_t launch_density_grid(const Grid& g, const Atoms& a, const Physics& ph, int precision,
                               CellFields out, hipStream_t st);
// Far-field node density: the atoms are split into at most POINT_SPLITS_MAX
// slices whose FP64 partials (4 x nsplit x np doubles in `part`) are summed
// in slice order.
constexpr int POINT_SPLITS_MAX = 16;
int points_split(int64_t np, int64_t natoms);
hipError_t launch_density_points(const double4* pts, int64_t np, const Atoms& a, const Physics& ph,
                                 int precision, double* part, double* ulj, double* ucfa,
                                 double* ex, double* ey, double* ez, hipStream_t st);
hipError_t launch_weighted_sum2(const double4* pts, const double* a, const double* b, int64_t np,
                                double* partial, int nblocks, double* out, hipStream_t st);

// One molecule of a batched far-field evaluation (FP32 point densities):
// what launch_density_points, launch_weighted_sum2 and the NaN fill of the
// near-tie cache take for it, its slices (nsplit, chunk) as there, and the
// index of its first point block in the launch.
struct FarDesc {
    const double4* pts;
    int64_t np;
    Atoms a;
    Physics ph;
    int nsplit;
    int64_t chunk;
    double* part;
    double* ulj;
    double* ucfa;
    double* ex;
    double* ey;
    double* ez;
    double* partial;   // nred x 2
    double* out;       // the two weighted sums
    double* u64cache;  // 2 x ncell
    int64_t ncell;
    int64_t block0;
};
// Point blocks of one molecule's far-field launch (node blocks x slices).
int64_t points_blocks(int64_t np, int64_t natoms);
// NaN fill, point densities, combine and the two-level sums of m molecules
// in five launches; the point blocks of molecule k are consecutive from
// d[k].block0 (block_mol maps each to its molecule).  The results equal the
// single-molecule launches' bit for bit.
hipError_t launch_far_batch(const FarDesc* d, const int* block_mol, int m, int64_t nblocks,
                            int64_t max_np, int64_t max_ncell, int nred, hipStream_t st);

// Batched density (FP32): variant 0 = 2 cells per lane on 16 x 8 x 4 bricks,
// 1 = 1 cell per lane on 16 x 8 x 2 bricks, 2 = 4 cells per lane on 16 x 8 x 8
// bricks.  block_mol maps each block to its molecule; a molecule's blocks are
// consecutive, from desc[m].brick0.
constexpr int DENSITY_VARIANTS = 3;
int64_t density_bricks(const Grid& g, int variant);
hipError_t launch_density_batch(const MolDesc* desc, const int* block_mol, int64_t nblocks,
                                int variant, hipStream_t st);

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st);
hipError_t launch_init_loose(const Grid& g, double R0, uint32_t* bits, hipStream_t st);
// bits must hold all-solvent labels; dmax >= scale * max_i sigma_i.
hipError_t launch_init_tight(const Grid& g, const Atoms& a, double scale, double dmax,
                             uint32_t* bits, hipStream_t st);
// In-box label bits from per-cell logits (solute where logit > 0).
hipError_t launch_labels_from_logits(const Grid& g, const float* logits, uint32_t* bits,
                                     hipStream_t st);
// u64cache: 2 x ncell FP64 (LJ parts, then CFA parts; NaN = not computed).
// gpass: pass index within the current minimisation call (sweep * p^3 + colour);
// stamp: one int per label word, filled with a value < -p^3 before the call.
hipError_t launch_flip_pass(const Grid& g, const Stencil& sc, const Atoms& a, const Physics& ph,
                            int colour, int sweep, int gpass, uint32_t* bits, int* stamp,
                            const CellFields& f, double* u64cache, int* sweep_flips,
                            int64_t* counters, hipStream_t st);
// The three colour passes 3 group + a, a = 0, 1, 2 (colour period 3: they
// share their rows), in one launch: the same decisions, flips and stamps as
// the three separate passes; gpass0 is the global index of the first.
hipError_t launch_flip_group3(const Grid& g, const Stencil& sc, const Atoms& a, const Physics& ph,
                              int group, int sweep, int gpass0, uint32_t* bits, int* stamp,
                              const CellFields& f, double* u64cache, int* sweep_flips,
                              int64_t* counters, hipStream_t st);
// FP64 density parts of cell (x, y, z) into u64cache (LJ at c, CFA at
// ncell + c), by one workgroup, as the colour passes compute near ties.
hipError_t launch_cell_density_f64(const Grid& g, const Atoms& a, const Physics& ph, int x, int y,
                                   int z, double* u64cache, hipStream_t st);
// Batched colour pass: flip_slots(g, p) thread slots per molecule (a multiple
// of the workgroup size).  Entry b of the block map is molecule |
// (logical block << BATCH_MOL_BITS), or -1 for an idle workgroup.
constexpr int FLIP_WG = 256;
constexpr int BATCH_MOL_BITS = 12;
constexpr int BATCH_MOLS = 1 << BATCH_MOL_BITS;  // molecules a batch may hold
int64_t flip_slots(const Grid& g, int p);
// Workgroups per molecule of the batched passes' block map: enough for the
// single-colour passes (flip_slots / FLIP_WG) and, with colour period 3, for
// the three-colour launches (whole rows per workgroup).
int64_t flip_blocks(const Grid& g, int p);
// The three-colour launch of launch_flip_group3 over a batch (block map as
// for launch_flip_pass_batch, built with flip_blocks).
hipError_t launch_flip_group3_batch(const MolDesc* descs, const int* block_mol, const int* done,
                                    const int* pass_base, int64_t nblocks, int group, int sweep,
                                    int gpass_off, hipStream_t st);
// One colour pass over a batch: done[k] != 0 skips molecule k; the pass
// index is *pass_base + gpass_off.
hipError_t launch_flip_pass_batch(const MolDesc* descs, const int* block_mol, const int* done,
                                  const int* pass_base, int64_t nblocks, int p, int colour,
                                  int sweep, int gpass_off, hipStream_t st);
// Colour-pass variants of a batch: 0 = the three colours that share their
// rows in one launch (colour period 3; one colour per launch with period 2),
// 1 = one colour per launch.
constexpr int FLIP_VARIANTS = 2;
// End of a group of nsweeps sweeps: flag molecules that had a sweep without
// flips, advance *pass_base by nsweeps * ncol.
hipError_t launch_batch_end_group(const MolDesc* descs, int m, int nsweeps, int ncol, int* done,
                                  int* pass_base, hipStream_t st);
hipError_t launch_batch_clear_flips(const MolDesc* descs, int m, int nsweeps, hipStream_t st);
// Stamps of every molecule set older than any pass, tie counters zeroed;
// max_words: the largest label word count of the m molecules.
hipError_t launch_batch_prepare(const MolDesc* descs, int m, int64_t max_words, hipStream_t st);
hipError_t launch_batch_gather_flips(const MolDesc* descs, int m, int nsweeps, int* out,
                                     hipStream_t st);
hipError_t launch_energy_volume(const Grid& g, const uint32_t* bits, const CellFields& f,
                                double* partial, int nblocks, double* out, hipStream_t st);
hipError_t launch_geom_counts(const Grid& g, const uint32_t* bits, int64_t* partial, int nblocks,
                              int64_t* out, hipStream_t st);
hipError_t launch_band_count(const Grid& g, const uint32_t* bits, int64_t* partial, int nblocks,
                             int64_t* out, hipStream_t st);

struct Bonds {
    int64_t nb;
    const int32_t* off;     // CSR offsets per atom (n + 1)
    const int32_t* other;   // partner atom per incidence
    const double* r0;       // rest length per incidence
    const double* k;        // constant per incidence
};

// Device scratch of the force computation: staged cells (sized for FP64),
// per-chunk counts and per-(chunk group, atom) partial gradients.
struct ForceSizes {
    int64_t partial_doubles = 0;
    size_t staged_bytes = 0;
    int64_t counts = 0;
};
struct ForceScratch {
    double* partial;
    int64_t partial_doubles;
    void* staged;
    size_t staged_bytes;
    int* count;
    int64_t counts;
};
ForceSizes force_sizes(const Grid& g, int64_t natoms, int64_t nfar);
// ex, ey, ez: the cell field as stored by the density kernel of the same
// precision (float for 32, double for 64).
hipError_t launch_forces(const Grid& g, const Atoms& a, const Physics& ph, int precision,
                         const uint32_t* bits, const void* ex, const void* ey,
                         const void* ez, const double4* far_pts, const double* far_ex,
                         const double* far_ey, const double* far_ez, int64_t nfar,
                         const Bonds& bonds, const double* g_extra, const ForceScratch& scr,
                         double* f_out, hipStream_t st);

hipError_t launch_bond_energy(const Atoms& a, const Bonds& bonds, double* partial, int nblocks,
                              double* out, hipStream_t st);

// Solute-solute terms beyond bonds (bending, torsion, non-bonded pairs) on
// the device.  slot: (3 nang + 4 ntor) x 3 gradient rows, angle t's rows
// 3t .. 3t+2 (atoms i, j, k), torsion t's rows 3 nang + 4t .. +3; inc_off /
// inc_slot list, per atom, the rows that act on it.  Exclusion partners per
// atom are sorted ascending.  pair_part: nsplit x n x 5 (used when
// nonbonded).  Outputs: grad (n x 3), eatom (n x 2).
constexpr int SOLUTE_SPLITS_MAX = 32;
struct Solute {
    int64_t n;
    const double4* pos;
    int64_t nang;
    const int4* ang;          // i, j (vertex), k, 0
    const double2* ang_prm;   // theta0, B
    int64_t ntor;
    const int4* tor;          // i, j, k, l
    const double* tor_prm;    // 8 per torsion: a0, K_1 .. K_6, 0
    double* slot;
    const int32_t* inc_off;
    const int32_t* inc_slot;
    int nonbonded;
    int nsplit;
    const double4* nb_prm;    // sigma / 2, sqrt(eps), Q, 0
    const int32_t* x_off;
    const int32_t* x_other;
    double kcoul;             // coulomb_k / eps_w
    double* pair_part;
    double* grad;
    double* eatom;
};
int solute_splits(int64_t natoms);
// partial: 4 x nblocks doubles (1 <= nblocks <= 4096); out[0..3] = bending,
// torsion, LJ and Coulomb energies.
hipError_t launch_solute(const Solute& s, double* partial, int nblocks, double* out,
                         hipStream_t st);

}  // namespace vesis
