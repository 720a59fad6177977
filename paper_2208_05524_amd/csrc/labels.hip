// Binary level set on the GPU: initial labels, colour flip passes, energy
// reductions.  Labels are bit-packed (see Grid in internal.h).
//
// Flip pass (Eqs. "dGj1", "dGj2"; Step 2.2).  For one colour c = (a, b, cc)
// only the x-rows with y = b (mod p), z = cc (mod p) hold candidates, and in
// them the cells with x = a (mod p).  One lane owns one 32-cell word of such
// a row: it forms the band mask of all 32 cells with a few shifts and XORs
// (a cell is in the band when a face neighbour carries the other label) and
// keeps the colour-a cells.  The workgroup lists its lanes' candidates and
// shares them out, one per thread, and for each evaluates
//     Delta E_j = phi_j (c S_j - h^3 U_j),  S_j = sum_{0<|o|<delta/h} phi_{j+o} K(|o|/rho_s)
// (the two cases of the paper's flip energy in one expression).  S_j is
// computed exactly as sum over squared offsets s of w_s * n_s with integer
// counts n_s = #solvent - #solute, read from 5-bit windows of 25 neighbour
// rows.  A candidate whose |Delta E| lies within h^3 times the density error
// bound is a near tie: the workgroup recomputes U_j in FP64 (each thread a
// strided share of the atoms, fixed tree sum), caches it, and decides.
// Cells of one colour lie outside each other's kernel support, so all
// decisions of a pass read only labels that the pass does not change.
#include <algorithm>
#include <cmath>

#include "internal.h"
#include "reduce.h"

namespace vesis {
namespace {

__global__ void fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void fill_f64(double* p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void fill_i64(int64_t* p, int64_t n, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// bits of a word for x = 32 w ... 32 w + 31 that lie inside the box
__device__ inline uint32_t valid_mask(int n, int x0) {
    const int m = n - x0;
    return m >= 32 ? 0xffffffffu : ((1u << m) - 1u);
}

// Cell centre c - L + (i + 1/2) h per axis, the grid's definition, evaluated
// without contraction so that label decisions on a sphere or a union of
// spheres round exactly as the definition reads.
__device__ inline double centre_coord(double c, double L, int i, double h) {
#pragma clang fp contract(off)
    return (c - L) + ((double)i + 0.5) * h;
}

// ---------------------------------------------------------------- init

__global__ void init_loose_kernel(Grid g, double R0, uint32_t* bits) {
#pragma clang fp contract(off)
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)g.nwin * g.n * g.n;
    if (tid >= total) return;
    const int w = (int)(tid % g.nwin);
    const int64_t r = tid / g.nwin;
    const int y = (int)(r % g.n), z = (int)(r / g.n);
    const double py = centre_coord(g.cy, g.L, y, g.h) - g.cy;
    const double pz = centre_coord(g.cz, g.L, z, g.h) - g.cz;
    uint32_t word = 0xffffffffu;
    const int x0 = 32 * w;
    for (int b = 0; b < 32 && x0 + b < g.n; ++b) {
        const double px = centre_coord(g.cx, g.L, x0 + b, g.h) - g.cx;
        if (sqrt(px * px + py * py + pz * pz) <= R0) word &= ~(1u << b);
    }
    bits[g.row(y, z) + 1 + w] = word;
}

// Tight surface: solute iff min_i (|x - r_i| - d_i) <= 0, d_i = scale sigma_i,
// i.e. the union over atoms of the cells within d_i of the atom.  Scattered
// from the atoms (after the labels are filled with solvent): one lane per
// (atom, row) of the atom's box of (2R+1)^2 rows around its cell, R covering
// the largest d_i; the cells of the row within the box are tested exactly as
// defined, in FP64, and the solute ones cleared with one atomic AND per word.
// The union does not depend on the order of the atoms.
__global__ __launch_bounds__(256) void init_tight_kernel(Grid g, Atoms a, double scale, int R,
                                                         uint32_t* bits) {
#pragma clang fp contract(off)
    const int side = 2 * R + 1;
    const int64_t rows = (int64_t)side * side;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= a.n * rows) return;
    const int64_t ai = tid / rows;
    const int r = (int)(tid - ai * rows);
    const double4 p = a.pos[ai];
    const double d = scale * a.prm64[ai].w;
    // the atom's cell along each axis
    const int ix = (int)floor((p.x - (g.cx - g.L)) / g.h);
    const int iy = (int)floor((p.y - (g.cy - g.L)) / g.h);
    const int iz = (int)floor((p.z - (g.cz - g.L)) / g.h);
    const int y = iy + r % side - R, z = iz + r / side - R;
    if (y < 0 || y >= g.n || z < 0 || z >= g.n) return;
    const double dy = centre_coord(g.cy, g.L, y, g.h) - p.y;
    const double dz = centre_coord(g.cz, g.L, z, g.h) - p.z;
    const double lim = d * (1.0 + 1e-9) + 1e-12;
    if (dy * dy + dz * dz > lim * lim) return;  // no cell of this row is within d
    const int xlo = max(0, ix - R), xhi = min(g.n - 1, ix + R);
    uint32_t* row = bits + g.row(y, z) + 1;
    for (int w = xlo >> 5; w <= (xhi >> 5); ++w) {
        uint32_t mask = 0;
        const int xa = max(xlo, 32 * w), xb = min(xhi, 32 * w + 31);
        for (int x = xa; x <= xb; ++x) {
            const double dx = centre_coord(g.cx, g.L, x, g.h) - p.x;
            if (sqrt(dx * dx + dy * dy + dz * dz) - d <= 0.0) mask |= 1u << (x & 31);
        }
        if (mask) atomicAnd(&row[w], ~mask);
    }
}

// ------------------------------------------------------------- stencil

// The 25 x-rows (y + dy, z + dz) with dy^2 + dz^2 <= 8 around a word, three
// words each (left, own, right), loaded once per lane.
struct Rows25 {
    uint32_t l[25], c[25], r[25];
};

__device__ inline void load_rows(const Grid& g, const uint32_t* bits, int w, int y, int z,
                                 Rows25& R) {
    int k = 0;
#pragma unroll
    for (int dz = -2; dz <= 2; ++dz) {
#pragma unroll
        for (int dy = -2; dy <= 2; ++dy) {
            if (dy * dy + dz * dz > 8) continue;
            const uint32_t* p = bits + g.row(y + dy, z + dz) + w;
            R.l[k] = p[0];
            R.c[k] = p[1];
            R.r[k] = p[2];
            ++k;
        }
    }
}

// Per row of Rows25, the labels of cells x0 - 2 .. x0 + 61 (x0 = 32 w) as two
// words: bit j of (hi:lo) is cell x0 - 2 + j, so the 5-cell window of the
// cell at bit b (bit 0 = x - 2, bit 2 = x) is the low 5 bits of
// alignbit(hi, lo, b).  Built once per word, shared by its candidates.
struct Win25 {
    uint32_t lo[25], hi[25];
};

__device__ inline void make_windows(const Rows25& R, Win25& W) {
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        W.lo[k] = __builtin_amdgcn_alignbit(R.c[k], R.l[k], 30u);
        W.hi[k] = __builtin_amdgcn_alignbit(R.r[k], R.c[k], 30u);
    }
}

// S_j = sum over offsets 0 < |o|^2 <= 8 of w_{|o|^2} phi_{j+o} for the cell
// at bit b of the lane's word.  cnt[s] counts the solvent neighbours at
// squared offset s, from the window of each row: for a row at dy^2 + dz^2 =
// q, the centre bit lies at s = q, the two bits at dx = +-1 at s = q + 1 and
// the two at dx = +-2 at s = q + 4.  With N_s offsets at squared distance s,
// sum_{|o|^2 = s} phi = 2 cnt[s] - N_s (phi = +1 solvent, -1 solute).
__device__ inline double stencil_sum(const Stencil& sc, const Win25& W, int b) {
    constexpr int N[9] = {0, 6, 12, 8, 6, 24, 24, 0, 12};
    int cnt[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) cnt[s] = 0;
    int k = 0;
#pragma unroll
    for (int dz = -2; dz <= 2; ++dz) {
#pragma unroll
        for (int dy = -2; dy <= 2; ++dy) {
            const int q = dy * dy + dz * dz;
            if (q > 8) continue;
            const uint32_t v = __builtin_amdgcn_alignbit(W.hi[k], W.lo[k], (uint32_t)b);
            if (q > 0) cnt[q] += __popc(v & 0x4u);
            if (q + 1 <= 8) cnt[q + 1] += __popc(v & 0xAu);
            if (q + 4 <= 8) cnt[q + 4] += __popc(v & 0x11u);
            ++k;
        }
    }
    double S = 0.0;
#pragma unroll
    for (int s = 1; s <= 8; ++s) S += sc.w[s] * (double)(2 * cnt[s] - N[s]);
    return S;
}

constexpr int FWG = 256;  // flip-pass workgroup: four wavefronts

// FP64 density parts at cell (x, y, z), summed by the whole workgroup:
// thread t takes atoms t, t + FWG, ...; the partial sums meet in a fixed
// tree in LDS, so the result does not depend on timing.  All threads call.
template <int TU>
__device__ inline void block_density_f64(const Grid& g, const Atoms& a, const Physics& ph, int x,
                                         int y, int z, double* sh, double& u_lj, double& u_cfa) {
    const int t = threadIdx.x;
    const double px = centre_coord(g.cx, g.L, x, g.h);
    const double py = centre_coord(g.cy, g.L, y, g.h);
    const double pz = centre_coord(g.cz, g.L, z, g.h);
    double lj = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    // TU atoms per thread in flight: their loads are issued together (indices
    // clamped to the last atom) and the atoms are added in index order with
    // no branch between them; a slot past the last atom adds +0.0, so each
    // thread's sum is the plain sequential one whatever TU is.
    for (int64_t i0 = t; i0 < a.n; i0 += TU * FWG) {
        double4 P[TU], Q[TU];
#pragma unroll
        for (int u = 0; u < TU; ++u) {
            const int64_t i = i0 + (int64_t)u * FWG < a.n ? i0 + (int64_t)u * FWG : a.n - 1;
            P[u] = a.pos[i];
            Q[u] = a.prm64[i];
        }
#pragma unroll
        for (int u = 0; u < TU; ++u) {
            const bool in = i0 + (int64_t)u * FWG < a.n;
            const double dx = px - P[u].x, dy = py - P[u].y, dz = pz - P[u].z;
            const double r2 = fmax(dx * dx + dy * dy + dz * dz, ph.r2min);
            // 1/r from the hardware estimate and two Newton steps (full FP64 accuracy)
            double ir = __builtin_amdgcn_rsq(r2);
            ir = ir * fma(-0.5 * r2, ir * ir, 1.5);
            ir = ir * fma(-0.5 * r2, ir * ir, 1.5);
            const double ir2 = ir * ir;
            const double s = Q[u].x * ir2;
            const double s3 = s * s * s;
            lj += in ? Q[u].y * (s3 * s3 - s3) : 0.0;
            const double f = Q[u].z * ir2 * ir;
            ex += in ? f * dx : 0.0;
            ey += in ? f * dy : 0.0;
            ez += in ? f * dz : 0.0;
        }
    }
    sh[t] = lj;
    sh[FWG + t] = ex;
    sh[2 * FWG + t] = ey;
    sh[3 * FWG + t] = ez;
    __syncthreads();
    for (int st = FWG / 2; st > 0; st >>= 1) {
        if (t < st) {
            sh[t] += sh[t + st];
            sh[FWG + t] += sh[FWG + t + st];
            sh[2 * FWG + t] += sh[2 * FWG + t + st];
            sh[3 * FWG + t] += sh[3 * FWG + t + st];
        }
        __syncthreads();
    }
    u_lj = sh[0];
    ex = sh[FWG];
    ey = sh[2 * FWG];
    ez = sh[3 * FWG];
    u_cfa = ph.ccfa * (ex * ex + ey * ey + ez * ez);
    __syncthreads();
}

// --------------------------------------------------------------- flip pass

// Activity stamps (one int per label word): a lane that flips cells of word
// (w, y, z) in global pass q writes q into the words w-1..w+1 of the rows
// y-2..y+2, z-2..z+2, which hold every cell whose flip energy or band status
// that flip can change.  The previous evaluation of a word in this colour was
// pass q - ncol; if its stamp is older than that, nothing in its cells'
// neighbourhoods changed since then, every decision would repeat (no flip),
// and the word is skipped.  The first sweep of a call evaluates every word.
// XCD-aware block order.  The chip hands consecutive workgroups of a launch
// to its NXCD dies in turn, and each die has its own L2.  A pass's logical
// blocks run along x, then the colour's rows along y, then z, and each block
// reads the label rows two either side of its own; so the logical blocks are
// dealt out in contiguous runs, one run per die (workgroup b takes logical
// block (b mod NXCD) xcd_blocks + b / NXCD), and each die's L2 serves a slab
// of rows instead of every die fetching rows from all over the grid.
// xcd_blocks = 0 keeps the launch order.
constexpr int NXCD = 8;
__device__ inline int64_t flip_block_of(unsigned b, int64_t xcd_blocks) {
    return xcd_blocks > 0 ? (int64_t)(b % NXCD) * xcd_blocks + b / NXCD : (int64_t)b;
}

// One colour pass of colour period P (2 or 3).  BATCH = false: one molecule,
// described by `one`, its logical blocks from flip_block_of; BATCH = true:
// workgroup b takes entry block_mol[b] = molecule | (logical block <<
// BATCH_MOL_BITS) of `descs` (-1: none), so a block never spans two molecules
// and the host chooses which die runs which molecule.  In a batch, molecules
// flagged in `done` are skipped and the pass index is *pass_base + gpass, so
// that one captured sequence of passes can be replayed.
template <bool BATCH, int P>
__global__ __launch_bounds__(FWG) void flip_pass_kernel(
    MolDesc one, const MolDesc* descs, const int* block_mol, const int* done,
    const int* pass_base, int colour, int sweep, int gpass, int ncol, int64_t xcd_blocks) {
    constexpr int K = (32 + P - 1) / P;  // cells of one colour in a word
    __shared__ double s_red[4 * FWG];
    __shared__ double s_cs[K * FWG];     // c S_j of the near ties, slot-major
    __shared__ int s_item[FWG * K];      // the workgroup's candidates: (owner << 5) | bit
    __shared__ int s_wsum[FWG / 64];     // candidates per wavefront
    __shared__ int s_wyz[3][FWG];        // each lane's word: w, y, z
    __shared__ uint32_t s_fm[FWG], s_tm[FWG];  // flip and near-tie bits per owner
    __shared__ int s_leader;
    __shared__ int s_tie[4];
    // the logical block this workgroup takes (see flip_block_of)
    int mol = 0;
    int64_t lblock = flip_block_of(blockIdx.x, xcd_blocks);
    if (BATCH) {
        const int ent = block_mol[blockIdx.x];
        if (ent < 0) return;  // padding at the end of a shorter XCD's list
        mol = ent & (BATCH_MOLS - 1);
        lblock = ent >> BATCH_MOL_BITS;
        if (done[mol]) return;
        gpass += *pass_base;
    }
    const MolDesc& D = BATCH ? descs[mol] : one;
    const Grid& g = D.g;
    const Stencil& sc = D.sc;
    const Atoms& a = D.a;
    const Physics& ph = D.ph;
    uint32_t* bits = D.bits;
    int* stamp = D.stamp;
    const CellFields& cf = D.f;
    double* u64cache = D.u64cache;
    int* sweep_flips = D.sweep_flips;
    int64_t* counters = D.counters;
    // a sweep that follows a sweep without flips has nothing to do
    if (sweep > 0 && sweep_flips[sweep - 1] == 0) return;
    const int ca = colour % P, cb = (colour / P) % P, cc = colour / (P * P);
    const int ny = (g.n - cb + P - 1) / P, nz = (g.n - cc + P - 1) / P;
    const int64_t total = (int64_t)g.nwin * ny * nz;
    const int64_t tid = lblock * FWG + threadIdx.x;
    const bool active = tid < total;
    int w = 0, y = 0, z = 0;
    if (active) {
        w = (int)(tid % g.nwin);
        const int64_t r = tid / g.nwin;
        y = cb + P * (int)(r % ny);
        z = cc + P * (int)(r / ny);
    }
    const int x0 = 32 * w;
    uint32_t* rowc = bits + g.row(y, z);
    uint32_t C = 0, cand = 0;
    if (active) {
        // the stamp and the band words are loaded together, so that a word
        // still to be evaluated waits for one round trip, not two
        const int stw = stamp[g.row(y, z) + 1 + w];
        C = rowc[w + 1];
        const uint32_t Lw = rowc[w], Rw = rowc[w + 2];
        const uint32_t ym = bits[g.row(y - 1, z) + w + 1], yp = bits[g.row(y + 1, z) + w + 1];
        const uint32_t zm = bits[g.row(y, z - 1) + w + 1], zp = bits[g.row(y, z + 1) + w + 1];
        const uint32_t fresh = (gpass >= ncol && stw < gpass - ncol) ? 0u : 0xffffffffu;
        const uint32_t left = (C << 1) | (Lw >> 31);
        const uint32_t right = (C >> 1) | (Rw << 31);
        const uint32_t band = (C ^ left) | (C ^ right) | (C ^ ym) | (C ^ yp) | (C ^ zm) | (C ^ zp);
        // bits b with (x0 + b) mod P == ca: a fixed pattern shifted by the
        // first such b
        const uint32_t cmask = (P == 2 ? 0x55555555u : 0x49249249u) << (((ca - x0) % P + P) % P);
        cand = band & cmask & valid_mask(g.n, x0) & fresh;
    }
    // The candidate cells are shared out over the workgroup: a prefix sum of
    // the lanes' counts lists them in LDS as (owner thread, bit), and the
    // workgroup takes the list FWG cells at a time, each thread one cell with
    // the owner word's rows (L2-resident), so that a lane with many
    // candidates does not hold its wavefront, nor the workgroup, for as many
    // rounds.  The decisions go back to the owner's masks in LDS; a near tie
    // also keeps c S_j there for the FP64 decision below.  Every cell is
    // evaluated exactly as its owner would.
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    s_fm[t] = 0u;
    s_tm[t] = 0u;
    s_wyz[0][t] = w;
    s_wyz[1][t] = y;
    s_wyz[2][t] = z;
    const int nc = __popc(cand);
    int incl = nc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    if (lane == 63) s_wsum[wv] = incl;
    __syncthreads();
    int base = 0, nitems = 0;
#pragma unroll
    for (int v = 0; v < FWG / 64; ++v) {
        base += v < wv ? s_wsum[v] : 0;
        nitems += s_wsum[v];
    }
    {
        int k = base + incl - nc;
        uint32_t cm = cand;
        while (cm) {
            const int b = __ffs(cm) - 1;
            cm &= cm - 1;
            s_item[k++] = (t << 5) | b;
        }
    }
    __syncthreads();
    for (int k0 = 0; k0 < nitems; k0 += FWG) {
        const int k = k0 + t;
        if (k >= nitems) continue;
        const int it = s_item[k];
        const int b = it & 31;
        const int to = it >> 5;
        const int wo = s_wyz[0][to], yo = s_wyz[1][to], zo = s_wyz[2][to];
        const int64_t c = (int64_t)(32 * wo + b) + (int64_t)g.n * (yo + (int64_t)g.n * zo);
        Win25 Wn;
        uint32_t Co;
        {
            Rows25 R;
            load_rows(g, bits, wo, yo, zo, R);
            Co = R.c[12];  // the owner's word (dy = dz = 0)
            make_windows(R, Wn);
        }
        const double S = stencil_sum(sc, Wn, b);
        const double phi = ((Co >> b) & 1u) ? 1.0 : -1.0;
        const double hU =
            ph.h3 * (cell_value(cf.ulj, cf.f32, c) + cell_value(cf.ucfa, cf.f32, c));
        const double cS = sc.c * S;
        const double dE = phi * (cS - hU);
        const double tol = ph.h3 * cell_value(cf.bound, cf.f32, c) + 4.0e-16 * (fabs(cS) + fabs(hU));
        if (!(fabs(dE) > tol)) {
            const int b0o = ((ca - 32 * wo) % P + P) % P;
            s_cs[((b - b0o) / P) * FWG + to] = cS;
            atomicOr(&s_tm[to], 1u << b);
        } else if (dE < 0.0) {
            atomicOr(&s_fm[to], 1u << b);
        }
    }
    __syncthreads();
    uint32_t flipmask = s_fm[t], tiemask = s_tm[t];
    const int b0 = ((ca - x0) % P + P) % P;  // first bit of this colour in the word
    // near ties: the whole workgroup resolves them one at a time in FP64,
    // lowest thread first; each cell's FP64 parts are computed once per atom
    // configuration and cached (2 x ncell doubles: LJ, then CFA; NaN = none)
    while (__syncthreads_or(tiemask != 0u)) {
        if (t == 0) s_leader = FWG;
        __syncthreads();
        if (tiemask) atomicMin(&s_leader, t);
        __syncthreads();
        const int leader = s_leader;
        if (t == leader) {
            s_tie[0] = __ffs(tiemask) - 1;
            s_tie[1] = y;
            s_tie[2] = z;
            s_tie[3] = x0;
        }
        __syncthreads();
        const int bL = s_tie[0], yL = s_tie[1], zL = s_tie[2], xL = s_tie[3] + bL;
        const int64_t cL = (int64_t)xL + (int64_t)g.n * (yL + (int64_t)g.n * zL);
        double lj = u64cache[cL], cfa = u64cache[g.ncell() + cL];
        if (isnan(lj)) {  // same value for every thread
            // one molecule leaves about one workgroup per CU, so latency
            // rules: 8 atoms in flight; a batch keeps several workgroups
            // per CU, so registers rule: 2
            block_density_f64<BATCH ? 2 : 8>(g, a, ph, xL, yL, zL, s_red, lj, cfa);
            if (t == leader) {
                u64cache[cL] = lj;
                u64cache[g.ncell() + cL] = cfa;
                atomicAdd((unsigned long long*)&counters[1], 1ull);
            }
        }
        if (t == leader) {
            const double cS = s_cs[((bL - b0) / P) * FWG + t];
            const double phi = ((C >> bL) & 1u) ? 1.0 : -1.0;
            const double dE = phi * (cS - ph.h3 * (lj + cfa));
            if (dE < 0.0) flipmask |= 1u << bL;
            tiemask &= ~(1u << bL);
            atomicAdd((unsigned long long*)&counters[0], 1ull);
        }
    }
    if (flipmask) {
        rowc[w + 1] = C ^ flipmask;
        for (int dz = -2; dz <= 2; ++dz)
            for (int dy = -2; dy <= 2; ++dy) {
                int* sr = stamp + g.row(y + dy, z + dz) + w;
                sr[0] = gpass;
                sr[1] = gpass;
                sr[2] = gpass;
            }
    }
    int nf = __popc(flipmask);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nf += __shfl_xor(nf, off);
    if ((t & 63) == 0 && nf) atomicAdd(&sweep_flips[sweep], nf);
}

// The three colour passes (a, cb, cc), a = 0, 1, 2, of colour period 3 in
// one launch.  They share their rows (y = cb, z = cc mod 3), and since the
// kernel reaches two cells, a cell of one of these rows sees no label of
// another of them: across the three passes each row depends on itself
// only.  A workgroup owns whole rows (one lane per word, nwin lanes per row)
// and runs the three passes back to back with its rows' words and their
// stamps in LDS; the other rows a candidate's stencil reads do not change
// during the launch and come from global memory.  Each decision is the one
// the separate passes take (same stencil sums, same stored values, the same
// FP64 near-tie path), so labels, flip counts and stamps are identical: a
// word's stamp is the pass of the latest flip in its neighbourhood, written
// with atomicMax at the end (within the launch only the row's own words can
// be stamped, and those stamps are tracked in LDS).
// BATCH as for flip_pass_kernel: workgroup b takes entry block_mol[b] of
// `descs` (a molecule and a logical block of its rows).
template <bool BATCH>
__global__ __launch_bounds__(FWG) void flip_group3_kernel(MolDesc one, const MolDesc* descs,
                                                          const int* block_mol, const int* done,
                                                          const int* pass_base, int cb, int cc,
                                                          int sweep, int gpass0, int ncol,
                                                          int64_t xcd_blocks) {
    constexpr int P = 3, K = 11;
    __shared__ double s_red[4 * FWG];
    __shared__ double s_cs[K * FWG];
    __shared__ int s_item[FWG * K];
    __shared__ int s_wsum[FWG / 64];
    __shared__ int s_wyz[3][FWG];
    __shared__ uint32_t s_fm[FWG], s_tm[FWG];
    __shared__ uint32_t s_word[FWG];  // each lane's own word, as the passes change it
    __shared__ int s_stw[FWG];        // its stamp, with this launch's flips in the row
    __shared__ int s_leader;
    __shared__ int s_tie[4];
    int mol = 0;
    int64_t lblock = flip_block_of(blockIdx.x, xcd_blocks);
    if (BATCH) {
        const int ent = block_mol[blockIdx.x];
        if (ent < 0) return;  // padding at the end of a shorter XCD's list
        mol = ent & (BATCH_MOLS - 1);
        lblock = ent >> BATCH_MOL_BITS;
        if (done[mol]) return;
        gpass0 += *pass_base;
    }
    const MolDesc& D = BATCH ? descs[mol] : one;
    const Grid& g = D.g;
    const Stencil& sc = D.sc;
    const Atoms& a = D.a;
    const Physics& ph = D.ph;
    uint32_t* bits = D.bits;
    int* stamp = D.stamp;
    const CellFields& cf = D.f;
    double* u64cache = D.u64cache;
    int* sweep_flips = D.sweep_flips;
    int64_t* counters = D.counters;
    if (sweep > 0 && sweep_flips[sweep - 1] == 0) return;
    const int nwin = g.nwin;
    const int rpw = FWG / nwin;  // whole rows per workgroup
    const int ny = (g.n - cb + P - 1) / P, nz = (g.n - cc + P - 1) / P;
    const int64_t nrows = (int64_t)ny * nz;
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int rl = t / nwin, w = t - rl * nwin;
    const int64_t rid = lblock * rpw + rl;
    const bool active = rl < rpw && rid < nrows;
    int y = 0, z = 0;
    if (active) {
        y = cb + P * (int)(rid % ny);
        z = cc + P * (int)(rid / ny);
    }
    const int x0 = 32 * w;
    uint32_t* rowc = bits + g.row(y, z);
    uint32_t C = 0, Lpad = 0, Rpad = 0, ym = 0, yp = 0, zm = 0, zp = 0;
    int stw = 0;
    if (active) {
        stw = stamp[g.row(y, z) + 1 + w];
        C = rowc[w + 1];
        Lpad = rowc[w];      // the row's left padding word when w == 0
        Rpad = rowc[w + 2];  // the right padding word when w == nwin - 1
        ym = bits[g.row(y - 1, z) + w + 1];
        yp = bits[g.row(y + 1, z) + w + 1];
        zm = bits[g.row(y, z - 1) + w + 1];
        zp = bits[g.row(y, z + 1) + w + 1];
    }
    s_word[t] = C;
    s_stw[t] = stw;
    s_wyz[0][t] = w;
    s_wyz[1][t] = y;
    s_wyz[2][t] = z;
    int nflips = 0, last = -1;  // this lane's flips in the launch, pass of its last
    for (int ca = 0; ca < P; ++ca) {
        const int gpass = gpass0 + ca;
        __syncthreads();  // the previous pass's words and stamps are in LDS
        C = s_word[t];
        stw = s_stw[t];
        uint32_t cand = 0;
        if (active) {
            const uint32_t Lw = w == 0 ? Lpad : s_word[t - 1];
            const uint32_t Rw = w == nwin - 1 ? Rpad : s_word[t + 1];
            const uint32_t fresh = (gpass >= ncol && stw < gpass - ncol) ? 0u : 0xffffffffu;
            const uint32_t left = (C << 1) | (Lw >> 31);
            const uint32_t right = (C >> 1) | (Rw << 31);
            const uint32_t band = (C ^ left) | (C ^ right) | (C ^ ym) | (C ^ yp) | (C ^ zm) | (C ^ zp);
            const uint32_t cmask = 0x49249249u << (((ca - x0) % P + P) % P);
            cand = band & cmask & valid_mask(g.n, x0) & fresh;
        }
        s_fm[t] = 0u;
        s_tm[t] = 0u;
        const int nc = __popc(cand);
        int incl = nc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        if (lane == 63) s_wsum[wv] = incl;
        __syncthreads();
        int base = 0, nitems = 0;
#pragma unroll
        for (int v = 0; v < FWG / 64; ++v) {
            base += v < wv ? s_wsum[v] : 0;
            nitems += s_wsum[v];
        }
        {
            int k = base + incl - nc;
            uint32_t cm = cand;
            while (cm) {
                const int b = __ffs(cm) - 1;
                cm &= cm - 1;
                s_item[k++] = (t << 5) | b;
            }
        }
        __syncthreads();
        for (int k0 = 0; k0 < nitems; k0 += FWG) {
            const int k = k0 + t;
            if (k >= nitems) continue;
            const int it = s_item[k];
            const int b = it & 31;
            const int to = it >> 5;
            const int wo = s_wyz[0][to], yo = s_wyz[1][to], zo = s_wyz[2][to];
            const int64_t c = (int64_t)(32 * wo + b) + (int64_t)g.n * (yo + (int64_t)g.n * zo);
            Win25 Wn;
            uint32_t Co;
            {
                Rows25 R;
                load_rows(g, bits, wo, yo, zo, R);
                // the owner's row (dy = dz = 0) as the earlier passes of this
                // launch left it; its padding words never change
                R.c[12] = s_word[to];
                if (wo > 0) R.l[12] = s_word[to - 1];
                if (wo < nwin - 1) R.r[12] = s_word[to + 1];
                Co = R.c[12];
                make_windows(R, Wn);
            }
            const double S = stencil_sum(sc, Wn, b);
            const double phi = ((Co >> b) & 1u) ? 1.0 : -1.0;
            const double hU =
                ph.h3 * (cell_value(cf.ulj, cf.f32, c) + cell_value(cf.ucfa, cf.f32, c));
            const double cS = sc.c * S;
            const double dE = phi * (cS - hU);
            const double tol = ph.h3 * cell_value(cf.bound, cf.f32, c) + 4.0e-16 * (fabs(cS) + fabs(hU));
            if (!(fabs(dE) > tol)) {
                const int b0o = ((ca - 32 * wo) % P + P) % P;
                s_cs[((b - b0o) / P) * FWG + to] = cS;
                atomicOr(&s_tm[to], 1u << b);
            } else if (dE < 0.0) {
                atomicOr(&s_fm[to], 1u << b);
            }
        }
        __syncthreads();
        uint32_t flipmask = s_fm[t], tiemask = s_tm[t];
        const int b0 = ((ca - x0) % P + P) % P;
        while (__syncthreads_or(tiemask != 0u)) {
            if (t == 0) s_leader = FWG;
            __syncthreads();
            if (tiemask) atomicMin(&s_leader, t);
            __syncthreads();
            const int leader = s_leader;
            if (t == leader) {
                s_tie[0] = __ffs(tiemask) - 1;
                s_tie[1] = y;
                s_tie[2] = z;
                s_tie[3] = x0;
            }
            __syncthreads();
            const int bL = s_tie[0], yL = s_tie[1], zL = s_tie[2], xL = s_tie[3] + bL;
            const int64_t cL = (int64_t)xL + (int64_t)g.n * (yL + (int64_t)g.n * zL);
            double lj = u64cache[cL], cfa = u64cache[g.ncell() + cL];
            if (isnan(lj)) {  // same value for every thread
                block_density_f64<BATCH ? 2 : 8>(g, a, ph, xL, yL, zL, s_red, lj, cfa);
                if (t == leader) {
                    u64cache[cL] = lj;
                    u64cache[g.ncell() + cL] = cfa;
                    atomicAdd((unsigned long long*)&counters[1], 1ull);
                }
            }
            if (t == leader) {
                const double cS = s_cs[((bL - b0) / P) * FWG + t];
                const double phi = ((C >> bL) & 1u) ? 1.0 : -1.0;
                const double dE = phi * (cS - ph.h3 * (lj + cfa));
                if (dE < 0.0) flipmask |= 1u << bL;
                tiemask &= ~(1u << bL);
                atomicAdd((unsigned long long*)&counters[0], 1ull);
            }
        }
        if (flipmask) {
            C ^= flipmask;
            s_word[t] = C;
            nflips += __popc(flipmask);
            last = gpass;
            // the row's own words that this flip stamps (w - 1 .. w + 1)
            atomicMax(&s_stw[t], gpass);
            if (w > 0) atomicMax(&s_stw[t - 1], gpass);
            if (w < nwin - 1) atomicMax(&s_stw[t + 1], gpass);
        }
    }
    if (last >= 0) {
        rowc[w + 1] = C;
        for (int dz = -2; dz <= 2; ++dz)
            for (int dy = -2; dy <= 2; ++dy) {
                int* sr = stamp + g.row(y + dy, z + dz) + w;
                atomicMax(&sr[0], last);
                atomicMax(&sr[1], last);
                atomicMax(&sr[2], last);
            }
    }
    int nf = nflips;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nf += __shfl_xor(nf, off);
    if (lane == 0 && nf) atomicAdd(&sweep_flips[sweep], nf);
}

// FP64 density parts of one cell into the near-tie cache (u64cache: LJ,
// then CFA), by one workgroup: the value the colour passes compute for a
// near tie, for the serial schedule's near ties.
__global__ __launch_bounds__(FWG) void cell_density_f64_kernel(Grid g, Atoms a, Physics ph, int x,
                                                               int y, int z, double* u64cache) {
    __shared__ double s_red[4 * FWG];
    double lj = 0.0, cfa = 0.0;
    block_density_f64<8>(g, a, ph, x, y, z, s_red, lj, cfa);
    if (threadIdx.x == 0) {
        const int64_t c = (int64_t)x + (int64_t)g.n * (y + (int64_t)g.n * z);
        u64cache[c] = lj;
        u64cache[g.ncell() + c] = cfa;
    }
}

// Labels from per-cell logits (FP32, x fastest): solute (bit 0) where the
// logit is positive; padding bits stay solvent.
__global__ void labels_from_logits_kernel(Grid g, const float* logits, uint32_t* bits) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)g.nwin * g.n * g.n;
    if (tid >= total) return;
    const int w = (int)(tid % g.nwin);
    const int64_t r = tid / g.nwin;
    const int y = (int)(r % g.n), z = (int)(r / g.n);
    uint32_t word = 0xffffffffu;
    for (int b = 0; b < 32; ++b) {
        const int x = 32 * w + b;
        if (x >= g.n) break;
        if (logits[(int64_t)x + (int64_t)g.n * (y + (int64_t)g.n * z)] > 0.f) word &= ~(1u << b);
    }
    bits[g.row(y, z) + 1 + w] = word;
}

// Before a batch's colour passes: every molecule's activity stamps set older
// than any pass (so its first sweep evaluates every word) and its near-tie
// counters zeroed.  Block (x, k) strides over molecule k's label words.
__global__ void batch_prepare(const MolDesc* descs) {
    const MolDesc& D = descs[blockIdx.y];
    const int64_t nw = D.g.nwords();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += stride)
        D.stamp[i] = -(1 << 30);
    if (blockIdx.x == 0 && threadIdx.x < 2) D.counters[threadIdx.x] = 0;
}

// Zero the sweep flip counters of every molecule of a batch.
__global__ void batch_clear_flips(const MolDesc* descs, int m, int nsweeps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m * nsweeps) descs[i / nsweeps].sweep_flips[i % nsweeps] = 0;
}

// After a group of nsweeps sweeps: a molecule whose group holds a sweep
// without flips is done; the pass counter advances by the group.
__global__ void batch_end_group(const MolDesc* descs, int m, int nsweeps, int ncol, int* done,
                                int* pass_base) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *pass_base += nsweeps * ncol;
    if (i >= m || done[i]) return;
    for (int sw = 0; sw < nsweeps; ++sw)
        if (descs[i].sweep_flips[sw] == 0) {
            done[i] = 1;
            return;
        }
}

// Gather the sweep flip counters of every molecule into one array.
__global__ void batch_gather_flips(const MolDesc* descs, int m, int nsweeps, int* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m * nsweeps) out[i] = descs[i / nsweeps].sweep_flips[i % nsweeps];
}

// ------------------------------------------------------------ reductions

// Sums (without the h^3 weight) of U_LJ and U_CFA over solvent cells, from
// U stored as T (float or double).  A wavefront takes whole x-rows, two at a
// time (lanes along x: each load instruction reads 64 consecutive values),
// rows strided over the grid; U is loaded for every cell
// and selected by its label bit, so the loads do not wait for the labels.
// Per-lane FP64 sums in a fixed order, then a fixed tree per workgroup.
template <typename T>
__global__ __launch_bounds__(RED_WG) void energy_volume_kernel(Grid g, const uint32_t* bits,
                                                               const T* ulj, const T* ucfa,
                                                               double* partial) {
    __shared__ double sh[RED_WG];
    double sa = 0.0, sb = 0.0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = g.n, nrows = g.n * g.n;
    const int wstride = gridDim.x * (RED_WG / 64);
    for (int r0 = blockIdx.x * (RED_WG / 64) + wv; r0 < nrows; r0 += 2 * wstride) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = r0 + k * wstride;
            if (r >= nrows) break;
            const int y = r % n, z = r / n;
            const uint32_t* wrow = bits + g.row(y, z) + 1;
            const T* a = ulj + (int64_t)r * n;
            const T* b = ucfa + (int64_t)r * n;
#pragma unroll 4
            for (int x = lane; x < n; x += 64) {
                const double va = (double)a[x], vb = (double)b[x];
                const bool solvent = (wrow[x >> 5] >> (x & 31)) & 1u;
                sa += solvent ? va : 0.0;
                sb += solvent ? vb : 0.0;
            }
        }
    }
    sa = block_sum(sa, sh);
    sb = block_sum(sb, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sa;
        partial[2 * blockIdx.x + 1] = sb;
    }
}

// T_s = number of (solute j, solvent k) pairs with |x_k - x_j|^2 = s h^2,
// s = 1..8, bit-parallel over the 32 cells of a word.
__global__ __launch_bounds__(RED_WG) void geom_counts_kernel(Grid g, const uint32_t* bits,
                                                             int64_t* partial) {
    __shared__ int64_t sh[RED_WG];
    int64_t cnt[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) cnt[s] = 0;
    const int64_t total = (int64_t)g.nwin * g.n * g.n;
    const int64_t stride = (int64_t)gridDim.x * RED_WG;
    for (int64_t tid = (int64_t)blockIdx.x * RED_WG + threadIdx.x; tid < total; tid += stride) {
        const int w = (int)(tid % g.nwin);
        const int64_t r = tid / g.nwin;
        const int y = (int)(r % g.n), z = (int)(r / g.n);
        const uint32_t C = bits[g.row(y, z) + 1 + w];
        const uint32_t m = ~C & valid_mask(g.n, 32 * w);
        if (!m) continue;
#pragma unroll
        for (int dz = -2; dz <= 2; ++dz) {
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy) {
                const int q = dy * dy + dz * dz;
                if (q > 8) continue;
                const uint32_t* rr = bits + g.row(y + dy, z + dz) + w;
                const uint32_t L = rr[0], Cn = rr[1], R = rr[2];
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx) {
                    const int s = q + dx * dx;
                    if (s == 0 || s > 8) continue;
                    uint32_t nb;
                    if (dx > 0)
                        nb = (Cn >> dx) | (R << (32 - dx));
                    else if (dx < 0)
                        nb = (Cn << (-dx)) | (L >> (32 + dx));
                    else
                        nb = Cn;
                    cnt[s] += __popc(m & nb);
                }
            }
        }
    }
    for (int s = 1; s <= 8; ++s) {
        const int64_t v = block_sum(cnt[s], sh);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * 8 + (s - 1)] = v;
    }
}

// number of band cells (face neighbour with the other label)
__global__ __launch_bounds__(RED_WG) void band_count_kernel(Grid g, const uint32_t* bits,
                                                            int64_t* partial) {
    __shared__ int64_t sh[RED_WG];
    int64_t cnt = 0;
    const int64_t total = (int64_t)g.nwin * g.n * g.n;
    const int64_t stride = (int64_t)gridDim.x * RED_WG;
    for (int64_t tid = (int64_t)blockIdx.x * RED_WG + threadIdx.x; tid < total; tid += stride) {
        const int w = (int)(tid % g.nwin);
        const int64_t r = tid / g.nwin;
        const int y = (int)(r % g.n), z = (int)(r / g.n);
        const uint32_t* rc = bits + g.row(y, z);
        const uint32_t C = rc[w + 1];
        const uint32_t left = (C << 1) | (rc[w] >> 31);
        const uint32_t right = (C >> 1) | (rc[w + 2] << 31);
        const uint32_t band = (C ^ left) | (C ^ right) | (C ^ bits[g.row(y - 1, z) + w + 1]) |
                              (C ^ bits[g.row(y + 1, z) + w + 1]) |
                              (C ^ bits[g.row(y, z - 1) + w + 1]) |
                              (C ^ bits[g.row(y, z + 1) + w + 1]);
        cnt += __popc(band & valid_mask(g.n, 32 * w));
    }
    cnt = block_sum(cnt, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = cnt;
}

inline unsigned nblk(int64_t n, int wg) { return (unsigned)((n + wg - 1) / wg); }

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i64, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_init_loose(const Grid& g, double R0, uint32_t* bits, hipStream_t st) {
    const int64_t total = (int64_t)g.nwin * g.n * g.n;
    hipLaunchKernelGGL(init_loose_kernel, dim3(nblk(total, 256)), dim3(256), 0, st, g, R0, bits);
    return hipGetLastError();
}

hipError_t launch_init_tight(const Grid& g, const Atoms& a, double scale, double dmax,
                             uint32_t* bits, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    // rows within dmax of the atom's cell, plus one for the cell's own offset
    const int R = (int)std::min(std::ceil(dmax / g.h) + 2.0, (double)g.n + 2.0);
    const int64_t threads = a.n * (int64_t)(2 * R + 1) * (2 * R + 1);
    hipLaunchKernelGGL(init_tight_kernel, dim3(nblk(threads, 256)), dim3(256), 0, st, g, a, scale,
                       R, bits);
    return hipGetLastError();
}

hipError_t launch_flip_pass(const Grid& g, const Stencil& sc, const Atoms& a, const Physics& ph,
                            int colour, int sweep, int gpass, uint32_t* bits, int* stamp,
                            const CellFields& f, double* u64cache, int* sweep_flips,
                            int64_t* counters, hipStream_t st) {
    const int p = sc.p;
    const int cb = (colour / p) % p, cc = colour / (p * p);
    const int64_t ny = (g.n - cb + p - 1) / p, nz = (g.n - cc + p - 1) / p;
    const int64_t total = (int64_t)g.nwin * ny * nz;
    if (total <= 0) return hipSuccess;
    MolDesc d{};
    d.g = g;
    d.sc = sc;
    d.a = a;
    d.ph = ph;
    d.f = f;
    d.bits = bits;
    d.stamp = stamp;
    d.u64cache = u64cache;
    d.sweep_flips = sweep_flips;
    d.counters = counters;
    const int64_t xb = (nblk(total, FWG) + NXCD - 1) / NXCD;  // logical blocks per die
    const dim3 grid((unsigned)(xb * NXCD));
    if (p == 2)
        hipLaunchKernelGGL((flip_pass_kernel<false, 2>), grid, dim3(FWG), 0, st, d, nullptr,
                           nullptr, nullptr, nullptr, colour, sweep, gpass, 8, xb);
    else if (p == 3)
        hipLaunchKernelGGL((flip_pass_kernel<false, 3>), grid, dim3(FWG), 0, st, d, nullptr,
                           nullptr, nullptr, nullptr, colour, sweep, gpass, 27, xb);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_flip_group3(const Grid& g, const Stencil& sc, const Atoms& a, const Physics& ph,
                              int group, int sweep, int gpass0, uint32_t* bits, int* stamp,
                              const CellFields& f, double* u64cache, int* sweep_flips,
                              int64_t* counters, hipStream_t st) {
    if (sc.p != 3 || group < 0 || group >= 9 || g.nwin > FWG) return hipErrorInvalidValue;
    const int cb = group % 3, cc = group / 3;
    const int64_t ny = (g.n - cb + 2) / 3, nz = (g.n - cc + 2) / 3;
    const int64_t nrows = ny * nz;
    if (nrows <= 0) return hipSuccess;
    MolDesc d{};
    d.g = g;
    d.sc = sc;
    d.a = a;
    d.ph = ph;
    d.f = f;
    d.bits = bits;
    d.stamp = stamp;
    d.u64cache = u64cache;
    d.sweep_flips = sweep_flips;
    d.counters = counters;
    const int64_t rpw = FWG / g.nwin;
    const int64_t xb = (nblk(nrows, rpw) + NXCD - 1) / NXCD;  // logical blocks per die
    hipLaunchKernelGGL(flip_group3_kernel<false>, dim3((unsigned)(xb * NXCD)), dim3(FWG), 0, st, d,
                       nullptr, nullptr, nullptr, nullptr, cb, cc, sweep, gpass0, 27, xb);
    return hipGetLastError();
}

hipError_t launch_flip_group3_batch(const MolDesc* descs, const int* block_mol, const int* done,
                                    const int* pass_base, int64_t nblocks, int group, int sweep,
                                    int gpass_off, hipStream_t st) {
    if (group < 0 || group >= 9) return hipErrorInvalidValue;
    if (nblocks <= 0) return hipSuccess;
    MolDesc unused{};
    hipLaunchKernelGGL(flip_group3_kernel<true>, dim3((unsigned)nblocks), dim3(FWG), 0, st, unused,
                       descs, block_mol, done, pass_base, group % 3, group / 3, sweep, gpass_off,
                       27, (int64_t)0);
    return hipGetLastError();
}

int64_t flip_blocks(const Grid& g, int p) {
    int64_t nb = flip_slots(g, p) / FWG;
    if (p == 3 && g.nwin <= FWG) {
        const int64_t ny = (g.n + 2) / 3, rpw = FWG / g.nwin;
        nb = std::max(nb, (ny * ny + rpw - 1) / rpw);
    }
    return nb;
}

static_assert(FWG == FLIP_WG, "flip-pass workgroup size");

hipError_t launch_labels_from_logits(const Grid& g, const float* logits, uint32_t* bits,
                                     hipStream_t st) {
    const int64_t total = (int64_t)g.nwin * g.n * g.n;
    hipLaunchKernelGGL(labels_from_logits_kernel, dim3(nblk(total, 256)), dim3(256), 0, st, g,
                       logits, bits);
    return hipGetLastError();
}

int64_t flip_slots(const Grid& g, int p) {
    const int64_t ny = (g.n + p - 1) / p;
    const int64_t slots = (int64_t)g.nwin * ny * ny;
    return (slots + FWG - 1) / FWG * FWG;
}

hipError_t launch_cell_density_f64(const Grid& g, const Atoms& a, const Physics& ph, int x, int y,
                                   int z, double* u64cache, hipStream_t st) {
    if (x < 0 || y < 0 || z < 0 || x >= g.n || y >= g.n || z >= g.n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cell_density_f64_kernel, dim3(1), dim3(FWG), 0, st, g, a, ph, x, y, z,
                       u64cache);
    return hipGetLastError();
}

hipError_t launch_flip_pass_batch(const MolDesc* descs, const int* block_mol, const int* done,
                                  const int* pass_base, int64_t nblocks, int p, int colour,
                                  int sweep, int gpass_off, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    MolDesc unused{};
    const dim3 grid((unsigned)nblocks);
    if (p == 2)
        hipLaunchKernelGGL((flip_pass_kernel<true, 2>), grid, dim3(FWG), 0, st, unused, descs,
                           block_mol, done, pass_base, colour, sweep, gpass_off, 8, (int64_t)0);
    else if (p == 3)
        hipLaunchKernelGGL((flip_pass_kernel<true, 3>), grid, dim3(FWG), 0, st, unused, descs,
                           block_mol, done, pass_base, colour, sweep, gpass_off, 27, (int64_t)0);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_batch_end_group(const MolDesc* descs, int m, int nsweeps, int ncol, int* done,
                                  int* pass_base, hipStream_t st) {
    hipLaunchKernelGGL(batch_end_group, dim3(nblk(m, 256)), dim3(256), 0, st, descs, m, nsweeps,
                       ncol, done, pass_base);
    return hipGetLastError();
}

hipError_t launch_batch_prepare(const MolDesc* descs, int m, int64_t max_words, hipStream_t st) {
    if (m <= 0 || max_words <= 0) return hipSuccess;
    const int64_t bx = std::min<int64_t>((max_words + 4 * 256 - 1) / (4 * 256), 1024);
    hipLaunchKernelGGL(batch_prepare, dim3((unsigned)bx, (unsigned)m), dim3(256), 0, st, descs);
    return hipGetLastError();
}

hipError_t launch_batch_clear_flips(const MolDesc* descs, int m, int nsweeps, hipStream_t st) {
    hipLaunchKernelGGL(batch_clear_flips, dim3(nblk((int64_t)m * nsweeps, 256)), dim3(256), 0, st,
                       descs, m, nsweeps);
    return hipGetLastError();
}

hipError_t launch_batch_gather_flips(const MolDesc* descs, int m, int nsweeps, int* out,
                                     hipStream_t st) {
    hipLaunchKernelGGL(batch_gather_flips, dim3(nblk((int64_t)m * nsweeps, 256)), dim3(256), 0, st,
                       descs, m, nsweeps, out);
    return hipGetLastError();
}

hipError_t launch_energy_volume(const Grid& g, const uint32_t* bits, const CellFields& f,
                                double* partial, int nblocks, double* out, hipStream_t st) {
    if (f.f32)
        hipLaunchKernelGGL(energy_volume_kernel<float>, dim3(nblocks), dim3(RED_WG), 0, st, g,
                           bits, static_cast<const float*>(f.ulj),
                           static_cast<const float*>(f.ucfa), partial);
    else
        hipLaunchKernelGGL(energy_volume_kernel<double>, dim3(nblocks), dim3(RED_WG), 0, st, g,
                           bits, static_cast<const double*>(f.ulj),
                           static_cast<const double*>(f.ucfa), partial);
    hipLaunchKernelGGL((reduce_partials<double, 2>), dim3(1), dim3(RED_WG), 0, st, partial,
                       nblocks, out);
    return hipGetLastError();
}

hipError_t launch_geom_counts(const Grid& g, const uint32_t* bits, int64_t* partial, int nblocks,
                              int64_t* out, hipStream_t st) {
    hipLaunchKernelGGL(geom_counts_kernel, dim3(nblocks), dim3(RED_WG), 0, st, g, bits, partial);
    hipLaunchKernelGGL((reduce_partials<int64_t, 8>), dim3(1), dim3(RED_WG), 0, st, partial,
                       nblocks, out);
    return hipGetLastError();
}

hipError_t launch_band_count(const Grid& g, const uint32_t* bits, int64_t* partial, int nblocks,
                             int64_t* out, hipStream_t st) {
    hipLaunchKernelGGL(band_count_kernel, dim3(nblocks), dim3(RED_WG), 0, st, g, bits, partial);
    hipLaunchKernelGGL((reduce_partials<int64_t, 1>), dim3(1), dim3(RED_WG), 0, st, partial,
                       nblocks, out);
    return hipGetLastError();
}

}  // namespace vesis
