// Energy density U over the cell grid and over far-field quadrature nodes.
//
// U(x) = rho_w sum_i 4 eps_i [(sigma_i/r)^12 - (sigma_i/r)^6]
//        + Ccfa |sum_i Q_i (x - r_i) / r^3|^2,   r = |x - r_i|   (Eq. "Ur")
//
// The grid kernel is the hot loop of the method (the paper's grid-parallel
// evaluation, Sec. "GPU Implementation"): every cell against every atom.
// Layout on gfx950:
//  * a workgroup of 256 lanes owns a 16 x 8 x 4 brick of cells, 2 cells per
//    lane stacked along z, so the x/y part of each distance is shared by the
//    lane's two cells (2 cells per lane keeps the kernel near 100 VGPRs and
//    5 wavefronts per SIMD, which measured faster than 4 or 8);
//  * atoms stream through LDS in tiles of 256: each lane stages one atom,
//    rebased in FP64 to the brick centre and rounded to FP32 (cell offsets
//    inside the brick are small, so the FP32 differences keep ~7 digits even
//    for the nearest atoms); all four wavefronts then read the tile by LDS
//    broadcast;
//  * the LJ powers come from r^-6 = (r^-2)^3 against per-atom constants
//    4 rho_w eps sigma^6 and 4 rho_w eps sigma^12;
//  * FP32 partial sums over 32 atoms are summed over the 256-atom tile in
//    FP32 and folded into FP64 once per tile;
//  * atoms within 16 cells of the brick centre are summed in FP64 (they
//    carry most of a cell's U, and with it most of the FP32 rounding);
//  * beside U the kernel keeps the absolute sum sum 4 eps (s^6 + s^3) per
//    cell and, per atom tile, a brick-wide bound on sum |Q|/r^2, from which
//    the epilogue writes a bound on |U_stored - U_exact| per cell; flip
//    decisions inside that bound are redone in FP64;
//  * U_LJ, U_CFA, the field E and the bound are stored as float (24 bytes
//    per cell); the FP64 kernel stores doubles.
#include "internal.h"
#include "reduce.h"

namespace vesis {
namespace {

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

constexpr int DWG = 256;
constexpr int BX = 16, BY = 8, BZ = 4, KC = 2;
constexpr int TILE = 256;

// Error bound of the FP32 path.  Atoms within NEAR_CELLS = 16 cells of the
// brick centre are summed in FP64; the others are at r >= 16h - |c| >= 7.6h
// from every cell of the 16 x 8 x 4 brick (|c| <= 8.4h).  The bound below is
// derived for |c|/r <= 2.4 (which held for a radius of 12 cells) and so holds
// with margin; with u = 2^-24:
//  * coordinates: d = fl(c - fl(r_i - O)) has |d_err| <= u (|a| + |c| + r)
//    <= u (2|c| + 2r), so rel(r^2) <= 4u(|c|/r + 1) + 2u <= 16u;
//  * rsqrt (1 ulp): rel(1/r) <= 9u; r^-2: 18.5u; r^-3 = r^-2 r^-1: 28.5u;
//    r^-6 = (r^-3)^2: 58u; the s^3 term c6 r^-6: 59u; the s^6 term
//    c12 r^-6 r^-6: 118u;
//  * sums: 32-term FP32 partials (31u), 8 of them summed in FP32 per tile
//    (7u), then FP64.
// So |U_LJ,fp32 - U_LJ| <= 156u sum_far 4 rho_w eps (s^6 + s^3) (KAPPA_LJ =
// 192 with margin) and each component of E carries <= 74u sum_far |Q|/r^2
// (Q r^-3: 29u, d: 6.8u relative to r; KAPPA_E = 96).  The FP64 near terms:
// a cell centre that is not a binary fraction puts an absolute error of
// ~u64 (|x| + r) on d, so a term's relative error is ~12 u64 |x| / r, largest
// for an atom almost on the cell centre (r at the r2_min floor); NEAR_REL =
// 1e-9 of their absolute sums covers |x| / r up to ~1e5 (e.g. a 13 nm box
// against the 1e-3 nm floor), for this kernel and for an FP64 reference that
// does not rebase coordinates alike.
constexpr double U32 = 5.9604644775390625e-08;   // 2^-24
constexpr double U64 = 1.1102230246251565e-16;   // 2^-53
constexpr double KAPPA_LJ = 192.0;
constexpr double KAPPA_E = 96.0;
constexpr double NEAR_REL = 1.0e-9;
constexpr int SUB = 32;                           // atoms per FP32 partial
// FP64 radius in cells.  The FP32 terms carry rounding that does not average
// out over a cell's sum: v_rsq_f32 returns the value one ulp below the
// correctly rounded one for about one input in ten (mean relative error
// -0.12 u over all inputs), which the power chain scales by 6 and 12 on the
// LJ terms, and each far atom's coordinates are rounded once per brick.  Both
// weigh by the size of the term, i.e. by the nearest far atoms (r^-6 for
// the attractive LJ term): moving the FP64 radius from 12 to 16 cells cuts
// the FP32 share of U_LJ at a far atom's closest approach by (3.6/7.6)^6 and
// the summed rounding of a small molecule's volume energy several-fold, for
// about 2 % more work on a 10^4-atom globule.
constexpr double NEAR_CELLS = 16.0;

// Bound on |U - U_exact| from a bound on the LJ part (errLJ) and a per-
// component bound on the field (errE): |E'|^2 - |E|^2 <= 2|E'| d + d^2 with
// d = sqrt(3) errE.
__device__ inline double cell_bound(double errLJ, double errE, double ex, double ey, double ez,
                                    double ccfa) {
    const double d = 1.7320508075688772 * errE * 1.001;
    const double emag = sqrt(ex * ex + ey * ey + ez * ez);
    return 1.001 * (errLJ + fabs(ccfa) * (2.0 * emag * d + d * d));
}

// The FP32 grid kernel's work for one brick of 16 x 8 x BZV cells (KCV cells
// per lane stacked along z), shared by the single-molecule and the batched
// launches.
template <int KCV, int BZV>
__device__ __forceinline__ void density_brick_f32(const Grid& g, const Atoms& a, const Physics& ph,
                                                  const CellFields& out, int64_t brick) {
    __shared__ float4 spos[TILE];     // far atoms: rebased FP32 position, |Q|
    __shared__ float4 sprm[TILE];     // far atoms: c6, c12, Q
    __shared__ double4 npos[TILE];    // near atoms: FP64 position, sigma^2
    __shared__ double4 nprm[TILE];    // near atoms: 4 rho_w eps, Q, |Q|
    __shared__ int wcnt[2][DWG / 64];
    __shared__ float sae[DWG / 64];  // per wavefront: bound on sum_far |Q|/r^2
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int tx = t & 15, ty = (t >> 4) & 7, tz = t >> 7;
    const int nbx = (g.n + BX - 1) / BX, nby = (g.n + BY - 1) / BY;
    int b = (int)brick;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby;
    const int bz = b / nby;
    const int i = bx * BX + tx, j = by * BY + ty, k0 = bz * BZV + tz * KCV;

    // brick centre in FP64; lane cell offsets from it in FP32 (far atoms)
    // and the lane's cell centres in FP64 (near atoms)
    const double ox = g.x0 + (bx * BX + 0.5 * (BX - 1)) * g.h;
    const double oy = g.y0 + (by * BY + 0.5 * (BY - 1)) * g.h;
    const double oz = g.z0 + (bz * BZV + 0.5 * (BZV - 1)) * g.h;
    const float cx = (float)((tx - 0.5 * (BX - 1)) * g.h);
    const float cy = (float)((ty - 0.5 * (BY - 1)) * g.h);
    const double x64 = g.x0 + i * g.h, y64 = g.y0 + j * g.h;
    float cz[KCV];
    double z64[KCV];
#pragma unroll
    for (int k = 0; k < KCV; ++k) {
        cz[k] = (float)((tz * KCV + k - 0.5 * (BZV - 1)) * g.h);
        z64[k] = g.z0 + (k0 + k) * g.h;
    }
    // atoms within NEAR_CELLS cells of the brick centre are "near": they are
    // summed in FP64; every other atom is at least (NEAR_CELLS - 8.4) h from
    // every cell (and beyond the r2_min floor)
    const double rnear = NEAR_CELLS * g.h + 4.0 * sqrt(ph.r2min);
    const float rnear2 = (float)(rnear * rnear);
    // half extents of the box spanned by the brick's cell centres
    const double hxe = 0.5 * (BX - 1) * g.h, hye = 0.5 * (BY - 1) * g.h, hze = 0.5 * (BZV - 1) * g.h;

    double dP[KCV], dQ[KCV], dEx[KCV], dEy[KCV], dEz[KCV], dMag[KCV], dAE[KCV], nMag[KCV], nAE[KCV];
#pragma unroll
    for (int k = 0; k < KCV; ++k)
        dP[k] = dQ[k] = dEx[k] = dEy[k] = dEz[k] = dMag[k] = dAE[k] = nMag[k] = nAE[k] = 0.0;

    for (int64_t base = 0; base < a.n; base += TILE) {
        // classify this tile's atoms and compact them, in atom order, into
        // the far (FP32) and near (FP64) lists
        const int64_t ai = base + t;
        bool far = false, near = false;
        double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
        float4 q32 = make_float4(0.f, 0.f, 0.f, 0.f);
        float ax = 0.f, ay = 0.f, az = 0.f;
        if (ai < a.n) {
            p = a.pos[ai];
            q32 = a.prm32[ai];
            ax = (float)(p.x - ox);
            ay = (float)(p.y - oy);
            az = (float)(p.z - oz);
            near = fmaf(ax, ax, fmaf(ay, ay, az * az)) < rnear2;
            far = !near;
        }
        const uint64_t bfar = __ballot(far), bnear = __ballot(near);
        const uint64_t below = (1ull << lane) - 1ull;
        __syncthreads();  // the previous tile has been consumed
        if (lane == 0) {
            wcnt[0][wv] = __popcll(bfar);
            wcnt[1][wv] = __popcll(bnear);
        }
        __syncthreads();
        int ofar = 0, onear = 0, nfar = 0, nnear = 0;
#pragma unroll
        for (int w2 = 0; w2 < DWG / 64; ++w2) {
            ofar += (w2 < wv) ? wcnt[0][w2] : 0;
            onear += (w2 < wv) ? wcnt[1][w2] : 0;
            nfar += wcnt[0][w2];
            nnear += wcnt[1][w2];
        }
        // sum over the tile's far atoms of |Q| / d^2, d the distance from the
        // atom to the box of the brick's cell centres: a bound on the tile's
        // sum |Q|/r^2 for every cell of the brick (FP32 terms and wavefront
        // sums; the 1.0001 below covers their rounding)
        float ae = 0.f;
        if (far) {
            const double ex_ = fmax(fabs(p.x - ox) - hxe, 0.0);
            const double ey_ = fmax(fabs(p.y - oy) - hye, 0.0);
            const double ez_ = fmax(fabs(p.z - oz) - hze, 0.0);
            ae = q32.w * __builtin_amdgcn_rcpf((float)(ex_ * ex_ + ey_ * ey_ + ez_ * ez_));
        }
        ae = wave_sum(ae);
        if (lane == 0) sae[wv] = ae;
        if (far) {
            // prm32 = (4 rho_w eps sigma^6, 4 rho_w eps sigma^12, Q, |Q|)
            const int at = ofar + __popcll(bfar & below);
            spos[at] = make_float4(ax, ay, az, q32.w);
            sprm[at] = make_float4(q32.x, q32.y, q32.z, 0.f);
        }
        if (near) {
            const double4 q = a.prm64[ai];   // sigma^2, 4 rho_w eps, Q, sigma
            const int at = onear + __popcll(bnear & below);
            npos[at] = make_double4(p.x, p.y, p.z, q.x);
            nprm[at] = make_double4(q.y, q.z, fabs(q.z), 0.0);
        }
        __syncthreads();

        // far atoms, FP32: 32-atom partials, summed over the tile in FP32,
        // folded into FP64 once per tile
        float TP[KCV], TQ[KCV], TEx[KCV], TEy[KCV], TEz[KCV];
#pragma unroll
        for (int k = 0; k < KCV; ++k) TP[k] = TQ[k] = TEx[k] = TEy[k] = TEz[k] = 0.f;
        for (int m0 = 0; m0 < nfar; m0 += SUB) {
            const int me = (m0 + SUB < nfar) ? m0 + SUB : nfar;
            float P[KCV], Q[KCV], Ex[KCV], Ey[KCV], Ez[KCV];
#pragma unroll
            for (int k = 0; k < KCV; ++k) P[k] = Q[k] = Ex[k] = Ey[k] = Ez[k] = 0.f;
#pragma unroll 2
            for (int m = m0; m < me; ++m) {
                const float4 pp = spos[m];
                const float4 q = sprm[m];
                const float dx = cx - pp.x, dy = cy - pp.y;
                const float dxy = fmaf(dx, dx, dy * dy);
#pragma unroll
                for (int k = 0; k < KCV; ++k) {
                    const float dz = cz[k] - pp.z;
                    // far atoms lie beyond 4 sqrt(r2_min): no floor needed
                    const float r2 = fmaf(dz, dz, dxy);
                    const float ir = __builtin_amdgcn_rsqf(r2);
                    const float ir2 = ir * ir;
                    const float ir3 = ir2 * ir;
                    const float ir6 = ir3 * ir3;
                    // 4 rho_w eps (s^6, s^3) = (c12 r^-12, c6 r^-6)
                    P[k] = fmaf(q.y * ir6, ir6, P[k]);
                    Q[k] = fmaf(q.x, ir6, Q[k]);
                    const float qr3 = q.z * ir3;
                    Ex[k] = fmaf(qr3, dx, Ex[k]);
                    Ey[k] = fmaf(qr3, dy, Ey[k]);
                    Ez[k] = fmaf(qr3, dz, Ez[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < KCV; ++k) {
                TP[k] += P[k];
                TQ[k] += Q[k];
                TEx[k] += Ex[k];
                TEy[k] += Ey[k];
                TEz[k] += Ez[k];
            }
        }
#pragma unroll
        for (int k = 0; k < KCV; ++k) {
            dP[k] += TP[k];
            dQ[k] += TQ[k];
            dEx[k] += TEx[k];
            dEy[k] += TEy[k];
            dEz[k] += TEz[k];
            dMag[k] += (double)TP[k] + (double)TQ[k];
            dAE[k] += 1.0001 * ((double)sae[0] + (double)sae[1] + (double)sae[2] + (double)sae[3]);
        }

        // near atoms, FP64 (1/r from the hardware estimate + two Newton steps)
        for (int m = 0; m < nnear; ++m) {
            const double4 pp = npos[m];
            const double4 q = nprm[m];
            const double dx = x64 - pp.x, dy = y64 - pp.y;
#pragma unroll
            for (int k = 0; k < KCV; ++k) {
                const double dz = z64[k] - pp.z;
                const double r2 = fmax(dx * dx + dy * dy + dz * dz, ph.r2min);
                double ir = __builtin_amdgcn_rsq(r2);
                ir = ir * fma(-0.5 * r2, ir * ir, 1.5);
                ir = ir * fma(-0.5 * r2, ir * ir, 1.5);
                const double ir2 = ir * ir;
                const double sg = pp.w * ir2;
                const double s3 = sg * sg * sg;
                const double es3 = q.x * s3;
                dP[k] += es3 * s3;
                dQ[k] += es3;
                nMag[k] += es3 * s3 + es3;
                const double qr3 = q.y * (ir2 * ir);
                dEx[k] += qr3 * dx;
                dEy[k] += qr3 * dy;
                dEz[k] += qr3 * dz;
                nAE[k] += q.z * ir2;
            }
        }
    }

    if (i >= g.n || j >= g.n) return;
    float* o_lj = static_cast<float*>(out.ulj);
    float* o_cfa = static_cast<float*>(out.ucfa);
    float* o_ex = static_cast<float*>(out.ex);
    float* o_ey = static_cast<float*>(out.ey);
    float* o_ez = static_cast<float*>(out.ez);
    float* o_b = static_cast<float*>(out.bound);
#pragma unroll
    for (int k = 0; k < KCV; ++k) {
        const int kk = k0 + k;
        if (kk >= g.n) continue;
        const int64_t c = (int64_t)i + (int64_t)g.n * (j + (int64_t)g.n * kk);
        const double e2 = dEx[k] * dEx[k] + dEy[k] * dEy[k] + dEz[k] * dEz[k];
        const double ulj = dP[k] - dQ[k], ucfa = ph.ccfa * e2;
        // FP32 storage: the bound adds the rounding of both parts to float
        // (u each) and is itself rounded up
        const double b = cell_bound(KAPPA_LJ * U32 * dMag[k] + NEAR_REL * nMag[k],
                                    KAPPA_E * U32 * dAE[k] + NEAR_REL * nAE[k], dEx[k], dEy[k],
                                    dEz[k], ph.ccfa) +
                         U32 * (fabs(ulj) + fabs(ucfa));
        o_lj[c] = (float)ulj;
        o_cfa[c] = (float)ucfa;
        o_ex[c] = (float)dEx[k];
        o_ey[c] = (float)dEy[k];
        o_ez[c] = (float)dEz[k];
        o_b[c] = (float)(b * (1.0 + 0x1p-22));
    }
}

// Four wavefronts per SIMD: at up to 128 VGPRs the loop keeps its two atoms
// x two cells in flight; the compiler's default allocation lands above 128
// and drops to three.
__global__ __launch_bounds__(DWG) __attribute__((amdgpu_waves_per_eu(4, 8))) void density_grid_f32(
    Grid g, Atoms a, Physics ph, CellFields out) {
    density_brick_f32<KC, BZ>(g, a, ph, out, blockIdx.x);
}

// Batched: block b works on brick b - brick0 of molecule block_mol[b].  Four
// cells per lane hold twice the accumulators: two wavefronts per SIMD.
template <int KCV, int BZV>
__global__ __launch_bounds__(DWG) __attribute__((amdgpu_waves_per_eu(KCV >= 4 ? 2 : 4, 8))) void density_batch_f32(
    const MolDesc* desc, const int* block_mol) {
    const MolDesc& d = desc[block_mol[blockIdx.x]];
    density_brick_f32<KCV, BZV>(d.g, d.a, d.ph, d.f, (int64_t)blockIdx.x - d.brick0);
}

// FP64 variant: same brick and tiling, FP64 arithmetic and accumulation
// throughout, correctly rounded sqrt and division.
__global__ __launch_bounds__(DWG) void density_grid_f64(Grid g, Atoms a, Physics ph,
                                                        CellFields out) {
    __shared__ double4 spos[TILE];
    __shared__ double4 sprm[TILE];
    const int t = threadIdx.x;
    const int tx = t & 15, ty = (t >> 4) & 7, tz = t >> 7;
    const int nbx = (g.n + BX - 1) / BX, nby = (g.n + BY - 1) / BY;
    int b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby;
    const int bz = b / nby;
    const int i = bx * BX + tx, j = by * BY + ty, k0 = bz * BZ + tz * KC;
    const double x = g.x0 + i * g.h, y = g.y0 + j * g.h;
    double z[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) z[k] = g.z0 + (k0 + k) * g.h;

    double P[KC], Q[KC], Ex[KC], Ey[KC], Ez[KC], AE[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        P[k] = Q[k] = Ex[k] = Ey[k] = Ez[k] = AE[k] = 0.0;
    }
    for (int64_t base = 0; base < a.n; base += TILE) {
        __syncthreads();
        const int64_t ai = base + t;
        if (ai < a.n) {
            const double4 p = a.pos[ai];
            const double4 q = a.prm64[ai];
            spos[t] = make_double4(p.x, p.y, p.z, q.x);
            sprm[t] = make_double4(q.y, q.z, fabs(q.z), 0.0);
        } else {
            spos[t] = make_double4(1.0e6, 1.0e6, 1.0e6, 0.0);
            sprm[t] = make_double4(0.0, 0.0, 0.0, 0.0);
        }
        __syncthreads();
        const int cnt = (int)((a.n - base) < TILE ? (a.n - base) : TILE);
        for (int m = 0; m < cnt; ++m) {
            const double4 p = spos[m];
            const double4 q = sprm[m];
            const double dx = x - p.x, dy = y - p.y;
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const double dz = z[k] - p.z;
                double r2 = dx * dx + dy * dy + dz * dz;
                r2 = fmax(r2, ph.r2min);
                const double ir2 = 1.0 / r2;
                const double ir = sqrt(ir2);
                const double s = p.w * ir2;
                const double s3 = s * s * s;
                const double es3 = q.x * s3;
                P[k] += es3 * s3;
                Q[k] += es3;
                const double qr3 = q.y * (ir2 * ir);
                Ex[k] += qr3 * dx;
                Ey[k] += qr3 * dy;
                Ez[k] += qr3 * dz;
                AE[k] += q.z * ir2;
            }
        }
    }
    if (i >= g.n || j >= g.n) return;
    // FP64: one sequential sum over all atoms; coordinates are not rebased,
    // so allow 1e7 u of relative error per term (|x| / r up to ~1e5)
    const double kappa = ((double)a.n + 1.0e7) * U64;
    double* o_lj = static_cast<double*>(out.ulj);
    double* o_cfa = static_cast<double*>(out.ucfa);
    double* o_ex = static_cast<double*>(out.ex);
    double* o_ey = static_cast<double*>(out.ey);
    double* o_ez = static_cast<double*>(out.ez);
    double* o_b = static_cast<double*>(out.bound);
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int kk = k0 + k;
        if (kk >= g.n) continue;
        const int64_t c = (int64_t)i + (int64_t)g.n * (j + (int64_t)g.n * kk);
        o_lj[c] = P[k] - Q[k];
        o_cfa[c] = ph.ccfa * (Ex[k] * Ex[k] + Ey[k] * Ey[k] + Ez[k] * Ez[k]);
        o_ex[c] = Ex[k];
        o_ey[c] = Ey[k];
        o_ez[c] = Ez[k];
        o_b[c] = cell_bound(kappa * (P[k] + Q[k]), kappa * AE[k], Ex[k], Ey[k], Ez[k], ph.ccfa);
    }
}

// Density at arbitrary points (far-field quadrature nodes).  The nodes are
// few (6 nf^2 ntau) against the cells, so the atom range is split across
// blockIdx.y to fill the chip: block (x, s) takes 256 nodes, one per lane,
// and the s-th slice of the atoms, staged through LDS rebased to the block's
// first node, with FP32 partials over 32 atoms folded into FP64.  Slices
// write FP64 partial LJ sums and fields; points_combine adds the slices in
// order and squares the field.
constexpr int PWG = 256;

template <typename T>
struct PTypes;
template <>
struct PTypes<float> {
    using T4 = float4;
    static __device__ float4 mk(float a, float b, float c, float d) { return make_float4(a, b, c, d); }
    // the hardware estimate refined by one Newton step on the residual
    // t = 1 - x y^2 (small, so an FMA keeps its relative accuracy): the
    // estimate's bias (one ulp low for about one input in ten) is removed,
    // which matters here because every node's sum is a sum of terms of one
    // sign; the grid kernel bounds this error by its FP64 radius instead
    static __device__ float rsq(float x) {
        const float y = __builtin_amdgcn_rsqf(x);
        const float t = fmaf(-x, y * y, 1.0f);
        return fmaf(0.5f * y, t, y);
    }
};
template <>
struct PTypes<double> {
    using T4 = double4;
    static __device__ double4 mk(double a, double b, double c, double d) {
        return make_double4(a, b, c, d);
    }
    static __device__ double rsq(double x) { return sqrt(1.0 / x); }
};

// Block (bx, sl) of a far-field evaluation: nodes bx * PWG ..., atom slice sl.
template <typename T>
__device__ __forceinline__ void points_part_block(const double4* pts, int64_t np, const Atoms& a,
                                                  const Physics& ph, int64_t chunk, int nsplit,
                                                  double* part, int64_t bx, int sl) {
    using T4 = typename PTypes<T>::T4;
    __shared__ T4 spos[TILE];
    __shared__ T4 sprm[TILE];
    const int t = threadIdx.x;
    const int64_t lo = (int64_t)sl * chunk;
    const int64_t hi = (lo + chunk < a.n) ? lo + chunk : a.n;
    const int64_t p0 = bx * PWG;
    const int64_t pi = p0 + t;
    const double4 o = pts[p0];
    const double4 me = pts[pi < np ? pi : p0];
    const T px = (T)(me.x - o.x), py = (T)(me.y - o.y), pz = (T)(me.z - o.z);
    const T r2min = (T)ph.r2min;
    double dP = 0, dQ = 0, dEx = 0, dEy = 0, dEz = 0;
    for (int64_t base = lo; base < hi; base += TILE) {
        __syncthreads();
        const int64_t ai = base + t;
        if (ai < hi) {
            const double4 p = a.pos[ai];
            const double4 q = a.prm64[ai];
            spos[t] = PTypes<T>::mk((T)(p.x - o.x), (T)(p.y - o.y), (T)(p.z - o.z), (T)q.x);
            sprm[t] = PTypes<T>::mk((T)q.y, (T)q.z, (T)0, (T)0);
        }
        __syncthreads();
        const int cnt = (int)((hi - base) < TILE ? (hi - base) : TILE);
        for (int m0 = 0; m0 < cnt; m0 += SUB) {
            const int me_ = (m0 + SUB < cnt) ? m0 + SUB : cnt;
            T P = 0, Q = 0, Ex = 0, Ey = 0, Ez = 0;
            for (int m = m0; m < me_; ++m) {
                const T4 p = spos[m];
                const T4 q = sprm[m];
                const T dx = px - p.x, dy = py - p.y, dz = pz - p.z;
                T r2 = dx * dx + dy * dy + dz * dz;
                r2 = r2 > r2min ? r2 : r2min;
                const T ir = PTypes<T>::rsq(r2);
                const T ir2 = ir * ir;
                const T s = p.w * ir2;
                const T s3 = s * s * s;
                const T es3 = q.x * s3;
                P += es3 * s3;
                Q += es3;
                const T qr3 = q.y * (ir2 * ir);
                Ex += qr3 * dx;
                Ey += qr3 * dy;
                Ez += qr3 * dz;
            }
            dP += P;
            dQ += Q;
            dEx += Ex;
            dEy += Ey;
            dEz += Ez;
        }
    }
    if (pi >= np) return;
    const int64_t stride = (int64_t)nsplit * np;
    const int64_t at = (int64_t)sl * np + pi;
    part[at] = dP - dQ;
    part[stride + at] = dEx;
    part[2 * stride + at] = dEy;
    part[3 * stride + at] = dEz;
}

template <typename T>
__global__ __launch_bounds__(PWG) void density_points_part(const double4* pts, int64_t np,
                                                           Atoms a, Physics ph, int64_t chunk,
                                                           int nsplit, double* part) {
    points_part_block<T>(pts, np, a, ph, chunk, nsplit, part, blockIdx.x, blockIdx.y);
}

// Batched: block b works on block b - block0 of molecule block_mol[b], laid
// out as in the single-molecule launch (node block fastest, then slice).
__global__ __launch_bounds__(PWG) void density_points_part_batch(const FarDesc* d,
                                                                 const int* block_mol) {
    const FarDesc& D = d[block_mol[blockIdx.x]];
    const int64_t local = (int64_t)blockIdx.x - D.block0;
    const int64_t nbx = (D.np + PWG - 1) / PWG;
    points_part_block<float>(D.pts, D.np, D.a, D.ph, D.chunk, D.nsplit, D.part, local % nbx,
                             (int)(local / nbx));
}

__device__ __forceinline__ void combine_point(int64_t p, int64_t np, int nsplit, const double* part,
                                              double ccfa, double* ulj, double* ucfa, double* ex,
                                              double* ey, double* ez);

__global__ void points_combine(int64_t np, int nsplit, const double* part, double ccfa,
                               double* ulj, double* ucfa, double* ex, double* ey, double* ez) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    combine_point(p, np, nsplit, part, ccfa, ulj, ucfa, ex, ey, ez);
}

// Batched: block (x, k) combines nodes x * 256 ... of molecule k.
__global__ void points_combine_batch(const FarDesc* d) {
    const FarDesc& D = d[blockIdx.y];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= D.np) return;
    combine_point(p, D.np, D.nsplit, D.part, D.ph.ccfa, D.ulj, D.ucfa, D.ex, D.ey, D.ez);
}

// The slices of node p added in order; the field squared.
__device__ __forceinline__ void combine_point(int64_t p, int64_t np, int nsplit, const double* part,
                                              double ccfa, double* ulj, double* ucfa, double* ex,
                                              double* ey, double* ez) {
    const int64_t stride = (int64_t)nsplit * np;
    double lj = 0, x = 0, y = 0, z = 0;
    for (int s = 0; s < nsplit; ++s) {
        const int64_t at = (int64_t)s * np + p;
        lj += part[at];
        x += part[stride + at];
        y += part[2 * stride + at];
        z += part[3 * stride + at];
    }
    ulj[p] = lj;
    ucfa[p] = ccfa * (x * x + y * y + z * z);
    ex[p] = x;
    ey[p] = y;
    ez[p] = z;
}

// Deterministic two-level sum of w_p a_p and w_p b_p (w = pts[p].w): block
// blk of nblk takes nodes blk * RED_WG + i * nblk * RED_WG.
__device__ __forceinline__ void wsum2_block(const double4* pts, const double* a, const double* b,
                                            int64_t np, double* partial, int blk, int nblk) {
    __shared__ double sh[RED_WG];
    double sa = 0.0, sb = 0.0;
    const int64_t stride = (int64_t)nblk * RED_WG;
    for (int64_t p = (int64_t)blk * RED_WG + threadIdx.x; p < np; p += stride) {
        const double w = pts[p].w;
        sa += w * a[p];
        sb += w * b[p];
    }
    sa = block_sum(sa, sh);
    sb = block_sum(sb, sh);
    if (threadIdx.x == 0) {
        partial[2 * blk] = sa;
        partial[2 * blk + 1] = sb;
    }
}

__global__ __launch_bounds__(RED_WG) void wsum2_stage1(const double4* pts, const double* a,
                                                       const double* b, int64_t np,
                                                       double* partial) {
    wsum2_block(pts, a, b, np, partial, blockIdx.x, gridDim.x);
}

// Batched: block (blk, k) of molecule k's far-field sums; then one block per
// molecule adds its partials as reduce_partials<double, 2> does.
__global__ __launch_bounds__(RED_WG) void wsum2_stage1_batch(const FarDesc* d) {
    const FarDesc& D = d[blockIdx.y];
    wsum2_block(D.pts, D.ulj, D.ucfa, D.np, D.partial, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(RED_WG) void wsum2_stage2_batch(const FarDesc* d, int nblk) {
    __shared__ double sh[RED_WG];
    const FarDesc& D = d[blockIdx.x];
    for (int k = 0; k < 2; ++k) {
        double s = 0;
        for (int i = threadIdx.x; i < nblk; i += RED_WG) s += D.partial[(int64_t)i * 2 + k];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) D.out[k] = s;
    }
}

// Batched: the FP64 near-tie cache of every molecule set to NaN.
__global__ void far_fill_nan_batch(const FarDesc* d) {
    const FarDesc& D = d[blockIdx.y];
    const int64_t n = 2 * D.ncell;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        D.u64cache[i] = __builtin_nan("");
}

}  // namespace

hipError_t launch_density_grid(const Grid& g, const Atoms& a, const Physics& ph, int precision,
                               CellFields out, hipStream_t st) {
    const int nbx = (g.n + BX - 1) / BX, nby = (g.n + BY - 1) / BY, nbz = (g.n + BZ - 1) / BZ;
    const unsigned nblk = (unsigned)(nbx * nby * nbz);
    if (precision == 64)
        hipLaunchKernelGGL(density_grid_f64, dim3(nblk), dim3(DWG), 0, st, g, a, ph, out);
    else
        hipLaunchKernelGGL(density_grid_f32, dim3(nblk), dim3(DWG), 0, st, g, a, ph, out);
    return hipGetLastError();
}

int64_t density_bricks(const Grid& g, int variant) {
    const int bz = variant == 1 ? 2 : (variant == 2 ? 8 : BZ);
    const int64_t nbx = (g.n + BX - 1) / BX, nby = (g.n + BY - 1) / BY, nbz = (g.n + bz - 1) / bz;
    return nbx * nby * nbz;
}

hipError_t launch_density_batch(const MolDesc* desc, const int* block_mol, int64_t nblocks,
                                int variant, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    if (variant == 1)
        hipLaunchKernelGGL((density_batch_f32<1, 2>), dim3((unsigned)nblocks), dim3(DWG), 0, st,
                           desc, block_mol);
    else if (variant == 2)
        hipLaunchKernelGGL((density_batch_f32<4, 8>), dim3((unsigned)nblocks), dim3(DWG), 0, st,
                           desc, block_mol);
    else
        hipLaunchKernelGGL((density_batch_f32<KC, BZ>), dim3((unsigned)nblocks), dim3(DWG), 0, st,
                           desc, block_mol);
    return hipGetLastError();
}

int points_split(int64_t np, int64_t natoms) {
    if (np <= 0) return 1;
    const int64_t nblk = (np + PWG - 1) / PWG;
    int64_t s = (2048 + nblk - 1) / nblk;
    s = s < 1 ? 1 : (s > POINT_SPLITS_MAX ? POINT_SPLITS_MAX : s);
    const int64_t by_atoms = (natoms + 63) / 64;  // at least 64 atoms per slice
    if (s > by_atoms) s = by_atoms < 1 ? 1 : by_atoms;
    return (int)s;
}

hipError_t launch_density_points(const double4* pts, int64_t np, const Atoms& a, const Physics& ph,
                                 int precision, double* part, double* ulj, double* ucfa,
                                 double* ex, double* ey, double* ez, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    const int nsplit = points_split(np, a.n);
    const int64_t chunk = (a.n + nsplit - 1) / nsplit;
    const dim3 grid((unsigned)((np + PWG - 1) / PWG), (unsigned)nsplit);
    if (precision == 64)
        hipLaunchKernelGGL(density_points_part<double>, grid, dim3(PWG), 0, st, pts, np, a, ph,
                           chunk, nsplit, part);
    else
        hipLaunchKernelGGL(density_points_part<float>, grid, dim3(PWG), 0, st, pts, np, a, ph,
                           chunk, nsplit, part);
    hipLaunchKernelGGL(points_combine, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np,
                       nsplit, part, ph.ccfa, ulj, ucfa, ex, ey, ez);
    return hipGetLastError();
}

int64_t points_blocks(int64_t np, int64_t natoms) {
    if (np <= 0) return 0;
    return (np + PWG - 1) / PWG * points_split(np, natoms);
}

hipError_t launch_far_batch(const FarDesc* d, const int* block_mol, int m, int64_t nblocks,
                            int64_t max_np, int64_t max_ncell, int nred, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const unsigned fx = (unsigned)std::min<int64_t>((2 * max_ncell + 1023) / 1024, 4096);
    hipLaunchKernelGGL(far_fill_nan_batch, dim3(fx, (unsigned)m), dim3(256), 0, st, d);
    if (nblocks > 0 && max_np > 0) {
        hipLaunchKernelGGL(density_points_part_batch, dim3((unsigned)nblocks), dim3(PWG), 0, st, d,
                           block_mol);
        hipLaunchKernelGGL(points_combine_batch, dim3((unsigned)((max_np + 255) / 256), (unsigned)m),
                           dim3(256), 0, st, d);
    }
    hipLaunchKernelGGL(wsum2_stage1_batch, dim3((unsigned)nred, (unsigned)m), dim3(RED_WG), 0, st,
                       d);
    hipLaunchKernelGGL(wsum2_stage2_batch, dim3((unsigned)m), dim3(RED_WG), 0, st, d, nred);
    return hipGetLastError();
}

hipError_t launch_weighted_sum2(const double4* pts, const double* a, const double* b, int64_t np,
                                double* partial, int nblocks, double* out, hipStream_t st) {
    hipLaunchKernelGGL(wsum2_stage1, dim3(nblocks), dim3(RED_WG), 0, st, pts, a, b, np, partial);
    hipLaunchKernelGGL((reduce_partials<double, 2>), dim3(1), dim3(RED_WG), 0, st, partial, nblocks,
                       out);
    return hipGetLastError();
}

}  // namespace vesis
