// Solvent forces: the adjoint of the density sum.
//
// At fixed labels the discrete energy depends on the atoms through
//   sum_j w_j U(x_j),  w_j = h^3 [phi_j = +1] on grid cells and the
//   quadrature weight on far-field nodes,
// so  dG/dr_n = sum_j w_j grad_{r_n} U(x_j) with, for d = x_j - r_n,
//   grad_{r_n} rho_w U_LJ = 24 rho_w eps_n (2 s^6 - s^3) d / r^2,  s = sigma_n^6/r^6
//   grad_{r_n} Ccfa |E|^2 = -2 Ccfa Q_n [E/r^3 - 3 (E.d) d / r^5]
// (the solvent terms of the Appendix gradient, taken as the exact derivative
// of the discrete energy; E_j comes from the density kernel).  Within the
// r2_min floor the LJ part is constant and E_n = Q_n d / r_min^3.
//
// Layout.  A staging kernel first compacts, per chunk of cells (a cubic
// 16^3 brick of the grid, or a run of 4096 far-field nodes), what the force
// sum visits, in the working precision.  A grid chunk keeps its x-rows of 16
// cells that hold at least one solvent cell, in row order: per row its
// (y, z) relative to the chunk centre and the span of its solvent cells
// (from the first to the last, widened to whole pairs), per cell (x
// relative to the centre, E); a solute cell of a kept row is staged at
// x = BIG with E = 0, where every term of the pair underflows to exactly
// zero, and the pairs outside the span are not visited (the weight h^3
// common to grid cells multiplies the sums of each tile instead).  Far-field nodes
// are staged one by one as (position, w) and w E.  The
// force kernel gives a workgroup 512 atoms (two per lane: every cell read
// from LDS serves two pairs, which halves the LDS traffic) and a group of
// consecutive chunks; the staged data of each chunk stream through a
// double-buffered LDS tile of 32 rows or 256 nodes (the next tile is fetched
// into registers while the current one is summed, one barrier per tile) and
// are read by broadcast.  The cells of a row share dy, dz and dy^2 + dz^2
// with an atom, and the y and z parts of the sum along d are the row's
// coefficient sum times dy and dz, so a grid pair costs about 20 VALU
// instructions against 24 for a node.  Every lane keeps FP32 partials per
// tile, folded into FP64.  Per
// pair the LJ term and the (E.d) d part of the CFA term share one
// coefficient along d; the E/r^3 part is summed separately.  The r2_min
// floor can only bind for an atom within the chunk's extent (plus a margin):
// waves with no such atom take a loop without the floor test.  Each
// (chunk group, atom) pair writes one FP64 partial gradient; a second kernel
// sums the groups of each atom in a fixed order and adds the bond terms, so
// the result is deterministic.
#include "internal.h"
#include "reduce.h"

namespace vesis {
namespace {

constexpr int AWG = 256;        // lanes per workgroup
constexpr int APL = 2;          // atoms per lane
constexpr int CT = 256;         // staged far-field nodes per LDS tile
constexpr int CB = 16;          // grid chunk edge (cells)
constexpr int CB3 = CB * CB * CB;
constexpr int RT = 2 * CT / CB; // staged grid rows per LDS tile (same LDS as CT nodes)
static_assert(CB * CB == 256, "the staging kernel gives one thread each row of a chunk");
static_assert(AWG == CT, "a force workgroup loads one tile unit per thread");
static_assert(CB <= 16 && 32 % CB == 0, "a chunk row lies within one label word");
constexpr int FAR_CHUNK = 4096; // far-field nodes per chunk
constexpr int GROUP = 4;        // chunks per force workgroup (at least)
constexpr int64_t MAX_GRID_Y = 65535;  // launch limit of the second grid dimension
constexpr int RSPLIT = 8;       // group slices per atom in the reduction
constexpr int RATOMS = 32;      // atoms per reduction workgroup

struct ChunkPlan {
    int ncx;              // grid chunks per axis
    int64_t ngrid;        // grid chunks
    int64_t nfar_chunks;  // far-field chunks
    int64_t nchunks() const { return ngrid + nfar_chunks; }
    // chunks per group: GROUP, or more where the groups would not fit the
    // second grid dimension (grids above ~1000 cells per axis)
    int64_t group() const {
        const int64_t g = (nchunks() + MAX_GRID_Y - 1) / MAX_GRID_Y;
        return g > GROUP ? g : GROUP;
    }
    int64_t ngroups() const { return (nchunks() + group() - 1) / group(); }
    // staged slots (each slot is two 4-vectors; a grid chunk's cells fill
    // the first CB3 4-vectors of its 2 CB3, its rows' (y, z) and spans the
    // rest)
    int64_t slots() const { return ngrid * CB3 + nfar_chunks * FAR_CHUNK; }
};

ChunkPlan chunk_plan(int n, int64_t nfar) {
    ChunkPlan p;
    p.ncx = (n + CB - 1) / CB;
    p.ngrid = (int64_t)p.ncx * p.ncx * p.ncx;
    p.nfar_chunks = (nfar + FAR_CHUNK - 1) / FAR_CHUNK;
    return p;
}

struct ForceArgs {
    Grid g;
    Atoms a;
    Physics ph;
    const uint32_t* bits;
    const void* ex;       // cell field, stored as T
    const void* ey;
    const void* ez;
    const double4* far_pts;
    const double* far_ex;
    const double* far_ey;
    const double* far_ez;
    int64_t nfar;
    int ncx;              // grid chunks per axis
    int64_t ngrid;        // grid chunks
    int64_t nchunks;      // grid + far chunks
    int64_t group;        // chunks per force workgroup
    void* staged;         // [slot][2] 4-vectors of the working precision
    int* count;           // staged rows (grid chunk) or nodes (far chunk)
    double* partial;      // [group][atom][3]
};

template <typename T>
struct V4 {};
template <>
struct V4<float> {
    using type = float4;
    using half = float2;
    // |d| at which r^-3 (hence every term but the r^-3-times-zero-field
    // ones) underflows to exactly zero in this precision
    static constexpr float BIG = 1e18f;
};
template <>
struct V4<double> {
    using type = double4;
    using half = double2;
    static constexpr double BIG = 1e110;
};

__device__ inline float2 mk2(float a, float b) { return make_float2(a, b); }
__device__ inline double2 mk2(double a, double b) { return make_double2(a, b); }
__device__ inline float4 mk4(float a, float b, float c, float d) { return make_float4(a, b, c, d); }
__device__ inline double4 mk4(double a, double b, double c, double d) {
    return make_double4(a, b, c, d);
}

template <typename T>
__device__ inline T rsq(T x);
template <>
__device__ inline float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ inline double rsq<double>(double x) { return sqrt(1.0 / x); }

__device__ inline int64_t chunk_slot0(const ForceArgs& f, int64_t chunk) {
    return chunk < f.ngrid ? chunk * CB3 : f.ngrid * CB3 + (chunk - f.ngrid) * FAR_CHUNK;
}

// Centre of a grid chunk's cell centres, or the first node of a far chunk.
__device__ inline void chunk_origin(const ForceArgs& f, int64_t chunk, double& ox, double& oy,
                                    double& oz) {
    if (chunk < f.ngrid) {
        const int ci = (int)(chunk % f.ncx), cj = (int)((chunk / f.ncx) % f.ncx),
                  ck = (int)(chunk / ((int64_t)f.ncx * f.ncx));
        ox = f.g.x0 + (ci * CB + 0.5 * (CB - 1)) * f.g.h;
        oy = f.g.y0 + (cj * CB + 0.5 * (CB - 1)) * f.g.h;
        oz = f.g.z0 + (ck * CB + 0.5 * (CB - 1)) * f.g.h;
    } else {
        const double4 o = f.far_pts[(chunk - f.ngrid) * FAR_CHUNK];
        ox = o.x;
        oy = o.y;
        oz = o.z;
    }
}

// One workgroup per chunk.  Grid chunk: its x-rows with a solvent cell, in
// row order (one thread per row finds them, then 16 threads per row write
// the row's cells).  Far chunk: its nodes in order.
template <typename T>
__global__ __launch_bounds__(256) void force_stage_kernel(ForceArgs f) {
    using T4 = typename V4<T>::type;
    using T2 = typename V4<T>::half;
    __shared__ int wcnt[4];
    __shared__ int run;
    __shared__ uint32_t s_seg[CB * CB];
    __shared__ int s_row[CB * CB];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t chunk = blockIdx.x;
    const Grid& g = f.g;
    T4* out = static_cast<T4*>(f.staged) + 2 * chunk_slot0(f, chunk);
    if (chunk < f.ngrid) {
        const int ci = (int)(chunk % f.ncx), cj = (int)((chunk / f.ncx) % f.ncx),
                  ck = (int)(chunk / ((int64_t)f.ncx * f.ncx));
        const int x0 = ci * CB;
        const int ly = t % CB, lz = t / CB, y = cj * CB + ly, z = ck * CB + lz;
        uint32_t seg = 0;  // solvent bits of the row's cells
        if (y < g.n && z < g.n) {
            const uint32_t word = f.bits[g.row(y, z) + 1 + (x0 >> 5)];
            seg = (word >> (x0 & 31)) & ((1u << CB) - 1u);
            if (g.n - x0 < CB) seg &= (1u << (g.n - x0)) - 1u;
        }
        const bool keep = seg != 0;
        const uint64_t bal = __ballot(keep);
        if (lane == 0) wcnt[wv] = __popcll(bal);
        __syncthreads();
        int k = __popcll(bal & ((1ull << lane) - 1ull)), nrows = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            k += (v < wv) ? wcnt[v] : 0;
            nrows += wcnt[v];
        }
        T2* rowpos = reinterpret_cast<T2*>(out + CB3);
        int* rowrange = reinterpret_cast<int*>(rowpos + CB * CB);
        if (keep) {
            s_seg[k] = seg;
            s_row[k] = t;
            rowpos[k] = mk2((T)((ly - 0.5 * (CB - 1)) * g.h), (T)((lz - 0.5 * (CB - 1)) * g.h));
            // the row's solvent cells lie in [first, last]; taken as whole
            // pairs (first even, last odd), the cells between being
            // sentinels that add exact zeros
            const int first = __builtin_ctz(seg) & ~1, last = (31 - __builtin_clz(seg)) | 1;
            rowrange[k] = first | (last << 8);
        }
        __syncthreads();
        const int lx = t % CB;
        const T xrel = (T)((lx - 0.5 * (CB - 1)) * g.h);
        for (int k0 = 0; k0 < nrows; k0 += 256 / CB) {
            const int kr = k0 + t / CB;
            if (kr >= nrows) break;
            T4 e = mk4(V4<T>::BIG, (T)0, (T)0, (T)0);
            if ((s_seg[kr] >> lx) & 1u) {
                const int r = s_row[kr];
                const int64_t c = (int64_t)(x0 + lx) +
                                  (int64_t)g.n * (cj * CB + r % CB + (int64_t)g.n * (ck * CB + r / CB));
                e = mk4(xrel, static_cast<const T*>(f.ex)[c], static_cast<const T*>(f.ey)[c],
                        static_cast<const T*>(f.ez)[c]);
            }
            out[kr * CB + lx] = e;
        }
        if (t == 0) f.count[chunk] = nrows;
        return;
    }
    double ox, oy, oz;
    chunk_origin(f, chunk, ox, oy, oz);
    const int64_t far0 = (chunk - f.ngrid) * FAR_CHUNK;
    const int64_t ncells = f.nfar - far0 < FAR_CHUNK ? f.nfar - far0 : FAR_CHUNK;
    if (t == 0) run = 0;
    for (int64_t base = 0; base < ncells; base += 256) {
        const int64_t li = base + t;
        T4 a = mk4((T)0, (T)0, (T)0, (T)0), b = a;
        bool keep = false;
        if (li < ncells) {
            const int64_t pidx = far0 + li;
            const double4 p = f.far_pts[pidx];
            a = mk4((T)(p.x - ox), (T)(p.y - oy), (T)(p.z - oz), (T)p.w);
            b = mk4((T)(p.w * f.far_ex[pidx]), (T)(p.w * f.far_ey[pidx]),
                    (T)(p.w * f.far_ez[pidx]), (T)0);
            keep = true;
        }
        const uint64_t bal = __ballot(keep);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wcnt[wv] = __popcll(bal);
        __syncthreads();
        int off = run, tot = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            off += (v < wv) ? wcnt[v] : 0;
            tot += wcnt[v];
        }
        if (keep) {
            out[2 * (off + before)] = a;
            out[2 * (off + before) + 1] = b;
        }
        __syncthreads();  // everyone has read run and wcnt
        if (t == 0) run += tot;
        __syncthreads();
    }
    if (t == 0) f.count[chunk] = run;
}

// Pairs of one staged tile for the APL atoms of a lane: each staged cell or
// node is read from LDS once and serves APL pairs.  With c1 = 48 rho_w eps
// sigma^12 and c2 = 24 rho_w eps sigma^6 the LJ part of the coefficient
// along d is w r^-8 (c1 r^-6 - c2) and the CFA part -k3 (wE.d) r^-5, so the
// coefficient is r^-5 [w r^-3 (c1 r^-6 - c2) - k3 (wE.d)] (powers from
// r^-1: r^-2, r^-3, r^-5 = r^-2 r^-3, r^-6 = (r^-3)^2).  FLOOR: apply the
// r2_min floor (only needed when an atom of the wave may lie within
// sqrt(r2_min) of a cell of the chunk).
//
// Far-field nodes: (position, w) and w E per node.
template <typename T>
__device__ __forceinline__ void tile_nodes(const typename V4<T>::type* sc, int cnt,
                                           const T (&ax)[APL], const T (&ay)[APL],
                                           const T (&az)[APL], const T (&c1)[APL],
                                           const T (&c2)[APL], const T (&k3)[APL], T r2min,
                                           T (&acc)[APL][6]) {
    using T4 = typename V4<T>::type;
    T s[APL][6];
#pragma unroll
    for (int q = 0; q < APL; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) s[q][k] = 0;
    for (int m = 0; m < cnt; ++m) {
        const T4 c = sc[2 * m];
        const T4 e = sc[2 * m + 1];
#pragma unroll
        for (int q = 0; q < APL; ++q) {
            const T dx = c.x - ax[q], dy = c.y - ay[q], dz = c.z - az[q];
            const T r2 = dx * dx + dy * dy + dz * dz;
            const bool inside = r2 < r2min;
            const T ir = rsq<T>(inside ? r2min : r2);
            const T ir2 = ir * ir;
            const T ir3 = ir2 * ir;
            const T ir5 = ir3 * ir2;
            const T ir6 = ir3 * ir3;
            const T ed = e.x * dx + e.y * dy + e.z * dz;
            const T lj3 = c.w * ir3 * (c1[q] * ir6 - c2[q]);
            const T coef = inside ? (T)0 : ir5 * (lj3 - k3[q] * ed);
            s[q][0] += coef * dx;
            s[q][1] += coef * dy;
            s[q][2] += coef * dz;
            s[q][3] += ir3 * e.x;
            s[q][4] += ir3 * e.y;
            s[q][5] += ir3 * e.z;
        }
    }
#pragma unroll
    for (int q = 0; q < APL; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[q][k] = s[q][k];
}

// Grid rows: (y, z) and the span [first, last] (packed first | last << 8)
// per row, (x, E) per cell, unit weight.  Per row and atom dy, dz and
// dy^2 + dz^2 once; per pair of the span dx, r^2 = dx^2 + (dy^2 + dz^2), the
// coefficient, its x part and its running sum over the row, whose y and z
// parts are taken once at the end of the row.
template <typename T, bool FLOOR>
__device__ __forceinline__ void tile_rows(const typename V4<T>::type* sc,
                                          const typename V4<T>::half* rows, const int* ranges,
                                          int nrows,
                                          const T (&ax)[APL], const T (&ay)[APL],
                                          const T (&az)[APL], const T (&c1)[APL],
                                          const T (&c2)[APL], const T (&k3)[APL], T r2min,
                                          T (&acc)[APL][6]) {
    using T4 = typename V4<T>::type;
    using T2 = typename V4<T>::half;
    T s[APL][6];
#pragma unroll
    for (int q = 0; q < APL; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) s[q][k] = 0;
    for (int r = 0; r < nrows; ++r) {
        const T2 yz = rows[r];
        T dy[APL], dz[APL], ryz[APL], cs[APL];
#pragma unroll
        for (int q = 0; q < APL; ++q) {
            dy[q] = yz.x - ay[q];
            dz[q] = yz.y - az[q];
            ryz[q] = dy[q] * dy[q] + dz[q] * dz[q];
            cs[q] = 0;
        }
        const int rg = ranges[r];
        const int lx1 = rg >> 8;
        // two cells per iteration: the fully unrolled row (16 cells, ~1,300
        // instructions per floor variant) ran 25 % slower than this
#pragma unroll 2
        for (int lx = rg & 255; lx <= lx1; ++lx) {
            const T4 c = sc[r * CB + lx];  // x, Ex, Ey, Ez
#pragma unroll
            for (int q = 0; q < APL; ++q) {
                const T dx = c.x - ax[q];
                const T r2 = dx * dx + ryz[q];
                bool inside = false;
                T ir;
                if (FLOOR) {
                    inside = r2 < r2min;
                    ir = rsq<T>(inside ? r2min : r2);
                } else {
                    ir = rsq<T>(r2);
                }
                const T ir2 = ir * ir;
                const T ir3 = ir2 * ir;
                const T ir5 = ir3 * ir2;
                const T ir6 = ir3 * ir3;
                const T ed = c.y * dx + c.z * dy[q] + c.w * dz[q];
                const T lj3 = ir3 * (c1[q] * ir6 - c2[q]);
                T coef = ir5 * (lj3 - k3[q] * ed);
                if (FLOOR) coef = inside ? (T)0 : coef;
                s[q][0] += coef * dx;
                cs[q] += coef;
                s[q][3] += ir3 * c.y;
                s[q][4] += ir3 * c.z;
                s[q][5] += ir3 * c.w;
            }
        }
#pragma unroll
        for (int q = 0; q < APL; ++q) {
            s[q][1] += cs[q] * dy[q];
            s[q][2] += cs[q] * dz[q];
        }
    }
#pragma unroll
    for (int q = 0; q < APL; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[q][k] = s[q][k];
}

template <typename T>
__global__ __launch_bounds__(AWG) void force_adjoint_kernel(ForceArgs f) {
    using T4 = typename V4<T>::type;
    using T2 = typename V4<T>::half;
    __shared__ T4 sbuf[2][2 * CT];  // 2 CT 4-vectors: CT nodes or RT rows of cells
    __shared__ T2 srow[2][RT];
    __shared__ int srng[2][RT];
    const int t = threadIdx.x;
    const Grid& g = f.g;
    const T4* staged = static_cast<const T4*>(f.staged);

    // lane t holds atoms base + t and base + AWG + t
    int64_t atom[APL];
    bool has[APL];
    double px[APL], py[APL], pz[APL], kq[APL];
    T c1[APL], c2[APL], k3[APL];
#pragma unroll
    for (int q = 0; q < APL; ++q) {
        atom[q] = (int64_t)blockIdx.x * (AWG * APL) + q * AWG + t;
        has[q] = atom[q] < f.a.n;
        px[q] = py[q] = pz[q] = kq[q] = 0.0;
        c1[q] = c2[q] = k3[q] = 0;
        if (has[q]) {
            const double4 p = f.a.pos[atom[q]];
            const double4 prm = f.a.prm64[atom[q]];  // sigma^2, 4 rho_w eps, Q, sigma
            px[q] = p.x;
            py[q] = p.y;
            pz[q] = p.z;
            const double s6 = prm.x * prm.x * prm.x;
            c2[q] = (T)(6.0 * prm.y * s6);
            c1[q] = (T)(12.0 * prm.y * s6 * s6);
            kq[q] = -2.0 * f.ph.ccfa * prm.z;
            k3[q] = (T)(3.0 * kq[q]);
        }
    }
    const T r2min = (T)f.ph.r2min;
    // an atom farther than this from the chunk centre along some axis is at
    // least 2 sqrt(r2_min) from every cell centre of the chunk
    const double reach = 0.5 * (CB - 1) * g.h + 2.0 * sqrt(f.ph.r2min);
    double gd[APL][3], ge[APL][3];
#pragma unroll
    for (int q = 0; q < APL; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) gd[q][k] = ge[q][k] = 0.0;

    const int64_t ch0 = (int64_t)blockIdx.y * f.group;
    const int64_t ch1 = ch0 + f.group < f.nchunks ? ch0 + f.group : f.nchunks;
    for (int64_t chunk = ch0; chunk < ch1; ++chunk) {
        const int cnt = f.count[chunk];
        if (cnt == 0) continue;  // uniform over the workgroup
        double ox, oy, oz;
        chunk_origin(f, chunk, ox, oy, oz);
        T ax[APL], ay[APL], az[APL];
        bool near = false;
#pragma unroll
        for (int q = 0; q < APL; ++q) {
            ax[q] = (T)(px[q] - ox);
            ay[q] = (T)(py[q] - oy);
            az[q] = (T)(pz[q] - oz);
            near = near || (has[q] && fabs(px[q] - ox) <= reach && fabs(py[q] - oy) <= reach &&
                            fabs(pz[q] - oz) <= reach);
        }
        const bool is_grid = chunk < f.ngrid;
        const bool floor = !is_grid || __ballot(near) != 0;
        const double wscale = is_grid ? f.ph.h3 : 1.0;
        const T4* src = staged + 2 * chunk_slot0(f, chunk);
        const T2* rsrc = reinterpret_cast<const T2*>(src + CB3);
        const int* gsrc = reinterpret_cast<const int*>(rsrc + CB * CB);
        // a tile is CT units of two 4-vectors: CT nodes, or RT rows of CB
        // cells (a row is CB / 2 units); rows are CT / RT units apart
        const int per = is_grid ? RT : CT;             // rows or nodes per tile
        const int units = is_grid ? cnt * (CB / 2) : cnt;
        const int ntiles = (cnt + per - 1) / per;
        T4 ra = mk4((T)0, (T)0, (T)0, (T)0), rb = ra;
        T2 rr = mk2((T)0, (T)0);
        int rq = 0;
        if (t < units) {
            ra = src[2 * t];
            rb = src[2 * t + 1];
        }
        if (is_grid && t < RT && t < cnt) {
            rr = rsrc[t];
            rq = gsrc[t];
        }
        sbuf[0][2 * t] = ra;
        sbuf[0][2 * t + 1] = rb;
        if (t < RT) {
            srow[0][t] = rr;
            srng[0][t] = rq;
        }
        __syncthreads();
        for (int tile = 0; tile < ntiles; ++tile) {
            const int nxt = (tile + 1) * CT + t;
            if (tile + 1 < ntiles && nxt < units) {
                ra = src[2 * nxt];
                rb = src[2 * nxt + 1];
            }
            const int nr = (tile + 1) * RT + t;
            if (is_grid && tile + 1 < ntiles && t < RT && nr < cnt) {
                rr = rsrc[nr];
                rq = gsrc[nr];
            }
            const int m = cnt - tile * per < per ? cnt - tile * per : per;
            T acc[APL][6];
            if (!is_grid)
                tile_nodes<T>(sbuf[tile & 1], m, ax, ay, az, c1, c2, k3, r2min, acc);
            else if (floor)
                tile_rows<T, true>(sbuf[tile & 1], srow[tile & 1], srng[tile & 1], m, ax, ay, az,
                                   c1, c2, k3, r2min, acc);
            else
                tile_rows<T, false>(sbuf[tile & 1], srow[tile & 1], srng[tile & 1], m, ax, ay,
                                    az, c1, c2, k3, r2min, acc);
#pragma unroll
            for (int q = 0; q < APL; ++q)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    gd[q][k] += wscale * acc[q][k];
                    ge[q][k] += wscale * acc[q][3 + k];
                }
            if (tile + 1 < ntiles) {
                // the other buffer was last read in tile - 1, before the
                // barrier that ended it
                sbuf[(tile + 1) & 1][2 * t] = ra;
                sbuf[(tile + 1) & 1][2 * t + 1] = rb;
                if (t < RT) {
                    srow[(tile + 1) & 1][t] = rr;
                    srng[(tile + 1) & 1][t] = rq;
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int q = 0; q < APL; ++q) {
        if (!has[q]) continue;
        double* out = f.partial + ((int64_t)blockIdx.y * f.a.n + atom[q]) * 3;
        out[0] = gd[q][0] + kq[q] * ge[q][0];
        out[1] = gd[q][1] + kq[q] * ge[q][1];
        out[2] = gd[q][2] + kq[q] * ge[q][2];
    }
}

// F_n = -(sum over chunk groups of the partial gradients + bond gradient +
// g_extra[n], the gradient of the other solute-solute terms, when given).
// Each of RSPLIT lanes per atom sums a fixed slice of the groups in order;
// the slices are then added in slice order.
__global__ __launch_bounds__(RATOMS * RSPLIT) void force_reduce_kernel(
    int64_t natoms, int64_t ngroups, const double* partial, const double4* pos, Bonds bonds,
    const double* g_extra, double* f_out) {
    __shared__ double sh[RSPLIT][RATOMS][3];
    const int la = threadIdx.x % RATOMS, sl = threadIdx.x / RATOMS;
    const int64_t atom = (int64_t)blockIdx.x * RATOMS + la;
    const int64_t per = (ngroups + RSPLIT - 1) / RSPLIT;
    const int64_t g0 = sl * per, g1 = g0 + per < ngroups ? g0 + per : ngroups;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (atom < natoms) {
        for (int64_t c = g0; c < g1; ++c) {
            const double* p = partial + (c * natoms + atom) * 3;
            s0 += p[0];
            s1 += p[1];
            s2 += p[2];
        }
    }
    sh[sl][la][0] = s0;
    sh[sl][la][1] = s1;
    sh[sl][la][2] = s2;
    __syncthreads();
    if (sl != 0 || atom >= natoms) return;
    double g0s = 0.0, g1s = 0.0, g2s = 0.0;
    for (int k = 0; k < RSPLIT; ++k) {
        g0s += sh[k][la][0];
        g1s += sh[k][la][1];
        g2s += sh[k][la][2];
    }
    if (bonds.nb > 0) {
        const double4 pa = pos[atom];
        for (int e = bonds.off[atom]; e < bonds.off[atom + 1]; ++e) {
            const double4 pb = pos[bonds.other[e]];
            const double dx = pa.x - pb.x, dy = pa.y - pb.y, dz = pa.z - pb.z;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double c = bonds.k[e] * (r - bonds.r0[e]) / r;
            g0s += c * dx;
            g1s += c * dy;
            g2s += c * dz;
        }
    }
    if (g_extra) {
        g0s += g_extra[3 * atom + 0];
        g1s += g_extra[3 * atom + 1];
        g2s += g_extra[3 * atom + 2];
    }
    f_out[3 * atom + 0] = -g0s;
    f_out[3 * atom + 1] = -g1s;
    f_out[3 * atom + 2] = -g2s;
}

// sum over bonds of (1/2) k (r - r0)^2, each bond counted from its lower end
constexpr int BWG = 256;
__global__ __launch_bounds__(BWG) void bond_energy_kernel(int64_t natoms, const double4* pos,
                                                          Bonds bonds, double* partial) {
    __shared__ double sh[BWG];
    double e = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BWG;
    for (int64_t a = (int64_t)blockIdx.x * BWG + threadIdx.x; a < natoms; a += stride) {
        const double4 pa = pos[a];
        for (int k = bonds.off[a]; k < bonds.off[a + 1]; ++k) {
            const int b = bonds.other[k];
            if (b < a) continue;
            const double4 pb = pos[b];
            const double dx = pa.x - pb.x, dy = pa.y - pb.y, dz = pa.z - pb.z;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            e += 0.5 * bonds.k[k] * (r - bonds.r0[k]) * (r - bonds.r0[k]);
        }
    }
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int s = BWG / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

}  // namespace

ForceSizes force_sizes(const Grid& g, int64_t natoms, int64_t nfar) {
    const ChunkPlan p = chunk_plan(g.n, nfar);
    ForceSizes s;
    s.partial_doubles = 3 * p.ngroups() * natoms;
    s.staged_bytes = 2 * sizeof(double4) * p.slots();
    s.counts = p.nchunks();
    return s;
}

hipError_t launch_forces(const Grid& g, const Atoms& a, const Physics& ph, int precision,
                         const uint32_t* bits, const void* ex, const void* ey,
                         const void* ez, const double4* far_pts, const double* far_ex,
                         const double* far_ey, const double* far_ez, int64_t nfar,
                         const Bonds& bonds, const double* g_extra, const ForceScratch& scr,
                         double* f_out, hipStream_t st) {
    const ChunkPlan p = chunk_plan(g.n, nfar);
    const ForceSizes need = force_sizes(g, a.n, nfar);
    if (need.partial_doubles > scr.partial_doubles || need.staged_bytes > scr.staged_bytes ||
        need.counts > scr.counts)
        return hipErrorInvalidValue;
    ForceArgs f;
    f.g = g;
    f.a = a;
    f.ph = ph;
    f.bits = bits;
    f.ex = ex;
    f.ey = ey;
    f.ez = ez;
    f.far_pts = far_pts;
    f.far_ex = far_ex;
    f.far_ey = far_ey;
    f.far_ez = far_ez;
    f.nfar = nfar;
    f.ncx = p.ncx;
    f.ngrid = p.ngrid;
    f.nchunks = p.nchunks();
    f.group = p.group();
    f.staged = scr.staged;
    f.count = scr.count;
    f.partial = scr.partial;
    const dim3 grid((unsigned)((a.n + AWG * APL - 1) / (AWG * APL)), (unsigned)p.ngroups());
    if (precision == 64) {
        hipLaunchKernelGGL(force_stage_kernel<double>, dim3((unsigned)p.nchunks()), dim3(256), 0,
                           st, f);
        hipLaunchKernelGGL(force_adjoint_kernel<double>, grid, dim3(AWG), 0, st, f);
    } else {
        hipLaunchKernelGGL(force_stage_kernel<float>, dim3((unsigned)p.nchunks()), dim3(256), 0,
                           st, f);
        hipLaunchKernelGGL(force_adjoint_kernel<float>, grid, dim3(AWG), 0, st, f);
    }
    hipLaunchKernelGGL(force_reduce_kernel, dim3((unsigned)((a.n + RATOMS - 1) / RATOMS)),
                       dim3(RATOMS * RSPLIT), 0, st, a.n, p.ngroups(), scr.partial, a.pos, bonds,
                       g_extra, f_out);
    return hipGetLastError();
}

hipError_t launch_bond_energy(const Atoms& a, const Bonds& bonds, double* partial, int nblocks,
                              double* out, hipStream_t st) {
    hipLaunchKernelGGL(bond_energy_kernel, dim3(nblocks), dim3(BWG), 0, st, a.n, a.pos, bonds,
                       partial);
    hipLaunchKernelGGL((reduce_partials<double, 1>), dim3(1), dim3(RED_WG), 0, st, partial, nblocks,
                       out);
    return hipGetLastError();
}

}  // namespace vesis
