// Solvent forces: the adjoint of the density sum.
//
// At fixed labels the discrete energy depends on the atoms through
//   sum_j w_j U(x_j),  w_j = h^3 [phi_j = +1] on grid cells and the
//   quadrature weight on far-field nodes,
// so  dG/dr_n = sum_j w_j grad_{r_n} U(x_j) with, for d = x_j - r_n,
//   grad_{r_n} rho_w U_LJ = 24 rho_w eps_n (2 s^6 - s^3) d / r^2,  s = sigma_n^2/r^2
//   grad_{r_n} Ccfa |E|^2 = -2 Ccfa Q_n [E/r^3 - 3 (E.d) d / r^5]
// (the solvent terms of the Appendix gradient, taken as the exact derivative
// of the discrete energy; E_j comes from the density kernel).  Within the
// r2_min floor the LJ part is constant and E_n = Q_n d / r_min^3.
//
// Layout: a workgroup owns 256 atoms (one per lane) and one chunk of cells
// (a cubic brick of the grid, or a run of far-field nodes).  Cells stream
// through LDS 256 at a time; the solvent cells of a tile (w != 0) are
// compacted in cell order (wave ballots, so the summation order is fixed)
// and staged once as (position relative to the chunk centre, w, w E) in FP32,
// read by broadcast; every lane keeps FP32 partials per tile folded into
// FP64.  Per pair the LJ term and the (E.d) d part of the CFA term share one
// coefficient along d, the E/r^3 part is summed separately.  Each (chunk, atom) pair writes one
// FP64 partial gradient; a second kernel sums the chunks of each atom in a
// fixed order and adds the bond terms, so the result is deterministic.
#include "internal.h"
#include "reduce.h"

namespace vesis {
namespace {

constexpr int AWG = 256;   // atoms per workgroup
constexpr int CT = 256;    // cells per LDS tile
constexpr int FAR_TILES = 16;

int chunk_edge(int n, int64_t natoms) {
    const int64_t ablk = (natoms + AWG - 1) / AWG;
    int cb = 64;
    while (cb > 8) {
        const int64_t nc = (int64_t)((n + cb - 1) / cb) * ((n + cb - 1) / cb) * ((n + cb - 1) / cb);
        if (nc * ablk >= 2048) break;
        cb /= 2;
    }
    return cb;
}

struct ForceArgs {
    Grid g;
    Atoms a;
    Physics ph;
    const uint32_t* bits;
    const double* ex;
    const double* ey;
    const double* ez;
    const double4* far_pts;
    const double* far_ex;
    const double* far_ey;
    const double* far_ez;
    int64_t nfar;
    int cb;          // grid chunk edge
    int ncx;         // grid chunks per axis
    int64_t ngrid_chunks;
    double* partial; // [chunk][atom][3]
};

template <typename T>
struct V4 {};
template <>
struct V4<float> { using type = float4; };
template <>
struct V4<double> { using type = double4; };

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

template <typename T>
__global__ __launch_bounds__(AWG) void force_adjoint_kernel(ForceArgs f) {
    using T4 = typename V4<T>::type;
    __shared__ T4 scell[CT];
    __shared__ T4 sfld[CT];
    __shared__ int wcnt[AWG / 64];
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int64_t chunk = blockIdx.y;
    const int64_t atom = (int64_t)blockIdx.x * AWG + t;
    const bool has_atom = atom < f.a.n;
    const Grid& g = f.g;

    // chunk origin and extent
    double ox, oy, oz;
    int64_t ncells;
    int ci = 0, cj = 0, ck = 0;
    int64_t far0 = 0;
    const bool is_grid = chunk < f.ngrid_chunks;
    if (is_grid) {
        ci = (int)(chunk % f.ncx);
        cj = (int)((chunk / f.ncx) % f.ncx);
        ck = (int)(chunk / ((int64_t)f.ncx * f.ncx));
        ox = g.x0 + (ci * f.cb + 0.5 * (f.cb - 1)) * g.h;
        oy = g.y0 + (cj * f.cb + 0.5 * (f.cb - 1)) * g.h;
        oz = g.z0 + (ck * f.cb + 0.5 * (f.cb - 1)) * g.h;
        ncells = (int64_t)f.cb * f.cb * f.cb;
    } else {
        far0 = (chunk - f.ngrid_chunks) * (int64_t)(CT * FAR_TILES);
        const double4 o = f.far_pts[far0];
        ox = o.x;
        oy = o.y;
        oz = o.z;
        const int64_t rem = f.nfar - far0;
        ncells = rem < CT * FAR_TILES ? rem : CT * FAR_TILES;
    }

    // per-lane atom: position relative to the chunk origin and the two
    // per-atom factors, 24 rho_w eps (LJ) and -2 Ccfa Q (CFA)
    T ax = 0, ay = 0, az = 0, sig2 = 0, e24 = 0, k3 = 0;
    double kq = 0.0;
    if (has_atom) {
        const double4 p = f.a.pos[atom];
        const double4 q = f.a.prm64[atom];
        ax = (T)(p.x - ox);
        ay = (T)(p.y - oy);
        az = (T)(p.z - oz);
        sig2 = (T)q.x;
        e24 = (T)(6.0 * q.y);
        kq = -2.0 * f.ph.ccfa * q.z;
        k3 = (T)(3.0 * kq);
    }
    const T r2min = (T)f.ph.r2min;
    double gd[3] = {0.0, 0.0, 0.0}, ge[3] = {0.0, 0.0, 0.0};

    for (int64_t base = 0; base < ncells; base += CT) {
        // stage the tile's cells with nonzero weight, in cell order
        const int64_t li = base + t;
        T px = 0, py = 0, pz = 0, w = 0, wx = 0, wy = 0, wz = 0;
        bool keep = false;
        if (li < ncells) {
            if (is_grid) {
                const int lx = (int)(li % f.cb), ly = (int)((li / f.cb) % f.cb),
                          lz = (int)(li / ((int64_t)f.cb * f.cb));
                const int x = ci * f.cb + lx, y = cj * f.cb + ly, z = ck * f.cb + lz;
                if (x < g.n && y < g.n && z < g.n) {
                    const uint32_t word = f.bits[g.row(y, z) + 1 + (x >> 5)];
                    if ((word >> (x & 31)) & 1u) {
                        const int64_t c = (int64_t)x + (int64_t)g.n * (y + (int64_t)g.n * z);
                        const double wd = f.ph.h3;
                        px = (T)((lx - 0.5 * (f.cb - 1)) * g.h);
                        py = (T)((ly - 0.5 * (f.cb - 1)) * g.h);
                        pz = (T)((lz - 0.5 * (f.cb - 1)) * g.h);
                        w = (T)wd;
                        wx = (T)(wd * f.ex[c]);
                        wy = (T)(wd * f.ey[c]);
                        wz = (T)(wd * f.ez[c]);
                        keep = true;
                    }
                }
            } else {
                const int64_t pidx = far0 + li;
                const double4 p = f.far_pts[pidx];
                px = (T)(p.x - ox);
                py = (T)(p.y - oy);
                pz = (T)(p.z - oz);
                w = (T)p.w;
                wx = (T)(p.w * f.far_ex[pidx]);
                wy = (T)(p.w * f.far_ey[pidx]);
                wz = (T)(p.w * f.far_ez[pidx]);
                keep = true;
            }
        }
        const uint64_t bal = __ballot(keep);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        __syncthreads();  // previous tile fully consumed
        if (lane == 0) wcnt[wv] = __popcll(bal);
        __syncthreads();
        int off = 0, cnt = 0;
#pragma unroll
        for (int k = 0; k < AWG / 64; ++k) {
            off += (k < wv) ? wcnt[k] : 0;
            cnt += wcnt[k];
        }
        if (keep) {
            scell[off + before] = mk4(px, py, pz, w);
            sfld[off + before] = mk4(wx, wy, wz, (T)0);
        }
        __syncthreads();
        T dx_ = 0, dy_ = 0, dz_ = 0, ex_ = 0, ey_ = 0, ez_ = 0;
#pragma unroll 2
        for (int m = 0; m < cnt; ++m) {
            const T4 c = scell[m];
            const T4 e = sfld[m];
            const T dx = c.x - ax, dy = c.y - ay, dz = c.z - az;
            const T r2 = dx * dx + dy * dy + dz * dz;
            const bool inside = r2 < r2min;
            const T ir = rsq<T>(inside ? r2min : r2);
            const T ir2 = ir * ir;
            const T ir3 = ir2 * ir;
            const T s = sig2 * ir2;
            const T s3 = s * s * s;
            const T lj = (c.w * ir2) * ((s3 + s3) * s3 - s3);
            const T ed = e.x * dx + e.y * dy + e.z * dz;
            T coef = e24 * lj - k3 * (ed * (ir3 * ir2));
            coef = inside ? (T)0 : coef;
            dx_ += coef * dx;
            dy_ += coef * dy;
            dz_ += coef * dz;
            ex_ += ir3 * e.x;
            ey_ += ir3 * e.y;
            ez_ += ir3 * e.z;
        }
        gd[0] += dx_;
        gd[1] += dy_;
        gd[2] += dz_;
        ge[0] += ex_;
        ge[1] += ey_;
        ge[2] += ez_;
    }
    if (!has_atom) return;
    double* out = f.partial + (chunk * f.a.n + atom) * 3;
    out[0] = gd[0] + kq * ge[0];
    out[1] = gd[1] + kq * ge[1];
    out[2] = gd[2] + kq * ge[2];
}

// F_n = -(sum over chunks of the partial gradients + bond gradient).
__global__ void force_reduce_kernel(int64_t natoms, int64_t nchunks, const double* partial,
                                    const double4* pos, Bonds bonds, double* f_out) {
    const int64_t atom = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (atom >= natoms) return;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int64_t c = 0; c < nchunks; ++c) {
        const double* p = partial + (c * natoms + atom) * 3;
        g0 += p[0];
        g1 += p[1];
        g2 += p[2];
    }
    if (bonds.nb > 0) {
        const double4 pa = pos[atom];
        for (int e = bonds.off[atom]; e < bonds.off[atom + 1]; ++e) {
            const double4 pb = pos[bonds.other[e]];
            const double dx = pa.x - pb.x, dy = pa.y - pb.y, dz = pa.z - pb.z;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double c = bonds.k[e] * (r - bonds.r0[e]) / r;
            g0 += c * dx;
            g1 += c * dy;
            g2 += c * dz;
        }
    }
    f_out[3 * atom + 0] = -g0;
    f_out[3 * atom + 1] = -g1;
    f_out[3 * atom + 2] = -g2;
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

int64_t force_partial_chunks(const Grid& g, int64_t natoms, int64_t nfar) {
    const int cb = chunk_edge(g.n, natoms);
    const int64_t ncx = (g.n + cb - 1) / cb;
    return ncx * ncx * ncx + (nfar + CT * FAR_TILES - 1) / (CT * FAR_TILES);
}

hipError_t launch_forces(const Grid& g, const Atoms& a, const Physics& ph, int precision,
                         const uint32_t* bits, const double* ex, const double* ey,
                         const double* ez, const double4* far_pts, const double* far_ex,
                         const double* far_ey, const double* far_ez, int64_t nfar,
                         const Bonds& bonds, double* partial, int64_t nchunk_cap,
                         double* f_out, hipStream_t st) {
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
    f.cb = chunk_edge(g.n, a.n);
    f.ncx = (g.n + f.cb - 1) / f.cb;
    f.ngrid_chunks = (int64_t)f.ncx * f.ncx * f.ncx;
    f.partial = partial;
    const int64_t nfar_chunks = (nfar + CT * FAR_TILES - 1) / (CT * FAR_TILES);
    const int64_t nchunks = f.ngrid_chunks + nfar_chunks;
    if (nchunks > nchunk_cap) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.n + AWG - 1) / AWG), (unsigned)nchunks);
    if (precision == 64)
        hipLaunchKernelGGL(force_adjoint_kernel<double>, grid, dim3(AWG), 0, st, f);
    else
        hipLaunchKernelGGL(force_adjoint_kernel<float>, grid, dim3(AWG), 0, st, f);
    hipLaunchKernelGGL(force_reduce_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st,
                       a.n, nchunks, partial, a.pos, bonds, f_out);
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
