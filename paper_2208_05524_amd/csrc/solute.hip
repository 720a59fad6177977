// Solute-solute terms of Eq. "Gss" beyond the bonds, and their gradients
// (Appendix, "Force calculations of molecular mechanical interactions"):
//
//   bending    (1/2) B (theta - theta0)^2 per triplet (i, j, k), theta the
//              angle at j between r_i - r_j and r_k - r_j;
//   torsion    sum_{n=0..6} C_n [1 + cos(n tau - psi_n)] per quadruple, tau
//              the angle between the planes (i, j, k) and (j, k, l), psi_n in
//              {0, pi}: with Lambda = cos tau this is a0 + sum_n K_n T_n(Lambda)
//              (T_n Chebyshev, K_n = C_n cos psi_n), evaluated by the
//              three-term recurrence, and dW/dLambda = sum_n n K_n U_{n-1}
//              (U_n of the second kind);
//   non-bonded 4 eps_ij [(sigma_ij/r)^12 - (sigma_ij/r)^6] + k Q_i Q_j/(eps_w r)
//              over every pair not on the exclusion list, sigma_ij the mean
//              and eps_ij the geometric mean of the atoms' values.
//
// Everything is FP64.  Bonded terms: one lane per term writes the term's
// gradient on each of its atoms to a slot row; a gather kernel adds, per
// atom, its slot rows in a fixed (CSR) order.  Non-bonded pairs: a
// workgroup holds 256 atoms i (one per lane) and one slice of the partner
// atoms j, staged through LDS 256 at a time and read by broadcast; each lane
// walks its sorted exclusion list alongside the ascending j.  Every pair is
// visited from both ends (half of its energy to each), so a lane owns its
// atom's sums and no atomics are needed; the gather kernel adds the slices
// in order.  All reductions have a fixed order: results are reproducible
// bit for bit.
#include <cmath>

#include "internal.h"
#include "reduce.h"

namespace vesis {
namespace {

constexpr int SWG = 256;

__device__ inline double3 sub(double4 a, double4 b) {
    return make_double3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ inline double dot(double3 a, double3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline double3 cross(double3 a, double3 b) {
    return make_double3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ inline double3 axpy(double a, double3 x, double3 y) {  // a x + y
    return make_double3(fma(a, x.x, y.x), fma(a, x.y, y.y), fma(a, x.z, y.z));
}
__device__ inline void put(double* slot, int64_t row, double3 g) {
    slot[3 * row + 0] = g.x;
    slot[3 * row + 1] = g.y;
    slot[3 * row + 2] = g.z;
}

// Smallest sin(theta) used in the bending gradient and smallest |u|, |v| in
// the torsion gradient: collinear atoms leave the direction undefined.
constexpr double SIN_FLOOR = 1e-12;
constexpr double CROSS_FLOOR2 = 1e-40;

__global__ __launch_bounds__(SWG) void bend_kernel(Solute s, double* partial) {
    __shared__ double sh[SWG];
    double e = 0.0;
    const int64_t stride = (int64_t)gridDim.x * SWG;
    for (int64_t t = (int64_t)blockIdx.x * SWG + threadIdx.x; t < s.nang; t += stride) {
        const int4 id = s.ang[t];
        const double2 pr = s.ang_prm[t];  // theta0, B
        const double4 pj = s.pos[id.y];
        const double3 a = sub(s.pos[id.x], pj), b = sub(s.pos[id.z], pj);
        const double aa = dot(a, a), bb = dot(b, b);
        const double iab = 1.0 / sqrt(aa * bb);
        const double c = fmin(1.0, fmax(-1.0, dot(a, b) * iab));
        const double th = acos(c);
        const double dth = th - pr.x;
        e += 0.5 * pr.y * dth * dth;
        const double sn = fmax(sqrt(fmax(0.0, 1.0 - c * c)), SIN_FLOOR);
        const double pre = pr.y * dth / sn;
        // B dth grad theta: grad_i = (c a/|a|^2 - b/(|a||b|)) / sin, and the
        // same with a, b exchanged for k; j takes minus their sum
        const double3 gi = axpy(pre * c / aa, a, make_double3(-pre * iab * b.x, -pre * iab * b.y,
                                                              -pre * iab * b.z));
        const double3 gk = axpy(pre * c / bb, b, make_double3(-pre * iab * a.x, -pre * iab * a.y,
                                                              -pre * iab * a.z));
        put(s.slot, 3 * t + 0, gi);
        put(s.slot, 3 * t + 1, make_double3(-gi.x - gk.x, -gi.y - gk.y, -gi.z - gk.z));
        put(s.slot, 3 * t + 2, gk);
    }
    e = block_sum(e, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = e;
}

__global__ __launch_bounds__(SWG) void torsion_kernel(Solute s, double* partial) {
    __shared__ double sh[SWG];
    double e = 0.0;
    const int64_t stride = (int64_t)gridDim.x * SWG;
    const int64_t base = 3 * s.nang;
    for (int64_t t = (int64_t)blockIdx.x * SWG + threadIdx.x; t < s.ntor; t += stride) {
        const int4 id = s.tor[t];
        const double* K = s.tor_prm + 8 * t;  // a0, K_1 .. K_6
        const double4 pi = s.pos[id.x], pj = s.pos[id.y], pk = s.pos[id.z], pl = s.pos[id.w];
        const double3 q1 = sub(pj, pi), q2 = sub(pk, pj), q3 = sub(pl, pk);
        const double3 u = cross(q1, q2), v = cross(q2, q3);
        const double uu = fmax(dot(u, u), CROSS_FLOOR2), vv = fmax(dot(v, v), CROSS_FLOOR2);
        const double iuv = 1.0 / sqrt(uu * vv);
        const double L = fmin(1.0, fmax(-1.0, dot(u, v) * iuv));
        // W = a0 + sum K_n T_n(L); dW/dL = sum n K_n U_{n-1}(L).  Entering
        // step n: tm, tn = T_{n-2}, T_{n-1} and um, un = U_{n-2}, U_{n-1}.
        double tm = 1.0, tn = L, w = K[0] + K[1] * L;
        double um = 1.0, un = 2.0 * L, dw = K[1];
#pragma unroll
        for (int n = 2; n <= 6; ++n) {
            const double tp = 2.0 * L * tn - tm;
            tm = tn;
            tn = tp;
            w += K[n] * tn;
            dw += n * K[n] * un;
            const double up = 2.0 * L * un - um;
            um = un;
            un = up;
        }
        e += w;
        // dL/du and dL/dv
        const double3 A = make_double3(v.x * iuv - L * u.x / uu, v.y * iuv - L * u.y / uu,
                                       v.z * iuv - L * u.z / uu);
        const double3 B = make_double3(u.x * iuv - L * v.x / vv, u.y * iuv - L * v.y / vv,
                                       u.z * iuv - L * v.z / vv);
        const double3 g1 = cross(q2, A);                      // dL/dq1
        const double3 a1 = cross(A, q1), b3 = cross(q3, B);
        const double3 g2 = make_double3(a1.x + b3.x, a1.y + b3.y, a1.z + b3.z);  // dL/dq2
        const double3 g3 = cross(B, q2);                      // dL/dq3
        const int64_t r = base + 4 * t;
        put(s.slot, r + 0, make_double3(-dw * g1.x, -dw * g1.y, -dw * g1.z));
        put(s.slot, r + 1, make_double3(dw * (g1.x - g2.x), dw * (g1.y - g2.y), dw * (g1.z - g2.z)));
        put(s.slot, r + 2, make_double3(dw * (g2.x - g3.x), dw * (g2.y - g3.y), dw * (g2.z - g3.z)));
        put(s.slot, r + 3, make_double3(dw * g3.x, dw * g3.y, dw * g3.z));
    }
    e = block_sum(e, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = e;
}

// Non-bonded pairs: blockIdx.x picks 256 atoms i, blockIdx.y the slice of
// partners j in [j0, j1).  Writes, per (slice, i): grad_i (3), half the LJ
// and half the Coulomb energy of its pairs.
__global__ __launch_bounds__(SWG) void pair_kernel(Solute s) {
    __shared__ double4 tp[SWG];
    __shared__ double4 tq[SWG];
    const int64_t n = s.n;
    const int64_t i = (int64_t)blockIdx.x * SWG + threadIdx.x;
    const int64_t per = (n + s.nsplit - 1) / s.nsplit;
    const int64_t j0 = (int64_t)blockIdx.y * per;
    const int64_t j1 = j0 + per < n ? j0 + per : n;
    const bool own = i < n;
    const double4 pi = own ? s.pos[i] : make_double4(0, 0, 0, 0);
    const double4 qi = own ? s.nb_prm[i] : make_double4(0, 0, 0, 0);
    int e = own ? s.x_off[i] : 0;
    const int e1 = own ? s.x_off[i + 1] : 0;
    while (e < e1 && s.x_other[e] < j0) ++e;
    int64_t nextx = e < e1 ? s.x_other[e] : INT64_MAX;
    double gx = 0.0, gy = 0.0, gz = 0.0, elj = 0.0, ecl = 0.0;
    const double kq = s.kcoul * qi.z;
    for (int64_t jt = j0; jt < j1; jt += SWG) {
        __syncthreads();
        const int64_t jl = jt + threadIdx.x;
        if (jl < j1) {
            tp[threadIdx.x] = s.pos[jl];
            tq[threadIdx.x] = s.nb_prm[jl];
        }
        __syncthreads();
        const int cnt = (int)(j1 - jt < SWG ? j1 - jt : SWG);
        if (!own) continue;
        for (int t = 0; t < cnt; ++t) {
            const int64_t j = jt + t;
            if (j == nextx) {
                ++e;
                nextx = e < e1 ? s.x_other[e] : INT64_MAX;
                continue;
            }
            if (j == i) continue;
            const double4 pj = tp[t], qj = tq[t];
            const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ir2 = 1.0 / r2;
            const double ir = sqrt(ir2);
            const double sg = qi.x + qj.x;          // (sigma_i + sigma_j) / 2
            const double ep4 = 4.0 * qi.y * qj.y;   // 4 sqrt(eps_i eps_j)
            const double s2 = sg * sg * ir2;
            const double s6 = s2 * s2 * s2;
            const double cq = kq * qj.z * ir;       // k Q_i Q_j / (eps_w r)
            elj += ep4 * (s6 * s6 - s6);
            ecl += cq;
            // -(dU/dr)/r = [4 eps (12 s^12 - 6 s^6) + k QQ / r] / r^2
            const double c = (ep4 * (12.0 * s6 * s6 - 6.0 * s6) + cq) * ir2;
            gx -= c * dx;
            gy -= c * dy;
            gz -= c * dz;
        }
    }
    if (!own) return;
    double* o = s.pair_part + ((int64_t)blockIdx.y * n + i) * 5;
    o[0] = gx;
    o[1] = gy;
    o[2] = gz;
    o[3] = 0.5 * elj;
    o[4] = 0.5 * ecl;
}

// Per atom: the slices of its pair sums in order, then its bonded slot rows
// in CSR order; writes the gradient and the atom's share of the pair
// energies.
__global__ __launch_bounds__(SWG) void gather_kernel(Solute s) {
    const int64_t a = (int64_t)blockIdx.x * SWG + threadIdx.x;
    if (a >= s.n) return;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0, elj = 0.0, ecl = 0.0;
    if (s.nonbonded) {
        for (int k = 0; k < s.nsplit; ++k) {
            const double* p = s.pair_part + ((int64_t)k * s.n + a) * 5;
            g0 += p[0];
            g1 += p[1];
            g2 += p[2];
            elj += p[3];
            ecl += p[4];
        }
    }
    for (int e = s.inc_off[a]; e < s.inc_off[a + 1]; ++e) {
        const double* p = s.slot + 3 * (int64_t)s.inc_slot[e];
        g0 += p[0];
        g1 += p[1];
        g2 += p[2];
    }
    s.grad[3 * a + 0] = g0;
    s.grad[3 * a + 1] = g1;
    s.grad[3 * a + 2] = g2;
    s.eatom[2 * a + 0] = elj;
    s.eatom[2 * a + 1] = ecl;
}

__global__ __launch_bounds__(SWG) void atom_sum2_kernel(const double* eatom, int64_t n,
                                                        double* partial) {
    __shared__ double sh[SWG];
    double a = 0.0, b = 0.0;
    const int64_t stride = (int64_t)gridDim.x * SWG;
    for (int64_t i = (int64_t)blockIdx.x * SWG + threadIdx.x; i < n; i += stride) {
        a += eatom[2 * i];
        b += eatom[2 * i + 1];
    }
    a = block_sum(a, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = a;
        partial[2 * blockIdx.x + 1] = b;
    }
}

}  // namespace

int solute_splits(int64_t natoms) {
    const int64_t s = (natoms + SWG - 1) / SWG;
    return (int)(s < 1 ? 1 : (s > SOLUTE_SPLITS_MAX ? SOLUTE_SPLITS_MAX : s));
}

hipError_t launch_solute(const Solute& s, double* partial, int nblocks, double* out,
                         hipStream_t st) {
    // partial: 4 x nblocks doubles; out[0..3] = bend, torsion, LJ, Coulomb
    if (nblocks < 1 || nblocks > 4096) return hipErrorInvalidValue;
    double* pb = partial;
    double* pt = partial + nblocks;
    double* pn = partial + 2 * nblocks;
    hipLaunchKernelGGL(bend_kernel, dim3(nblocks), dim3(SWG), 0, st, s, pb);
    hipLaunchKernelGGL((reduce_partials<double, 1>), dim3(1), dim3(RED_WG), 0, st, pb, nblocks,
                       out + 0);
    hipLaunchKernelGGL(torsion_kernel, dim3(nblocks), dim3(SWG), 0, st, s, pt);
    hipLaunchKernelGGL((reduce_partials<double, 1>), dim3(1), dim3(RED_WG), 0, st, pt, nblocks,
                       out + 1);
    const unsigned gx = (unsigned)((s.n + SWG - 1) / SWG);
    if (s.nonbonded)
        hipLaunchKernelGGL(pair_kernel, dim3(gx, (unsigned)s.nsplit), dim3(SWG), 0, st, s);
    hipLaunchKernelGGL(gather_kernel, dim3(gx), dim3(SWG), 0, st, s);
    hipLaunchKernelGGL(atom_sum2_kernel, dim3(nblocks), dim3(SWG), 0, st, s.eatom, s.n, pn);
    hipLaunchKernelGGL((reduce_partials<double, 2>), dim3(1), dim3(RED_WG), 0, st, pn, nblocks,
                       out + 2);
    return hipGetLastError();
}

}  // namespace vesis
