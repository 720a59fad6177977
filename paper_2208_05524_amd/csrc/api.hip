// Host runtime and C ABI of libvesis (see include/vesis.h).
//
// The context keeps host copies of the inputs, validates them, lays out the
// caller's device workspace, and sequences the kernels on the caller's
// stream.  All arithmetic of the hot path runs in the kernels; the host does
// bookkeeping, the adaptive-mobility accept/reject logic on a handful of
// scalars, and the trial positions R - dt omega M grad G.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>

#include "../../include/vesis.h"
#include "internal.h"

using namespace vesis;

namespace {

constexpr int RED_BLOCKS = 1024;   // partial sums per reduction
constexpr int SWEEP_BATCH = 8;     // colour sweeps launched between host checks
constexpr double PI = 3.14159265358979323846;

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_m from
// the asymptotic first guess, P_m and P_m' from the three-term recurrence.
void gauss_legendre_rule(int m, std::vector<double>& x, std::vector<double>& w) {
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int i = 0; i < (m + 1) / 2; ++i) {
        double z = std::cos(PI * (i + 0.75) / (m + 0.5));
        double pm = 0.0, dpm = 1.0;
        for (int it = 0; it < 64; ++it) {
            double a = 1.0, b = z;  // P_0, P_1
            for (int k = 2; k <= m; ++k) {
                const double c = ((2 * k - 1) * z * b - (k - 1) * a) / k;
                a = b;
                b = c;
            }
            pm = (m == 1) ? z : b;
            const double pm1 = (m == 1) ? 1.0 : a;
            dpm = m * (pm1 - z * pm) / (1.0 - z * z);
            const double step = pm / dpm;
            z -= step;
            if (std::fabs(step) <= 1e-16 * std::fabs(z) + 1e-300) break;
        }
        double a = 1.0, b = z;
        for (int k = 2; k <= m; ++k) {
            const double c = ((2 * k - 1) * z * b - (k - 1) * a) / k;
            a = b;
            b = c;
        }
        const double pm1 = (m == 1) ? 1.0 : a;
        pm = (m == 1) ? z : b;
        dpm = m * (pm1 - z * pm) / (1.0 - z * z);
        x[i] = -z;
        x[m - 1 - i] = z;
        w[i] = w[m - 1 - i] = 2.0 / ((1.0 - z * z) * dpm * dpm);
    }
}

struct Layout {
    size_t pos, prm64, prm32, pos_stage;
    size_t boff, bother, br0, bk;
    size_t ulj, ucfa, ex, ey, ez, bound, u64cache;
    size_t bits, stamp;
    size_t far_pts, far_ulj, far_ucfa, far_ex, far_ey, far_ez, far_part;
    size_t red_d, red_i, scal_d, scal_i, sweep_flips;
    size_t fpart, fstage, fcount, fout;
    size_t s_ang, s_angp, s_tor, s_torp, s_slot, s_incoff, s_incslot, s_nbp, s_xoff, s_xother;
    size_t s_part, s_grad, s_eatom, s_red;
    int s_nsplit;
    size_t total;
    ForceSizes fsz;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__global__ void pack_positions(const double* xyz, int64_t n, double4* pos) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pos[i] = make_double4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], 0.0);
}

struct PendingEvent {
    int kind;
    hipEvent_t a, b;
};

}  // namespace

struct vesis_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    bool has_params = false;
    vesis_params prm{};
    bool has_grid = false;
    Grid g{};
    Stencil sc{};
    bool has_atoms = false;
    int64_t na = 0;
    std::vector<double> xyz, q, sigma, eps;
    std::vector<uint8_t> movable;
    int64_t nb = 0;
    std::vector<int32_t> b_off, b_other;
    std::vector<double> b_r0, b_k;
    // solute-solute terms beyond bonds (bending, torsion, non-bonded pairs)
    int64_t nang = 0, ntor = 0;
    std::vector<int32_t> ang;      // 4 per angle: i, j, k, 0
    std::vector<double> ang_prm;   // theta0, B
    std::vector<int32_t> tor;      // 4 per torsion
    std::vector<double> tor_prm;   // 8 per torsion: a0, K_1 .. K_6, 0
    std::vector<int32_t> inc_off, inc_slot;
    bool nonbonded = false;
    std::vector<double> sig_ss, eps_ss;  // empty: the atoms' sigma and eps
    std::vector<int32_t> x_off, x_other;
    std::vector<double> far_host;  // x, y, z, w per node
    int64_t nfar = 0;

    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool has_ws = false;
    Layout lay{};
    int64_t lay_na = -1, lay_nb = -1, lay_nfar = -1;
    int64_t lay_nang = 0, lay_ntor = 0, lay_nxo = 0;
    int lay_cell_bytes = 0;  // bytes per stored cell value of the planned layout
    bool lay_nonbonded = false;
    int lay_n = -1;

    bool has_labels = false;
    bool atoms_uploaded = false;
    bool far_uploaded = false;
    bool bonds_uploaded = false;
    bool ss_uploaded = false;
    bool ss_valid = false;       // solute-solute energies and gradient are current
    bool dens_valid = false;
    bool forces_valid = false;

    hipStream_t capture = nullptr;  // private stream for graph capture (made on first use)
    // the captured group of batched sweeps, kept across calls while the
    // batch workspace, molecule count, pass grid, colour period and flip
    // variant stay the same
    hipGraph_t bgraph = nullptr;
    hipGraphExec_t bexec = nullptr;
    const void* bkey_ws = nullptr;
    int bkey_m = 0, bkey_p = 0, bkey_fv = 0;
    int64_t bkey_nblocks = 0;
    hipEvent_t bev[2] = {nullptr, nullptr};  // completion of the two groups in flight
    // pinned host staging of the batch calls' tables (descriptors, block
    // maps, read-backs), so that their copies need not be waited for
    char* hstage = nullptr;
    size_t hstage_bytes = 0;
    bool hstage_busy = false;  // a copy from it may still be pending

    bool prof = false;
    double prof_ms[K_NKINDS] = {0};
    int64_t prof_n[K_NKINDS] = {0};
    std::vector<PendingEvent> pending;
};

namespace {

vesis_status fail(vesis_ctx* c, vesis_status s, const std::string& m) {
    if (c) c->err = m;
    return s;
}

#define CK(call)                                                                             \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, VESIS_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool finite_all(const double* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

template <typename T>
T* at(vesis_ctx* c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

Atoms dev_atoms(vesis_ctx* c) {
    Atoms a;
    a.n = c->na;
    a.pos = at<double4>(c, c->lay.pos);
    a.prm64 = at<double4>(c, c->lay.prm64);
    a.prm32 = at<float4>(c, c->lay.prm32);
    return a;
}

Physics dev_physics(vesis_ctx* c) {
    Physics ph;
    ph.ccfa = c->prm.coulomb_k / (8.0 * PI) * (1.0 / c->prm.eps_w - 1.0 / c->prm.eps_m);
    ph.r2min = c->prm.r2_min;
    ph.rho_w = c->prm.rho_w;
    ph.h3 = c->g.h * c->g.h * c->g.h;
    return ph;
}

Bonds dev_bonds(vesis_ctx* c) {
    Bonds b;
    b.nb = c->nb;
    b.off = at<int32_t>(c, c->lay.boff);
    b.other = at<int32_t>(c, c->lay.bother);
    b.r0 = at<double>(c, c->lay.br0);
    b.k = at<double>(c, c->lay.bk);
    return b;
}

// Kernel timing: record events around a launch when profiling is on.
struct Timed {
    vesis_ctx* c;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(vesis_ctx* c_, int k) : c(c_), kind(k) {
        if (c->prof) {
            (void)hipEventCreate(&a);
            (void)hipEventCreate(&b);
            (void)hipEventRecord(a, c->stream);
        }
    }
    ~Timed() {
        if (c->prof) {
            (void)hipEventRecord(b, c->stream);
            c->pending.push_back({kind, a, b});
        }
    }
};

void drain_events(vesis_ctx* c) {
    for (auto& e : c->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
            c->prof_ms[e.kind] += ms;
            c->prof_n[e.kind] += 1;
        }
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    c->pending.clear();
}

void compute_stencil(vesis_ctx* c) {
    const double rs = c->prm.rho_s;
    for (int s = 0; s < 9; ++s) {
        const double r = std::sqrt((double)s) / rs;
        double v = 0.0;
        if (s > 0 && (double)s < rs * rs) {
            const double sn = std::sin(PI * r);
            v = sn * sn;
        }
        c->sc.w[s] = v;
    }
    const double C0 = 8.0 * PI / (PI * PI - 3.0);  // = 1 / (pi int_0^1 r^3 sin^2(pi r) dr)
    const double h = c->g.h;
    c->sc.c = c->prm.gamma0 * C0 * h * h / (rs * rs * rs * rs);  // gamma0 C0 h^6 / delta^4
    c->sc.p = (int)std::ceil(rs);
}

void compute_far_nodes(vesis_ctx* c) {
    std::vector<double> gx, gw, tx, tw;
    const int nf = c->prm.far_nf, nt = c->prm.far_ntau;
    gauss_legendre_rule(nf, gx, gw);
    gauss_legendre_rule(nt, tx, tw);
    const double L = c->g.L;
    const double ctr[3] = {c->g.cx, c->g.cy, c->g.cz};
    c->nfar = 6LL * nf * nf * nt;
    c->far_host.assign(4 * c->nfar, 0.0);
    int64_t m = 0;
    for (int face = 0; face < 6; ++face) {
        const int ax = face / 2;
        const double sg = (face & 1) ? -1.0 : 1.0;
        const int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
        for (int it = 0; it < nt; ++it) {
            const double tau = 0.5 * (tx[it] + 1.0), wt = 0.5 * tw[it];
            for (int iv = 0; iv < nf; ++iv)
                for (int iu = 0; iu < nf; ++iu) {
                    double y[3];
                    y[ax] = sg * L;
                    y[a1] = L * gx[iu];
                    y[a2] = L * gx[iv];
                    double* o = &c->far_host[4 * m];
                    for (int d = 0; d < 3; ++d) o[d] = ctr[d] + y[d] / tau;
                    // dV = L tau^-4 du dv dtau on the cone over a face
                    o[3] = (L * gw[iu]) * (L * gw[iv]) * wt * L / (tau * tau * tau * tau);
                    ++m;
                }
        }
    }
    c->far_uploaded = false;
}

// Bytes per stored per-cell density value: float with FP32 sums, double
// with FP64 sums.
int cell_bytes(const vesis_ctx* c) { return c->prm.precision == 64 ? 8 : 4; }

Layout plan(const vesis_ctx* c) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += align256(bytes ? bytes : 1);
        return r;
    };
    const int64_t na = c->na, ncell = c->g.ncell(), nfar = c->nfar;
    const int64_t nbi = 2 * c->nb;
    L.pos = take(32 * na);
    L.prm64 = take(32 * na);
    L.prm32 = take(16 * na);
    L.pos_stage = take(24 * na);
    L.boff = take(4 * (na + 1));
    L.bother = take(4 * nbi);
    L.br0 = take(8 * nbi);
    L.bk = take(8 * nbi);
    // density outputs in the precision of the sums (float for FP32)
    const int64_t cb = cell_bytes(c);
    L.ulj = take(cb * ncell);
    L.ucfa = take(cb * ncell);
    L.ex = take(cb * ncell);
    L.ey = take(cb * ncell);
    L.ez = take(cb * ncell);
    L.bound = take(cb * ncell);
    L.u64cache = take(16 * ncell);
    L.bits = take(4 * c->g.nwords());
    L.stamp = take(4 * c->g.nwords());
    L.far_pts = take(32 * nfar);
    L.far_ulj = take(8 * nfar);
    L.far_ucfa = take(8 * nfar);
    L.far_ex = take(8 * nfar);
    L.far_ey = take(8 * nfar);
    L.far_ez = take(8 * nfar);
    L.far_part = take(8 * 4 * (size_t)POINT_SPLITS_MAX * nfar);
    L.red_d = take(8 * 2 * RED_BLOCKS);
    L.red_i = take(8 * 8 * RED_BLOCKS);
    L.scal_d = take(8 * 16);
    L.scal_i = take(8 * 16);
    L.sweep_flips = take(4 * SWEEP_BATCH);
    L.fsz = force_sizes(c->g, na, nfar);
    L.fpart = take(8 * (size_t)L.fsz.partial_doubles);
    L.fstage = take(L.fsz.staged_bytes);
    L.fcount = take(4 * (size_t)L.fsz.counts);
    L.fout = take(8 * 3 * na);
    const int64_t nslot = 3 * c->nang + 4 * c->ntor;
    L.s_ang = take(16 * c->nang);
    L.s_angp = take(16 * c->nang);
    L.s_tor = take(16 * c->ntor);
    L.s_torp = take(64 * c->ntor);
    L.s_slot = take(24 * nslot);
    L.s_incoff = take(4 * (na + 1));
    L.s_incslot = take(4 * nslot);
    L.s_nbp = take(32 * na);
    L.s_xoff = take(4 * (na + 1));
    L.s_xother = take(4 * c->x_other.size());
    L.s_nsplit = solute_splits(na);
    L.s_part = take(c->nonbonded ? 40 * (size_t)L.s_nsplit * na : 0);
    L.s_grad = take(24 * na);
    L.s_eatom = take(16 * na);
    L.s_red = take(8 * 4 * RED_BLOCKS);
    L.total = o;
    return L;
}

// scalar slots
enum { SD_VOL = 0, SD_FAR = 2, SD_BOND = 4, SD_SS = 8 };
enum { SI_GEOM = 0, SI_BAND = 8, SI_CNT = 10 };

vesis_status need(vesis_ctx* ctx, bool labels) {
    if (!ctx->has_params) return fail(ctx, VESIS_E_STATE, "parameters not set");
    if (!ctx->has_grid) return fail(ctx, VESIS_E_STATE, "grid not set");
    if (!ctx->has_atoms) return fail(ctx, VESIS_E_STATE, "atoms not set");
    if (!ctx->has_ws) return fail(ctx, VESIS_E_WORKSPACE, "workspace not set");
    if (labels && !ctx->has_labels) return fail(ctx, VESIS_E_STATE, "labels not initialised");
    return VESIS_OK;
}

vesis_status upload_inputs(vesis_ctx* ctx) {
    hipStream_t st = ctx->stream;
    if (!ctx->atoms_uploaded) {
        const int64_t n = ctx->na;
        std::vector<double> pos(4 * n), p64(4 * n);
        std::vector<float> p32(4 * n);
        for (int64_t i = 0; i < n; ++i) {
            pos[4 * i + 0] = ctx->xyz[3 * i + 0];
            pos[4 * i + 1] = ctx->xyz[3 * i + 1];
            pos[4 * i + 2] = ctx->xyz[3 * i + 2];
            pos[4 * i + 3] = 0.0;
            const double s2 = ctx->sigma[i] * ctx->sigma[i];
            const double e4 = 4.0 * ctx->prm.rho_w * ctx->eps[i];
            p64[4 * i + 0] = s2;
            p64[4 * i + 1] = e4;
            p64[4 * i + 2] = ctx->q[i];
            p64[4 * i + 3] = ctx->sigma[i];
            const double c6 = e4 * s2 * s2 * s2;
            p32[4 * i + 0] = (float)c6;
            p32[4 * i + 1] = (float)(c6 * s2 * s2 * s2);
            p32[4 * i + 2] = (float)ctx->q[i];
            p32[4 * i + 3] = (float)std::fabs(ctx->q[i]);
        }
        CK(hipMemcpyAsync(ctx->ws + ctx->lay.pos, pos.data(), 32 * n, hipMemcpyHostToDevice, st));
        CK(hipMemcpyAsync(ctx->ws + ctx->lay.prm64, p64.data(), 32 * n, hipMemcpyHostToDevice, st));
        CK(hipMemcpyAsync(ctx->ws + ctx->lay.prm32, p32.data(), 16 * n, hipMemcpyHostToDevice, st));
        CK(hipStreamSynchronize(st));
        ctx->atoms_uploaded = true;
    }
    if (!ctx->bonds_uploaded) {
        if (ctx->nb > 0) {
            const size_t nbi = ctx->b_other.size();
            CK(hipMemcpyAsync(ctx->ws + ctx->lay.boff, ctx->b_off.data(), 4 * (ctx->na + 1),
                              hipMemcpyHostToDevice, st));
            CK(hipMemcpyAsync(ctx->ws + ctx->lay.bother, ctx->b_other.data(), 4 * nbi,
                              hipMemcpyHostToDevice, st));
            CK(hipMemcpyAsync(ctx->ws + ctx->lay.br0, ctx->b_r0.data(), 8 * nbi,
                              hipMemcpyHostToDevice, st));
            CK(hipMemcpyAsync(ctx->ws + ctx->lay.bk, ctx->b_k.data(), 8 * nbi,
                              hipMemcpyHostToDevice, st));
            CK(hipStreamSynchronize(st));
        }
        ctx->bonds_uploaded = true;
    }
    if (!ctx->ss_uploaded) {
        const Layout& L = ctx->lay;
        const int64_t n = ctx->na;
        auto up = [&](size_t off, const void* src, size_t bytes) {
            return bytes ? hipMemcpyAsync(ctx->ws + off, src, bytes, hipMemcpyHostToDevice, st)
                         : hipSuccess;
        };
        std::vector<double> nbp(4 * n);
        for (int64_t i = 0; i < n; ++i) {
            const double sg = ctx->sig_ss.empty() ? ctx->sigma[i] : ctx->sig_ss[i];
            const double ep = ctx->eps_ss.empty() ? ctx->eps[i] : ctx->eps_ss[i];
            nbp[4 * i + 0] = 0.5 * sg;
            nbp[4 * i + 1] = std::sqrt(ep);
            nbp[4 * i + 2] = ctx->q[i];
            nbp[4 * i + 3] = 0.0;
        }
        if (ctx->inc_off.size() != (size_t)(n + 1)) ctx->inc_off.assign(n + 1, 0);
        if (ctx->x_off.size() != (size_t)(n + 1)) ctx->x_off.assign(n + 1, 0);
        CK(up(L.s_ang, ctx->ang.data(), 16 * ctx->nang));
        CK(up(L.s_angp, ctx->ang_prm.data(), 16 * ctx->nang));
        CK(up(L.s_tor, ctx->tor.data(), 16 * ctx->ntor));
        CK(up(L.s_torp, ctx->tor_prm.data(), 64 * ctx->ntor));
        CK(up(L.s_incoff, ctx->inc_off.data(), 4 * (n + 1)));
        CK(up(L.s_incslot, ctx->inc_slot.data(), 4 * ctx->inc_slot.size()));
        CK(up(L.s_nbp, nbp.data(), 32 * n));
        CK(up(L.s_xoff, ctx->x_off.data(), 4 * (n + 1)));
        CK(up(L.s_xother, ctx->x_other.data(), 4 * ctx->x_other.size()));
        CK(hipStreamSynchronize(st));
        ctx->ss_uploaded = true;
    }
    if (!ctx->far_uploaded) {
        CK(hipMemcpyAsync(ctx->ws + ctx->lay.far_pts, ctx->far_host.data(), 32 * ctx->nfar,
                          hipMemcpyHostToDevice, st));
        CK(hipStreamSynchronize(st));
        ctx->far_uploaded = true;
    }
    return VESIS_OK;
}

vesis_status density_tail(vesis_ctx* ctx);

CellFields cell_fields(vesis_ctx* ctx) {
    CellFields cf;
    cf.ulj = ctx->ws + ctx->lay.ulj;
    cf.ucfa = ctx->ws + ctx->lay.ucfa;
    cf.ex = ctx->ws + ctx->lay.ex;
    cf.ey = ctx->ws + ctx->lay.ey;
    cf.ez = ctx->ws + ctx->lay.ez;
    cf.bound = ctx->ws + ctx->lay.bound;
    cf.f32 = ctx->prm.precision == 64 ? 0 : 1;
    return cf;
}

// U, E and the error bound on every cell, the far field at every node, and
// the far-field sums; resets the FP64 near-tie cache.
vesis_status ensure_density(vesis_ctx* ctx) {
    vesis_status s = upload_inputs(ctx);
    if (s != VESIS_OK) return s;
    if (ctx->dens_valid) return VESIS_OK;
    hipStream_t st = ctx->stream;
    const Atoms a = dev_atoms(ctx);
    const Physics ph = dev_physics(ctx);
    const CellFields cf = cell_fields(ctx);
    {
        Timed t(ctx, K_DENSITY);
        CK(launch_density_grid(ctx->g, a, ph, ctx->prm.precision, cf, st));
    }
    return density_tail(ctx);
}

// After the grid density: reset the FP64 near-tie cache, evaluate the far
// field and its sums.
vesis_status density_tail(vesis_ctx* ctx) {
    hipStream_t st = ctx->stream;
    const Atoms a = dev_atoms(ctx);
    const Physics ph = dev_physics(ctx);
    {
        Timed t(ctx, K_OTHER);
        CK(launch_fill_f64(at<double>(ctx, ctx->lay.u64cache), 2 * ctx->g.ncell(), NAN, st));
    }
    {
        Timed t(ctx, K_FAR);
        CK(launch_density_points(at<double4>(ctx, ctx->lay.far_pts), ctx->nfar, a, ph,
                                 ctx->prm.precision, at<double>(ctx, ctx->lay.far_part),
                                 at<double>(ctx, ctx->lay.far_ulj),
                                 at<double>(ctx, ctx->lay.far_ucfa), at<double>(ctx, ctx->lay.far_ex),
                                 at<double>(ctx, ctx->lay.far_ey), at<double>(ctx, ctx->lay.far_ez),
                                 st));
        CK(launch_weighted_sum2(at<double4>(ctx, ctx->lay.far_pts), at<double>(ctx, ctx->lay.far_ulj),
                                at<double>(ctx, ctx->lay.far_ucfa), ctx->nfar,
                                at<double>(ctx, ctx->lay.red_d), RED_BLOCKS,
                                at<double>(ctx, ctx->lay.scal_d) + SD_FAR, st));
    }
    ctx->dens_valid = true;
    return VESIS_OK;
}

bool has_solute_terms(const vesis_ctx* c) { return c->nang > 0 || c->ntor > 0 || c->nonbonded; }

// Bending, torsion and non-bonded energies (scalar slots SD_SS..SD_SS+3)
// and their gradient (s_grad) at the current positions.
vesis_status ensure_solute(vesis_ctx* ctx) {
    if (!has_solute_terms(ctx) || ctx->ss_valid) return VESIS_OK;
    vesis_status s = upload_inputs(ctx);
    if (s != VESIS_OK) return s;
    const Layout& L = ctx->lay;
    Solute so;
    so.n = ctx->na;
    so.pos = at<double4>(ctx, L.pos);
    so.nang = ctx->nang;
    so.ang = at<int4>(ctx, L.s_ang);
    so.ang_prm = at<double2>(ctx, L.s_angp);
    so.ntor = ctx->ntor;
    so.tor = at<int4>(ctx, L.s_tor);
    so.tor_prm = at<double>(ctx, L.s_torp);
    so.slot = at<double>(ctx, L.s_slot);
    so.inc_off = at<int32_t>(ctx, L.s_incoff);
    so.inc_slot = at<int32_t>(ctx, L.s_incslot);
    so.nonbonded = ctx->nonbonded ? 1 : 0;
    so.nsplit = L.s_nsplit;
    so.nb_prm = at<double4>(ctx, L.s_nbp);
    so.x_off = at<int32_t>(ctx, L.s_xoff);
    so.x_other = at<int32_t>(ctx, L.s_xother);
    so.kcoul = ctx->prm.coulomb_k / ctx->prm.eps_w;
    so.pair_part = at<double>(ctx, L.s_part);
    so.grad = at<double>(ctx, L.s_grad);
    so.eatom = at<double>(ctx, L.s_eatom);
    {
        Timed t(ctx, K_SOLUTE);
        CK(launch_solute(so, at<double>(ctx, L.s_red), RED_BLOCKS,
                         at<double>(ctx, L.scal_d) + SD_SS, ctx->stream));
    }
    ctx->ss_valid = true;
    return VESIS_OK;
}

vesis_status compute_energy(vesis_ctx* ctx, vesis_energy_parts* out) {
    vesis_status s = ensure_density(ctx);
    if (s != VESIS_OK) return s;
    s = ensure_solute(ctx);
    if (s != VESIS_OK) return s;
    hipStream_t st = ctx->stream;
    const uint32_t* bits = at<uint32_t>(ctx, ctx->lay.bits);
    {
        Timed t(ctx, K_ENERGY);
        CK(launch_energy_volume(ctx->g, bits, cell_fields(ctx), at<double>(ctx, ctx->lay.red_d),
                                RED_BLOCKS, at<double>(ctx, ctx->lay.scal_d) + SD_VOL, st));
        CK(launch_geom_counts(ctx->g, bits, at<int64_t>(ctx, ctx->lay.red_i), RED_BLOCKS,
                              at<int64_t>(ctx, ctx->lay.scal_i) + SI_GEOM, st));
        if (ctx->nb > 0)
            CK(launch_bond_energy(dev_atoms(ctx), dev_bonds(ctx), at<double>(ctx, ctx->lay.red_d),
                                  RED_BLOCKS, at<double>(ctx, ctx->lay.scal_d) + SD_BOND, st));
    }
    double sd[16];
    int64_t si[16];
    CK(hipMemcpyAsync(sd, ctx->ws + ctx->lay.scal_d, sizeof(sd), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(si, ctx->ws + ctx->lay.scal_i, sizeof(si), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const double h3 = ctx->g.h * ctx->g.h * ctx->g.h;
    double geom = 0.0;
    for (int s2 = 1; s2 <= 8; ++s2) geom += ctx->sc.w[s2] * (double)si[SI_GEOM + s2 - 1];
    out->geom = ctx->sc.c * geom;
    out->vdw_in = h3 * sd[SD_VOL];
    out->elec_in = h3 * sd[SD_VOL + 1];
    out->vdw_far = sd[SD_FAR];
    out->elec_far = sd[SD_FAR + 1];
    out->bond = ctx->nb > 0 ? sd[SD_BOND] : 0.0;
    const bool ss = has_solute_terms(ctx);
    out->bend = ss ? sd[SD_SS] : 0.0;
    out->torsion = ss ? sd[SD_SS + 1] : 0.0;
    out->vdw_ss = ss ? sd[SD_SS + 2] : 0.0;
    out->elec_ss = ss ? sd[SD_SS + 3] : 0.0;
    out->total = out->geom + out->vdw_in + out->vdw_far + out->elec_in + out->elec_far + out->bond +
                 out->bend + out->torsion + out->vdw_ss + out->elec_ss;
    return VESIS_OK;
}

ForceScratch force_scratch(vesis_ctx* ctx) {
    const Layout& L = ctx->lay;
    return ForceScratch{at<double>(ctx, L.fpart), L.fsz.partial_doubles, ctx->ws + L.fstage,
                        L.fsz.staged_bytes, at<int>(ctx, L.fcount), L.fsz.counts};
}

vesis_status compute_forces(vesis_ctx* ctx, double* f_host) {
    vesis_status s = ensure_density(ctx);
    if (s != VESIS_OK) return s;
    s = ensure_solute(ctx);
    if (s != VESIS_OK) return s;
    hipStream_t st = ctx->stream;
    const Physics ph = dev_physics(ctx);
    if (!ctx->forces_valid) {
        Timed t(ctx, K_FORCE);
        CK(launch_forces(ctx->g, dev_atoms(ctx), ph, ctx->prm.precision,
                         at<uint32_t>(ctx, ctx->lay.bits), ctx->ws + ctx->lay.ex,
                         ctx->ws + ctx->lay.ey, ctx->ws + ctx->lay.ez,
                         at<double4>(ctx, ctx->lay.far_pts), at<double>(ctx, ctx->lay.far_ex),
                         at<double>(ctx, ctx->lay.far_ey), at<double>(ctx, ctx->lay.far_ez),
                         ctx->nfar, dev_bonds(ctx),
                         has_solute_terms(ctx) ? at<double>(ctx, ctx->lay.s_grad) : nullptr,
                         force_scratch(ctx), at<double>(ctx, ctx->lay.fout), st));
        ctx->forces_valid = true;
    }
    CK(hipMemcpyAsync(f_host, ctx->ws + ctx->lay.fout, 24 * ctx->na, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    return VESIS_OK;
}

vesis_status put_positions(vesis_ctx* ctx, const double* xyz) {
    std::memcpy(ctx->xyz.data(), xyz, sizeof(double) * 3 * ctx->na);
    std::vector<double> pos(4 * ctx->na);
    for (int64_t i = 0; i < ctx->na; ++i) {
        pos[4 * i] = xyz[3 * i];
        pos[4 * i + 1] = xyz[3 * i + 1];
        pos[4 * i + 2] = xyz[3 * i + 2];
        pos[4 * i + 3] = 0.0;
    }
    CK(hipMemcpyAsync(ctx->ws + ctx->lay.pos, pos.data(), 32 * ctx->na, hipMemcpyHostToDevice,
                      ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    ctx->dens_valid = false;
    ctx->ss_valid = false;
    ctx->forces_valid = false;
    return VESIS_OK;
}

bool inside_box(const vesis_ctx* c, const double* xyz, int64_t n) {
    const double ctr[3] = {c->g.cx, c->g.cy, c->g.cz};
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d)
            if (!(std::fabs(xyz[3 * i + d] - ctr[d]) < c->g.L)) return false;
    return true;
}

// Per-atom list of the gradient rows of the bending and torsion terms, in
// term order (angle rows first).
void rebuild_incidence(vesis_ctx* c) {
    const int64_t n = c->na;
    std::vector<int32_t> deg(n + 1, 0);
    for (int64_t t = 0; t < c->nang; ++t)
        for (int r = 0; r < 3; ++r) deg[c->ang[4 * t + r]]++;
    for (int64_t t = 0; t < c->ntor; ++t)
        for (int r = 0; r < 4; ++r) deg[c->tor[4 * t + r]]++;
    c->inc_off.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) c->inc_off[i + 1] = c->inc_off[i] + deg[i];
    std::vector<int32_t> fill(c->inc_off.begin(), c->inc_off.end() - 1);
    c->inc_slot.assign(c->inc_off[n], 0);
    for (int64_t t = 0; t < c->nang; ++t)
        for (int r = 0; r < 3; ++r) c->inc_slot[fill[c->ang[4 * t + r]]++] = (int32_t)(3 * t + r);
    for (int64_t t = 0; t < c->ntor; ++t)
        for (int r = 0; r < 4; ++r)
            c->inc_slot[fill[c->tor[4 * t + r]]++] = (int32_t)(3 * c->nang + 4 * t + r);
}

// The workspace stays usable while every solute-solute array fits the
// layout it was planned for.
void check_solute_layout(vesis_ctx* c) {
    if (c->nang > c->lay_nang || c->ntor > c->lay_ntor ||
        (int64_t)c->x_other.size() > c->lay_nxo || (c->nonbonded && !c->lay_nonbonded))
        c->has_ws = false;
    c->ss_uploaded = false;
    c->ss_valid = false;
    c->forces_valid = false;
}

bool distinct(const int32_t* id, int m) {
    for (int a = 0; a < m; ++a)
        for (int b = a + 1; b < m; ++b)
            if (id[a] == id[b]) return false;
    return true;
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

vesis_status vesis_create(int32_t device, void* stream, vesis_ctx** out) {
    if (!out) return VESIS_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return VESIS_E_NO_DEVICE;
    if (device < 0 || device >= count) return VESIS_E_NO_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return VESIS_E_NO_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return VESIS_E_NO_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return VESIS_E_DEVICE;
    vesis_ctx* c = new vesis_ctx();
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    *out = c;
    return VESIS_OK;
}

void vesis_destroy(vesis_ctx* ctx) {
    if (!ctx) return;
    if (!ctx->pending.empty()) drain_events(ctx);
    if (ctx->bexec) (void)hipGraphExecDestroy(ctx->bexec);
    if (ctx->bgraph) (void)hipGraphDestroy(ctx->bgraph);
    for (hipEvent_t e : ctx->bev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    if (ctx->hstage) (void)hipHostFree(ctx->hstage);
    delete ctx;
}

const char* vesis_last_error(const vesis_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

vesis_status vesis_set_params(vesis_ctx* ctx, const vesis_params* p) {
    if (!ctx || !p) return fail(ctx, VESIS_E_ARG, "null argument");
    const double v[7] = {p->rho_w, p->gamma0, p->eps_m, p->eps_w, p->coulomb_k, p->rho_s, p->r2_min};
    if (!finite_all(v, 7)) return fail(ctx, VESIS_E_NONFINITE, "non-finite parameter");
    if (p->rho_w < 0 || p->gamma0 < 0 || p->eps_m <= 0 || p->eps_w <= 0 || p->r2_min <= 0)
        return fail(ctx, VESIS_E_ARG, "rho_w, gamma0 >= 0, eps_m, eps_w, r2_min > 0 required");
    if (!(p->rho_s > 1.0 && p->rho_s <= 3.0))
        return fail(ctx, VESIS_E_ARG, "rho_s = delta/h must lie in (1, 3]");
    if (p->far_nf < 1 || p->far_nf > 128 || p->far_ntau < 1 || p->far_ntau > 128)
        return fail(ctx, VESIS_E_ARG, "far_nf, far_ntau must lie in [1, 128]");
    if (p->precision != 32 && p->precision != 64)
        return fail(ctx, VESIS_E_ARG, "precision must be 32 or 64");
    const bool far_changed = !ctx->has_params || p->far_nf != ctx->prm.far_nf ||
                             p->far_ntau != ctx->prm.far_ntau;
    const bool rho_changed = !ctx->has_params || p->rho_w != ctx->prm.rho_w;
    ctx->prm = *p;
    ctx->has_params = true;
    // the stored densities change size with the precision
    if (ctx->has_ws && ctx->lay_cell_bytes != cell_bytes(ctx)) ctx->has_ws = false;
    ctx->dens_valid = false;
    ctx->ss_valid = false;
    ctx->forces_valid = false;
    if (rho_changed) ctx->atoms_uploaded = false;
    if (ctx->has_grid) {
        compute_stencil(ctx);
        if (far_changed) {
            compute_far_nodes(ctx);
            ctx->has_ws = ctx->has_ws && ctx->lay_nfar == ctx->nfar;
        }
    }
    return VESIS_OK;
}

vesis_status vesis_set_grid(vesis_ctx* ctx, int32_t n, const double center[3], double h) {
    if (!ctx || !center) return fail(ctx, VESIS_E_ARG, "null argument");
    if (!ctx->has_params) return fail(ctx, VESIS_E_STATE, "parameters not set");
    if (n < 4 || n > 1024) return fail(ctx, VESIS_E_ARG, "n must lie in [4, 1024]");
    const double v[4] = {center[0], center[1], center[2], h};
    if (!finite_all(v, 4)) return fail(ctx, VESIS_E_NONFINITE, "non-finite grid");
    if (!(h > 0)) return fail(ctx, VESIS_E_ARG, "h must be positive");
    Grid& g = ctx->g;
    g.n = n;
    g.nwin = (n + 31) / 32;
    g.W = g.nwin + 2;
    g.rdim = n + 4;
    g.h = h;
    g.L = 0.5 * (double)n * h;
    g.cx = center[0];
    g.cy = center[1];
    g.cz = center[2];
    g.x0 = (g.cx - g.L) + 0.5 * h;
    g.y0 = (g.cy - g.L) + 0.5 * h;
    g.z0 = (g.cz - g.L) + 0.5 * h;
    ctx->has_grid = true;
    compute_stencil(ctx);
    compute_far_nodes(ctx);
    ctx->has_ws = false;
    ctx->has_labels = false;
    ctx->dens_valid = false;
    ctx->ss_valid = false;
    ctx->forces_valid = false;
    if (ctx->has_atoms && !inside_box(ctx, ctx->xyz.data(), ctx->na)) {
        ctx->has_atoms = false;
        return fail(ctx, VESIS_E_OUT_OF_BOX, "an atom lies outside the new box; set atoms again");
    }
    return VESIS_OK;
}

vesis_status vesis_set_atoms(vesis_ctx* ctx, int64_t n, const double* xyz, const double* q,
                             const double* sigma, const double* eps, const uint8_t* movable) {
    if (!ctx || !xyz || !q || !sigma || !eps) return fail(ctx, VESIS_E_ARG, "null argument");
    if (!ctx->has_grid) return fail(ctx, VESIS_E_STATE, "grid not set");
    if (n < 1 || n > (1LL << 26)) return fail(ctx, VESIS_E_ARG, "atom count out of range");
    if (!finite_all(xyz, 3 * n) || !finite_all(q, n) || !finite_all(sigma, n) || !finite_all(eps, n))
        return fail(ctx, VESIS_E_NONFINITE, "non-finite atom data");
    for (int64_t i = 0; i < n; ++i)
        if (!(sigma[i] > 0) || eps[i] < 0) return fail(ctx, VESIS_E_ARG, "sigma > 0, eps >= 0 required");
    if (!inside_box(ctx, xyz, n)) return fail(ctx, VESIS_E_OUT_OF_BOX, "an atom lies outside the box");
    if (n != ctx->na) {
        ctx->has_ws = false;
        ctx->nb = 0;
        ctx->b_off.assign(n + 1, 0);
        ctx->b_other.clear();
        ctx->b_r0.clear();
        ctx->b_k.clear();
        ctx->nang = ctx->ntor = 0;
        ctx->ang.clear();
        ctx->ang_prm.clear();
        ctx->tor.clear();
        ctx->tor_prm.clear();
        ctx->inc_off.assign(n + 1, 0);
        ctx->inc_slot.clear();
        ctx->nonbonded = false;
        ctx->sig_ss.clear();
        ctx->eps_ss.clear();
        ctx->x_off.assign(n + 1, 0);
        ctx->x_other.clear();
    }
    ctx->na = n;
    ctx->xyz.assign(xyz, xyz + 3 * n);
    ctx->q.assign(q, q + n);
    ctx->sigma.assign(sigma, sigma + n);
    ctx->eps.assign(eps, eps + n);
    ctx->movable.assign(n, 1);
    if (movable)
        for (int64_t i = 0; i < n; ++i) ctx->movable[i] = movable[i] ? 1 : 0;
    if (ctx->b_off.size() != (size_t)(n + 1)) ctx->b_off.assign(n + 1, 0);
    ctx->has_atoms = true;
    ctx->atoms_uploaded = false;
    ctx->bonds_uploaded = false;
    ctx->ss_uploaded = false;
    ctx->dens_valid = false;
    ctx->ss_valid = false;
    ctx->forces_valid = false;
    return VESIS_OK;
}

vesis_status vesis_set_positions(vesis_ctx* ctx, const double* xyz, int32_t on_device) {
    if (!ctx || !xyz) return fail(ctx, VESIS_E_ARG, "null argument");
    if (!ctx->has_atoms) return fail(ctx, VESIS_E_STATE, "atoms not set");
    if (on_device) {
        if (!ctx->has_ws) return fail(ctx, VESIS_E_WORKSPACE, "workspace not set");
        vesis_status s = upload_inputs(ctx);
        if (s != VESIS_OK) return s;
        hipStream_t st = ctx->stream;
        CK(hipMemcpyAsync(ctx->ws + ctx->lay.pos_stage, xyz, 24 * ctx->na, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(pack_positions, dim3((unsigned)((ctx->na + 255) / 256)), dim3(256), 0, st,
                           at<double>(ctx, ctx->lay.pos_stage), ctx->na, at<double4>(ctx, ctx->lay.pos));
        CK(hipGetLastError());
        CK(hipMemcpyAsync(ctx->xyz.data(), ctx->ws + ctx->lay.pos_stage, 24 * ctx->na,
                          hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        ctx->dens_valid = false;
        ctx->ss_valid = false;
        ctx->forces_valid = false;
        return VESIS_OK;
    }
    if (!finite_all(xyz, 3 * ctx->na)) return fail(ctx, VESIS_E_NONFINITE, "non-finite positions");
    if (!inside_box(ctx, xyz, ctx->na)) return fail(ctx, VESIS_E_OUT_OF_BOX, "an atom lies outside the box");
    if (!ctx->has_ws || !ctx->atoms_uploaded) {
        ctx->xyz.assign(xyz, xyz + 3 * ctx->na);
        ctx->atoms_uploaded = false;
        ctx->dens_valid = false;
        ctx->ss_valid = false;
        ctx->forces_valid = false;
        return VESIS_OK;
    }
    return put_positions(ctx, xyz);
}

vesis_status vesis_get_positions(vesis_ctx* ctx, double* xyz) {
    if (!ctx || !xyz) return fail(ctx, VESIS_E_ARG, "null argument");
    if (!ctx->has_atoms) return fail(ctx, VESIS_E_STATE, "atoms not set");
    std::memcpy(xyz, ctx->xyz.data(), sizeof(double) * 3 * ctx->na);
    return VESIS_OK;
}

vesis_status vesis_set_bonds(vesis_ctx* ctx, int64_t nb, const int32_t* ij, const double* r0,
                             const double* k) {
    if (!ctx) return VESIS_E_ARG;
    if (!ctx->has_atoms) return fail(ctx, VESIS_E_STATE, "atoms not set");
    if (nb < 0 || (nb > 0 && (!ij || !r0 || !k))) return fail(ctx, VESIS_E_ARG, "bad bond arrays");
    if (nb > 0 && (!finite_all(r0, nb) || !finite_all(k, nb)))
        return fail(ctx, VESIS_E_NONFINITE, "non-finite bond data");
    for (int64_t b = 0; b < nb; ++b) {
        const int32_t i = ij[2 * b], j = ij[2 * b + 1];
        if (i < 0 || j < 0 || i >= ctx->na || j >= ctx->na || i == j)
            return fail(ctx, VESIS_E_ARG, "bond atom index out of range");
    }
    const int64_t n = ctx->na;
    std::vector<int32_t> deg(n + 1, 0);
    for (int64_t b = 0; b < nb; ++b) {
        deg[ij[2 * b]]++;
        deg[ij[2 * b + 1]]++;
    }
    std::vector<int32_t> off(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + deg[i];
    std::vector<int32_t> fill(off.begin(), off.end() - 1), other(2 * nb);
    std::vector<double> rr(2 * nb), kk(2 * nb);
    for (int64_t b = 0; b < nb; ++b) {
        const int32_t i = ij[2 * b], j = ij[2 * b + 1];
        other[fill[i]] = j;
        rr[fill[i]] = r0[b];
        kk[fill[i]++] = k[b];
        other[fill[j]] = i;
        rr[fill[j]] = r0[b];
        kk[fill[j]++] = k[b];
    }
    if (nb > ctx->lay_nb) ctx->has_ws = false;
    ctx->nb = nb;
    ctx->b_off = off;
    ctx->b_other = other;
    ctx->b_r0 = rr;
    ctx->b_k = kk;
    ctx->bonds_uploaded = false;
    ctx->forces_valid = false;
    return VESIS_OK;
}

vesis_status vesis_set_angles(vesis_ctx* ctx, int64_t nang, const int32_t* ijk,
                              const double* theta0, const double* k) {
    if (!ctx) return VESIS_E_ARG;
    if (!ctx->has_atoms) return fail(ctx, VESIS_E_STATE, "atoms not set");
    if (nang < 0 || nang > (1LL << 28) || (nang > 0 && (!ijk || !theta0 || !k)))
        return fail(ctx, VESIS_E_ARG, "bad angle arrays");
    if (nang > 0 && (!finite_all(theta0, nang) || !finite_all(k, nang)))
        return fail(ctx, VESIS_E_NONFINITE, "non-finite angle data");
    for (int64_t t = 0; t < nang; ++t) {
        for (int r = 0; r < 3; ++r)
            if (ijk[3 * t + r] < 0 || ijk[3 * t + r] >= ctx->na)
                return fail(ctx, VESIS_E_ARG, "angle atom index out of range");
        if (!distinct(ijk + 3 * t, 3)) return fail(ctx, VESIS_E_ARG, "angle atoms must differ");
        if (theta0[t] < 0 || theta0[t] > PI)
            return fail(ctx, VESIS_E_ARG, "theta0 must lie in [0, pi]");
    }
    ctx->nang = nang;
    ctx->ang.assign(4 * nang, 0);
    ctx->ang_prm.assign(2 * nang, 0.0);
    for (int64_t t = 0; t < nang; ++t) {
        for (int r = 0; r < 3; ++r) ctx->ang[4 * t + r] = ijk[3 * t + r];
        ctx->ang_prm[2 * t] = theta0[t];
        ctx->ang_prm[2 * t + 1] = k[t];
    }
    rebuild_incidence(ctx);
    check_solute_layout(ctx);
    return VESIS_OK;
}

vesis_status vesis_set_torsions(vesis_ctx* ctx, int64_t ntor, const int32_t* ijkl,
                                const double* c, const double* psi) {
    if (!ctx) return VESIS_E_ARG;
    if (!ctx->has_atoms) return fail(ctx, VESIS_E_STATE, "atoms not set");
    if (ntor < 0 || ntor > (1LL << 28) || (ntor > 0 && (!ijkl || !c || !psi)))
        return fail(ctx, VESIS_E_ARG, "bad torsion arrays");
    if (ntor > 0 && (!finite_all(c, 7 * ntor) || !finite_all(psi, 7 * ntor)))
        return fail(ctx, VESIS_E_NONFINITE, "non-finite torsion data");
    std::vector<double> prm(8 * ntor, 0.0);
    for (int64_t t = 0; t < ntor; ++t) {
        for (int r = 0; r < 4; ++r)
            if (ijkl[4 * t + r] < 0 || ijkl[4 * t + r] >= ctx->na)
                return fail(ctx, VESIS_E_ARG, "torsion atom index out of range");
        if (!distinct(ijkl + 4 * t, 4)) return fail(ctx, VESIS_E_ARG, "torsion atoms must differ");
        // C_n [1 + cos(n tau - psi_n)] = C_n + C_n cos(psi_n) T_n(cos tau) when sin psi_n = 0
        double a0 = 0.0;
        for (int m = 0; m <= 6; ++m) {
            const double ps = psi[7 * t + m];
            if (std::fabs(std::sin(ps)) > 1e-9)
                return fail(ctx, VESIS_E_ARG, "every psi_n must be 0 or pi");
            const double cp = std::cos(ps) > 0 ? 1.0 : -1.0;
            const double cn = c[7 * t + m];
            a0 += cn;
            if (m == 0)
                a0 += cn * cp;
            else
                prm[8 * t + m] = cn * cp;
        }
        prm[8 * t] = a0;
    }
    ctx->ntor = ntor;
    ctx->tor.assign(ijkl, ijkl + 4 * ntor);
    ctx->tor_prm = prm;
    rebuild_incidence(ctx);
    check_solute_layout(ctx);
    return VESIS_OK;
}

vesis_status vesis_set_nonbonded(vesis_ctx* ctx, int32_t enable, const double* sigma_ss,
                                 const double* eps_ss, int64_t nexcl, const int32_t* excl) {
    if (!ctx) return VESIS_E_ARG;
    if (!ctx->has_atoms) return fail(ctx, VESIS_E_STATE, "atoms not set");
    const int64_t n = ctx->na;
    if (nexcl < 0 || nexcl > (1LL << 28) || (nexcl > 0 && !excl))
        return fail(ctx, VESIS_E_ARG, "bad exclusion arrays");
    if ((sigma_ss && !finite_all(sigma_ss, n)) || (eps_ss && !finite_all(eps_ss, n)))
        return fail(ctx, VESIS_E_NONFINITE, "non-finite solute-solute LJ parameters");
    for (int64_t i = 0; i < n; ++i)
        if ((sigma_ss && !(sigma_ss[i] > 0)) || (eps_ss && eps_ss[i] < 0))
            return fail(ctx, VESIS_E_ARG, "sigma_ss > 0, eps_ss >= 0 required");
    for (int64_t e = 0; e < nexcl; ++e) {
        const int32_t i = excl[2 * e], j = excl[2 * e + 1];
        if (i < 0 || j < 0 || i >= n || j >= n || i == j)
            return fail(ctx, VESIS_E_ARG, "exclusion atom index out of range");
    }
    std::vector<std::vector<int32_t>> part(n);
    for (int64_t e = 0; e < nexcl; ++e) {
        part[excl[2 * e]].push_back(excl[2 * e + 1]);
        part[excl[2 * e + 1]].push_back(excl[2 * e]);
    }
    ctx->x_off.assign(n + 1, 0);
    ctx->x_other.clear();
    for (int64_t i = 0; i < n; ++i) {
        std::sort(part[i].begin(), part[i].end());
        part[i].erase(std::unique(part[i].begin(), part[i].end()), part[i].end());
        ctx->x_other.insert(ctx->x_other.end(), part[i].begin(), part[i].end());
        ctx->x_off[i + 1] = (int32_t)ctx->x_other.size();
    }
    ctx->nonbonded = enable != 0;
    if (sigma_ss) ctx->sig_ss.assign(sigma_ss, sigma_ss + n); else ctx->sig_ss.clear();
    if (eps_ss) ctx->eps_ss.assign(eps_ss, eps_ss + n); else ctx->eps_ss.clear();
    check_solute_layout(ctx);
    return VESIS_OK;
}

vesis_status vesis_workspace_size(vesis_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return fail(ctx, VESIS_E_ARG, "null argument");
    if (!ctx->has_params || !ctx->has_grid || !ctx->has_atoms)
        return fail(ctx, VESIS_E_STATE, "params, grid and atoms must be set first");
    *bytes = plan(ctx).total;
    return VESIS_OK;
}

vesis_status vesis_set_workspace(vesis_ctx* ctx, void* device_ptr, size_t bytes) {
    if (!ctx || !device_ptr) return fail(ctx, VESIS_E_ARG, "null argument");
    if (!ctx->has_params || !ctx->has_grid || !ctx->has_atoms)
        return fail(ctx, VESIS_E_STATE, "params, grid and atoms must be set first");
    if (reinterpret_cast<uintptr_t>(device_ptr) & 255)
        return fail(ctx, VESIS_E_ARG, "workspace must be 256-byte aligned");
    const Layout L = plan(ctx);
    if (bytes < L.total)
        return fail(ctx, VESIS_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total) +
                                                " bytes, got " + std::to_string(bytes));
    const bool same = ctx->has_ws && ctx->ws == device_ptr && ctx->lay_n == ctx->g.n;
    ctx->ws = static_cast<char*>(device_ptr);
    ctx->ws_bytes = bytes;
    ctx->lay = L;
    ctx->lay_na = ctx->na;
    ctx->lay_nb = ctx->nb;
    ctx->lay_nang = ctx->nang;
    ctx->lay_ntor = ctx->ntor;
    ctx->lay_nxo = (int64_t)ctx->x_other.size();
    ctx->lay_nonbonded = ctx->nonbonded;
    ctx->lay_nfar = ctx->nfar;
    ctx->lay_cell_bytes = cell_bytes(ctx);
    ctx->lay_n = ctx->g.n;
    ctx->has_ws = true;
    ctx->atoms_uploaded = false;
    ctx->bonds_uploaded = false;
    ctx->far_uploaded = false;
    ctx->ss_uploaded = false;
    ctx->dens_valid = false;
    ctx->ss_valid = false;
    ctx->forces_valid = false;
    if (!same) ctx->has_labels = false;
    return VESIS_OK;
}

vesis_status vesis_init_labels(vesis_ctx* ctx, int32_t mode, double param, const int8_t* user) {
    if (!ctx) return VESIS_E_ARG;
    vesis_status s = need(ctx, false);
    if (s != VESIS_OK) return s;
    if (mode < 0 || mode > 2) return fail(ctx, VESIS_E_ARG, "mode must be 0, 1 or 2");
    if (mode != 2 && (!std::isfinite(param) || !(param > 0)))
        return fail(ctx, VESIS_E_ARG, "param must be positive and finite");
    if (mode == 2 && !user) return fail(ctx, VESIS_E_ARG, "user labels missing");
    s = upload_inputs(ctx);
    if (s != VESIS_OK) return s;
    hipStream_t st = ctx->stream;
    const Grid& g = ctx->g;
    uint32_t* bits = at<uint32_t>(ctx, ctx->lay.bits);
    if (mode == 2) {
        const int64_t nc = g.ncell();
        for (int64_t c = 0; c < nc; ++c)
            if (user[c] != 1 && user[c] != -1) return fail(ctx, VESIS_E_ARG, "labels must be -1 or +1");
        std::vector<uint32_t> host(g.nwords(), 0xffffffffu);
        for (int z = 0; z < g.n; ++z)
            for (int y = 0; y < g.n; ++y)
                for (int x = 0; x < g.n; ++x)
                    if (user[x + (int64_t)g.n * (y + (int64_t)g.n * z)] == -1)
                        host[g.row(y, z) + 1 + (x >> 5)] &= ~(1u << (x & 31));
        CK(hipMemcpyAsync(bits, host.data(), 4 * host.size(), hipMemcpyHostToDevice, st));
        CK(hipStreamSynchronize(st));
    } else {
        Timed t(ctx, K_INIT);
        CK(launch_fill_u32(bits, g.nwords(), 0xffffffffu, st));
        if (mode == 0)
            CK(launch_init_loose(g, param, bits, st));
        else {
            double smax = 0.0;
            for (double sg : ctx->sigma) smax = std::max(smax, sg);
            CK(launch_init_tight(g, dev_atoms(ctx), param, param * smax, bits, st));
        }
    }
    ctx->has_labels = true;
    ctx->forces_valid = false;
    return VESIS_OK;
}

vesis_status vesis_init_labels_logits(vesis_ctx* ctx, const float* logits) {
    if (!ctx) return VESIS_E_ARG;
    vesis_status s = need(ctx, false);
    if (s != VESIS_OK) return s;
    if (!logits) return fail(ctx, VESIS_E_ARG, "logits missing");
    s = upload_inputs(ctx);
    if (s != VESIS_OK) return s;
    hipStream_t st = ctx->stream;
    uint32_t* bits = at<uint32_t>(ctx, ctx->lay.bits);
    {
        Timed t(ctx, K_INIT);
        CK(launch_fill_u32(bits, ctx->g.nwords(), 0xffffffffu, st));
        CK(launch_labels_from_logits(ctx->g, logits, bits, st));
    }
    ctx->has_labels = true;
    ctx->forces_valid = false;
    return VESIS_OK;
}

vesis_status vesis_minimize_interface(vesis_ctx* ctx, int32_t max_sweeps, vesis_min_stats* out) {
    if (!ctx) return VESIS_E_ARG;
    vesis_status s = need(ctx, true);
    if (s != VESIS_OK) return s;
    if (max_sweeps < 1) return fail(ctx, VESIS_E_ARG, "max_sweeps must be >= 1");
    s = ensure_density(ctx);
    if (s != VESIS_OK) return s;
    hipStream_t st = ctx->stream;
    const Atoms a = dev_atoms(ctx);
    const Physics ph = dev_physics(ctx);
    const CellFields cf = cell_fields(ctx);
    const int ncol = ctx->sc.p * ctx->sc.p * ctx->sc.p;
    uint32_t* bits = at<uint32_t>(ctx, ctx->lay.bits);
    int* flips = at<int>(ctx, ctx->lay.sweep_flips);
    int64_t* counters = at<int64_t>(ctx, ctx->lay.scal_i) + SI_CNT;
    CK(launch_fill_i64(counters, 2, 0, st));
    int* stamp = at<int>(ctx, ctx->lay.stamp);
    CK(launch_fill_u32(reinterpret_cast<uint32_t*>(stamp), ctx->g.nwords(),
                       (uint32_t)(-(1 << 30)), st));
    int64_t total_flips = 0;
    int sweeps = 0;
    bool converged = false;
    while (sweeps < max_sweeps && !converged) {
        const int nb = std::min(SWEEP_BATCH, max_sweeps - sweeps);
        CK(launch_fill_u32(reinterpret_cast<uint32_t*>(flips), SWEEP_BATCH, 0u, st));
        {
            Timed t(ctx, K_FLIP);
            for (int sw = 0; sw < nb; ++sw) {
                if (ctx->sc.p == 3) {
                    // colour period 3: the colours sharing their rows go three
                    // to a launch
                    for (int grp = 0; grp < 9; ++grp)
                        CK(launch_flip_group3(ctx->g, ctx->sc, a, ph, grp, sw,
                                              (sweeps + sw) * ncol + 3 * grp, bits, stamp, cf,
                                              at<double>(ctx, ctx->lay.u64cache), flips,
                                              counters, st));
                } else {
                    for (int c = 0; c < ncol; ++c)
                        CK(launch_flip_pass(ctx->g, ctx->sc, a, ph, c, sw,
                                            (sweeps + sw) * ncol + c, bits, stamp, cf,
                                            at<double>(ctx, ctx->lay.u64cache), flips, counters,
                                            st));
                }
            }
        }
        int hf[SWEEP_BATCH];
        CK(hipMemcpyAsync(hf, flips, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        for (int sw = 0; sw < nb; ++sw) {
            total_flips += hf[sw];
            ++sweeps;
            if (hf[sw] == 0) {
                converged = true;
                break;
            }
        }
    }
    if (total_flips > 0) ctx->forces_valid = false;
    if (out) {
        int64_t cnt[2] = {0, 0}, band = 0;
        CK(launch_band_count(ctx->g, bits, at<int64_t>(ctx, ctx->lay.red_i), RED_BLOCKS,
                             at<int64_t>(ctx, ctx->lay.scal_i) + SI_BAND, st));
        CK(hipMemcpyAsync(cnt, counters, sizeof(cnt), hipMemcpyDeviceToHost, st));
        CK(hipMemcpyAsync(&band, ctx->ws + ctx->lay.scal_i + 8 * SI_BAND, sizeof(band),
                          hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        out->sweeps = sweeps;
        out->converged = converged ? 1 : 0;
        out->flips = total_flips;
        out->band_cells = band;
        out->near_ties = cnt[0];
        out->fp64_recomputes = cnt[1];
    }
    return converged ? VESIS_OK : VESIS_NOT_CONVERGED;
}

vesis_status vesis_energy(vesis_ctx* ctx, vesis_energy_parts* out) {
    if (!ctx || !out) return fail(ctx, VESIS_E_ARG, "null argument");
    vesis_status s = need(ctx, true);
    if (s != VESIS_OK) return s;
    return compute_energy(ctx, out);
}

vesis_status vesis_forces(vesis_ctx* ctx, double* f_out) {
    if (!ctx || !f_out) return fail(ctx, VESIS_E_ARG, "null argument");
    vesis_status s = need(ctx, true);
    if (s != VESIS_OK) return s;
    return compute_forces(ctx, f_out);
}

vesis_status vesis_atom_step(vesis_ctx* ctx, vesis_mobility* st, vesis_step_info* info) {
    if (!ctx || !st || !info) return fail(ctx, VESIS_E_ARG, "null argument");
    vesis_status s = need(ctx, true);
    if (s != VESIS_OK) return s;
    const double sv[6] = {st->M, st->alpha, st->dt, st->dG_frac, st->M_min, 0.0};
    if (!finite_all(sv, 6) || !(st->M > 0) || !(st->alpha > 0 && st->alpha < 1) || !(st->dt > 0) ||
        st->dG_frac < 0 || st->N_cnt_max < 0 || st->max_retries < 0)
        return fail(ctx, VESIS_E_ARG, "bad mobility state");
    const int64_t n = ctx->na;
    vesis_energy_parts e{};
    s = compute_energy(ctx, &e);
    if (s != VESIS_OK) return s;
    const double G_old = e.total;
    std::vector<double> f(3 * n), R(ctx->xyz), trial(3 * n);
    s = compute_forces(ctx, f.data());
    if (s != VESIS_OK) return s;
    double gmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!ctx->movable[i]) continue;
        for (int d = 0; d < 3; ++d) gmax = std::max(gmax, std::fabs(f[3 * i + d]));
    }
    info->accepted = 0;
    info->retries = 0;
    info->G_old = G_old;
    info->G_new = G_old;
    info->max_grad = gmax;
    info->omega = 0.0;
    if (gmax == 0.0) {
        st->G_old = G_old;
        return fail(ctx, VESIS_NOT_CONVERGED, "zero gradient");
    }
    const double omega = 1.0 / gmax;
    info->omega = omega;
    for (;;) {
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) {
                const double gr = -f[3 * i + d];
                trial[3 * i + d] = ctx->movable[i] ? R[3 * i + d] - st->dt * omega * st->M * gr
                                                   : R[3 * i + d];
            }
        s = put_positions(ctx, trial.data());
        if (s != VESIS_OK) return s;
        s = compute_energy(ctx, &e);
        if (s != VESIS_OK) return s;
        const double dG = e.total - G_old;
        const double dGs = st->dG_frac * std::fabs(G_old);
        const bool reject = (dG > dGs) || (st->N_cnt >= st->N_cnt_max && dG > 0.0 && dG <= dGs);
        info->G_new = e.total;
        if (!reject) {
            st->N_cnt += 1;
            st->k += 1;
            st->G_old = e.total;
            info->accepted = 1;
            return VESIS_OK;
        }
        st->M *= st->alpha;
        st->N_cnt = 0;
        info->retries += 1;
        if (st->M < st->M_min || info->retries > st->max_retries) {
            st->G_old = G_old;
            s = put_positions(ctx, R.data());
            if (s != VESIS_OK) return s;
            return fail(ctx, VESIS_NOT_CONVERGED, "mobility fell below M_min or retries ran out");
        }
    }
}

vesis_status vesis_relax(vesis_ctx* ctx, const vesis_relax_opts* o, vesis_mobility* st,
                         vesis_relax_report* rep) {
    if (!ctx || !o || !st || !rep) return fail(ctx, VESIS_E_ARG, "null argument");
    vesis_status s = need(ctx, true);
    if (s != VESIS_OK) return s;
    if (o->max_iters < 1 || o->persist < 1 || o->max_sweeps < 1 || !(o->tol_grad >= 0) ||
        !(o->tol_energy >= 0))
        return fail(ctx, VESIS_E_ARG, "bad relax options");
    std::memset(rep, 0, sizeof(*rep));
    const int64_t n = ctx->na;
    std::vector<double> f(3 * n);
    double G_prev = NAN;
    int calm = 0, reason = 3;
    for (int k = 0; k < o->max_iters; ++k) {
        rep->iters = k + 1;
        // Step 2: interface at fixed atoms
        vesis_min_stats ms{};
        s = vesis_minimize_interface(ctx, o->max_sweeps, &ms);
        if (s < 0) return s;
        rep->sweeps += ms.sweeps;
        // Steps 3.1-3.2: gradient test
        s = vesis_forces(ctx, f.data());
        if (s < 0) return s;
        double gmax = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!ctx->movable[i]) continue;
            for (int d = 0; d < 3; ++d) gmax = std::max(gmax, std::fabs(f[3 * i + d]));
        }
        rep->max_grad = gmax;
        if (gmax < o->tol_grad) {
            vesis_energy_parts e{};
            s = compute_energy(ctx, &e);
            if (s < 0) return s;
            rep->G_final = e.total;
            reason = 1;
            break;
        }
        // Steps 3.3-3.4: one accepted step
        vesis_step_info info{};
        s = vesis_atom_step(ctx, st, &info);
        if (s < 0) return s;
        rep->retries += info.retries;
        if (s == VESIS_NOT_CONVERGED) {
            rep->G_final = info.G_old;
            reason = 4;
            break;
        }
        // Steps 4-5: change of G between iterations
        const double G = info.G_new;
        rep->G_final = G;
        if (!std::isnan(G_prev)) {
            rep->dG_abs = std::fabs(G - G_prev);
            rep->dG_rel = rep->dG_abs / std::fabs(G_prev);
            calm = (rep->dG_rel < o->tol_energy || rep->dG_abs < o->tol_energy) ? calm + 1 : 0;
            if (calm >= o->persist) {
                reason = 2;
                break;
            }
        }
        G_prev = G;
    }
    rep->stop_reason = reason;
    ctx->err.clear();
    return reason == 3 ? VESIS_NOT_CONVERGED : VESIS_OK;
}

// ------------------------------------------------------------------ batches

namespace {

constexpr int BATCH_MAX = BATCH_MOLS;
constexpr int NXCD_BATCH = 8;  // dies (XCDs) of the chip, each with its own L2

struct BatchLayout {
    size_t desc, dmap, fmap, flips, done, pass, far, farmap, total;
};

BatchLayout batch_layout(int m, int64_t dens_blocks, int64_t flip_blocks, int64_t far_blocks) {
    BatchLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += align256(bytes ? bytes : 1);
        return r;
    };
    L.desc = take(sizeof(MolDesc) * (size_t)m);
    L.dmap = take(4 * (size_t)dens_blocks);
    L.fmap = take(4 * (size_t)flip_blocks);
    L.flips = take(4 * (size_t)m * SWEEP_BATCH);
    L.done = take(4 * (size_t)m);
    L.pass = take(4);
    L.far = take(sizeof(FarDesc) * (size_t)m);
    L.farmap = take(4 * (size_t)far_blocks);
    L.total = o;
    return L;
}

// Host staging of a batch call (in the first context's pinned buffer):
// density descriptors and brick map, colour-pass descriptors and block map,
// three int64 read-backs per molecule, and two slots of per-sweep flip
// counts (one per group of sweeps in flight).  The regions are disjoint, so a
// call never overwrites a table whose copy may still be pending; every call
// ends synchronised, so the next one may reuse them.
struct StageLayout {
    size_t ddesc, dmap, fdesc, fmap, far, farmap, stats, flips2, total;
};

StageLayout stage_layout(int m, int64_t dens_blocks, int64_t flip_blocks, int64_t far_blocks) {
    StageLayout S{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += align256(bytes ? bytes : 1);
        return r;
    };
    S.ddesc = take(sizeof(MolDesc) * (size_t)m);
    S.dmap = take(4 * (size_t)dens_blocks);
    S.fdesc = take(sizeof(MolDesc) * (size_t)m);
    S.fmap = take(4 * (size_t)flip_blocks);
    S.far = take(sizeof(FarDesc) * (size_t)m);
    S.farmap = take(4 * (size_t)far_blocks);
    S.stats = take(8 * 3 * (size_t)m);
    S.flips2 = take(2 * 4 * (size_t)m * SWEEP_BATCH);
    S.total = o;
    return S;
}

// Grows the pinned staging buffer of c to at least `bytes` (waiting for the
// stream first, so that no copy from the old buffer is pending).
vesis_status ensure_stage(vesis_ctx* c, size_t bytes) {
    vesis_ctx* ctx = c;
    if (c->hstage_busy) {  // a call that stopped early may have left copies queued
        CK(hipStreamSynchronize(c->stream));
        c->hstage_busy = false;
    }
    if (c->hstage_bytes >= bytes) return VESIS_OK;
    if (c->hstage) {
        (void)hipHostFree(c->hstage);
        c->hstage = nullptr;
        c->hstage_bytes = 0;
    }
    void* p = nullptr;
    CK(hipHostMalloc(&p, bytes, hipHostMallocDefault));
    c->hstage = static_cast<char*>(p);
    c->hstage_bytes = bytes;
    return VESIS_OK;
}

// The largest block counts any density variant or the flip passes need.
void batch_blocks(vesis_ctx* const* c, int m, int64_t& dens, int64_t& flip, int64_t& far) {
    dens = 0;
    flip = 0;
    far = 0;
    for (int i = 0; i < m; ++i) far += points_blocks(c[i]->nfar, c[i]->na);
    for (int v = 0; v < DENSITY_VARIANTS; ++v) {
        int64_t s = 0;
        for (int i = 0; i < m; ++i) s += density_bricks(c[i]->g, v);
        dens = std::max(dens, s);
    }
    // the colour passes' block map: every molecule's blocks, dealt to the
    // dies, padded to the longest die's list (at most one molecule longer
    // than the even share)
    int64_t most = 0;
    for (int i = 0; i < m; ++i) {
        const int64_t nb = flip_blocks(c[i]->g, c[i]->sc.p);
        flip += nb;
        most = std::max(most, nb);
    }
    flip = NXCD_BATCH * ((flip + NXCD_BATCH - 1) / NXCD_BATCH + most);
}

MolDesc mol_desc(vesis_ctx* c) {
    MolDesc d{};
    d.g = c->g;
    d.sc = c->sc;
    d.a = dev_atoms(c);
    d.ph = dev_physics(c);
    d.f = cell_fields(c);
    d.bits = at<uint32_t>(c, c->lay.bits);
    d.stamp = at<int>(c, c->lay.stamp);
    d.u64cache = at<double>(c, c->lay.u64cache);
    d.sweep_flips = at<int>(c, c->lay.sweep_flips);
    d.counters = at<int64_t>(c, c->lay.scal_i) + SI_CNT;
    return d;
}

// Common checks of a batch call; on success `L` is the batch workspace layout.
vesis_status batch_check(vesis_ctx* const* c, int32_t m, void* bws, size_t bytes, bool labels,
                         BatchLayout& L, StageLayout& S) {
    if (!c || m < 1 || m > BATCH_MAX)
        return fail(m >= 1 && c ? c[0] : nullptr, VESIS_E_ARG, "need 1 to 4096 contexts");
    vesis_ctx* c0 = c[0];
    if (!c0) return VESIS_E_ARG;
    for (int i = 0; i < m; ++i) {
        if (!c[i]) return fail(c0, VESIS_E_ARG, "null context in batch");
        for (int j = 0; j < i; ++j)
            if (c[j] == c[i]) return fail(c0, VESIS_E_ARG, "context repeated in batch");
        vesis_status s = need(c[i], labels);
        if (s != VESIS_OK) {
            c0->err = "batch member " + std::to_string(i) + ": " + c[i]->err;
            return s;
        }
        if (c[i]->device != c0->device || c[i]->stream != c0->stream)
            return fail(c0, VESIS_E_ARG, "batch members must share device and stream");
        if (c[i]->prm.precision != 32)
            return fail(c0, VESIS_E_ARG, "batched minimisation needs FP32 densities");
        if (c[i]->sc.p != c0->sc.p)
            return fail(c0, VESIS_E_ARG, "batch members must share the colour period");
    }
    int64_t db, fb;
    int64_t pb;
    batch_blocks(c, m, db, fb, pb);
    L = batch_layout(m, db, fb, pb);
    if (!bws || (reinterpret_cast<uintptr_t>(bws) & 255))
        return fail(c0, VESIS_E_ARG, "batch workspace must be a 256-byte aligned device pointer");
    if (bytes < L.total)
        return fail(c0, VESIS_E_WORKSPACE, "batch workspace too small: need " +
                                               std::to_string(L.total) + " bytes");
    S = stage_layout(m, db, fb, pb);
    vesis_status se = ensure_stage(c0, S.total);
    if (se != VESIS_OK) return se;
    for (int i = 0; i < m; ++i) {
        vesis_status s = upload_inputs(c[i]);
        if (s != VESIS_OK) {
            c0->err = "batch member " + std::to_string(i) + ": " + c[i]->err;
            return s;
        }
    }
    return VESIS_OK;
}

// One batched density launch over the listed molecules, heaviest first (the
// blocks of the costliest molecules are dispatched first, the light ones
// fill the tail).
vesis_status batch_density(vesis_ctx* c0, vesis_ctx* const* c, const std::vector<int>& which,
                           char* bws, const BatchLayout& L, const StageLayout& S, int variant) {
    vesis_ctx* ctx = c0;
    hipStream_t st = c0->stream;
    if (which.empty()) return VESIS_OK;
    std::vector<int> order(which);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return (double)c[x]->na * (double)c[x]->g.ncell() > (double)c[y]->na * (double)c[y]->g.ncell();
    });
    // the tables go through the pinned staging buffer, so nothing here waits
    // for the device
    MolDesc* desc = reinterpret_cast<MolDesc*>(c0->hstage + S.ddesc);
    int* map = reinterpret_cast<int*>(c0->hstage + S.dmap);
    int64_t nmap = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        desc[k] = mol_desc(c[order[k]]);
        desc[k].brick0 = nmap;
        const int64_t nb = density_bricks(c[order[k]]->g, variant);
        for (int64_t j = 0; j < nb; ++j) map[nmap + j] = (int)k;
        nmap += nb;
    }
    c0->hstage_busy = true;
    CK(hipMemcpyAsync(bws + L.desc, desc, sizeof(MolDesc) * order.size(), hipMemcpyHostToDevice,
                      st));
    CK(hipMemcpyAsync(bws + L.dmap, map, 4 * (size_t)nmap, hipMemcpyHostToDevice, st));
    {
        Timed t(c0, K_DENSITY);
        CK(launch_density_batch(reinterpret_cast<const MolDesc*>(bws + L.desc),
                                reinterpret_cast<const int*>(bws + L.dmap), nmap, variant, st));
    }
    return VESIS_OK;
}

// After batch_density: what density_tail does for each molecule in `which`
// (NaN fill of the near-tie cache, far field, its sums), in five launches.
vesis_status batch_far(vesis_ctx* c0, vesis_ctx* const* c, const std::vector<int>& which,
                       char* bws, const BatchLayout& L, const StageLayout& S) {
    vesis_ctx* ctx = c0;
    hipStream_t st = c0->stream;
    if (which.empty()) return VESIS_OK;
    FarDesc* fd = reinterpret_cast<FarDesc*>(c0->hstage + S.far);
    int* map = reinterpret_cast<int*>(c0->hstage + S.farmap);
    int64_t nmap = 0, max_np = 0, max_ncell = 0;
    for (size_t k = 0; k < which.size(); ++k) {
        vesis_ctx* x = c[which[k]];
        FarDesc& d = fd[k];
        d.pts = at<double4>(x, x->lay.far_pts);
        d.np = x->nfar;
        d.a = dev_atoms(x);
        d.ph = dev_physics(x);
        d.nsplit = points_split(x->nfar, x->na);
        d.chunk = (x->na + d.nsplit - 1) / d.nsplit;
        d.part = at<double>(x, x->lay.far_part);
        d.ulj = at<double>(x, x->lay.far_ulj);
        d.ucfa = at<double>(x, x->lay.far_ucfa);
        d.ex = at<double>(x, x->lay.far_ex);
        d.ey = at<double>(x, x->lay.far_ey);
        d.ez = at<double>(x, x->lay.far_ez);
        d.partial = at<double>(x, x->lay.red_d);
        d.out = at<double>(x, x->lay.scal_d) + SD_FAR;
        d.u64cache = at<double>(x, x->lay.u64cache);
        d.ncell = x->g.ncell();
        d.block0 = nmap;
        const int64_t nb = x->nfar > 0 ? points_blocks(x->nfar, x->na) : 0;
        for (int64_t j = 0; j < nb; ++j) map[nmap + j] = (int)k;
        nmap += nb;
        max_np = std::max(max_np, x->nfar);
        max_ncell = std::max(max_ncell, d.ncell);
    }
    c0->hstage_busy = true;
    CK(hipMemcpyAsync(bws + L.far, fd, sizeof(FarDesc) * which.size(), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(bws + L.farmap, map, 4 * (size_t)std::max<int64_t>(nmap, 1),
                      hipMemcpyHostToDevice, st));
    {
        Timed t(c0, K_FAR);
        CK(launch_far_batch(reinterpret_cast<const FarDesc*>(bws + L.far),
                            reinterpret_cast<const int*>(bws + L.farmap), (int)which.size(), nmap,
                            max_np, max_ncell, RED_BLOCKS, st));
    }
    for (int i : which) c[i]->dens_valid = true;
    return VESIS_OK;
}

}  // namespace

vesis_status vesis_batch_workspace_size(vesis_ctx* const* ctxs, int32_t m, size_t* bytes) {
    if (!ctxs || !bytes || m < 1 || m > BATCH_MAX) return VESIS_E_ARG;
    for (int i = 0; i < m; ++i)
        if (!ctxs[i] || !ctxs[i]->has_grid || !ctxs[i]->has_params)
            return fail(ctxs[0], VESIS_E_STATE, "batch members need parameters and a grid");
    int64_t db, fb;
    int64_t pb;
    batch_blocks(ctxs, m, db, fb, pb);
    *bytes = batch_layout(m, db, fb, pb).total;
    return VESIS_OK;
}

// The colour-pass tables of a batch call: descriptors and the block map,
// staged and copied to the batch workspace; returns the pass grid.
int64_t batch_pass_tables(vesis_ctx* ctx, vesis_ctx* const* ctxs, int m, char* b,
                          const BatchLayout& L, const StageLayout& S, int64_t& max_words,
                          MolDesc*& desc) {
    const int p = ctx->sc.p;
    desc = reinterpret_cast<MolDesc*>(ctx->hstage + S.fdesc);
    int* map = reinterpret_cast<int*>(ctx->hstage + S.fmap);
    max_words = 0;
    // Each molecule's blocks go to one die (its labels then stay in that
    // die's L2 for the pass), largest molecules first, each to the die with
    // the fewest blocks so far; workgroup NXCD j + x runs entry j of die x.
    std::vector<int64_t> nbm(m);
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) {
        desc[i] = mol_desc(ctxs[i]);
        desc[i].slot0 = 0;
        nbm[i] = flip_blocks(ctxs[i]->g, p);
        order[i] = i;
        max_words = std::max(max_words, ctxs[i]->g.nwords());
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b2) { return nbm[a] > nbm[b2]; });
    std::vector<std::vector<int>> lists(NXCD_BATCH);
    std::vector<int64_t> load(NXCD_BATCH, 0);
    for (int i : order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (int64_t j = 0; j < nbm[i]; ++j) lists[x].push_back(i | (int)(j << BATCH_MOL_BITS));
        load[x] += nbm[i];
    }
    int64_t longest = 0;
    for (const auto& l : lists) longest = std::max<int64_t>(longest, (int64_t)l.size());
    const int64_t nmap = NXCD_BATCH * longest;
    for (int64_t j = 0; j < longest; ++j)
        for (int x = 0; x < NXCD_BATCH; ++x)
            map[NXCD_BATCH * j + x] = j < (int64_t)lists[x].size() ? lists[x][j] : -1;
    ctx->hstage_busy = true;
    (void)hipMemcpyAsync(b + L.desc, desc, sizeof(MolDesc) * m, hipMemcpyHostToDevice, ctx->stream);
    (void)hipMemcpyAsync(b + L.fmap, map, 4 * (size_t)nmap, hipMemcpyHostToDevice, ctx->stream);
    return nmap;
}

// One sweep of colour passes over a batch.  Colour-pass variant 0 with
// colour period 3 runs the colours that share their rows three to a launch
// (launch_flip_group3_batch); otherwise one launch per colour, variant v
// selecting the register budget of flip_pass_kernel.
constexpr int TUNE_SWEEPS = 4;  // colour-pass sweeps the tuner times
static_assert(TUNE_SWEEPS <= SWEEP_BATCH, "the sweep flip counts the tuner clears");

hipError_t launch_batch_sweep(const MolDesc* ddesc, const int* dmap, const int* ddone, const int* dpass,
                              int64_t nblocks, int p, int sw, int fvar, hipStream_t st) {
    const int ncol = p * p * p;
    hipError_t e = hipSuccess;
    if (p == 3 && fvar == 0) {
        for (int grp = 0; grp < 9 && e == hipSuccess; ++grp)
            e = launch_flip_group3_batch(ddesc, dmap, ddone, dpass, nblocks, grp, sw,
                                         sw * ncol + 3 * grp, st);
        return e;
    }
    for (int c = 0; c < ncol && e == hipSuccess; ++c)
        e = launch_flip_pass_batch(ddesc, dmap, ddone, dpass, nblocks, p, c, sw, sw * ncol + c,
                                   st);
    return e;
}

vesis_status vesis_batch_tune(vesis_ctx* const* ctxs, int32_t m, void* bws, size_t bytes,
                              int32_t* best, double* ms) {
    BatchLayout L;
    StageLayout S;
    vesis_status s = batch_check(ctxs, m, bws, bytes, false, L, S);
    if (s != VESIS_OK) return s;
    if (!best) return fail(ctxs[0], VESIS_E_ARG, "null argument");
    vesis_ctx* ctx = ctxs[0];
    hipStream_t st = ctx->stream;
    char* b = static_cast<char*>(bws);
    std::vector<int> all(m);
    for (int i = 0; i < m; ++i) all[i] = i;
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    auto elapsed = [&](float& t) -> hipError_t {
        hipError_t e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        return e;
    };
    // density tilings
    int dbest = 0;
    double tbest = 0.0;
    for (int v = 0; v < DENSITY_VARIANTS && s == VESIS_OK; ++v) {
        double tv = 1e300;
        for (int rep = 0; rep < 2; ++rep) {  // the first run also warms the caches
            CK(hipEventRecord(e0, st));
            s = batch_density(ctx, ctxs, all, b, L, S, v);
            if (s != VESIS_OK) break;
            CK(hipEventRecord(e1, st));
            float t = 0.f;
            CK(elapsed(t));
            ctx->hstage_busy = false;
            tv = std::min(tv, (double)t);
        }
        if (s != VESIS_OK) break;
        if (ms) ms[v] = tv;
        if (v == 0 || tv < tbest) {
            tbest = tv;
            dbest = v;
        }
    }
    // colour-pass variants: the first TUNE_SWEEPS sweeps over the batch
    // from its current labels, which are saved first and put back
    // after each run (in each molecule's force staging scratch, which no
    // result depends on between calls).  Needs labels on every molecule.
    bool labelled = s == VESIS_OK;
    for (int i = 0; i < m && labelled; ++i) labelled = ctxs[i]->has_labels;
    int fbest = 0;
    for (int v = 0; v < FLIP_VARIANTS && ms; ++v) ms[DENSITY_VARIANTS + v] = -1.0;
    if (labelled) {
        const int p = ctx->sc.p;
        int64_t max_words = 0;
        MolDesc* desc = nullptr;
        const int64_t nblocks = batch_pass_tables(ctx, ctxs, m, b, L, S, max_words, desc);
        const MolDesc* ddesc = reinterpret_cast<const MolDesc*>(b + L.desc);
        const int* dmap = reinterpret_cast<const int*>(b + L.fmap);
        int* ddone = reinterpret_cast<int*>(b + L.done);
        int* dpass = reinterpret_cast<int*>(b + L.pass);
        for (int i = 0; i < m; ++i)
            CK(hipMemcpyAsync(ctxs[i]->ws + ctxs[i]->lay.fstage, desc[i].bits,
                              4 * (size_t)ctxs[i]->g.nwords(), hipMemcpyDeviceToDevice, st));
        double fb = 0.0;
        // with colour period 2 both variants launch one colour at a time
        const int nfv = p == 3 ? FLIP_VARIANTS : 1;
        for (int v = 0; v < nfv; ++v) {
            double tv = 1e300;
            for (int rep = 0; rep < 2; ++rep) {
                CK(launch_batch_prepare(ddesc, m, max_words, st));
                CK(launch_fill_u32(reinterpret_cast<uint32_t*>(ddone), m, 0u, st));
                CK(launch_fill_u32(reinterpret_cast<uint32_t*>(dpass), 1, 0u, st));
                CK(launch_batch_clear_flips(ddesc, m, SWEEP_BATCH, st));
                CK(hipEventRecord(e0, st));
                // the first sweeps from the start: the first, where every
                // band cell is a candidate, and the lighter ones after it
                for (int sw = 0; sw < TUNE_SWEEPS; ++sw)
                    CK(launch_batch_sweep(ddesc, dmap, ddone, dpass, nblocks, p, sw, v, st));
                CK(hipEventRecord(e1, st));
                float t = 0.f;
                CK(elapsed(t));
                tv = std::min(tv, (double)t);
                for (int i = 0; i < m; ++i)
                    CK(hipMemcpyAsync(desc[i].bits, ctxs[i]->ws + ctxs[i]->lay.fstage,
                                      4 * (size_t)ctxs[i]->g.nwords(), hipMemcpyDeviceToDevice,
                                      st));
            }
            if (ms) ms[DENSITY_VARIANTS + v] = tv;
            if (v == 0 || tv < fb) {
                fb = tv;
                fbest = v;
            }
        }
        CK(hipStreamSynchronize(st));
        ctx->hstage_busy = false;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *best = dbest + DENSITY_VARIANTS * fbest;
    // the densities now come from the last variant tried: recompute on use
    for (int i = 0; i < m; ++i) {
        ctxs[i]->dens_valid = false;
        ctxs[i]->ss_valid = false;
        ctxs[i]->forces_valid = false;
    }
    return s;
}

void release_batch_graph(vesis_ctx* c) {
    if (c->bexec) (void)hipGraphExecDestroy(c->bexec);
    if (c->bgraph) (void)hipGraphDestroy(c->bgraph);
    c->bexec = nullptr;
    c->bgraph = nullptr;
}

vesis_status vesis_minimize_batch(vesis_ctx* const* ctxs, int32_t m, void* bws, size_t bytes,
                                  int32_t max_sweeps, int32_t variant, int32_t flags,
                                  vesis_min_stats* out) {
    BatchLayout L;
    StageLayout S;
    vesis_status s = batch_check(ctxs, m, bws, bytes, true, L, S);
    if (s != VESIS_OK) return s;
    vesis_ctx* ctx = ctxs[0];
    if (max_sweeps < 1) return fail(ctx, VESIS_E_ARG, "max_sweeps must be >= 1");
    if (variant < 0 || variant >= DENSITY_VARIANTS * FLIP_VARIANTS)
        return fail(ctx, VESIS_E_ARG, "batch variant out of range");
    const int dvar = variant % DENSITY_VARIANTS, fvar = variant / DENSITY_VARIANTS;
    hipStream_t st = ctx->stream;
    char* b = static_cast<char*>(bws);
    // a1 + a2: one density launch over every molecule whose atoms changed
    std::vector<int> stale;
    for (int i = 0; i < m; ++i)
        if (!ctxs[i]->dens_valid) stale.push_back(i);
    s = batch_density(ctx, ctxs, stale, b, L, S, dvar);
    if (s != VESIS_OK) return s;
    s = batch_far(ctx, ctxs, stale, b, L, S);
    if (s != VESIS_OK) return s;
    // a3 + a4: one launch per colour pass over every unconverged molecule
    const int p = ctx->sc.p, ncol = p * p * p;
    int64_t max_words = 0;
    MolDesc* desc = nullptr;
    const int64_t nblocks = batch_pass_tables(ctx, ctxs, m, b, L, S, max_words, desc);
    std::vector<char> done(m, 0);
    std::vector<int> msweeps(m, 0);
    std::vector<int64_t> mflips(m, 0);
    const MolDesc* ddesc = reinterpret_cast<const MolDesc*>(b + L.desc);
    const int* dmap = reinterpret_cast<const int*>(b + L.fmap);
    int* ddone = reinterpret_cast<int*>(b + L.done);
    int* dpass = reinterpret_cast<int*>(b + L.pass);
    int* dflips = reinterpret_cast<int*>(b + L.flips);
    int* hflips = reinterpret_cast<int*>(ctx->hstage + S.flips2);
    // every molecule's stamps older than any pass and its tie counters zero
    CK(launch_batch_prepare(ddesc, m, max_words, st));
    CK(launch_fill_u32(reinterpret_cast<uint32_t*>(ddone), m, 0u, st));
    CK(launch_fill_u32(reinterpret_cast<uint32_t*>(dpass), 1, 0u, st));
    // one group of sweeps: every pass of every colour over the molecules not
    // yet done, then the done flags, the pass counter and the flip counts
    auto enqueue_group = [&](hipStream_t s2, int nb) -> hipError_t {
        hipError_t e = launch_batch_clear_flips(ddesc, m, SWEEP_BATCH, s2);
        for (int sw = 0; sw < nb && e == hipSuccess; ++sw)
            e = launch_batch_sweep(ddesc, dmap, ddone, dpass, nblocks, p, sw, fvar, s2);
        if (e == hipSuccess) e = launch_batch_end_group(ddesc, m, nb, ncol, ddone, dpass, s2);
        if (e == hipSuccess) e = launch_batch_gather_flips(ddesc, m, SWEEP_BATCH, dflips, s2);
        return e;
    };
    const bool use_graph = !(flags & VESIS_BATCH_EAGER);
    if (ctx->bexec && !(ctx->bkey_ws == bws && ctx->bkey_m == m && ctx->bkey_nblocks == nblocks &&
                        ctx->bkey_p == p && ctx->bkey_fv == fvar))
        release_batch_graph(ctx);
    // a full group is the same sequence of launches every time: captured once
    // on a private stream, replayed on the caller's stream (no memset nodes:
    // counters are cleared by kernels)
    auto launch_group = [&](int nb) -> hipError_t {
        hipError_t e = hipSuccess;
        if (use_graph && nb == SWEEP_BATCH) {
            if (!ctx->bexec) {
                if (!ctx->capture) {
                    e = hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking);
                    if (e != hipSuccess) ctx->capture = nullptr;
                }
                if (e == hipSuccess) e = hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeRelaxed);
                if (e == hipSuccess) {
                    const hipError_t e1 = enqueue_group(ctx->capture, nb);
                    const hipError_t e2 = hipStreamEndCapture(ctx->capture, &ctx->bgraph);
                    e = e1 != hipSuccess ? e1 : e2;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&ctx->bexec, ctx->bgraph, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    release_batch_graph(ctx);
                    return e;
                }
                ctx->bkey_ws = bws;
                ctx->bkey_m = m;
                ctx->bkey_nblocks = nblocks;
                ctx->bkey_p = p;
                ctx->bkey_fv = fvar;
            }
            Timed t(ctx, K_FLIP);
            return hipGraphLaunch(ctx->bexec, st);
        }
        Timed t(ctx, K_FLIP);
        return enqueue_group(st, nb);
    };
    for (int k = 0; k < 2; ++k)
        if (!ctx->bev[k]) CK(hipEventCreateWithFlags(&ctx->bev[k], hipEventDisableTiming));
    // Groups are issued ahead of the host: while more than an eighth of the
    // molecules are still relaxing, the next group is queued before the
    // host waits for the current one's flip counts, so the device does not
    // idle through the round trip; near the end, when a queued group would
    // mostly find every molecule done, the host waits first.  At most two
    // groups are in flight (two host slots for their counts).
    struct Inflight { int slot, nb; };
    Inflight q[2];
    int nq = 0, next_slot = 0, enq = 0, sweeps = 0, active = m;
    auto issue = [&]() -> hipError_t {
        const int nb = std::min(SWEEP_BATCH, max_sweeps - enq);
        hipError_t e = launch_group(nb);
        const int slot = next_slot;
        if (e == hipSuccess)
            e = hipMemcpyAsync(hflips + (size_t)slot * m * SWEEP_BATCH, dflips,
                               4 * (size_t)m * SWEEP_BATCH, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(ctx->bev[slot], st);
        if (e == hipSuccess) {
            q[nq++] = Inflight{slot, nb};
            next_slot ^= 1;
            enq += nb;
        }
        return e;
    };
    hipError_t e = issue();
    while (e == hipSuccess && nq > 0) {
        if (nq == 1 && enq < max_sweeps && active > std::max(1, m / 8)) e = issue();
        if (e != hipSuccess) break;
        const Inflight g = q[0];
        q[0] = q[1];
        --nq;
        e = hipEventSynchronize(ctx->bev[g.slot]);
        if (e != hipSuccess) break;
        const int* hf = hflips + (size_t)g.slot * m * SWEEP_BATCH;
        for (int i = 0; i < m; ++i) {
            if (done[i]) continue;
            for (int sw = 0; sw < g.nb; ++sw) {
                const int f = hf[(size_t)i * SWEEP_BATCH + sw];
                mflips[i] += f;
                ++msweeps[i];
                if (f == 0) {
                    done[i] = 1;
                    --active;
                    break;
                }
            }
        }
        sweeps += g.nb;
        if (active == 0) break;  // a group still queued finds every molecule done
        if (nq == 0 && enq < max_sweeps) e = issue();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    ctx->hstage_busy = false;
    if (e != hipSuccess) {
        release_batch_graph(ctx);
        return fail(ctx, VESIS_E_DEVICE, std::string("batched sweeps: ") + hipGetErrorString(e));
    }
    for (int i = 0; i < m; ++i)
        if (mflips[i] > 0) ctxs[i]->forces_valid = false;
    if (out) {
        // every molecule's band count and tie counters, read back together
        int64_t* hs = reinterpret_cast<int64_t*>(ctx->hstage + S.stats);
        ctx->hstage_busy = true;
        for (int i = 0; i < m; ++i) {
            vesis_ctx* c = ctxs[i];
            CK(launch_band_count(c->g, at<uint32_t>(c, c->lay.bits), at<int64_t>(c, c->lay.red_i),
                                 RED_BLOCKS, at<int64_t>(c, c->lay.scal_i) + SI_BAND, st));
            CK(hipMemcpyAsync(hs + 3 * i, desc[i].counters, 2 * sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
            CK(hipMemcpyAsync(hs + 3 * i + 2, c->ws + c->lay.scal_i + 8 * SI_BAND, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
        }
        CK(hipStreamSynchronize(st));
        ctx->hstage_busy = false;
        for (int i = 0; i < m; ++i) {
            out[i].sweeps = msweeps[i];
            out[i].converged = done[i] ? 1 : 0;
            out[i].flips = mflips[i];
            out[i].band_cells = hs[3 * i + 2];
            out[i].near_ties = hs[3 * i];
            out[i].fp64_recomputes = hs[3 * i + 1];
        }
    }
    ctx->err.clear();
    (void)sweeps;
    return active == 0 ? VESIS_OK : VESIS_NOT_CONVERGED;
}

// ------------------------------------------------ serial (min-heap) schedule

namespace {

struct HeapItem {
    double key;
    int64_t idx;
    int64_t ver;
};
// min-heap order on (Delta E, cell index): std::push_heap keeps the largest
// first, so "less" means "later"
struct HeapLater {
    bool operator()(const HeapItem& a, const HeapItem& b) const {
        return a.key != b.key ? a.key > b.key : a.idx > b.idx;
    }
};

}  // namespace

vesis_status vesis_minimize_heap(vesis_ctx* ctx, int64_t max_flips, vesis_min_stats* out) {
    if (!ctx) return VESIS_E_ARG;
    if (max_flips < 0) return fail(ctx, VESIS_E_ARG, "max_flips must be >= 0");
    vesis_status s = need(ctx, true);
    if (s != VESIS_OK) return s;
    s = ensure_density(ctx);
    if (s != VESIS_OK) return s;
    hipStream_t st = ctx->stream;
    const Grid& g = ctx->g;
    const int n = g.n;
    const int64_t ncell = g.ncell();
    // the labels and the stored densities and bounds, on the host
    std::vector<int8_t> phi(ncell);
    s = vesis_get_labels(ctx, phi.data());
    if (s != VESIS_OK) return s;
    std::vector<double> U(ncell), B(ncell);
    {
        std::vector<double> lj(ncell), cfa(ncell);
        s = vesis_get_density(ctx, lj.data(), cfa.data(), B.data());
        if (s != VESIS_OK) return s;
        for (int64_t c = 0; c < ncell; ++c) U[c] = lj[c] + cfa[c];
    }
    const double h3 = g.h * g.h * g.h, cc = ctx->sc.c;
    const Atoms a = dev_atoms(ctx);
    const Physics ph = dev_physics(ctx);
    double* u64 = at<double>(ctx, ctx->lay.u64cache);
    std::vector<double> exact(ncell, NAN);  // FP64 U of near-tie cells, once each
    int64_t near_ties = 0, recomputes = 0;
    auto label = [&](int x, int y, int z) -> int {
        if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return 1;  // outside: solvent
        return phi[x + (int64_t)n * (y + (int64_t)n * z)];
    };
    auto in_band = [&](int x, int y, int z) {
        const int me = label(x, y, z);
        return label(x - 1, y, z) != me || label(x + 1, y, z) != me || label(x, y - 1, z) != me ||
               label(x, y + 1, z) != me || label(x, y, z - 1) != me || label(x, y, z + 1) != me;
    };
    hipError_t herr = hipSuccess;
    // the stencil's offsets (squared length 1..8) and, per cell, the number
    // of solvent cells at each squared offset (outside the box: solvent),
    // kept up to date flip by flip
    struct Off {
        int dx, dy, dz, q;
    };
    std::vector<Off> offs;
    for (int dz = -2; dz <= 2; ++dz)
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                const int q = dx * dx + dy * dy + dz * dz;
                if (q >= 1 && q <= 8) offs.push_back({dx, dy, dz, q});
            }
    std::vector<uint8_t> cnt(9 * (size_t)ncell, 0);
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                uint8_t* cc9 = &cnt[9 * (size_t)(x + (int64_t)n * (y + (int64_t)n * z))];
                for (const Off& o : offs) cc9[o.q] += label(x + o.dx, y + o.dy, z + o.dz) == 1;
            }
    // Delta E of cell (x, y, z), decided as a colour pass decides it: the
    // stored U unless |Delta E| is within the cell's bound, then FP64 U
    auto delta_e = [&](int x, int y, int z) -> double {
        static const int NS[9] = {0, 6, 12, 8, 6, 24, 24, 0, 12};
        const int64_t c = x + (int64_t)n * (y + (int64_t)n * z);
        const uint8_t* cc9 = &cnt[9 * (size_t)c];
        double S = 0.0;
        for (int q = 1; q <= 8; ++q) S += ctx->sc.w[q] * (double)(2 * (int)cc9[q] - NS[q]);
        const double p = phi[c] == 1 ? 1.0 : -1.0;
        const double cS = cc * S, hU = h3 * U[c];
        const double dE = p * (cS - hU);
        if (std::fabs(dE) > h3 * B[c] + 4.0e-16 * (std::fabs(cS) + std::fabs(hU))) return dE;
        ++near_ties;
        if (std::isnan(exact[c])) {
            double two[2];
            if (herr == hipSuccess) herr = launch_cell_density_f64(g, a, ph, x, y, z, u64, st);
            if (herr == hipSuccess) herr = hipMemcpyAsync(&two[0], u64 + c, 8, hipMemcpyDeviceToHost, st);
            if (herr == hipSuccess)
                herr = hipMemcpyAsync(&two[1], u64 + ncell + c, 8, hipMemcpyDeviceToHost, st);
            if (herr == hipSuccess) herr = hipStreamSynchronize(st);
            if (herr != hipSuccess) return 0.0;
            exact[c] = two[0] + two[1];
            ++recomputes;
        }
        return p * (cS - h3 * exact[c]);
    };
    // the paper's flipping process: every band cell's Delta E in a min-heap;
    // while the smallest is negative, flip that cell and re-evaluate the
    // cells whose Delta E or band membership it changed (within two cells
    // along each axis: the kernel's support); stale entries are dropped by a
    // per-cell version
    std::vector<int64_t> ver(ncell, 0);
    std::vector<HeapItem> heap;
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x)
                if (in_band(x, y, z))
                    heap.push_back({delta_e(x, y, z), x + (int64_t)n * (y + (int64_t)n * z), 0});
    std::make_heap(heap.begin(), heap.end(), HeapLater());
    int64_t flips = 0;
    bool converged = false;
    while (herr == hipSuccess) {
        if (heap.empty()) {
            converged = true;
            break;
        }
        std::pop_heap(heap.begin(), heap.end(), HeapLater());
        const HeapItem it = heap.back();
        heap.pop_back();
        if (it.ver != ver[it.idx]) continue;
        if (it.key >= 0.0) {
            converged = true;
            break;
        }
        if (flips == max_flips) break;
        phi[it.idx] = (int8_t)(-phi[it.idx]);
        ++flips;
        const int x0 = (int)(it.idx % n), y0 = (int)((it.idx / n) % n), z0 = (int)(it.idx / ((int64_t)n * n));
        // the flipped cell's stencil neighbours gain or lose a solvent cell
        // at their offset; they and the cell itself are re-evaluated (the
        // rest of the 5 x 5 x 5 cube keeps its Delta E and band membership)
        auto reevaluate = [&](int x, int y, int z) {
            const int64_t c = x + (int64_t)n * (y + (int64_t)n * z);
            ++ver[c];
            if (in_band(x, y, z)) {
                heap.push_back({delta_e(x, y, z), c, ver[c]});
                std::push_heap(heap.begin(), heap.end(), HeapLater());
            }
        };
        const int add = phi[it.idx] == 1 ? 1 : -1;
        for (const Off& o : offs) {
            const int x = x0 + o.dx, y = y0 + o.dy, z = z0 + o.dz;
            if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) continue;
            cnt[9 * (size_t)(x + (int64_t)n * (y + (int64_t)n * z)) + o.q] += add;
        }
        reevaluate(x0, y0, z0);
        for (const Off& o : offs) {
            const int x = x0 + o.dx, y = y0 + o.dy, z = z0 + o.dz;
            if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) continue;
            reevaluate(x, y, z);
        }
    }
    if (herr != hipSuccess)
        return fail(ctx, VESIS_E_DEVICE, std::string("FP64 near-tie density: ") + hipGetErrorString(herr));
    // the new labels back to the device
    s = vesis_init_labels(ctx, 2, 0.0, phi.data());
    if (s != VESIS_OK) return s;
    if (out) {
        int64_t band = 0;
        for (int z = 0; z < n; ++z)
            for (int y = 0; y < n; ++y)
                for (int x = 0; x < n; ++x) band += in_band(x, y, z);
        out->sweeps = 0;
        out->converged = converged ? 1 : 0;
        out->flips = flips;
        out->band_cells = band;
        out->near_ties = near_ties;
        out->fp64_recomputes = recomputes;
    }
    ctx->err.clear();
    return converged ? VESIS_OK : VESIS_NOT_CONVERGED;
}

vesis_status vesis_get_labels(vesis_ctx* ctx, int8_t* out) {
    if (!ctx || !out) return fail(ctx, VESIS_E_ARG, "null argument");
    vesis_status s = need(ctx, true);
    if (s != VESIS_OK) return s;
    const Grid& g = ctx->g;
    std::vector<uint32_t> host(g.nwords());
    CK(hipMemcpyAsync(host.data(), ctx->ws + ctx->lay.bits, 4 * host.size(), hipMemcpyDeviceToHost,
                      ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    for (int z = 0; z < g.n; ++z)
        for (int y = 0; y < g.n; ++y)
            for (int x = 0; x < g.n; ++x)
                out[x + (int64_t)g.n * (y + (int64_t)g.n * z)] =
                    ((host[g.row(y, z) + 1 + (x >> 5)] >> (x & 31)) & 1u) ? 1 : -1;
    return VESIS_OK;
}

vesis_status vesis_get_density(vesis_ctx* ctx, double* u_lj, double* u_cfa, double* bound) {
    if (!ctx || !u_lj || !u_cfa) return fail(ctx, VESIS_E_ARG, "null argument");
    vesis_status s = need(ctx, false);
    if (s != VESIS_OK) return s;
    s = ensure_density(ctx);
    if (s != VESIS_OK) return s;
    const size_t ncell = (size_t)ctx->g.ncell();
    if (ctx->prm.precision == 64) {
        const size_t nb = 8 * ncell;
        CK(hipMemcpyAsync(u_lj, ctx->ws + ctx->lay.ulj, nb, hipMemcpyDeviceToHost, ctx->stream));
        CK(hipMemcpyAsync(u_cfa, ctx->ws + ctx->lay.ucfa, nb, hipMemcpyDeviceToHost, ctx->stream));
        if (bound)
            CK(hipMemcpyAsync(bound, ctx->ws + ctx->lay.bound, nb, hipMemcpyDeviceToHost,
                              ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        return VESIS_OK;
    }
    // FP32 storage: copied as stored, widened on the host
    std::vector<float> tmp(ncell);
    double* dst[3] = {u_lj, u_cfa, bound};
    const size_t off[3] = {ctx->lay.ulj, ctx->lay.ucfa, ctx->lay.bound};
    for (int k = 0; k < 3; ++k) {
        if (!dst[k]) continue;
        CK(hipMemcpyAsync(tmp.data(), ctx->ws + off[k], 4 * ncell, hipMemcpyDeviceToHost,
                          ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        for (size_t c = 0; c < ncell; ++c) dst[k][c] = (double)tmp[c];
    }
    return VESIS_OK;
}

vesis_status vesis_profile(vesis_ctx* ctx, int32_t enable) {
    if (!ctx) return VESIS_E_ARG;
    if (!ctx->pending.empty()) drain_events(ctx);
    ctx->prof = enable != 0;
    for (int k = 0; k < K_NKINDS; ++k) {
        ctx->prof_ms[k] = 0.0;
        ctx->prof_n[k] = 0;
    }
    return VESIS_OK;
}

vesis_status vesis_profile_read(vesis_ctx* ctx, int32_t kind, double* total_ms, int64_t* launches) {
    if (!ctx || !total_ms || !launches) return fail(ctx, VESIS_E_ARG, "null argument");
    if (kind < 0 || kind >= K_NKINDS) return fail(ctx, VESIS_E_ARG, "kind out of range");
    drain_events(ctx);
    *total_ms = ctx->prof_ms[kind];
    *launches = ctx->prof_n[kind];
    return VESIS_OK;
}

}  // extern "C"
