/* Seeded self-avoiding globule walk: the same draws and the same decisions
 * as synth.globule's Python loop (SplitMix64 counter stream, directions by
 * rejection in the cube in batches of 6 * trials uniforms, first valid
 * candidate wins, backtrack on failure), only faster.  Input generation
 * only: no arithmetic of the method lives here.  Built with
 * -ffp-contract=off so every operation rounds as the numpy code does. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t seed, count;
} sm64;

static uint64_t sm64_at(const sm64* r, uint64_t k) {
    uint64_t z = r->seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* m unit vectors, exactly as _unit_vectors: rounds of 6m uniforms in
 * [-1, 1), triples with 1e-4 < r2 <= 1 kept in order, normalised. */
static void unit_vectors(sm64* r, int m, double* out, double* tmp) {
    int got = 0;
    while (got < m) {
        const int nu = 6 * m;
        for (int k = 0; k < nu; ++k) {
            const uint64_t z = sm64_at(r, r->count + 1 + (uint64_t)k);
            const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
            tmp[k] = -1.0 + 2.0 * u;
        }
        r->count += (uint64_t)nu;
        for (int t = 0; t < 2 * m; ++t) {
            const double x = tmp[3 * t], y = tmp[3 * t + 1], zz = tmp[3 * t + 2];
            const double r2 = x * x + y * y + zz * zz;
            if (r2 > 1e-4 && r2 <= 1.0) {
                if (got < m) {
                    const double s = sqrt(r2);
                    out[3 * got] = x / s;
                    out[3 * got + 1] = y / s;
                    out[3 * got + 2] = zz / s;
                }
                ++got;
            }
        }
    }
}

typedef struct {
    int64_t* head; /* per bin: first atom or -1 */
    int64_t* next; /* per atom */
    int64_t* prev;
    int64_t nb;    /* bins per axis */
    int64_t off;   /* bin index offset */
} grid_t;

static int64_t bin_of(const grid_t* g, const double* p, double w, int64_t* k) {
    for (int d = 0; d < 3; ++d) k[d] = (int64_t)floor(p[d] / w) + g->off;
    return (k[2] * g->nb + k[1]) * g->nb + k[0];
}

/* Returns 0 on success, 1 if the walk did not finish. */
int synth_globule(int64_t natoms, uint64_t seed, double bond, double min_sep, double min_sep2,
                  double density, int trials, int backtrack, double* pos) {
    sm64 rng = {seed, 0};
    const double pi = 3.141592653589793;
    const double rconf = pow(3.0 * (double)natoms / (4.0 * pi * density), 1.0 / 3.0);
    const double w = min_sep;
    grid_t g;
    g.off = (int64_t)ceil(rconf / w) + 4;
    g.nb = 2 * g.off + 1;
    const int64_t nbins = g.nb * g.nb * g.nb;
    g.head = malloc(sizeof(int64_t) * (size_t)nbins);
    g.next = malloc(sizeof(int64_t) * (size_t)natoms);
    g.prev = malloc(sizeof(int64_t) * (size_t)natoms);
    int64_t* binof = malloc(sizeof(int64_t) * (size_t)natoms);
    double* cand = malloc(sizeof(double) * 3 * (size_t)trials);
    double* tmp = malloc(sizeof(double) * 6 * (size_t)trials);
    for (int64_t b = 0; b < nbins; ++b) g.head[b] = -1;
    memset(pos, 0, sizeof(double) * 3 * (size_t)natoms);
    const double ms2 = min_sep * min_sep, ms22 = min_sep2 * min_sep2;
    /* bins keep atoms in insertion order (Python appends to a list and the
     * scan order does not change the accept/reject decision anyway) */
    int64_t kk[3];
#define ADD(i)                                                   \
    do {                                                         \
        const int64_t b_ = bin_of(&g, pos + 3 * (i), w, kk);     \
        binof[i] = b_;                                           \
        g.next[i] = g.head[b_];                                  \
        g.prev[i] = -1;                                          \
        if (g.head[b_] >= 0) g.prev[g.head[b_]] = (i);           \
        g.head[b_] = (i);                                        \
    } while (0)
#define REMOVE(i)                                                \
    do {                                                         \
        const int64_t b_ = binof[i];                             \
        if (g.prev[i] >= 0) g.next[g.prev[i]] = g.next[i];       \
        else g.head[b_] = g.next[i];                             \
        if (g.next[i] >= 0) g.prev[g.next[i]] = g.prev[i];       \
    } while (0)
    ADD(0);
    int64_t i = 1, guard = 0;
    int rc = 0;
    while (i < natoms) {
        if (++guard > 200 * natoms) {
            rc = 1;
            break;
        }
        unit_vectors(&rng, trials, cand, tmp);
        int placed = 0;
        for (int t = 0; t < trials && !placed; ++t) {
            double c[3];
            for (int d = 0; d < 3; ++d) c[d] = pos[3 * (i - 1) + d] + bond * cand[3 * t + d];
            if (c[0] * c[0] + c[1] * c[1] + c[2] * c[2] > rconf * rconf) continue;
            int64_t k[3];
            bin_of(&g, c, w, k);
            int ok = 1;
            for (int64_t az = k[2] - 1; az <= k[2] + 1 && ok; ++az)
                for (int64_t ay = k[1] - 1; ay <= k[1] + 1 && ok; ++ay)
                    for (int64_t ax = k[0] - 1; ax <= k[0] + 1 && ok; ++ax) {
                        for (int64_t j = g.head[(az * g.nb + ay) * g.nb + ax]; j >= 0; j = g.next[j]) {
                            if (j >= i - 1) continue;
                            const double dx = c[0] - pos[3 * j], dy = c[1] - pos[3 * j + 1],
                                         dz = c[2] - pos[3 * j + 2];
                            const double lim = (j == i - 2) ? ms22 : ms2;
                            if (dx * dx + dy * dy + dz * dz < lim) {
                                ok = 0;
                                break;
                            }
                        }
                    }
            if (ok) {
                for (int d = 0; d < 3; ++d) pos[3 * i + d] = c[d];
                ADD(i);
                ++i;
                placed = 1;
            }
        }
        if (!placed) {
            int64_t back = backtrack < i - 1 ? backtrack : i - 1;
            for (int64_t j = i - 1; j > i - 1 - back; --j) REMOVE(j);
            i -= back;
        }
    }
    free(g.head); free(g.next); free(g.prev); free(binof); free(cand); free(tmp);
    return rc;
}
