// The learned warm start: a 3-D U-Net on the cell grid, its layers as HIP
// kernels for gfx950.
//
// Activations are BF16 in channels-last order (n, z, y, x, c), so that the
// K dimension of a convolution (27 taps x Cin channels) is contiguous per
// tap.  A 3x3x3 convolution with zero padding is an implicit GEMM
//   Y[p][co] = sum_{tap, ci} X[p + off(tap)][ci] W[tap][co][ci]
// with M = positions, N = output channels, K = 27 Cin, computed with the
// CDNA4 BF16 matrix instruction v_mfma_f32_32x32x16_bf16 (32 x 32 x 16,
// FP32 accumulation).  Its operand layout (checked on the device): lane i
// holds A[i % 32][8 (i / 32) + j] and B[8 (i / 32) + j][i % 32] for
// j = 0..7, and the 16 results D[8 (r / 4) + 4 (i / 32) + r % 4][i % 32],
// r = 0..15.  A wavefront computes 32 positions x 32 NT output channels;
// a workgroup of four wavefronts 128 consecutive positions.
//
// The data gradient is the same convolution of dY with the weights flipped
// in space and transposed in channels; the weight gradient is a GEMM over
// positions (M = Cout, N = Cin per tap, K = positions) split over position
// chunks whose FP32 partial tiles are summed in a fixed order.
#include "internal.h"
#include "reduce.h"

namespace vesis {
namespace nn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int CWG = 256;  // convolution workgroup: four wavefronts

__device__ inline void pos_coords(int64_t p, int D, int H, int W, int& n, int& z, int& y, int& x) {
    x = (int)(p % W);
    int64_t r = p / W;
    y = (int)(r % H);
    r /= H;
    z = (int)(r % D);
    n = (int)(r / D);
}

// 8 consecutive BF16 values (16 bytes) as an MFMA operand.
__device__ inline bf16x8 load8(const __bf16* p) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    bf16x8 r;
    __builtin_memcpy(&r, &v, 16);
    return r;
}

// Y = [relu](conv3x3x3(X, Wt) + bias).  X: (P, Cin), Wt: (27, Cout, Cin),
// Y: (P, Cout); Cin % 16 == 0, Cout % (32 NT) == 0.
template <int NT, bool RELU>
__global__ __launch_bounds__(CWG) void conv3_fwd_kernel(const __bf16* __restrict__ X,
                                                        const __bf16* __restrict__ Wt,
                                                        const float* __restrict__ bias,
                                                        __bf16* __restrict__ Y, int N, int D,
                                                        int H, int W, int Cin, int Cout) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t P = (int64_t)N * D * H * W;
    const int64_t p0 = (int64_t)blockIdx.x * 128 + wv * 32;
    const int co0 = blockIdx.y * 32 * NT;
    const int row = lane & 31, half = lane >> 5;
    // the position whose A row this lane loads
    const int64_t pa = p0 + row;
    int n, z, y, x;
    pos_coords(pa < P ? pa : 0, D, H, W, n, z, y, x);
    const bool pa_ok = pa < P;
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x16{};
    // K = 27 taps x Cin/16 steps, flattened; the operands of step k + 1 are
    // loaded before the matrix instructions of step k issue
    const int ncb = Cin / 16, K = 27 * ncb;
    auto a_ptr = [&](int tap, bool& ok) {
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        const int zz = z + dz, yy = y + dy, xx = x + dx;
        ok = pa_ok && zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
        const int64_t q = (((int64_t)n * D + zz) * H + yy) * W + xx;
        return X + (ok ? q : 0) * Cin + 8 * half;
    };
    const __bf16* wrow = Wt + ((int64_t)co0 + row) * Cin + 8 * half;
    bool ok;
    const __bf16* xa = a_ptr(0, ok);
    bf16x8 a = load8(xa);
    if (!ok) a = bf16x8{};
    bf16x8 bb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bb[t] = load8(wrow + (int64_t)t * 32 * Cin);
    for (int k = 0; k < K; ++k) {
        bf16x8 an = bf16x8{}, bn[NT];
        const int k1 = k + 1 < K ? k + 1 : k;
        const int tap1 = k1 / ncb, c1 = (k1 - tap1 * ncb) * 16;
        bool ok1;
        const __bf16* xa1 = a_ptr(tap1, ok1);
        an = load8(xa1 + c1);
        if (!ok1) an = bf16x8{};
        const __bf16* wb1 = wrow + (int64_t)tap1 * Cout * Cin + c1;
#pragma unroll
        for (int t = 0; t < NT; ++t) bn[t] = load8(wb1 + (int64_t)t * 32 * Cin);
#pragma unroll
        for (int t = 0; t < NT; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb[t], acc[t], 0, 0, 0);
        a = an;
#pragma unroll
        for (int t = 0; t < NT; ++t) bb[t] = bn[t];
    }
    // D[8 (r/4) + 4 half + r%4][row]: position p0 + that, channel co0 + 32 t + row
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = co0 + 32 * t + row;
        const float bv = bias ? bias[co] : 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t p = p0 + 8 * (r / 4) + 4 * half + (r % 4);
            if (p >= P) continue;
            float v = acc[t][r] + bv;
            if (RELU) v = v > 0.f ? v : 0.f;
            Y[p * Cout + co] = (__bf16)v;
        }
    }
}

// The same convolution with the input staged in LDS.  A workgroup owns a
// tile of 4 MT x-rows of 32 positions (TY = 4 rows in y, TZ = MT in z) and
// 32 NT output channels; per chunk of 16 input channels it stages the tile
// with its one-cell halo (TZ+2) x 6 x 34 positions in LDS (16 channels =
// 32 bytes per position: the 32 rows of an operand are one contiguous
// kilobyte, though eight lanes' 16-byte reads then fall on every other 16
// bytes, a two-way bank conflict the z-reuse kernel below avoids), then
// runs the 27 taps:
// wavefront w takes y-row w of each of the MT z-layers of the tile (MT
// operands of 32 positions) against NT output-channel tiles, the weights
// read from global memory (shared by every workgroup, they stay in cache).
//
// The input may be the channel concatenation [up2(A) | B] read in place:
// channels [0, ca) come from A, which holds them at half resolution
// (nearest-neighbour upsampling: position (z, y, x) reads A at (z/2, y/2,
// x/2)) when `up` is set, and channels [ca, Cin) from B at full
// resolution.  ca is a multiple of 16, so a staged chunk of 16 channels
// comes from one tensor; the staged values, and hence the result, are those
// of the convolution of the materialised concatenation.
struct ConvIn {
    const __bf16* a;
    int ca;
    int up;
    const __bf16* b;
};

constexpr int TX = 32, TY = 4, HX = TX + 2, HY = TY + 2;
template <int MT, int NT, bool RELU>
__global__ __launch_bounds__(CWG) void conv3_fwd_lds_kernel(const ConvIn in,
                                                            const __bf16* __restrict__ Wt,
                                                            const float* __restrict__ bias,
                                                            __bf16* __restrict__ Y, int N, int D,
                                                            int H, int W, int Cin, int Cout) {
    constexpr int TZ = MT, HZ = TZ + 2, HPOS = HZ * HY * HX;
    __shared__ __attribute__((aligned(16))) __bf16 tile[HPOS * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = lane & 31, half = lane >> 5;
    const int ntx = (W + TX - 1) / TX, nty = (H + TY - 1) / TY, ntz = (D + TZ - 1) / TZ;
    const int x0 = (blockIdx.x % ntx) * TX;
    const int y0 = ((int)(blockIdx.x / ntx) % nty) * TY;
    const int co0 = blockIdx.y * 32 * NT;
    const int z0 = ((int)blockIdx.z % ntz) * TZ;
    const int nb = (int)blockIdx.z / ntz;
    f32x16 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[i][t] = f32x16{};
    const __bf16* wrow = Wt + ((int64_t)co0 + row) * Cin + 8 * half;
    const int cb = Cin - in.ca;
    const int Da = in.up ? D / 2 : D, Ha = in.up ? H / 2 : H, Wa = in.up ? W / 2 : W;
    for (int c0 = 0; c0 < Cin; c0 += 16) {
        __syncthreads();  // the previous chunk's reads are done
        const bool from_a = c0 < in.ca;  // uniform over the workgroup
        // stage the halo tile: two lanes per position, 8 channels each
        for (int e = threadIdx.x; e < 2 * HPOS; e += CWG) {
            const int hp = e >> 1, hh = e & 1;
            const int hx = hp % HX, hy = (hp / HX) % HY, hz = hp / (HX * HY);
            const int xx = x0 + hx - 1, yy = y0 + hy - 1, zz = z0 + hz - 1;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (xx >= 0 && xx < W && yy >= 0 && yy < H && zz >= 0 && zz < D) {
                const __bf16* src;
                if (from_a) {
                    const int za = in.up ? zz >> 1 : zz, ya = in.up ? yy >> 1 : yy,
                              xa = in.up ? xx >> 1 : xx;
                    src = in.a + ((((int64_t)nb * Da + za) * Ha + ya) * Wa + xa) * in.ca + c0;
                } else {
                    src = in.b + ((((int64_t)nb * D + zz) * H + yy) * W + xx) * cb + (c0 - in.ca);
                }
                v = *reinterpret_cast<const uint4*>(src + 8 * hh);
            }
            *reinterpret_cast<uint4*>(&tile[hp * 16 + 8 * hh]) = v;
        }
        __syncthreads();
#pragma unroll 3
        for (int tap = 0; tap < 27; ++tap) {
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;  // halo offsets 0..2
            bf16x8 b[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t)
                b[t] = load8(wrow + ((int64_t)tap * Cout + 32 * t) * Cin + c0);
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                // x-row: z layer i, y row wv of the tile
                const int hp = ((i + dz) * HY + (wv + dy)) * HX + (row + dx);
                const bf16x8 a = load8(&tile[hp * 16 + 8 * half]);
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[i][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[t], acc[i][t], 0, 0, 0);
            }
        }
    }
    // D[8 (r/4) + 4 half + r%4][row]: x = x0 + that, channel co0 + 32 t + row
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const int z = z0 + i, y = y0 + wv;
        if (z >= D || y >= H) continue;
        const int64_t rowbase = (((int64_t)nb * D + z) * H + y) * W;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = co0 + 32 * t + row;
            const float bv = bias ? bias[co] : 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int x = x0 + 8 * (r / 4) + 4 * half + (r % 4);
                if (x >= W) continue;
                float v = acc[i][t][r] + bv;
                if (RELU) v = v > 0.f ? v : 0.f;
                Y[(rowbase + x) * Cout + co] = (__bf16)v;
            }
        }
    }
}

// The large layers: tile reuse along z, operands from LDS only.  A
// workgroup of ZW groups of four wavefronts owns ZW TZ z-layers x 4 y-rows
// x 32 x-positions and 32 output channels; wavefront w of group zg takes
// y-row w of layers zg TZ .. zg TZ + TZ - 1 (TZ accumulators).  Per chunk of
// 16 input channels the halo tile (ZW TZ + 2) x 6 x 34 and the chunk's
// weights (27 taps x 32 output channels x 16 channels) sit in LDS, and the
// next chunk's are loaded into registers (every load issued before any is
// waited for) while the current one is multiplied.  The 27 taps run as 9
// (dy, dx) pairs: the pair's three weight fragments (dz = 0, 1, 2) are read
// once, and each staged operand of halo layer hz (32 positions of row wv +
// dy, shifted by dx) is read once and multiplied into output layers hz - dz
// for all three dz: per chunk and wavefront 27 TZ matrix instructions
// against 9 (TZ + 2) + 27 operand reads.  LDS holds each operand as two planes of 8 channels
// (16 bytes per position), so the 16-byte reads of eight consecutive lanes
// cover 128 contiguous bytes (no bank conflict); the second plane is offset
// by 64 bytes so the staging writes, which alternate planes, do not
// conflict either.  The staged pieces' element offsets are computed once per
// workgroup (32-bit: the host checks that they fit).  Workgroups are dealt
// to the chip's dies in contiguous runs of tiles (XCD-aware, as the colour
// passes), so the halo rows neighbouring tiles share are served by one L2.
constexpr int NXCD_CONV = 8;

// One chunk's staged pieces into registers: input piece k from element
// offset oa[k] (channels [0, ca), tensor A) or ob[k] (tensor B) plus the
// chunk's first channel, zero where bit k of okm is clear; weight piece k
// from ow[k] plus the chunk's first channel.  Every load is issued before
// any result is used.
template <int NA, int NW>
__device__ __forceinline__ void conv_fetch(u32x4 (&pa)[NA], u32x4 (&pw)[NW], const int (&oa)[NA],
                                           const int (&ob)[NA], uint32_t okm, const int (&ow)[NW],
                                           const __bf16* abase, const __bf16* bbase,
                                           const __bf16* Wt, int ca, int c0) {
    const bool from_a = c0 < ca;  // uniform over the workgroup
    const __bf16* base = from_a ? abase + c0 : bbase + (c0 - ca);
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const u32x4 v = *reinterpret_cast<const u32x4*>(base + (from_a ? oa[k] : ob[k]));
        pa[k] = (okm >> k) & 1u ? v : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int k = 0; k < NW; ++k) pw[k] = *reinterpret_cast<const u32x4*>(Wt + ow[k] + c0);
}

template <int TZ, int ZW, bool RELU>
__global__ __launch_bounds__(CWG * ZW) __attribute__((amdgpu_waves_per_eu(2, 8))) void conv3_fwd_zp_kernel(const ConvIn in,
                                                           const __bf16* __restrict__ Wt,
                                                           const float* __restrict__ bias,
                                                           __bf16* __restrict__ Y, int N, int D,
                                                           int H, int W, int Cin, int Cout,
                                                           int64_t ntiles, int64_t per_die) {
    constexpr int NT = CWG * ZW;             // threads: ZW groups of four wavefronts
    constexpr int HZ = ZW * TZ + 2, HPOS = HZ * HY * HX;
    constexpr int PT = HPOS * 8 + 32;       // elements per plane of the input tile
    constexpr int PW = 27 * 32 * 8 + 32;    // elements per plane of the weights
    constexpr int NA = (2 * HPOS + NT - 1) / NT;
    constexpr int WQ = 27 * 32 * 2;
    constexpr int NW = (WQ + NT - 1) / NT;
    __shared__ __attribute__((aligned(16))) __bf16 tile[2 * PT];
    __shared__ __attribute__((aligned(16))) __bf16 wts[2 * PW];
    const int64_t tid = (int64_t)(blockIdx.x % NXCD_CONV) * per_die + blockIdx.x / NXCD_CONV;
    if (tid >= ntiles) return;  // whole workgroup: no barrier is skipped by part of it
    const int lane = threadIdx.x & 63, wv = (threadIdx.x >> 6) & 3, zg = threadIdx.x >> 8;
    const int row = lane & 31, half = lane >> 5;
    const int ntx = (W + TX - 1) / TX, nty = (H + TY - 1) / TY, ntz = (D + ZW * TZ - 1) / (ZW * TZ);
    const int ncot = Cout / 32;
    int64_t r = tid;
    const int x0 = (int)(r % ntx) * TX;
    r /= ntx;
    const int y0 = (int)(r % nty) * TY;
    r /= nty;
    const int co0 = (int)(r % ncot) * 32;
    r /= ncot;
    const int z0 = (int)(r % ntz) * (ZW * TZ);
    const int nb = (int)(r / ntz);
    const int cb = Cin - in.ca;
    const int Da = in.up ? D / 2 : D, Ha = in.up ? H / 2 : H, Wa = in.up ? W / 2 : W;
    const float bv = bias ? bias[co0 + row] : 0.f;  // loaded with the first chunk
    f32x16 acc[TZ];
#pragma unroll
    for (int i = 0; i < TZ; ++i) acc[i] = f32x16{};
    // each thread's staged pieces as element offsets within this molecule's
    // input (A and B) and within the weights, computed once: a chunk's fetch
    // is then one add and one load per piece; pieces outside the volume load
    // offset 0 and are replaced by zero
    const __bf16* abase = in.a + (int64_t)nb * Da * Ha * Wa * in.ca;
    const __bf16* bbase = cb > 0 ? in.b + (int64_t)nb * D * H * W * cb : abase;
    int oa[NA], ob[NA];
    uint32_t okm = 0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int e = threadIdx.x + k * NT;
        const int hp = e >> 1, hh = e & 1;
        const int hx = hp % HX, hy = (hp / HX) % HY, hz = hp / (HX * HY);
        const int xx = x0 + hx - 1, yy = y0 + hy - 1, zz = z0 + hz - 1;
        const bool ok = e < 2 * HPOS && xx >= 0 && xx < W && yy >= 0 && yy < H && zz >= 0 &&
                        zz < D;
        const int za = in.up ? zz >> 1 : zz, ya = in.up ? yy >> 1 : yy, xa = in.up ? xx >> 1 : xx;
        oa[k] = ok ? ((za * Ha + ya) * Wa + xa) * in.ca + 8 * hh : 0;
        ob[k] = ok && cb > 0 ? ((zz * H + yy) * W + xx) * cb + 8 * hh : 0;
        okm |= ok ? 1u << k : 0u;
    }
    int ow[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int e = threadIdx.x + k * NT;
        const int tap = e >> 6, co = (e >> 1) & 31, hh = e & 1;
        ow[k] = e < WQ ? (tap * Cout + co0 + co) * Cin + 8 * hh : 0;
    }
    u32x4 pa[NA], pw[NW];
    conv_fetch(pa, pw, oa, ob, okm, ow, abase, bbase, Wt, in.ca, 0);
    for (int c0 = 0; c0 < Cin; c0 += 16) {
        __syncthreads();  // the previous chunk's LDS reads are done
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < 2 * HPOS) *reinterpret_cast<u32x4*>(&tile[(e & 1) * PT + (e >> 1) * 8]) = pa[k];
        }
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < WQ) *reinterpret_cast<u32x4*>(&wts[(e & 1) * PW + (e >> 1) * 8]) = pw[k];
        }
        __syncthreads();
        if (c0 + 16 < Cin) conv_fetch(pa, pw, oa, ob, okm, ow, abase, bbase, Wt, in.ca, c0 + 16);
        const __bf16* wl = &wts[half * PW + row * 8];
        const __bf16* tl = &tile[half * PT + ((zg * TZ * HY + wv) * HX + row) * 8];
#pragma unroll
        for (int yx = 0; yx < 9; ++yx) {
            const int dy = yx / 3, dx = yx - 3 * dy;
            bf16x8 b[3];
#pragma unroll
            for (int dz = 0; dz < 3; ++dz) b[dz] = load8(wl + (dz * 9 + yx) * 32 * 8);
#pragma unroll
            for (int hz = 0; hz < HZ; ++hz) {
                const bf16x8 a = load8(tl + ((hz * HY + dy) * HX + dx) * 8);
#pragma unroll
                for (int dz = 0; dz < 3; ++dz) {
                    const int z = hz - dz;
                    if (z >= 0 && z < TZ)
                        acc[z] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[dz], acc[z], 0, 0, 0);
                }
            }
        }
    }
    // D[8 (r/4) + 4 half + r%4][row]: x = x0 + that, channel co0 + row; a
    // tile wholly inside the row stores at fixed offsets from one pointer
    const bool full_x = x0 + TX <= W;
#pragma unroll
    for (int i = 0; i < TZ; ++i) {
        const int z = z0 + zg * TZ + i, y = y0 + wv;
        if (z >= D || y >= H) continue;
        __bf16* yr = Y + ((((int64_t)nb * D + z) * H + y) * W + x0 + 4 * half) * Cout + co0 + row;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int dxq = 8 * (q / 4) + (q % 4);
            if (!full_x && x0 + 4 * half + dxq >= W) continue;
            float v = acc[i][q] + bv;
            if (RELU) v = v > 0.f ? v : 0.f;
            yr[(int64_t)dxq * Cout] = (__bf16)v;
        }
    }
}

// Weight gradient partials: for one tap, a 32 x 32 (co, ci) tile and one
// chunk of positions: part[chunk][tap][co][ci] = sum_p dY[p][co] X[p+off][ci].
// Per step a wavefront takes 16 consecutive positions: each lane loads 8
// channels of one position of dY and of the shifted X (16-byte loads),
// stores them transposed (channel-major) in the wavefront's own LDS tiles,
// and the matrix operands (8 consecutive positions per lane) come back as
// 16-byte LDS reads.  The four wavefronts take interleaved steps; their
// tiles are added in LDS in wavefront order.
constexpr int WCHUNK = 8192;  // positions per chunk
__global__ __launch_bounds__(CWG) void conv3_wgrad_kernel(const __bf16* __restrict__ X,
                                                          const __bf16* __restrict__ dY,
                                                          float* __restrict__ part, int N, int D,
                                                          int H, int W, int Cin, int Cout) {
    __shared__ float red[4][32 * 32];
    __shared__ __attribute__((aligned(16))) __bf16 sA[4][32][16];
    __shared__ __attribute__((aligned(16))) __bf16 sB[4][32][16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = lane & 31, half = lane >> 5;
    const int64_t P = (int64_t)N * D * H * W;
    const int64_t chunk = blockIdx.x;
    const int nco = Cout / 32, nci = Cin / 32;
    int t2 = blockIdx.y;
    const int cit = t2 % nci;
    t2 /= nci;
    const int cot = t2 % nco;
    const int tap = t2 / nco;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    // loader role of this lane: position j of the 16, channels 8 o .. 8 o + 7
    const int j = lane >> 2, o = lane & 3;
    f32x16 acc = f32x16{};
    const int64_t pbeg = chunk * WCHUNK;
    const int64_t pend = pbeg + WCHUNK < P ? pbeg + WCHUNK : P;
    // coordinates of this lane's position, advanced by 64 positions per step
    int n, z, y, x;
    pos_coords(pbeg + 16 * wv + j, D, H, W, n, z, y, x);
    for (int64_t g0 = pbeg + 16 * wv; g0 < pend; g0 += 64) {
        const int64_t p = g0 + j;
        uint4 va = make_uint4(0, 0, 0, 0), vb = make_uint4(0, 0, 0, 0);
        if (p < pend) {
            va = *reinterpret_cast<const uint4*>(dY + p * Cout + cot * 32 + 8 * o);
            const int zz = z + dz, yy = y + dy, xx = x + dx;
            if (zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W)
                vb = *reinterpret_cast<const uint4*>(
                    X + ((((int64_t)n * D + zz) * H + yy) * W + xx) * Cin + cit * 32 + 8 * o);
        }
        __bf16 ea[8], eb[8];
        __builtin_memcpy(ea, &va, 16);
        __builtin_memcpy(eb, &vb, 16);
        __builtin_amdgcn_wave_barrier();  // the previous step's LDS reads are done
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            sA[wv][8 * o + e][j] = ea[e];
            sB[wv][8 * o + e][j] = eb[e];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const bf16x8 a = load8(&sA[wv][row][8 * half]);
        const bf16x8 b = load8(&sB[wv][row][8 * half]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        x += 64;
        while (x >= W) {
            x -= W;
            if (++y == H) {
                y = 0;
                if (++z == D) {
                    z = 0;
                    ++n;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wv][(8 * (r / 4) + 4 * half + (r % 4)) * 32 + row] = acc[r];
    __syncthreads();
    float* out = part + ((chunk * 27 + tap) * (int64_t)Cout) * Cin;
    for (int e = threadIdx.x; e < 32 * 32; e += CWG) {
        const float v = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
        const int r_ = e / 32, c_ = e % 32;
        out[(int64_t)(cot * 32 + r_) * Cin + cit * 32 + c_] = v;
    }
}

// dW[i] = sum over chunks, in order, of part[chunk][i].
__global__ void wgrad_reduce_kernel(const float* part, int64_t nchunks, int64_t nw, float* dW) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    float s = 0.f;
    for (int64_t c = 0; c < nchunks; ++c) s += part[c * nw + i];
    dW[i] = s;
}

// Per-channel sums over positions, in chunks of RCH positions:
// partial[chunk][c] = sum_p (A ? A[p][c] : 1) (scale ? scale[p] : 1);
// 64 channels x 4 position lanes per workgroup (loads coalesced along c).
constexpr int RCH = 1024;
__global__ __launch_bounds__(256) void channel_partial_kernel(const __bf16* A, const float* scale,
                                                              int64_t P, int C, float* partial) {
    __shared__ float sh[4][64];
    const int cl = threadIdx.x & 63, pl = threadIdx.x >> 6;
    const int c = blockIdx.y * 64 + cl;
    const int64_t p0 = (int64_t)blockIdx.x * RCH;
    float s = 0.f;
    if (c < C) {
        for (int k = pl; k < RCH; k += 4) {
            const int64_t p = p0 + k;
            if (p >= P) break;
            const float v = A ? (float)A[p * C + c] : 1.f;
            s += scale ? v * scale[p] : v;
        }
    }
    sh[pl][cl] = s;
    __syncthreads();
    if (pl == 0 && c < C)
        partial[blockIdx.x * (int64_t)C + c] = ((sh[0][cl] + sh[1][cl]) + sh[2][cl]) + sh[3][cl];
}

// out[c] = sum over chunks, in order, of partial[chunk][c] (FP64 sum).
__global__ void channel_reduce_kernel(const float* partial, int64_t nch, int C, float* out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    double s = 0.0;
    for (int64_t k = 0; k < nch; ++k) s += partial[k * C + c];
    out[c] = (float)s;
}

hipError_t channel_sums(const __bf16* A, const float* scale, int64_t P, int C, float* partial,
                        float* out, hipStream_t st) {
    const int64_t nch = (P + RCH - 1) / RCH;
    hipLaunchKernelGGL(channel_partial_kernel, dim3((unsigned)nch, (unsigned)((C + 63) / 64)),
                       dim3(256), 0, st, A, scale, P, C, partial);
    hipLaunchKernelGGL(channel_reduce_kernel, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, st,
                       partial, nch, C, out);
    return hipGetLastError();
}

size_t channel_sums_bytes(int64_t P, int C) {
    return sizeof(float) * (size_t)((P + RCH - 1) / RCH) * (size_t)C;
}

// BF16 forward weights and the spatially flipped, channel-transposed
// weights of the data gradient, from the FP32 master copy (27, Cout, Cin).
__global__ void prep_weights_kernel(const float* W32, int Cout, int Cin, __bf16* Wf, __bf16* Wb) {
    const int64_t n = 27LL * Cout * Cin;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ci = (int)(i % Cin);
    const int64_t r = i / Cin;
    const int co = (int)(r % Cout);
    const int tap = (int)(r / Cout);
    const __bf16 v = (__bf16)W32[i];
    Wf[i] = v;
    Wb[((int64_t)(26 - tap) * Cin + ci) * Cout + co] = v;
}

// dPre = dY where Y > 0 (the ReLU was applied to the pre-activation).
__global__ void relu_bwd_kernel(const __bf16* Y, const __bf16* dY, __bf16* dPre, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dPre[i] = (float)Y[i] > 0.f ? dY[i] : (__bf16)0.f;
}

// 2x2x2 average pooling and its adjoint (even sizes).
// Eight channels per thread (C % 8 == 0): 16-byte loads and stores; the
// eight inputs of each output are summed in the same order as below.
__global__ void pool2_fwd_vec_kernel(const __bf16* X, __bf16* Y, int N, int D, int H, int W, int C) {
    const int d = D / 2, h = H / 2, w = W / 2, C8 = C / 8;
    const int64_t n_out = (int64_t)N * d * h * w * C8;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    const int c = (int)(i % C8) * 8;
    int n, z, y, x;
    pos_coords(i / C8, d, h, w, n, z, y, x);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < 8; ++k) {
        const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
        const bf16x8 v = load8(X + ((((int64_t)n * D + zz) * H + yy) * W + xx) * C + c);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] += (float)v[j];
    }
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = (__bf16)(0.125f * s[j]);
    *reinterpret_cast<bf16x8*>(Y + (i / C8) * C + c) = o;
}
__global__ void pool2_fwd_kernel(const __bf16* X, __bf16* Y, int N, int D, int H, int W, int C) {
    const int d = D / 2, h = H / 2, w = W / 2;
    const int64_t n_out = (int64_t)N * d * h * w * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    const int c = (int)(i % C);
    int n, z, y, x;
    pos_coords(i / C, d, h, w, n, z, y, x);
    float s = 0.f;
    for (int k = 0; k < 8; ++k) {
        const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
        s += (float)X[((((int64_t)n * D + zz) * H + yy) * W + xx) * C + c];
    }
    Y[i] = (__bf16)(0.125f * s);
}
__global__ void pool2_bwd_kernel(const __bf16* dY, __bf16* dX, int N, int D, int H, int W, int C) {
    const int64_t n_in = (int64_t)N * D * H * W * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_in) return;
    const int c = (int)(i % C);
    int n, z, y, x;
    pos_coords(i / C, D, H, W, n, z, y, x);
    const int d = D / 2, h = H / 2, w = W / 2;
    dX[i] = (__bf16)(0.125f * (float)dY[((((int64_t)n * d + z / 2) * h + y / 2) * w + x / 2) * C + c]);
}

// Nearest 2x upsampling (X: half size) and its adjoint.
__global__ void up2_fwd_kernel(const __bf16* X, __bf16* Y, int N, int D, int H, int W, int C) {
    const int64_t n_out = (int64_t)N * D * H * W * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    const int c = (int)(i % C);
    int n, z, y, x;
    pos_coords(i / C, D, H, W, n, z, y, x);
    const int d = D / 2, h = H / 2, w = W / 2;
    Y[i] = X[((((int64_t)n * d + z / 2) * h + y / 2) * w + x / 2) * C + c];
}
__global__ void up2_bwd_kernel(const __bf16* dY, __bf16* dX, int N, int D, int H, int W, int C) {
    const int d = D / 2, h = H / 2, w = W / 2;
    const int64_t n_small = (int64_t)N * d * h * w * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_small) return;
    const int c = (int)(i % C);
    int n, z, y, x;
    pos_coords(i / C, d, h, w, n, z, y, x);
    float s = 0.f;
    for (int k = 0; k < 8; ++k) {
        const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
        s += (float)dY[((((int64_t)n * D + zz) * H + yy) * W + xx) * C + c];
    }
    dX[i] = (__bf16)s;
}

// Channel concatenation Y = [A | B] and its adjoint (dA = dY[:, :Ca],
// dB (+)= dY[:, Ca:]).
__global__ void concat_kernel(const __bf16* A, int Ca, const __bf16* B, int Cb, __bf16* Y,
                              int64_t P) {
    const int C = Ca + Cb;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * C) return;
    const int64_t p = i / C;
    const int c = (int)(i % C);
    Y[i] = c < Ca ? A[p * Ca + c] : B[p * Cb + (c - Ca)];
}
__global__ void split_kernel(const __bf16* dY, int Ca, int Cb, __bf16* dA, __bf16* dB,
                             int accumulate_b, int64_t P) {
    const int C = Ca + Cb;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * C) return;
    const int64_t p = i / C;
    const int c = (int)(i % C);
    if (c < Ca) {
        dA[p * Ca + c] = dY[i];
    } else {
        const int64_t j = p * Cb + (c - Ca);
        dB[j] = accumulate_b ? (__bf16)((float)dB[j] + (float)dY[i]) : dY[i];
    }
}

// Y = A + B (BF16, added in FP32).
__global__ void add_kernel(const __bf16* A, const __bf16* B, __bf16* Y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Y[i] = (__bf16)((float)A[i] + (float)B[i]);
}

// 1x1x1 head: logits[p] = w . X[p] + b (FP32), and its adjoint.
// One position per thread; channels added in order (16-byte loads when
// C % 8 == 0).
__global__ void head_fwd_kernel(const __bf16* X, const float* w, const float* b, float* logits,
                                int64_t P, int C) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    float s = b[0];
    if (C % 8 == 0) {
        for (int c = 0; c < C; c += 8) {
            const bf16x8 v = load8(X + p * C + c);
#pragma unroll
            for (int j = 0; j < 8; ++j) s += w[c + j] * (float)v[j];
        }
    } else {
        for (int c = 0; c < C; ++c) s += w[c] * (float)X[p * C + c];
    }
    logits[p] = s;
}
__global__ void head_bwd_x_kernel(const float* dlogit, const float* w, __bf16* dX, int64_t P,
                                  int C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * C) return;
    dX[i] = (__bf16)(dlogit[i / C] * w[i % C]);
}
// Weighted binary cross-entropy with logits against labels (target 1 for
// solute, phi = -1), mean over cells: per-block FP64 partial losses and the
// gradient dlogit = w (sigmoid(l) - t) / P.
__global__ __launch_bounds__(256) void bce_kernel(const float* logits, const int8_t* labels,
                                                  int64_t P, float pos_weight, float* dlogit,
                                                  double* partial) {
    __shared__ double sh[256];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += stride) {
        const float l = logits[p];
        const float t = labels[p] < 0 ? 1.f : 0.f;
        const float wt = t > 0.f ? pos_weight : 1.f;
        // log(1 + exp(-|l|)) + max(l, 0) - l t
        const float sp = log1pf(expf(-fabsf(l))) + fmaxf(l, 0.f) - l * t;
        s += (double)(wt * sp);
        const float sg = 1.f / (1.f + expf(-l));
        dlogit[p] = wt * (sg - t) / (float)P;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s / (double)P;
}

// Adam on FP32 master parameters.
__global__ void adam_kernel(float* w, const float* g, float* m, float* v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Input features on the cell grid (n^3 cells of edge h, first centre x0):
// channel 0 = sum_i exp(-|x - r_i|^2 / (2 s_i^2)), channel 1 = the same
// weighted by q_i, with s_i = sigma_i / 2, cut at 4 s_i; channels 2..C-1 = 0.
// A workgroup takes an 8 x 8 x 4 brick of cells; per tile of 256 atoms it
// keeps, in atom order, those whose distance to the brick's box of cell
// centres is below the cut (with a margin for rounding), and every cell then
// applies the exact cut to those: the same terms, summed in the same order,
// as a loop over all atoms.
constexpr int FBX = 8, FBY = 8, FBZ = 4;
__global__ __launch_bounds__(256) void featurize_kernel(const double4* pos, const double* sigma,
                                                        const double* q, int64_t na, int n,
                                                        double h, double x0, double y0, double z0,
                                                        int C, __bf16* X) {
    __shared__ float4 sa[256];
    __shared__ float2 sp[256];
    __shared__ int wcnt[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int nbx = (n + FBX - 1) / FBX, nby = (n + FBY - 1) / FBY;
    int b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby;
    const int bz = b / nby;
    const int x = bx * FBX + (t % FBX), y = by * FBY + ((t / FBX) % FBY), z = bz * FBZ + t / (FBX * FBY);
    const float cx = (float)(x0 + x * h), cy = (float)(y0 + y * h), cz = (float)(z0 + z * h);
    // box of the brick's cell centres (clipped to the grid)
    const int xe = min(bx * FBX + FBX - 1, n - 1), ye = min(by * FBY + FBY - 1, n - 1),
              ze = min(bz * FBZ + FBZ - 1, n - 1);
    const float lx = (float)(x0 + bx * FBX * h), hx = (float)(x0 + xe * h);
    const float ly = (float)(y0 + by * FBY * h), hy = (float)(y0 + ye * h);
    const float lz = (float)(z0 + bz * FBZ * h), hz = (float)(z0 + ze * h);
    float d0 = 0.f, d1 = 0.f;
    for (int64_t base = 0; base < na; base += 256) {
        const int64_t a = base + t;
        bool keep = false;
        float4 pa = make_float4(0.f, 0.f, 0.f, 0.f);
        float2 pq = make_float2(0.f, 0.f);
        if (a < na) {
            const double4 p = pos[a];
            const float s = (float)(0.5 * sigma[a]);
            pa = make_float4((float)p.x, (float)p.y, (float)p.z, 1.f / (2.f * s * s));
            pq = make_float2((float)q[a], 16.f * s * s);
            const float ex = fmaxf(fmaxf(lx - pa.x, pa.x - hx), 0.f);
            const float ey = fmaxf(fmaxf(ly - pa.y, pa.y - hy), 0.f);
            const float ez = fmaxf(fmaxf(lz - pa.z, pa.z - hz), 0.f);
            keep = ex * ex + ey * ey + ez * ez < 1.001f * pq.y;
        }
        const uint64_t bal = __ballot(keep);
        __syncthreads();  // the previous tile has been read
        if (lane == 0) wcnt[wv] = __popcll(bal);
        __syncthreads();
        int off = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            off += k < wv ? wcnt[k] : 0;
            tot += wcnt[k];
        }
        if (keep) {
            const int at = off + __popcll(bal & ((1ull << lane) - 1ull));
            sa[at] = pa;
            sp[at] = pq;
        }
        __syncthreads();
        for (int k = 0; k < tot; ++k) {
            const float4 p = sa[k];
            const float dx = cx - p.x, dy = cy - p.y, dz = cz - p.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < sp[k].y) {
                const float e = __expf(-r2 * p.w);
                d0 += e;
                d1 += sp[k].x * e;
            }
        }
    }
    if (x >= n || y >= n || z >= n) return;
    const int64_t cell = (int64_t)x + (int64_t)n * (y + (int64_t)n * z);
    for (int c = 0; c < C; ++c) X[cell * C + c] = (__bf16)(c == 0 ? d0 : (c == 1 ? d1 : 0.f));
}

inline unsigned nblk(int64_t n, int wg) { return (unsigned)((n + wg - 1) / wg); }

}  // namespace
}  // namespace nn
}  // namespace vesis

// ------------------------------------------------------------------ C ABI

#include <mutex>

#include "vesis_nn.h"

using namespace vesis::nn;

// Scratch of the allocation-free head gradient (vesis_nn_head_bwd_noalloc):
// the per-chunk channel partial sums, one float per (chunk of 1024
// positions, channel), at most HEAD_SCRATCH_FLOATS of them (1 MiB).  Each GPU
// the library runs on holds its own copy until the process ends; host code
// reaches it only through the device address looked up per device below.
constexpr int64_t HEAD_SCRATCH_FLOATS = 262144;
static __device__ __align__(256) float scratch[HEAD_SCRATCH_FLOATS];

namespace {
inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
inline int status(hipError_t e) { return e == hipSuccess ? 0 : VESIS_NN_E_DEVICE; }
inline const __bf16* B(const void* p) { return static_cast<const __bf16*>(p); }
inline __bf16* Bm(void* p) { return static_cast<__bf16*>(p); }
bool dims_ok(int N, int D, int H, int W) { return N > 0 && D > 0 && H > 0 && W > 0; }

// Device address of the current GPU's copy of `scratch`, looked up once per
// device (with that device current) and kept.
constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
float* scratch_ptr[SCRATCH_DEVICES] = {};

int head_scratch(float** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_DEVICES)
        return VESIS_NN_E_DEVICE;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return VESIS_NN_E_DEVICE;
        scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = scratch_ptr[dev];
    return 0;
}

// The head's adjoint with its channel partials in ws (at least
// channel_sums_bytes(p, c) bytes): dx, then dw, then db (which reuses ws
// after the dw sums have read it: same stream).
int head_bwd(hipStream_t st, const float* dlogit, const void* x, const float* w, void* dx,
             float* dw, float* db, float* ws, int64_t p, int c) {
    hipLaunchKernelGGL(head_bwd_x_kernel, dim3(nblk(p * c, 256)), dim3(256), 0, st, dlogit, w,
                       Bm(dx), p, c);
    if (channel_sums(B(x), dlogit, p, c, ws, dw, st) != hipSuccess ||
        channel_sums(nullptr, dlogit, p, 1, ws, db, st) != hipSuccess)
        return VESIS_NN_E_DEVICE;
    return status(hipGetLastError());
}

// Layers with at least 256 tiles of 4 z-layers take the z-reuse kernel
// (when its 32-bit element offsets fit: the inputs of one molecule and the
// weights each below 2^31 elements); smaller ones take
// conv3_fwd_lds_kernel<1, 1> (one z-layer per workgroup: more, smaller
// workgroups).
template <int TZ, int ZW>
void launch_conv3_zp(hipStream_t st, const ConvIn& in, const void* w, const float* bias, void* y,
                     int n, int d, int h, int wd, int cin, int cout, int relu) {
    const int64_t ntiles = (int64_t)((wd + TX - 1) / TX) * ((h + TY - 1) / TY) * (cout / 32) *
                           ((d + ZW * TZ - 1) / (ZW * TZ)) * n;
    const int64_t per = (ntiles + NXCD_CONV - 1) / NXCD_CONV;
    const dim3 grid((unsigned)(per * NXCD_CONV));
    if (relu)
        hipLaunchKernelGGL((conv3_fwd_zp_kernel<TZ, ZW, true>), grid, dim3(CWG * ZW), 0, st, in, B(w), bias, Bm(y), n, d, h, wd, cin, cout, ntiles, per);
    else
        hipLaunchKernelGGL((conv3_fwd_zp_kernel<TZ, ZW, false>), grid, dim3(CWG * ZW), 0, st, in, B(w), bias, Bm(y), n, d, h, wd, cin, cout, ntiles, per);
}

void launch_conv3_lds(hipStream_t st, const ConvIn& in, const void* w, const float* bias, void* y,
                      int n, int d, int h, int wd, int cin, int cout, int relu) {
    const unsigned nt_xy = (unsigned)(((wd + TX - 1) / TX) * ((h + TY - 1) / TY));
    const int64_t big = (int64_t)nt_xy * (cout / 32) * ((d + 3) / 4) * n;
    const int64_t lim = (int64_t)1 << 31;
    const int64_t pos = (int64_t)d * h * wd;
    const int64_t apos = in.up ? (int64_t)(d / 2) * (h / 2) * (wd / 2) : pos;
    const bool fits = apos * in.ca < lim && pos * (cin - in.ca) < lim && 27LL * cout * cin < lim;
    if (big >= 256 && fits) {
        // 2 z-layers per wavefront: 126 registers, four wavefronts per SIMD;
        // the tile is shared by two groups of four wavefronts (4 z-layers),
        // or by four (8 z-layers) when the chunks are many (each chunk's
        // staging then serves twice the outputs)
        if (cin <= 64)
            launch_conv3_zp<2, 2>(st, in, w, bias, y, n, d, h, wd, cin, cout, relu);
        else
            launch_conv3_zp<2, 4>(st, in, w, bias, y, n, d, h, wd, cin, cout, relu);
        return;
    }
    const dim3 grid(nt_xy, (unsigned)(cout / 32), (unsigned)(n * d));
    if (relu)
        hipLaunchKernelGGL((conv3_fwd_lds_kernel<1, 1, true>), grid, dim3(CWG), 0, st, in, B(w), bias, Bm(y), n, d, h, wd, cin, cout);
    else
        hipLaunchKernelGGL((conv3_fwd_lds_kernel<1, 1, false>), grid, dim3(CWG), 0, st, in, B(w), bias, Bm(y), n, d, h, wd, cin, cout);
}
}  // namespace

extern "C" {

int vesis_nn_conv3_fwd(void* stream, const void* x, const void* w, const float* bias, void* y,
                       int n, int d, int h, int wd, int cin, int cout, int relu) {
    if (!x || !w || !y || !dims_ok(n, d, h, wd) || cin <= 0 || cin % 16 || cout <= 0 || cout % 32)
        return VESIS_NN_E_ARG;
    const int64_t P = (int64_t)n * d * h * wd;
    const bool two = cout % 64 == 0;
    if (wd >= TX / 2) {
        launch_conv3_lds(S(stream), ConvIn{B(x), cin, 0, nullptr}, w, bias, y, n, d, h, wd, cin,
                         cout, relu);
        return status(hipGetLastError());
    }
    const dim3 grid(nblk(P, 128), (unsigned)(cout / (two ? 64 : 32)));
    if (two && relu)
        hipLaunchKernelGGL((conv3_fwd_kernel<2, true>), grid, dim3(CWG), 0, S(stream), B(x), B(w), bias, Bm(y), n, d, h, wd, cin, cout);
    else if (two)
        hipLaunchKernelGGL((conv3_fwd_kernel<2, false>), grid, dim3(CWG), 0, S(stream), B(x), B(w), bias, Bm(y), n, d, h, wd, cin, cout);
    else if (relu)
        hipLaunchKernelGGL((conv3_fwd_kernel<1, true>), grid, dim3(CWG), 0, S(stream), B(x), B(w), bias, Bm(y), n, d, h, wd, cin, cout);
    else
        hipLaunchKernelGGL((conv3_fwd_kernel<1, false>), grid, dim3(CWG), 0, S(stream), B(x), B(w), bias, Bm(y), n, d, h, wd, cin, cout);
    return status(hipGetLastError());
}

int vesis_nn_conv3_fwd_upcat(void* stream, const void* a, int ca, const void* b, int cb,
                             const void* w, const float* bias, void* y, int n, int d, int h,
                             int wd, int cout, int relu) {
    if (!a || !b || !w || !y || !dims_ok(n, d, h, wd) || d % 2 || h % 2 || wd % 2 ||
        wd < TX / 2 || ca <= 0 || ca % 16 || cb <= 0 || cb % 16 || cout <= 0 || cout % 32)
        return VESIS_NN_E_ARG;
    launch_conv3_lds(S(stream), ConvIn{B(a), ca, 1, B(b)}, w, bias, y, n, d, h, wd, ca + cb,
                     cout, relu);
    return status(hipGetLastError());
}

int vesis_nn_wgrad_workspace(int n, int d, int h, int wd, int cin, int cout, size_t* bytes) {
    if (!bytes || !dims_ok(n, d, h, wd) || cin % 32 || cout % 32) return VESIS_NN_E_ARG;
    const int64_t P = (int64_t)n * d * h * wd;
    const size_t wpart = sizeof(float) * (size_t)((P + WCHUNK - 1) / WCHUNK) * 27 * cout * cin;
    const size_t bpart = channel_sums_bytes(P, cout);
    *bytes = wpart + bpart + 256;
    return 0;
}

int vesis_nn_conv3_wgrad(void* stream, const void* x, const void* dy, float* dw, float* db,
                         float* ws, size_t ws_bytes, int n, int d, int h, int wd, int cin,
                         int cout) {
    size_t need = 0;
    if (!x || !dy || !dw || !ws || vesis_nn_wgrad_workspace(n, d, h, wd, cin, cout, &need) != 0)
        return VESIS_NN_E_ARG;
    if (ws_bytes < need) return VESIS_NN_E_ARG;
    const int64_t P = (int64_t)n * d * h * wd;
    const int64_t nch = (P + WCHUNK - 1) / WCHUNK;
    hipLaunchKernelGGL(conv3_wgrad_kernel, dim3((unsigned)nch, (unsigned)(27 * (cout / 32) * (cin / 32))),
                       dim3(CWG), 0, S(stream), B(x), B(dy), ws, n, d, h, wd, cin, cout);
    const int64_t nw = 27LL * cout * cin;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(nblk(nw, 256)), dim3(256), 0, S(stream), ws, nch, nw, dw);
    if (db) {
        // bias partials after the weight partials (256-byte aligned)
        const size_t off = (sizeof(float) * (size_t)nch * nw + 255) / 256 * 256 / sizeof(float);
        if (channel_sums(B(dy), nullptr, P, cout, ws + off, db, S(stream)) != hipSuccess)
            return VESIS_NN_E_DEVICE;
    }
    return status(hipGetLastError());
}

int vesis_nn_prep_weights(void* stream, const float* w32, int cout, int cin, void* wf, void* wb) {
    if (!w32 || !wf || !wb || cout <= 0 || cin <= 0) return VESIS_NN_E_ARG;
    const int64_t n = 27LL * cout * cin;
    hipLaunchKernelGGL(prep_weights_kernel, dim3(nblk(n, 256)), dim3(256), 0, S(stream), w32, cout, cin, Bm(wf), Bm(wb));
    return status(hipGetLastError());
}

int vesis_nn_relu_bwd(void* stream, const void* y, const void* dy, void* dpre, int64_t count) {
    if (!y || !dy || !dpre || count < 0) return VESIS_NN_E_ARG;
    if (count == 0) return 0;
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(nblk(count, 256)), dim3(256), 0, S(stream), B(y), B(dy), Bm(dpre), count);
    return status(hipGetLastError());
}

int vesis_nn_pool2(void* stream, const void* x, void* y, int n, int d, int h, int wd, int c, int backward) {
    if (!x || !y || !dims_ok(n, d, h, wd) || c <= 0 || d % 2 || h % 2 || wd % 2) return VESIS_NN_E_ARG;
    if (backward) {
        const int64_t cnt = (int64_t)n * d * h * wd * c;
        hipLaunchKernelGGL(pool2_bwd_kernel, dim3(nblk(cnt, 256)), dim3(256), 0, S(stream), B(x), Bm(y), n, d, h, wd, c);
    } else {
        const int64_t cnt = (int64_t)n * (d / 2) * (h / 2) * (wd / 2) * c;
        if (c % 8 == 0)
            hipLaunchKernelGGL(pool2_fwd_vec_kernel, dim3(nblk(cnt / 8, 256)), dim3(256), 0, S(stream), B(x), Bm(y), n, d, h, wd, c);
        else
            hipLaunchKernelGGL(pool2_fwd_kernel, dim3(nblk(cnt, 256)), dim3(256), 0, S(stream), B(x), Bm(y), n, d, h, wd, c);
    }
    return status(hipGetLastError());
}

int vesis_nn_up2(void* stream, const void* x, void* y, int n, int d, int h, int wd, int c, int backward) {
    if (!x || !y || !dims_ok(n, d, h, wd) || c <= 0 || d % 2 || h % 2 || wd % 2) return VESIS_NN_E_ARG;
    if (backward) {
        const int64_t cnt = (int64_t)n * (d / 2) * (h / 2) * (wd / 2) * c;
        hipLaunchKernelGGL(up2_bwd_kernel, dim3(nblk(cnt, 256)), dim3(256), 0, S(stream), B(x), Bm(y), n, d, h, wd, c);
    } else {
        const int64_t cnt = (int64_t)n * d * h * wd * c;
        hipLaunchKernelGGL(up2_fwd_kernel, dim3(nblk(cnt, 256)), dim3(256), 0, S(stream), B(x), Bm(y), n, d, h, wd, c);
    }
    return status(hipGetLastError());
}

int vesis_nn_concat(void* stream, const void* a, int ca, const void* b, int cb, void* y, int64_t p) {
    if (!a || !b || !y || ca <= 0 || cb <= 0 || p <= 0) return VESIS_NN_E_ARG;
    hipLaunchKernelGGL(concat_kernel, dim3(nblk(p * (ca + cb), 256)), dim3(256), 0, S(stream), B(a), ca, B(b), cb, Bm(y), p);
    return status(hipGetLastError());
}

int vesis_nn_split(void* stream, const void* dy, int ca, int cb, void* da, void* db,
                   int accumulate_b, int64_t p) {
    if (!dy || !da || !db || ca <= 0 || cb <= 0 || p <= 0) return VESIS_NN_E_ARG;
    hipLaunchKernelGGL(split_kernel, dim3(nblk(p * (ca + cb), 256)), dim3(256), 0, S(stream), B(dy), ca, cb, Bm(da), Bm(db), accumulate_b, p);
    return status(hipGetLastError());
}

int vesis_nn_add(void* stream, const void* a, const void* b, void* y, int64_t count) {
    if (!a || !b || !y || count < 0) return VESIS_NN_E_ARG;
    if (count == 0) return 0;
    hipLaunchKernelGGL(add_kernel, dim3(nblk(count, 256)), dim3(256), 0, S(stream), B(a), B(b), Bm(y), count);
    return status(hipGetLastError());
}

int vesis_nn_head_fwd(void* stream, const void* x, const float* w, const float* b, float* logits,
                      int64_t p, int c) {
    if (!x || !w || !b || !logits || p <= 0 || c <= 0) return VESIS_NN_E_ARG;
    hipLaunchKernelGGL(head_fwd_kernel, dim3(nblk(p, 256)), dim3(256), 0, S(stream), B(x), w, b, logits, p, c);
    return status(hipGetLastError());
}

int vesis_nn_head_bwd(void* stream, const float* dlogit, const void* x, const float* w, void* dx,
                      float* dw, float* db, float* ws, size_t ws_bytes, int64_t p, int c) {
    if (!dlogit || !x || !w || !dx || !dw || !db || !ws || p <= 0 || c <= 0) return VESIS_NN_E_ARG;
    if (ws_bytes < channel_sums_bytes(p, c)) return VESIS_NN_E_ARG;
    return head_bwd(S(stream), dlogit, x, w, dx, dw, db, ws, p, c);
}

int vesis_nn_head_bwd_noalloc(void* stream, const float* dlogit, const void* x, const float* w,
                              void* dx, float* dw, float* db, int64_t p, int c) {
    if (!dlogit || !x || !w || !dx || !dw || !db || p <= 0 || c <= 0) return VESIS_NN_E_ARG;
    if (channel_sums_bytes(p, c) > sizeof(float) * (size_t)HEAD_SCRATCH_FLOATS)
        return VESIS_NN_E_SCRATCH;
    float* ws = nullptr;
    const int rc = head_scratch(&ws);
    if (rc != 0) return rc;
    return head_bwd(S(stream), dlogit, x, w, dx, dw, db, ws, p, c);
}

int vesis_nn_bce(void* stream, const float* logits, const int8_t* labels, int64_t p,
                 float pos_weight, float* dlogit, double* partial, int nblocks, double* loss) {
    if (!logits || !labels || !dlogit || !partial || !loss || p <= 0 || nblocks < 1 || nblocks > 4096)
        return VESIS_NN_E_ARG;
    hipLaunchKernelGGL(bce_kernel, dim3((unsigned)nblocks), dim3(256), 0, S(stream), logits, labels, p, pos_weight, dlogit, partial);
    hipLaunchKernelGGL((vesis::reduce_partials<double, 1>), dim3(1), dim3(vesis::RED_WG), 0, S(stream), partial, nblocks, loss);
    return status(hipGetLastError());
}

int vesis_nn_adam(void* stream, float* w, const float* g, float* m, float* v, int64_t count,
                  float lr, float b1, float b2, float eps, int step) {
    if (!w || !g || !m || !v || count <= 0 || step < 1) return VESIS_NN_E_ARG;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(count, 256)), dim3(256), 0, S(stream), w, g, m, v, count, lr, b1, b2, eps, c1, c2);
    return status(hipGetLastError());
}

int vesis_nn_featurize(void* stream, const double* pos4, const double* sigma, const double* q,
                       int64_t na, int n, double h, const double* center, int c, void* x) {
    if (!pos4 || !sigma || !q || !center || !x || na < 0 || n <= 0 || c < 2) return VESIS_NN_E_ARG;
    const double L = 0.5 * n * h;
    const unsigned nbricks = (unsigned)(((n + FBX - 1) / FBX) * ((n + FBY - 1) / FBY) * ((n + FBZ - 1) / FBZ));
    hipLaunchKernelGGL(featurize_kernel, dim3(nbricks), dim3(256), 0, S(stream),
                       reinterpret_cast<const double4*>(pos4), sigma, q, na, n, h,
                       center[0] - L + 0.5 * h, center[1] - L + 0.5 * h, center[2] - L + 0.5 * h, c, Bm(x));
    return status(hipGetLastError());
}

}  // extern "C"
