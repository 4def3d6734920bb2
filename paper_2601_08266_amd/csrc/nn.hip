// Learned warm start: 3x3x3 convolutions on the node lattice with BF16 operands
// and FP32 accumulation on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16),
// plus the small kernels of training (loss, bias gradient, Adam) and the
// packing of solver fields into network channels.
//
// Layouts: activations channels-last [V][C] (C a multiple of 32, voxel v =
// i + nx (j + ny k)); weights [27][Cout][Cin] with tap = dx + 3 (dy + 3 dz)
// reading the neighbour at offset (dx - 1, dy - 1, dz - 1); zero padding.
//
// Forward / data gradient (implicit GEMM): a block owns a brick of 8 x 8 x 4 voxels
// x 64 output channels, each wave a 64-voxel z-slice of it x 64 channels (16
// accumulator tiles).  Per 32-channel input chunk the brick's halo is staged in
// LDS once and the 27 taps read shifted input fragments from it; each tap's
// weights are staged in LDS once per block (one load per thread, fetched a tap
// ahead) and each weight fragment feeds 4 MFMAs, each input fragment 4.  The
// products are weights x inputs, so a lane ends with 4 consecutive channels of
// one voxel.  The data gradient is the same kernel on flipped, transposed
// weights, with the ReLU mask of the previous layer applied in the epilogue.
// Weight gradient (split K): block (voxel range, tap) stages 64 voxels of dY
// and of the shifted input, transposed, in LDS and accumulates the 64x64 tap
// block with 16 MFMA tiles; the 27 tap blocks of a range run together on one
// XCD; ranges are summed in a fixed order afterwards (deterministic).
#include "nn.hpp"
#include "profile.hpp"

namespace fsi {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf8 load8(const uint16_t *p)
{
    return *reinterpret_cast<const bf8 *>(p);
}

__device__ __forceinline__ bf8 zero8()
{
    const uint4 z = make_uint4(0, 0, 0, 0);
    return __builtin_bit_cast(bf8, z);
}

// ---------------------------------------------------------------- forward / dgrad
// A block owns a brick of 8 x 8 x 4 voxels and 64 output channels; wave w the z-slice w of
// the brick, as four 16-voxel M tiles (8 x 2 voxel patches: rows y = 2m, 2m + 1).  Per
// 32-channel input chunk the block stages the brick's halo (10 x 10 x 6 voxels, zero outside
// the grid) in LDS once; the 27 taps then read their shifted A fragments from it at offsets
// fixed at compile time, so the tap loop has no address or bounds arithmetic.  The weight
// fragments (B) come straight from memory (a layer's weights stay in L2), two taps ahead.
constexpr int CF_BX = 8, CF_BY = 8, CF_BZ = 4;
constexpr int CF_HX = CF_BX + 2, CF_HY = CF_BY + 2, CF_HZ = CF_BZ + 2;
constexpr int CF_HV = CF_HX * CF_HY * CF_HZ;   // halo voxels (600)
constexpr int CF_RS = 32;                      // LDS row (bf16) of a halo voxel or a weight row: 64 bytes,
                                               // its four 16-byte parts XOR-swizzled (cf_hslot, cf_wslot)
constexpr int CF_PIECES = CF_HV * 4;           // 16-byte pieces of a staged chunk
constexpr int CF_PPT = (CF_PIECES + 255) / 256;

// LDS bank spreading: the 16-byte part `part` of halo voxel row (halo x = hx) and of weight row
// i sits in slot part ^ g.  With these g the fragment reads (16 lanes: an 8 x 2 voxel patch at any
// shift, or 16 consecutive weight rows) and the staging writes touch every bank once, both with
// 32 banks per 8 lanes and with 64 banks per 16 lanes.
__device__ __forceinline__ int cf_hslot(int part, int hx) { return part ^ ((hx >> 1) & 3); }
__device__ __forceinline__ int cf_wslot(int part, int i) { return part ^ (((i >> 1) ^ (i >> 2)) & 3); }

// Buffer loads of 16 bytes: the resource (base and byte size) in SGPRs, the lane's offset in
// a VGPR, the uniform part in an SGPR; an offset at or past the size reads zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t cf_rsrc(const void *base, int64_t bytes)
{
    const int32_t n = bytes > (int64_t)0x7fffffff ? 0x7fffffff : (int32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, n, 0x00020000);
}
__device__ __forceinline__ bf8 cf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(bf8, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
constexpr uint32_t CF_OOB = 0x80000000u;   // a lane offset past every resource: the load reads zeros

// Block b -> brick: blocks are dealt to the 8 XCDs round-robin, each XCD gets a contiguous
// range of bricks (x fastest), so bricks sharing halo voxels mostly run under one L2.
__device__ __forceinline__ uint32_t cf_brick(uint32_t b, uint32_t nb)
{
    const uint32_t q = nb >> 3, r = nb & 7u, xcd = b & 7u, idx = b >> 3;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// X: [V][cin] bf16 with V * cin * 2 < 2^31 bytes (checked by the launcher); W: [27][cout][cin].
__global__ __launch_bounds__(256, 3) void conv_fwd_k(int nx, int ny, int nz, int cin, int cout,
                                                     const uint16_t *__restrict__ X,
                                                     const uint16_t *__restrict__ W,
                                                     const float *__restrict__ bias, int relu,
                                                     const uint16_t *__restrict__ gate,
                                                     uint16_t *__restrict__ Ybf,
                                                     float *__restrict__ Yf)
{
    // the brick's input halo for one 32-channel chunk, and three taps' 64 x 32 weights (buffer
    // dx for the taps of x shift dx)
    __shared__ __attribute__((aligned(16))) uint16_t sH[CF_HV * CF_RS];
    __shared__ __attribute__((aligned(16))) uint16_t sW[3][64 * CF_RS];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int nbx = (nx + CF_BX - 1) / CF_BX, nby = (ny + CF_BY - 1) / CF_BY;
    const uint32_t brick = cf_brick(blockIdx.x, gridDim.x);
    const uint32_t bxy = brick / (uint32_t)nbx;
    const int bx = (int)(brick - bxy * (uint32_t)nbx), by = (int)(bxy % (uint32_t)nby), bz = (int)(bxy / (uint32_t)nby);
    const int co0 = blockIdx.y * 64;
    const int ntiles = (cout - co0) >= 64 ? 4 : (cout - co0) / 16;
    const int64_t V = (int64_t)nx * ny * nz;
    const __amdgpu_buffer_rsrc_t rX = cf_rsrc(X, V * cin * 2);
    const __amdgpu_buffer_rsrc_t rW = cf_rsrc(W, (int64_t)27 * cout * cin * 2);
    // this lane's A row: voxel (lane & 7, (lane >> 3) & 1) of an 8 x 2 patch, 8 channels
    // 8 (lane >> 4) .. + 7 (part lane >> 4), whose slot depends on the tap's x shift dx through the halo x
    const int arow = ((lane & 7) + CF_HX * ((lane >> 3) & 1) + CF_HX * CF_HY * w) * CF_RS;
    int abase[3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) abase[dx] = arow + 8 * cf_hslot(lane >> 4, (lane & 7) + dx);
    // this lane's B column in LDS: output channel 16 q + (lane & 15), part lane >> 4
    const int bbase = (lane & 15) * CF_RS + 8 * cf_wslot(lane >> 4, lane & 15);
    // staging of a tap's weights: thread t brings 8 input channels (t & 3) of output channel t >> 2
    const int sco = t >> 2, spart = t & 3;
    const int sslot = sco * CF_RS + 8 * cf_wslot(spart, sco);
    const bool sval = co0 + sco < cout;
    const uint32_t svoff = sval ? (uint32_t)(((co0 + sco) * cin + 8 * spart) * 2) : CF_OOB;
    auto fetch_w = [&](int tap, int c0) { return cf_load(rW, svoff, (uint32_t)((tap * cout * cin + c0) * 2)); };
    f4 acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[m][q] = (f4){0.f, 0.f, 0.f, 0.f};
    const int gx0 = bx * CF_BX - 1, gy0 = by * CF_BY - 1, gz0 = bz * CF_BZ - 1;
    for (int c0 = 0; c0 < cin; c0 += 32) {
        bf8 wn = fetch_w(0, c0);
        if (c0 > 0) __syncthreads();   // every wave is done with the previous chunk's halo and weights
        // stage the halo: piece p = 8 channels (16 bytes) of halo voxel p / 4, in two batches
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            constexpr int NH = (CF_PPT + 1) / 2;
            bf8 hv[NH];
#pragma unroll
            for (int j = 0; j < NH; ++j) {
                const int p = t + 256 * (half * NH + j);
                const int v = p >> 2, part = p & 3;
                const int hx = v % CF_HX, hy = (v / CF_HX) % CF_HY, hz = v / (CF_HX * CF_HY);
                const int gx = gx0 + hx, gy = gy0 + hy, gz = gz0 + hz;
                const bool inb = p < CF_PIECES && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
                const uint32_t off = (uint32_t)(((gx + (int64_t)nx * (gy + (int64_t)ny * gz)) * cin + 8 * part) * 2);
                hv[j] = cf_load(rX, inb ? off : CF_OOB, (uint32_t)(c0 * 2));
            }
#pragma unroll
            for (int j = 0; j < NH; ++j) {
                const int p = t + 256 * (half * NH + j);
                if (half * NH + j < CF_PPT && p < CF_PIECES)
                    *reinterpret_cast<bf8 *>(&sH[(p >> 2) * CF_RS + 8 * cf_hslot(p & 3, (p >> 2) % CF_HX)]) = hv[j];
            }
        }
        *reinterpret_cast<bf8 *>(&sW[0][sslot]) = wn;
        wn = fetch_w(1, c0);
        __syncthreads();
        // one (dy, dz) row of three taps per iteration.  Tap t reads its weights from buffer
        // t % 3 and writes tap t + 1's into the next one, last read in tap t - 2: one barrier per tap
#pragma unroll 1
        for (int row = 0; row < 9; ++row) {
            const int dy = row % 3, dz = row / 3;   // halo offsets (shift + 1)
            const int roff = (CF_HX * dy + CF_HX * CF_HY * dz) * CF_RS;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int tap = 3 * row + dx;
                bf8 a[4], b[4];
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    a[m] = *reinterpret_cast<const bf8 *>(&sH[abase[dx] + roff + (dx + 2 * CF_HX * m) * CF_RS]);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    b[q] = q < ntiles ? *reinterpret_cast<const bf8 *>(&sW[dx][bbase + 16 * q * CF_RS]) : zero8();
                if (tap + 1 < 27) {
                    *reinterpret_cast<bf8 *>(&sW[(dx + 1) % 3][sslot]) = wn;
                    if (tap + 2 < 27) wn = fetch_w(tap + 2, c0);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q < ntiles) {
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            acc[m][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[q], a[m], acc[m][q], 0, 0, 0);
                    }
                }
                __syncthreads();   // the next tap's weights are in place
            }
        }
    }
    // The products are weights x inputs, so the 16 x 16 tile (m, q) is channels x voxels: lane
    // holds output channels 16 q + 4 (lane >> 4) + e, e = 0..3, of patch voxel r = lane & 15
    // (x = r & 7, y = 2 m + (r >> 3)): four consecutive channels, one 8- or 16-byte store.
    const int oz = bz * CF_BZ + w;
    const int r = lane & 15;
    const int cq = 4 * (lane >> 4);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= ntiles) continue;
        const int co = co0 + 16 * q + cq;
        float bv[4] = {0.f, 0.f, 0.f, 0.f};
        if (bias) {
#pragma unroll
            for (int e = 0; e < 4; ++e) bv[e] = bias[co + e];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int ox = bx * CF_BX + (r & 7), oy = by * CF_BY + 2 * m + (r >> 3);
            if (ox >= nx || oy >= ny || oz >= nz) continue;
            const int64_t at = (ox + (int64_t)nx * (oy + (int64_t)ny * oz)) * cout + co;
            float val[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) val[e] = acc[m][q][e] + bv[e];
            if (gate) {
                const uint2 gb = *reinterpret_cast<const uint2 *>(gate + at);
                const uint16_t gv[4] = {(uint16_t)(gb.x & 0xffffu), (uint16_t)(gb.x >> 16),
                                        (uint16_t)(gb.y & 0xffffu), (uint16_t)(gb.y >> 16)};
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (!(bf2f(gv[e]) > 0.f)) val[e] = 0.f;
            }
            if (relu) {
#pragma unroll
                for (int e = 0; e < 4; ++e) val[e] = val[e] > 0.f ? val[e] : 0.f;
            }
            if (Yf) *reinterpret_cast<float4 *>(Yf + at) = make_float4(val[0], val[1], val[2], val[3]);
            if (Ybf)
                *reinterpret_cast<uint2 *>(Ybf + at) =
                    make_uint2((uint32_t)f2bf(val[0]) | ((uint32_t)f2bf(val[1]) << 16),
                               (uint32_t)f2bf(val[2]) | ((uint32_t)f2bf(val[3]) << 16));
        }
    }
}

// ---------------------------------------------------------------- weight gradient
constexpr int WG_K = 64;          // voxels per K step
constexpr int WG_S = WG_K + 8;    // LDS row stride (bf16) of a transposed tile: 144 B, so the 16 rows
                                  // one 16-lane group reads start on distinct 4-bank groups

// Both MFMA operands need 8 consecutive voxels of one channel per lane, while the activations are
// channel-contiguous: each step stages 64 voxels x 64 channels of dY and of the shifted input
// transposed in LDS ([channel][voxel], pairs of voxels packed in one 32-bit write), so a fragment
// is one 128-bit LDS read.  The tiles are double buffered: the next step's global loads are in
// flight during this step's MFMAs, one barrier per step.
__global__ __launch_bounds__(256) void conv_wgrad_k(int nx, int ny, int nz, int cin, int cout,
                                                    int range, const uint16_t *__restrict__ dY,
                                                    const uint16_t *__restrict__ X,
                                                    float *__restrict__ partial)
{
    __shared__ __attribute__((aligned(16))) uint16_t sdy[2][64 * WG_S];
    __shared__ __attribute__((aligned(16))) uint16_t sx[2][64 * WG_S];
    const int64_t V = (int64_t)nx * ny * nz;
    // block -> (range, tap): the 27 taps of a voxel range are consecutive blocks of one XCD
    // (blocks are dealt to the 8 XCDs round-robin), so the range's dY and input tiles come from
    // that XCD's L2 after the first tap instead of from memory 27 times
    const int xcd = blockIdx.x & 7, t2 = blockIdx.x >> 3;
    const int tap = t2 % 27, r = (t2 / 27) * 8 + xcd;
    const int nr = (int)((V + range - 1) / range);
    if (r >= nr) return;
    const int co0 = blockIdx.z / ((cin + 63) / 64) * 64;
    const int ci0 = blockIdx.z % ((cin + 63) / 64) * 64;
    const int mco = cout - co0 < 64 ? cout - co0 : 64;
    const int nci = cin - ci0 < 64 ? cin - ci0 : 64;
    const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // staging role: voxels 2p, 2p + 1 of the step, channels 8g .. 8g + 7
    const int p = threadIdx.x & 31, g = threadIdx.x >> 5;
    const bool gy = 8 * g < mco, gx = 8 * g < nci;
    const int64_t vbeg = (int64_t)r * range;
    const int64_t vend = vbeg + range < V ? vbeg + range : V;
    const int nsteps = (int)((vend - vbeg + WG_K - 1) / WG_K);
    uint4 ry[2], rx[2];
    auto load = [&](int step) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t v = vbeg + (int64_t)step * WG_K + 2 * p + h;
            uint4 zy = make_uint4(0, 0, 0, 0), zx = make_uint4(0, 0, 0, 0);
            if (v < vend) {
                if (gy) zy = *reinterpret_cast<const uint4 *>(dY + v * cout + co0 + 8 * g);
                // lattices hold fewer than 2^31 voxels: 32-bit index arithmetic
                const uint32_t u = (uint32_t)v, uxy = u / (uint32_t)nx;
                const int x = (int)(u - uxy * (uint32_t)nx), y = (int)(uxy % (uint32_t)ny), z = (int)(uxy / (uint32_t)ny);
                const int xs = x + dx, ys = y + dy, zs = z + dz;
                if (gx && xs >= 0 && xs < nx && ys >= 0 && ys < ny && zs >= 0 && zs < nz) {
                    const int64_t vs = xs + (int64_t)nx * (ys + (int64_t)ny * zs);
                    zx = *reinterpret_cast<const uint4 *>(X + vs * cin + ci0 + 8 * g);
                }
            }
            ry[h] = zy;
            rx[h] = zx;
        }
    };
    auto store = [&](int buf) {
        const uint32_t y0[4] = {ry[0].x, ry[0].y, ry[0].z, ry[0].w}, y1[4] = {ry[1].x, ry[1].y, ry[1].z, ry[1].w};
        const uint32_t x0[4] = {rx[0].x, rx[0].y, rx[0].z, rx[0].w}, x1[4] = {rx[1].x, rx[1].y, rx[1].z, rx[1].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // channel 8g + 2q: low halves of the two voxels' words; channel 8g + 2q + 1: high halves
            const int c = 8 * g + 2 * q;
            *reinterpret_cast<uint32_t *>(&sdy[buf][c * WG_S + 2 * p]) = (y0[q] & 0xffffu) | (y1[q] << 16);
            *reinterpret_cast<uint32_t *>(&sdy[buf][(c + 1) * WG_S + 2 * p]) = (y0[q] >> 16) | (y1[q] & 0xffff0000u);
            *reinterpret_cast<uint32_t *>(&sx[buf][c * WG_S + 2 * p]) = (x0[q] & 0xffffu) | (x1[q] << 16);
            *reinterpret_cast<uint32_t *>(&sx[buf][(c + 1) * WG_S + 2 * p]) = (x0[q] >> 16) | (x1[q] & 0xffff0000u);
        }
    };
    // this wave's 4 tiles of the 4x4 grid of 16x16 tiles: (mt = w, nt = 0..3)
    f4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (f4){0.f, 0.f, 0.f, 0.f};
    if (nsteps > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    const int kq = 8 * (lane >> 4);
    for (int step = 0; step < nsteps; ++step) {
        const int buf = step & 1;
        const bool more = step + 1 < nsteps;
        if (more) load(step + 1);
#pragma unroll
        for (int kh = 0; kh < WG_K / 32; ++kh) {
            // A (M = co, K = voxel): row co = 16 w + lane % 16; B (K = voxel, N = ci): column lane % 16
            const bf8 a = *reinterpret_cast<const bf8 *>(&sdy[buf][(16 * w + (lane & 15)) * WG_S + 32 * kh + kq]);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bf8 b = *reinterpret_cast<const bf8 *>(&sx[buf][(16 * t + (lane & 15)) * WG_S + 32 * kh + kq]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
            }
        }
        // the other buffer was last read in the previous step, which every wave has finished
        if (more) store(buf ^ 1);
        __syncthreads();
    }
    // partial[r][tap][co][ci]
    float *out = partial + ((int64_t)r * 27 + tap) * cout * cin;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = co0 + 16 * w + 4 * (lane >> 4) + e;
            const int ci = ci0 + 16 * t + (lane & 15);
            if (co < cout && ci < cin) out[(int64_t)co * cin + ci] = acc[t][e];
        }
}

__global__ __launch_bounds__(256) void sum_ranges_k(int64_t n, int nranges, const float *__restrict__ partial,
                                                    float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int r = 0; r < nranges; ++r) s += partial[(int64_t)r * n + i];
    out[i] = s;
}

// Few outputs over many ranges (the bias gradient): one block per output, thread t sums ranges
// t, t + 256, ... in order, then a fixed pairing tree in LDS (deterministic).
__global__ __launch_bounds__(256) void sum_ranges_wide_k(int64_t n, int nranges, const float *__restrict__ partial,
                                                         float *__restrict__ out)
{
    __shared__ float red[256];
    const int64_t i = blockIdx.x;
    float s = 0.f;
    for (int r = threadIdx.x; r < nranges; r += 256) s += partial[(int64_t)r * n + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
}

// db partials: partial[r][c] = sum_{v in range r} dY[v][c]
// (c <= 256: the block's 256 / c voxel groups take interleaved voxels of the range, four
// independent sums per thread, then the groups are added in a fixed order through LDS)
__global__ __launch_bounds__(256) void bias_grad_k(int64_t V, int c, int range, const uint16_t *__restrict__ dY,
                                                   float *__restrict__ partial)
{
    __shared__ float red[256];
    const int r = blockIdx.x;
    const int64_t vb = (int64_t)r * range, ve = vb + range < V ? vb + range : V;
    if (c > 256) {
        for (int ch = threadIdx.x; ch < c; ch += 256) {
            float s = 0.f;
            for (int64_t v = vb; v < ve; ++v) s += bf2f(dY[v * c + ch]);
            partial[(int64_t)r * c + ch] = s;
        }
        return;
    }
    const int t = threadIdx.x, groups = 256 / c, ch = t % c, grp = t / c;
    float s = 0.f;
    if (grp < groups) {
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
        int64_t v = vb + grp;
        for (; v + 3 * groups < ve; v += 4 * groups) {
            s0 += bf2f(dY[v * c + ch]);
            s1 += bf2f(dY[(v + groups) * c + ch]);
            s2 += bf2f(dY[(v + 2 * groups) * c + ch]);
            s3 += bf2f(dY[(v + 3 * groups) * c + ch]);
        }
        for (; v < ve; v += groups) s0 += bf2f(dY[v * c + ch]);
        s = (s0 + s1) + (s2 + s3);
    }
    red[t] = s;
    __syncthreads();
    if (t < c) {
        float acc = 0.f;
        for (int gi = 0; gi < groups; ++gi) acc += red[gi * c + t];
        partial[(int64_t)r * c + t] = acc;
    }
}

// Wd[tap'][ci][co] = W[26 - tap'][co][ci]
__global__ __launch_bounds__(256) void flip_transpose_k(int cin, int cout, const uint16_t *__restrict__ W,
                                                        uint16_t *__restrict__ Wd)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)27 * cin * cout;
    if (i >= n) return;
    const int tap = (int)(i / ((int64_t)cin * cout));
    const int rem = (int)(i % ((int64_t)cin * cout));
    const int ci = rem / cout, co = rem % cout;
    Wd[i] = W[((int64_t)(26 - tap) * cout + co) * cin + ci];
}

// MSE over the first `used` channels: dpred = 2 (pred - target) / (V used), loss partials per block
__global__ __launch_bounds__(256) void mse_k(int64_t V, int c, int used, const float *__restrict__ pred,
                                             const float *__restrict__ target,
                                             uint16_t *__restrict__ dpred, double *__restrict__ partial)
{
    __shared__ double red[256];
    const double scale = 2.0 / ((double)V * used);
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < V * c; i += (int64_t)gridDim.x * 256) {
        const int ch = (int)(i % c);
        float g = 0.f;
        if (ch < used) {
            const double d = (double)pred[i] - (double)target[i];
            s += d * d;
            g = (float)(scale * d);
        }
        if (dpred) dpred[i] = f2bf(g);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// one block: thread t sums partials t, t + 256, ... in order, then a fixed pairing tree
__global__ __launch_bounds__(256) void sum_partials_d(int n, const double *__restrict__ partial,
                                                      double *__restrict__ out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ __launch_bounds__(256) void adam_k(int64_t n, float *__restrict__ w, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v,
                                              uint16_t *__restrict__ wbf, float lr, float b1, float b2,
                                              float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wbf) wbf[i] = f2bf(wi);
}

__global__ __launch_bounds__(256) void to_bf16_k(int64_t n, const float *__restrict__ in, uint16_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = f2bf(in[i]);
}

__global__ __launch_bounds__(256) void pack_k(int64_t V, int c, NnPack p, float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= V * c) return;
    const int64_t v = i / c;
    const int ch = (int)(i % c);
    float r = 0.f;
    if (ch < p.nch) {
        double val = p.cst[ch];
        if (p.a[ch]) val += p.ca[ch] * p.a[ch][v];
        if (p.b[ch]) val += p.cb[ch] * p.b[ch][v];
        if (p.c[ch]) val += p.cc[ch] * p.c[ch][v];
        r = (float)((val - p.shift[ch]) * p.scale[ch]);
    }
    out[i] = r;
}

// per-channel sum and sum of squares, partial per block (fixed order reduce on the host side)
__global__ __launch_bounds__(256) void moments_k(int64_t V, int c, const float *__restrict__ data,
                                                 double *__restrict__ partial)
{
    // one block per channel slice: blockIdx.y = channel, blockIdx.x = voxel range
    __shared__ double r1[256], r2[256];
    const int ch = blockIdx.y;
    double s = 0.0, q = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256) {
        const double x = data[v * c + ch];
        s += x;
        q += x * x;
    }
    r1[threadIdx.x] = s;
    r2[threadIdx.x] = q;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            r1[threadIdx.x] += r1[threadIdx.x + off];
            r2[threadIdx.x] += r2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[((int64_t)ch * gridDim.x + blockIdx.x) * 2 + 0] = r1[0];
        partial[((int64_t)ch * gridDim.x + blockIdx.x) * 2 + 1] = r2[0];
    }
}

// x[f][v] = base[f][v] + out[v][f] / scale_f + shift_f for f < 4, then Dirichlet values
__global__ __launch_bounds__(256) void unpack_k(int64_t V, int c, const float *__restrict__ out,
                                                const double *__restrict__ base, NnUnpack u,
                                                const uint32_t *__restrict__ mask,
                                                const double *__restrict__ gD, double *__restrict__ x)
{
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= V) return;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        double val = base[f * V + v] + (double)out[v * c + f] / u.scale[f] + u.shift[f];
        if (f < 3 && mask_bit(mask, f * V + v)) val = gD ? gD[f * V + v] : 0.0;
        x[f * V + v] = val;
    }
}

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int nn_conv_fwd(const int32_t *dims, int cin, int cout, const uint16_t *X, const uint16_t *W,
                const float *bias, int relu, const uint16_t *gate, uint16_t *Ybf, float *Yf,
                hipStream_t st)
{
    ProfileScope prof("conv3d_fwd", st);
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2];
    if (((uintptr_t)X | (uintptr_t)W) & 15 || (uintptr_t)Yf & 15 || ((uintptr_t)Ybf | (uintptr_t)gate) & 7) {
        set_error("conv3d: X, W and Y_f32 must be 16-byte aligned, Y_bf16 and gate 8-byte aligned");
        return FSI_ERR_ARG;
    }
    if (V * cin * 2 >= ((int64_t)1 << 31)) {
        set_error("conv3d: the input ([V][cin] bf16, %lld bytes) must stay below 2 GiB", (long long)(V * cin * 2));
        return FSI_ERR_ARG;
    }
    // bricks of 8 x 8 x 4 voxels (fewer than the lattice's voxels, which the ABI keeps below 2^31)
    const int64_t nbk = (int64_t)((dims[0] + CF_BX - 1) / CF_BX) * ((dims[1] + CF_BY - 1) / CF_BY) *
                        ((dims[2] + CF_BZ - 1) / CF_BZ);
    dim3 grid((unsigned)nbk, (unsigned)((cout + 63) / 64));
    hipLaunchKernelGGL(conv_fwd_k, grid, dim3(256), 0, st, dims[0], dims[1], dims[2], cin, cout, X, W,
                       bias, relu, gate, Ybf, Yf);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

size_t nn_wgrad_workspace(const int32_t *dims, int cin, int cout)
{
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2];
    const int64_t nr = (V + NN_WG_RANGE - 1) / NN_WG_RANGE;
    const int64_t nrb = (V + NN_BG_RANGE - 1) / NN_BG_RANGE;
    return align_up((size_t)nr * 27 * cin * cout * sizeof(float)) +
           align_up((size_t)nrb * cout * sizeof(float));
}

int nn_conv_wgrad(const int32_t *dims, int cin, int cout, const uint16_t *dY, const uint16_t *X, float *dW,
                  float *db, void *ws, hipStream_t st)
{
    ProfileScope prof("conv3d_wgrad", st);
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2];
    const int nr = (int)((V + NN_WG_RANGE - 1) / NN_WG_RANGE);
    float *part = reinterpret_cast<float *>(ws);
    float *bpart = reinterpret_cast<float *>(reinterpret_cast<char *>(ws) +
                                             align_up((size_t)nr * 27 * cin * cout * sizeof(float)));
    const int groups = ((cout + 63) / 64) * ((cin + 63) / 64);
    const unsigned nrt = (unsigned)(8 * 27 * ((nr + 7) / 8));   // (range, tap) blocks, ranges padded to 8
    hipLaunchKernelGGL(conv_wgrad_k, dim3(nrt, 1, groups), dim3(256), 0, st, dims[0], dims[1], dims[2], cin,
                       cout, NN_WG_RANGE, dY, X, part);
    FSI_LAUNCH_CHECK();
    const int64_t nw = (int64_t)27 * cin * cout;
    hipLaunchKernelGGL(sum_ranges_k, dim3(nb(nw)), dim3(256), 0, st, nw, nr, part, dW);
    FSI_LAUNCH_CHECK();
    if (db) {
        const int nrb = (int)((V + NN_BG_RANGE - 1) / NN_BG_RANGE);
        hipLaunchKernelGGL(bias_grad_k, dim3(nrb), dim3(256), 0, st, V, cout, NN_BG_RANGE, dY, bpart);
        FSI_LAUNCH_CHECK();
        hipLaunchKernelGGL(sum_ranges_wide_k, dim3(cout), dim3(256), 0, st, (int64_t)cout, nrb, bpart, db);
        FSI_LAUNCH_CHECK();
    }
    return FSI_OK;
}

int nn_flip_transpose(int cin, int cout, const uint16_t *W, uint16_t *Wd, hipStream_t st)
{
    const int64_t n = (int64_t)27 * cin * cout;
    hipLaunchKernelGGL(flip_transpose_k, dim3(nb(n)), dim3(256), 0, st, cin, cout, W, Wd);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

size_t nn_mse_workspace() { return align_up(1025 * sizeof(double)); }

int nn_mse(int64_t V, int c, int used, const float *pred, const float *target, uint16_t *dpred,
           double *loss_host, void *ws, hipStream_t st)
{
    double *part = reinterpret_cast<double *>(ws);
    hipLaunchKernelGGL(mse_k, dim3(1024), dim3(256), 0, st, V, c, used, pred, target, dpred, part);
    FSI_LAUNCH_CHECK();
    hipLaunchKernelGGL(sum_partials_d, dim3(1), dim3(256), 0, st, 1024, part, part + 1024);
    FSI_LAUNCH_CHECK();
    if (loss_host) {
        double s = 0.0;
        FSI_HIP(hipMemcpyAsync(&s, part + 1024, sizeof(double), hipMemcpyDeviceToHost, st));
        FSI_HIP(hipStreamSynchronize(st));
        *loss_host = s / ((double)V * used);
    }
    return FSI_OK;
}

int nn_adam(int64_t n, float *w, const float *g, float *m, float *v, uint16_t *wbf, int t, float lr, float b1,
            float b2, float eps, hipStream_t st)
{
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_k, dim3(nb(n)), dim3(256), 0, st, n, w, g, m, v, wbf, lr, b1, b2, eps, c1, c2);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int nn_to_bf16(int64_t n, const float *in, uint16_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(to_bf16_k, dim3(nb(n)), dim3(256), 0, st, n, in, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

int nn_pack(int64_t V, int c, const NnPack &p, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(pack_k, dim3(nb(V * c)), dim3(256), 0, st, V, c, p, out);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

size_t nn_moments_workspace(int c) { return align_up((size_t)c * 256 * 2 * sizeof(double)); }

int nn_moments(int64_t V, int c, const float *data, double *sums_host, void *ws, hipStream_t st)
{
    double *part = reinterpret_cast<double *>(ws);
    hipLaunchKernelGGL(moments_k, dim3(256, c), dim3(256), 0, st, V, c, data, part);
    FSI_LAUNCH_CHECK();
    std::vector<double> h((size_t)c * 256 * 2);
    FSI_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    FSI_HIP(hipStreamSynchronize(st));
    for (int ch = 0; ch < c; ++ch) {
        double s = 0.0, q = 0.0;
        for (int b = 0; b < 256; ++b) {
            s += h[((size_t)ch * 256 + b) * 2];
            q += h[((size_t)ch * 256 + b) * 2 + 1];
        }
        sums_host[2 * ch] = s;
        sums_host[2 * ch + 1] = q;
    }
    return FSI_OK;
}

int nn_unpack(int64_t V, int c, const float *out, const double *base, const NnUnpack &u,
              const uint32_t *mask, const double *gD, double *x, hipStream_t st)
{
    hipLaunchKernelGGL(unpack_k, dim3(nb(V)), dim3(256), 0, st, V, c, out, base, u, mask, gD, x);
    FSI_LAUNCH_CHECK();
    return FSI_OK;
}

}  // namespace fsi
