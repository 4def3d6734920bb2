// Learned warm start: 3x3x3 convolutions on the node lattice with BF16 operands
// and FP32 accumulation on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16),
// plus the small kernels of training (loss, bias gradient, Adam) and the
// packing of solver fields into network channels.
//
// Layouts: activations channels-last [V][C] (C a multiple of 32, voxel v =
// i + nx (j + ny k)); weights [27][Cout][Cin] with tap = dx + 3 (dy + 3 dz)
// reading the neighbour at offset (dx - 1, dy - 1, dz - 1); zero padding.
//
// Forward / data gradient (implicit GEMM): a block owns 128 voxels x 64 output
// channels, each wave 32 voxels x 64 channels (8 accumulator tiles; 5 waves per
// SIMD, where 64-voxel waves fit 3 and left the second round of blocks at 65^3
// mostly empty).  The K loop runs over the 27 taps x Cin/32 chunks; per step the
// block stages the chunk's 64 x 32 weights in LDS (double buffered, one barrier
// per step), and each lane loads 8 consecutive input channels of its 2 (shifted)
// voxels, so a weight fragment feeds 2 MFMAs and an input fragment 4.  The data gradient is
// the same kernel on flipped, transposed weights, with the ReLU mask of the
// previous layer applied in the epilogue.
// Weight gradient (split K): block (voxel range, tap) stages 64 voxels of dY
// and of the shifted input, transposed, in LDS and accumulates the 64x64 tap
// block with 16 MFMA tiles; ranges are summed in a fixed order afterwards
// (deterministic).
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
constexpr int CF_MT = 2;                 // 16-voxel M tiles per wave
constexpr int CF_VB = 64 * CF_MT;        // voxels per block (4 waves)
constexpr int CF_WS = 40;                // LDS row stride (bf16) of a staged weight chunk: 32 + 8 pad

// 16 zero bytes that out-of-range fragment loads read instead (a pointer choice before the
// load, so the loads can stay in flight: no select on the loaded value)
__device__ __attribute__((aligned(16))) uint16_t cf_zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};

__global__ __launch_bounds__(256) void conv_fwd_k(int nx, int ny, int nz, int cin, int cout,
                                                  const uint16_t *__restrict__ X,
                                                  const uint16_t *__restrict__ W,
                                                  const float *__restrict__ bias, int relu,
                                                  const uint16_t *__restrict__ gate,
                                                  uint16_t *__restrict__ Ybf,
                                                  float *__restrict__ Yf)
{
    // weights of one (tap, 32-channel chunk) for the block's 64 output channels, double buffered
    __shared__ __attribute__((aligned(16))) uint16_t sW[2][64 * CF_WS];
    const int64_t V = (int64_t)nx * ny * nz;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t vw = (int64_t)blockIdx.x * CF_VB + 16 * CF_MT * w;   // first voxel of this wave
    const int co0 = blockIdx.y * 64;
    const int ntiles = (cout - co0) >= 64 ? 4 : (cout - co0) / 16;
    const int kq = 8 * (lane >> 4);
    int ax[CF_MT], ay[CF_MT], az[CF_MT];
    bool vin[CF_MT];
#pragma unroll
    for (int m = 0; m < CF_MT; ++m) {
        const int64_t va = vw + 16 * m + (lane & 15);
        vin[m] = va < V;
        ax[m] = (int)(va % nx);
        ay[m] = (int)((va / nx) % ny);
        az[m] = (int)(va / ((int64_t)nx * ny));
    }
    f4 acc[CF_MT][4];
#pragma unroll
    for (int m = 0; m < CF_MT; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[m][q] = (f4){0.f, 0.f, 0.f, 0.f};
    const int nchunks = cin / 32, nsteps = 27 * nchunks;
    // software pipeline: the weights of step s+1 and the input fragments of step s+1 are in
    // flight while step s runs its MFMAs; the weights go to the other LDS buffer at the end
    // thread t stages 8 channels of output channel co0 + t/4
    const int sco = t >> 2, sci = (t & 3) * 8;
    auto load_w = [&](int step) -> bf8 {
        const int tap = step / nchunks, c0 = (step % nchunks) * 32;
        const uint16_t *p = co0 + sco < cout ? W + ((int64_t)tap * cout + co0 + sco) * cin + c0 + sci : cf_zero;
        return load8(p);
    };
    auto load_a = [&](int step, bf8 *a) {
        const int tap = step / nchunks, c0 = (step % nchunks) * 32;
        const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
#pragma unroll
        for (int m = 0; m < CF_MT; ++m) {
            const int xs = ax[m] + dx, ys = ay[m] + dy, zs = az[m] + dz;
            const bool inb = vin[m] && xs >= 0 && xs < nx && ys >= 0 && ys < ny && zs >= 0 && zs < nz;
            const int64_t vs = xs + (int64_t)nx * (ys + (int64_t)ny * zs);
            a[m] = load8(inb ? X + vs * cin + c0 + kq : cf_zero);
        }
    };
    *reinterpret_cast<bf8 *>(&sW[0][sco * CF_WS + sci]) = load_w(0);
    bf8 a0[CF_MT], a1[CF_MT];
    load_a(0, a0);
    bf8 w_nxt = nsteps > 1 ? load_w(1) : zero8();
    __syncthreads();
    // one step: MFMAs on `a_use` (this step's input fragments) while `a_fill` receives the next
    // step's; the two register sets swap roles every step (the loop below is unrolled by two)
    auto run_step = [&](int step, bf8 *a_use, bf8 *a_fill) {
        const int buf = step & 1;
        const bool more = step + 1 < nsteps;
        if (more) load_a(step + 1, a_fill);
        bf8 bq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            bq[q] = *reinterpret_cast<const bf8 *>(&sW[buf][(16 * q + (lane & 15)) * CF_WS + kq]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < ntiles) {
#pragma unroll
                for (int m = 0; m < CF_MT; ++m)
                    acc[m][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_use[m], bq[q], acc[m][q], 0, 0, 0);
            }
        }
        if (more) {
            *reinterpret_cast<bf8 *>(&sW[buf ^ 1][sco * CF_WS + sci]) = w_nxt;
            if (step + 2 < nsteps) w_nxt = load_w(step + 2);
        }
        __syncthreads();
    };
    for (int step = 0; step < nsteps; step += 2) {
        run_step(step, a0, a1);
        if (step + 1 < nsteps) run_step(step + 1, a1, a0);
    }
    // D layout: lane holds rows 4*(lane/16) + e (voxels), column lane%16 (channel)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= ntiles) continue;
        const int co = co0 + 16 * q + (lane & 15);
        const float bv = bias ? bias[co] : 0.f;
#pragma unroll
        for (int m = 0; m < CF_MT; ++m)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t vo = vw + 16 * m + 4 * (lane >> 4) + e;
                if (vo >= V) continue;
                float val = acc[m][q][e] + bv;
                if (gate && !(bf2f(gate[vo * cout + co]) > 0.f)) val = 0.f;
                if (relu) val = val > 0.f ? val : 0.f;
                if (Yf) Yf[vo * cout + co] = val;
                if (Ybf) Ybf[vo * cout + co] = f2bf(val);
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
    const int r = blockIdx.x, tap = blockIdx.y;
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
    dim3 grid((unsigned)((V + CF_VB - 1) / CF_VB), (unsigned)((cout + 63) / 64));
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
    hipLaunchKernelGGL(conv_wgrad_k, dim3(nr, 27, groups), dim3(256), 0, st, dims[0], dims[1], dims[2], cin,
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
