// Kernels of the learned warm start: a small 3-D convolutional
// encoder-decoder trained on steady temperature fields the solver produces.
//
// Activations are BF16, channels-last [n][z][y][x][c]; weights of a 3x3x3
// convolution are BF16 [cout][Kpad] with k = tap * cin + ci, tap = (dz*3 +
// dy)*3 + dx for offsets -1..1, zero-padded to Kpad = 32 * ceil(27 cin / 32);
// accumulation is FP32 on the matrix cores (v_mfma_f32_16x16x32_bf16).
// Convolution = implicit GEMM: M = voxels, N = cout, K = 27 cin.  A lane of a
// 16x16x32 product holds 8 consecutive k of one row, i.e. 8 channels of one
// tap: one 16-byte load of the channels-last activations.
// Padding per axis: circular (periodic cell sides) or zero (the walls of the
// gradient axis).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nn_internal.h"

namespace mrt {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));



// coordinates of voxel v (flattened over n, z, y, x; fewer than 2^31 voxels,
// checked on the host), computed once per voxel with 32-bit arithmetic
struct VoxPos {
    int x, y, z, nb;
};

__device__ __forceinline__ VoxPos vox_pos(const ConvGeom &g, int v) {
    const unsigned u = (unsigned)v;
    const unsigned r = u / (unsigned)g.W;
    const unsigned r2 = r / (unsigned)g.H;
    VoxPos p;
    p.x = (int)(u - r * (unsigned)g.W);
    p.y = (int)(r - r2 * (unsigned)g.H);
    p.nb = (int)(r2 / (unsigned)g.D);
    p.z = (int)(r2 - (unsigned)p.nb * (unsigned)g.D);
    return p;
}

// neighbour of a voxel at tap offset ((tap / 9, tap / 3 % 3, tap % 3) - 1);
// -1 if it falls into zero padding
__device__ __forceinline__ int neighbour_at(const ConvGeom &g, const VoxPos &p, int tap) {
    int px = p.x + tap % 3 - 1, py = p.y + (tap / 3) % 3 - 1, pz = p.z + tap / 9 - 1;
    if (px < 0 || px >= g.W) { if (!(g.circ & 1)) return -1; px = px < 0 ? px + g.W : px - g.W; }
    if (py < 0 || py >= g.H) { if (!(g.circ & 2)) return -1; py = py < 0 ? py + g.H : py - g.H; }
    if (pz < 0 || pz >= g.D) { if (!(g.circ & 4)) return -1; pz = pz < 0 ? pz + g.D : pz - g.D; }
    return ((p.nb * g.D + pz) * g.H + py) * g.W + px;
}

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; e++) z[e] = (bf16)0.0f;
    return z;
}

// one wave: 16*MT voxels x 16*NT output channels; 4 waves per block along voxels
template <int MT, int NT>
__global__ void __launch_bounds__(256) k_conv_fwd(const bf16 *__restrict__ in, const bf16 *__restrict__ w,
                                                  const float *__restrict__ bias, ConvGeom g, int relu,
                                                  bf16 *__restrict__ out, float *__restrict__ out_f32) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long nvox = (long long)g.n * g.D * g.H * g.W;
    const long long v0 = ((long long)blockIdx.x * 4 + wave) * (16 * MT);
    const int n0 = blockIdx.y * (16 * NT);
    f32x4 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    VoxPos vrow[MT];
#pragma unroll
    for (int i = 0; i < MT; i++) {
        const long long v = v0 + i * 16 + (lane & 15);
        vrow[i] = vox_pos(g, (int)(v < nvox ? v : nvox - 1));
    }
    const int kq = (lane >> 4) * 8;  // this lane's first k inside a 32-wide chunk
    const int K27 = 27 * g.cin;
    for (int k0 = 0; k0 < g.kpad; k0 += 32) {
        const int k = k0 + kq;
        bf16x8 a[MT], b[NT];
        const int tap = k / g.cin, c0 = k - tap * g.cin;
#pragma unroll
        for (int i = 0; i < MT; i++) {
            const int p = (k < K27) ? neighbour_at(g, vrow[i], tap) : -1;
            a[i] = (p >= 0) ? *reinterpret_cast<const bf16x8 *>(in + (long long)p * g.cin + c0) : zero8();
        }
#pragma unroll
        for (int j = 0; j < NT; j++) {
            const int co = n0 + j * 16 + (lane & 15);
            b[j] = *reinterpret_cast<const bf16x8 *>(w + (long long)co * g.kpad + k);
        }
#pragma unroll
        for (int i = 0; i < MT; i++)
#pragma unroll
            for (int j = 0; j < NT; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // result of a 16x16 tile: lane holds rows 4*(lane/16) + r, column lane % 16
#pragma unroll
    for (int i = 0; i < MT; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) {
            const int co = n0 + j * 16 + (lane & 15);
            const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const long long v = v0 + i * 16 + (lane >> 4) * 4 + r;
                if (v >= nvox) continue;
                float y = acc[i][j][r] + bb;
                if (relu) y = fmaxf(y, 0.0f);
                if (out_f32) out_f32[v * g.cout + co] = y;
                else out[v * g.cout + co] = (bf16)y;
            }
        }
}

// neighbour of a voxel at offset (dx, dy, dz) in {-1, 0, 1}^3, or -1 if it
// falls into zero padding; selects instead of branches
__device__ __forceinline__ int neighbour_off(const ConvGeom &g, const VoxPos &p, int dx, int dy, int dz) {
    int px = p.x + dx, py = p.y + dy, pz = p.z + dz;
    const bool ox = px < 0 || px >= g.W, oy = py < 0 || py >= g.H, oz = pz < 0 || pz >= g.D;
    px += px < 0 ? g.W : (px >= g.W ? -g.W : 0);
    py += py < 0 ? g.H : (py >= g.H ? -g.H : 0);
    pz += pz < 0 ? g.D : (pz >= g.D ? -g.D : 0);
    const bool ok = (!ox || (g.circ & 1)) && (!oy || (g.circ & 2)) && (!oz || (g.circ & 4));
    return ok ? ((p.nb * g.D + pz) * g.H + py) * g.W + px : -1;
}

// k_conv_fwd for a channel count known at compile time (8, 16, 32, 64 or
// 128): the tap and channel of a lane's k are shifts and masks, and with 32
// or more channels (whole 32-wide k-chunks per tap) each tile's neighbour
// is found once per tap instead of once per chunk.  Same tiles, operands
// and accumulation order as k_conv_fwd, so the same results bit for bit.
template <int MT, int NT, int CIN>
__global__ void __launch_bounds__(256) k_conv_fwd_c(const bf16 *__restrict__ in, const bf16 *__restrict__ w,
                                                    const float *__restrict__ bias, ConvGeom g, int relu,
                                                    bf16 *__restrict__ out, float *__restrict__ out_f32) {
    static_assert(CIN == 8 || CIN == 16 || CIN % 32 == 0, "channel count");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long nvox = (long long)g.n * g.D * g.H * g.W;
    const long long v0 = ((long long)blockIdx.x * 4 + wave) * (16 * MT);
    const int n0 = blockIdx.y * (16 * NT);
    f32x4 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    VoxPos vrow[MT];
#pragma unroll
    for (int i = 0; i < MT; i++) {
        const long long v = v0 + i * 16 + (lane & 15);
        vrow[i] = vox_pos(g, (int)(v < nvox ? v : nvox - 1));
    }
    const int kq = (lane >> 4) * 8;  // this lane's first k inside a 32-wide chunk
    const bf16 *wrow[NT];
#pragma unroll
    for (int j = 0; j < NT; j++) wrow[j] = w + (long long)(n0 + j * 16 + (lane & 15)) * g.kpad + kq;
    if constexpr (CIN >= 32) {
        for (int tap = 0; tap < 27; tap++) {
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            const bf16 *src[MT];
#pragma unroll
            for (int i = 0; i < MT; i++) {
                const int p = neighbour_off(g, vrow[i], dx, dy, dz);
                src[i] = p >= 0 ? in + (long long)p * CIN + kq : nullptr;
            }
#pragma unroll
            for (int c = 0; c < CIN / 32; c++) {
                bf16x8 a[MT], b[NT];
#pragma unroll
                for (int i = 0; i < MT; i++)
                    a[i] = src[i] ? *reinterpret_cast<const bf16x8 *>(src[i] + c * 32) : zero8();
#pragma unroll
                for (int j = 0; j < NT; j++)
                    b[j] = *reinterpret_cast<const bf16x8 *>(wrow[j] + tap * CIN + c * 32);
#pragma unroll
                for (int i = 0; i < MT; i++)
#pragma unroll
                    for (int j = 0; j < NT; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
    } else {
        // a 32-wide chunk spans 32 / CIN taps; this lane's 8 channels belong
        // to tap TPC * q + sub of chunk q (tap 27 and beyond: zero padding)
        constexpr int TPC = 32 / CIN;
        const int sub = kq / CIN, c0 = kq % CIN;
#pragma unroll
        for (int q = 0; q < (27 + TPC - 1) / TPC; q++) {
            const int tap = q * TPC + sub;
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            bf16x8 a[MT], b[NT];
#pragma unroll
            for (int i = 0; i < MT; i++) {
                const int p = tap < 27 ? neighbour_off(g, vrow[i], dx, dy, dz) : -1;
                a[i] = p >= 0 ? *reinterpret_cast<const bf16x8 *>(in + (long long)p * CIN + c0) : zero8();
            }
#pragma unroll
            for (int j = 0; j < NT; j++) b[j] = *reinterpret_cast<const bf16x8 *>(wrow[j] + q * 32);
#pragma unroll
            for (int i = 0; i < MT; i++)
#pragma unroll
                for (int j = 0; j < NT; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < MT; i++)
#pragma unroll
        for (int j = 0; j < NT; j++) {
            const int co = n0 + j * 16 + (lane & 15);
            const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const long long v = v0 + i * 16 + (lane >> 4) * 4 + r;
                if (v >= nvox) continue;
                float y = acc[i][j][r] + bb;
                if (relu) y = fmaxf(y, 0.0f);
                if (out_f32) out_f32[v * g.cout + co] = y;
                else out[v * g.cout + co] = (bf16)y;
            }
        }
}

// weights of the adjoint convolution: wt[ci][flip(tap) * cout + co] = w[co][tap * cin + ci]
__global__ void k_weight_flip(const bf16 *__restrict__ w, int cin, int cout, int kpad, int kpad_t, bf16 *__restrict__ wt) {
    const long long total = (long long)cin * kpad_t;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int ci = (int)(i / kpad_t), kt = (int)(i % kpad_t);
        bf16 val = (bf16)0.0f;
        if (kt < 27 * cout) {
            const int tapt = kt / cout, co = kt % cout;
            val = w[(long long)co * kpad + (26 - tapt) * cin + ci];
        }
        wt[i] = val;
    }
}

// Weight gradient through LDS.  dW[co][k] = sum_v dy[v][co] x[nb(v, tap(k))][ci(k)]
// is a product with the voxels as its inner dimension, while both operands
// sit channels-last in memory; each wave therefore stages, per chunk of 32
// voxels, the chunk's dy and the x columns of the block's k-range into LDS
// transposed (voxels contiguous, rows padded to 40 elements so that the
// 16-byte operand reads of one MFMA hit 64 distinct banks), and feeds the
// 16x16x32 MFMA from there: A = dy^T rows (output channels), B = x columns
// (k).  Block: 4 waves, KT 32-wide k-tiles (KT * cout / 2 accumulator
// registers); the waves take every fourth chunk of the block's voxel split,
// their sums are added in a fixed order and the block writes one partial per
// split, summed over the splits in a fixed order afterwards.
constexpr int WG_ROW = 40;  // padded LDS row, in bf16

template <int MT, int KT>
__global__ void __launch_bounds__(256) k_conv_wgrad_lds(const bf16 *__restrict__ x, const bf16 *__restrict__ dy,
                                                        ConvGeom g, long long vox_per_split,
                                                        float *__restrict__ partials) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cout = g.cout, cin = g.cin, K27 = 27 * g.cin;
    // this wave's staging area: dy^T [cout][WG_ROW] then x^T [32 KT][WG_ROW]
    bf16 *dyT = reinterpret_cast<bf16 *>(smem_raw) + (size_t)wave * (cout + 32 * KT) * WG_ROW;
    bf16 *xT = dyT + (size_t)cout * WG_ROW;
    const int kbase = blockIdx.x * 32 * KT;
    const int s = blockIdx.y;
    const long long nvox = (long long)g.n * g.D * g.H * g.W;
    const long long vb = s * vox_per_split, ve = min(nvox, vb + vox_per_split);
    f32x4 acc[MT][2 * KT];  // MT = cout / 16 row tiles
#pragma unroll
    for (int i = 0; i < MT; i++)
#pragma unroll
        for (int j = 0; j < 2 * KT; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int vl = lane & 31;  // the voxel of the chunk this lane stages
    for (long long v0 = vb + 32LL * wave; v0 < ve; v0 += 128) {
        const long long v = v0 + vl;
        const bool inside = v < ve;
        // dy rows of the chunk, transposed
        for (int u = lane; u < 4 * cout; u += 64) {
            const int c8 = (u >> 5) * 8;
            bf16x8 val = inside ? *reinterpret_cast<const bf16x8 *>(dy + v * cout + c8) : zero8();
#pragma unroll
            for (int e = 0; e < 8; e++) dyT[(c8 + e) * WG_ROW + vl] = val[e];
        }
        // x columns kbase .. kbase + 32 KT of the chunk's neighbours, transposed
        const VoxPos pos = vox_pos(g, (int)(inside ? v : vb));
        for (int u = lane; u < 128 * KT; u += 64) {
            const int grp = u >> 5;
            const int k8 = kbase + grp * 8;
            bf16x8 val = zero8();
            if (inside && k8 < K27) {
                const int tap = k8 / cin, ci0 = k8 - tap * cin;
                const int p = neighbour_at(g, pos, tap);
                if (p >= 0) val = *reinterpret_cast<const bf16x8 *>(x + (long long)p * cin + ci0);
            }
#pragma unroll
            for (int e = 0; e < 8; e++) xT[(grp * 8 + e) * WG_ROW + vl] = val[e];
        }
        // the wave's own LDS writes complete before its reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int r = lane & 15, q = (lane >> 4) * 8;
        bf16x8 b[2 * KT];
#pragma unroll
        for (int j = 0; j < 2 * KT; j++) b[j] = *reinterpret_cast<const bf16x8 *>(xT + (j * 16 + r) * WG_ROW + q);
#pragma unroll
        for (int i = 0; i < MT; i++) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(dyT + (i * 16 + r) * WG_ROW + q);
#pragma unroll
            for (int j = 0; j < 2 * KT; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
        }
        // the reads complete before the next chunk overwrites the staging area
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the four waves' sums added in a fixed order through LDS (waves 2, 3
    // into 0, 1, then 1 into 0), one partial per split: tile rows = output
    // channels, columns = k
    __syncthreads();
    float *red = reinterpret_cast<float *>(smem_raw);  // [2][MT][2 KT][4][64]
    constexpr int TILE = MT * 2 * KT * 4;
    if (wave >= 2) {
#pragma unroll
        for (int i = 0; i < MT; i++)
#pragma unroll
            for (int j = 0; j < 2 * KT; j++)
#pragma unroll
                for (int rr = 0; rr < 4; rr++) red[(((wave - 2) * TILE) + (i * 2 * KT + j) * 4 + rr) * 64 + lane] = acc[i][j][rr];
    }
    __syncthreads();
    if (wave < 2) {
#pragma unroll
        for (int i = 0; i < MT; i++)
#pragma unroll
            for (int j = 0; j < 2 * KT; j++)
#pragma unroll
                for (int rr = 0; rr < 4; rr++) acc[i][j][rr] += red[((wave * TILE) + (i * 2 * KT + j) * 4 + rr) * 64 + lane];
    }
    __syncthreads();
    if (wave == 1) {
#pragma unroll
        for (int i = 0; i < MT; i++)
#pragma unroll
            for (int j = 0; j < 2 * KT; j++)
#pragma unroll
                for (int rr = 0; rr < 4; rr++) red[((i * 2 * KT + j) * 4 + rr) * 64 + lane] = acc[i][j][rr];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int i = 0; i < MT; i++) {
#pragma unroll
            for (int j = 0; j < 2 * KT; j++) {
                const int kc = kbase + j * 16 + (lane & 15);
#pragma unroll
                for (int rr = 0; rr < 4; rr++) {
                    const float v = acc[i][j][rr] + red[((i * 2 * KT + j) * 4 + rr) * 64 + lane];
                    const int orow = i * 16 + (lane >> 4) * 4 + rr;
                    if (kc < g.kpad) partials[((long long)s * cout + orow) * g.kpad + kc] = v;
                }
            }
        }
    }
}

// fixed-order sum over splits; optional accumulate into dw
// fixed-order sum over splits: a block of 256 threads takes 16 consecutive
// outputs; thread (o, g) adds splits g, g + 16, g + 32, ... of output o in
// that order, and the 16 group sums are added in group order
constexpr int SUM_GROUPS = 16;
__global__ void __launch_bounds__(256) k_sum_splits(const float *__restrict__ partials, long long len, int splits,
                                                    float *__restrict__ out) {
    __shared__ float red[SUM_GROUPS][256 / SUM_GROUPS];
    const int o = threadIdx.x % (256 / SUM_GROUPS), grp = threadIdx.x / (256 / SUM_GROUPS);
    const long long i = (long long)blockIdx.x * (256 / SUM_GROUPS) + o;
    float acc = 0.0f;
    if (i < len)
        for (int s = grp; s < splits; s += SUM_GROUPS) acc += partials[(long long)s * len + i];
    red[grp][o] = acc;
    __syncthreads();
    if (grp == 0 && i < len) {
        float sum = 0.0f;
        for (int k = 0; k < SUM_GROUPS; k++) sum += red[k][o];
        out[i] = sum;
    }
}

static inline int sum_blocks(long long len) { return (int)((len + 256 / SUM_GROUPS - 1) / (256 / SUM_GROUPS)); }

__global__ void k_sum_rows(const float *__restrict__ p, int rows, float scale, float *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float acc = 0.0f;
        for (int i = 0; i < rows; i++) acc += p[i];
        out[0] = acc * scale;
    }
}

// bias gradient partials: partials[s][c] = sum over the split's voxels of dy[v][c].
// With c <= BIAS_THREADS the block's threads form BIAS_THREADS / c voxel lanes
// (thread t: channel t % c, lane t / c), so a wave reads whole voxel rows;
// lane l sums voxels vb + l, vb + l + lanes, ..., and the lanes' sums are
// added in lane order.  Wider layers keep one thread per channel.
constexpr int BIAS_THREADS = 256;

__global__ void __launch_bounds__(BIAS_THREADS)
k_bias_grad(const bf16 *__restrict__ dy, long long nvox, int c, long long vox_per_split, float *__restrict__ partials) {
    __shared__ float red[BIAS_THREADS];
    const int s = blockIdx.x, t = threadIdx.x;
    const long long vb = s * vox_per_split, ve = min(nvox, vb + vox_per_split);
    if (c > BIAS_THREADS) {
        for (int ch = t; ch < c; ch += BIAS_THREADS) {
            float acc = 0.0f;
            for (long long v = vb; v < ve; v++) acc += (float)dy[v * c + ch];
            partials[(long long)s * c + ch] = acc;
        }
        return;
    }
    const int lanes = BIAS_THREADS / c, ch = t % c, lane = t / c;
    float acc = 0.0f;
    if (lane < lanes)
        for (long long v = vb + lane; v < ve; v += lanes) acc += (float)dy[v * c + ch];
    red[t] = acc;
    __syncthreads();
    if (t < c) {
        float sum = 0.0f;
        for (int l = 0; l < lanes; l++) sum += red[l * c + t];
        partials[(long long)s * c + t] = sum;
    }
}

__global__ void k_relu_bwd(const bf16 *__restrict__ y, const bf16 *__restrict__ dy, bf16 *__restrict__ dx, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dx[i] = ((float)y[i] > 0.0f) ? dy[i] : (bf16)0.0f;
}

__global__ void k_add(const bf16 *__restrict__ a, const bf16 *__restrict__ b, bf16 *__restrict__ out, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = (bf16)((float)a[i] + (float)b[i]);
}

// the same on 8 channels (16 bytes) per thread; the launchers use these when
// the counts are multiples of 8 and the arrays 16-byte aligned
__global__ void k_relu_bwd8(const bf16x8 *__restrict__ y, const bf16x8 *__restrict__ dy, bf16x8 *__restrict__ dx,
                            long long n8) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n8; i += (long long)gridDim.x * blockDim.x) {
        const bf16x8 a = y[i], g = dy[i];
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; e++) o[e] = ((float)a[e] > 0.0f) ? g[e] : (bf16)0.0f;
        dx[i] = o;
    }
}

__global__ void k_add8(const bf16x8 *__restrict__ a, const bf16x8 *__restrict__ b, bf16x8 *__restrict__ out,
                       long long n8) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n8; i += (long long)gridDim.x * blockDim.x) {
        const bf16x8 u = a[i], v = b[i];
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; e++) o[e] = (bf16)((float)u[e] + (float)v[e]);
        out[i] = o;
    }
}

// 2x2x2 average pooling, channels-last; (D, H, W) are the input extents
__global__ void k_pool2_fwd(const bf16 *__restrict__ in, int n, int D, int H, int W, int c, bf16 *__restrict__ out) {
    const int Do = D / 2, Ho = H / 2, Wo = W / 2;
    const long long total = (long long)n * Do * Ho * Wo * c;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        long long r = i / c;
        const int x = (int)(r % Wo); r /= Wo;
        const int y = (int)(r % Ho); r /= Ho;
        const int z = (int)(r % Do);
        const long long nb = r / Do;
        float acc = 0.0f;
        for (int dz = 0; dz < 2; dz++)
            for (int dy = 0; dy < 2; dy++)
                for (int dx = 0; dx < 2; dx++)
                    acc += (float)in[((((nb * D + 2 * z + dz) * H) + 2 * y + dy) * W + 2 * x + dx) * c + ch];
        out[i] = (bf16)(acc * 0.125f);
    }
}

__global__ void k_pool2_bwd(const bf16 *__restrict__ dout, int n, int D, int H, int W, int c, bf16 *__restrict__ din) {
    const long long total = (long long)n * D * H * W * c;
    const int Do = D / 2, Ho = H / 2, Wo = W / 2;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        long long r = i / c;
        const int x = (int)(r % W); r /= W;
        const int y = (int)(r % H); r /= H;
        const int z = (int)(r % D);
        const long long nb = r / D;
        din[i] = (bf16)((float)dout[(((nb * Do + z / 2) * Ho + y / 2) * Wo + x / 2) * c + ch] * 0.125f);
    }
}

// nearest 2x upsampling; (D, H, W) are the input extents
__global__ void k_up2_fwd(const bf16 *__restrict__ in, int n, int D, int H, int W, int c, bf16 *__restrict__ out) {
    const int D2 = 2 * D, H2 = 2 * H, W2 = 2 * W;
    const long long total = (long long)n * D2 * H2 * W2 * c;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        long long r = i / c;
        const int x = (int)(r % W2); r /= W2;
        const int y = (int)(r % H2); r /= H2;
        const int z = (int)(r % D2);
        const long long nb = r / D2;
        out[i] = in[(((nb * D + z / 2) * H + y / 2) * W + x / 2) * c + ch];
    }
}

// k_up2_fwd on 8 channels per thread (c8 = c / 8 groups per voxel)
__global__ void k_up2_fwd8(const bf16x8 *__restrict__ in, int n, int D, int H, int W, int c8, bf16x8 *__restrict__ out) {
    const int D2 = 2 * D, H2 = 2 * H, W2 = 2 * W;
    const long long total = (long long)n * D2 * H2 * W2 * c8;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int cg = (int)(i % c8);
        long long r = i / c8;
        const int x = (int)(r % W2); r /= W2;
        const int y = (int)(r % H2); r /= H2;
        const int z = (int)(r % D2);
        const long long nb = r / D2;
        out[i] = in[(((nb * D + z / 2) * H + y / 2) * W + x / 2) * c8 + cg];
    }
}

__global__ void k_up2_bwd(const bf16 *__restrict__ dout, int n, int D, int H, int W, int c, bf16 *__restrict__ din) {
    const long long total = (long long)n * D * H * W * c;
    const int H2 = 2 * H, W2 = 2 * W, D2 = 2 * D;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        long long r = i / c;
        const int x = (int)(r % W); r /= W;
        const int y = (int)(r % H); r /= H;
        const int z = (int)(r % D);
        const long long nb = r / D;
        float acc = 0.0f;
        for (int dz = 0; dz < 2; dz++)
            for (int dy = 0; dy < 2; dy++)
                for (int dx = 0; dx < 2; dx++)
                    acc += (float)dout[((((nb * D2 + 2 * z + dz) * H2) + 2 * y + dy) * W2 + 2 * x + dx) * c + ch];
        din[i] = (bf16)acc;
    }
}

// mean squared error of channel 0 of pred[v][cpred] against target[v];
// dpred[v][c] = 2 (pred - target) / nvox on channel 0, zero elsewhere;
// partials[block] = sum of squares of the block's voxels
__global__ void __launch_bounds__(256) k_mse(const float *__restrict__ pred, int cpred, const float *__restrict__ target,
                                             long long nvox, bf16 *__restrict__ dpred, float *__restrict__ partials) {
    __shared__ float red[256];
    float acc = 0.0f;
    for (long long v = blockIdx.x * 256LL + threadIdx.x; v < nvox; v += (long long)gridDim.x * 256) {
        const float d = pred[v * cpred] - target[v];
        acc += d * d;
        dpred[v * cpred] = (bf16)(2.0f * d / (float)nvox);
        for (int ch = 1; ch < cpred; ch++) dpred[v * cpred + ch] = (bf16)0.0f;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// Adam on FP32 master weights; also writes the BF16 copy used by the kernels
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       long long n, float lr, float b1, float b2, float eps, float c1, float c2,
                       bf16 *__restrict__ wb) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        if (wb) wb[i] = (bf16)wi;
    }
}

__global__ void k_to_bf16(const float *__restrict__ a, long long n, bf16 *__restrict__ out) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = (bf16)a[i];
}

// network input: per voxel the six tensor entries of its phase (feat[phase][6])
// and the coordinate along x, (x + 1/2) / W - 1/2; channel 7 is zero
__global__ void k_features(const uint8_t *__restrict__ phase, int D, int H, int W, const float *__restrict__ feat,
                           bf16 *__restrict__ out) {
    const long long total = (long long)D * H * W;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < total; v += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(v % W);
        const float *f = feat + 6 * phase[v];
        bf16 *o = out + v * 8;
        for (int c = 0; c < 6; c++) o[c] = (bf16)f[c];
        o[6] = (bf16)(((float)x + 0.5f) / (float)W - 0.5f);
        o[7] = (bf16)0.0f;
    }
}

// first fine index of coarse cell c when n fine voxels are resampled to nc:
// fine voxel i belongs to the coarse cell that holds its centre, i.e. to
// floor((2i + 1) nc / (2n)); the first i of cell c solves (2i + 1) nc >= 2 c n
__device__ __forceinline__ int box_lo(int c, int n, int nc) {
    const long long num = 2LL * c * n - nc;
    return num <= 0 ? 0 : (int)((num + 2LL * nc - 1) / (2LL * nc));
}

// Network input on a coarse grid (Dc, Hc, Wc) for a medium of (D, H, W)
// voxels: channels 0..5 average feat[phase] over the fine voxels whose
// centres lie in the coarse voxel (a coarse voxel with none, when the grid
// is refined, takes the fine voxel under its centre), channel 6 is the
// coarse voxel's own x coordinate, channel 7 is zero.
__global__ void k_features_resampled(const uint8_t *__restrict__ phase, int D, int H, int W,
                                     const float *__restrict__ feat, int Dc, int Hc, int Wc, bf16 *__restrict__ out) {
    const long long total = (long long)Dc * Hc * Wc;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < total; v += (long long)gridDim.x * blockDim.x) {
        const int cx = (int)(v % Wc);
        const long long r = v / Wc;
        const int cy = (int)(r % Hc), cz = (int)(r / Hc);
        int x0 = box_lo(cx, W, Wc), x1 = box_lo(cx + 1, W, Wc);
        int y0 = box_lo(cy, H, Hc), y1 = box_lo(cy + 1, H, Hc);
        int z0 = box_lo(cz, D, Dc), z1 = box_lo(cz + 1, D, Dc);
        if (x1 <= x0) { x0 = (int)(((2LL * cx + 1) * W) / (2LL * Wc)); x1 = x0 + 1; }
        if (y1 <= y0) { y0 = (int)(((2LL * cy + 1) * H) / (2LL * Hc)); y1 = y0 + 1; }
        if (z1 <= z0) { z0 = (int)(((2LL * cz + 1) * D) / (2LL * Dc)); z1 = z0 + 1; }
        float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int z = z0; z < z1; z++)
            for (int y = y0; y < y1; y++)
                for (int x = x0; x < x1; x++) {
                    const float *f = feat + 6 * phase[((long long)z * H + y) * W + x];
                    for (int c = 0; c < 6; c++) acc[c] += f[c];
                }
        const float inv = 1.0f / (float)((z1 - z0) * (y1 - y0) * (x1 - x0));
        bf16 *o = out + v * 8;
        for (int c = 0; c < 6; c++) o[c] = (bf16)(acc[c] * inv);
        o[6] = (bf16)(((float)cx + 0.5f) / (float)Wc - 0.5f);
        o[7] = (bf16)0.0f;
    }
}

// training target: scale * (T - T_lin(x)), T_lin = 1 - (x + 1/2) / W (walls 1 -> 0)
__global__ void k_target(const float *__restrict__ T, int D, int H, int W, float scale, float *__restrict__ out) {
    const long long total = (long long)D * H * W;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < total; v += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(v % W);
        out[v] = scale * (T[v] - (1.0f - ((float)x + 0.5f) / (float)W));
    }
}

// Temperature start field on a (D, H, W) grid from a prediction on a
// (Dc, Hc, Wc) grid covering the same cell (pred[v][cpred], channel 0 =
// scale * (T - T_lin)): trilinear interpolation between coarse voxel centres
// (periodic in y and z, clamped in x), then T = T_lin(x) + pred / scale.
// bad[block] counts values that are not finite or outside [-margin, 1 + margin].
__global__ void k_to_temperature(const float *__restrict__ pred, int cpred, int Dc, int Hc, int Wc, int D, int H, int W,
                                 float scale, float margin, float *__restrict__ T, int *__restrict__ bad) {
    const long long total = (long long)D * H * W;
    const float rx = (float)Wc / (float)W, ry = (float)Hc / (float)H, rz = (float)Dc / (float)D;
    int nbad = 0;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < total; v += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(v % W);
        const long long r = v / W;
        const int y = (int)(r % H), z = (int)(r / H);
        // fine voxel centre in coarse-voxel-centre coordinates
        const float cx = ((float)x + 0.5f) * rx - 0.5f, cy = ((float)y + 0.5f) * ry - 0.5f,
                    cz = ((float)z + 0.5f) * rz - 0.5f;
        const float fx = floorf(cx), fy = floorf(cy), fz = floorf(cz);
        const float tx = cx - fx, ty = cy - fy, tz = cz - fz;
        float acc = 0.0f;
        for (int dz = 0; dz < 2; dz++)
            for (int dy = 0; dy < 2; dy++)
                for (int dx = 0; dx < 2; dx++) {
                    int ix = (int)fx + dx, iy = (int)fy + dy, iz = (int)fz + dz;
                    ix = min(max(ix, 0), Wc - 1);
                    iy = ((iy % Hc) + Hc) % Hc;
                    iz = ((iz % Dc) + Dc) % Dc;
                    const float wgt = (dx ? tx : 1.0f - tx) * (dy ? ty : 1.0f - ty) * (dz ? tz : 1.0f - tz);
                    acc += wgt * pred[(((long long)iz * Hc + iy) * Wc + ix) * cpred];
                }
        const float t = (1.0f - ((float)x + 0.5f) / (float)W) + acc / scale;
        T[v] = t;
        if (!(t >= -margin && t <= 1.0f + margin)) nbad++;
    }
    // per-thread counts summed on the host side through a block reduction
    __shared__ int red[256];
    red[threadIdx.x] = nbad;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) bad[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline int g1(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}

// Tiles of a wave: 16 * mt voxels x 16 * nt output channels.  Large tiles
// reuse each gathered operand over more products, but a coarse level (8^3
// voxels, 128 channels) then fills a few dozen blocks; tiles shrink until a
// launch has 1024 blocks or they are 16 x 16.  Every output element sums the
// same products in the same k order whatever the tile, so the results do
// not depend on the choice.
hipError_t nn_conv_fwd(const void *in, const void *w, const float *bias, const ConvGeom &g, int relu, void *out,
                       float *out_f32, hipStream_t s) {
    const long long nvox = (long long)g.n * g.D * g.H * g.W;
    int mt = 2, nt = (g.cout % 64 == 0) ? 4 : ((g.cout % 32 == 0) ? 2 : 1);
    auto blocks = [&](int m, int n) { return ((nvox + 16 * m - 1) / (16 * m) + 3) / 4 * (g.cout / (16 * n)); };
    while (blocks(mt, nt) < 1024 && (nt > 1 || mt > 1)) {
        if (nt > 1) nt >>= 1;
        else mt = 1;
    }
    const long long vtiles = (nvox + 16 * mt - 1) / (16 * mt);
    const dim3 grid((unsigned)((vtiles + 3) / 4), g.cout / (16 * nt)), block(256);
    const bf16 *i = (const bf16 *)in;
    const bf16 *ww = (const bf16 *)w;
    bf16 *o = (bf16 *)out;
#define FWD_C(MT_, NT_, CIN_) \
    hipLaunchKernelGGL((k_conv_fwd_c<MT_, NT_, CIN_>), grid, block, 0, s, i, ww, bias, g, relu, o, out_f32)
#define FWD_T(MT_, NT_)                                                                                     \
    switch (g.cin) {                                                                                        \
        case 8: FWD_C(MT_, NT_, 8); break;                                                                  \
        case 16: FWD_C(MT_, NT_, 16); break;                                                                \
        case 32: FWD_C(MT_, NT_, 32); break;                                                                \
        case 64: FWD_C(MT_, NT_, 64); break;                                                                \
        case 128: FWD_C(MT_, NT_, 128); break;                                                              \
        default: hipLaunchKernelGGL((k_conv_fwd<MT_, NT_>), grid, block, 0, s, i, ww, bias, g, relu, o, out_f32); \
    }
    if (mt == 2) {
        if (nt == 4) { FWD_T(2, 4) }
        else if (nt == 2) { FWD_T(2, 2) }
        else { FWD_T(2, 1) }
    } else {
        FWD_T(1, 1)
    }
#undef FWD_T
#undef FWD_C
    return hipGetLastError();
}

hipError_t nn_weight_flip(const void *w, int cin, int cout, int kpad, int kpad_t, void *wt, hipStream_t s) {
    hipLaunchKernelGGL(k_weight_flip, dim3(g1((long long)cin * kpad_t)), dim3(256), 0, s, (const bf16 *)w, cin, cout,
                       kpad, kpad_t, (bf16 *)wt);
    return hipGetLastError();
}

// k-tiles per block of the LDS weight gradient: KT * cout / 2 accumulator
// registers, at most 64
static inline int wgrad_kt(const ConvGeom &g) {
    const int kt = g.cout > 64 ? 1 : (g.cout > 32 ? 2 : 4);
    const int ktiles = g.kpad / 32;
    return kt > ktiles ? (ktiles >= 2 ? 2 : 1) : kt;
}

// voxel splits of the weight gradient: about 1024 blocks (the fixed-order
// sum over splits afterwards reads every split's partial), at least 128
// voxels (one chunk per wave) per split
int nn_wgrad_splits(const ConvGeom &g) {
    const long long nvox = (long long)g.n * g.D * g.H * g.W;
    const int kt = wgrad_kt(g);
    const long long kblocks = (g.kpad / 32 + kt - 1) / kt;
    long long s = (1024 + kblocks - 1) / kblocks;
    const long long maxs = (nvox + 127) / 128;
    if (s > maxs) s = maxs;
    if (s > 1024) s = 1024;
    return (int)(s < 1 ? 1 : s);
}

// partial sums the weight gradient leaves in its scratch (one per split)
int nn_wgrad_partials(const ConvGeom &g) { return nn_wgrad_splits(g); }

hipError_t nn_conv_wgrad(const void *x, const void *dy, const ConvGeom &g, int splits, float *partials, float *dw,
                         hipStream_t s) {
    if (g.cout % 16 || g.cout > 128 || g.cin % 8) return hipErrorInvalidValue;
    const long long nvox = (long long)g.n * g.D * g.H * g.W;
    long long per = (nvox + splits - 1) / splits;
    per = (per + 127) / 128 * 128;
    const int kt = wgrad_kt(g);
    const dim3 grid((g.kpad / 32 + kt - 1) / kt, splits);
    const size_t sh = (size_t)4 * (g.cout + 32 * kt) * WG_ROW * sizeof(bf16);
    const bf16 *xx = (const bf16 *)x, *dd = (const bf16 *)dy;
#define WG_LAUNCH(MT, KT) hipLaunchKernelGGL((k_conv_wgrad_lds<MT, KT>), grid, dim3(256), sh, s, xx, dd, g, per, partials)
    switch (g.cout / 16 * 8 + kt) {
        case 8 + 4: WG_LAUNCH(1, 4); break;
        case 8 + 2: WG_LAUNCH(1, 2); break;
        case 8 + 1: WG_LAUNCH(1, 1); break;
        case 16 + 4: WG_LAUNCH(2, 4); break;
        case 16 + 2: WG_LAUNCH(2, 2); break;
        case 16 + 1: WG_LAUNCH(2, 1); break;
        case 24 + 4: WG_LAUNCH(3, 4); break;
        case 24 + 2: WG_LAUNCH(3, 2); break;
        case 24 + 1: WG_LAUNCH(3, 1); break;
        case 32 + 4: WG_LAUNCH(4, 4); break;
        case 32 + 2: WG_LAUNCH(4, 2); break;
        case 32 + 1: WG_LAUNCH(4, 1); break;
        default:
            if (g.cout <= 80) WG_LAUNCH(5, 1);
            else if (g.cout <= 96) WG_LAUNCH(6, 1);
            else if (g.cout <= 112) WG_LAUNCH(7, 1);
            else WG_LAUNCH(8, 1);
            break;
    }
#undef WG_LAUNCH
    const long long len = (long long)g.cout * g.kpad;
    hipLaunchKernelGGL(k_sum_splits, dim3(sum_blocks(len)), dim3(256), 0, s, partials, len, splits, dw);
    return hipGetLastError();
}

hipError_t nn_bias_grad(const void *dy, long long nvox, int c, int splits, float *partials, float *db, hipStream_t s) {
    long long per = (nvox + splits - 1) / splits;
    hipLaunchKernelGGL(k_bias_grad, dim3(splits), dim3(BIAS_THREADS), 0, s, (const bf16 *)dy, nvox, c, per, partials);
    hipLaunchKernelGGL(k_sum_splits, dim3(sum_blocks(c)), dim3(256), 0, s, partials, (long long)c, splits, db);
    return hipGetLastError();
}

static inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

hipError_t nn_relu_bwd(const void *y, const void *dy, void *dx, long long n, hipStream_t s) {
    if (n % 8 == 0 && aligned16(y) && aligned16(dy) && aligned16(dx))
        hipLaunchKernelGGL(k_relu_bwd8, dim3(g1(n / 8)), dim3(256), 0, s, (const bf16x8 *)y, (const bf16x8 *)dy,
                           (bf16x8 *)dx, n / 8);
    else
        hipLaunchKernelGGL(k_relu_bwd, dim3(g1(n)), dim3(256), 0, s, (const bf16 *)y, (const bf16 *)dy, (bf16 *)dx, n);
    return hipGetLastError();
}

hipError_t nn_add(const void *a, const void *b, void *out, long long n, hipStream_t s) {
    if (n % 8 == 0 && aligned16(a) && aligned16(b) && aligned16(out))
        hipLaunchKernelGGL(k_add8, dim3(g1(n / 8)), dim3(256), 0, s, (const bf16x8 *)a, (const bf16x8 *)b,
                           (bf16x8 *)out, n / 8);
    else
        hipLaunchKernelGGL(k_add, dim3(g1(n)), dim3(256), 0, s, (const bf16 *)a, (const bf16 *)b, (bf16 *)out, n);
    return hipGetLastError();
}

hipError_t nn_pool2(int fwd, const void *in, int n, int D, int H, int W, int c, void *out, hipStream_t s) {
    const long long big = (long long)n * D * H * W * c;
    if (fwd) hipLaunchKernelGGL(k_pool2_fwd, dim3(g1(big / 8)), dim3(256), 0, s, (const bf16 *)in, n, D, H, W, c, (bf16 *)out);
    else hipLaunchKernelGGL(k_pool2_bwd, dim3(g1(big)), dim3(256), 0, s, (const bf16 *)in, n, D, H, W, c, (bf16 *)out);
    return hipGetLastError();
}

hipError_t nn_up2(int fwd, const void *in, int n, int D, int H, int W, int c, void *out, hipStream_t s) {
    const long long small = (long long)n * D * H * W * c;
    if (fwd && c % 8 == 0 && aligned16(in) && aligned16(out))
        hipLaunchKernelGGL(k_up2_fwd8, dim3(g1(small)), dim3(256), 0, s, (const bf16x8 *)in, n, D, H, W, c / 8,
                           (bf16x8 *)out);
    else if (fwd) hipLaunchKernelGGL(k_up2_fwd, dim3(g1(small * 8)), dim3(256), 0, s, (const bf16 *)in, n, D, H, W, c, (bf16 *)out);
    else hipLaunchKernelGGL(k_up2_bwd, dim3(g1(small)), dim3(256), 0, s, (const bf16 *)in, n, D, H, W, c, (bf16 *)out);
    return hipGetLastError();
}

hipError_t nn_sum_rows(const float *p, int rows, float scale, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(64), 0, s, p, rows, scale, out);
    return hipGetLastError();
}

int nn_mse_blocks(long long nvox) { return g1(nvox) > 1024 ? 1024 : g1(nvox); }

hipError_t nn_mse(const float *pred, int cpred, const float *target, long long nvox, void *dpred, float *partials,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_mse, dim3(nn_mse_blocks(nvox)), dim3(256), 0, s, pred, cpred, target, nvox, (bf16 *)dpred,
                       partials);
    return hipGetLastError();
}

hipError_t nn_adam(float *w, const float *g, float *m, float *v, long long n, float lr, float b1, float b2, float eps,
                   int t, void *wb, hipStream_t s) {
    float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(g1(n)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2, (bf16 *)wb);
    return hipGetLastError();
}

hipError_t nn_to_bf16(const float *a, long long n, void *out, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3(g1(n)), dim3(256), 0, s, a, n, (bf16 *)out);
    return hipGetLastError();
}

hipError_t nn_features(const uint8_t *phase, int D, int H, int W, const float *feat, void *out, hipStream_t s) {
    hipLaunchKernelGGL(k_features, dim3(g1((long long)D * H * W)), dim3(256), 0, s, phase, D, H, W, feat, (bf16 *)out);
    return hipGetLastError();
}

hipError_t nn_features_resampled(const uint8_t *phase, int D, int H, int W, const float *feat, int Dc, int Hc, int Wc,
                                 void *out, hipStream_t s) {
    hipLaunchKernelGGL(k_features_resampled, dim3(g1((long long)Dc * Hc * Wc)), dim3(256), 0, s, phase, D, H, W, feat,
                       Dc, Hc, Wc, (bf16 *)out);
    return hipGetLastError();
}

hipError_t nn_target(const float *T, int D, int H, int W, float scale, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_target, dim3(g1((long long)D * H * W)), dim3(256), 0, s, T, D, H, W, scale, out);
    return hipGetLastError();
}

int nn_temp_blocks(long long n) { return g1(n) > 2048 ? 2048 : g1(n); }

hipError_t nn_to_temperature(const float *pred, int cpred, int Dc, int Hc, int Wc, int D, int H, int W, float scale,
                             float margin, float *T, int *bad, hipStream_t s) {
    const long long n = (long long)D * H * W;
    hipLaunchKernelGGL(k_to_temperature, dim3(nn_temp_blocks(n)), dim3(256), 0, s, pred, cpred, Dc, Hc, Wc, D, H, W,
                       scale, margin, T, bad);
    return hipGetLastError();
}

}  // namespace mrt
