// Device-side building blocks shared by the single-cell and the batched
// kernels: vector loads/stores, the per-node update of one lattice Boltzmann
// step and the FP64 observable accumulators.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm_internal.h"

namespace mrt {


template <typename real, int VEC>
struct Vec {
    real v[VEC];
};

// NT: streaming (non-temporal) cache policy for the state loads / stores.
template <typename real, int VEC, bool NT = false>
__device__ __forceinline__ Vec<real, VEC> vload(const real *__restrict__ p) {
    Vec<real, VEC> r;
    if constexpr (VEC == 1) {
        r.v[0] = NT ? __builtin_nontemporal_load(p) : p[0];
    } else {
        typedef real vt __attribute__((ext_vector_type(VEC)));
        vt t = NT ? __builtin_nontemporal_load(reinterpret_cast<const vt *>(p)) : *reinterpret_cast<const vt *>(p);
#pragma unroll
        for (int i = 0; i < VEC; i++) r.v[i] = t[i];
    }
    return r;
}

template <typename real, int VEC, bool NT = false>
__device__ __forceinline__ void vstore(real *__restrict__ p, const Vec<real, VEC> &r) {
    if constexpr (VEC == 1) {
        if constexpr (NT) __builtin_nontemporal_store(r.v[0], p);
        else p[0] = r.v[0];
    } else {
        typedef real vt __attribute__((ext_vector_type(VEC)));
        vt t;
#pragma unroll
        for (int i = 0; i < VEC; i++) t[i] = r.v[i];
        if constexpr (NT) __builtin_nontemporal_store(t, reinterpret_cast<vt *>(p));
        else *reinterpret_cast<vt *>(p) = t;
    }
}

template <int VEC>
__device__ __forceinline__ void load_phase(const uint8_t *__restrict__ p, int *out) {
    if constexpr (VEC == 4) {
        uint32_t w = *reinterpret_cast<const uint32_t *>(p);
        out[0] = w & 0xff; out[1] = (w >> 8) & 0xff; out[2] = (w >> 16) & 0xff; out[3] = w >> 24;
    } else if constexpr (VEC == 2) {
        uint32_t w = *reinterpret_cast<const uint16_t *>(p);
        out[0] = w & 0xff; out[1] = w >> 8;
    } else {
        out[0] = p[0];
    }
}

// FP64 accumulators of the check step
struct Acc {
    double v[NRED];
    __device__ void zero() {
#pragma unroll
        for (int i = 0; i < NRED; i++) v[i] = 0.0;
    }
};

// Where a thread finds the x-neighbour elements it does not hold: lane srcL
// holds g_1 of node x0 - 1 (or, for x0 == 0 on a periodic axis, of the row's
// last node) and lane srcR holds g_2 of node x0 + VEC (or of the row's first
// node).  haveL / haveR say whether that lane really holds it (same row or
// whole row inside the wave); otherwise the element is loaded.
struct XLink {
    int srcL, srcR;
    bool haveL, haveR;
};

// MODE 0: step; 1: step + observables; 2: observables only; 3: as 2 + flux field.
// NT bit 0: non-temporal state loads; bit 1: non-temporal state stores.
template <typename real, int VEC, int MODE, int NT = 0>
__device__ __forceinline__ void node_update(const Cell<real> &c, const real *__restrict__ tab, int xv, int y, int z,
                                            bool active, const XLink &xl, Acc &acc, real *__restrict__ qout,
                                            real qscale) {
    const long long N = c.N;
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const int x0 = xv * VEC;
    const long long base = ((long long)z * ny + y) * nx + x0;
    const real *__restrict__ s = c.src;

    // neighbour rows/planes; on a non-periodic wall redirect to the opposite
    // population of the node itself (the reflected link)
    int ym = y - 1, yp = y + 1, pym = 3, pyp = 4;
    const bool ylo = (y == 0), yhi = (y == ny - 1);
    if (ylo) { if (c.per[1]) ym = ny - 1; else { ym = y; pym = 4; } }
    if (yhi) { if (c.per[1]) yp = 0; else { yp = y; pyp = 3; } }
    int zm = z - 1, zp = z + 1, pzm = 5, pzp = 6;
    const bool zlo = (z == 0), zhi = (z == nz - 1);
    if (zlo) { if (c.per[2]) zm = nz - 1; else { zm = z; pzm = 6; } }
    if (zhi) { if (c.per[2]) zp = 0; else { zp = z; pzp = 5; } }

    Vec<real, VEC> c0 = vload<real, VEC, (NT & 1) != 0>(s + base);
    Vec<real, VEC> a1 = vload<real, VEC, (NT & 1) != 0>(s + N + base);
    Vec<real, VEC> a2 = vload<real, VEC, (NT & 1) != 0>(s + 2 * N + base);
    Vec<real, VEC> b3 = vload<real, VEC, (NT & 1) != 0>(s + pym * N + ((long long)z * ny + ym) * nx + x0);
    Vec<real, VEC> b4 = vload<real, VEC, (NT & 1) != 0>(s + pyp * N + ((long long)z * ny + yp) * nx + x0);
    Vec<real, VEC> b5 = vload<real, VEC, (NT & 1) != 0>(s + pzm * N + ((long long)zm * ny + y) * nx + x0);
    Vec<real, VEC> b6 = vload<real, VEC, (NT & 1) != 0>(s + pzp * N + ((long long)zp * ny + y) * nx + x0);
    int ph[VEC];
    load_phase<VEC>(c.phase + base, ph);
    Vec<real, VEC> o3, o4, o5, o6;
    if constexpr (MODE != 0) {  // own post-collision populations: T(t) for the residual
        o3 = vload<real, VEC>(s + 3 * N + base);
        o4 = vload<real, VEC>(s + 4 * N + base);
        o5 = vload<real, VEC>(s + 5 * N + base);
        o6 = vload<real, VEC>(s + 6 * N + base);
    }

    // x exchange inside the wave: my last g1 feeds the next lane's first
    // node, my first g2 feeds the previous lane's last node
    const real gotL = __shfl(a1.v[VEC - 1], min(max(xl.srcL, 0), 63), 64);
    const real gotR = __shfl(a2.v[0], min(max(xl.srcR, 0), 63), 64);
    real left, right;
    const real hx = c.h[0], hy = c.h[1], hz = c.h[2];
    real rawHotX = 0, rawColdX = 0;
    if (x0 == 0) {
        if (c.per[0]) left = xl.haveL ? gotL : s[N + base + nx - 1];
        else { rawHotX = a2.v[0]; left = c.sgn[0] * a2.v[0]; }
    } else {
        left = xl.haveL ? gotL : s[N + base - 1];
    }
    if (x0 + VEC == nx) {
        if (c.per[0]) right = xl.haveR ? gotR : s[2 * N + base - x0];
        else { rawColdX = a1.v[VEC - 1]; right = c.sgn[0] * a1.v[VEC - 1]; }
    } else {
        right = xl.haveR ? gotR : s[2 * N + base + VEC];
    }
    const real sy3 = (ylo && !c.per[1]) ? c.sgn[1] : real(1);
    const real sy4 = (yhi && !c.per[1]) ? c.sgn[1] : real(1);
    const real sz5 = (zlo && !c.per[2]) ? c.sgn[2] : real(1);
    const real sz6 = (zhi && !c.per[2]) ? c.sgn[2] : real(1);

    Vec<real, VEC> out[Q];
#pragma unroll
    for (int v = 0; v < VEC; v++) {
        const real f0 = c0.v[v];
        const real r1 = (v == 0 ? left : a1.v[v - 1]);
        const real r2 = (v == VEC - 1 ? right : a2.v[v + 1]);
        const real r3 = sy3 * b3.v[v], r4 = sy4 * b4.v[v];
        const real r5 = sz5 * b5.v[v], r6 = sz6 * b6.v[v];
        const real f1 = r1 + hx, f2 = r2 - hx;
        const real f3 = r3 + hy, f4 = r4 - hy;
        const real f5 = r5 + hz, f6 = r6 - hz;
        const real T = f0 + f1 + f2 + f3 + f4 + f5 + f6;
        const real jx = f1 - f2, jy = f3 - f4, jz = f5 - f6;
        const real *tb = tab + ph[v] * TABW;  // half of (I - tau^-1)
        const real hjx = tb[0] * jx + tb[3] * jy + tb[4] * jz;
        const real hjy = tb[3] * jx + tb[1] * jy + tb[5] * jz;
        const real hjz = tb[4] * jx + tb[5] * jy + tb[2] * jz;
        const real t8 = T * real(0.125);
        out[0].v[v] = T * real(0.25);
        out[1].v[v] = t8 + hjx;
        out[2].v[v] = t8 - hjx;
        out[3].v[v] = t8 + hjy;
        out[4].v[v] = t8 - hjy;
        out[5].v[v] = t8 + hjz;
        out[6].v[v] = t8 - hjz;
        if constexpr (MODE != 0) {
            if (active) {
                const real Told = c0.v[v] + a1.v[v] + a2.v[v] + o3.v[v] + o4.v[v] + o5.v[v] + o6.v[v];
                const double dT = fabs((double)T - (double)Told);
                const double qx = 0.5 * (double)jx + (double)hjx;
                const double qy = 0.5 * (double)jy + (double)hjy;
                const double qz = 0.5 * (double)jz + (double)hjz;
                acc.v[R_QX] += qx;
                acc.v[R_QY] += qy;
                acc.v[R_QZ] += qz;
                acc.v[R_TSUM] += (double)T;
                // rounding energy of this node: stored outputs minus the
                // pulled inputs, both summed exactly in FP64 (the +-h
                // shifts cancel within a node)
                double din = (double)f0 + (double)r1 + (double)r2 + (double)r3 + (double)r4 + (double)r5 + (double)r6;
                double dout = 0.0;
#pragma unroll
                for (int i = 0; i < Q; i++) dout += (double)out[i].v[v];
                acc.v[R_LEAK] += dout - din;
                if (!(dT <= 1e300)) acc.v[R_NONFINITE] += 1.0;
                else acc.v[R_RESID] = fmax(acc.v[R_RESID], dT);
                if constexpr (MODE == 3) {
                    const long long i = base + v;
                    qout[i] = (real)(qx * (double)qscale);
                    qout[N + i] = (real)(qy * (double)qscale);
                    qout[2 * N + i] = (real)(qz * (double)qscale);
                }
            }
        }
    }

    if constexpr (MODE != 0) {
        if (active) {
            // wall link fluxes through the isothermal faces:
            // hot:  eps (T_hot - T_lin(0)) - 2 g_out = h - 2 g_out
            // cold: 2 g_out + eps (T_lin(n-1) - T_cold) = 2 g_out + h
            const int g = c.gaxis;
            const double hg = (double)c.h[g];
            if (g == 0) {
                if (x0 == 0) acc.v[R_PHI_HOT] += hg - 2.0 * (double)rawHotX;
                if (x0 + VEC == nx) acc.v[R_PHI_COLD] += 2.0 * (double)rawColdX + hg;
            } else if (g == 1) {
                if (ylo) for (int v = 0; v < VEC; v++) acc.v[R_PHI_HOT] += hg - 2.0 * (double)b3.v[v];
                if (yhi) for (int v = 0; v < VEC; v++) acc.v[R_PHI_COLD] += 2.0 * (double)b4.v[v] + hg;
            } else {
                if (zlo) for (int v = 0; v < VEC; v++) acc.v[R_PHI_HOT] += hg - 2.0 * (double)b5.v[v];
                if (zhi) for (int v = 0; v < VEC; v++) acc.v[R_PHI_COLD] += 2.0 * (double)b6.v[v] + hg;
            }
        }
    }

    if constexpr (MODE <= 1) {
        if (active) {
            real *__restrict__ d = c.dst;
#pragma unroll
            for (int i = 0; i < Q; i++) vstore<real, VEC, (NT & 2) != 0>(d + i * N + base, out[i]);
        }
    }
}

template <typename real>
__device__ __forceinline__ void load_table(const Cell<real> &c, real *tab) {
    const int n = c.nphase * TABW;
    for (int i = threadIdx.y * blockDim.x + threadIdx.x; i < n; i += blockDim.x * blockDim.y) tab[i] = c.tab[i];
    __syncthreads();
}

// deterministic block reduction of the 8 accumulators (sums, one max)
__device__ __forceinline__ void block_reduce_store(Acc &acc, double *out) {
    __shared__ double red[16][NRED];
#pragma unroll
    for (int k = 0; k < NRED; k++) {
        double v = acc.v[k];
        for (int off = 32; off >= 1; off >>= 1) {
            double o = __shfl_xor(v, off, 64);
            v = (k == R_RESID) ? fmax(v, o) : v + o;
        }
        acc.v[k] = v;
    }
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int wave = tid >> 6, nw = (blockDim.x * blockDim.y + 63) >> 6;
    if ((tid & 63) == 0)
        for (int k = 0; k < NRED; k++) red[wave][k] = acc.v[k];
    __syncthreads();
    if (tid < NRED) {
        double v = red[0][tid];
        for (int w = 1; w < nw; w++) v = (tid == R_RESID) ? fmax(v, red[w][tid]) : v + red[w][tid];
        out[tid] = v;
    }
}


}  // namespace mrt
