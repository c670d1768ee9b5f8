// Device-side building blocks shared by the single-cell and the batched
// kernels: vector loads/stores, the per-node update of one lattice Boltzmann
// step and the FP64 observable accumulators.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lbm_internal.h"

// Every kernel that includes this file must perform exactly the same
// floating-point operations per node (population vs moment storage, single
// vs batched launches, any block shape), so the compiler may not fuse a
// multiply and an add on its own; the fused operations are written out.
#pragma clang fp contract(off)

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

// What one thread pulled for its VEC nodes: the rest population, the six
// streamed populations before the gradient-axis shift (wall links already
// reflected), the node's own populations summed (T(t), check modes only), the
// phases, and the populations that left through an isothermal wall.
template <typename real, int VEC>
struct Pulled {
    real f0[VEC], r[6][VEC];
    real told[VEC];
    int ph[VEC];
    double out_hot, out_cold;  // sums of the outgoing wall populations of this thread's nodes
    bool hot, cold;            // this thread holds nodes on the hot / cold face
};

// Distribution storage: state [7][N].
// MODE 0: step; 1: step + observables; 2: observables only; 3: as 2 + flux field.
// NT bit 0: non-temporal state loads; bit 1: non-temporal state stores.
template <typename real, int VEC, int MODE, int NT>
__device__ __forceinline__ void pull_dist(const Cell<real> &c, int xv, int y, int z, const XLink &xl,
                                          Pulled<real, VEC> &P) {
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
    constexpr bool NL = (NT & 1) != 0;
    Vec<real, VEC> c0 = vload<real, VEC, NL>(s + base);
    Vec<real, VEC> a1 = vload<real, VEC, NL>(s + N + base);
    Vec<real, VEC> a2 = vload<real, VEC, NL>(s + 2 * N + base);
    Vec<real, VEC> b3 = vload<real, VEC, NL>(s + pym * N + ((long long)z * ny + ym) * nx + x0);
    Vec<real, VEC> b4 = vload<real, VEC, NL>(s + pyp * N + ((long long)z * ny + yp) * nx + x0);
    Vec<real, VEC> b5 = vload<real, VEC, NL>(s + pzm * N + ((long long)zm * ny + y) * nx + x0);
    Vec<real, VEC> b6 = vload<real, VEC, NL>(s + pzp * N + ((long long)zp * ny + y) * nx + x0);
    load_phase<VEC>(c.phase + base, P.ph);
    if constexpr (MODE != 0) {  // own post-collision populations: T(t) for the residual
        Vec<real, VEC> o3 = vload<real, VEC>(s + 3 * N + base);
        Vec<real, VEC> o4 = vload<real, VEC>(s + 4 * N + base);
        Vec<real, VEC> o5 = vload<real, VEC>(s + 5 * N + base);
        Vec<real, VEC> o6 = vload<real, VEC>(s + 6 * N + base);
#pragma unroll
        for (int v = 0; v < VEC; v++)
            P.told[v] = c0.v[v] + a1.v[v] + a2.v[v] + o3.v[v] + o4.v[v] + o5.v[v] + o6.v[v];
    }
    // x exchange inside the wave: my last g1 feeds the next lane's first
    // node, my first g2 feeds the previous lane's last node
    const real gotL = __shfl(a1.v[VEC - 1], min(max(xl.srcL, 0), 63), 64);
    const real gotR = __shfl(a2.v[0], min(max(xl.srcR, 0), 63), 64);
    real left, right;
    real rawHotX = 0, rawColdX = 0;
    if (x0 == 0) {
        if (c.per[0]) left = xl.haveL ? gotL : s[N + base + nx - 1];
        else { rawHotX = a2.v[0]; left = c.sgn[0] * a2.v[0] + c.phi[0][0]; }
    } else {
        left = xl.haveL ? gotL : s[N + base - 1];
    }
    if (x0 + VEC == nx) {
        if (c.per[0]) right = xl.haveR ? gotR : s[2 * N + base - x0];
        else { rawColdX = a1.v[VEC - 1]; right = c.sgn[0] * a1.v[VEC - 1] + c.phi[0][1]; }
    } else {
        right = xl.haveR ? gotR : s[2 * N + base + VEC];
    }
    // wall links: reflection sign and the imposed inflow (Eq. 24; zero on
    // Dirichlet and zero-flux faces)
    const bool wy3 = ylo && !c.per[1], wy4 = yhi && !c.per[1], wz5 = zlo && !c.per[2], wz6 = zhi && !c.per[2];
    const real sy3 = wy3 ? c.sgn[1] : real(1), py3 = wy3 ? c.phi[1][0] : real(0);
    const real sy4 = wy4 ? c.sgn[1] : real(1), py4 = wy4 ? c.phi[1][1] : real(0);
    const real sz5 = wz5 ? c.sgn[2] : real(1), pz5 = wz5 ? c.phi[2][0] : real(0);
    const real sz6 = wz6 ? c.sgn[2] : real(1), pz6 = wz6 ? c.phi[2][1] : real(0);
#pragma unroll
    for (int v = 0; v < VEC; v++) {
        P.f0[v] = c0.v[v];
        P.r[0][v] = (v == 0 ? left : a1.v[v - 1]);
        P.r[1][v] = (v == VEC - 1 ? right : a2.v[v + 1]);
        P.r[2][v] = fma(sy3, b3.v[v], py3);
        P.r[3][v] = fma(sy4, b4.v[v], py4);
        P.r[4][v] = fma(sz5, b5.v[v], pz5);
        P.r[5][v] = fma(sz6, b6.v[v], pz6);
    }
    if constexpr (MODE != 0) {
        P.out_hot = P.out_cold = 0.0;
        const int g = c.gaxis;
        if (g == 0) {
            P.hot = (x0 == 0);
            P.cold = (x0 + VEC == nx);
            P.out_hot = rawHotX;
            P.out_cold = rawColdX;
        } else {
            const Vec<real, VEC> &bh = (g == 1) ? b3 : b5;
            const Vec<real, VEC> &bc = (g == 1) ? b4 : b6;
            P.hot = (g == 1) ? ylo : zlo;
            P.cold = (g == 1) ? yhi : zhi;
#pragma unroll
            for (int v = 0; v < VEC; v++) {
                P.out_hot += (double)bh.v[v];
                P.out_cold += (double)bc.v[v];
            }
        }
    }
}

// Moment storage: state [4][N] = (T - T_lin, jhat_x / 2, jhat_y / 2, jhat_z / 2).
// With tau_4 = tau_5 = tau_6 = 1 the post-collision populations are
// g_0 = T/4 and g_{2a+1, 2a+2} = T/8 +- jhat_a/2.  In FP64 they are
// recomputed here with the very operations that produce them in population
// storage, so the two storages evolve bit for bit alike; the FP32 moment
// path (pull_mom_exact below) keeps them exact instead.
template <typename real>
__device__ __forceinline__ real gplus(real T, real z) { return fma(T, real(0.125), z); }
template <typename real>
__device__ __forceinline__ real gminus(real T, real z) { return fma(T, real(0.125), -z); }

template <typename real, int VEC, int MODE, int NT>
__device__ __forceinline__ void pull_mom(const Cell<real> &c, int xv, int y, int z, const XLink &xl,
                                         Pulled<real, VEC> &P) {
    const long long N = c.N;
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const int x0 = xv * VEC;
    const long long row = (long long)z * ny + y;
    const long long base = row * nx + x0;
    const real *__restrict__ sT = c.src;
    const real *__restrict__ sX = c.src + N;
    const real *__restrict__ sY = c.src + 2 * N;
    const real *__restrict__ sZ = c.src + 3 * N;
    const bool ylo = (y == 0), yhi = (y == ny - 1), zlo = (z == 0), zhi = (z == nz - 1);
    // a wall link reads the node's own opposite population: own row, other sign of jhat
    const int ym = ylo ? (c.per[1] ? ny - 1 : y) : y - 1;
    const int yp = yhi ? (c.per[1] ? 0 : y) : y + 1;
    const int zm = zlo ? (c.per[2] ? nz - 1 : z) : z - 1;
    const int zp = zhi ? (c.per[2] ? 0 : z) : z + 1;
    const bool wym = ylo && !c.per[1], wyp = yhi && !c.per[1], wzm = zlo && !c.per[2], wzp = zhi && !c.per[2];
    constexpr bool NL = (NT & 1) != 0;
    Vec<real, VEC> Tc = vload<real, VEC, NL>(sT + base);
    Vec<real, VEC> Xc = vload<real, VEC, NL>(sX + base);
    const long long rym = ((long long)z * ny + ym) * nx + x0, ryp = ((long long)z * ny + yp) * nx + x0;
    const long long rzm = ((long long)zm * ny + y) * nx + x0, rzp = ((long long)zp * ny + y) * nx + x0;
    Vec<real, VEC> Tym = vload<real, VEC, NL>(sT + rym), Yym = vload<real, VEC, NL>(sY + rym);
    Vec<real, VEC> Typ = vload<real, VEC, NL>(sT + ryp), Yyp = vload<real, VEC, NL>(sY + ryp);
    Vec<real, VEC> Tzm = vload<real, VEC, NL>(sT + rzm), Zzm = vload<real, VEC, NL>(sZ + rzm);
    Vec<real, VEC> Tzp = vload<real, VEC, NL>(sT + rzp), Zzp = vload<real, VEC, NL>(sZ + rzp);
    load_phase<VEC>(c.phase + base, P.ph);
    // all loads of this node are out: back to the normal wave priority (raised
    // on entry to the moment step)
    __builtin_amdgcn_s_setprio(0);
    // x: my last g1 feeds the next lane, my first g2 the previous lane
    const real mine1 = gplus(Tc.v[VEC - 1], Xc.v[VEC - 1]);
    const real mine2 = gminus(Tc.v[0], Xc.v[0]);
    const real gotL = __shfl(mine1, min(max(xl.srcL, 0), 63), 64);
    const real gotR = __shfl(mine2, min(max(xl.srcR, 0), 63), 64);
    real left, right;
    if (x0 == 0) {
        if (c.per[0]) left = xl.haveL ? gotL : gplus(sT[base + nx - 1], sX[base + nx - 1]);
        else left = c.sgn[0] * mine2 + c.phi[0][0];
    } else {
        left = xl.haveL ? gotL : gplus(sT[base - 1], sX[base - 1]);
    }
    if (x0 + VEC == nx) {
        if (c.per[0]) right = xl.haveR ? gotR : gminus(sT[base - x0], sX[base - x0]);
        else right = c.sgn[0] * mine1 + c.phi[0][1];
    } else {
        right = xl.haveR ? gotR : gminus(sT[base + VEC], sX[base + VEC]);
    }
    Vec<real, VEC> Yc, Zc;
    if constexpr (MODE != 0) {
        Yc = vload<real, VEC>(sY + base);
        Zc = vload<real, VEC>(sZ + base);
    }
#pragma unroll
    for (int v = 0; v < VEC; v++) {
        P.f0[v] = Tc.v[v] * real(0.25);
        P.r[0][v] = (v == 0) ? left : gplus(Tc.v[v - 1], Xc.v[v - 1]);
        P.r[1][v] = (v == VEC - 1) ? right : gminus(Tc.v[v + 1], Xc.v[v + 1]);
        P.r[2][v] = wym ? fma(c.sgn[1], gminus(Tym.v[v], Yym.v[v]), c.phi[1][0]) : gplus(Tym.v[v], Yym.v[v]);
        P.r[3][v] = wyp ? fma(c.sgn[1], gplus(Typ.v[v], Yyp.v[v]), c.phi[1][1]) : gminus(Typ.v[v], Yyp.v[v]);
        P.r[4][v] = wzm ? fma(c.sgn[2], gminus(Tzm.v[v], Zzm.v[v]), c.phi[2][0]) : gplus(Tzm.v[v], Zzm.v[v]);
        P.r[5][v] = wzp ? fma(c.sgn[2], gplus(Tzp.v[v], Zzp.v[v]), c.phi[2][1]) : gminus(Tzp.v[v], Zzp.v[v]);
        if constexpr (MODE != 0) {
            const real t = Tc.v[v];
            P.told[v] = t * real(0.25) + gplus(t, Xc.v[v]) + gminus(t, Xc.v[v]) + gplus(t, Yc.v[v]) +
                        gminus(t, Yc.v[v]) + gplus(t, Zc.v[v]) + gminus(t, Zc.v[v]);
        }
    }
    if constexpr (MODE != 0) {
        P.out_hot = P.out_cold = 0.0;
        const int g = c.gaxis;
        if (g == 0) {
            P.hot = (x0 == 0);
            P.cold = (x0 + VEC == nx);
            P.out_hot = (double)mine2;
            P.out_cold = (double)mine1;
        } else {
            P.hot = (g == 1) ? ylo : zlo;
            P.cold = (g == 1) ? yhi : zhi;
#pragma unroll
            for (int v = 0; v < VEC; v++) {
                const real jh = (g == 1) ? Yc.v[v] : Zc.v[v];
                P.out_hot += (double)gminus(Tc.v[v], jh);
                P.out_cold += (double)gplus(Tc.v[v], jh);
            }
        }
    }
}

// FP32 state: round values computed in FP64 to FP32 with a dither.
// Close to steady state the slowest mode changes a node's T by less than
// half an FP32 ulp per step; round-to-nearest then drops every such
// increment and the iteration stalls at a fixed point of the rounded map whose
// error grows like the mode's relaxation time (N_g^2).  Where the field is
// smooth, round-to-nearest also makes neighbouring nodes err the same way, a
// coherent energy source.  Rounding up with probability equal to the
// discarded fraction keeps every increment in expectation and decorrelates
// the errors.  The random bits are a hash of the value and of a per-node,
// per-quantity key, so the result is a deterministic function of the state
// (independent of launch shape, batching and storage); they change whenever
// the state does.  Mechanism: add 29 random bits below the 23 FP32 fraction
// bits of the FP64 value and truncate; the truncated value is exact in FP32.
// one multiply carries every input bit into the top bits used below
__device__ __forceinline__ unsigned mix32(unsigned a) {
    a ^= a >> 16;
    a *= 0x7feb352du;
    a ^= a >> 15;
    return a;
}

__device__ __forceinline__ float dither_to_float(double x, unsigned long long node) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned key = mix32((unsigned)b ^ (unsigned)(b >> 32) ^ ((unsigned)node * 0x9E3779B9u) ^
                               (unsigned)(node >> 32));
    const unsigned long long r = (unsigned long long)(key >> 3);  // 29 bits
    return (float)__longlong_as_double((long long)((b + r) & ~0x1FFFFFFFull));
}

// Post-collision population T/8 +- jhat_a/2 as population storage keeps it:
// FP64 rounds to nearest; FP32 is dithered (the sum is exact in FP64), so
// that T/8 is not lost, always in the same direction, where it falls below
// half an ulp of jhat_a/2.  a = axis, s = 0 (+) or 1 (-).
template <typename real>
__device__ __forceinline__ real out_pop(real T, real hj, long long node, int a, int s) {
    if constexpr (sizeof(real) == 4) {
        const double e = s ? (double)T * 0.125 - (double)hj : (double)T * 0.125 + (double)hj;
        return dither_to_float(e, ((unsigned long long)node * 8ull + (unsigned long long)(2 * a + s)) ^ (1ull << 62));
    } else {
        return s ? gminus(T, hj) : gplus(T, hj);
    }
}

// General relaxation of the three remaining moments of Eq. 11 (rows 5-7:
// e = 6 f_0 - sum_{i>0} f_i, p_xx = 2 (f_1 + f_2) - (f_3 + f_4 + f_5 + f_6),
// p_ww = f_3 + f_4 - f_5 - f_6) with 1/tau_4..6 of Eq. 12 towards their
// equilibria (3T/4, 0, 0), then f_hat = M^-1 m_hat using the orthogonality of
// M's rows (squared norms 7, 2, 2, 2, 42, 12, 4).
// srel: 1/tau_4, 1/tau_5, 1/tau_6.
template <typename real>
__device__ __forceinline__ void relax_general(const real *srel, real f0, real f1, real f2, real f3, real f4,
                                              real f5, real f6, real T, real hjx, real hjy, real hjz, real *o) {
    const real e = real(6) * f0 - (((((f1 + f2) + f3) + f4) + f5) + f6);
    const real pxx = real(2) * (f1 + f2) - (((f3 + f4) + f5) + f6);
    const real pww = (f3 + f4) - (f5 + f6);
    const real eh = e - srel[0] * (e - real(0.75) * T);
    const real pxxh = pxx - srel[1] * pxx;
    const real pwwh = pww - srel[2] * pww;
    const real base = T * real(1.0 / 7.0) - eh * real(1.0 / 42.0);
    const real ax = base + pxxh * real(1.0 / 6.0);
    const real ay = (base - pxxh * real(1.0 / 12.0)) + pwwh * real(0.25);
    const real az = (base - pxxh * real(1.0 / 12.0)) - pwwh * real(0.25);
    o[0] = (T + eh) * real(1.0 / 7.0);
    o[1] = ax + hjx;
    o[2] = ax - hjx;
    o[3] = ay + hjy;
    o[4] = ay - hjy;
    o[5] = az + hjz;
    o[6] = az - hjz;
}

// Collision (shared by all storages), FP64 observables, and the stores.
// STORAGE 0: 7 populations; 1: 4 moments; 2: 7 populations, general tau_4..6.
template <typename real, int VEC, int MODE, int NT, int STORAGE>
__device__ __forceinline__ void collide_store(const Cell<real> &c, const real *__restrict__ tab, int xv, int y, int z,
                                              bool active, const Pulled<real, VEC> &P, Acc &acc,
                                              real *__restrict__ qout, real qscale) {
    const long long N = c.N;
    const long long base = ((long long)z * c.ny + y) * c.nx + xv * VEC;
    const real hx = c.h[0], hy = c.h[1], hz = c.h[2];
    Vec<real, VEC> T_, X_, Y_, Z_;
    Vec<real, VEC> G_[STORAGE == 2 ? Q : 1];  // general relaxation: the seven outputs
#pragma unroll
    for (int v = 0; v < VEC; v++) {
        const real f0 = P.f0[v];
        const real f1 = P.r[0][v] + hx, f2 = P.r[1][v] - hx;
        const real f3 = P.r[2][v] + hy, f4 = P.r[3][v] - hy;
        const real f5 = P.r[4][v] + hz, f6 = P.r[5][v] - hz;
        const real *tb = tab + P.ph[v] * TABW;  // half of (I - tau^-1)
        real T, jx, jy, jz, hjx, hjy, hjz;
        if constexpr (sizeof(real) == 4) {
            // T and jhat/2 from the FP32 inputs in FP64 (exact sums and
            // differences), each dithered to FP32 with its own random bits
            const unsigned long long key = (unsigned long long)(base + v) * 4ull;
            const double T64 = (((((((double)f0 + (double)f1) + (double)f2) + (double)f3) + (double)f4) +
                                 (double)f5) + (double)f6);
            const double jx64 = (double)f1 - (double)f2, jy64 = (double)f3 - (double)f4,
                         jz64 = (double)f5 - (double)f6;
            const double hx64 = fma((double)tb[4], jz64, fma((double)tb[3], jy64, (double)tb[0] * jx64));
            const double hy64 = fma((double)tb[5], jz64, fma((double)tb[1], jy64, (double)tb[3] * jx64));
            const double hz64 = fma((double)tb[2], jz64, fma((double)tb[5], jy64, (double)tb[4] * jx64));
            T = dither_to_float(T64, key);
            hjx = dither_to_float(hx64, key + 1);
            hjy = dither_to_float(hy64, key + 2);
            hjz = dither_to_float(hz64, key + 3);
            jx = (real)jx64;
            jy = (real)jy64;
            jz = (real)jz64;
        } else {
            T = f0 + f1 + f2 + f3 + f4 + f5 + f6;
            jx = f1 - f2;
            jy = f3 - f4;
            jz = f5 - f6;
            hjx = fma(tb[4], jz, fma(tb[3], jy, tb[0] * jx));
            hjy = fma(tb[5], jz, fma(tb[1], jy, tb[3] * jx));
            hjz = fma(tb[2], jz, fma(tb[5], jy, tb[4] * jx));
        }
        T_.v[v] = T;
        X_.v[v] = hjx;
        Y_.v[v] = hjy;
        Z_.v[v] = hjz;
        if constexpr (STORAGE == 2) {
            real o[Q];
            relax_general(c.srel, f0, f1, f2, f3, f4, f5, f6, T, hjx, hjy, hjz, o);
#pragma unroll
            for (int i = 0; i < Q; i++) G_[i].v[v] = o[i];
        }
        if constexpr (MODE != 0) {
            if (active) {
                const double dT = fabs((double)T - (double)P.told[v]);
                const double qx = 0.5 * (double)jx + (double)hjx;
                const double qy = 0.5 * (double)jy + (double)hjy;
                const double qz = 0.5 * (double)jz + (double)hjz;
                acc.v[R_QX] += qx;
                acc.v[R_QY] += qy;
                acc.v[R_QZ] += qz;
                acc.v[R_TSUM] += (double)T;
                // rounding energy of this node: the populations the next step
                // will stream minus the ones pulled now, both summed exactly
                // in FP64 (the +-h shifts cancel within a node)
                const double din = (double)f0 + (double)P.r[0][v] + (double)P.r[1][v] + (double)P.r[2][v] +
                                   (double)P.r[3][v] + (double)P.r[4][v] + (double)P.r[5][v];
                double dout;
                if constexpr (STORAGE == 2) {
                    dout = (double)G_[0].v[v] + (double)G_[1].v[v] + (double)G_[2].v[v] + (double)G_[3].v[v] +
                           (double)G_[4].v[v] + (double)G_[5].v[v] + (double)G_[6].v[v];
                } else {
                    const long long i = base + v;
                    dout = (double)(T * real(0.25)) + (double)out_pop(T, hjx, i, 0, 0) +
                           (double)out_pop(T, hjx, i, 0, 1) + (double)out_pop(T, hjy, i, 1, 0) +
                           (double)out_pop(T, hjy, i, 1, 1) + (double)out_pop(T, hjz, i, 2, 0) +
                           (double)out_pop(T, hjz, i, 2, 1);
                }
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
            const double hg = (double)c.h[c.gaxis];
            const double nodes = (c.gaxis == 0) ? 1.0 : (double)VEC;
            if (P.hot) acc.v[R_PHI_HOT] += nodes * hg - 2.0 * P.out_hot;
            if (P.cold) acc.v[R_PHI_COLD] += 2.0 * P.out_cold + nodes * hg;
        }
    }
    if constexpr (MODE <= 1) {
        if (active) {
            real *__restrict__ d = c.dst;
            constexpr bool NS = (NT & 2) != 0;
            if constexpr (STORAGE == 0) {
                Vec<real, VEC> o;
#pragma unroll
                for (int v = 0; v < VEC; v++) o.v[v] = T_.v[v] * real(0.25);
                vstore<real, VEC, NS>(d + base, o);
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const Vec<real, VEC> &hj = (a == 0) ? X_ : ((a == 1) ? Y_ : Z_);
                    Vec<real, VEC> p, m;
#pragma unroll
                    for (int v = 0; v < VEC; v++) {
                        p.v[v] = out_pop(T_.v[v], hj.v[v], base + v, a, 0);
                        m.v[v] = out_pop(T_.v[v], hj.v[v], base + v, a, 1);
                    }
                    vstore<real, VEC, NS>(d + (2 * a + 1) * N + base, p);
                    vstore<real, VEC, NS>(d + (2 * a + 2) * N + base, m);
                }
            } else if constexpr (STORAGE == 2) {
#pragma unroll
                for (int i = 0; i < Q; i++) vstore<real, VEC, NS>(d + i * N + base, G_[i]);
            } else {
                vstore<real, VEC, NS>(d + base, T_);
                vstore<real, VEC, NS>(d + N + base, X_);
                vstore<real, VEC, NS>(d + 2 * N + base, Y_);
                vstore<real, VEC, NS>(d + 3 * N + base, Z_);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 moment storage, exact populations.  Every pulled population is
// T/8 +- jhat_a/2 of the FP32 moments of its source node; in FP64 that sum is
// exact, and so are the seven-term T, the differences j and the wall terms.
// The only roundings of a step are then those of the new T and jhat/2 to
// FP32, both dithered.  (Rounding the populations to FP32, as population
// storage must, loses T/8 wherever it is below half an ulp of jhat/2 -- near
// the surface T = T_lin -- with the same sign over whole regions: a coherent
// energy sink.)
// ---------------------------------------------------------------------------

template <int VEC, int MODE>
struct PulledX {
    // exact T(t+1) of each node; its pre-collision j in FP32 (the stored
    // jhat is formed from it, identically in every mode) and, for the
    // observables, exactly
    double T[VEC];
    float j[3][VEC];
    typename std::conditional<MODE != 0, double, char>::type j64[3][VEC];
    float told[VEC];           // the node's stored T(t)
    int ph[VEC];
    double out_hot, out_cold;
    bool hot, cold;
};

__device__ __forceinline__ double pop_plus(float T, float z) { return (double)T * 0.125 + (double)z; }
__device__ __forceinline__ double pop_minus(float T, float z) { return (double)T * 0.125 - (double)z; }

template <int VEC, int MODE, int NT>
__device__ __forceinline__ void pull_mom_exact(const Cell<float> &c, int xv, int y, int z, const XLink &xl,
                                               PulledX<VEC, MODE> &P) {
    const long long N = c.N;
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const int x0 = xv * VEC;
    const long long base = ((long long)z * ny + y) * nx + x0;
    const float *__restrict__ sT = c.src;
    const float *__restrict__ sX = c.src + N;
    const float *__restrict__ sY = c.src + 2 * N;
    const float *__restrict__ sZ = c.src + 3 * N;
    const bool ylo = (y == 0), yhi = (y == ny - 1), zlo = (z == 0), zhi = (z == nz - 1);
    const int ym = ylo ? (c.per[1] ? ny - 1 : y) : y - 1;
    const int yp = yhi ? (c.per[1] ? 0 : y) : y + 1;
    const int zm = zlo ? (c.per[2] ? nz - 1 : z) : z - 1;
    const int zp = zhi ? (c.per[2] ? 0 : z) : z + 1;
    const bool wym = ylo && !c.per[1], wyp = yhi && !c.per[1], wzm = zlo && !c.per[2], wzp = zhi && !c.per[2];
    constexpr bool NL = (NT & 1) != 0;
    // jhat_x/2 of a node is read only by that node (its x neighbours take it
    // by lane exchange), never again by another block: always streamed
    // non-temporally, unlike T, jhat_y and jhat_z, which the y and z
    // neighbours re-read from L2
    Vec<float, VEC> Tc = vload<float, VEC, NL>(sT + base);
    Vec<float, VEC> Xc = vload<float, VEC, true>(sX + base);
    const long long rym = ((long long)z * ny + ym) * nx + x0, ryp = ((long long)z * ny + yp) * nx + x0;
    const long long rzm = ((long long)zm * ny + y) * nx + x0, rzp = ((long long)zp * ny + y) * nx + x0;
    Vec<float, VEC> Tym = vload<float, VEC, NL>(sT + rym), Yym = vload<float, VEC, NL>(sY + rym);
    Vec<float, VEC> Typ = vload<float, VEC, NL>(sT + ryp), Yyp = vload<float, VEC, NL>(sY + ryp);
    Vec<float, VEC> Tzm = vload<float, VEC, NL>(sT + rzm), Zzm = vload<float, VEC, NL>(sZ + rzm);
    Vec<float, VEC> Tzp = vload<float, VEC, NL>(sT + rzp), Zzp = vload<float, VEC, NL>(sZ + rzp);
    load_phase<VEC>(c.phase + base, P.ph);
    // every load of this node is in flight: back to the normal wave priority
    // (the step kernel raises it on entry so the load issue of the waves
    // resident on a SIMD is not interleaved with another wave's arithmetic)
    __builtin_amdgcn_s_setprio(0);
    // x: the moments of my last node feed the next lane, of my first node the previous lane
    const int sl = min(max(xl.srcL, 0), 63), sr = min(max(xl.srcR, 0), 63);
    const float gotLT = __shfl(Tc.v[VEC - 1], sl, 64), gotLX = __shfl(Xc.v[VEC - 1], sl, 64);
    const float gotRT = __shfl(Tc.v[0], sr, 64), gotRX = __shfl(Xc.v[0], sr, 64);
    double left, right;
    if (x0 == 0) {
        if (c.per[0]) left = xl.haveL ? pop_plus(gotLT, gotLX) : pop_plus(sT[base + nx - 1], sX[base + nx - 1]);
        else left = (double)c.sgn[0] * pop_minus(Tc.v[0], Xc.v[0]) + (double)c.phi[0][0];
    } else {
        left = xl.haveL ? pop_plus(gotLT, gotLX) : pop_plus(sT[base - 1], sX[base - 1]);
    }
    if (x0 + VEC == nx) {
        if (c.per[0]) right = xl.haveR ? pop_minus(gotRT, gotRX) : pop_minus(sT[base - x0], sX[base - x0]);
        else right = (double)c.sgn[0] * pop_plus(Tc.v[VEC - 1], Xc.v[VEC - 1]) + (double)c.phi[0][1];
    } else {
        right = xl.haveR ? pop_minus(gotRT, gotRX) : pop_minus(sT[base + VEC], sX[base + VEC]);
    }
    const double s1 = (double)c.sgn[1], s2 = (double)c.sgn[2];
    // the gradient-axis shifts +-h of a population pair cancel in T and
    // add 2h to j
    const float h2x = 2.0f * c.h[0], h2y = 2.0f * c.h[1], h2z = 2.0f * c.h[2];
#pragma unroll
    for (int v = 0; v < VEC; v++) {
        const double p1 = (v == 0) ? left : pop_plus(Tc.v[v - 1], Xc.v[v - 1]);
        const double p2 = (v == VEC - 1) ? right : pop_minus(Tc.v[v + 1], Xc.v[v + 1]);
        const double p3 = wym ? s1 * pop_minus(Tym.v[v], Yym.v[v]) + (double)c.phi[1][0]
                              : pop_plus(Tym.v[v], Yym.v[v]);
        const double p4 = wyp ? s1 * pop_plus(Typ.v[v], Yyp.v[v]) + (double)c.phi[1][1]
                              : pop_minus(Typ.v[v], Yyp.v[v]);
        const double p5 = wzm ? s2 * pop_minus(Tzm.v[v], Zzm.v[v]) + (double)c.phi[2][0]
                              : pop_plus(Tzm.v[v], Zzm.v[v]);
        const double p6 = wzp ? s2 * pop_plus(Tzp.v[v], Zzp.v[v]) + (double)c.phi[2][1]
                              : pop_minus(Tzp.v[v], Zzp.v[v]);
        P.T[v] = (double)Tc.v[v] * 0.25 + p1 + p2 + p3 + p4 + p5 + p6;
        P.j[0][v] = (float)(p1 - p2) + h2x;
        P.j[1][v] = (float)(p3 - p4) + h2y;
        P.j[2][v] = (float)(p5 - p6) + h2z;
        if constexpr (MODE != 0) {
            P.j64[0][v] = (p1 - p2) + (double)h2x;
            P.j64[1][v] = (p3 - p4) + (double)h2y;
            P.j64[2][v] = (p5 - p6) + (double)h2z;
        }
        P.told[v] = Tc.v[v];
    }
    if constexpr (MODE != 0) {
        P.out_hot = P.out_cold = 0.0;
        const int g = c.gaxis;
        if (g == 0) {
            P.hot = (x0 == 0);
            P.cold = (x0 + VEC == nx);
            P.out_hot = pop_minus(Tc.v[0], Xc.v[0]);
            P.out_cold = pop_plus(Tc.v[VEC - 1], Xc.v[VEC - 1]);
        } else {
            const Vec<float, VEC> Jc = vload<float, VEC>((g == 1 ? sY : sZ) + base);
            P.hot = (g == 1) ? ylo : zlo;
            P.cold = (g == 1) ? yhi : zhi;
#pragma unroll
            for (int v = 0; v < VEC; v++) {
                P.out_hot += pop_minus(Tc.v[v], Jc.v[v]);
                P.out_cold += pop_plus(Tc.v[v], Jc.v[v]);
            }
        }
    }
}

template <int VEC, int MODE, int NT>
__device__ __forceinline__ void collide_store_exact(const Cell<float> &c, const float *__restrict__ tab, int xv, int y,
                                                    int z, bool active, const PulledX<VEC, MODE> &P, Acc &acc,
                                                    float *__restrict__ qout, float qscale) {
    const long long N = c.N;
    const long long base = ((long long)z * c.ny + y) * c.nx + xv * VEC;
    Vec<float, VEC> T_, X_, Y_, Z_;
#pragma unroll
    for (int v = 0; v < VEC; v++) {
        const float *tb = tab + P.ph[v] * TABW;  // half of (I - tau^-1)
        // only T needs the dither: jhat relaxes within a few steps, and its
        // rounding moves no energy (the exact populations sum to T anyway)
        const float T = dither_to_float(P.T[v], (unsigned long long)(base + v));
        const float jx = P.j[0][v], jy = P.j[1][v], jz = P.j[2][v];
        T_.v[v] = T;
        X_.v[v] = fmaf(tb[4], jz, fmaf(tb[3], jy, tb[0] * jx));
        Y_.v[v] = fmaf(tb[5], jz, fmaf(tb[1], jy, tb[3] * jx));
        Z_.v[v] = fmaf(tb[2], jz, fmaf(tb[5], jy, tb[4] * jx));
        if constexpr (MODE != 0) {
            if (active) {
                const double jx64 = P.j64[0][v], jy64 = P.j64[1][v], jz64 = P.j64[2][v];
                const double hx = fma((double)tb[4], jz64, fma((double)tb[3], jy64, (double)tb[0] * jx64));
                const double hy = fma((double)tb[5], jz64, fma((double)tb[1], jy64, (double)tb[3] * jx64));
                const double hz = fma((double)tb[2], jz64, fma((double)tb[5], jy64, (double)tb[4] * jx64));
                const double qx = 0.5 * jx64 + hx, qy = 0.5 * jy64 + hy, qz = 0.5 * jz64 + hz;
                acc.v[R_QX] += qx;
                acc.v[R_QY] += qy;
                acc.v[R_QZ] += qz;
                acc.v[R_TSUM] += (double)T;
                // the next step's populations of this node sum exactly to the
                // stored T, so the rounding energy is that of T alone
                acc.v[R_LEAK] += (double)T - P.T[v];
                const double dT = fabs((double)T - (double)P.told[v]);
                if (!(dT <= 1e300)) acc.v[R_NONFINITE] += 1.0;
                else acc.v[R_RESID] = fmax(acc.v[R_RESID], dT);
                if constexpr (MODE == 3) {
                    const long long i = base + v;
                    qout[i] = (float)(qx * (double)qscale);
                    qout[N + i] = (float)(qy * (double)qscale);
                    qout[2 * N + i] = (float)(qz * (double)qscale);
                }
            }
        }
    }
    if constexpr (MODE != 0) {
        if (active) {
            const double hg = (double)c.h[c.gaxis];
            const double nodes = (c.gaxis == 0) ? 1.0 : (double)VEC;
            if (P.hot) acc.v[R_PHI_HOT] += nodes * hg - 2.0 * P.out_hot;
            if (P.cold) acc.v[R_PHI_COLD] += 2.0 * P.out_cold + nodes * hg;
        }
    }
    if constexpr (MODE <= 1) {
        if (active) {
            float *__restrict__ d = c.dst;
            constexpr bool NS = (NT & 2) != 0;
            vstore<float, VEC, NS>(d + base, T_);
            vstore<float, VEC, NS>(d + N + base, X_);
            vstore<float, VEC, NS>(d + 2 * N + base, Y_);
            vstore<float, VEC, NS>(d + 3 * N + base, Z_);
        }
    }
}

// FP32 population storage: the pulled populations with their gradient-axis
// shift, T, j and jhat all in FP64 from the FP32 inputs (exact sums and
// differences), the seven outputs -- T/4, T/8 +- jhat_a/2, or with RELAX the
// general relaxation of the three remaining moments (Eq. 12, tau_4..6 not
// all 1) -- formed in FP64 and each dithered to FP32: these are the only
// roundings of the step.
template <int VEC, int MODE, int NT, bool RELAX>
__device__ __forceinline__ void collide_store_pop32(const Cell<float> &c, const float *__restrict__ tab, int xv, int y,
                                                    int z, bool active, const Pulled<float, VEC> &P, Acc &acc,
                                                    float *__restrict__ qout, float qscale) {
    const long long N = c.N;
    const long long base = ((long long)z * c.ny + y) * c.nx + xv * VEC;
    const double hx = c.h[0], hy = c.h[1], hz = c.h[2];
    double srel[3];
    if constexpr (RELAX) {
        srel[0] = c.srel[0];
        srel[1] = c.srel[1];
        srel[2] = c.srel[2];
    }
    Vec<float, VEC> G[Q];
#pragma unroll
    for (int v = 0; v < VEC; v++) {
        const double f0 = P.f0[v];
        const double f1 = (double)P.r[0][v] + hx, f2 = (double)P.r[1][v] - hx;
        const double f3 = (double)P.r[2][v] + hy, f4 = (double)P.r[3][v] - hy;
        const double f5 = (double)P.r[4][v] + hz, f6 = (double)P.r[5][v] - hz;
        const double T = ((((((f0 + f1) + f2) + f3) + f4) + f5) + f6);
        const double jx = f1 - f2, jy = f3 - f4, jz = f5 - f6;
        const float *tb = tab + P.ph[v] * TABW;  // half of (I - tau^-1)
        const double hjx = fma((double)tb[4], jz, fma((double)tb[3], jy, (double)tb[0] * jx));
        const double hjy = fma((double)tb[5], jz, fma((double)tb[1], jy, (double)tb[3] * jx));
        const double hjz = fma((double)tb[2], jz, fma((double)tb[5], jy, (double)tb[4] * jx));
        const unsigned long long key = (unsigned long long)(base + v) * 8ull;
        if constexpr (RELAX) {
            double o[Q];
            relax_general<double>(srel, f0, f1, f2, f3, f4, f5, f6, T, hjx, hjy, hjz, o);
#pragma unroll
            for (int i = 0; i < Q; i++) G[i].v[v] = dither_to_float(o[i], key + i);
        } else {
            G[0].v[v] = dither_to_float(T * 0.25, key);
            G[1].v[v] = dither_to_float(fma(T, 0.125, hjx), key + 1);
            G[2].v[v] = dither_to_float(fma(T, 0.125, -hjx), key + 2);
            G[3].v[v] = dither_to_float(fma(T, 0.125, hjy), key + 3);
            G[4].v[v] = dither_to_float(fma(T, 0.125, -hjy), key + 4);
            G[5].v[v] = dither_to_float(fma(T, 0.125, hjz), key + 5);
            G[6].v[v] = dither_to_float(fma(T, 0.125, -hjz), key + 6);
        }
        if constexpr (MODE != 0) {
            if (active) {
                // T(t+1) as the next step sums it; the rounding energy is its
                // difference to the exact T
                const double Tn = (double)G[0].v[v] + (double)G[1].v[v] + (double)G[2].v[v] + (double)G[3].v[v] +
                                  (double)G[4].v[v] + (double)G[5].v[v] + (double)G[6].v[v];
                const double qx = 0.5 * jx + hjx, qy = 0.5 * jy + hjy, qz = 0.5 * jz + hjz;
                acc.v[R_QX] += qx;
                acc.v[R_QY] += qy;
                acc.v[R_QZ] += qz;
                acc.v[R_TSUM] += Tn;
                acc.v[R_LEAK] += Tn - T;
                const double dT = fabs(Tn - (double)P.told[v]);
                if (!(dT <= 1e300)) acc.v[R_NONFINITE] += 1.0;
                else acc.v[R_RESID] = fmax(acc.v[R_RESID], dT);
                if constexpr (MODE == 3) {
                    const long long i = base + v;
                    qout[i] = (float)(qx * (double)qscale);
                    qout[N + i] = (float)(qy * (double)qscale);
                    qout[2 * N + i] = (float)(qz * (double)qscale);
                }
            }
        }
    }
    if constexpr (MODE != 0) {
        if (active) {
            const double hg = (double)c.h[c.gaxis];
            const double nodes = (c.gaxis == 0) ? 1.0 : (double)VEC;
            if (P.hot) acc.v[R_PHI_HOT] += nodes * hg - 2.0 * P.out_hot;
            if (P.cold) acc.v[R_PHI_COLD] += 2.0 * P.out_cold + nodes * hg;
        }
    }
    if constexpr (MODE <= 1) {
        if (active) {
            float *__restrict__ d = c.dst;
            constexpr bool NS = (NT & 2) != 0;
#pragma unroll
            for (int i = 0; i < Q; i++) vstore<float, VEC, NS>(d + i * N + base, G[i]);
        }
    }
}

// One node update: pull, then `between(tab)` (the single-cell step kernel
// finishes staging the phase table in LDS there and may point tab at it, so
// that the state loads are already in flight meanwhile), then collide and
// store.
struct NoOp {
    template <typename T>
    __device__ void operator()(const T *&) const {}
};

template <typename real, int VEC, int MODE, int NT = 0, int STORAGE = 0, typename Between = NoOp>
__device__ __forceinline__ void node_update(const Cell<real> &c, const real *tab, int xv, int y, int z,
                                            bool active, const XLink &xl, Acc &acc, real *__restrict__ qout,
                                            real qscale, const Between &between = Between()) {
    if constexpr (STORAGE == 1 && sizeof(real) == 4) {
        PulledX<VEC, MODE> P;
        pull_mom_exact<VEC, MODE, NT>(c, xv, y, z, xl, P);
        between(tab);
        collide_store_exact<VEC, MODE, NT>(c, tab, xv, y, z, active, P, acc, qout, qscale);
    } else if constexpr ((STORAGE == 0 || STORAGE == 2) && sizeof(real) == 4) {
        Pulled<float, VEC> P;
        pull_dist<float, VEC, MODE, NT>(c, xv, y, z, xl, P);
        between(tab);
        collide_store_pop32<VEC, MODE, NT, STORAGE == 2>(c, tab, xv, y, z, active, P, acc, qout, qscale);
    } else {
        Pulled<real, VEC> P;
        if constexpr (STORAGE == 1) pull_mom<real, VEC, MODE, NT>(c, xv, y, z, xl, P);
        else pull_dist<real, VEC, MODE, NT>(c, xv, y, z, xl, P);
        between(tab);
        collide_store<real, VEC, MODE, NT, STORAGE>(c, tab, xv, y, z, active, P, acc, qout, qscale);
    }
}

template <typename real>
__device__ __forceinline__ void load_table(const Cell<real> &c, real *tab) {
    const int n = c.nphase * TABW;
    for (int i = threadIdx.y * blockDim.x + threadIdx.x; i < n; i += blockDim.x * blockDim.y) tab[i] = c.tab[i];
    __syncthreads();
}

// The phase table staged in two halves: the first value of each thread is
// read into a register before the state loads are issued, and written to
// LDS (with the rest of the table, when it has more entries than the block
// has threads) after them.
template <typename real>
struct TablePrefetch {
    real v;
};

template <typename real>
__device__ __forceinline__ TablePrefetch<real> table_prefetch(const Cell<real> &c) {
    const int i = threadIdx.y * blockDim.x + threadIdx.x;
    TablePrefetch<real> t;
    t.v = (i < c.nphase * TABW) ? c.tab[i] : real(0);
    return t;
}

template <typename real>
__device__ __forceinline__ void table_commit(const Cell<real> &c, real *tab, const TablePrefetch<real> &t) {
    const int n = c.nphase * TABW, nt = blockDim.x * blockDim.y;
    const int i0 = threadIdx.y * blockDim.x + threadIdx.x;
    if (i0 < n) tab[i0] = t.v;
    for (int i = i0 + nt; i < n; i += nt) tab[i] = c.tab[i];
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
