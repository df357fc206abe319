// Contrast kernels of the LS operator: f = B u = -E^T (dC (E u)) + w^2 drho u  (Eq 8, 11-12, 17-18).
//
// E is the Voigt engineering strain by second-order central differences, with the first-order
// one-sided difference on the model boundary (Eq 18); E^T is its exact discrete adjoint, so the
// divergence of the contrast stress is -E^T tau.  Per cell, tau = dC eps with dC the symmetric
// 6x6 of the cell (21 packed values).  The first kernel writes tau for every cell, the second
// forms f and writes it straight into the zero-padded FFT work buffer.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "fft_reg.h"

namespace ls {

namespace {

constexpr int kThreads = 256;

// packed index of the upper-triangle entry (I, J), I <= J, row order 11,12,...,16,22,...,66
__host__ __device__ constexpr int packed(int I, int J) {
    return I <= J ? I * 6 - I * (I - 1) / 2 + (J - I) : J * 6 - J * (J - 1) / 2 + (I - J);
}

// packed indices of the nine entries of an orthotropic stiffness (11, 12, 13, 22, 23, 33, 44, 55, 66) and of the
// twelve others, which vanish for isotropic, VTI and orthorhombic media in the grid axes
constexpr int kOrtho9[9] = {0, 1, 2, 6, 7, 11, 15, 18, 20};
constexpr int kOffOrtho[12] = {3, 4, 5, 8, 9, 10, 12, 13, 14, 16, 17, 19};

// d/dx_a at index i of an axis with n cells (Eq 18): central inside, one-sided at the ends
template <typename T>
__device__ __forceinline__ cpx<T> deriv(const cpx<T>* __restrict__ f, long long p, long long stride, int i, int n,
                                        T inv_h) {
    if (i == 0) return inv_h * (f[p + stride] - f[p]);
    if (i == n - 1) return inv_h * (f[p] - f[p - stride]);
    return (T(0.5) * inv_h) * (f[p + stride] - f[p - stride]);
}

// (D^T v)(i) along one axis: coefficients of v(i-1), v(i), v(i+1) in row sums of D
template <typename T>
__device__ __forceinline__ cpx<T> deriv_t(const cpx<T>* __restrict__ v, long long p, long long stride, int i, int n,
                                          T inv_h) {
    cpx<T> acc = {T(0), T(0)};
    if (i >= 1) {
        const T cm = (i - 1 == 0) ? inv_h : T(0.5) * inv_h;
        acc = acc + cm * v[p - stride];
    }
    if (i == 0) acc = acc - inv_h * v[p];
    if (i == n - 1) acc = acc + inv_h * v[p];
    if (i <= n - 2) {
        const T cp = (i + 1 == n - 1) ? -inv_h : T(-0.5) * inv_h;
        acc = acc + cp * v[p + stride];
    }
    return acc;
}

// Voigt strain at the cell with grid indices (i, j, k) of an N1 x N2 x N3 grid; the field's values sit
// at element p of three component arrays n apart, with neighbours 1, sy and sz elements away (the
// grid itself, or a tile of it staged in LDS).
template <typename T>
__device__ __forceinline__ void strain_at_strided(const cpx<T>* __restrict__ u, long long n, long long p, int i,
                                                  int j, int k, long long sy, long long sz, int N1, int N2, int N3,
                                                  T inv_h, cpx<T> eps[6]) {
    const long long sx = 1;
    const cpx<T>* u0 = u;
    const cpx<T>* u1 = u + n;
    const cpx<T>* u2 = u + 2 * n;
    eps[0] = deriv(u0, p, sx, i, N1, inv_h);
    eps[1] = deriv(u1, p, sy, j, N2, inv_h);
    eps[2] = deriv(u2, p, sz, k, N3, inv_h);
    eps[3] = deriv(u1, p, sz, k, N3, inv_h) + deriv(u2, p, sy, j, N2, inv_h);
    eps[4] = deriv(u0, p, sz, k, N3, inv_h) + deriv(u2, p, sx, i, N1, inv_h);
    eps[5] = deriv(u0, p, sy, j, N2, inv_h) + deriv(u1, p, sx, i, N1, inv_h);
}

template <typename T>
__device__ __forceinline__ void strain_at(const cpx<T>* __restrict__ u, long long n, long long p, int i, int j,
                                          int k, int N1, int N2, int N3, T inv_h, cpx<T> eps[6]) {
    const long long sx = 1, sy = N1, sz = (long long)N1 * N2;
    const cpx<T>* u0 = u;
    const cpx<T>* u1 = u + n;
    const cpx<T>* u2 = u + 2 * n;
    eps[0] = deriv(u0, p, sx, i, N1, inv_h);
    eps[1] = deriv(u1, p, sy, j, N2, inv_h);
    eps[2] = deriv(u2, p, sz, k, N3, inv_h);
    eps[3] = deriv(u1, p, sz, k, N3, inv_h) + deriv(u2, p, sy, j, N2, inv_h);
    eps[4] = deriv(u0, p, sz, k, N3, inv_h) + deriv(u2, p, sx, i, N1, inv_h);
    eps[5] = deriv(u0, p, sy, j, N2, inv_h) + deriv(u1, p, sx, i, N1, inv_h);
}

// tau[r][6][n] = dC(p) eps(u at slot sm.slot[r])(p)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_strain_stress(const cpx<T>* __restrict__ u, cpx<T>* __restrict__ tau,
                                                            const T* __restrict__ dc, SlotMap sm, int nrhs, int N1,
                                                            int N2, int N3, T inv_h) {
    const long long n = (long long)N1 * N2 * N3;
    const long long lb = xcd_logical_block(blockIdx.x, (n + kThreads - 1) / kThreads);
    const long long p = lb * kThreads + threadIdx.x;
    if (lb < 0 || p >= n) return;
    const int i = (int)(p % N1);
    const int j = (int)((p / N1) % N2);
    const int k = (int)(p / ((long long)N1 * N2));
    T C[21];
#pragma unroll
    for (int q = 0; q < 21; ++q) C[q] = dc[q * n + p];
    for (int r = 0; r < nrhs; ++r) {
        cpx<T> eps[6];
        strain_at(u + (long long)sm.slot[r] * 3 * n, n, p, i, j, k, N1, N2, N3, inv_h, eps);
        cpx<T>* tr = tau + (long long)r * 6 * n;
#pragma unroll
        for (int I = 0; I < 6; ++I) {
            cpx<T> acc = {T(0), T(0)};
#pragma unroll
            for (int J = 0; J < 6; ++J) acc = acc + C[packed(I, J)] * eps[J];
            tr[I * n + p] = acc;
        }
    }
}

// f_c(p) = -sum_a (D_a^T tau_{V(a,c)})(p) + w^2 drho(p) u_c(p), for position r (tau[r]) on field slot
// sw.slot[r] at w^2 = sw.w2[r].
// OUT 0: f written to the padded work buffer at position r (layout of zplane_offset; component pitch N3 L2 L1).
// OUT 1: the transposed operator's epilogue, work[compact] = y - f (work is then a compact field array,
// indexed by slot like y).
template <typename T, int OUT>
__global__ __launch_bounds__(kThreads) void k_divergence(const cpx<T>* __restrict__ tau, const cpx<T>* __restrict__ u,
                                                         const T* __restrict__ drho, cpx<T>* __restrict__ work,
                                                         SlotW2<T> sw, int nrhs, int N1, int N2, int N3, int L1,
                                                         int L2, T inv_h, const cpx<T>* __restrict__ y, int zbs) {
    const long long n = (long long)N1 * N2 * N3;
    const long long lb = xcd_logical_block(blockIdx.x, (n + kThreads - 1) / kThreads);
    const long long p = lb * kThreads + threadIdx.x;
    if (lb < 0 || p >= n) return;
    const int i = (int)(p % N1);
    const int j = (int)((p / N1) % N2);
    const int k = (int)(p / ((long long)N1 * N2));
    const long long sx = 1, sy = N1, sz = (long long)N1 * N2;
    const T dr = drho[p];
    const long long cpitch = (long long)N3 * L2 * L1;
    const long long wpos = zplane_offset(k, zbs, L2, L1) + zrow_offset(j, zbs, L1) + i;
    for (int r = 0; r < nrhs; ++r) {
        const T wr = sw.w2[r] * dr;
        const long long so = (long long)sw.slot[r] * 3 * n;
        const cpx<T>* t = tau + (long long)r * 6 * n;
        const cpx<T>* ur = u + so;
        // Voigt index of the pair (a, c): 11->0, 22->1, 33->2, 23->3, 13->4, 12->5
        const cpx<T> f0 = deriv_t(t + 0 * n, p, sx, i, N1, inv_h) + deriv_t(t + 5 * n, p, sy, j, N2, inv_h) +
                          deriv_t(t + 4 * n, p, sz, k, N3, inv_h);
        const cpx<T> f1 = deriv_t(t + 5 * n, p, sx, i, N1, inv_h) + deriv_t(t + 1 * n, p, sy, j, N2, inv_h) +
                          deriv_t(t + 3 * n, p, sz, k, N3, inv_h);
        const cpx<T> f2 = deriv_t(t + 4 * n, p, sx, i, N1, inv_h) + deriv_t(t + 3 * n, p, sy, j, N2, inv_h) +
                          deriv_t(t + 2 * n, p, sz, k, N3, inv_h);
        if constexpr (OUT == 0) {
            cpx<T>* wr_ = work + (long long)r * 3 * cpitch + wpos;
            wr_[0] = wr * ur[p] - f0;
            wr_[cpitch] = wr * ur[n + p] - f1;
            wr_[2 * cpitch] = wr * ur[2 * n + p] - f2;
        } else {
            const cpx<T>* yr = y + so;
            cpx<T>* o = work + so;
            o[p] = yr[p] - (wr * ur[p] - f0);
            o[n + p] = yr[n + p] - (wr * ur[n + p] - f1);
            o[2 * n + p] = yr[2 * n + p] - (wr * ur[2 * n + p] - f2);
        }
    }
}

// Weights of the values at i-1, i, i+1 in one derivative along an axis of n >= 2 cells: of the
// strain stencil d/dx (Eq 18: central inside, one-sided at the ends) and of its transpose D^T.
template <typename T>
struct W3 {
    T m, z, p;
};

template <typename T>
__device__ __forceinline__ W3<T> d_weights(int i, int n, T inv_h) {
    if (i == 0) return {T(0), -inv_h, inv_h};
    if (i == n - 1) return {-inv_h, inv_h, T(0)};
    return {T(-0.5) * inv_h, T(0), T(0.5) * inv_h};
}

template <typename T>
__device__ __forceinline__ W3<T> dt_weights(int i, int n, T inv_h) {
    W3<T> w;
    w.m = i >= 1 ? (i - 1 == 0 ? inv_h : T(0.5) * inv_h) : T(0);
    w.z = (i == 0 ? -inv_h : T(0)) + (i == n - 1 ? inv_h : T(0));
    w.p = i <= n - 2 ? (i + 1 == n - 1 ? -inv_h : T(-0.5) * inv_h) : T(0);
    return w;
}

template <typename T>
__device__ __forceinline__ cpx<T> w3(const W3<T>& w, cpx<T> fm, cpx<T> f0, cpx<T> fp) {
    return w.m * fm + w.z * f0 + w.p * fp;
}

// Fused contrast, marching in z: f = w^2 drho u - E^T (dC E u) in one pass over u.
//
// One block = one right-hand side, one BX x BY column of cells and a chunk of z planes.  LDS holds a
// ring of four u planes with a 2-cell xy halo and two tau planes with a 1-cell xy halo (no corners).
// Thread roles: the first BX*BY threads own one cell each (full tau, then f); the next 2*BX threads
// take the halo rows below and above the column and the next 2*BY the halo columns left and right,
// and compute only the tau components that the divergence reads there (Voigt 22, 23, 12 across a y
// face; 11, 13, 12 across an x face).  With BX = 32 every wave has one role, so each step is one
// tau pass per wave.  The z neighbours of tau at the owned cells stay in registers, so step k
// computes tau(k+1) and f(k) between the same two barriers (details at the loop).  Each u plane is read from HBM once per chunk (plus the xy halo, served
// mostly from L2), each dC once per chunk and right-hand side (from the tile-packed copy: one contiguous run
// of 21 BX BY values per tile and plane instead of 21 x BY short rows, 7 % faster in FP32, 11 % in FP64) (right-hand sides are the fastest
// logical block index, so the blocks of one column share dC through one L2), and f is written once
// as full 128-byte rows.  Derivatives use per-lane weights (no divergent branches at the model
// boundary): every LDS value they touch is finite, since u planes are stored whole (zeros outside the
// grid) and the tau planes start zeroed and only ever receive finite values.
// OUT 0: f into the padded work buffer; OUT 1: out = y - f (the transposed operator's epilogue).
// Launch position rhs works on field slot sw.slot[rhs] of u (and y, out for OUT 1) at w^2 = sw.w2[rhs]; OUT 0
// writes position rhs of the work buffer.
template <typename T, int BX, int BY, int NT, int MINB, bool DB, int OUT, int K>
__global__ __launch_bounds__(NT, MINB) void k_contrast_zmarch(
    const cpx<T>* __restrict__ u, const T* __restrict__ dcp, const T* __restrict__ drho, cpx<T>* __restrict__ out,
    const cpx<T>* __restrict__ y, SlotW2<T> sw, int nrhs, int N1, int N2, int N3, int L1, int L2, T inv_h, int tx,
    int ty, int nzc, long long nb_real, int zbs) {
    constexpr int NOWN = BX * BY;
    constexpr int UX = BX + 4, UY = BY + 4, UP = UX * UY;  // u plane (halo 2)
    constexpr int SX = BX + 2, SY = BY + 2, SP = SX * SY;  // tau plane (halo 1)
    constexpr int NLOAD = (3 * UP + NT - 1) / NT;
    constexpr int NRING = 2 * BX + 2 * BY;
    static_assert(NOWN + NRING <= NT, "one tau cell per thread");
    static_assert(NLOAD <= 32, "validity mask of the plane loads");
    __shared__ cpx<T> us[4 * 3 * UP];
    __shared__ cpx<T> ts[2 * 6 * SP];

    const long long lb = xcd_logical_block(blockIdx.x, nb_real);
    if (lb < 0) return;
    const int t = threadIdx.x;
    const int rhs = (int)(lb % nrhs);
    const long long col = lb / nrhs;
    const int x0 = (int)(col % tx) * BX;
    const int y0 = (int)((col / tx) % ty) * BY;
    const int z0 = (int)(col / ((long long)tx * ty)) * nzc;
    const int zend = min(z0 + nzc, N3);
    const long long n = (long long)N1 * N2 * N3;
    const long long plane = (long long)N1 * N2;
    const long long so = (long long)sw.slot[rhs] * 3 * n;   // this position's field slot
    const T w2 = sw.w2[rhs];
    const cpx<T>* ur = u + so;

    // role: 0 owned cell, 1 y-face halo cell, 2 x-face halo cell, 3 idle; (lx, ly) in plane coordinates
    int role, lx, ly;
    if (t < NOWN) {
        role = 0, lx = t % BX, ly = t / BX;
    } else if (t < NOWN + 2 * BX) {
        const int r = t - NOWN;
        role = 1, lx = r % BX, ly = r < BX ? -1 : BY;
    } else if (t < NOWN + NRING) {
        const int r = t - NOWN - 2 * BX;
        role = 2, lx = r < BY ? -1 : BX, ly = r % BY;
    } else {
        role = 3, lx = 0, ly = 0;
    }
    const int gx = x0 + lx, gy = y0 + ly;
    const bool cell = role != 3 && gx >= 0 && gx < N1 && gy >= 0 && gy < N2;
    const bool own = role == 0 && cell;
    const W3<T> dxw = d_weights(gx, N1, inv_h), dyw = d_weights(gy, N2, inv_h);
    const W3<T> txw = dt_weights(gx, N1, inv_h), tyw = dt_weights(gy, N2, inv_h);
    const unsigned cell_xy = cell ? (unsigned)(gy * N1 + gx) : 0u;  // clamped: never used when !cell
    // the cell's place in the tile-packed contrast (k_pack_contrast): its tile's run of K x BX x BY values
    // on a z plane, then its position in the tile
    static_assert(K == 21 || K == 9, "general or orthotropic contrast");
    constexpr int TILE = BX * BY;
    const int pgx = cell ? gx : 0, pgy = cell ? gy : 0;
    const long long pplane = (long long)tx * ty * K * TILE;
    const unsigned pxy = (unsigned)(((pgy / BY) * tx + pgx / BX) * K * TILE + (pgy % BY) * BX + pgx % BX);

    // plane loads: element e = t + m NT of the [3][UY][UX] box; its offset in plane 0 and validity
    unsigned ldoff[NLOAD];
    unsigned ldok = 0;
#pragma unroll
    for (int m = 0; m < NLOAD; ++m) {
        const int e = t + m * NT;
        const int c = e / UP, rem = e - c * UP;
        const int bly = rem / UX, blx = rem - bly * UX;
        const int bx = x0 - 2 + blx, by = y0 - 2 + bly;
        ldoff[m] = 0;
        if (e < 3 * UP && bx >= 0 && bx < N1 && by >= 0 && by < N2) {
            ldoff[m] = (unsigned)(c * n + (long long)by * N1 + bx);
            ldok |= 1u << m;
        }
    }
    // Prefetched plane, raw (scalar arrays: kept in registers).  Loads are unconditional (invalid
    // elements read a valid address: ldoff = 0 of a clamped plane), so no load sits behind a branch,
    // and the zeroing select is applied only when the plane is stored, a step later, so that the
    // load's latency is not waited for at the load.
    T pfr[NLOAD], pfi[NLOAD];
    bool pf_in = false;
    auto load_plane = [&](int q) __attribute__((always_inline)) {
        pf_in = q >= 0 && q < N3;
        const cpx<T>* src = ur + (long long)min(max(q, 0), N3 - 1) * plane;
#pragma unroll
        for (int m = 0; m < NLOAD; ++m) {
            const cpx<T> v = src[ldoff[m]];
            pfr[m] = v.x;
            pfi[m] = v.y;
        }
    };
    auto store_plane = [&](int q) __attribute__((always_inline)) {
        cpx<T>* s = us + (q & 3) * 3 * UP;
#pragma unroll
        for (int m = 0; m < NLOAD; ++m) {
            const int e = t + m * NT;
            const bool ok = pf_in && ((ldok >> m) & 1u);
            if (e < 3 * UP) s[e] = cpx<T>{ok ? pfr[m] : T(0), ok ? pfi[m] : T(0)};
        }
    };
    // dC of this thread's cell (a clamped valid cell when the thread has none): C for the tau plane of
    // this step; with DB, Cn is loaded for the next one at the top of the step, else C is reloaded
    // right after its tau plane (fewer registers)
    T C[21], Cn[DB ? 21 : 1];
    // K = 9: the twelve entries off the orthotropic pattern are compile-time zeros, so their loads and products
    // drop out (adding the exact zeros they would contribute leaves every sum bitwise unchanged)
    auto load_C = [&](T* dst, int q) __attribute__((always_inline)) {
        const T* base = dcp + (long long)min(max(q, 0), N3 - 1) * pplane + pxy;
        if constexpr (K == 21) {
#pragma unroll
            for (int qq = 0; qq < 21; ++qq) dst[qq] = base[qq * TILE];
        } else {
#pragma unroll
            for (int qq = 0; qq < 12; ++qq) dst[kOffOrtho[qq]] = T(0);
#pragma unroll
            for (int qq = 0; qq < 9; ++qq) dst[kOrtho9[qq]] = base[qq * TILE];
        }
    };
    // tau on plane q at this thread's cell, from u planes q-1, q, q+1: rows I of dC eps for which
    // the mask bit I is set
    // tau on plane q at this thread's cell, from u planes q-1, q, q+1: rows I of dC eps for which the
    // mask bit I is set; the owned cell also returns its z components (Voigt 33, 23, 13) in zc
    auto tau_cell = [&](int q, auto rows, cpx<T>* zc, const T* C) __attribute__((always_inline)) {
        constexpr int mask = decltype(rows)::value;
        const cpx<T>* um = us + ((q - 1) & 3) * 3 * UP;
        const cpx<T>* u0 = us + (q & 3) * 3 * UP;
        const cpx<T>* up = us + ((q + 1) & 3) * 3 * UP;
        const W3<T> dz = d_weights(q, N3, inv_h);
        const int pu = (ly + 2) * UX + (lx + 2);
        auto ddx = [&](int c) __attribute__((always_inline)) {
            const cpx<T>* f = u0 + c * UP + pu;
            return w3(dxw, f[-1], f[0], f[1]);
        };
        auto ddy = [&](int c) __attribute__((always_inline)) {
            const cpx<T>* f = u0 + c * UP + pu;
            return w3(dyw, f[-UX], f[0], f[UX]);
        };
        auto ddz = [&](int c) __attribute__((always_inline)) {
            return w3(dz, um[c * UP + pu], u0[c * UP + pu], up[c * UP + pu]);
        };
        cpx<T> eps[6];
        eps[0] = ddx(0);
        eps[1] = ddy(1);
        eps[2] = ddz(2);
        eps[3] = ddz(1) + ddy(2);
        eps[4] = ddz(0) + ddx(2);
        eps[5] = ddy(0) + ddx(1);
        cpx<T>* s = ts + (q & 1) * 6 * SP + (ly + 1) * SX + (lx + 1);
#pragma unroll
        for (int I = 0; I < 6; ++I) {
            if (!((mask >> I) & 1)) continue;
            cpx<T> acc = {T(0), T(0)};
#pragma unroll
            for (int J = 0; J < 6; ++J) acc = acc + C[packed(I, J)] * eps[J];
            s[I * SP] = acc;
            if constexpr (mask == 0x3f) {
                if (I >= 2 && I <= 4) zc[I - 2] = acc;
            }
        }
    };
    auto tau_plane = [&](int q, cpx<T>* zc, const T* C) __attribute__((always_inline)) {
        if (q < 0 || q >= N3 || !cell) return;  // never read with a nonzero weight
        if (role == 0)
            tau_cell(q, std::integral_constant<int, 0x3f>{}, zc, C);
        else if (role == 1)
            tau_cell(q, std::integral_constant<int, (1 << 1) | (1 << 3) | (1 << 5)>{}, zc, C);
        else
            tau_cell(q, std::integral_constant<int, (1 << 0) | (1 << 4) | (1 << 5)>{}, zc, C);
    };

    // prologue: zero tau planes; u planes z0-2 .. z0+2; tau planes z0-1 and z0 (the owned cell's z
    // components of tau in registers: tprev, tcur, tnext for planes k-1, k, k+1)
    for (int e = t; e < 2 * 6 * SP; e += NT) ts[e] = cpx<T>{T(0), T(0)};
    for (int q = z0 - 2; q <= z0 + 1; ++q) {
        load_plane(q);
        store_plane(q);
    }
    __syncthreads();
    cpx<T> tprev[3] = {}, tcur[3] = {}, tnext[3] = {};
    load_C(C, z0 - 1);
    tau_plane(z0 - 1, tprev, C);
    load_C(C, z0);
    tau_plane(z0, tcur, C);
    __syncthreads();  // tau(z0-1) has read u(z0-2), whose ring slot u(z0+2) takes
    load_plane(z0 + 2);
    store_plane(z0 + 2);
    if (z0 + 3 <= zend + 1) load_plane(z0 + 3);
    load_C(C, z0 + 1);
    T dro = (drho + (long long)z0 * plane)[cell_xy], dron = T(0);
    __syncthreads();
    const int po = (ly + 1) * SX + (lx + 1);

    // One barrier per step: step k computes tau(k+1) into one tau plane and f(k) from the other, and
    // stores u(k+3) into the ring slot of u(k-1), which nothing reads in this step.  The dC and drho of
    // the next step are requested at the top of the step and the next u plane right after the store,
    // so each load has about a whole step to land.  The loop is unrolled by two with the dC and drho of
    // alternate steps in alternate registers (C, Cn and dro, dron): no loaded value is copied, so the first
    // wait for a load comes in the step that uses it, not at the end of the step that issued it (the wait
    // counter retires loads in order, so such a wait also waits for every load issued before it).
    auto step = [&](int k, T* Cu, T* Cx, T& du, T& dx) __attribute__((always_inline)) {
        const bool more = k + 1 < zend;
        if (more) {
            if constexpr (DB) load_C(Cx, k + 2);
            dx = (drho + (long long)(k + 1) * plane)[cell_xy];
        }
        tau_plane(k + 1, tnext, Cu);
        if constexpr (!DB) {
            if (more) load_C(Cu, k + 2);
        }
        if (own) {
            const cpx<T>* s0 = ts + (k & 1) * 6 * SP + po;
            const W3<T> tz = dt_weights(k, N3, inv_h);
            auto tdx = [&](int I) __attribute__((always_inline)) {
                const cpx<T>* v = s0 + I * SP;
                return w3(txw, v[-1], v[0], v[1]);
            };
            auto tdy = [&](int I) __attribute__((always_inline)) {
                const cpx<T>* v = s0 + I * SP;
                return w3(tyw, v[-SX], v[0], v[SX]);
            };
            // tnext holds stale finite values on the last plane, where its weight is 0
            const cpx<T> f0 = tdx(0) + tdy(5) + w3(tz, tprev[2], tcur[2], tnext[2]);
            const cpx<T> f1 = tdx(5) + tdy(1) + w3(tz, tprev[1], tcur[1], tnext[1]);
            const cpx<T> f2 = tdx(4) + tdy(3) + w3(tz, tprev[0], tcur[0], tnext[0]);
            const long long p = (long long)k * plane + cell_xy;
            const cpx<T>* uk = us + (k & 3) * 3 * UP + (ly + 2) * UX + (lx + 2);
            const T wr = w2 * du;
            const cpx<T> g0 = wr * uk[0] - f0, g1 = wr * uk[UP] - f1, g2 = wr * uk[2 * UP] - f2;
            if constexpr (OUT == 0) {
                const long long cpitch = (long long)N3 * L2 * L1;
                cpx<T>* w_ = out + (long long)rhs * 3 * cpitch + zplane_offset(k, zbs, L2, L1) + zrow_offset(gy, zbs, L1) + gx;
                // written once and read by the next pass: non-temporal stores (measured 1-2 % faster)
                store_nt(&w_[0], g0);
                store_nt(&w_[cpitch], g1);
                store_nt(&w_[2 * cpitch], g2);
            } else {
                const cpx<T>* yr = y + so;
                cpx<T>* o_ = out + so;
                o_[p] = yr[p] - g0;
                o_[n + p] = yr[n + p] - g1;
                o_[2 * n + p] = yr[2 * n + p] - g2;
            }
        }
        if (k + 3 <= zend + 1) {
            store_plane(k + 3);
            if (k + 4 <= zend + 1) load_plane(k + 4);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            tprev[c] = tcur[c];
            tcur[c] = tnext[c];
        }
        __syncthreads();
    };
    for (int k = z0; k < zend; k += 2) {
        if constexpr (DB) {
            step(k, C, Cn, dro, dron);
            if (k + 1 < zend) step(k + 1, Cn, C, dron, dro);
        } else {
            step(k, C, C, dro, dron);
            if (k + 1 < zend) step(k + 1, C, C, dron, dro);
        }
    }
}

// Tile-packed contrast for k_contrast_zmarch with BX x BY tiles: stored value q of cell (x, y, z) goes to
// ((z TY + y / BY) TX + x / BX) K BX BY + q BX BY + (y mod BY) BX + x mod BX (TX x TY tiles per plane; the
// entries of cells outside the grid in edge tiles stay zero).  K = 21 stores every packed entry, K = 9 the
// orthotropic ones (kOrtho9).
template <typename T, int BX, int BY, int K>
__global__ void k_pack_contrast(const double* __restrict__ dc, T* __restrict__ dcp, int N1, int N2, int N3) {
    const long long n = (long long)N1 * N2 * N3;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int x = (int)(p % N1), y = (int)((p / N1) % N2), z = (int)(p / ((long long)N1 * N2));
    const int TX = (N1 + BX - 1) / BX, TY = (N2 + BY - 1) / BY;
    constexpr int TILE = BX * BY;
    const long long o = (((long long)z * TY + y / BY) * TX + x / BX) * K * TILE + (y % BY) * BX + x % BX;
    for (int q = 0; q < K; ++q) dcp[o + q * TILE] = (T)dc[(K == 21 ? q : kOrtho9[q]) * n + p];
}

// flag = 1 if any cell's contrast has a nonzero entry off the orthotropic pattern
__global__ void k_off_ortho(const double* __restrict__ dc, long long n, int* __restrict__ flag) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    for (int q = 0; q < 12; ++q)
        if (dc[kOffOrtho[q] * n + p] != 0.0) {
            atomicOr(flag, 1);
            return;
        }
}

// compact field f[slot][c][n] -> zero-padded work buffer at position r (layout of zplane_offset; data cells only)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_to_work(const cpx<T>* __restrict__ f, cpx<T>* __restrict__ work,
                                                      SlotMap sm, int nrhs, int N1, int N2, int N3, int L1, int L2,
                                                      int zbs) {
    const long long n = (long long)N1 * N2 * N3;
    const long long p = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n) return;
    const int i = (int)(p % N1);
    const int j = (int)((p / N1) % N2);
    const int k = (int)(p / ((long long)N1 * N2));
    const long long cpitch = (long long)N3 * L2 * L1;
    const long long wpos = zplane_offset(k, zbs, L2, L1) + zrow_offset(j, zbs, L1) + i;
    for (int r = 0; r < nrhs; ++r)
        for (int c = 0; c < 3; ++c) work[(3LL * r + c) * cpitch + wpos] = f[(3LL * sm.slot[r] + c) * n + p];
}

// Absorbing-layer weight of cell (i, j, k) (Eq 23-25): 1 - exp(-l^2 / (N_a h^2)) within d cells of a face,
// 1 elsewhere; l is the distance from the cell centre to where the ray from the model centre through it
// leaves the box (faces half a cell outside the outer cell centres), N_a the cell count along the axis of
// the face it crosses (the lower axis on ties).  Lengths in cells.
__device__ double taper_weight(int i, int j, int k, int N1, int N2, int N3, int d) {
    if (d <= 0) return 1.0;
    const int p[3] = {i, j, k}, n[3] = {N1, N2, N3};
    bool layer = false;
    for (int a = 0; a < 3; ++a) layer = layer || p[a] < d || p[a] > n[a] - 1 - d;
    if (!layer) return 1.0;
    double v[3], best = 0.0;
    int axis = -1;
    for (int a = 0; a < 3; ++a) {
        const double c = 0.5 * (n[a] - 1);
        v[a] = p[a] - c;
        if (v[a] == 0.0) continue;
        const double face = v[a] > 0.0 ? n[a] - 0.5 : -0.5;
        const double s = (face - c) / v[a];
        if (axis < 0 || s < best) best = s, axis = a;
    }
    if (axis < 0) return 1.0;
    const double l = (best - 1.0) * sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    return 1.0 - exp(-l * l / n[axis]);
}

// Gradient of a real misfit with respect to the contrast at every cell, for forward fields u and
// adjoint-side fields mu = conj(Gconv lambda_bar) (lambda_bar solving A^T lambda_bar = conj(P^H r)):
//   g21[JK](p) += -Re[conj(eps_J(mu)) eps_K(u) + (J != K) conj(eps_K(mu)) eps_J(u)]   (packed J <= K)
//   grho(p)    += w^2 Re[sum_c conj(mu_c) u_c]
// summed over the nrhs (u, mu) pairs.
__global__ __launch_bounds__(kThreads) void k_grad_contrast(const z128* __restrict__ u, const z128* __restrict__ mu,
                                                            double* __restrict__ g21, double* __restrict__ grho,
                                                            int nrhs, int N1, int N2, int N3, double inv_h, double w2,
                                                            int taper) {
    const long long n = (long long)N1 * N2 * N3;
    const long long p = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n) return;
    const int i = (int)(p % N1);
    const int j = (int)((p / N1) % N2);
    const int k = (int)(p / ((long long)N1 * N2));
    double acc[21];
#pragma unroll
    for (int q = 0; q < 21; ++q) acc[q] = 0.0;
    double ar = 0.0;
    for (int r = 0; r < nrhs; ++r) {
        const z128* ur = u + (long long)r * 3 * n;
        const z128* mr = mu + (long long)r * 3 * n;
        z128 eu[6], em[6];
        strain_at(ur, n, p, i, j, k, N1, N2, N3, inv_h, eu);
        strain_at(mr, n, p, i, j, k, N1, N2, N3, inv_h, em);
#pragma unroll
        for (int I = 0; I < 6; ++I)
#pragma unroll
            for (int J = I; J < 6; ++J) {
                double v = cmulc(em[I], eu[J]).x;
                if (J != I) v += cmulc(em[J], eu[I]).x;
                acc[packed(I, J)] -= v;
            }
#pragma unroll
        for (int c = 0; c < 3; ++c) ar += cmulc(mr[c * n + p], ur[c * n + p]).x;
    }
    // the contrast the operator sees is the input times the absorbing-layer weight
    const double tw = taper_weight(i, j, k, N1, N2, N3, taper);
#pragma unroll
    for (int q = 0; q < 21; ++q) g21[q * n + p] += tw * acc[q];
    grho[p] += tw * w2 * ar;
}

// a[p] = conj(a[p])
__global__ void k_conj(z128* __restrict__ a, long long m) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m) a[p].y = -a[p].y;
}

// Moment-tensor gradient: gM[r][J] = Re[e^{i w t0_r} conj(eps_J(mu_r)(s_r))] / h^3 (one thread per
// right-hand side; s_r inside the grid, checked on the host)
__global__ void k_grad_moment(const z128* __restrict__ mu, const int* __restrict__ src, const double* __restrict__ t0,
                              double* __restrict__ gM, int nrhs, int N1, int N2, int N3, double inv_h, double w,
                              double inv_h3) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    const long long n = (long long)N1 * N2 * N3;
    const int i = src[3 * r], j = src[3 * r + 1], k = src[3 * r + 2];
    const long long p = ((long long)k * N2 + j) * N1 + i;
    z128 eps[6];
    strain_at(mu + (long long)r * 3 * n, n, p, i, j, k, N1, N2, N3, inv_h, eps);
    double sn, cs;
    sincos(w * t0[r], &sn, &cs);
#pragma unroll
    for (int J = 0; J < 6; ++J) gM[6 * r + J] = (cs * eps[J].x + sn * eps[J].y) * inv_h3;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_strain_out(const cpx<T>* __restrict__ u, cpx<T>* __restrict__ eps_out,
                                                         int nrhs, int N1, int N2, int N3, T inv_h) {
    const long long n = (long long)N1 * N2 * N3;
    const long long p = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n) return;
    const int i = (int)(p % N1);
    const int j = (int)((p / N1) % N2);
    const int k = (int)(p / ((long long)N1 * N2));
    for (int r = 0; r < nrhs; ++r) {
        cpx<T> eps[6];
        strain_at(u + (long long)r * 3 * n, n, p, i, j, k, N1, N2, N3, inv_h, eps);
#pragma unroll
        for (int J = 0; J < 6; ++J) eps_out[((long long)r * 6 + J) * n + p] = eps[J];
    }
}

// total contrast = (input contrast + background fold) x absorbing-layer weight, in FP64 and FP32
__global__ void k_fold(const double* __restrict__ dc_in, const double* __restrict__ drho_in, double* __restrict__ dc,
                       double* __restrict__ drho, float* __restrict__ dc32, float* __restrict__ drho32, int N1, int N2,
                       int N3, int taper, const double* __restrict__ fold21) {
    const long long n = (long long)N1 * N2 * N3;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double w = taper_weight((int)(p % N1), (int)((p / N1) % N2), (int)(p / ((long long)N1 * N2)), N1, N2, N3,
                                  taper);
    for (int q = 0; q < 21; ++q) {
        const double v = (dc_in[q * n + p] + fold21[q]) * w;
        dc[q * n + p] = v;
        if (dc32) dc32[q * n + p] = (float)v;
    }
    drho[p] = drho_in[p] * w;
    if (drho32) drho32[p] = (float)(drho_in[p] * w);
}

template <typename T>
const T* contrast_of(const Ctx* c);
template <>
const double* contrast_of<double>(const Ctx* c) { return c->dc; }
template <>
const float* contrast_of<float>(const Ctx* c) { return c->dc32; }
template <typename T>
const T* contrast_packed_of(const Ctx* c);
template <>
const double* contrast_packed_of<double>(const Ctx* c) { return c->dcp; }
template <>
const float* contrast_packed_of<float>(const Ctx* c) { return c->dcp32; }
template <typename T>
const T* density_of(const Ctx* c);
template <>
const double* density_of<double>(const Ctx* c) { return c->drho; }
template <>
const float* density_of<float>(const Ctx* c) { return c->drho32; }

}  // namespace

// LS_CONTRAST=split selects the two-kernel contrast (strain/stress, then divergence) everywhere; both
// paths are kept under test.
bool use_fused_contrast() {
    static const bool fused = [] {
        const char* e = std::getenv("LS_CONTRAST");
        return !(e && std::strcmp(e, "split") == 0);
    }();
    return fused;
}

// z chunk of the fused kernel: blocks run in rounds of (CUs x resident blocks per CU), each block
// costs its chunk plus about three planes of prologue; pick the chunk (at least 8 planes) that
// minimises rounds x (chunk + 3).
inline int fused_z_chunk(int n3, long long cols, long long slots) {
    int best = n3;
    long long best_cost = -1;
    for (int nzc = std::min(8, n3); nzc <= n3; ++nzc) {
        const long long nb = cols * ((n3 + nzc - 1) / nzc);
        const long long cost = ((nb + slots - 1) / slots) * (nzc + 3);
        if (best_cost < 0 || cost < best_cost) best = nzc, best_cost = cost;
    }
    return best;
}

// Tile, block size and resident blocks per CU: c64 32x4 cells, 256 threads (128 owned, 72 halo), 47 KB
// LDS, three blocks per CU; c128 32x8 cells, 384 threads (256 owned, 80 halo), 145 KB LDS, one block.
template <typename T>
struct FusedShape;
template <>
struct FusedShape<float> {
    static constexpr int BX = 32, BY = 4, NT = 256, PER_CU = 3;
    static constexpr bool DB = true;
};
template <>
struct FusedShape<double> {
    static constexpr int BX = 32, BY = 8, NT = 384, PER_CU = 1;
    static constexpr bool DB = false;
};

template <typename T>
size_t packed_elems(const Ctx* c) {
    using S = FusedShape<T>;
    const size_t tx = (c->n1 + S::BX - 1) / S::BX, ty = (c->n2 + S::BY - 1) / S::BY;
    return tx * ty * (size_t)c->n3 * 21 * S::BX * S::BY;
}

template <typename T>
int pack_contrast(Ctx* c, T* dst) {
    using S = FusedShape<T>;
    LS_HIP(hipMemsetAsync(dst, 0, packed_elems<T>(c) * sizeof(T), c->stream));
    const long long n = c->ncell;
    const dim3 g((unsigned)((n + 255) / 256));
    if (c->contrast_k == 9)
        hipLaunchKernelGGL((k_pack_contrast<T, S::BX, S::BY, 9>), g, dim3(256), 0, c->stream, c->dc, dst, c->n1, c->n2, c->n3);
    else
        hipLaunchKernelGGL((k_pack_contrast<T, S::BX, S::BY, 21>), g, dim3(256), 0, c->stream, c->dc, dst, c->n1, c->n2,
                           c->n3);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

// values per cell of the packed contrast: 9 if the folded contrast has the orthotropic pattern at every cell,
// else 21; LS_CONTRAST_K=21 in the environment keeps the general form (both are kept under test)
int choose_contrast_k(Ctx* c) {
    const char* e = std::getenv("LS_CONTRAST_K");
    if (e && std::strcmp(e, "21") == 0) {
        c->contrast_k = 21;
        return LS_OK;
    }
    int* flag = (int*)c->stage;   // staging area of the context, free at set-up
    LS_HIP(hipMemsetAsync(flag, 0, sizeof(int), c->stream));
    hipLaunchKernelGGL(k_off_ortho, dim3((unsigned)((c->ncell + 255) / 256)), dim3(256), 0, c->stream, c->dc, c->ncell,
                       flag);
    LS_HIP(hipGetLastError());
    int h = 0;
    LS_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    LS_HIP(hipStreamSynchronize(c->stream));
    c->contrast_k = h ? 21 : 9;
    return LS_OK;
}

template <typename T>
SlotW2<T> slot_w2(const Ctx* c, const RhsSet& set) {
    SlotW2<T> sw{};
    for (int r = 0; r < set.n; ++r) {
        const double w = c->omega[set.freq[r]];
        sw.slot[r] = set.slot[r];
        sw.w2[r] = T(w * w);
    }
    return sw;
}

template <typename T, int OUT>
int launch_fused(Ctx* c, const RhsSet& set, const cpx<T>* u, cpx<T>* out, const cpx<T>* y) {
    using S = FusedShape<T>;
    const int nrhs = set.n;
    const int tx = (c->n1 + S::BX - 1) / S::BX, ty = (c->n2 + S::BY - 1) / S::BY;
    const long long cols = (long long)tx * ty * nrhs;
    const int nzc = fused_z_chunk(c->n3, cols, (long long)c->num_cu * S::PER_CU);
    const long long nb = cols * ((c->n3 + nzc - 1) / nzc);
    const unsigned nbl = (unsigned)((nb + 7) / 8 * 8);
    c->prof.begin(c->stream, OUT == 0 ? LS_PNAME(T, "contrast_fused") : LS_PNAME(T, "contrast_fused_T"), nrhs);
    if (c->contrast_k == 9)
        hipLaunchKernelGGL((k_contrast_zmarch<T, S::BX, S::BY, S::NT, S::PER_CU, S::DB, OUT, 9>), dim3(nbl), dim3(S::NT), 0,
                           c->stream, u, contrast_packed_of<T>(c), density_of<T>(c), out, y, slot_w2<T>(c, set), nrhs, c->n1,
                           c->n2, c->n3, c->L1, c->L2, T(1.0 / c->h), tx, ty, nzc, nb, c->zbs);
    else
        hipLaunchKernelGGL((k_contrast_zmarch<T, S::BX, S::BY, S::NT, S::PER_CU, S::DB, OUT, 21>), dim3(nbl), dim3(S::NT), 0,
                           c->stream, u, contrast_packed_of<T>(c), density_of<T>(c), out, y, slot_w2<T>(c, set), nrhs, c->n1,
                           c->n2, c->n3, c->L1, c->L2, T(1.0 / c->h), tx, ty, nzc, nb, c->zbs);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

template <typename T>
int contrast_to_work(Ctx* c, const RhsSet& set, const cpx<T>* u, cpx<T>* work, cpx<T>* tau) {
    if (use_fused_contrast()) return launch_fused<T, 0>(c, set, u, work, nullptr);
    const long long n = c->ncell;
    // XCD-aware order: grid padded to a multiple of 8, neighbouring cells share an L2
    const unsigned nb = (unsigned)(((n + kThreads - 1) / kThreads + 7) / 8 * 8);
    const T inv_h = T(1.0 / c->h);
    const SlotW2<T> sw = slot_w2<T>(c, set);
    c->prof.begin(c->stream, LS_PNAME(T, "contrast_strain_stress"), set.n);
    hipLaunchKernelGGL((k_strain_stress<T>), dim3(nb), dim3(kThreads), 0, c->stream, u, tau, contrast_of<T>(c),
                       slot_map(set), set.n, c->n1, c->n2, c->n3, inv_h);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    c->prof.begin(c->stream, LS_PNAME(T, "contrast_divergence"), set.n);
    hipLaunchKernelGGL((k_divergence<T, 0>), dim3(nb), dim3(kThreads), 0, c->stream, tau, u, density_of<T>(c), work,
                       sw, set.n, c->n1, c->n2, c->n3, c->L1, c->L2, inv_h, nullptr, c->zbs);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

template int contrast_to_work<double>(Ctx*, const RhsSet&, const z128*, z128*, z128*);
template int contrast_to_work<float>(Ctx*, const RhsSet&, const z64*, z64*, z64*);

// out = y - B g  (the last step of the transposed operator A^T y = y - B Gconv y, with g = Gconv y)
template <typename T>
int contrast_transposed_epilogue(Ctx* c, const RhsSet& set, const cpx<T>* g, const cpx<T>* y, cpx<T>* out,
                                 cpx<T>* tau) {
    if (use_fused_contrast()) return launch_fused<T, 1>(c, set, g, out, y);
    const long long n = c->ncell;
    const unsigned nb = (unsigned)(((n + kThreads - 1) / kThreads + 7) / 8 * 8);
    const T inv_h = T(1.0 / c->h);
    c->prof.begin(c->stream, LS_PNAME(T, "contrast_strain_stress"), set.n);
    hipLaunchKernelGGL((k_strain_stress<T>), dim3(nb), dim3(kThreads), 0, c->stream, g, tau, contrast_of<T>(c),
                       slot_map(set), set.n, c->n1, c->n2, c->n3, inv_h);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    c->prof.begin(c->stream, LS_PNAME(T, "contrast_divergence_T"), set.n);
    hipLaunchKernelGGL((k_divergence<T, 1>), dim3(nb), dim3(kThreads), 0, c->stream, tau, g, density_of<T>(c), out,
                       slot_w2<T>(c, set), set.n, c->n1, c->n2, c->n3, c->L1, c->L2, inv_h, y, c->zbs);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

template int contrast_transposed_epilogue<double>(Ctx*, const RhsSet&, const z128*, const z128*, z128*, z128*);
template int contrast_transposed_epilogue<float>(Ctx*, const RhsSet&, const z64*, const z64*, z64*, z64*);

template <typename T>
int to_work(Ctx* c, const RhsSet& set, const cpx<T>* f, cpx<T>* work) {
    const long long n = c->ncell;
    const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
    c->prof.begin(c->stream, LS_PNAME(T, "to_work"), set.n);
    hipLaunchKernelGGL((k_to_work<T>), dim3(nb), dim3(kThreads), 0, c->stream, f, work, slot_map(set), set.n, c->n1,
                       c->n2, c->n3, c->L1, c->L2, c->zbs);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

template int to_work<double>(Ctx*, const RhsSet&, const z128*, z128*);
template int to_work<float>(Ctx*, const RhsSet&, const z64*, z64*);

int grad_contrast_launch(Ctx* c, int i_omega, const z128* u, const z128* mu, int nrhs, double* g21, double* grho) {
    const long long n = c->ncell;
    const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
    const double w = c->omega[i_omega];
    c->prof.begin(c->stream, "grad_contrast.c128", nrhs);
    hipLaunchKernelGGL(k_grad_contrast, dim3(nb), dim3(kThreads), 0, c->stream, u, mu, g21, grho, nrhs, c->n1, c->n2,
                       c->n3, 1.0 / c->h, w * w, c->taper);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

int conj_launch(Ctx* c, z128* a, long long m) {
    hipLaunchKernelGGL(k_conj, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, c->stream, a, m);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

// src: host [nrhs][3] cells (inside the grid); t0: host [nrhs]; gM: host [nrhs][6].  Stages src and t0
// through the context's staging area and waits for the result.
int grad_moment_launch(Ctx* c, int i_omega, const z128* mu, int nrhs, const int* src, const double* t0, double* gM) {
    char* st = (char*)c->stage;
    int* dsrc = (int*)st;
    double* dt0 = (double*)(st + 1024);
    double* dgM = (double*)(st + 2048);
    LS_HIP(hipMemcpyAsync(dsrc, src, 3 * nrhs * sizeof(int), hipMemcpyHostToDevice, c->stream));
    LS_HIP(hipMemcpyAsync(dt0, t0, nrhs * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const double h3 = c->h * c->h * c->h;
    hipLaunchKernelGGL(k_grad_moment, dim3((unsigned)((nrhs + 63) / 64)), dim3(64), 0, c->stream, mu, dsrc, dt0, dgM,
                       nrhs, c->n1, c->n2, c->n3, 1.0 / c->h, c->omega[i_omega], 1.0 / h3);
    LS_HIP(hipGetLastError());
    LS_HIP(hipMemcpyAsync(gM, dgM, 6 * nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LS_HIP(hipStreamSynchronize(c->stream));
    return LS_OK;
}

int strain_launch(Ctx* c, const z128* u, z128* eps, int nrhs) {
    const long long n = c->ncell;
    const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((k_strain_out<double>), dim3(nb), dim3(kThreads), 0, c->stream, u, eps, nrhs, c->n1, c->n2,
                       c->n3, 1.0 / c->h);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

size_t contrast_packed_elems(const Ctx* c, bool fp32) {
    return fp32 ? packed_elems<float>(c) : packed_elems<double>(c);
}

int fold_background(Ctx* c, const double* dc_in, const double* drho_in, const double fold21[21]) {
    double* dfold = nullptr;
    LS_HIP(hipMallocAsync((void**)&dfold, 21 * sizeof(double), c->stream));
    LS_HIP(hipMemcpyAsync(dfold, fold21, 21 * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const long long n = c->ncell;
    hipLaunchKernelGGL(k_fold, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, dc_in, drho_in, c->dc, c->drho,
                       c->dc32, c->drho32, c->n1, c->n2, c->n3, c->taper, dfold);
    LS_HIP(hipGetLastError());
    int rc = choose_contrast_k(c);
    if (rc == LS_OK) rc = pack_contrast<double>(c, c->dcp);
    if (rc == LS_OK && c->dcp32) rc = pack_contrast<float>(c, c->dcp32);
    LS_HIP(hipStreamSynchronize(c->stream));
    LS_HIP(hipFreeAsync(dfold, c->stream));
    LS_HIP(hipStreamSynchronize(c->stream));
    return rc;
}

}  // namespace ls
