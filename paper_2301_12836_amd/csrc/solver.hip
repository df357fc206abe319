// BiCGSTAB for A u = u0 (Eq 21-22) over a batch of right-hand sides, and its mixed-precision
// form: an FP64 iterative-refinement loop (true residual b - A u with the FP64 operator) around
// an inner BiCGSTAB on the FP32 operator with FP64 inner products.
//
// Van der Vorst's Bi-CGSTAB, unpreconditioned, shadow residual r^ = r0, Hermitian products:
//   rho = r^H r;  beta = (rho / rho_old)(alpha / omega);  p = r + beta (p - omega v);  v = A p;
//   alpha = rho / (r^H v);  s = r - alpha v  [stop if ||s|| <= tol ||b||: x += alpha p];
//   t = A s;  omega = (t^H s)/(t^H t);  x += alpha p + omega s;  r = s - omega t.
// Every scalar lives on the device: each reduction ends in a one-block kernel that also updates
// the right-hand side's scalars and its active flag, so an iteration is a fixed sequence of
// stream-ordered launches; the host only reads the flags to decide when to stop.  Reductions
// use a fixed number of blocks and a fixed tree, so results are bitwise reproducible.
// Every kernel covers the systems of a slot map (grid dimension y, or x for the one-block kernels): the
// systems still iterating, at any mix of frequencies, so a system computes the same iterates whichever
// other systems share its launches, and converged systems drop out of the launches.
#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>

#include "common.h"

namespace ls {

namespace {

constexpr int kThreads = 256;

// state layout per right-hand side
enum {
    S_RHO = 0,       // complex
    S_ALPHA = 2,     // complex
    S_OMEGA = 4,     // complex
    S_BETA = 6,      // complex
    S_BNORM2 = 8,
    S_SNORM2 = 9,
    S_RNORM2 = 10,
    S_ACTIVE = 11,   // 1: iterating
    S_FLAG = 12,     // 0 ok, 1 converged at a half step (x += alpha p pending), 2 breakdown, 3 non-finite
    S_ITERS = 13,
    S_TOL2 = 14,     // tol^2 ||b||^2
    S_DONE = 15      // 1: converged
};

__device__ __forceinline__ double2 block_reduce2(double a, double b, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = a;
    sh[kThreads + tid] = b;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            sh[tid] += sh[tid + w];
            sh[kThreads + tid] += sh[kThreads + tid + w];
        }
        __syncthreads();
    }
    return make_double2(sh[0], sh[kThreads]);
}

__device__ __forceinline__ void write_partials(double* partials, int r, int slot, double a, double b, double* sh) {
    const double2 s = block_reduce2(a, b, sh);
    if (threadIdx.x == 0) {
        partials[((long long)r * kRedSlots + slot) * kRedBlocks + blockIdx.x] = s.x;
        partials[((long long)r * kRedSlots + slot + 1) * kRedBlocks + blockIdx.x] = s.y;
    }
}

template <typename T>
__device__ __forceinline__ cpx<double> wide(cpx<T> a) {
    return {(double)a.x, (double)a.y};
}

// Loop helper: element indices of this thread for one right-hand side of length m; the system is
// rr = sm.slot[blockIdx.y].
#define LS_FOR_ELEMS(m) for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < (m); e += (long long)kRedBlocks * kThreads)

// The Bi-CGSTAB updates stream their vectors once: non-temporal access (about 1 % per solve step).

// r = b - ax (ax may be null), rhat = r, p = v = 0; partials: ||b||^2, ||r||^2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_init(const cpx<T>* __restrict__ b, const cpx<T>* __restrict__ ax,
                                                   cpx<T>* __restrict__ r, cpx<T>* __restrict__ rhat,
                                                   cpx<T>* __restrict__ p, cpx<T>* __restrict__ v, long long m,
                                                   double* partials, SlotMap sm) {
    __shared__ double sh[2 * kThreads];
    const int rr = sm.slot[blockIdx.y];
    const long long off = (long long)rr * m;
    double bb = 0, nr = 0;
    LS_FOR_ELEMS(m) {
        const cpx<T> bv = b[off + e];
        cpx<T> rv = bv;
        if (ax) rv = bv - ax[off + e];
        r[off + e] = rv;
        rhat[off + e] = rv;
        p[off + e] = {T(0), T(0)};
        v[off + e] = {T(0), T(0)};
        bb += (double)bv.x * bv.x + (double)bv.y * bv.y;
        nr += (double)rv.x * rv.x + (double)rv.y * rv.y;
    }
    write_partials(partials, rr, 0, bb, nr, sh);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_update_p(const cpx<T>* __restrict__ r, cpx<T>* __restrict__ p,
                                                       const cpx<T>* __restrict__ v, long long m,
                                                       const double* __restrict__ state, SlotMap sm) {
    const int rr = sm.slot[blockIdx.y];
    const double* st = state + rr * kStateLen;
    if (st[S_ACTIVE] == 0.0) return;
    const cpx<T> beta = {(T)st[S_BETA], (T)st[S_BETA + 1]};
    const cpx<T> om = {(T)st[S_OMEGA], (T)st[S_OMEGA + 1]};
    const long long off = (long long)rr * m;
    LS_FOR_ELEMS(m) {
        const cpx<T> pv = load_nt(&p[off + e]), vv = load_nt(&v[off + e]);
        store_nt(&p[off + e], load_nt(&r[off + e]) + beta * (pv - om * vv));
    }
}

// partials: r^H v (complex)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot(const cpx<T>* __restrict__ a, const cpx<T>* __restrict__ b,
                                                  long long m, const double* __restrict__ state, double* partials,
                                                  SlotMap sm) {
    __shared__ double sh[2 * kThreads];
    const int rr = sm.slot[blockIdx.y];
    if (state[rr * kStateLen + S_ACTIVE] == 0.0) return;
    const long long off = (long long)rr * m;
    double re = 0, im = 0;
    LS_FOR_ELEMS(m) {
        const cpx<double> z = cmulc(wide(a[off + e]), wide(b[off + e]));
        re += z.x;
        im += z.y;
    }
    write_partials(partials, rr, 0, re, im, sh);
}

// s = r - alpha v; partials ||s||^2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update_s(const cpx<T>* __restrict__ r, const cpx<T>* __restrict__ v,
                                                       cpx<T>* __restrict__ s, long long m,
                                                       const double* __restrict__ state, double* partials,
                                                       SlotMap sm) {
    __shared__ double sh[2 * kThreads];
    const int rr = sm.slot[blockIdx.y];
    const double* st = state + rr * kStateLen;
    if (st[S_ACTIVE] == 0.0) return;
    const cpx<T> al = {(T)st[S_ALPHA], (T)st[S_ALPHA + 1]};
    const long long off = (long long)rr * m;
    double ss = 0;
    LS_FOR_ELEMS(m) {
        const cpx<T> sv = load_nt(&r[off + e]) - al * load_nt(&v[off + e]);
        store_nt(&s[off + e], sv);
        ss += (double)sv.x * sv.x + (double)sv.y * sv.y;
    }
    write_partials(partials, rr, 0, ss, 0.0, sh);
}

// Right preconditioning by the block-Jacobi matrix M (or M^T for the transposed operator): the operator
// is applied to M^-1 p and M^-1 s, which the updates of p and s form cell by cell (the three components of a
// cell sit n apart) while they write p and s; x takes its steps along M^-1 p and M^-1 s.
#define LS_FOR_CELLS(n) for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < (n); e += (long long)kRedBlocks * kThreads)

template <typename T>
__device__ __forceinline__ void minv_apply(const cpx<T>* __restrict__ M, long long n, long long e, int trans,
                                           const cpx<T> v[3], cpx<T> y[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cpx<T> acc = {T(0), T(0)};
#pragma unroll
        for (int b = 0; b < 3; ++b) acc = acc + M[(trans ? 3 * b + a : 3 * a + b) * n + e] * v[b];
        y[a] = acc;
    }
}

// p = r + beta (p - omega v);  ph = M^-1 p
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update_p_pre(const cpx<T>* __restrict__ r, cpx<T>* __restrict__ p,
                                                           const cpx<T>* __restrict__ v, cpx<T>* __restrict__ ph,
                                                           long long n, const double* __restrict__ state,
                                                           SlotMap sm, PreTabs<T> pt) {
    const int rr = sm.slot[blockIdx.y];
    const double* st = state + rr * kStateLen;
    if (st[S_ACTIVE] == 0.0) return;
    const cpx<T> beta = {(T)st[S_BETA], (T)st[S_BETA + 1]};
    const cpx<T> om = {(T)st[S_OMEGA], (T)st[S_OMEGA + 1]};
    const cpx<T>* M = pt.m[blockIdx.y];
    const long long off = (long long)rr * 3 * n;
    LS_FOR_CELLS(n) {
        cpx<T> pn[3], y[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const long long q = off + a * n + e;
            pn[a] = load_nt(&r[q]) + beta * (load_nt(&p[q]) - om * load_nt(&v[q]));
            store_nt(&p[q], pn[a]);
        }
        minv_apply(M, n, e, pt.trans, pn, y);
#pragma unroll
        for (int a = 0; a < 3; ++a) store_nt(&ph[off + a * n + e], y[a]);
    }
}

// s = r - alpha v;  sh = M^-1 s;  partials ||s||^2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update_s_pre(const cpx<T>* __restrict__ r, const cpx<T>* __restrict__ v,
                                                           cpx<T>* __restrict__ s, cpx<T>* __restrict__ sh,
                                                           long long n, const double* __restrict__ state,
                                                           double* partials, SlotMap sm, PreTabs<T> pt) {
    __shared__ double shm[2 * kThreads];
    const int rr = sm.slot[blockIdx.y];
    const double* st = state + rr * kStateLen;
    if (st[S_ACTIVE] == 0.0) return;
    const cpx<T> al = {(T)st[S_ALPHA], (T)st[S_ALPHA + 1]};
    const cpx<T>* M = pt.m[blockIdx.y];
    const long long off = (long long)rr * 3 * n;
    double ss = 0;
    LS_FOR_CELLS(n) {
        cpx<T> sv[3], y[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const long long q = off + a * n + e;
            sv[a] = load_nt(&r[q]) - al * load_nt(&v[q]);
            store_nt(&s[q], sv[a]);
            ss += (double)sv[a].x * sv[a].x + (double)sv[a].y * sv[a].y;
        }
        minv_apply(M, n, e, pt.trans, sv, y);
#pragma unroll
        for (int a = 0; a < 3; ++a) store_nt(&sh[off + a * n + e], y[a]);
    }
    write_partials(partials, rr, 0, ss, 0.0, shm);
}

// x += alpha p for the systems that converged at the half step
template <typename T, typename X>
__global__ __launch_bounds__(kThreads) void k_update_x_half(cpx<X>* __restrict__ x, const cpx<T>* __restrict__ p,
                                                            long long m, double* __restrict__ state, SlotMap sm) {
    const int rr = sm.slot[blockIdx.y];
    const double* st = state + rr * kStateLen;
    if (st[S_FLAG] != 1.0) return;
    const cpx<X> al = {(X)st[S_ALPHA], (X)st[S_ALPHA + 1]};
    const long long off = (long long)rr * m;
    LS_FOR_ELEMS(m) {
        const cpx<T> pv = p[off + e];
        x[off + e] = x[off + e] + al * cpx<X>{(X)pv.x, (X)pv.y};
    }
}

// partials: t^H s (complex), t^H t
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot_ts(const cpx<T>* __restrict__ t, const cpx<T>* __restrict__ s,
                                                     long long m, const double* __restrict__ state,
                                                     double* partials, SlotMap sm) {
    __shared__ double sh[2 * kThreads];
    const int rr = sm.slot[blockIdx.y];
    if (state[rr * kStateLen + S_ACTIVE] == 0.0) return;
    const long long off = (long long)rr * m;
    double re = 0, im = 0, tt = 0;
    LS_FOR_ELEMS(m) {
        const cpx<double> tv = wide(t[off + e]);
        const cpx<double> z = cmulc(tv, wide(s[off + e]));
        re += z.x;
        im += z.y;
        tt += tv.x * tv.x + tv.y * tv.y;
    }
    write_partials(partials, rr, 0, re, im, sh);
    write_partials(partials, rr, 2, tt, 0.0, sh);
}

// x += alpha p + omega s; r = s - omega t; partials ||r||^2, r^H r (complex)
// PRE: the x step takes xs (M^-1 s) instead of s
template <typename T, typename X, bool PRE>
__global__ __launch_bounds__(kThreads) void k_update_xr(cpx<X>* __restrict__ x, const cpx<T>* __restrict__ p,
                                                        const cpx<T>* __restrict__ s, const cpx<T>* __restrict__ xs,
                                                        const cpx<T>* __restrict__ t, cpx<T>* __restrict__ r,
                                                        const cpx<T>* __restrict__ rhat, long long m,
                                                        const double* __restrict__ state, double* partials,
                                                        SlotMap sm) {
    __shared__ double sh[2 * kThreads];
    const int rr = sm.slot[blockIdx.y];
    const double* st = state + rr * kStateLen;
    if (st[S_ACTIVE] == 0.0) return;
    const cpx<X> alx = {(X)st[S_ALPHA], (X)st[S_ALPHA + 1]};
    const cpx<X> omx = {(X)st[S_OMEGA], (X)st[S_OMEGA + 1]};
    const cpx<T> om = {(T)st[S_OMEGA], (T)st[S_OMEGA + 1]};
    const long long off = (long long)rr * m;
    double nr = 0, re = 0, im = 0;
    LS_FOR_ELEMS(m) {
        const cpx<T> pv = load_nt(&p[off + e]), sv = load_nt(&s[off + e]);
        const cpx<T> xsv = PRE ? load_nt(&xs[off + e]) : sv;
        const cpx<X> xv = load_nt(&x[off + e]);
        store_nt(&x[off + e], xv + alx * cpx<X>{(X)pv.x, (X)pv.y} + omx * cpx<X>{(X)xsv.x, (X)xsv.y});
        const cpx<T> rv = sv - om * load_nt(&t[off + e]);
        store_nt(&r[off + e], rv);
        const cpx<double> rw = wide(rv);
        nr += rw.x * rw.x + rw.y * rw.y;
        const cpx<double> z = cmulc(wide(load_nt(&rhat[off + e])), rw);
        re += z.x;
        im += z.y;
    }
    write_partials(partials, rr, 0, nr, 0.0, sh);
    write_partials(partials, rr, 2, re, im, sh);
}

// r = b - ax; partials ||r||^2, ||b||^2   (FP64 true residual)
__global__ __launch_bounds__(kThreads) void k_residual(const z128* __restrict__ b, const z128* __restrict__ ax,
                                                       z128* __restrict__ r, long long m, double* partials,
                                                       SlotMap sm) {
    __shared__ double sh[2 * kThreads];
    const int rr = sm.slot[blockIdx.y];
    const long long off = (long long)rr * m;
    double nr = 0, bb = 0;
    LS_FOR_ELEMS(m) {
        const z128 bv = b[off + e];
        const z128 rv = bv - ax[off + e];
        if (r) r[off + e] = rv;
        nr += rv.x * rv.x + rv.y * rv.y;
        bb += bv.x * bv.x + bv.y * bv.y;
    }
    write_partials(partials, rr, 0, nr, bb, sh);
}

// out = scale_r * in (FP64 -> FP32), optionally zero a second buffer
__global__ __launch_bounds__(kThreads) void k_to32(const z128* __restrict__ in, z64* __restrict__ out, long long m,
                                                   const double* __restrict__ scale, z64* __restrict__ zero_out,
                                                   SlotMap sm) {
    const int rr = sm.slot[blockIdx.y];
    const double sc = scale[rr];
    const long long off = (long long)rr * m;
    LS_FOR_ELEMS(m) {
        const z128 v = in[off + e];
        out[off + e] = {(float)(sc * v.x), (float)(sc * v.y)};
        if (zero_out) zero_out[off + e] = {0.f, 0.f};
    }
}

// x += scale_r * d (FP32 correction into the FP64 iterate)
__global__ __launch_bounds__(kThreads) void k_add32(z128* __restrict__ x, const z64* __restrict__ d, long long m,
                                                    const double* __restrict__ scale, SlotMap sm) {
    const int rr = sm.slot[blockIdx.y];
    const double sc = scale[rr];
    if (sc == 0.0) return;
    const long long off = (long long)rr * m;
    LS_FOR_ELEMS(m) {
        const z64 dv = d[off + e];
        x[off + e] = x[off + e] + sc * z128{(double)dv.x, (double)dv.y};
    }
}

__global__ void k_copy(const z128* __restrict__ a, z128* __restrict__ b, long long m, SlotMap sm) {
    const long long off = (long long)sm.slot[blockIdx.y] * m;
    LS_FOR_ELEMS(m) { b[off + e] = a[off + e]; }
}

// Sum the kRedBlocks partials of each slot in a fixed order, then advance the scalars.
enum Phase { PH_INIT = 0, PH_ALPHA = 1, PH_S = 2, PH_OMEGA = 3, PH_RHO = 4, PH_RESID = 5 };

// partials: [rhs][kRedSlots][nparts] (nparts = kRedBlocks, or the x-inverse epilogue's blocks per right-hand
// side for the inner products fused there).  PH_INIT: tolerance tol2v[rr] (squared) per system, or tol2.
// PH_RESID: out[rr] and out[kRedBlocks + rr] by slot.
__global__ __launch_bounds__(kThreads) void k_finalize(const double* __restrict__ partials, int nparts,
                                                       double* __restrict__ state, int phase, int nslots, double tol2,
                                                       double* __restrict__ out, const double* __restrict__ tol2v,
                                                       SlotMap sm) {
    __shared__ double sh[kRedSlots][kThreads];
    const int rr = sm.slot[blockIdx.x];
    double* st = state + rr * kStateLen;
    const int tid = threadIdx.x;
    if (phase != PH_INIT && phase != PH_RESID && st[S_ACTIVE] == 0.0) return;
    for (int q = 0; q < nslots; ++q) {
        double a = 0;
        for (int k = tid; k < nparts; k += kThreads) a += partials[((long long)rr * kRedSlots + q) * nparts + k];
        sh[q][tid] = a;
    }
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (tid < w)
            for (int q = 0; q < nslots; ++q) sh[q][tid] += sh[q][tid + w];
        __syncthreads();
    }
    if (tid != 0) return;
    double v[kRedSlots];
    for (int q = 0; q < nslots; ++q) v[q] = sh[q][0];
    auto bad = [](double x) { return !(fabs(x) <= 1.7e308); };
    switch (phase) {
        case PH_INIT: {  // v = (||b||^2, ||r||^2)
            if (tol2v) tol2 = tol2v[rr];
            st[S_BNORM2] = v[0];
            st[S_RNORM2] = v[1];
            st[S_RHO] = v[1];
            st[S_RHO + 1] = 0.0;
            st[S_ALPHA] = 1.0;
            st[S_ALPHA + 1] = 0.0;
            st[S_OMEGA] = 1.0;
            st[S_OMEGA + 1] = 0.0;
            st[S_BETA] = 0.0;
            st[S_BETA + 1] = 0.0;
            st[S_TOL2] = tol2 * v[0];
            st[S_ITERS] = 0.0;
            st[S_FLAG] = 0.0;
            const bool done = v[1] <= tol2 * v[0];
            st[S_DONE] = done ? 1.0 : 0.0;
            st[S_ACTIVE] = done ? 0.0 : 1.0;
            if (bad(v[0]) || bad(v[1])) {
                st[S_FLAG] = 3.0;
                st[S_ACTIVE] = 0.0;
            }
            break;
        }
        case PH_ALPHA: {  // v = r^H v
            const double dr = v[0], di = v[1];
            const double den = dr * dr + di * di;
            st[S_ITERS] += 1.0;
            if (!(den > 0.0) || bad(den)) {
                st[S_FLAG] = bad(den) ? 3.0 : 2.0;
                st[S_ACTIVE] = 0.0;
                break;
            }
            const double rr_ = st[S_RHO], ri = st[S_RHO + 1];
            st[S_ALPHA] = (rr_ * dr + ri * di) / den;
            st[S_ALPHA + 1] = (ri * dr - rr_ * di) / den;
            break;
        }
        case PH_S: {  // v = ||s||^2
            st[S_SNORM2] = v[0];
            if (bad(v[0])) {
                st[S_FLAG] = 3.0;
                st[S_ACTIVE] = 0.0;
            } else if (v[0] <= st[S_TOL2]) {
                st[S_FLAG] = 1.0;
                st[S_ACTIVE] = 0.0;
                st[S_DONE] = 1.0;
                st[S_RNORM2] = v[0];
            }
            break;
        }
        case PH_OMEGA: {  // v = (t^H s re, im, t^H t)
            const double tt = v[2];
            if (!(tt > 0.0) || bad(tt)) {
                st[S_FLAG] = bad(tt) ? 3.0 : 2.0;
                st[S_ACTIVE] = 0.0;
                break;
            }
            st[S_OMEGA] = v[0] / tt;
            st[S_OMEGA + 1] = v[1] / tt;
            break;
        }
        case PH_RHO: {  // v = (||r||^2, 0, r^H r re, im)
            st[S_RNORM2] = v[0];
            const double nr = v[2], ni = v[3];
            if (bad(v[0])) {
                st[S_FLAG] = 3.0;
                st[S_ACTIVE] = 0.0;
                break;
            }
            if (v[0] <= st[S_TOL2]) {
                st[S_ACTIVE] = 0.0;
                st[S_DONE] = 1.0;
                break;
            }
            // beta = (rho_new / rho)(alpha / omega)
            const double pr = st[S_RHO], pi = st[S_RHO + 1];
            const double ar = st[S_ALPHA], ai = st[S_ALPHA + 1];
            const double orr = st[S_OMEGA], oi = st[S_OMEGA + 1];
            const double d1 = pr * pr + pi * pi, d2 = orr * orr + oi * oi;
            if (!(d1 > 0.0) || !(d2 > 0.0) || !(nr * nr + ni * ni > 0.0)) {
                st[S_FLAG] = 2.0;
                st[S_ACTIVE] = 0.0;
                break;
            }
            const double q1r = (nr * pr + ni * pi) / d1, q1i = (ni * pr - nr * pi) / d1;
            const double q2r = (ar * orr + ai * oi) / d2, q2i = (ai * orr - ar * oi) / d2;
            st[S_BETA] = q1r * q2r - q1i * q2i;
            st[S_BETA + 1] = q1r * q2i + q1i * q2r;
            st[S_RHO] = nr;
            st[S_RHO + 1] = ni;
            break;
        }
        case PH_RESID: {  // v = (||r||^2, ||b||^2) -> out[rr] = ||r|| / ||b||
            out[rr] = v[1] > 0.0 ? sqrt(v[0] / v[1]) : 0.0;
            out[kRedBlocks + rr] = sqrt(v[0]);
            break;
        }
    }
}

__global__ void k_clear_half(double* state, int n, SlotMap sm) {
    if ((int)threadIdx.x >= n) return;
    const int rr = sm.slot[threadIdx.x];
    if (state[rr * kStateLen + S_FLAG] == 1.0) state[rr * kStateLen + S_FLAG] = 0.0;
}

struct Vecs64 {
    z128 *r, *rhat, *p, *v, *s, *t;
};
struct Vecs32 {
    z64 *r, *rhat, *p, *v, *s, *t;
};

dim3 vgrid(int nrhs) { return dim3(kRedBlocks, nrhs); }

int finalize(Ctx* c, const RhsSet& set, int phase, int nslots, double tol2 = 0.0, double* out = nullptr,
             const double* parts = nullptr, int nparts = kRedBlocks, const double* tol2v = nullptr) {
    hipLaunchKernelGGL(k_finalize, dim3(set.n), dim3(kThreads), 0, c->stream, parts ? parts : c->partials, nparts,
                       c->state, phase, nslots, tol2, out, tol2v, slot_map(set));
    LS_HIP(hipGetLastError());
    return LS_OK;
}

// the systems of `all` whose state says they are still iterating (host copy of the state)
RhsSet active_subset(const RhsSet& all, const double* host_state) {
    RhsSet a;
    for (int r = 0; r < all.n; ++r)
        if (host_state[(size_t)all.slot[r] * kStateLen + S_ACTIVE] != 0.0) {
            a.slot[a.n] = all.slot[r];
            a.freq[a.n] = all.freq[r];
            ++a.n;
        }
    return a;
}

bool same_set(const RhsSet& a, const RhsSet& b) {
    if (a.n != b.n) return false;
    for (int r = 0; r < a.n; ++r)
        if (a.slot[r] != b.slot[r] || a.freq[r] != b.freq[r]) return false;
    return true;
}

RhsSet one_slot(int q) {
    RhsSet s;
    s.n = 1;
    s.slot[0] = q;
    return s;
}

// The iterate with the smallest recursive residual seen, saved whenever that residual halves (so at most
// about log2(1/tol) copies per system): a solve that stops short of tol returns it, not its last iterate.
struct BestIterate {
    z128* x = nullptr;           // [nrhs][3 ncell]
    std::vector<double> r2;      // residual norm^2 of the saved iterate, per system
    int save(Ctx* c, const z128* from, int q, long long m) {
        hipLaunchKernelGGL(k_copy, dim3(kRedBlocks, 1), dim3(kThreads), 0, c->stream, from, x, m,
                           slot_map(one_slot(q)));
        LS_HIP(hipGetLastError());
        return LS_OK;
    }
    int restore(Ctx* c, z128* to, int q, long long m) {
        hipLaunchKernelGGL(k_copy, dim3(kRedBlocks, 1), dim3(kThreads), 0, c->stream, (const z128*)x, to, m,
                           slot_map(one_slot(q)));
        LS_HIP(hipGetLastError());
        return LS_OK;
    }
};

// Iterations without a 10 % gain on the best residual norm after which an FP32 inner solve stops:
// 30 once the residual is within 1e-4 of the inner right-hand side (FP32's attainable accuracy is
// near), 300 above that, where hard systems (high frequency, many wavelengths) cross long plateaus.
inline int stall_window(double r2, double b2) { return r2 < 1e-8 * b2 ? 30 : 300; }

// Generic BiCGSTAB over the systems of `all` (their slots in every vector).  T: vector precision, X: iterate
// precision (x is cpx<X>), ApplyFn(set, in, out) applies the operator to the systems of a set.  tol2v:
// device array of each slot's squared relative tolerance.  Every iteration covers only the systems still
// iterating; the iteration over a given set is captured once into a graph and replayed until the set
// shrinks.  iters: per slot.
template <typename T, typename X, typename ApplyFn>
int bicgstab(Ctx* c, const RhsSet& all, const cpx<T>* b, cpx<X>* x, const cpx<T>* ax0, cpx<T>* r, cpx<T>* rhat,
             cpx<T>* p, cpx<T>* v, cpx<T>* s, cpx<T>* t, const double* tol2v, int maxit, ApplyFn apply,
             std::vector<int>& iters, const double* hscale = nullptr, BestIterate* keep = nullptr, bool fuse = false,
             cpx<T>* ph = nullptr, cpx<T>* sh = nullptr, int pre = 0) {
    const long long m = (long long)c->field_elems();
    int ns = 0;   // slots spanned by the set (state entries read back)
    for (int q = 0; q < all.n; ++q) ns = std::max(ns, all.slot[q] + 1);
    // r^H v and (t^H s, t^H t) come from the x-inverse epilogue of the operator call that writes v and t,
    // when it can compute them (forward operator, register four-step x pass)
    // (not with a preconditioner: t^H s needs s, while the operator is applied to M^-1 s)
    const int fblocks = fuse && !pre ? fused_dot_blocks<T>(c) : 0;
    const long long flines = 3LL * c->n3 * c->n2;
    hipLaunchKernelGGL((k_init<T>), dim3(kRedBlocks, all.n), dim3(kThreads), 0, c->stream, b, ax0, r, rhat, p, v, m,
                       c->partials, slot_map(all));
    LS_HIP(hipGetLastError());
    int rc = finalize(c, all, PH_INIT, 2, 0.0, nullptr, nullptr, kRedBlocks, tol2v);
    if (rc) return rc;
    auto read_state = [&]() -> int {
        LS_HIP(hipMemcpyAsync(c->red_host, c->state, sizeof(double) * ns * kStateLen, hipMemcpyDeviceToHost,
                              c->stream));
        LS_HIP(hipStreamSynchronize(c->stream));
        return LS_OK;
    };
    if ((rc = read_state())) return rc;
    if constexpr (sizeof(X) == 8) {
        if (keep && keep->r2.empty()) {
            keep->r2.assign(ns, std::numeric_limits<double>::infinity());
            for (int q = 0; q < all.n; ++q) keep->r2[all.slot[q]] = c->red_host[all.slot[q] * kStateLen + S_RNORM2];
            hipLaunchKernelGGL(k_copy, dim3(kRedBlocks, all.n), dim3(kThreads), 0, c->stream, (const z128*)x, keep->x,
                               m, slot_map(all));
            LS_HIP(hipGetLastError());
        }
    }
    // One iteration over the systems of `cur` is a fixed sequence of launches whose scalars live on the
    // device, so it is captured once into a graph and replayed; the host only reads the active flags in
    // between.
    auto body = [&](const RhsSet& cur) -> int {
        int brc;
        const dim3 g(kRedBlocks, cur.n);
        const SlotMap sm = slot_map(cur);
        PreTabs<T> pt{};
        if (pre) {
            for (int q = 0; q < cur.n; ++q)
                pt.m[q] = sizeof(T) == 8 ? (const cpx<T>*)c->minv[cur.freq[q]] : (const cpx<T>*)c->minv32[cur.freq[q]];
            pt.trans = pre == 2 ? 1 : 0;
        }
        c->prof.begin(c->stream, LS_PNAME(T, "blas1"), cur.n);
        if (pre)
            hipLaunchKernelGGL((k_update_p_pre<T>), g, dim3(kThreads), 0, c->stream, r, p, v, ph, m / 3, c->state, sm,
                               pt);
        else
            hipLaunchKernelGGL((k_update_p<T>), g, dim3(kThreads), 0, c->stream, r, p, v, m, c->state, sm);
        c->prof.end(c->stream);
        if (fblocks) c->dot = {1, rhat, c->dparts, flines, fblocks};
        brc = apply(cur, pre ? ph : p, v);
        c->dot = {};
        if (brc) return brc;
        if (fblocks) {
            if ((brc = finalize(c, cur, PH_ALPHA, 2, 0.0, nullptr, c->dparts, fblocks))) return brc;
        } else {
            c->prof.begin(c->stream, LS_PNAME(T, "blas1"), cur.n);
            hipLaunchKernelGGL((k_dot<T>), g, dim3(kThreads), 0, c->stream, rhat, v, m, c->state, c->partials, sm);
            c->prof.end(c->stream);
            if ((brc = finalize(c, cur, PH_ALPHA, 2))) return brc;
        }
        c->prof.begin(c->stream, LS_PNAME(T, "blas1"), cur.n);
        if (pre)
            hipLaunchKernelGGL((k_update_s_pre<T>), g, dim3(kThreads), 0, c->stream, r, v, s, sh, m / 3, c->state,
                               c->partials, sm, pt);
        else
            hipLaunchKernelGGL((k_update_s<T>), g, dim3(kThreads), 0, c->stream, r, v, s, m, c->state, c->partials,
                               sm);
        c->prof.end(c->stream);
        if ((brc = finalize(c, cur, PH_S, 1))) return brc;
        hipLaunchKernelGGL((k_update_x_half<T, X>), g, dim3(kThreads), 0, c->stream, x, pre ? ph : p, m, c->state, sm);
        hipLaunchKernelGGL(k_clear_half, dim3(1), dim3(kMaxRhs), 0, c->stream, c->state, cur.n, sm);
        if (fblocks) c->dot = {2, nullptr, c->dparts, flines, fblocks};
        brc = apply(cur, pre ? sh : s, t);
        c->dot = {};
        if (brc) return brc;
        if (fblocks) {
            if ((brc = finalize(c, cur, PH_OMEGA, 3, 0.0, nullptr, c->dparts, fblocks))) return brc;
        } else {
            c->prof.begin(c->stream, LS_PNAME(T, "blas1"), cur.n);
            hipLaunchKernelGGL((k_dot_ts<T>), g, dim3(kThreads), 0, c->stream, t, s, m, c->state, c->partials, sm);
            c->prof.end(c->stream);
            if ((brc = finalize(c, cur, PH_OMEGA, 3))) return brc;
        }
        c->prof.begin(c->stream, LS_PNAME(T, "blas1"), cur.n);
        if (pre)
            hipLaunchKernelGGL((k_update_xr<T, X, true>), g, dim3(kThreads), 0, c->stream, x, ph, s, sh, t, r, rhat, m,
                               c->state, c->partials, sm);
        else
            hipLaunchKernelGGL((k_update_xr<T, X, false>), g, dim3(kThreads), 0, c->stream, x, p, s, s, t, r, rhat, m,
                               c->state, c->partials, sm);
        c->prof.end(c->stream);
        if ((brc = finalize(c, cur, PH_RHO, 4))) return brc;
        LS_HIP(hipGetLastError());
        return LS_OK;
    };
    struct GraphGuard {
        hipGraphExec_t exec = nullptr;
        RhsSet set;   // the systems the captured iteration covers
        void reset() {
            if (exec) (void)hipGraphExecDestroy(exec);
            exec = nullptr;
        }
        ~GraphGuard() { reset(); }
    } guard;
    const bool graphs = !(c->flags & LS_FLAG_NO_GRAPH) && !c->prof.on && c->stream != nullptr;
    auto capture = [&](const RhsSet& cur) -> int {
        guard.reset();
        LS_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        const int brc = body(cur);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(c->stream, &graph);
        if (brc) {
            if (graph) (void)hipGraphDestroy(graph);
            return brc;
        }
        if (e != hipSuccess) return hip_fail(e, "BiCGSTAB iteration capture");
        const hipError_t e2 = hipGraphInstantiate(&guard.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) {
            guard.exec = nullptr;
            return hip_fail(e2, "BiCGSTAB iteration graph instantiation");
        }
        guard.set = cur;
        return LS_OK;
    };
    // FP32 inner solves stop a right-hand side whose residual has not improved on its best by 10 % for
    // a stall window of iterations (see stall_window; the FP64 refinement restarts from the true
    // residual).  FP64 solves run to tol or maxit.
    std::vector<double> best(ns, std::numeric_limits<double>::infinity());
    std::vector<int> since(ns, 0), last_it(ns, 0);
    static const double zero = 0.0;
    RhsSet cur = active_subset(all, c->red_host);
    for (int it = 0; it < maxit && cur.n > 0; ++it) {
        if (graphs) {
            if (!guard.exec || !same_set(cur, guard.set))
                if ((rc = capture(cur))) return rc;
            LS_HIP(hipGraphLaunch(guard.exec, c->stream));
        } else if ((rc = body(cur))) {
            return rc;
        }
        if ((rc = read_state())) return rc;
        for (int r = 0; r < cur.n; ++r) {
            const int q = cur.slot[r];
            double* sq = &c->red_host[q * kStateLen];
            // relative residual of each completed iteration (scaled to the caller's system)
            if ((int)sq[S_ITERS] > last_it[q] && sq[S_BNORM2] > 0.0 && (size_t)q < c->history.size()) {
                last_it[q] = (int)sq[S_ITERS];
                c->history[q].push_back(std::sqrt(sq[S_RNORM2] / sq[S_BNORM2]) * (hscale ? hscale[q] : 1.0));
            }
            if constexpr (sizeof(X) == 8) {
                if (keep && sq[S_DONE] != 1.0 && sq[S_RNORM2] < 0.25 * keep->r2[q]) {
                    keep->r2[q] = sq[S_RNORM2];
                    if ((rc = keep->save(c, (const z128*)x, q, m))) return rc;
                }
            }
            if (sq[S_ACTIVE] == 0.0) continue;
            if (sizeof(T) == 4) {
                if (sq[S_RNORM2] < 0.81 * best[q]) {  // 10 % on the norm
                    best[q] = sq[S_RNORM2];
                    since[q] = 0;
                } else if (++since[q] >= stall_window(sq[S_RNORM2], sq[S_BNORM2])) {
                    LS_HIP(hipMemcpyAsync(c->state + q * kStateLen + S_ACTIVE, &zero, sizeof(double),
                                          hipMemcpyHostToDevice, c->stream));
                    sq[S_ACTIVE] = 0.0;
                }
            }
        }
        cur = active_subset(cur, c->red_host);
    }
    if ((rc = read_state())) return rc;
    iters.assign(ns, 0);
    for (int q = 0; q < all.n; ++q) iters[all.slot[q]] = (int)c->red_host[all.slot[q] * kStateLen + S_ITERS];
    return LS_OK;
}

// ---------------------------------------------------------------------------------------------
// BiCGSTAB(l) (Sleijpen and Fokkema): l Bi-CG steps, then the minimal-residual polynomial of degree l
// over the residuals r_0 .. r_l the steps built (r_j = A r_{j-1}).  Per right-hand side:
//   Bi-CG step j:  rho1 = r^H r_j;  beta = alpha rho1 / rho0;  rho0 = rho1;  u_i = r_i - beta u_i (i <= j);
//                  u_{j+1} = A u_j;  alpha = rho0 / (r^H u_{j+1});  r_i -= alpha u_{i+1} (i <= j);
//                  x += alpha u_0;  r_{j+1} = A r_j
//   MR part:       gamma = argmin ||r_0 - sum_{j>=1} gamma_j r_j||, from the Gram matrix Z = R^H R
//                  (normal equations, Cholesky on the host);  r_0 -= sum gamma_j r_j;
//                  u_0 -= sum gamma_j u_j;  x += sum gamma_j r_{j-1};  omega = gamma_l;  next rho0 = -omega rho0.
// The scalars of the cycle are computed on the host from deterministic device reductions (fixed
// block count and order), one round trip per inner product, so the iteration is not captured in a
// graph; a cycle costs 2 l matvecs and 2 l + 1 round trips.  l = 1 uses the graph-captured Bi-CGSTAB.

constexpr int kMaxL = 4;
constexpr int kGramSlots = (kMaxL + 1) * (kMaxL + 2);  // re, im of the upper triangle of Z
constexpr int kCoef = 12;                              // per right-hand side: up to l complex + active flag

template <typename T>
struct VecSet {
    cpx<T>* v[kMaxL + 1];
};

// nq per-thread values summed over the block in a fixed order (wavefront shuffles, then the four
// wavefronts in order) into gp[(rr kGramSlots + q) kRedBlocks + block]
template <int NQ>
__device__ __forceinline__ void block_partials(const double (&a)[NQ], int nq, double* gp, int rr) {
    __shared__ double sh[kThreads / 64][NQ];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (q >= nq) break;
        double v = a[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) sh[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < nq) {
        double v = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) v += sh[w][threadIdx.x];
        gp[((long long)rr * kGramSlots + threadIdx.x) * kRedBlocks + blockIdx.x] = v;
    }
}

// (a^H b, ||b||^2) per right-hand side
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot_l(const cpx<T>* __restrict__ a, const cpx<T>* __restrict__ b,
                                                    long long m, const double* __restrict__ coef, double* gp) {
    const int rr = blockIdx.y;
    if (coef[rr * kCoef + kCoef - 1] == 0.0) return;
    const long long off = (long long)rr * m;
    double acc[3] = {0.0, 0.0, 0.0};
    LS_FOR_ELEMS(m) {
        const cpx<double> av = wide(a[off + e]), bv = wide(b[off + e]);
        acc[0] += av.x * bv.x + av.y * bv.y;
        acc[1] += av.x * bv.y - av.y * bv.x;
        acc[2] += bv.x * bv.x + bv.y * bv.y;
    }
    block_partials<3>(acc, 3, gp, rr);
}

// u_i = r_i - beta u_i, i <= j
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bicg_u(VecSet<T> R, VecSet<T> U, int j, long long m,
                                                     const double* __restrict__ coef) {
    const int rr = blockIdx.y;
    const double* cf = coef + rr * kCoef;
    if (cf[kCoef - 1] == 0.0) return;
    const cpx<T> beta = {(T)cf[0], (T)cf[1]};
    const long long off = (long long)rr * m;
    LS_FOR_ELEMS(m) {
        for (int i = 0; i <= j; ++i) U.v[i][off + e] = R.v[i][off + e] - beta * U.v[i][off + e];
    }
}

// r_i -= alpha u_{i+1} (i <= j), x += alpha u_0; partials ||r_0||^2
template <typename T, typename X>
__global__ __launch_bounds__(kThreads) void k_bicg_r(VecSet<T> R, VecSet<T> U, int j, cpx<X>* __restrict__ x,
                                                     long long m, const double* __restrict__ coef, double* gp) {
    const int rr = blockIdx.y;
    const double* cf = coef + rr * kCoef;
    if (cf[kCoef - 1] == 0.0) return;
    const cpx<T> alpha = {(T)cf[0], (T)cf[1]};
    const cpx<X> alx = {(X)cf[0], (X)cf[1]};
    const long long off = (long long)rr * m;
    double acc[1] = {0.0};
    LS_FOR_ELEMS(m) {
        for (int i = 0; i <= j; ++i) {
            const cpx<T> v = R.v[i][off + e] - alpha * U.v[i + 1][off + e];
            R.v[i][off + e] = v;
            if (i == 0) acc[0] += (double)v.x * v.x + (double)v.y * v.y;
        }
        const cpx<T> u0 = U.v[0][off + e];
        x[off + e] = x[off + e] + alx * cpx<X>{(X)u0.x, (X)u0.y};
    }
    block_partials<1>(acc, 1, gp, rr);
}

// Z_ab = r_a^H r_b, a <= b <= L (row by row), as (re, im) pairs
template <typename T, int L>
__global__ __launch_bounds__(kThreads) void k_gram(VecSet<T> R, long long m, const double* __restrict__ coef,
                                                   double* gp) {
    const int rr = blockIdx.y;
    if (coef[rr * kCoef + kCoef - 1] == 0.0) return;
    constexpr int NQ = (L + 1) * (L + 2);
    const long long off = (long long)rr * m;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    LS_FOR_ELEMS(m) {
        cpx<double> v[L + 1];
#pragma unroll
        for (int a = 0; a <= L; ++a) v[a] = wide(R.v[a][off + e]);
        int q = 0;
#pragma unroll
        for (int a = 0; a <= L; ++a)
#pragma unroll
            for (int b = a; b <= L; ++b, q += 2) {
                acc[q] += v[a].x * v[b].x + v[a].y * v[b].y;
                acc[q + 1] += v[a].x * v[b].y - v[a].y * v[b].x;
            }
    }
    block_partials<NQ>(acc, NQ, gp, rr);
}

// r_0 -= sum_j g_j r_j;  u_0 -= sum_j g_j u_j;  x += sum_j g_j r_{j-1}   (j = 1..L)
template <typename T, typename X, int L>
__global__ __launch_bounds__(kThreads) void k_mr(VecSet<T> R, VecSet<T> U, cpx<X>* __restrict__ x, long long m,
                                                 const double* __restrict__ coef) {
    const int rr = blockIdx.y;
    const double* cf = coef + rr * kCoef;
    if (cf[kCoef - 1] == 0.0) return;
    cpx<T> g[L + 1];
#pragma unroll
    for (int j = 1; j <= L; ++j) g[j] = {(T)cf[2 * (j - 1)], (T)cf[2 * (j - 1) + 1]};
    const long long off = (long long)rr * m;
    LS_FOR_ELEMS(m) {
        cpx<T> rv[L + 1];
#pragma unroll
        for (int a = 0; a <= L; ++a) rv[a] = R.v[a][off + e];
        cpx<T> r0 = rv[0], u0 = U.v[0][off + e];
        cpx<X> dx = {(X)0, (X)0};
#pragma unroll
        for (int j = 1; j <= L; ++j) {
            r0 = r0 - g[j] * rv[j];
            u0 = u0 - g[j] * U.v[j][off + e];
            const cpx<T> t = g[j] * rv[j - 1];
            dx = dx + cpx<X>{(X)t.x, (X)t.y};
        }
        R.v[0][off + e] = r0;
        U.v[0][off + e] = u0;
        x[off + e] = x[off + e] + dx;
    }
}

// sums of the first nq partial slots of each right-hand side, in a fixed order -> out[rr kGramSlots + q]
__global__ __launch_bounds__(kThreads) void k_reduce_slots(const double* __restrict__ gp, int nq,
                                                           double* __restrict__ out) {
    __shared__ double sh[kThreads];
    const int rr = blockIdx.x, tid = threadIdx.x;
    for (int q = 0; q < nq; ++q) {
        double a = 0.0;
        for (int k = tid; k < kRedBlocks; k += kThreads) a += gp[((long long)rr * kGramSlots + q) * kRedBlocks + k];
        sh[tid] = a;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (tid < w) sh[tid] += sh[tid + w];
            __syncthreads();
        }
        if (tid == 0) out[rr * kGramSlots + q] = sh[0];
        __syncthreads();
    }
}

struct LState {
    int iters = 0, matvecs = 0;
    int status = 0;          // 0 running / converged, 1 not converged, 2 breakdown, 3 non-finite
    bool active = true, done = false;
    double bnorm2 = 0, rnorm2 = 0, best = 0;
    int since = 0;
    std::complex<double> rho0 = 1.0, alpha = 0.0, omega = 1.0;
};

// Solve min ||r_0 - sum_{j=1..l} g_j r_j|| from Z (upper triangle, row-major pairs): Z[1:,1:] g = Z[1:,0].
bool mr_coefficients(const double* z, int l, std::complex<double>* g) {
    using C = std::complex<double>;
    // entry (a, b) of the Hermitian Gram matrix from its stored upper triangle
    auto Z = [&](int a, int b) -> C {
        const bool lower = a > b;
        if (lower) std::swap(a, b);
        int q = 0;
        for (int i = 0; i < a; ++i) q += l + 1 - i;
        q += b - a;
        const C v(z[2 * q], z[2 * q + 1]);
        return lower ? std::conj(v) : v;
    };
    C M[kMaxL][kMaxL], rhs[kMaxL];
    for (int a = 0; a < l; ++a) {
        for (int b = 0; b < l; ++b) M[a][b] = Z(a + 1, b + 1);
        rhs[a] = Z(a + 1, 0);
    }
    // Cholesky M = L L^H
    C Lm[kMaxL][kMaxL] = {};
    for (int a = 0; a < l; ++a) {
        for (int b = 0; b <= a; ++b) {
            C sacc = M[a][b];
            for (int k = 0; k < b; ++k) sacc -= Lm[a][k] * std::conj(Lm[b][k]);
            if (a == b) {
                if (!(sacc.real() > 0.0) || !std::isfinite(sacc.real())) return false;
                Lm[a][a] = std::sqrt(sacc.real());
            } else {
                Lm[a][b] = sacc / Lm[b][b].real();
            }
        }
    }
    C y[kMaxL];
    for (int a = 0; a < l; ++a) {
        C sacc = rhs[a];
        for (int k = 0; k < a; ++k) sacc -= Lm[a][k] * y[k];
        y[a] = sacc / Lm[a][a].real();
    }
    for (int a = l - 1; a >= 0; --a) {
        C sacc = y[a];
        for (int k = a + 1; k < l; ++k) sacc -= std::conj(Lm[k][a]) * g[k + 1];
        g[a + 1] = sacc / Lm[a][a].real();
        if (!std::isfinite(g[a + 1].real()) || !std::isfinite(g[a + 1].imag())) return false;
    }
    return true;
}

template <typename T, typename X, typename ApplyFn>
int bicgstab_l(Ctx* c, const cpx<T>* b, cpx<X>* x, const cpx<T>* ax0, cpx<T>* const* vecs, int l, int nrhs,
               double tol, int maxit, ApplyFn apply, std::vector<LState>& st, const double* hscale = nullptr,
               BestIterate* best = nullptr) {
    using Cd = std::complex<double>;
    const long long m = (long long)c->field_elems();
    const dim3 g = vgrid(nrhs);
    VecSet<T> R{}, U{};
    for (int i = 0; i <= l; ++i) {
        R.v[i] = vecs[i];
        U.v[i] = vecs[l + 1 + i];
    }
    cpx<T>* rhat = vecs[2 * l + 2];
    double* coef = c->red + 3 * kRedBlocks;
    double* out = c->red;
    std::vector<double> hc((size_t)nrhs * kCoef, 0.0);
    std::vector<int> stale(nrhs, 0);
    st.assign(nrhs, LState());
    // r_0 = b - A x0, rhat = r_0, u_0 = 0 (systems 0..nrhs-1 on slots 0..nrhs-1)
    const RhsSet ids = RhsSet::uniform(nrhs, 0);
    hipLaunchKernelGGL((k_init<T>), g, dim3(kThreads), 0, c->stream, b, ax0, R.v[0], rhat, U.v[0], U.v[1], m,
                       c->partials, slot_map(ids));
    LS_HIP(hipGetLastError());
    int rc = finalize(c, ids, PH_INIT, 2, tol * tol);
    if (rc) return rc;
    LS_HIP(hipMemcpyAsync(c->red_host, c->state, sizeof(double) * nrhs * kStateLen, hipMemcpyDeviceToHost, c->stream));
    LS_HIP(hipStreamSynchronize(c->stream));
    const double tol2 = tol * tol;
    if constexpr (sizeof(X) == 8) {
        if (best) {
            best->r2.resize(nrhs);
            for (int q = 0; q < nrhs; ++q) best->r2[q] = c->red_host[q * kStateLen + S_RNORM2];
            hipLaunchKernelGGL(k_copy, g, dim3(kThreads), 0, c->stream, (const z128*)x, best->x, m, slot_map(ids));
            LS_HIP(hipGetLastError());
        }
    }
    for (int q = 0; q < nrhs; ++q) {
        st[q].bnorm2 = c->red_host[q * kStateLen + S_BNORM2];
        st[q].rnorm2 = c->red_host[q * kStateLen + S_RNORM2];
        st[q].best = st[q].rnorm2;
        if (!std::isfinite(st[q].bnorm2) || !std::isfinite(st[q].rnorm2)) {
            st[q].status = 3;
            st[q].active = false;
        } else if (st[q].rnorm2 <= tol2 * st[q].bnorm2) {
            st[q].active = false;
            st[q].done = true;
        }
    }
    // hc holds the coefficients of the active systems; the last slot carries the active flag
    auto push = [&]() -> int {
        for (int q = 0; q < nrhs; ++q) hc[(size_t)q * kCoef + kCoef - 1] = st[q].active ? 1.0 : 0.0;
        LS_HIP(hipMemcpyAsync(coef, hc.data(), sizeof(double) * nrhs * kCoef, hipMemcpyHostToDevice, c->stream));
        return LS_OK;
    };
    auto reduce = [&](int nq) -> int {
        hipLaunchKernelGGL(k_reduce_slots, dim3(nrhs), dim3(kThreads), 0, c->stream, c->gpart, nq, out);
        LS_HIP(hipGetLastError());
        LS_HIP(hipMemcpyAsync(c->red_host, out, sizeof(double) * nrhs * kGramSlots, hipMemcpyDeviceToHost, c->stream));
        LS_HIP(hipStreamSynchronize(c->stream));
        return LS_OK;
    };
    auto any_active = [&]() {
        for (auto& q : st)
            if (q.active) return true;
        return false;
    };
    int save_rc = LS_OK;
    auto record = [&](int q, double r2) {
        st[q].rnorm2 = r2;
        stale[q] = 0;
        if constexpr (sizeof(X) == 8) {
            if (best && r2 < 0.25 * best->r2[q] && !(r2 <= tol2 * st[q].bnorm2)) {
                best->r2[q] = r2;
                if (save_rc == LS_OK) save_rc = best->save(c, (const z128*)x, q, m);
            }
        }
        if ((size_t)q < c->history.size() && st[q].bnorm2 > 0.0)
            c->history[q].push_back(std::sqrt(r2 / st[q].bnorm2) * (hscale ? hscale[q] : 1.0));
    };
    // converged, non-finite, or (FP32 inner solves) no 10 % gain on the best norm for 30 checks
    auto check = [&](int q, double r2) {
        if (!std::isfinite(r2)) {
            st[q].status = 3;
            st[q].active = false;
        } else if (r2 <= tol2 * st[q].bnorm2) {
            st[q].active = false;
            st[q].done = true;
        } else if (sizeof(T) == 4) {
            if (r2 < 0.81 * st[q].best) {
                st[q].best = r2;
                st[q].since = 0;
            } else if (++st[q].since >= stall_window(r2, st[q].bnorm2)) {
                st[q].active = false;
            }
        }
    };
    auto halt = [&](int q, bool finite) {
        st[q].status = finite ? 2 : 3;
        st[q].active = false;
    };
    bool first = true;
    while (any_active()) {
        for (auto& q : st)
            if (q.active && q.iters + l > maxit) q.active = false;
        if (!any_active()) break;
        for (auto& q : st)
            if (q.active) q.rho0 = -q.omega * q.rho0;
        for (int j = 0; j < l && any_active(); ++j) {
            // rho1 = rhat^H r_j; at j = 0 also ||r_0||^2, the residual after the last minimal-residual update
            if ((rc = push())) return rc;
            hipLaunchKernelGGL((k_dot_l<T>), g, dim3(kThreads), 0, c->stream, rhat, R.v[j], m, coef, c->gpart);
            LS_HIP(hipGetLastError());
            if ((rc = reduce(3))) return rc;
            for (int q = 0; q < nrhs; ++q) {
                if (!st[q].active) continue;
                const double* o = &c->red_host[q * kGramSlots];
                if (j == 0 && !first) {
                    record(q, o[2]);
                    check(q, o[2]);
                    if (!st[q].active) continue;
                }
                const Cd rho1(o[0], o[1]);
                if (!(std::abs(st[q].rho0) > 0.0) || !(std::abs(rho1) > 0.0) || !std::isfinite(std::abs(rho1))) {
                    halt(q, std::isfinite(std::abs(rho1)));
                    continue;
                }
                const Cd beta = st[q].alpha * rho1 / st[q].rho0;
                st[q].rho0 = rho1;
                hc[(size_t)q * kCoef] = beta.real();
                hc[(size_t)q * kCoef + 1] = beta.imag();
            }
            if (!any_active()) break;
            // u_i = r_i - beta u_i;  u_{j+1} = A u_j
            if ((rc = push())) return rc;
            c->prof.begin(c->stream, LS_PNAME(T, "blas1"), nrhs);
            hipLaunchKernelGGL((k_bicg_u<T>), g, dim3(kThreads), 0, c->stream, R, U, j, m, coef);
            c->prof.end(c->stream);
            LS_HIP(hipGetLastError());
            if ((rc = apply(U.v[j], U.v[j + 1]))) return rc;
            for (auto& q : st)
                if (q.active) q.matvecs += 1;
            // alpha = rho0 / (rhat^H u_{j+1})
            hipLaunchKernelGGL((k_dot_l<T>), g, dim3(kThreads), 0, c->stream, rhat, U.v[j + 1], m, coef, c->gpart);
            LS_HIP(hipGetLastError());
            if ((rc = reduce(3))) return rc;
            for (int q = 0; q < nrhs; ++q) {
                if (!st[q].active) continue;
                const double* o = &c->red_host[q * kGramSlots];
                const Cd gam(o[0], o[1]);
                if (!(std::abs(gam) > 0.0) || !std::isfinite(std::abs(gam))) {
                    halt(q, std::isfinite(std::abs(gam)));
                    continue;
                }
                st[q].alpha = st[q].rho0 / gam;
                hc[(size_t)q * kCoef] = st[q].alpha.real();
                hc[(size_t)q * kCoef + 1] = st[q].alpha.imag();
            }
            if (!any_active()) break;
            // r_i -= alpha u_{i+1};  x += alpha u_0;  ||r_0||^2
            if ((rc = push())) return rc;
            c->prof.begin(c->stream, LS_PNAME(T, "blas1"), nrhs);
            hipLaunchKernelGGL((k_bicg_r<T, X>), g, dim3(kThreads), 0, c->stream, R, U, j, x, m, coef, c->gpart);
            c->prof.end(c->stream);
            LS_HIP(hipGetLastError());
            if ((rc = reduce(1))) return rc;
            for (int q = 0; q < nrhs; ++q) {
                if (!st[q].active) continue;
                const double r2 = c->red_host[q * kGramSlots];
                st[q].iters += 1;
                check(q, r2);
                if (j < l - 1 || !st[q].active) record(q, r2);
            }
            if (!any_active()) break;
            // r_{j+1} = A r_j
            if ((rc = apply(R.v[j], R.v[j + 1]))) return rc;
            for (auto& q : st)
                if (q.active) q.matvecs += 1;
        }
        if (!any_active()) break;
        // minimal-residual part: the Gram matrix of r_0 .. r_l, the normal equations on the host
        const int nq = (l + 1) * (l + 2);
        if ((rc = push())) return rc;
        c->prof.begin(c->stream, LS_PNAME(T, "blas1"), nrhs);
        switch (l) {
            case 2: hipLaunchKernelGGL((k_gram<T, 2>), g, dim3(kThreads), 0, c->stream, R, m, coef, c->gpart); break;
            case 3: hipLaunchKernelGGL((k_gram<T, 3>), g, dim3(kThreads), 0, c->stream, R, m, coef, c->gpart); break;
            default: hipLaunchKernelGGL((k_gram<T, 4>), g, dim3(kThreads), 0, c->stream, R, m, coef, c->gpart); break;
        }
        c->prof.end(c->stream);
        LS_HIP(hipGetLastError());
        if ((rc = reduce(nq))) return rc;
        for (int q = 0; q < nrhs; ++q) {
            if (!st[q].active) continue;
            Cd gm[kMaxL + 1];
            if (!mr_coefficients(&c->red_host[q * kGramSlots], l, gm)) {
                halt(q, true);
                continue;
            }
            st[q].omega = gm[l];
            for (int j = 1; j <= l; ++j) {
                hc[(size_t)q * kCoef + 2 * (j - 1)] = gm[j].real();
                hc[(size_t)q * kCoef + 2 * (j - 1) + 1] = gm[j].imag();
            }
            stale[q] = 1;
        }
        if (!any_active()) break;
        if ((rc = push())) return rc;
        c->prof.begin(c->stream, LS_PNAME(T, "blas1"), nrhs);
        switch (l) {
            case 2: hipLaunchKernelGGL((k_mr<T, X, 2>), g, dim3(kThreads), 0, c->stream, R, U, x, m, coef); break;
            case 3: hipLaunchKernelGGL((k_mr<T, X, 3>), g, dim3(kThreads), 0, c->stream, R, U, x, m, coef); break;
            default: hipLaunchKernelGGL((k_mr<T, X, 4>), g, dim3(kThreads), 0, c->stream, R, U, x, m, coef); break;
        }
        c->prof.end(c->stream);
        LS_HIP(hipGetLastError());
        first = false;
    }
    // systems whose last operation was a minimal-residual update: their residual norm
    bool any_stale = false;
    for (int q = 0; q < nrhs; ++q) {
        const bool want = stale[q] && st[q].status == 0;
        any_stale = any_stale || want;
        hc[(size_t)q * kCoef + kCoef - 1] = want ? 1.0 : 0.0;
    }
    if (any_stale) {
        LS_HIP(hipMemcpyAsync(coef, hc.data(), sizeof(double) * nrhs * kCoef, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL((k_dot_l<T>), g, dim3(kThreads), 0, c->stream, rhat, R.v[0], m, coef, c->gpart);
        LS_HIP(hipGetLastError());
        if ((rc = reduce(3))) return rc;
        for (int q = 0; q < nrhs; ++q)
            if (stale[q] && st[q].status == 0) {
                const double r2 = c->red_host[q * kGramSlots + 2];
                record(q, r2);
                if (!std::isfinite(r2)) st[q].status = 3;
                else if (r2 <= tol2 * st[q].bnorm2) st[q].done = true;
            }
    }
    for (auto& q : st)
        if (!q.done && q.status == 0) q.status = 1;
    return save_rc;
}

// the operator or its transpose over the systems of a set, in launches of at most c->launch_rhs systems
// (0: one launch for the whole set)
template <typename T>
int op_apply(Ctx* c, const RhsSet& set, const cpx<T>* in, cpx<T>* out, bool transposed) {
    const int w = c->launch_rhs > 0 ? c->launch_rhs : set.n;
    for (int r0 = 0; r0 < set.n; r0 += w) {
        RhsSet sub;
        sub.n = std::min(w, set.n - r0);
        for (int r = 0; r < sub.n; ++r) sub.slot[r] = set.slot[r0 + r], sub.freq[r] = set.freq[r0 + r];
        const int rc = transposed ? apply_T_op<T>(c, sub, in, out) : apply_op<T>(c, sub, in, out);
        if (rc) return rc;
    }
    return LS_OK;
}

// ||b - A x|| / ||b|| (rel) and ||b - A x|| (abs_) of the systems of a set with the FP64 operator, into the
// entries of their slots; writes r = b - A x if r != null.
int true_residual(Ctx* c, const RhsSet& set, const z128* b, const z128* x, z128* ax, z128* r, std::vector<double>& rel,
                  std::vector<double>& abs_, bool transposed) {
    int rc = op_apply<double>(c, set, x, ax, transposed);
    if (rc) return rc;
    const long long m = (long long)c->field_elems();
    hipLaunchKernelGGL(k_residual, dim3(kRedBlocks, set.n), dim3(kThreads), 0, c->stream, b, ax, r, m, c->partials,
                       slot_map(set));
    LS_HIP(hipGetLastError());
    if ((rc = finalize(c, set, PH_RESID, 2, 0.0, c->red))) return rc;
    LS_HIP(hipMemcpyAsync(c->red_host, c->red, sizeof(double) * 2 * kRedBlocks, hipMemcpyDeviceToHost, c->stream));
    LS_HIP(hipStreamSynchronize(c->stream));
    for (int i = 0; i < set.n; ++i) {
        const int q = set.slot[i];
        if ((size_t)q >= rel.size()) rel.resize(q + 1, 0.0);
        if ((size_t)q >= abs_.size()) abs_.resize(q + 1, 0.0);
        rel[q] = c->red_host[q];
        abs_[q] = c->red_host[kRedBlocks + q];
    }
    return LS_OK;
}

// the vectors of BiCGSTAB(l) in the order r_0..r_l, u_0..u_l, rhat: the six of Bi-CGSTAB, then the extras
template <typename T>
std::vector<cpx<T>*> krylov_vectors(Ctx* c) {
    std::vector<cpx<T>*> v;
    if (sizeof(T) == 8) {
        for (z128* p : {c->r, c->rhat, c->p, c->v, c->s, c->t}) v.push_back((cpx<T>*)p);
        for (void* p : c->kry128) v.push_back((cpx<T>*)p);
    } else {
        for (z64* p : {c->r32, c->rhat32, c->p32, c->v32, c->s32, c->t32}) v.push_back((cpx<T>*)p);
        for (void* p : c->kry64) v.push_back((cpx<T>*)p);
    }
    return v;
}

}  // namespace

int krylov_setup(Ctx* c) {
    const int l = c->bicgstab_l;
    if (l < 2) return LS_OK;
    const size_t fe = c->field_elems() * (size_t)c->max_rhs;
    int rc = LS_OK;
    if (!c->gpart) rc = dalloc(c, (void**)&c->gpart, (size_t)c->max_rhs * kGramSlots * kRedBlocks * sizeof(double));
    const size_t extra = (size_t)std::max(0, 2 * l + 3 - 6);
    while (rc == LS_OK && c->kry128.size() < extra) {
        void* p = nullptr;
        rc = dalloc(c, &p, fe * sizeof(z128));
        if (rc == LS_OK) c->kry128.push_back(p);
    }
    while (rc == LS_OK && c->mixed && c->kry64.size() < extra) {
        void* p = nullptr;
        rc = dalloc(c, &p, fe * sizeof(z64));
        if (rc == LS_OK) c->kry64.push_back(p);
    }
    return rc;
}

int solve_systems(Ctx* c, const int* freq, const z128* b, int nrhs, double tol, int maxit, int precision, const z128* x0,
                  z128* u_out, ls_info* info, bool transposed) {
    const long long m = (long long)c->field_elems();
    RhsSet all;   // system q on slot q at frequency freq[q]
    all.n = nrhs;
    for (int q = 0; q < nrhs; ++q) all.slot[q] = q, all.freq[q] = freq[q];
    const dim3 gall(kRedBlocks, nrhs);
    std::vector<ls_info> inf(nrhs);
    for (auto& q : inf) q = ls_info{0, 0, 0, LS_OK, 0.0, 0.0};
    c->history.assign(nrhs, std::vector<double>());
    // x = x0 or 0
    if (x0) {
        if (x0 != u_out) {
            hipLaunchKernelGGL(k_copy, gall, dim3(kThreads), 0, c->stream, x0, u_out, m, slot_map(all));
            LS_HIP(hipGetLastError());
        }
    } else {
        LS_HIP(hipMemsetAsync(u_out, 0, sizeof(z128) * m * nrhs, c->stream));
    }
    // each slot's squared relative tolerance for the Bi-CGSTAB initialisation
    double* tol2v = c->red + 4 * kRedBlocks;
    std::vector<double> t2(nrhs, tol * tol);
    auto push_tol2 = [&]() -> int {
        LS_HIP(hipMemcpyAsync(tol2v, t2.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
        return LS_OK;
    };
    std::vector<double> rel(nrhs, 0.0), nrm(nrhs, 0.0);
    std::vector<int> iters;
    int rc = LS_OK;
    // block-Jacobi right preconditioning: M^-1 (1), or M^-T for the transposed operator (2)
    const int pre = c->precond == LS_PRECOND_BLOCK_JACOBI ? (transposed ? 2 : 1) : 0;
    if (precision == LS_PREC_C128 && c->bicgstab_l > 1) {
        auto apply = [&](const z128* in, z128* out) { return op_apply<double>(c, all, in, out, transposed); };
        const std::vector<z128*> vec = krylov_vectors<double>(c);
        const z128* ax0 = nullptr;
        if (x0) {
            if ((rc = apply(u_out, vec[1]))) return rc;   // r_1's vector is free until the first cycle
            ax0 = vec[1];
        }
        std::vector<LState> ls;
        BestIterate best{c->xbest, {}};
        rc = bicgstab_l<double, double>(c, b, u_out, ax0, vec.data(), c->bicgstab_l, nrhs, tol, maxit, apply, ls,
                                        nullptr, &best);
        if (rc) return rc;
        for (int q = 0; q < nrhs; ++q)
            if (ls[q].status == 1 && best.r2[q] < ls[q].rnorm2) {
                if ((rc = best.restore(c, u_out, q, m))) return rc;
                ls[q].rnorm2 = best.r2[q];
            }
        if ((rc = true_residual(c, all, b, u_out, c->v, nullptr, rel, nrm, transposed))) return rc;
        for (int q = 0; q < nrhs; ++q) {
            inf[q].iters = ls[q].iters;
            inf[q].matvecs = ls[q].matvecs + (x0 ? 1 : 0) + 1;
            inf[q].rel_res = ls[q].bnorm2 > 0 ? std::sqrt(ls[q].rnorm2 / ls[q].bnorm2) : 0.0;
            inf[q].rel_res_true = rel[q];
            if (ls[q].status == 3 || !std::isfinite(rel[q]))
                inf[q].status = LS_ERR_NONFINITE;
            else if (ls[q].status == 2)
                inf[q].status = LS_ERR_BREAKDOWN;
            else if (ls[q].status == 1)
                inf[q].status = LS_ERR_NOT_CONVERGED;
        }
    } else if (precision == LS_PREC_C128) {
        auto apply = [&](const RhsSet& set, const z128* in, z128* out) {
            return op_apply<double>(c, set, in, out, transposed);
        };
        if ((rc = push_tol2())) return rc;
        // A breakdown (rho = 0 or rhat^H v = 0) restarts once from the current iterate, which re-seeds the
        // shadow residual with the current residual; only the systems that broke down take the restart.
        std::vector<double> st((size_t)nrhs * kStateLen, 0.0);
        std::vector<int> total(nrhs, 0), extra(nrhs, 0);
        BestIterate best{c->xbest, {}};
        RhsSet todo = all;
        for (int attempt = 0; attempt < 2 && todo.n > 0; ++attempt) {
            const z128* ax0 = nullptr;
            if (x0 || attempt > 0) {
                if ((rc = op_apply<double>(c, todo, u_out, c->t, transposed))) return rc;
                ax0 = c->t;
                for (int i = 0; i < todo.n; ++i) extra[todo.slot[i]] += 1;
            }
            rc = bicgstab<double, double>(c, todo, b, u_out, ax0, c->r, c->rhat, c->p, c->v, c->s, c->t, tol2v, maxit,
                                          apply, iters, nullptr, &best, !transposed, c->ph, c->sh, pre);
            if (rc) return rc;
            RhsSet broken;
            for (int i = 0; i < todo.n; ++i) {
                const int q = todo.slot[i];
                std::copy(c->red_host + (size_t)q * kStateLen, c->red_host + (size_t)(q + 1) * kStateLen,
                          st.begin() + (size_t)q * kStateLen);
                const double* sq = &st[(size_t)q * kStateLen];
                const bool half = sq[S_DONE] == 1.0 && sq[S_SNORM2] == sq[S_RNORM2];
                total[q] += iters[q];
                extra[q] += 2 * iters[q] - (half ? 1 : 0);
                if (sq[S_FLAG] == 2.0) broken.slot[broken.n] = q, broken.freq[broken.n++] = freq[q];
            }
            todo = broken;
        }
        // a system that stopped short of tol returns its best iterate
        for (int q = 0; q < nrhs; ++q) {
            double* sq = &st[(size_t)q * kStateLen];
            if (sq[S_DONE] != 1.0 && sq[S_FLAG] != 3.0 && best.r2[q] < sq[S_RNORM2]) {
                if ((rc = best.restore(c, u_out, q, m))) return rc;
                sq[S_RNORM2] = best.r2[q];
            }
        }
        if ((rc = true_residual(c, all, b, u_out, c->v, nullptr, rel, nrm, transposed))) return rc;
        for (int q = 0; q < nrhs; ++q) {
            const double* sq = &st[(size_t)q * kStateLen];
            inf[q].iters = total[q];
            inf[q].matvecs = extra[q] + 1;
            inf[q].rel_res = sq[S_BNORM2] > 0 ? std::sqrt(sq[S_RNORM2] / sq[S_BNORM2]) : 0.0;
            inf[q].rel_res_true = rel[q];
            if (sq[S_FLAG] == 3.0 || !std::isfinite(rel[q]))
                inf[q].status = LS_ERR_NONFINITE;
            else if (sq[S_FLAG] == 2.0)
                inf[q].status = LS_ERR_BREAKDOWN;
            else if (sq[S_DONE] != 1.0)
                inf[q].status = LS_ERR_NOT_CONVERGED;
        }
    } else {
        if (!c->mixed) return fail(LS_ERR_STATE, "mixed precision needs a context built with LS_PREC_MIXED");
        // outer FP64 refinement: r = b - A x (FP64), inner FP32 BiCGSTAB on A d = r / ||r||.  A correction
        // that does not lower the FP64 true residual is taken back and ends that system's refinement (the
        // iterate stays the best one found); one that lowers it by less than 10 % is kept and ends it too.
        // Every decision is per system, so a system's result does not depend on the others in the batch.
        const int max_outer = 30;
        // The inner FP32 solve aims at kInnerAim tol: the FP64 true residual then lands above the inner one by
        // about the FP32 operator's error (at most 2.5e-7 relative on the 128^3 TTI model, 8 frequencies to 40 Hz,
        // where every system meets 1e-6 after one inner solve with aims 0.3, 0.5 and 0.7: 2078, 2004 and 1958
        // matvecs).  A system that misses tol refines again from its true residual.
        constexpr double kInnerAim = 0.5;
        std::vector<double> scale(nrhs), inv(nrhs), prev(nrhs, 0.0), undo(nrhs, 0.0);
        std::vector<int> active(nrhs, 1), stopped(nrhs, 0);
        int outer = 0;
        double* dscale = c->red + 2 * kRedBlocks;
        auto subset = [&](const std::vector<int>& pick) {
            RhsSet s_;
            for (int q = 0; q < nrhs; ++q)
                if (pick[q]) s_.slot[s_.n] = q, s_.freq[s_.n++] = freq[q];
            return s_;
        };
        for (; outer <= max_outer; ++outer) {
            if (outer == 0 && !x0) {
                // x = 0, so A x = 0 and r = b
                LS_HIP(hipMemsetAsync(c->v, 0, sizeof(z128) * m * nrhs, c->stream));
                hipLaunchKernelGGL(k_residual, gall, dim3(kThreads), 0, c->stream, b, c->v, c->r, m, c->partials,
                                   slot_map(all));
                LS_HIP(hipGetLastError());
                if ((rc = finalize(c, all, PH_RESID, 2, 0.0, c->red))) return rc;
                LS_HIP(hipMemcpyAsync(c->red_host, c->red, sizeof(double) * 2 * kRedBlocks, hipMemcpyDeviceToHost,
                                      c->stream));
                LS_HIP(hipStreamSynchronize(c->stream));
                rel.assign(c->red_host, c->red_host + nrhs);
                nrm.assign(c->red_host + kRedBlocks, c->red_host + kRedBlocks + nrhs);
            } else {
                // the true residual of every system still refining (all of them at the first step)
                const RhsSet rs = outer == 0 ? all : subset(active);
                if ((rc = true_residual(c, rs, b, u_out, c->v, c->r, rel, nrm, transposed))) return rc;
                std::vector<int> to_undo(nrhs, 0);
                bool any_undo = false;
                for (int i = 0; i < rs.n; ++i) {
                    const int q = rs.slot[i];
                    inf[q].matvecs += 1;
                    undo[q] = 0.0;
                    if (outer == 0 || !std::isfinite(rel[q])) continue;
                    if (!(rel[q] < prev[q])) {
                        undo[q] = -inv[q];
                        to_undo[q] = 1;
                        any_undo = true;
                        rel[q] = prev[q];
                        stopped[q] = 1;
                    } else if (rel[q] > 0.9 * prev[q]) {
                        stopped[q] = 1;
                    }
                }
                if (any_undo) {
                    // x -= d for the systems whose last correction raised the true residual (x32 still holds d)
                    const RhsSet us = subset(to_undo);
                    LS_HIP(hipMemcpyAsync(dscale, undo.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice,
                                          c->stream));
                    hipLaunchKernelGGL(k_add32, dim3(kRedBlocks, us.n), dim3(kThreads), 0, c->stream, u_out, c->x32,
                                       m, dscale, slot_map(us));
                    LS_HIP(hipGetLastError());
                    LS_HIP(hipStreamSynchronize(c->stream));
                }
            }
            bool any = false;
            for (int q = 0; q < nrhs; ++q) {
                prev[q] = rel[q];
                active[q] = active[q] && !stopped[q] && rel[q] > tol && std::isfinite(rel[q]) && nrm[q] > 0.0;
                any = any || active[q];
            }
            if (!any || outer == max_outer) break;
            // inner tolerance per system: the reduction that reaches kInnerAim tol, capped at 0.1 and floored at
            // 1e-7 (near the FP32 operator's relative accuracy; a stagnating inner solve is stopped early anyway)
            for (int q = 0; q < nrhs; ++q) {
                const double eta = active[q] ? std::min(1e-1, std::max(1e-7, kInnerAim * tol / rel[q])) : 1e-1;
                t2[q] = eta * eta;
                scale[q] = active[q] ? 1.0 / nrm[q] : 0.0;
                inv[q] = active[q] ? nrm[q] : 0.0;
            }
            const RhsSet inner = subset(active);
            if ((rc = push_tol2())) return rc;
            LS_HIP(hipMemcpyAsync(dscale, scale.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(k_to32, dim3(kRedBlocks, inner.n), dim3(kThreads), 0, c->stream, c->r, c->b32, m, dscale,
                               c->x32, slot_map(inner));
            LS_HIP(hipGetLastError());
            if (c->bicgstab_l > 1) {
                // BiCGSTAB(l) runs over slots 0..n-1 with host-side activity flags; inactive systems' FP32
                // right-hand sides are zero (scale 0), so they finish at once
                hipLaunchKernelGGL(k_to32, gall, dim3(kThreads), 0, c->stream, c->r, c->b32, m, dscale, c->x32,
                                   slot_map(all));
                LS_HIP(hipGetLastError());
                auto apply32 = [&](const z64* in, z64* out) { return op_apply<float>(c, all, in, out, transposed); };
                const std::vector<z64*> vec = krylov_vectors<float>(c);
                std::vector<LState> ls;
                double worst = 0.0;
                for (int q = 0; q < nrhs; ++q)
                    if (active[q]) worst = std::max(worst, rel[q]);
                const double eta = std::min(1e-1, std::max(1e-7, kInnerAim * tol / worst));
                rc = bicgstab_l<float, float>(c, c->b32, c->x32, nullptr, vec.data(), c->bicgstab_l, nrhs, eta, maxit,
                                              apply32, ls, rel.data());
                if (rc) return rc;
                for (int q = 0; q < nrhs; ++q) {
                    if (!active[q]) continue;
                    inf[q].iters += ls[q].iters;
                    inf[q].matvecs += ls[q].matvecs;
                }
            } else {
                auto apply32 = [&](const RhsSet& set, const z64* in, z64* out) {
                    return op_apply<float>(c, set, in, out, transposed);
                };
                rc = bicgstab<float, float>(c, inner, c->b32, c->x32, nullptr, c->r32, c->rhat32, c->p32, c->v32,
                                            c->s32, c->t32, tol2v, maxit, apply32, iters, rel.data(), nullptr,
                                            !transposed, c->ph32, c->sh32, pre);
                if (rc) return rc;
                for (int i = 0; i < inner.n; ++i) {
                    const int q = inner.slot[i];
                    const double* sq = &c->red_host[(size_t)q * kStateLen];
                    const bool half = sq[S_DONE] == 1.0 && sq[S_SNORM2] == sq[S_RNORM2];
                    inf[q].iters += iters[q];
                    inf[q].matvecs += 2 * iters[q] - (half ? 1 : 0);
                }
            }
            LS_HIP(hipMemcpyAsync(dscale, inv.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(k_add32, dim3(kRedBlocks, inner.n), dim3(kThreads), 0, c->stream, u_out, c->x32, m,
                               dscale, slot_map(inner));
            LS_HIP(hipGetLastError());
            LS_HIP(hipStreamSynchronize(c->stream));
            for (int q = 0; q < nrhs; ++q)
                if (active[q]) inf[q].refinements += 1;
        }
        for (int q = 0; q < nrhs; ++q) {
            inf[q].rel_res_true = rel[q];
            inf[q].rel_res = rel[q];
            if (!std::isfinite(rel[q]))
                inf[q].status = LS_ERR_NONFINITE;
            else if (rel[q] > tol && nrm[q] > 0.0)
                inf[q].status = LS_ERR_NOT_CONVERGED;
        }
    }
    int worst = LS_OK;
    for (int q = 0; q < nrhs; ++q) {
        if (info) info[q] = inf[q];
        if (inf[q].status != LS_OK && worst == LS_OK) worst = inf[q].status;
    }
    if (worst != LS_OK) set_error("one or more systems did not reach the tolerance (see info[].status)");
    return worst;
}

}  // namespace ls
