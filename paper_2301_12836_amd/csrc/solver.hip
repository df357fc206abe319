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
#include <cmath>

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

// Loop helper: element indices of this thread for one right-hand side of length m.
#define LS_FOR_ELEMS(m) for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < (m); e += (long long)kRedBlocks * kThreads)

// r = b - ax (ax may be null), rhat = r, p = v = 0; partials: ||b||^2, ||r||^2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_init(const cpx<T>* __restrict__ b, const cpx<T>* __restrict__ ax,
                                                   cpx<T>* __restrict__ r, cpx<T>* __restrict__ rhat,
                                                   cpx<T>* __restrict__ p, cpx<T>* __restrict__ v, long long m,
                                                   double* partials) {
    __shared__ double sh[2 * kThreads];
    const int rr = blockIdx.y;
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
                                                       const double* __restrict__ state) {
    const int rr = blockIdx.y;
    const double* st = state + rr * kStateLen;
    if (st[S_ACTIVE] == 0.0) return;
    const cpx<T> beta = {(T)st[S_BETA], (T)st[S_BETA + 1]};
    const cpx<T> om = {(T)st[S_OMEGA], (T)st[S_OMEGA + 1]};
    const long long off = (long long)rr * m;
    LS_FOR_ELEMS(m) { p[off + e] = r[off + e] + beta * (p[off + e] - om * v[off + e]); }
}

// partials: r^H v (complex)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot(const cpx<T>* __restrict__ a, const cpx<T>* __restrict__ b,
                                                  long long m, const double* __restrict__ state, double* partials) {
    __shared__ double sh[2 * kThreads];
    const int rr = blockIdx.y;
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
                                                       const double* __restrict__ state, double* partials) {
    __shared__ double sh[2 * kThreads];
    const int rr = blockIdx.y;
    const double* st = state + rr * kStateLen;
    if (st[S_ACTIVE] == 0.0) return;
    const cpx<T> al = {(T)st[S_ALPHA], (T)st[S_ALPHA + 1]};
    const long long off = (long long)rr * m;
    double ss = 0;
    LS_FOR_ELEMS(m) {
        const cpx<T> sv = r[off + e] - al * v[off + e];
        s[off + e] = sv;
        ss += (double)sv.x * sv.x + (double)sv.y * sv.y;
    }
    write_partials(partials, rr, 0, ss, 0.0, sh);
}

// x += alpha p for the systems that converged at the half step
template <typename T, typename X>
__global__ __launch_bounds__(kThreads) void k_update_x_half(cpx<X>* __restrict__ x, const cpx<T>* __restrict__ p,
                                                            long long m, double* __restrict__ state) {
    const int rr = blockIdx.y;
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
                                                     double* partials) {
    __shared__ double sh[2 * kThreads];
    const int rr = blockIdx.y;
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
template <typename T, typename X>
__global__ __launch_bounds__(kThreads) void k_update_xr(cpx<X>* __restrict__ x, const cpx<T>* __restrict__ p,
                                                        const cpx<T>* __restrict__ s, const cpx<T>* __restrict__ t,
                                                        cpx<T>* __restrict__ r, const cpx<T>* __restrict__ rhat,
                                                        long long m, const double* __restrict__ state,
                                                        double* partials) {
    __shared__ double sh[2 * kThreads];
    const int rr = blockIdx.y;
    const double* st = state + rr * kStateLen;
    if (st[S_ACTIVE] == 0.0) return;
    const cpx<X> alx = {(X)st[S_ALPHA], (X)st[S_ALPHA + 1]};
    const cpx<X> omx = {(X)st[S_OMEGA], (X)st[S_OMEGA + 1]};
    const cpx<T> om = {(T)st[S_OMEGA], (T)st[S_OMEGA + 1]};
    const long long off = (long long)rr * m;
    double nr = 0, re = 0, im = 0;
    LS_FOR_ELEMS(m) {
        const cpx<T> pv = p[off + e], sv = s[off + e];
        x[off + e] = x[off + e] + alx * cpx<X>{(X)pv.x, (X)pv.y} + omx * cpx<X>{(X)sv.x, (X)sv.y};
        const cpx<T> rv = sv - om * t[off + e];
        r[off + e] = rv;
        const cpx<double> rw = wide(rv);
        nr += rw.x * rw.x + rw.y * rw.y;
        const cpx<double> z = cmulc(wide(rhat[off + e]), rw);
        re += z.x;
        im += z.y;
    }
    write_partials(partials, rr, 0, nr, 0.0, sh);
    write_partials(partials, rr, 2, re, im, sh);
}

// r = b - ax; partials ||r||^2, ||b||^2   (FP64 true residual)
__global__ __launch_bounds__(kThreads) void k_residual(const z128* __restrict__ b, const z128* __restrict__ ax,
                                                       z128* __restrict__ r, long long m, double* partials) {
    __shared__ double sh[2 * kThreads];
    const int rr = blockIdx.y;
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
                                                   const double* __restrict__ scale, z64* __restrict__ zero_out) {
    const int rr = blockIdx.y;
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
                                                    const double* __restrict__ scale) {
    const int rr = blockIdx.y;
    const double sc = scale[rr];
    if (sc == 0.0) return;
    const long long off = (long long)rr * m;
    LS_FOR_ELEMS(m) {
        const z64 dv = d[off + e];
        x[off + e] = x[off + e] + sc * z128{(double)dv.x, (double)dv.y};
    }
}

__global__ void k_copy(const z128* __restrict__ a, z128* __restrict__ b, long long m) {
    LS_FOR_ELEMS(m) { b[(long long)blockIdx.y * m + e] = a[(long long)blockIdx.y * m + e]; }
}

// Sum the kRedBlocks partials of each slot in a fixed order, then advance the scalars.
enum Phase { PH_INIT = 0, PH_ALPHA = 1, PH_S = 2, PH_OMEGA = 3, PH_RHO = 4, PH_RESID = 5 };

__global__ __launch_bounds__(kThreads) void k_finalize(const double* __restrict__ partials, double* __restrict__ state,
                                                       int phase, int nslots, double tol2, double* __restrict__ out) {
    __shared__ double sh[kRedSlots][kThreads];
    const int rr = blockIdx.x;
    double* st = state + rr * kStateLen;
    const int tid = threadIdx.x;
    if (phase != PH_INIT && phase != PH_RESID && st[S_ACTIVE] == 0.0) return;
    for (int q = 0; q < nslots; ++q) {
        double a = 0;
        for (int k = tid; k < kRedBlocks; k += kThreads) a += partials[((long long)rr * kRedSlots + q) * kRedBlocks + k];
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

__global__ void k_clear_half(double* state, int nrhs) {
    const int rr = threadIdx.x;
    if (rr < nrhs && state[rr * kStateLen + S_FLAG] == 1.0) state[rr * kStateLen + S_FLAG] = 0.0;
}

struct Vecs64 {
    z128 *r, *rhat, *p, *v, *s, *t;
};
struct Vecs32 {
    z64 *r, *rhat, *p, *v, *s, *t;
};

dim3 vgrid(int nrhs) { return dim3(kRedBlocks, nrhs); }

int finalize(Ctx* c, int phase, int nslots, int nrhs, double tol2 = 0.0, double* out = nullptr) {
    hipLaunchKernelGGL(k_finalize, dim3(nrhs), dim3(kThreads), 0, c->stream, c->partials, c->state, phase, nslots, tol2,
                       out);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

// Generic BiCGSTAB.  T: vector precision, X: iterate precision (x is cpx<X>), ApplyFn(in, out).
template <typename T, typename X, typename ApplyFn>
int bicgstab(Ctx* c, const cpx<T>* b, cpx<X>* x, const cpx<T>* ax0, cpx<T>* r, cpx<T>* rhat, cpx<T>* p, cpx<T>* v,
             cpx<T>* s, cpx<T>* t, int nrhs, double tol, int maxit, ApplyFn apply, std::vector<int>& iters,
             const double* hscale = nullptr) {
    const long long m = (long long)c->field_elems();
    const dim3 g = vgrid(nrhs);
    hipLaunchKernelGGL((k_init<T>), g, dim3(kThreads), 0, c->stream, b, ax0, r, rhat, p, v, m, c->partials);
    LS_HIP(hipGetLastError());
    int rc = finalize(c, PH_INIT, 2, nrhs, tol * tol);
    if (rc) return rc;
    // One iteration is a fixed sequence of launches whose scalars live on the device, so it is
    // captured once into a graph and replayed; the host only reads the active flags in between.
    auto body = [&]() -> int {
        int brc;
        c->prof.begin(c->stream, LS_PNAME(T, "blas1"));
        hipLaunchKernelGGL((k_update_p<T>), g, dim3(kThreads), 0, c->stream, r, p, v, m, c->state);
        c->prof.end(c->stream);
        if ((brc = apply(p, v))) return brc;
        c->prof.begin(c->stream, LS_PNAME(T, "blas1"));
        hipLaunchKernelGGL((k_dot<T>), g, dim3(kThreads), 0, c->stream, rhat, v, m, c->state, c->partials);
        c->prof.end(c->stream);
        if ((brc = finalize(c, PH_ALPHA, 2, nrhs))) return brc;
        c->prof.begin(c->stream, LS_PNAME(T, "blas1"));
        hipLaunchKernelGGL((k_update_s<T>), g, dim3(kThreads), 0, c->stream, r, v, s, m, c->state, c->partials);
        c->prof.end(c->stream);
        if ((brc = finalize(c, PH_S, 1, nrhs))) return brc;
        hipLaunchKernelGGL((k_update_x_half<T, X>), g, dim3(kThreads), 0, c->stream, x, p, m, c->state);
        hipLaunchKernelGGL(k_clear_half, dim3(1), dim3(64), 0, c->stream, c->state, nrhs);
        if ((brc = apply(s, t))) return brc;
        c->prof.begin(c->stream, LS_PNAME(T, "blas1"));
        hipLaunchKernelGGL((k_dot_ts<T>), g, dim3(kThreads), 0, c->stream, t, s, m, c->state, c->partials);
        c->prof.end(c->stream);
        if ((brc = finalize(c, PH_OMEGA, 3, nrhs))) return brc;
        c->prof.begin(c->stream, LS_PNAME(T, "blas1"));
        hipLaunchKernelGGL((k_update_xr<T, X>), g, dim3(kThreads), 0, c->stream, x, p, s, t, r, rhat, m, c->state,
                           c->partials);
        c->prof.end(c->stream);
        if ((brc = finalize(c, PH_RHO, 4, nrhs))) return brc;
        LS_HIP(hipGetLastError());
        return LS_OK;
    };
    struct GraphGuard {
        hipGraphExec_t exec = nullptr;
        ~GraphGuard() {
            if (exec) (void)hipGraphExecDestroy(exec);
        }
    } guard;
    if (!(c->flags & LS_FLAG_NO_GRAPH) && !c->prof.on && c->stream != nullptr) {
        LS_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        const int brc = body();
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
    }
    // FP32 inner solves stop a right-hand side whose residual has not improved on its best by 10 % for
    // kStall iterations (its attainable accuracy is reached; the FP64 refinement restarts from the true
    // residual).  FP64 solves run to tol or maxit.
    constexpr int kStall = 30;
    std::vector<double> best(nrhs, std::numeric_limits<double>::infinity());
    std::vector<int> since(nrhs, 0), last_it(nrhs, 0);
    static const double zero = 0.0;
    for (int it = 0; it < maxit; ++it) {
        if (guard.exec) {
            LS_HIP(hipGraphLaunch(guard.exec, c->stream));
        } else if ((rc = body())) {
            return rc;
        }
        LS_HIP(hipMemcpyAsync(c->red_host, c->state, sizeof(double) * nrhs * kStateLen, hipMemcpyDeviceToHost,
                              c->stream));
        LS_HIP(hipStreamSynchronize(c->stream));
        bool any = false;
        for (int q = 0; q < nrhs; ++q) {
            const double* sq = &c->red_host[q * kStateLen];
            // relative residual of each completed iteration (scaled to the caller's system)
            if ((int)sq[S_ITERS] > last_it[q] && sq[S_BNORM2] > 0.0 && (size_t)q < c->history.size()) {
                last_it[q] = (int)sq[S_ITERS];
                c->history[q].push_back(std::sqrt(sq[S_RNORM2] / sq[S_BNORM2]) * (hscale ? hscale[q] : 1.0));
            }
            if (sq[S_ACTIVE] == 0.0) continue;
            if (sizeof(T) == 4) {
                if (sq[S_RNORM2] < 0.81 * best[q]) {  // 10 % on the norm
                    best[q] = sq[S_RNORM2];
                    since[q] = 0;
                } else if (++since[q] >= kStall) {
                    LS_HIP(hipMemcpyAsync(c->state + q * kStateLen + S_ACTIVE, &zero, sizeof(double),
                                          hipMemcpyHostToDevice, c->stream));
                    continue;
                }
            }
            any = true;
        }
        if (!any) break;
    }
    LS_HIP(hipMemcpyAsync(c->red_host, c->state, sizeof(double) * nrhs * kStateLen, hipMemcpyDeviceToHost, c->stream));
    LS_HIP(hipStreamSynchronize(c->stream));
    iters.resize(nrhs);
    for (int q = 0; q < nrhs; ++q) iters[q] = (int)c->red_host[q * kStateLen + S_ITERS];
    return LS_OK;
}

// ||b - A x|| / ||b|| per system with the FP64 operator; writes r = b - A x if r != null.
// the operator or its transpose
template <typename T>
int op_apply(Ctx* c, int i_omega, const cpx<T>* in, cpx<T>* out, int nrhs, bool transposed) {
    return transposed ? apply_T_op<T>(c, i_omega, in, out, nrhs) : apply_op<T>(c, i_omega, in, out, nrhs);
}

int true_residual(Ctx* c, int i_omega, const z128* b, const z128* x, z128* ax, z128* r, int nrhs,
                  std::vector<double>& rel, std::vector<double>& abs_, bool transposed) {
    int rc = op_apply<double>(c, i_omega, x, ax, nrhs, transposed);
    if (rc) return rc;
    const long long m = (long long)c->field_elems();
    hipLaunchKernelGGL(k_residual, vgrid(nrhs), dim3(kThreads), 0, c->stream, b, ax, r, m, c->partials);
    LS_HIP(hipGetLastError());
    if ((rc = finalize(c, PH_RESID, 2, nrhs, 0.0, c->red))) return rc;
    LS_HIP(hipMemcpyAsync(c->red_host, c->red, sizeof(double) * 2 * kRedBlocks, hipMemcpyDeviceToHost, c->stream));
    LS_HIP(hipStreamSynchronize(c->stream));
    rel.assign(c->red_host, c->red_host + nrhs);
    abs_.assign(c->red_host + kRedBlocks, c->red_host + kRedBlocks + nrhs);
    return LS_OK;
}

}  // namespace

int solve_systems(Ctx* c, int i_omega, const z128* b, int nrhs, double tol, int maxit, int precision, const z128* x0,
                  z128* u_out, ls_info* info, bool transposed) {
    const long long m = (long long)c->field_elems();
    std::vector<ls_info> inf(nrhs);
    for (auto& q : inf) q = ls_info{0, 0, 0, LS_OK, 0.0, 0.0};
    c->history.assign(nrhs, std::vector<double>());
    // x = x0 or 0
    if (x0) {
        hipLaunchKernelGGL(k_copy, vgrid(nrhs), dim3(kThreads), 0, c->stream, x0, u_out, m);
        LS_HIP(hipGetLastError());
    } else {
        LS_HIP(hipMemsetAsync(u_out, 0, sizeof(z128) * m * nrhs, c->stream));
    }
    std::vector<double> rel, nrm;
    std::vector<int> iters;
    int rc = LS_OK;
    if (precision == LS_PREC_C128) {
        auto apply = [&](const z128* in, z128* out) { return op_apply<double>(c, i_omega, in, out, nrhs, transposed); };
        // A breakdown (rho = 0 or rhat^H v = 0) restarts once from the current iterate, which re-seeds the
        // shadow residual with the current residual; systems already within tol take no further iteration.
        std::vector<double> st;
        std::vector<int> total(nrhs, 0), extra(nrhs, 0);
        for (int attempt = 0; attempt < 2; ++attempt) {
            const z128* ax0 = nullptr;
            if (x0 || attempt > 0) {
                if ((rc = op_apply<double>(c, i_omega, u_out, c->t, nrhs, transposed))) return rc;
                ax0 = c->t;
                for (int q = 0; q < nrhs; ++q) extra[q] += 1;
            }
            rc = bicgstab<double, double>(c, b, u_out, ax0, c->r, c->rhat, c->p, c->v, c->s, c->t, nrhs, tol, maxit,
                                          apply, iters);
            if (rc) return rc;
            st.assign(c->red_host, c->red_host + (size_t)nrhs * kStateLen);
            bool broke = false;
            for (int q = 0; q < nrhs; ++q) {
                const double* sq = &st[(size_t)q * kStateLen];
                const bool half = sq[S_DONE] == 1.0 && sq[S_SNORM2] == sq[S_RNORM2];
                total[q] += iters[q];
                extra[q] += 2 * iters[q] - (half ? 1 : 0);
                broke = broke || sq[S_FLAG] == 2.0;
            }
            if (!broke) break;
        }
        if ((rc = true_residual(c, i_omega, b, u_out, c->v, nullptr, nrhs, rel, nrm, transposed))) return rc;
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
        // outer FP64 refinement: r = b - A x (FP64), inner FP32 BiCGSTAB on A d = r / ||r||
        const int max_outer = 30;
        std::vector<double> scale(nrhs), inv(nrhs);
        std::vector<int> active(nrhs, 1);
        int outer = 0;
        double* dscale = c->red + 2 * kRedBlocks;
        for (; outer <= max_outer; ++outer) {
            if (outer == 0 && !x0) {
                // x = 0, so A x = 0 and r = b
                LS_HIP(hipMemsetAsync(c->v, 0, sizeof(z128) * m * nrhs, c->stream));
                hipLaunchKernelGGL(k_residual, vgrid(nrhs), dim3(kThreads), 0, c->stream, b, c->v, c->r, m,
                                   c->partials);
                LS_HIP(hipGetLastError());
                if ((rc = finalize(c, PH_RESID, 2, nrhs, 0.0, c->red))) return rc;
                LS_HIP(hipMemcpyAsync(c->red_host, c->red, sizeof(double) * 2 * kRedBlocks, hipMemcpyDeviceToHost,
                                      c->stream));
                LS_HIP(hipStreamSynchronize(c->stream));
                rel.assign(c->red_host, c->red_host + nrhs);
                nrm.assign(c->red_host + kRedBlocks, c->red_host + kRedBlocks + nrhs);
            } else {
                if ((rc = true_residual(c, i_omega, b, u_out, c->v, c->r, nrhs, rel, nrm, transposed))) return rc;
                for (int q = 0; q < nrhs; ++q) inf[q].matvecs += 1;
            }
            bool any = false;
            double worst = 0.0;
            for (int q = 0; q < nrhs; ++q) {
                active[q] = rel[q] > tol && std::isfinite(rel[q]) && nrm[q] > 0.0;
                any = any || active[q];
                if (active[q]) worst = std::max(worst, rel[q]);
            }
            if (!any || outer == max_outer) break;
            // inner tolerance: the reduction that reaches 0.3 tol, capped at 0.1 and floored at 1e-7 (near
            // the FP32 operator's relative accuracy; a stagnating inner solve is stopped early anyway)
            const double eta = std::min(1e-1, std::max(1e-7, 0.3 * tol / worst));
            for (int q = 0; q < nrhs; ++q) {
                scale[q] = active[q] ? 1.0 / nrm[q] : 0.0;
                inv[q] = active[q] ? nrm[q] : 0.0;
            }
            LS_HIP(hipMemcpyAsync(dscale, scale.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(k_to32, vgrid(nrhs), dim3(kThreads), 0, c->stream, c->r, c->b32, m, dscale, c->x32);
            LS_HIP(hipGetLastError());
            auto apply32 = [&](const z64* in, z64* out) {
                return op_apply<float>(c, i_omega, in, out, nrhs, transposed);
            };
            rc = bicgstab<float, float>(c, c->b32, c->x32, nullptr, c->r32, c->rhat32, c->p32, c->v32, c->s32, c->t32,
                                        nrhs, eta, maxit, apply32, iters, rel.data());
            if (rc) return rc;
            for (int q = 0; q < nrhs; ++q) {
                if (!active[q]) continue;
                const double* sq = &c->red_host[(size_t)q * kStateLen];
                const bool half = sq[S_DONE] == 1.0 && sq[S_SNORM2] == sq[S_RNORM2];
                inf[q].iters += iters[q];
                inf[q].matvecs += 2 * iters[q] - (half ? 1 : 0);
            }
            LS_HIP(hipMemcpyAsync(dscale, inv.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(k_add32, vgrid(nrhs), dim3(kThreads), 0, c->stream, u_out, c->x32, m, dscale);
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
