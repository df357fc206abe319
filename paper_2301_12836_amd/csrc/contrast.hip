// Contrast kernels of the LS operator: f = B u = -E^T (dC (E u)) + w^2 drho u  (Eq 8, 11-12, 17-18).
//
// E is the Voigt engineering strain by second-order central differences, with the first-order
// one-sided difference on the model boundary (Eq 18); E^T is its exact discrete adjoint, so the
// divergence of the contrast stress is -E^T tau.  Per cell, tau = dC eps with dC the symmetric
// 6x6 of the cell (21 packed values).  The first kernel writes tau for every cell, the second
// forms f and writes it straight into the zero-padded FFT work buffer.
#include "fft_reg.h"

namespace ls {

namespace {

constexpr int kThreads = 256;

// packed index of the upper-triangle entry (I, J), I <= J, row order 11,12,...,16,22,...,66
__host__ __device__ constexpr int packed(int I, int J) {
    return I <= J ? I * 6 - I * (I - 1) / 2 + (J - I) : J * 6 - J * (J - 1) / 2 + (I - J);
}

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

// tau[r][6][n] = dC(p) eps(u_r)(p)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_strain_stress(const cpx<T>* __restrict__ u, cpx<T>* __restrict__ tau,
                                                            const T* __restrict__ dc, int nrhs, int N1, int N2,
                                                            int N3, T inv_h) {
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
        strain_at(u + (long long)r * 3 * n, n, p, i, j, k, N1, N2, N3, inv_h, eps);
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

// f_c(p) = -sum_a (D_a^T tau_{V(a,c)})(p) + w^2 drho(p) u_c(p).
// OUT 0: f written to work[r][c][z][y][x] (row pitch L1, plane pitch L2 L1, component pitch N3 L2 L1).
// OUT 1: the transposed operator's epilogue, work[compact] = y - f (work is then a compact field array).
template <typename T, int OUT>
__global__ __launch_bounds__(kThreads) void k_divergence(const cpx<T>* __restrict__ tau, const cpx<T>* __restrict__ u,
                                                         const T* __restrict__ drho, cpx<T>* __restrict__ work,
                                                         int nrhs, int N1, int N2, int N3, int L1, int L2, T inv_h,
                                                         T w2, const cpx<T>* __restrict__ y) {
    const long long n = (long long)N1 * N2 * N3;
    const long long lb = xcd_logical_block(blockIdx.x, (n + kThreads - 1) / kThreads);
    const long long p = lb * kThreads + threadIdx.x;
    if (lb < 0 || p >= n) return;
    const int i = (int)(p % N1);
    const int j = (int)((p / N1) % N2);
    const int k = (int)(p / ((long long)N1 * N2));
    const long long sx = 1, sy = N1, sz = (long long)N1 * N2;
    const T wr = w2 * drho[p];
    const long long cpitch = (long long)N3 * L2 * L1;
    const long long wpos = ((long long)k * L2 + j) * L1 + i;
    for (int r = 0; r < nrhs; ++r) {
        const cpx<T>* t = tau + (long long)r * 6 * n;
        const cpx<T>* ur = u + (long long)r * 3 * n;
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
            const cpx<T>* yr = y + (long long)r * 3 * n;
            cpx<T>* o = work + (long long)r * 3 * n;
            o[p] = yr[p] - (wr * ur[p] - f0);
            o[n + p] = yr[n + p] - (wr * ur[n + p] - f1);
            o[2 * n + p] = yr[2 * n + p] - (wr * ur[2 * n + p] - f2);
        }
    }
}

// compact field f[r][c][n] -> zero-padded work[r][c][z][y][x] (data cells only)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_to_work(const cpx<T>* __restrict__ f, cpx<T>* __restrict__ work,
                                                      int nrhs, int N1, int N2, int N3, int L1, int L2) {
    const long long n = (long long)N1 * N2 * N3;
    const long long p = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n) return;
    const int i = (int)(p % N1);
    const int j = (int)((p / N1) % N2);
    const int k = (int)(p / ((long long)N1 * N2));
    const long long cpitch = (long long)N3 * L2 * L1;
    const long long wpos = ((long long)k * L2 + j) * L1 + i;
    for (int r = 0; r < 3 * nrhs; ++r) work[r * cpitch + wpos] = f[r * n + p];
}

// Gradient of a real misfit with respect to the contrast at every cell, for forward fields u and
// adjoint-side fields mu = conj(Gconv lambda_bar) (lambda_bar solving A^T lambda_bar = conj(P^H r)):
//   g21[JK](p) += -Re[conj(eps_J(mu)) eps_K(u) + (J != K) conj(eps_K(mu)) eps_J(u)]   (packed J <= K)
//   grho(p)    += w^2 Re[sum_c conj(mu_c) u_c]
// summed over the nrhs (u, mu) pairs.
__global__ __launch_bounds__(kThreads) void k_grad_contrast(const z128* __restrict__ u, const z128* __restrict__ mu,
                                                            double* __restrict__ g21, double* __restrict__ grho,
                                                            int nrhs, int N1, int N2, int N3, double inv_h, double w2) {
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
#pragma unroll
    for (int q = 0; q < 21; ++q) g21[q * n + p] += acc[q];
    grho[p] += w2 * ar;
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

__global__ void k_fold(const double* __restrict__ dc_in, const double* __restrict__ drho_in, double* __restrict__ dc,
                       double* __restrict__ drho, float* __restrict__ dc32, float* __restrict__ drho32, long long n,
                       const double* __restrict__ fold21) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    for (int q = 0; q < 21; ++q) {
        const double v = dc_in[q * n + p] + fold21[q];
        dc[q * n + p] = v;
        if (dc32) dc32[q * n + p] = (float)v;
    }
    drho[p] = drho_in[p];
    if (drho32) drho32[p] = (float)drho_in[p];
}

template <typename T>
const T* contrast_of(const Ctx* c);
template <>
const double* contrast_of<double>(const Ctx* c) { return c->dc; }
template <>
const float* contrast_of<float>(const Ctx* c) { return c->dc32; }
template <typename T>
const T* density_of(const Ctx* c);
template <>
const double* density_of<double>(const Ctx* c) { return c->drho; }
template <>
const float* density_of<float>(const Ctx* c) { return c->drho32; }

}  // namespace

template <typename T>
int contrast_to_work(Ctx* c, int i_omega, const cpx<T>* u, cpx<T>* work, cpx<T>* tau, int nrhs) {
    const long long n = c->ncell;
    // XCD-aware order: grid padded to a multiple of 8, neighbouring cells share an L2
    const unsigned nb = (unsigned)(((n + kThreads - 1) / kThreads + 7) / 8 * 8);
    const T inv_h = T(1.0 / c->h);
    const double w = c->omega[i_omega];
    c->prof.begin(c->stream, LS_PNAME(T, "contrast_strain_stress"));
    hipLaunchKernelGGL((k_strain_stress<T>), dim3(nb), dim3(kThreads), 0, c->stream, u, tau, contrast_of<T>(c), nrhs,
                       c->n1, c->n2, c->n3, inv_h);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    c->prof.begin(c->stream, LS_PNAME(T, "contrast_divergence"));
    hipLaunchKernelGGL((k_divergence<T, 0>), dim3(nb), dim3(kThreads), 0, c->stream, tau, u, density_of<T>(c), work,
                       nrhs, c->n1, c->n2, c->n3, c->L1, c->L2, inv_h, T(w * w), nullptr);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

template int contrast_to_work<double>(Ctx*, int, const z128*, z128*, z128*, int);
template int contrast_to_work<float>(Ctx*, int, const z64*, z64*, z64*, int);

// out = y - B g  (the last step of the transposed operator A^T y = y - B Gconv y, with g = Gconv y)
template <typename T>
int contrast_transposed_epilogue(Ctx* c, int i_omega, const cpx<T>* g, const cpx<T>* y, cpx<T>* out, cpx<T>* tau,
                                 int nrhs) {
    const long long n = c->ncell;
    const unsigned nb = (unsigned)(((n + kThreads - 1) / kThreads + 7) / 8 * 8);
    const T inv_h = T(1.0 / c->h);
    const double w = c->omega[i_omega];
    c->prof.begin(c->stream, LS_PNAME(T, "contrast_strain_stress"));
    hipLaunchKernelGGL((k_strain_stress<T>), dim3(nb), dim3(kThreads), 0, c->stream, g, tau, contrast_of<T>(c), nrhs,
                       c->n1, c->n2, c->n3, inv_h);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    c->prof.begin(c->stream, LS_PNAME(T, "contrast_divergence_T"));
    hipLaunchKernelGGL((k_divergence<T, 1>), dim3(nb), dim3(kThreads), 0, c->stream, tau, g, density_of<T>(c), out,
                       nrhs, c->n1, c->n2, c->n3, c->L1, c->L2, inv_h, T(w * w), y);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

template int contrast_transposed_epilogue<double>(Ctx*, int, const z128*, const z128*, z128*, z128*, int);
template int contrast_transposed_epilogue<float>(Ctx*, int, const z64*, const z64*, z64*, z64*, int);

template <typename T>
int to_work(Ctx* c, const cpx<T>* f, cpx<T>* work, int nrhs) {
    const long long n = c->ncell;
    const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
    c->prof.begin(c->stream, LS_PNAME(T, "to_work"));
    hipLaunchKernelGGL((k_to_work<T>), dim3(nb), dim3(kThreads), 0, c->stream, f, work, nrhs, c->n1, c->n2, c->n3,
                       c->L1, c->L2);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

template int to_work<double>(Ctx*, const z128*, z128*, int);
template int to_work<float>(Ctx*, const z64*, z64*, int);

int grad_contrast_launch(Ctx* c, int i_omega, const z128* u, const z128* mu, int nrhs, double* g21, double* grho) {
    const long long n = c->ncell;
    const unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
    const double w = c->omega[i_omega];
    c->prof.begin(c->stream, "grad_contrast.c128");
    hipLaunchKernelGGL(k_grad_contrast, dim3(nb), dim3(kThreads), 0, c->stream, u, mu, g21, grho, nrhs, c->n1, c->n2,
                       c->n3, 1.0 / c->h, w * w);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
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

int fold_background(Ctx* c, const double* dc_in, const double* drho_in, const double fold21[21]) {
    double* dfold = nullptr;
    LS_HIP(hipMallocAsync((void**)&dfold, 21 * sizeof(double), c->stream));
    LS_HIP(hipMemcpyAsync(dfold, fold21, 21 * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const long long n = c->ncell;
    hipLaunchKernelGGL(k_fold, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, dc_in, drho_in, c->dc, c->drho,
                       c->dc32, c->drho32, n, dfold);
    LS_HIP(hipGetLastError());
    LS_HIP(hipStreamSynchronize(c->stream));
    LS_HIP(hipFreeAsync(dfold, c->stream));
    LS_HIP(hipStreamSynchronize(c->stream));
    return LS_OK;
}

}  // namespace ls
