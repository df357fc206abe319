// Point-block Jacobi preconditioner of the LS system A u = u0 (Eq 19-21), applied on the right inside
// Bi-CGSTAB: M = blockdiag_x D(x), with D(x) the 3x3 block of A = I - Gconv B that couples the three
// components at cell x with themselves,
//   D(x)_ic = delta_ic - sum_{x'} sum_j h^3 G_ij(x - x') B[(j, x'), (c, x)].
// Column (c, x) of B = -E^T dC E + w^2 drho is a strain stencil followed by its adjoint: the strain of the unit
// displacement e_c at x lives on x and its six face neighbours r, and its divergence on the neighbours q of
// those, so only the Green's tensor at offsets within [-2, 2]^3 enters:
//   D(x)_ic = delta_ic + sum_r sum_b sum_{q = r + t e_b} D_b[r, q] sum_j h^3 G_ij(x - q) tau_{V(b, j)}(r)
//             - w^2 drho(x) h^3 G_ic(0),
//   tau(r) = dC(r) eps(r),  eps_J(r) = sum_a [V(a, c) = J] D_a[r, x],
// with D_a the one-dimensional derivative of Eq 18 along axis a (central inside, one-sided at the ends) and
// V the Voigt index.  The blocks are built per frequency at set-up in FP64, inverted (adjugate over the
// determinant) and kept as M^-1 in FP64 and, for mixed precision, FP32.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace ls {

namespace {

constexpr int kThreads = 256;

// packed upper-triangle index of the Voigt pair (I, J), row order 11,12,...,16,22,...,66
__device__ __forceinline__ int packed21(int I, int J) {
    if (I > J) {
        const int t = I;
        I = J;
        J = t;
    }
    return I * 6 - I * (I - 1) / 2 + (J - I);
}

// Voigt index of the pair of axes (a, b), order 11 22 33 23 13 12 (also the order of the six stored
// components of the symmetric Green's tensor)
__device__ __forceinline__ int voigt(int a, int b) {
    if (a == b) return a;
    const int s = a + b;   // (1,2) -> 3, (0,2) -> 4, (0,1) -> 5
    return s == 3 ? 3 : (s == 2 ? 4 : 5);
}

// entry (row, col) of the derivative matrix along an axis of n cells (Eq 18)
__device__ __forceinline__ double dcoef(int row, int col, int n, double ih) {
    if (row == 0) return col == 0 ? -ih : (col == 1 ? ih : 0.0);
    if (row == n - 1) return col == n - 1 ? ih : (col == n - 2 ? -ih : 0.0);
    return col == row + 1 ? 0.5 * ih : (col == row - 1 ? -0.5 * ih : 0.0);
}

// per cell: D (FP64), its inverse into minv[(3 a + b) n + p] (and minv32); bad counts singular or
// non-finite blocks
__global__ __launch_bounds__(kThreads) void k_block_jacobi(const double* __restrict__ dc,
                                                           const double* __restrict__ drho,
                                                           const z128* __restrict__ loc, double w2, int N1, int N2,
                                                           int N3, double ih, z128* __restrict__ minv,
                                                           z64* __restrict__ minv32, int* __restrict__ bad) {
    const long long n = (long long)N1 * N2 * N3;
    const long long p = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n) return;
    const int P[3] = {(int)(p % N1), (int)((p / N1) % N2), (int)(p / ((long long)N1 * N2))};
    const int NN[3] = {N1, N2, N3};
    const long long stride[3] = {1, N1, (long long)N1 * N2};
    z128 D[3][3];
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) D[i][c] = {i == c ? 1.0 : 0.0, 0.0};
    for (int c = 0; c < 3; ++c) {
        // r runs over x (ra = -1) and x +- e_ra
        for (int cand = 0; cand < 7; ++cand) {
            const int ra = cand == 0 ? -1 : (cand - 1) >> 1;
            const int rs = cand == 0 ? 0 : ((cand & 1) ? -1 : 1);
            int R[3] = {P[0], P[1], P[2]};
            if (ra >= 0) R[ra] += rs;
            if (ra >= 0 && (R[ra] < 0 || R[ra] >= NN[ra])) continue;
            double eps[6] = {0, 0, 0, 0, 0, 0};
            bool any = false;
            for (int a = 0; a < 3; ++a) {
                if (ra >= 0 && ra != a) continue;   // r differs from x along ra only
                const double w = dcoef(R[a], P[a], NN[a], ih);
                if (w == 0.0) continue;
                eps[voigt(a, c)] += w;
                any = true;
            }
            if (!any) continue;
            const long long rp = p + (ra >= 0 ? rs * stride[ra] : 0);
            double tau[6];
            for (int I = 0; I < 6; ++I) {
                double acc = 0.0;
                for (int J = 0; J < 6; ++J) acc += dc[packed21(I, J) * n + rp] * eps[J];
                tau[I] = acc;
            }
            for (int b = 0; b < 3; ++b)
                for (int t = -1; t <= 1; ++t) {
                    const int qb = R[b] + t;
                    if (qb < 0 || qb >= NN[b]) continue;
                    const double d = dcoef(R[b], qb, NN[b], ih);
                    if (d == 0.0) continue;
                    // offset x - q
                    int o[3] = {P[0] - R[0], P[1] - R[1], P[2] - R[2]};
                    o[b] -= t;
                    const z128* g = loc + (((o[2] + 2) * 5 + (o[1] + 2)) * 5 + (o[0] + 2)) * 6;
                    for (int i = 0; i < 3; ++i) {
                        z128 acc = {0.0, 0.0};
                        for (int j = 0; j < 3; ++j) acc = acc + tau[voigt(b, j)] * g[voigt(i, j)];
                        D[i][c] = D[i][c] + d * acc;
                    }
                }
        }
    }
    const double wr = w2 * drho[p];
    const z128* g0 = loc + 62 * 6;   // offset 0
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) D[i][c] = D[i][c] - wr * g0[voigt(i, c)];
    // inverse by the adjugate
    z128 A[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
            A[i][j] = D[i1][j1] * D[i2][j2] - D[i1][j2] * D[i2][j1];   // cofactor (j, i)
        }
    const z128 det = D[0][0] * A[0][0] + D[0][1] * A[1][0] + D[0][2] * A[2][0];
    const double dd = det.x * det.x + det.y * det.y;
    z128 inv[3][3];
    if (!(dd > 0.0) || !(dd < 1e300)) {
        atomicAdd(bad, 1);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) inv[i][j] = {i == j ? 1.0 : 0.0, 0.0};
    } else {
        const z128 idet = {det.x / dd, -det.y / dd};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) inv[i][j] = A[i][j] * idet;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            minv[(3 * i + j) * n + p] = inv[i][j];
            if (minv32) minv32[(3 * i + j) * n + p] = {(float)inv[i][j].x, (float)inv[i][j].y};
        }
}

}  // namespace

int build_block_jacobi(Ctx* c) {
    if (!c->precond) return LS_OK;
    const long long n = c->ncell;
    int* bad = (int*)c->stage;
    LS_HIP(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
    for (size_t i = 0; i < c->omega.size(); ++i) {
        int rc = local_green_table(c, (int)i, c->gloc);
        if (rc) return rc;
        const double w = c->omega[i];
        hipLaunchKernelGGL(k_block_jacobi, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                           c->stream, c->dc, c->drho, (const z128*)c->gloc, w * w, c->n1, c->n2, c->n3, 1.0 / c->h,
                           c->minv[i], c->mixed ? c->minv32[i] : nullptr, bad);
        LS_HIP(hipGetLastError());
    }
    int hbad = 0;
    LS_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    LS_HIP(hipStreamSynchronize(c->stream));
    if (hbad) return fail(LS_ERR_NONFINITE, "block-Jacobi preconditioner: " + std::to_string(hbad) +
                                                " diagonal blocks of the operator are singular or not finite");
    return LS_OK;
}

}  // namespace ls
