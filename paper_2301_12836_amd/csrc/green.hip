// Background Green's tensor (Eq 7, Appendix A), its k-space table for the convolution of Eq 21,
// and the incident fields of point forces and moment tensors (Eq 6, 13-16).
//
// Isotropic background, time convention e^{-i w t}:
//   exact     G = gg e^{i w r/a}/(4 pi rho a^2 r) + (I - gg) e^{i w r/b}/(4 pi rho b^2 r)
//                 + (3 gg - I) J(r)/(4 pi rho r^3),  J(r) = int_{r/a}^{r/b} tau e^{i w tau} dtau,
//             the closed-form solution of Eq 7 (its 1/r part is the far-field tensor A.5 and its
//             last term tends to the near-field tensor A.4 as w -> 0);
//   paper_sum G = A.4 + A.5.
// The cell at zero offset takes the average of the exact tensor over the sphere of volume h^3:
//   h^3 G(0) = [I(w/a)/(3 a^2) + 2 I(w/b)/(3 b^2)] / rho * Identity,  I(k) = int_0^R r e^{i k r} dr,
//   R = (3/(4 pi))^{1/3} h  (the angular mean of gg is I/3, that of 3gg - I is 0).
#include <cmath>

#include "common.h"

namespace ls {

namespace {

constexpr double kPi = 3.14159265358979323846;

struct GreenParams {
    double w, alpha, beta, rho;
    int mode;
};

// J = int_{t1}^{t2} tau e^{i w tau} dtau.  Closed form [e^{i w tau}(1/w^2 - i tau/w)]; where
// |w t2| < 0.5 the two terms cancel to O((w t)^2) and the integrated power series of the
// exponential is summed instead: J = sum_n (i w)^n/n! (t2^{n+2} - t1^{n+2})/(n+2).
__host__ __device__ inline z128 tau_moment(double w, double t1, double t2) {
    if (fabs(w * t2) < 0.5) {
        z128 acc = {0.0, 0.0};
        z128 coef = {1.0, 0.0};
        double p1 = t1 * t1, p2 = t2 * t2;
        for (int n = 0; n < 40; ++n) {
            const double d = (p2 - p1) / (n + 2);
            acc.x += coef.x * d;
            acc.y += coef.y * d;
            // coef *= i w / (n + 1)
            const double s = w / (n + 1);
            const z128 nc = {-coef.y * s, coef.x * s};
            coef = nc;
            p1 *= t1;
            p2 *= t2;
        }
        return acc;
    }
    double s2, c2, s1, c1;
    sincos(w * t2, &s2, &c2);
    sincos(w * t1, &s1, &c1);
    const double a = 1.0 / (w * w);
    // e^{i w t}(a - i t / w) = (c + i s)(a - i b),  b = t / w
    const double b2 = t2 / w, b1 = t1 / w;
    const z128 f2 = {c2 * a + s2 * b2, s2 * a - c2 * b2};
    const z128 f1 = {c1 * a + s1 * b1, s1 * a - c1 * b1};
    return {f2.x - f1.x, f2.y - f1.y};
}

// the six distinct components (11, 22, 33, 23, 13, 12) of G at offset (dx, dy, dz) != 0
__device__ inline void green6(double dx, double dy, double dz, const GreenParams& P, z128 g[6]) {
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double ir = 1.0 / r;
    const double gm[3] = {dx * ir, dy * ir, dz * ir};
    const double four_pi_rho = 4.0 * kPi * P.rho;
    double sp, cp, ss, cs;
    sincos(P.w * r / P.alpha, &sp, &cp);
    sincos(P.w * r / P.beta, &ss, &cs);
    const double ap = 1.0 / (four_pi_rho * P.alpha * P.alpha * r);
    const double as = 1.0 / (four_pi_rho * P.beta * P.beta * r);
    const z128 pt = {ap * cp, ap * sp};
    const z128 st = {as * cs, as * ss};
    z128 cgg, cdel;  // G_ij = gg_ij * cgg + delta_ij * cdel
    if (P.mode == LS_GREEN_EXACT) {
        const z128 J = tau_moment(P.w, r / P.alpha, r / P.beta);
        const double an = 1.0 / (four_pi_rho * r * r * r);
        const z128 nt = {an * J.x, an * J.y};
        cgg = {pt.x - st.x + 3.0 * nt.x, pt.y - st.y + 3.0 * nt.y};
        cdel = {st.x - nt.x, st.y - nt.y};
    } else {
        // A.4: -(1/(8 pi rho r b^2))(1 - b^2/a^2)(I - 3 gg)
        const double cnf = -(1.0 - (P.beta * P.beta) / (P.alpha * P.alpha)) / (8.0 * kPi * P.rho * r * P.beta * P.beta);
        cgg = {pt.x - st.x - 3.0 * cnf, pt.y - st.y};
        cdel = {st.x + cnf, st.y};
    }
    const int pa[6] = {0, 1, 2, 1, 0, 0};
    const int pb[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double gg = gm[pa[q]] * gm[pb[q]];
        g[q] = {gg * cgg.x, gg * cgg.y};
        if (q < 3) {
            g[q].x += cdel.x;
            g[q].y += cdel.y;
        }
    }
}

// h^3 G(0) / Identity: the sphere-averaged self-term
__host__ inline z128 self_term(double h, const GreenParams& P) {
    const double R = std::cbrt(3.0 / (4.0 * kPi)) * h;
    const z128 ip = tau_moment(P.w / P.alpha, 0.0, R);
    const z128 is = tau_moment(P.w / P.beta, 0.0, R);
    const double cp = 1.0 / (3.0 * P.alpha * P.alpha * P.rho), cs = 2.0 / (3.0 * P.beta * P.beta * P.rho);
    return {cp * ip.x + cs * is.x, cp * ip.y + cs * is.y};
}

// Padded real-space table of one component: T(m) = h^3 G(m h) at m mod L, m in [-(N-1), N-1],
// self-term at m = 0, zero in the gap between N - 1 and L - (N - 1).
__global__ void k_sample_table(z128* __restrict__ buf, int comp, int L1, int L2, int L3, int N1, int N2, int N3,
                               double h, GreenParams P, z128 self) {
    const long long total = (long long)L1 * L2 * L3;
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int x = (int)(q % L1), y = (int)((q / L1) % L2), z = (int)(q / ((long long)L1 * L2));
    auto offset = [](int i, int L, int N, int& m) -> bool {
        if (i <= N - 1) {
            m = i;
            return true;
        }
        if (i >= L - (N - 1)) {
            m = i - L;
            return true;
        }
        return false;
    };
    int mx, my, mz;
    z128 v = {0.0, 0.0};
    if (offset(x, L1, N1, mx) && offset(y, L2, N2, my) && offset(z, L3, N3, mz)) {
        if (mx == 0 && my == 0 && mz == 0) {
            if (comp < 3) v = self;
        } else {
            z128 g[6];
            green6(mx * h, my * h, mz * h, P, g);
            const double h3 = h * h * h;
            v = {h3 * g[comp].x, h3 * g[comp].y};
        }
    }
    buf[q] = v;
}

// copy the octant k_a <= L_a/2 of one transformed component, scaled by 1/(L1 L2 L3), into the
// component-interleaved table [L3/2+1][L2/2+1][L1/2+1][6]
__global__ void k_extract_octant(const z128* __restrict__ buf, z128* __restrict__ g, z64* __restrict__ g32, int comp,
                                 int L1, int L2, int L3, double scale) {
    const int O1 = L1 / 2 + 1, O2 = L2 / 2 + 1, O3 = L3 / 2 + 1;
    const long long total = (long long)O1 * O2 * O3;
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int x = (int)(q % O1), y = (int)((q / O1) % O2), z = (int)(q / ((long long)O1 * O2));
    const z128 v = buf[((long long)z * L2 + y) * L1 + x];
    const z128 s = {v.x * scale, v.y * scale};
    g[q * 6 + comp] = s;
    if (g32) g32[q * 6 + comp] = {(float)s.x, (float)s.y};
}

// b_i(x) = phase * sum_q [ G_ij(x - q) F_j(q)  (x != q);  self/h^3 F_i(q)  (x == q) ]
__global__ void k_rhs_points(z128* __restrict__ b, int N1, int N2, int N3, double h, GreenParams P, z128 self_over_h3,
                             const int* __restrict__ cells, const double* __restrict__ F, int npts, z128 phase) {
    const long long n = (long long)N1 * N2 * N3;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int i = (int)(p % N1), j = (int)((p / N1) % N2), k = (int)(p / ((long long)N1 * N2));
    z128 acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int t = 0; t < npts; ++t) {
        const int di = i - cells[3 * t], dj = j - cells[3 * t + 1], dk = k - cells[3 * t + 2];
        const double f0 = F[3 * t], f1 = F[3 * t + 1], f2 = F[3 * t + 2];
        if (di == 0 && dj == 0 && dk == 0) {
            acc[0] = acc[0] + f0 * self_over_h3;
            acc[1] = acc[1] + f1 * self_over_h3;
            acc[2] = acc[2] + f2 * self_over_h3;
        } else {
            z128 g[6];
            green6(di * h, dj * h, dk * h, P, g);
            // rows of the symmetric G: (11 12 13), (12 22 23), (13 23 33)
            acc[0] = acc[0] + f0 * g[0] + f1 * g[5] + f2 * g[4];
            acc[1] = acc[1] + f0 * g[5] + f1 * g[1] + f2 * g[3];
            acc[2] = acc[2] + f0 * g[4] + f1 * g[3] + f2 * g[2];
        }
    }
    b[p] = phase * acc[0];
    b[n + p] = phase * acc[1];
    b[2 * n + p] = phase * acc[2];
}

GreenParams params_of(const Ctx* c, int i) { return {c->omega[i], c->alpha, c->beta, c->rho0, c->green_mode}; }

}  // namespace

int build_green_tables(Ctx* c) {
    const int L1 = c->L1, L2 = c->L2, L3 = c->L3;
    const long long total = (long long)L1 * L2 * L3;
    const long long oct = (long long)(L1 / 2 + 1) * (L2 / 2 + 1) * (L3 / 2 + 1);
    z128* buf = nullptr;
    LS_HIP(hipMallocAsync((void**)&buf, total * sizeof(z128), c->stream));
    int rc = LS_OK;
    for (size_t i = 0; i < c->omega.size() && rc == LS_OK; ++i) {
        const GreenParams P = params_of(c, (int)i);
        const z128 self = self_term(c->h, P);
        for (int comp = 0; comp < 6 && rc == LS_OK; ++comp) {
            hipLaunchKernelGGL(k_sample_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream, buf,
                               comp, L1, L2, L3, c->n1, c->n2, c->n3, c->h, P, self);
            if (hipGetLastError() != hipSuccess) {
                rc = fail(LS_ERR_HIP, "table sampling launch failed");
                break;
            }
            rc = fft_full_3d_forward<double>(c, buf);
            if (rc) break;
            hipLaunchKernelGGL(k_extract_octant, dim3((unsigned)((oct + 255) / 256)), dim3(256), 0, c->stream, buf,
                               c->ghat[i], c->mixed ? c->ghat32[i] : nullptr, comp, L1, L2, L3,
                               1.0 / (double)total);
            if (hipGetLastError() != hipSuccess) rc = fail(LS_ERR_HIP, "octant extraction launch failed");
        }
    }
    hipError_t e1 = hipStreamSynchronize(c->stream);
    hipError_t e2 = hipFreeAsync(buf, c->stream);
    hipError_t e3 = hipStreamSynchronize(c->stream);
    if (rc) return rc;
    if (e1 != hipSuccess) return hip_fail(e1, "table build");
    if (e2 != hipSuccess) return hip_fail(e2, "table scratch free");
    if (e3 != hipSuccess) return hip_fail(e3, "table build sync");
    return LS_OK;
}

// cells: host int[3 npts], forces: host double[3 npts] (already h^3 times the force density)
int rhs_points_launch(Ctx* c, int i_omega, const int* cells, const double* forces, int npts, double t0, z128* b) {
    if (npts > 16) return fail(LS_ERR_ARG, "too many source points");
    // small host arrays are passed through the context's device staging area
    int* dcells = (int*)c->stage;
    double* dF = (double*)((char*)c->stage + 1024);
    LS_HIP(hipMemcpyAsync(dcells, cells, sizeof(int) * 3 * npts, hipMemcpyHostToDevice, c->stream));
    LS_HIP(hipMemcpyAsync(dF, forces, sizeof(double) * 3 * npts, hipMemcpyHostToDevice, c->stream));
    const GreenParams P = params_of(c, i_omega);
    const z128 self = self_term(c->h, P);
    const double h3 = c->h * c->h * c->h;
    const z128 self_h3 = {self.x / h3, self.y / h3};
    const double ph = c->omega[i_omega] * t0;
    const z128 phase = {std::cos(ph), std::sin(ph)};
    const long long n = c->ncell;
    c->prof.begin(c->stream, "rhs_points");
    hipLaunchKernelGGL(k_rhs_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, b, c->n1, c->n2, c->n3,
                       c->h, P, self_h3, dcells, dF, npts, phase);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    // the staging area is reused by the next call: wait for the copies to be consumed
    LS_HIP(hipStreamSynchronize(c->stream));
    return LS_OK;
}

}  // namespace ls
