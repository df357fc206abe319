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
#include <algorithm>
#include <cmath>
#include <vector>

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
// greal (LS_GREEN_ANISO): the octant table h^3 G, read with the mirror signs, or (half) the half-space
// table, read at -m for m_x < 0; else the closed form.
__global__ void k_rhs_points(z128* __restrict__ b, int N1, int N2, int N3, double h, GreenParams P, z128 self_over_h3,
                             const int* __restrict__ cells, const double* __restrict__ F, int npts, z128 phase,
                             const z128* __restrict__ greal, int half) {
    const long long n = (long long)N1 * N2 * N3;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int i = (int)(p % N1), j = (int)((p / N1) % N2), k = (int)(p / ((long long)N1 * N2));
    z128 acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int t = 0; t < npts; ++t) {
        const int di = i - cells[3 * t], dj = j - cells[3 * t + 1], dk = k - cells[3 * t + 2];
        const double f0 = F[3 * t], f1 = F[3 * t + 1], f2 = F[3 * t + 2];
        if (greal && half) {
            const int s = di < 0 ? -1 : 1;
            const z128* e = greal + (((long long)(s * dk + N3 - 1) * (2 * N2 - 1) + (s * dj + N2 - 1)) * N1 + s * di) * 6;
            const double ih3 = 1.0 / (h * h * h);
            z128 g[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) g[q] = ih3 * e[q];
            acc[0] = acc[0] + f0 * g[0] + f1 * g[5] + f2 * g[4];
            acc[1] = acc[1] + f0 * g[5] + f1 * g[1] + f2 * g[3];
            acc[2] = acc[2] + f0 * g[4] + f1 * g[3] + f2 * g[2];
        } else if (greal) {
            const z128* e = greal + (((long long)abs(dk) * N2 + abs(dj)) * N1 + abs(di)) * 6;
            const double ih3 = 1.0 / (h * h * h);
            const double syz = ((dj < 0) != (dk < 0)) ? -ih3 : ih3;
            const double sxz = ((di < 0) != (dk < 0)) ? -ih3 : ih3;
            const double sxy = ((di < 0) != (dj < 0)) ? -ih3 : ih3;
            const z128 g0 = ih3 * e[0], g1 = ih3 * e[1], g2 = ih3 * e[2];
            const z128 g3 = syz * e[3], g4 = sxz * e[4], g5 = sxy * e[5];
            acc[0] = acc[0] + f0 * g0 + f1 * g5 + f2 * g4;
            acc[1] = acc[1] + f0 * g5 + f1 * g1 + f2 * g3;
            acc[2] = acc[2] + f0 * g4 + f1 * g3 + f2 * g2;
        } else if (di == 0 && dj == 0 && dk == 0) {
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

// ---------------------------------------------------------------------------------------------
// Anisotropic background (LS_GREEN_ANISO).
//
// With Gamma(n) the Christoffel matrix, lambda_m, P_m its eigenvalues and eigenprojectors and
// k_m = w sqrt(rho / lambda_m), the outgoing solution of Eq 7 has the plane-wave form (the inverse
// Fourier transform of (Gamma(k) - rho w^2)^{-1}, split into its w = 0 part and the rest)
//   G(x) = 1/(8 pi^2 r) int_{n.x=0} Gamma(n)^{-1} dphi
//        + i/(8 pi^2) int_{n.x>0} sum_m P_m k_m/lambda_m e^{i k_m n.x} dS(n),
// and the zero-offset cell takes the integral over the sphere of volume h^3,
//   1/(4 pi) int_{S^2} sum_m P_m I(k_m)/lambda_m dS,  I(k) = int_0^R r e^{i k r} dr.
// Every homogeneous medium gives G(-x) = G(x); a background with the three coordinate mirror planes also
// gives G_ab(s x) = s_a s_b G_ab(x).  So one octant of offsets (mirror planes) or one half-space
// (x >= 0, any stiffness) is evaluated, one thread per offset, and the padded table is filled from it.
//
// Per quadrature node the matrix function sum_m f(lambda_m) P_m is formed without eigenvectors:
// the quasi-P eigenvalue lambda_c (the largest, kept apart from the other two by a set-up check)
// comes from the trigonometric solution of the characteristic cubic, its projector from
// P_c = (Gamma^2 - s Gamma + p I) / ((lambda_c - lambda_a)(lambda_c - lambda_b)) with
// s = lambda_a + lambda_b = tr Gamma - lambda_c and p = lambda_a lambda_b = det Gamma / lambda_c, and the
// quasi-S pair, which may coincide, enters only through s, p and the divided difference
// D = (f(lambda_a) - f(lambda_b)) / (lambda_a - lambda_b) (f' at a double eigenvalue):
//   sum_m f(lambda_m) P_m = (f_c - f_m - D (lambda_c - s/2)) P_c + (f_m - D s/2) I + D Gamma,
// f_m = (f(lambda_a) + f(lambda_b)) / 2.

// Christoffel matrix as a quadratic form: component q of Gamma(n) = sum_m a[q][m] mono_m(n), the monomials
// (n1 n1, n2 n2, n3 n3, n2 n3, n1 n3, n1 n2).  Symmetric 3x3 matrices are stored as (00, 11, 22, 12, 02,
// 01), the table's component order.
struct Quad {
    double a[6][6];
};

__host__ __device__ inline void christoffel(const Quad& Q, double n1, double n2, double n3, double g[6]) {
    const double mono[6] = {n1 * n1, n2 * n2, n3 * n3, n2 * n3, n1 * n3, n1 * n2};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) v += Q.a[q][m] * mono[m];
        g[q] = v;
    }
}

__host__ __device__ inline double det_sym(const double g[6]) {
    return g[0] * (g[1] * g[2] - g[3] * g[3]) - g[5] * (g[5] * g[2] - g[3] * g[4]) + g[4] * (g[5] * g[3] - g[1] * g[4]);
}

// largest eigenvalue of a symmetric 3x3 (trigonometric solution of the characteristic cubic)
__device__ inline double largest_eigenvalue(const double g[6]) {
    const double m = (g[0] + g[1] + g[2]) * (1.0 / 3.0);
    const double k[6] = {g[0] - m, g[1] - m, g[2] - m, g[3], g[4], g[5]};
    const double p2 = (k[0] * k[0] + k[1] * k[1] + k[2] * k[2] + 2.0 * (k[3] * k[3] + k[4] * k[4] + k[5] * k[5])) *
                      (1.0 / 6.0);
    if (!(p2 > 0.0)) return m;
    const double p = sqrt(p2);
    const double r = fmin(1.0, fmax(-1.0, det_sym(k) / (2.0 * p2 * p)));
    return m + 2.0 * p * cos(acos(r) * (1.0 / 3.0));
}

// f(lambda) = (k / lambda) e^{i k ru},  k = wsr / sqrt(lambda),  wsr = w sqrt(rho)
__device__ inline z128 f_plane(double lam, double wsr, double ru) {
    const double il = 1.0 / lam;
    const double k = wsr * sqrt(il);
    double sn, cs;
    sincos(k * ru, &sn, &cs);
    const double a = k * il;
    return {a * cs, a * sn};
}

// f'(lambda) = -(k / lambda^2) (3/2 + i k ru / 2) e^{i k ru}
__device__ inline z128 f_plane_deriv(double lam, double wsr, double ru) {
    const double il = 1.0 / lam;
    const double k = wsr * sqrt(il);
    double sn, cs;
    sincos(k * ru, &sn, &cs);
    const double a = -k * il * il;
    const z128 t = {1.5 * a, 0.5 * a * k * ru};
    return t * z128{cs, sn};
}

struct AnisoParams {
    Quad m;
    double wsr;      // w sqrt(rho)
    double kmax;     // upper bound of w / v over directions and modes
    double h;
    int N1, N2, N3;
    z128 self[6];    // zero-offset entry
};

constexpr int kGlLevels = 64;   // Gauss-Legendre rules with 8 l nodes, l = 1..64
constexpr int kCircleNodes = 64;

// h^3 G at the offsets of one octant or one half-space; out [D3][D2][D1][6] with (D1, D2, D3) =
// (N1, N2, N3) for the octant (offset (i, j, k)) and (N1, 2 N2 - 1, 2 N3 - 1) for the half-space
// (offset (i, j - N2 + 1, k - N3 + 1)).  A block is a 4 x 4 x 4 cube of offsets, so the node counts
// (which grow with r) vary little within a wavefront.  gl: rule l at pairs 4 l (l - 1) .. 4 l (l + 1) - 1
// of (node, weight) on [0, 1].
template <bool HALF>
__global__ __launch_bounds__(64) void k_green_aniso(z128* __restrict__ out, AnisoParams P,
                                                    const double* __restrict__ gl) {
    const int t = threadIdx.x;
    const int D1 = P.N1, D2 = HALF ? 2 * P.N2 - 1 : P.N2, D3 = HALF ? 2 * P.N3 - 1 : P.N3;
    const int bx = (D1 + 3) / 4, by = (D2 + 3) / 4;
    const int b = blockIdx.x;
    const int i = 4 * (b % bx) + (t & 3);
    const int j = 4 * ((b / bx) % by) + ((t >> 2) & 3);
    const int k = 4 * (b / (bx * by)) + (t >> 4);
    if (i >= D1 || j >= D2 || k >= D3) return;
    z128* o = out + (((long long)k * D2 + j) * D1 + i) * 6;
    const int mx = i, my = HALF ? j - (P.N2 - 1) : j, mz = HALF ? k - (P.N3 - 1) : k;
    if (mx == 0 && my == 0 && mz == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) o[q] = P.self[q];
        return;
    }
    const double x0 = mx * P.h, x1 = my * P.h, x2 = mz * P.h;
    const double r = sqrt(x0 * x0 + x1 * x1 + x2 * x2);
    const double ir = 1.0 / r;
    const double xh[3] = {x0 * ir, x1 * ir, x2 * ir};
    // orthonormal frame (xh, e1, e2): e1 = xh x (the axis least aligned with xh), normalised
    int ax = 0;
    if (fabs(xh[1]) < fabs(xh[ax])) ax = 1;
    if (fabs(xh[2]) < fabs(xh[ax])) ax = 2;
    double e1[3] = {ax == 0 ? 0.0 : (ax == 1 ? -xh[2] : xh[1]), ax == 1 ? 0.0 : (ax == 0 ? xh[2] : -xh[0]),
                    ax == 2 ? 0.0 : (ax == 0 ? -xh[1] : xh[0])};
    const double in1 = 1.0 / sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    e1[0] *= in1;
    e1[1] *= in1;
    e1[2] *= in1;
    const double e2[3] = {xh[1] * e1[2] - xh[2] * e1[1], xh[2] * e1[0] - xh[0] * e1[2], xh[0] * e1[1] - xh[1] * e1[0]};

    // static part: the circle n . x = 0 (trapezoid)
    double gs[6] = {0, 0, 0, 0, 0, 0};
    {
        double sd, cd;
        sincospi(2.0 / kCircleNodes, &sd, &cd);
        double cp = 1.0, sp = 0.0;
        for (int q = 0; q < kCircleNodes; ++q) {
            double g[6];
            christoffel(P.m, cp * e1[0] + sp * e2[0], cp * e1[1] + sp * e2[1], cp * e1[2] + sp * e2[2], g);
            const double id = 1.0 / det_sym(g);
            gs[0] += (g[1] * g[2] - g[3] * g[3]) * id;
            gs[1] += (g[0] * g[2] - g[4] * g[4]) * id;
            gs[2] += (g[0] * g[1] - g[5] * g[5]) * id;
            gs[3] += (g[5] * g[4] - g[0] * g[3]) * id;
            gs[4] += (g[5] * g[3] - g[1] * g[4]) * id;
            gs[5] += (g[4] * g[3] - g[5] * g[2]) * id;
            const double c2 = cp * cd - sp * sd;
            sp = sp * cd + cp * sd;
            cp = c2;
        }
    }

    // regular part: the half sphere n . x > 0, u = n . xh (Gauss-Legendre) times phi (trapezoid)
    const double kr = P.kmax * r;
    int nu = (int)ceil(0.3 * kr) + 32;
    nu = min(8 * kGlLevels, (nu + 7) & ~7);
    const int lev = nu / 8;
    const double* rule = gl + 2 * (4 * lev * (lev - 1));
    const int nphi = (int)ceil(0.3 * kr) + 64;
    double sd, cd;
    sincospi(2.0 / nphi, &sd, &cd);
    z128 acc[6] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int iu = 0; iu < nu; ++iu) {
        const double u = rule[2 * iu], wu = rule[2 * iu + 1];
        const double su = sqrt(fmax(0.0, 1.0 - u * u));
        const double ru = r * u;
        const double a0 = u * xh[0], a1 = u * xh[1], a2 = u * xh[2];
        z128 ring[6] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
        double cp = 1.0, sp = 0.0;
        for (int ip = 0; ip < nphi; ++ip) {
            double g[6];
            christoffel(P.m, a0 + su * (cp * e1[0] + sp * e2[0]), a1 + su * (cp * e1[1] + sp * e2[1]),
                        a2 + su * (cp * e1[2] + sp * e2[2]), g);
            const double lc = largest_eigenvalue(g);
            const double s = g[0] + g[1] + g[2] - lc;
            const double pp = det_sym(g) / lc;
            const double iden = 1.0 / (lc * lc - s * lc + pp);
            const double g2[6] = {g[0] * g[0] + g[5] * g[5] + g[4] * g[4], g[5] * g[5] + g[1] * g[1] + g[3] * g[3],
                                  g[4] * g[4] + g[3] * g[3] + g[2] * g[2], g[5] * g[4] + g[1] * g[3] + g[3] * g[2],
                                  g[0] * g[4] + g[5] * g[3] + g[4] * g[2], g[0] * g[5] + g[5] * g[1] + g[4] * g[3]};
            const double d = sqrt(fmax(0.0, s * s - 4.0 * pp));
            const z128 fc = f_plane(lc, P.wsr, ru);
            const z128 fa = f_plane(0.5 * (s + d), P.wsr, ru);
            const z128 fb = f_plane(0.5 * (s - d), P.wsr, ru);
            const z128 fm = 0.5 * (fa + fb);
            const z128 D = d > 1e-7 * s ? (1.0 / d) * (fa - fb) : f_plane_deriv(0.5 * s, P.wsr, ru);
            const z128 aP = fc - fm - (lc - 0.5 * s) * D;
            const z128 aI = fm - (0.5 * s) * D;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const double pc = (g2[q] - s * g[q] + (q < 3 ? pp : 0.0)) * iden;
                ring[q] = ring[q] + pc * aP + g[q] * D;
                if (q < 3) ring[q] = ring[q] + aI;
            }
            const double c2 = cp * cd - sp * sd;
            sp = sp * cd + cp * sd;
            cp = c2;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) acc[q] = acc[q] + wu * ring[q];
    }
    const double h3 = P.h * P.h * P.h;
    const double cs = h3 * (2.0 * kPi / kCircleNodes) / (8.0 * kPi * kPi * r);
    const double cr = h3 * (2.0 * kPi / nphi) / (8.0 * kPi * kPi);
#pragma unroll
    for (int q = 0; q < 6; ++q) o[q] = {cs * gs[q] - cr * acc[q].y, cr * acc[q].x};   // i * acc
}

// one component of the padded real-space table: from the octant, T_ab(m) = s_a s_b greal_ab(|m|); from
// the half-space, T(m) = greal(m) for m_x >= 0 and greal(-m) otherwise
template <bool HALF>
__global__ void k_fill_aniso(z128* __restrict__ buf, const z128* __restrict__ greal, int comp, int L1, int L2, int L3,
                             int N1, int N2, int N3) {
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
        if constexpr (HALF) {
            if (mx < 0) {
                mx = -mx;
                my = -my;
                mz = -mz;
            }
            v = greal[(((long long)(mz + N3 - 1) * (2 * N2 - 1) + (my + N2 - 1)) * N1 + mx) * 6 + comp];
        } else {
            v = greal[(((long long)abs(mz) * N2 + abs(my)) * N1 + abs(mx)) * 6 + comp];
            const bool sx = mx < 0, sy = my < 0, sz = mz < 0;
            const bool neg = comp == 3 ? (sy != sz) : comp == 4 ? (sx != sz) : comp == 5 ? (sx != sy) : false;
            if (neg) v = {-v.x, -v.y};
        }
    }
    buf[q] = v;
}

// the half-space k_x <= L1/2 of one transformed component, scaled, into [L3][L2][L1/2+1][6]
__global__ void k_extract_half(const z128* __restrict__ buf, z128* __restrict__ g, z64* __restrict__ g32, int comp,
                               int L1, int L2, int L3, double scale) {
    const int O1 = L1 / 2 + 1;
    const long long total = (long long)O1 * L2 * L3;
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int x = (int)(q % O1), y = (int)((q / O1) % L2), z = (int)(q / ((long long)O1 * L2));
    const z128 v = buf[((long long)z * L2 + y) * L1 + x];
    const z128 s = {v.x * scale, v.y * scale};
    g[q * 6 + comp] = s;
    if (g32) g32[q * 6 + comp] = {(float)s.x, (float)s.y};
}

// Gauss-Legendre nodes and weights of n points on [-1, 1] (Newton's method on P_n from the
// Chebyshev-like initial guesses)
void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 30; ++it) {
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; ++m) {
                const double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 4e-16) break;
        }
        // recompute the derivative at the converged node for the weight
        double p0 = 1.0, p1 = z;
        for (int m = 2; m <= n; ++m) {
            const double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// eigenvalues (ascending) and orthonormal eigenvectors (columns of V) of a symmetric 3x3 by cyclic Jacobi
void jacobi3(const double g[6], double lam[3], double V[3][3]) {
    double A[3][3] = {{g[0], g[5], g[4]}, {g[5], g[1], g[3]}, {g[4], g[3], g[2]}};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) V[a][b] = a == b ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-34 * dia) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < 3; ++k) {   // A <- A J
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - sn * akq;
                    A[k][q] = sn * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {   // A <- J^T A
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - sn * aqk;
                    A[q][k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {   // V <- V J
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - sn * vkq;
                    V[k][q] = sn * vkp + c * vkq;
                }
            }
    }
    int idx[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (A[idx[b]][idx[b]] < A[idx[a]][idx[a]]) std::swap(idx[a], idx[b]);
    double W[3][3];
    for (int m = 0; m < 3; ++m) {
        lam[m] = A[idx[m]][idx[m]];
        for (int k = 0; k < 3; ++k) W[k][m] = V[k][idx[m]];
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) V[a][b] = W[a][b];
}

// Gamma_ik(n) = c_ijkl n_j n_l as a quadratic form in n, from the Voigt stiffness (row-major 6x6): the
// coefficient of n_j n_j is c_ijkj, that of n_j n_l (j < l) is c_ijkl + c_ilkj.
Quad quad_of(const double* C) {
    auto voigt = [](int a, int b) { return a == b ? a : 6 - a - b; };   // 00 11 22 -> 0 1 2; 12 -> 3, 02 -> 4, 01 -> 5
    auto c4 = [&](int i, int j, int k, int l) { return C[voigt(i, j) * 6 + voigt(k, l)]; };
    const int pi[6] = {0, 1, 2, 1, 0, 0}, pk[6] = {0, 1, 2, 2, 2, 1};   // component q = (i, k)
    const int mj[6] = {0, 1, 2, 1, 0, 0}, ml[6] = {0, 1, 2, 2, 2, 1};   // monomial m = n_j n_l
    Quad Q;
    for (int q = 0; q < 6; ++q)
        for (int m = 0; m < 6; ++m) {
            const int i = pi[q], k = pk[q], j = mj[m], l = ml[m];
            Q.a[q][m] = j == l ? c4(i, j, k, j) : c4(i, j, k, l) + c4(i, l, k, j);
        }
    return Q;
}

// Set-up quantities of the anisotropic table from a sampling of the sphere (GL 48 in cos(theta),
// 96 azimuths): the smallest eigenvalue (kmax = 1.1 w sqrt(rho / lambda_min)), the quasi-P gap check,
// and the zero-offset entry 1/(4 pi) int sum_m P_m I(k_m) / lambda_m dS for each frequency.
int aniso_setup(const Ctx* c, double w, double* kmax, z128 self[6]) {
    const Quad m = quad_of(c->C0);
    constexpr int NT = 48, NP = 96;
    double tx[NT], tw[NT];
    gauss_legendre(NT, tx, tw);
    const double R = std::cbrt(3.0 / (4.0 * kPi)) * c->h;
    double lmin = 1e300, worst_gap = 1e300;
    double S[6][2] = {{0}};
    for (int a = 0; a < NT; ++a)
        for (int b = 0; b < NP; ++b) {
            const double st = std::sqrt(std::max(0.0, 1.0 - tx[a] * tx[a]));
            const double ph = 2.0 * kPi * b / NP;
            double g[6], lam[3], V[3][3];
            christoffel(m, st * std::cos(ph), st * std::sin(ph), tx[a], g);
            jacobi3(g, lam, V);
            lmin = std::min(lmin, lam[0]);
            worst_gap = std::min(worst_gap, (lam[2] - lam[1]) / lam[2]);
            const double wt = tw[a] * (2.0 * kPi / NP) / (4.0 * kPi);
            for (int mo = 0; mo < 3; ++mo) {
                if (!(lam[mo] > 0)) continue;
                const z128 I = tau_moment(w * std::sqrt(c->rho0 / lam[mo]), 0.0, R);
                const double f = wt / lam[mo];
                const int pa[6] = {0, 1, 2, 1, 0, 0}, pb[6] = {0, 1, 2, 2, 2, 1};
                for (int q = 0; q < 6; ++q) {
                    const double pq = V[pa[q]][mo] * V[pb[q]][mo] * f;
                    S[q][0] += pq * I.x;
                    S[q][1] += pq * I.y;
                }
            }
        }
    if (!(lmin > 0)) return fail(LS_ERR_ARG, "LS_GREEN_ANISO: the background stiffness is not positive definite");
    if (!(worst_gap >= 0.05))
        return fail(LS_ERR_ARG, "LS_GREEN_ANISO: the quasi-P eigenvalue comes within 5 % of a quasi-S one");
    *kmax = 1.1 * w * std::sqrt(c->rho0 / lmin);
    const double rmax = c->h * std::sqrt((double)(c->n1 - 1) * (c->n1 - 1) + (double)(c->n2 - 1) * (c->n2 - 1) +
                                         (double)(c->n3 - 1) * (c->n3 - 1));
    if (*kmax * rmax > 1600.0)
        return fail(LS_ERR_ARG, "LS_GREEN_ANISO: the grid spans more than 1600 rad of phase (too many wavelengths)");
    for (int q = 0; q < 6; ++q) self[q] = {S[q][0], S[q][1]};
    return LS_OK;
}

// Gauss-Legendre rules of 8 l points on [0, 1], l = 1..kGlLevels, as (node, weight) pairs
std::vector<double> gl_levels() {
    std::vector<double> out;
    for (int l = 1; l <= kGlLevels; ++l) {
        const int n = 8 * l;
        std::vector<double> x(n), w(n);
        gauss_legendre(n, x.data(), w.data());
        for (int i = 0; i < n; ++i) {
            out.push_back(0.5 * (x[i] + 1.0));
            out.push_back(0.5 * w[i]);
        }
    }
    return out;
}

int build_aniso_real(Ctx* c, int i) {
    if (!c->gl_nodes) {
        const std::vector<double> gl = gl_levels();
        int rc = dalloc(c, (void**)&c->gl_nodes, gl.size() * sizeof(double));
        if (rc) return rc;
        LS_HIP(hipMemcpy(c->gl_nodes, gl.data(), gl.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    AnisoParams P;
    P.m = quad_of(c->C0);
    P.wsr = c->omega[i] * std::sqrt(c->rho0);
    P.h = c->h;
    P.N1 = c->n1;
    P.N2 = c->n2;
    P.N3 = c->n3;
    int rc = aniso_setup(c, c->omega[i], &P.kmax, P.self);
    if (rc) return rc;
    const int D2 = c->green_half ? 2 * c->n2 - 1 : c->n2, D3 = c->green_half ? 2 * c->n3 - 1 : c->n3;
    const long long blocks = (long long)((c->n1 + 3) / 4) * ((D2 + 3) / 4) * ((D3 + 3) / 4);
    if (c->green_half)
        hipLaunchKernelGGL(k_green_aniso<true>, dim3((unsigned)blocks), dim3(64), 0, c->stream, c->greal[i], P,
                           c->gl_nodes);
    else
        hipLaunchKernelGGL(k_green_aniso<false>, dim3((unsigned)blocks), dim3(64), 0, c->stream, c->greal[i], P,
                           c->gl_nodes);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

GreenParams params_of(const Ctx* c, int i) { return {c->omega[i], c->alpha, c->beta, c->rho0, c->green_mode}; }

}  // namespace

int build_green_tables(Ctx* c) {
    const int L1 = c->L1, L2 = c->L2, L3 = c->L3;
    const long long total = (long long)L1 * L2 * L3;
    const long long oct = (long long)(L1 / 2 + 1) * (L2 / 2 + 1) * (L3 / 2 + 1);
    const long long half = (long long)(L1 / 2 + 1) * L2 * L3;
    z128* buf = nullptr;
    LS_HIP(hipMallocAsync((void**)&buf, total * sizeof(z128), c->stream));
    int rc = LS_OK;
    const bool aniso = c->green_mode == LS_GREEN_ANISO;
    for (size_t i = 0; i < c->omega.size() && rc == LS_OK; ++i) {
        const GreenParams P = params_of(c, (int)i);
        const z128 self = aniso ? z128{0.0, 0.0} : self_term(c->h, P);
        if (aniso && (rc = build_aniso_real(c, (int)i))) break;
        for (int comp = 0; comp < 6 && rc == LS_OK; ++comp) {
            if (aniso && c->green_half)
                hipLaunchKernelGGL(k_fill_aniso<true>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream,
                                   buf, (const z128*)c->greal[i], comp, L1, L2, L3, c->n1, c->n2, c->n3);
            else if (aniso)
                hipLaunchKernelGGL(k_fill_aniso<false>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream,
                                   buf, (const z128*)c->greal[i], comp, L1, L2, L3, c->n1, c->n2, c->n3);
            else
                hipLaunchKernelGGL(k_sample_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream,
                                   buf, comp, L1, L2, L3, c->n1, c->n2, c->n3, c->h, P, self);
            if (hipGetLastError() != hipSuccess) {
                rc = fail(LS_ERR_HIP, "table sampling launch failed");
                break;
            }
            rc = fft_full_3d_forward<double>(c, buf);
            if (rc) break;
            if (c->green_half)
                hipLaunchKernelGGL(k_extract_half, dim3((unsigned)((half + 255) / 256)), dim3(256), 0, c->stream, buf,
                                   c->ghat[i], c->mixed ? c->ghat32[i] : nullptr, comp, L1, L2, L3,
                                   1.0 / (double)total);
            else
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

namespace {

// h^3 G at the offsets m in [-2, 2]^3, entry ((mz + 2) 5 + my + 2) 5 + mx + 2, six components (11, 22, 33, 23,
// 13, 12): the closed form with the self term at m = 0, or the sampled LS_GREEN_ANISO table (octant with
// mirror signs, or half-space read at -m for m_x < 0).  Offsets that do not fit in the grid are left zero.
__global__ void k_local_table(z128* __restrict__ out, int N1, int N2, int N3, double h, GreenParams P, z128 self,
                              const z128* __restrict__ greal, int half) {
    const int t = threadIdx.x;
    if (t >= 125) return;
    const int mx = t % 5 - 2, my = (t / 5) % 5 - 2, mz = t / 25 - 2;
    z128 g[6] = {};
    if (abs(mx) < N1 && abs(my) < N2 && abs(mz) < N3) {
        if (greal && half) {
            const int s = mx < 0 ? -1 : 1;
            const z128* e = greal + (((long long)(s * mz + N3 - 1) * (2 * N2 - 1) + (s * my + N2 - 1)) * N1 + s * mx) * 6;
            for (int q = 0; q < 6; ++q) g[q] = e[q];
        } else if (greal) {
            const z128* e = greal + (((long long)abs(mz) * N2 + abs(my)) * N1 + abs(mx)) * 6;
            const double sg[6] = {1.0, 1.0, 1.0, ((my < 0) != (mz < 0)) ? -1.0 : 1.0,
                                  ((mx < 0) != (mz < 0)) ? -1.0 : 1.0, ((mx < 0) != (my < 0)) ? -1.0 : 1.0};
            for (int q = 0; q < 6; ++q) g[q] = sg[q] * e[q];
        } else if (mx == 0 && my == 0 && mz == 0) {
            g[0] = g[1] = g[2] = self;
        } else {
            green6(mx * h, my * h, mz * h, P, g);
            const double h3 = h * h * h;
            for (int q = 0; q < 6; ++q) g[q] = h3 * g[q];
        }
    }
    for (int q = 0; q < 6; ++q) out[t * 6 + q] = g[q];
}

}  // namespace

int local_green_table(Ctx* c, int i_omega, z128* out) {
    const GreenParams P = params_of(c, i_omega);
    const bool aniso = c->green_mode == LS_GREEN_ANISO;
    const z128 self = aniso ? z128{0.0, 0.0} : self_term(c->h, P);
    hipLaunchKernelGGL(k_local_table, dim3(1), dim3(128), 0, c->stream, out, c->n1, c->n2, c->n3, c->h, P, self,
                       aniso ? (const z128*)c->greal[i_omega] : nullptr, c->green_half ? 1 : 0);
    LS_HIP(hipGetLastError());
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
                       c->h, P, self_h3, dcells, dF, npts, phase,
                       c->green_mode == LS_GREEN_ANISO ? (const z128*)c->greal[i_omega] : nullptr,
                       c->green_half ? 1 : 0);
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    // the staging area is reused by the next call: wait for the copies to be consumed
    LS_HIP(hipStreamSynchronize(c->stream));
    return LS_OK;
}

}  // namespace ls
