// Zero-padded 3-D FFT passes of the matrix-free LS operator (Eq 21) and the k-space Green's
// tensor multiply.
//
// Work buffer layout (per right-hand side r, component c): W[r][c][z < N3][y < L2][x < L1].
// The convolution of a force density f (supported on the N1 x N2 x N3 cells) with the Green's
// table is linear (not periodic) because every FFT length L_a >= 2 N_a - 1.  The passes prune
// the zeros: the forward x pass reads N1 inputs per line and runs only on the N2 x N3 lines
// that carry data; the forward y pass reads N2 inputs; the fused z pass reads N3 inputs, runs
// the forward z FFT, multiplies by the 3x3 symmetric table G^(k), runs the inverse z FFT and
// keeps N3 outputs; the inverse y pass keeps N2 outputs and the inverse x pass keeps N1 outputs
// and writes Au = u - v (or v) into the compact caller array.  Every pass except the last is
// in place, so W holds 3 N3 L2 L1 complex values per right-hand side.
#include <cstdlib>
#include <cstring>

#include "fft_reg.h"

namespace ls {

namespace {

constexpr int kThreads = 256;

// Lines per block of the contiguous (x) pass: about 32 KB of LDS.
template <typename T, int L>
constexpr int contig_lines() {
    constexpr int elems = 32768 / (int)sizeof(cpx<T>);
    return elems / L > 1 ? elems / L : 1;
}
// Adjacent columns per block of the strided (y, z) passes: 128-byte row segments.
template <typename T>
constexpr int strided_cols() {
    return 128 / (int)sizeof(cpx<T>);
}
// Adjacent columns per block of the fused z pass (three components resident in LDS).
template <typename T, int L>
constexpr int zpass_cols() {
    constexpr int budget = 49152;  // bytes of LDS
    constexpr int tx = budget / (3 * L * (int)sizeof(cpx<T>));
    return tx >= 8 ? 8 : (tx >= 4 ? 4 : (tx >= 2 ? 2 : 1));
}

// Row of the compact field [.. component ..][z][y] that x line `line` of the padded work buffer holds:
// with z blocks of 2^zbs planes (zplane_offset) the lines of a block run (y, z mod B) with z fastest,
// D2 = N2 B lines per block; zbs = 0 is the identity.
__device__ __forceinline__ long long compact_row(long long line, int D2, int zbs) {
    if (zbs == 0) return line;
    const long long g = line / D2, rem = line - g * D2;
    return g * D2 + (rem & ((1 << zbs) - 1)) * (D2 >> zbs) + (rem >> zbs);
}

// k-space Green's table of each launch position (z passes), by value
template <typename T>
struct GreenTabs {
    const cpx<T>* g[kMaxRhs];
};

// Row of the compact field arrays (indexed by slot) that x line `line` of the work buffer (indexed by
// position) ends in: lines run over positions in blocks of lpr = 3 N3 N2 lines (a multiple of D2).  rr is
// the line's position; line counts stay below 2^31 (at most 3 x 64 x 256 x 256 lines).
__device__ __forceinline__ long long slot_row(long long line, long long lpr, unsigned rr, const SlotMap& sm, int D2,
                                              int zbs) {
    return (long long)sm.slot[rr] * lpr + compact_row(line - (long long)rr * lpr, D2, zbs);
}
// position of a line: block-uniform (scalar) when every block of TY lines lies in one position
template <int TY>
__device__ __forceinline__ unsigned line_position(long long line, long long lpr) {
    if (lpr % TY == 0) return (unsigned)(((unsigned)blockIdx.x * (unsigned)TY) / (unsigned)lpr);
    return (unsigned)line / (unsigned)lpr;
}

// MODE 0: in place into data; 1: out = u - v (compact, slot rows); 2: out = v (compact, slot rows)
template <typename T, int L, int TY, int SIGN, int MODE>
__global__ __launch_bounds__(kThreads) void k_fft_contig(cpx<T>* __restrict__ data, long long nlines, int D2,
                                                         long long S1, long long S2, int n_in, int n_out,
                                                         const cpx<T>* __restrict__ tw,
                                                         const cpx<T>* __restrict__ u, cpx<T>* __restrict__ out,
                                                         int zbs, SlotMap sm, long long lpr) {
    constexpr int LDP = TY + 1;
    __shared__ cpx<T> s[L * LDP];
    const int tid = threadIdx.x;
    const long long line0 = (long long)blockIdx.x * TY;
    for (int idx = tid; idx < L * TY; idx += kThreads) {
        const int e = idx % L, ln = idx / L;
        const long long line = line0 + ln;
        cpx<T> val = {T(0), T(0)};
        if (line < nlines && e < n_in) {
            const long long o1 = line / D2, o2 = line - o1 * D2;
            val = data[o1 * S1 + o2 * S2 + e];
        }
        s[e * LDP + ln] = val;
    }
    __syncthreads();
    lds_fft<T, L, TY, LDP, kThreads, SIGN>(s, tw, tid);
    for (int idx = tid; idx < L * TY; idx += kThreads) {
        const int e = idx % L, ln = idx / L;
        const long long line = line0 + ln;
        if (line < nlines && e < n_out) {
            const cpx<T> v = s[e * LDP + ln];
            if constexpr (MODE == 0) {
                const long long o1 = line / D2, o2 = line - o1 * D2;
                data[o1 * S1 + o2 * S2 + e] = v;
            } else {
                const long long q = slot_row(line, lpr, line_position<TY>(line, lpr), sm, D2, zbs) * n_out + e;
                if constexpr (MODE == 1)
                    out[q] = u[q] - v;
                else
                    out[q] = v;
            }
        }
    }
}

template <typename T, int L, int TX, int SIGN>
__global__ __launch_bounds__(kThreads) void k_fft_strided(cpx<T>* __restrict__ data, long long S1, long long S2,
                                                          long long ES, int n_in, int n_out,
                                                          const cpx<T>* __restrict__ tw) {
    __shared__ cpx<T> s[L * TX];
    const int tid = threadIdx.x;
    cpx<T>* base = data + (long long)blockIdx.z * S1 + (long long)blockIdx.y * S2 + (long long)blockIdx.x * TX;
    for (int idx = tid; idx < L * TX; idx += kThreads) {
        const int t = idx % TX, e = idx / TX;
        cpx<T> val = {T(0), T(0)};
        if (e < n_in) val = base[e * ES + t];
        s[e * TX + t] = val;
    }
    __syncthreads();
    lds_fft<T, L, TX, TX, kThreads, SIGN>(s, tw, tid);
    for (int idx = tid; idx < L * TX; idx += kThreads) {
        const int t = idx % TX, e = idx / TX;
        if (e < n_out) base[e * ES + t] = s[e * TX + t];
    }
}

// Visit y and its mirror L2 - y in consecutive blocks so both read the same octant rows of G^: a
// permutation of 0..L2-1 for any count (an even count ends on its self-mirrored middle row L2/2).
__device__ __forceinline__ int paired_row(int by, int L2) {
    if (by == 0) return 0;
    if (L2 % 2 == 0 && by == L2 - 1) return L2 / 2;
    const int m = (by + 1) >> 1;
    return (by & 1) ? m : L2 - m;
}

// the six table entries of one k-point: 48 (c64) or 96 (c128) contiguous bytes, read as 16-byte vectors
__device__ __forceinline__ void load_g6(const z64* __restrict__ ghat, long long idx, z64 g[6]) {
    const float4* p = reinterpret_cast<const float4*>(ghat + idx * 6);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float4 a = p[k];
        g[2 * k] = {a.x, a.y};
        g[2 * k + 1] = {a.z, a.w};
    }
}
__device__ __forceinline__ void load_g6(const z128* __restrict__ ghat, long long idx, z128 g[6]) {
    const double2* p = reinterpret_cast<const double2*>(ghat + idx * 6);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double2 a = p[k];
        g[k] = {a.x, a.y};
    }
}

// Fused z pass: forward z FFT of the three components, v^ = G^(k) f^, inverse z FFT.
// G^ holds the octant [L3/2+1][L2/2+1][L1/2+1][6] (Voigt order 11,22,33,23,13,12); under
// k_a -> L_a - k_a an off-diagonal component ij changes sign once for each of i, j equal to a.
// HALF: G^ holds the half-space [L3][L2][L1/2+1][6] (backgrounds without the mirror planes) and
// k_x > L1/2 reads the entry at -k (G^ is even), with no sign change.
template <typename T, int L, int TX, bool HALF = false, int ZBS = 0>
__global__ __launch_bounds__(kThreads) void k_fft_zgreen(cpx<T>* __restrict__ data, int nrhs, int L1, int L2,
                                                         long long CS, long long RS, long long ES, int n3,
                                                         GreenTabs<T> gt, const cpx<T>* __restrict__ tw) {
    constexpr int zbs = ZBS;   // work buffer layout (zplane_offset), fixed at compile time
    constexpr int NL = 3 * TX;
    __shared__ cpx<T> s[L * NL];
    const int tid = threadIdx.x;
    const int rhs = blockIdx.x % nrhs;
    const int x0 = (blockIdx.x / nrhs) * TX;
    const int y = paired_row(blockIdx.y, L2);
    const cpx<T>* __restrict__ ghat = gt.g[rhs];
    (void)ES;   // the plane pitch: element offsets follow zplane_offset
    cpx<T>* base = data + (long long)rhs * RS + zrow_offset(y, zbs, L1) + x0;
    for (int idx = tid; idx < L * NL; idx += kThreads) {
        const int t = idx % TX, c = (idx / TX) % 3, e = idx / NL;
        cpx<T> val = {T(0), T(0)};
        if (e < n3) val = base[c * CS + zplane_offset(e, zbs, L2, L1) + t];
        s[e * NL + c * TX + t] = val;
    }
    __syncthreads();
    lds_fft<T, L, NL, NL, kThreads, -1>(s, tw, tid);

    const int O1 = L1 / 2 + 1, O2 = L2 / 2 + 1, O3 = L / 2 + 1;
    (void)O3;
    const bool fy = y > L2 / 2;
    const int ky = fy ? L2 - y : y;
    for (int idx = tid; idx < L * TX; idx += kThreads) {
        const int t = idx % TX, kz0 = idx / TX;
        const int kx0 = x0 + t;
        cpx<T> g[6];
        if constexpr (HALF) {
            const bool neg = kx0 > L1 / 2;
            const int hx = neg ? L1 - kx0 : kx0, hy = neg ? (L2 - y) % L2 : y, hz = neg ? (L - kz0) % L : kz0;
            load_g6(ghat, ((long long)hz * L2 + hy) * O1 + hx, g);
        } else {
            const bool fx = kx0 > L1 / 2, fz = kz0 > L / 2;
            const int kx = fx ? L1 - kx0 : kx0, kz = fz ? L - kz0 : kz0;
            load_g6(ghat, ((long long)kz * O2 + ky) * O1 + kx, g);
            if (fy != fz) g[3] = T(-1) * g[3];
            if (fx != fz) g[4] = T(-1) * g[4];
            if (fx != fy) g[5] = T(-1) * g[5];
        }
        const cpx<T> g11 = g[0], g22 = g[1], g33 = g[2], g23 = g[3], g13 = g[4], g12 = g[5];
        cpx<T>* row = s + kz0 * NL + t;
        const cpx<T> f1 = row[0], f2 = row[TX], f3 = row[2 * TX];
        row[0] = g11 * f1 + g12 * f2 + g13 * f3;
        row[TX] = g12 * f1 + g22 * f2 + g23 * f3;
        row[2 * TX] = g13 * f1 + g23 * f2 + g33 * f3;
    }
    __syncthreads();
    lds_fft<T, L, NL, NL, kThreads, +1>(s, tw, tid);
    for (int idx = tid; idx < L * NL; idx += kThreads) {
        const int t = idx % TX, c = (idx / TX) % 3, e = idx / NL;
        if (e < n3) base[c * CS + zplane_offset(e, zbs, L2, L1) + t] = s[e * NL + c * TX + t];
    }
}

// ------------------------------------------------------------------------------------------
// Register four-step passes (fft_reg.h).  Each thread keeps its N2 elements of a line in registers;
// one LDS transpose per direction replaces the Stockham stages, and a block covers 128 bytes of
// adjacent columns (strided passes) or lines (contiguous passes).

template <typename T>
constexpr int seg_cols() {
    return 128 / (int)sizeof(cpx<T>);
}

// usable for powers of two whose transpose buffer stays within 64 KB (all but c128 at 512); the lengths
// with a factor 3 have register kernels of their own (k_fs_strided3, k_fs_contig3, k_fs_zgreen3 and the
// paired forms at 384)
template <typename T, int L>
constexpr bool fs_ok() {
    return (L & (L - 1)) == 0 && L * seg_cols<T>() * (int)sizeof(cpx<T>) <= 65536;
}

template <typename T, int L>
constexpr int fs_threads() {
    return seg_cols<T>() * FourStep<L>::N1;
}

// Twiddles e^{-2 pi i m / L} copied to LDS once per block (cheaper than per-use global loads).
template <typename T, int L>
__device__ __forceinline__ void stage_twiddles(cpx<T>* tws, const cpx<T>* __restrict__ tw, int tid, int nthreads) {
    for (int m = tid; m < L; m += nthreads) tws[m] = tw[m];
}

// Non-temporal access (load_nt, store_nt) is used where it measured faster at 128^3, 6 right-hand
// sides: the y forward, z and x-inverse passes and the loads of the y inverse (c64 apply 2.43 -> 2.31
// ms); the x forward and the y-inverse stores measured no faster or slower with it.

// Natural-layout element j of a line is zero by construction (PRUNE: the data occupy the first
// half, n < L/2, which always holds for the zero-padded convolution) or beyond n_in.
template <int L, bool PRUNE>
__device__ __forceinline__ constexpr bool half_slot(int j) {
    return PRUNE && j >= FourStep<L>::N2 / 2;
}

// Strided pass.  Forward: natural input (n_in values), all L outputs.  Inverse: all L inputs,
// natural output (n_out values).  In place: a block reads its columns before any write.
template <typename T, int L, int TX, int SIGN, bool PRUNE>
__global__ __launch_bounds__(TX * FourStep<L>::N1) void k_fs_strided(cpx<T>* __restrict__ data, long long S1,
                                                                     long long S2, long long ES, int n_in, int n_out,
                                                                     const cpx<T>* __restrict__ tw) {
    using F = FourStep<L>;
    __shared__ cpx<T> lds[L * TX];
    __shared__ cpx<T> tws[L];
    const int tid = threadIdx.x, t = tid % TX, q = tid / TX;
    stage_twiddles<T, L>(tws, tw, tid, TX * F::N1);
    cpx<T>* base = data + (long long)blockIdx.z * S1 + (long long)blockIdx.y * S2 + (long long)blockIdx.x * TX + t;
    cpx<T> v[F::N2];
    if constexpr (SIGN < 0) {
#pragma unroll
        for (int j = 0; j < F::N2; ++j) {
            const int e = q + F::N1 * j;
            v[j] = (!half_slot<L, PRUNE>(j) && e < n_in) ? load_nt(&base[e * ES]) : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        fs_forward<T, L, TX, SIGN>(v, lds, tws, t, q);
#pragma unroll
        for (int i = 0; i < F::N2; ++i) {
            const int k = spectral_index<L>(q, i);
            if (k < n_out) store_nt(&base[k * ES], v[i]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < F::N2; ++i) {
            const int k = spectral_index<L>(q, i);
            v[i] = k < n_in ? load_nt(&base[k * ES]) : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        fs_backward<T, L, TX, SIGN>(v, lds, tws, t, q);
#pragma unroll
        for (int j = 0; j < F::N2; ++j) {
            const int e = q + F::N1 * j;
            if (!half_slot<L, PRUNE>(j) && e < n_out) base[e * ES] = v[j];
        }
    }
}

// Strided pass at the lengths with a factor 3: the asymmetric four-step of k_fs_zgreen3 (L = A x 16, A = 3, 6,
// 12, 16 threads per column) for one component, without the Green multiply.  Forward: natural input (threads
// q < A hold elements q + A j), outputs X[q + 16 k1] in slot k1; inverse: the reverse, natural outputs.
// Threads q >= A transform zeros or a copy of row A - 1 and write nothing (no divergent merge).
template <typename T, int L, int TX, int SIGN, bool PRUNE>
__global__ __launch_bounds__(TX * 16) void k_fs_strided3(cpx<T>* __restrict__ data, long long S1, long long S2,
                                                          long long ES, int n_in, int n_out,
                                                          const cpx<T>* __restrict__ tw) {
    constexpr int B = 16, A = L / B;
    static_assert(A * B == L && (A == 3 || A == 6 || A == 12), "lengths 48, 96, 192");
    __shared__ cpx<T> lds[L * TX];
    __shared__ cpx<T> tws[L];
    const int tid = threadIdx.x, t = tid % TX, q = tid / TX;
    stage_twiddles<T, L>(tws, tw, tid, TX * B);
    cpx<T>* base = data + (long long)blockIdx.z * S1 + (long long)blockIdx.y * S2 + (long long)blockIdx.x * TX + t;
    const bool s1 = q < A;
    const int qa = s1 ? q : A - 1;
    cpx<T> v[B];
    if constexpr (SIGN < 0) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int e = q + A * j;
            v[j] = (s1 && !(PRUNE && j >= B / 2) && e < n_in) ? load_nt(&base[e * ES]) : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        reg_dft<SIGN, B, T, PRUNE>(v);
#pragma unroll
        for (int k2 = 1; k2 < B; ++k2) v[k2] = v[k2] * tw_at<SIGN>(tws, qa * k2);
        if (s1) {
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) lds[(k2 * A + q) * TX + t] = v[k2];
        }
        __syncthreads();
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) v[n1] = lds[(q * A + n1) * TX + t];
        reg_dft3<SIGN, A, T>(v);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            const int k = q + B * k1;
            if (k < n_out) store_nt(&base[k * ES], v[k1]);
        }
    } else {
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            const int k = q + B * k1;
            v[k1] = k < n_in ? load_nt(&base[k * ES]) : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        reg_dft3<SIGN, A, T>(v);
#pragma unroll
        for (int n1 = 1; n1 < A; ++n1) v[n1] = v[n1] * tw_at<SIGN>(tws, n1 * q);
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) lds[(n1 * B + q) * TX + t] = v[n1];
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) v[k2] = lds[(qa * B + k2) * TX + t];
        reg_dft<SIGN, B, T>(v);
        if (s1) {
#pragma unroll
            for (int j = 0; j < B; ++j) {
                const int e = q + A * j;
                if (!(PRUNE && j >= B / 2) && e < n_out) base[e * ES] = v[j];
            }
        }
    }
}

// Strided pass at length 384 = 24 x 16: the paired asymmetric four-step of k_fs_zgreen3p for one component.
// Forward: thread p = 2 k2 + h ends with X[k2 + 16 (i + 12 h)] in slot i; inverse: the reverse.
template <typename T, int TX, int SIGN, bool PRUNE>
__global__ __launch_bounds__(TX * 32) void k_fs_strided3p(cpx<T>* __restrict__ data, long long S1, long long S2,
                                                           long long ES, int n_in, int n_out,
                                                           const cpx<T>* __restrict__ tw) {
    constexpr int L = 384, B = 16, A = 24, H = 12;
    static_assert(2 * TX <= 64, "partner lanes share a wavefront");
    __shared__ cpx<T> lds[L * TX];
    __shared__ cpx<T> tws[L];
    const int tid = threadIdx.x, t = tid % TX, q = tid / TX;
    stage_twiddles<T, L>(tws, tw, tid, TX * 32);
    cpx<T>* base = data + (long long)blockIdx.z * S1 + (long long)blockIdx.y * S2 + (long long)blockIdx.x * TX + t;
    const bool s1 = q < A;
    const int qa = s1 ? q : A - 1;
    const int k2 = q >> 1;
    const bool h = q & 1;
    cpx<T> v[B];
    if constexpr (SIGN < 0) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int e = q + A * j;
            v[j] = (s1 && !(PRUNE && j >= B / 2) && e < n_in) ? load_nt(&base[e * ES]) : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        reg_dft<SIGN, B, T, PRUNE>(v);
#pragma unroll
        for (int kk = 1; kk < B; ++kk) v[kk] = v[kk] * tw_at<SIGN>(tws, qa * kk);
        if (s1) {
#pragma unroll
            for (int kk = 0; kk < B; ++kk) lds[(kk * A + q) * TX + t] = v[kk];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < H; ++m) v[m] = lds[(k2 * A + 2 * m + (int)h) * TX + t];
        reg_dft3<SIGN, H, T>(v);
#pragma unroll
        for (int i = 0; i < H; ++i) {
            cpx<T> mine = v[i];
            if (i > 0) mine = sel(h, mine * tw_at<SIGN>(tws, i * B), mine);
            const cpx<T> other = lane_xor<TX>(mine);
            const cpx<T> x = sel(h, other - mine, mine + other);
            const int k = k2 + B * (i + H * (int)h);
            if (k < n_out) store_nt(&base[k * ES], x);
        }
    } else {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const int k = k2 + B * (i + H * (int)h);
            v[i] = k < n_in ? load_nt(&base[k * ES]) : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const cpx<T> mine = v[i];
            const cpx<T> other = lane_xor<TX>(mine);
            const cpx<T> d = other - mine;
            const cpx<T> dw = (i > 0) ? d * tw_at<SIGN>(tws, i * B) : d;
            v[i] = sel(h, dw, mine + other);
        }
        reg_dft3<SIGN, H, T>(v);
#pragma unroll
        for (int m = 0; m < H; ++m) {
            const int n1 = 2 * m + (int)h;
            lds[(n1 * B + k2) * TX + t] = v[m] * tw_at<SIGN>(tws, n1 * k2);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < B; ++kk) v[kk] = lds[(qa * B + kk) * TX + t];
        reg_dft<SIGN, B, T>(v);
        if (s1) {
#pragma unroll
            for (int j = 0; j < B; ++j) {
                const int e = q + A * j;
                if (!(PRUNE && j >= B / 2) && e < n_out) base[e * ES] = v[j];
            }
        }
    }
}

// x-inverse epilogue of one output element qq, with u (and, for DOT 1, a) loaded before the inverse transform so
// that their latency overlaps it (x-inverse 6-RHS launch at 128^3: c64 0.284 -> 0.215 ms, c128 0.463 -> 0.391 ms):
// MODE 1 out = u - v, with the inner products of DOT accumulated (1: a^H out; 2: out^H u and |out|^2); MODE 2
// out = v
template <typename T, int MODE, int DOT>
__device__ __forceinline__ void contig_out_pre(cpx<T> v, cpx<T> uu, cpx<T> a, long long qq, cpx<T>* __restrict__ out,
                                               double acc[3]) {
    if constexpr (MODE == 1) {
        const cpx<T> o = uu - v;
        store_nt(&out[qq], o);
        if constexpr (DOT == 1) {   // a^H o
            acc[0] += (double)a.x * o.x + (double)a.y * o.y;
            acc[1] += (double)a.x * o.y - (double)a.y * o.x;
        } else if constexpr (DOT == 2) {   // o^H u, |o|^2
            acc[0] += (double)o.x * uu.x + (double)o.y * uu.y;
            acc[1] += (double)o.x * uu.y - (double)o.y * uu.x;
            acc[2] += (double)o.x * o.x + (double)o.y * o.y;
        }
    } else {
        store_nt(&out[qq], v);
    }
}

// Fixed-order block sum of the fused inner products of an x-inverse block of NT threads holding TY lines:
// wavefront shuffles, then the wavefronts in order, into dot_parts[(rhs kRedSlots + slot) nparts + block of
// the right-hand side].
template <int NT, int TY, int DOT>
__device__ __forceinline__ void contig_dot_parts(const double acc[3], int tid, double* __restrict__ dot_parts,
                                                 long long dot_lines, int dot_nparts, const SlotMap& sm) {
    constexpr int NW = (NT + 63) / 64;   // whole wavefronts only (checked by fused_dot_blocks)
    constexpr int NS = DOT == 1 ? 2 : 3;
    __shared__ double red[NW][NS];
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double x = acc[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if (lane == 0) red[wave][k] = x;
    }
    __syncthreads();
    if (tid < NS) {
        double x = 0.0;
        for (int w = 0; w < NW; ++w) x += red[w][tid];
        const long long l0 = (long long)blockIdx.x * TY;
        const long long rr = l0 / dot_lines, blk = (l0 - rr * dot_lines) / TY;
        dot_parts[((long long)sm.slot[rr] * kRedSlots + tid) * dot_nparts + blk] = x;
    }
}

// The x passes' transposes take the bank-swizzled LDS slots (fs_slot) in FP32: 6-RHS launches at 128^3 x
// forward 0.184 -> 0.143 ms, x inverse 0.213 -> 0.205 ms; in FP64 they measured no faster (0.353 against 0.356
// ms at 128^3), so FP64 keeps the padded layout.
template <typename T, int L, int LDP>
constexpr bool kSwzX = sizeof(T) == 4 && (L == 128 || L == 256 || L == 512) && (LDP - 1) * FourStep<L>::N1 <= L;

// Contiguous (x) pass over TY lines per block.  MODE 0: forward in place; MODE 1: inverse with
// out = u - v (compact); MODE 2: inverse with out = v (compact).
// DOT (MODE 1 only): inner products of the written field, fused for the Bi-CGSTAB iteration that
// called the operator: 1 = a^H out (slots re, im), 2 = out^H u and ||out||^2 (slots re, im, norm),
// summed over the block in a fixed order into dot_parts[(rhs kRedSlots + slot) nparts + block of the
// right-hand side] (every block holds lines of one right-hand side: dot_lines, the lines per
// right-hand side, is a multiple of TY).
template <typename T, int L, int TY, int SIGN, int MODE, bool PRUNE, int DOT = 0>
__global__ __launch_bounds__(TY * FourStep<L>::N1) void k_fs_contig(cpx<T>* __restrict__ data, long long nlines,
                                                                    int D2, long long S1, long long S2, int n_in,
                                                                    int n_out, const cpx<T>* __restrict__ tw,
                                                                    const cpx<T>* __restrict__ u,
                                                                    cpx<T>* __restrict__ out,
                                                                    const cpx<T>* __restrict__ dot_a,
                                                                    double* __restrict__ dot_parts,
                                                                    long long dot_lines, int dot_nparts,
                                                                    int zbs, SlotMap sm, long long lpr) {
    using F = FourStep<L>;
    constexpr int LDP = TY + 1;
    __shared__ cpx<T> lds[L * LDP];
    __shared__ cpx<T> tws[L];
    const int tid = threadIdx.x, q = tid % F::N1, ln = tid / F::N1;
    stage_twiddles<T, L>(tws, tw, tid, TY * F::N1);
    const long long line = (long long)blockIdx.x * TY + ln;
    const bool valid = line < nlines;
    // compact output row of this thread's line (MODE 1, 2), computed once
    const long long orow = (MODE == 0 || !valid) ? 0 : slot_row(line, lpr, line_position<TY>(line, lpr), sm, D2, zbs);
    const long long o1 = line / D2, o2 = line - o1 * D2;
    cpx<T>* base = data + o1 * S1 + o2 * S2;
    cpx<T> v[F::N2];
    if constexpr (MODE == 0) {
#pragma unroll
        for (int j = 0; j < F::N2; ++j) {
            const int e = q + F::N1 * j;
            v[j] = (!half_slot<L, PRUNE>(j) && valid && e < n_in) ? base[e] : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        fs_forward<T, L, LDP, SIGN, false, kSwzX<T, L, LDP>>(v, lds, tws, ln, q);
        if (valid) {
#pragma unroll
            for (int i = 0; i < F::N2; ++i) {
                const int k = spectral_index<L>(q, i);
                if (k < n_out) base[k] = v[i];
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < F::N2; ++i) {
            const int k = spectral_index<L>(q, i);
            v[i] = (valid && k < n_in) ? load_nt(&base[k]) : cpx<T>{T(0), T(0)};
        }
        // the epilogue's u requested before the transform; r^ for DOT 1 as well in FP64, after it in FP32
        // (there the late loads took the 6-RHS launch at 128^3 from 0.313 to 0.296 ms, and in FP64 the early
        // ones measured 0.462 against 0.469 ms)
        constexpr bool late_a = sizeof(T) == 4;
        cpx<T> up[F::N2], ap[F::N2];
        auto load_a = [&]() __attribute__((always_inline)) {
#pragma unroll
            for (int j = 0; j < F::N2; ++j) {
                const int e = q + F::N1 * j;
                const bool ok = MODE == 1 && DOT == 1 && valid && !half_slot<L, PRUNE>(j) && e < n_out;
                ap[j] = ok ? load_nt(&dot_a[orow * n_out + e]) : cpx<T>{T(0), T(0)};
            }
        };
#pragma unroll
        for (int j = 0; j < F::N2; ++j) {
            const int e = q + F::N1 * j;
            const bool ok = MODE == 1 && valid && !half_slot<L, PRUNE>(j) && e < n_out;
            up[j] = ok ? load_nt(&u[orow * n_out + e]) : cpx<T>{T(0), T(0)};
        }
        if constexpr (!late_a) load_a();
        __syncthreads();
        fs_backward<T, L, LDP, SIGN, kSwzX<T, L, LDP>>(v, lds, tws, ln, q);
        if constexpr (late_a) load_a();
        double acc[3] = {0.0, 0.0, 0.0};
        if (valid) {
#pragma unroll
            for (int j = 0; j < F::N2; ++j) {
                const int e = q + F::N1 * j;
                if (!half_slot<L, PRUNE>(j) && e < n_out)
                    contig_out_pre<T, MODE, DOT>(v[j], up[j], ap[j], orow * n_out + e, out, acc);
            }
        }
        if constexpr (MODE == 1 && DOT != 0)
            contig_dot_parts<TY * F::N1, TY, DOT>(acc, tid, dot_parts, dot_lines, dot_nparts, sm);
    }
}

// Contiguous (x) pass at the lengths with a factor 3 (L = A x 16, A = 3, 6, 12): the asymmetric four-step of
// k_fs_strided3 along lines, 16 threads per line (thread q = tid mod 16) and TY lines per block; MODE and DOT
// as in k_fs_contig.  Threads q >= A transform zeros or a copy of element row A - 1 and write nothing.
template <typename T, int L, int TY, int SIGN, int MODE, bool PRUNE, int DOT = 0>
__global__ __launch_bounds__(TY * 16) void k_fs_contig3(cpx<T>* __restrict__ data, long long nlines, int D2,
                                                         long long S1, long long S2, int n_in, int n_out,
                                                         const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ u,
                                                         cpx<T>* __restrict__ out, const cpx<T>* __restrict__ dot_a,
                                                         double* __restrict__ dot_parts, long long dot_lines,
                                                         int dot_nparts, int zbs, SlotMap sm, long long lpr) {
    constexpr int B = 16, A = L / B;
    static_assert(A * B == L && (A == 3 || A == 6 || A == 12), "lengths 48, 96, 192");
    constexpr int LDP = TY + 1;
    __shared__ cpx<T> lds[L * LDP];
    __shared__ cpx<T> tws[L];
    const int tid = threadIdx.x, q = tid % B, ln = tid / B;
    stage_twiddles<T, L>(tws, tw, tid, TY * B);
    const long long line = (long long)blockIdx.x * TY + ln;
    const bool valid = line < nlines;
    const long long orow = (MODE == 0 || !valid) ? 0 : slot_row(line, lpr, line_position<TY>(line, lpr), sm, D2, zbs);
    const long long o1 = line / D2, o2 = line - o1 * D2;
    cpx<T>* base = data + o1 * S1 + o2 * S2;
    const bool s1 = q < A;
    const int qa = s1 ? q : A - 1;
    cpx<T> v[B];
    if constexpr (MODE == 0) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int e = q + A * j;
            v[j] = (s1 && !(PRUNE && j >= B / 2) && valid && e < n_in) ? base[e] : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        reg_dft<SIGN, B, T, PRUNE>(v);
#pragma unroll
        for (int k2 = 1; k2 < B; ++k2) v[k2] = v[k2] * tw_at<SIGN>(tws, qa * k2);
        if (s1) {
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) lds[(k2 * A + q) * LDP + ln] = v[k2];
        }
        __syncthreads();
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) v[n1] = lds[(q * A + n1) * LDP + ln];
        reg_dft3<SIGN, A, T>(v);
        if (valid) {
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) {
                const int k = q + B * k1;
                if (k < n_out) base[k] = v[k1];
            }
        }
    } else {
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            const int k = q + B * k1;
            v[k1] = (valid && k < n_in) ? load_nt(&base[k]) : cpx<T>{T(0), T(0)};
        }
        // the epilogue's u (and r^ for DOT 1) requested before the transform
        cpx<T> up[B], ap[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int e = q + A * j;
            const bool ok = MODE == 1 && valid && s1 && !(PRUNE && j >= B / 2) && e < n_out;
            up[j] = ok ? load_nt(&u[orow * n_out + e]) : cpx<T>{T(0), T(0)};
            ap[j] = (ok && DOT == 1) ? load_nt(&dot_a[orow * n_out + e]) : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        reg_dft3<SIGN, A, T>(v);
#pragma unroll
        for (int n1 = 1; n1 < A; ++n1) v[n1] = v[n1] * tw_at<SIGN>(tws, n1 * q);
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) lds[(n1 * B + q) * LDP + ln] = v[n1];
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) v[k2] = lds[(qa * B + k2) * LDP + ln];
        reg_dft<SIGN, B, T>(v);
        double acc[3] = {0.0, 0.0, 0.0};
        if (valid && s1) {
#pragma unroll
            for (int j = 0; j < B; ++j) {
                const int e = q + A * j;
                if (!(PRUNE && j >= B / 2) && e < n_out)
                    contig_out_pre<T, MODE, DOT>(v[j], up[j], ap[j], orow * n_out + e, out, acc);
            }
        }
        if constexpr (MODE == 1 && DOT != 0) contig_dot_parts<TY * B, TY, DOT>(acc, tid, dot_parts, dot_lines, dot_nparts, sm);
    }
}

// Contiguous (x) pass at length 384 = 24 x 16: the paired asymmetric four-step of k_fs_strided3p along lines,
// 32 threads per line (thread p = tid mod 32, partner p ^ 1 one lane away); MODE and DOT as in k_fs_contig.
template <typename T, int TY, int SIGN, int MODE, bool PRUNE, int DOT = 0>
__global__ __launch_bounds__(TY * 32) void k_fs_contig3p(cpx<T>* __restrict__ data, long long nlines, int D2,
                                                          long long S1, long long S2, int n_in, int n_out,
                                                          const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ u,
                                                          cpx<T>* __restrict__ out, const cpx<T>* __restrict__ dot_a,
                                                          double* __restrict__ dot_parts, long long dot_lines,
                                                          int dot_nparts, int zbs, SlotMap sm, long long lpr) {
    constexpr int L = 384, B = 16, A = 24, H = 12, NL = 32;
    constexpr int LDP = TY + 1;
    __shared__ cpx<T> lds[L * LDP];
    __shared__ cpx<T> tws[L];
    const int tid = threadIdx.x, q = tid % NL, ln = tid / NL;
    stage_twiddles<T, L>(tws, tw, tid, TY * NL);
    const long long line = (long long)blockIdx.x * TY + ln;
    const bool valid = line < nlines;
    const long long orow = (MODE == 0 || !valid) ? 0 : slot_row(line, lpr, line_position<TY>(line, lpr), sm, D2, zbs);
    const long long o1 = line / D2, o2 = line - o1 * D2;
    cpx<T>* base = data + o1 * S1 + o2 * S2;
    const bool s1 = q < A;
    const int qa = s1 ? q : A - 1;
    const int k2 = q >> 1;
    const bool h = q & 1;
    cpx<T> v[B];
    if constexpr (MODE == 0) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int e = q + A * j;
            v[j] = (s1 && !(PRUNE && j >= B / 2) && valid && e < n_in) ? base[e] : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        reg_dft<SIGN, B, T, PRUNE>(v);
#pragma unroll
        for (int kk = 1; kk < B; ++kk) v[kk] = v[kk] * tw_at<SIGN>(tws, qa * kk);
        if (s1) {
#pragma unroll
            for (int kk = 0; kk < B; ++kk) lds[(kk * A + q) * LDP + ln] = v[kk];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < H; ++m) v[m] = lds[(k2 * A + 2 * m + (int)h) * LDP + ln];
        reg_dft3<SIGN, H, T>(v);
#pragma unroll
        for (int i = 0; i < H; ++i) {
            cpx<T> mine = v[i];
            if (i > 0) mine = sel(h, mine * tw_at<SIGN>(tws, i * B), mine);
            const cpx<T> other = lane_xor<1>(mine);
            const cpx<T> x = sel(h, other - mine, mine + other);
            const int k = k2 + B * (i + H * (int)h);
            if (valid && k < n_out) base[k] = x;
        }
    } else {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const int k = k2 + B * (i + H * (int)h);
            v[i] = (valid && k < n_in) ? load_nt(&base[k]) : cpx<T>{T(0), T(0)};
        }
        // the epilogue's u (and r^ for DOT 1) requested before the transform
        cpx<T> up[B], ap[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int e = q + A * j;
            const bool ok = MODE == 1 && valid && s1 && !(PRUNE && j >= B / 2) && e < n_out;
            up[j] = ok ? load_nt(&u[orow * n_out + e]) : cpx<T>{T(0), T(0)};
            ap[j] = (ok && DOT == 1) ? load_nt(&dot_a[orow * n_out + e]) : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const cpx<T> mine = v[i];
            const cpx<T> other = lane_xor<1>(mine);
            const cpx<T> d = other - mine;
            const cpx<T> dw = (i > 0) ? d * tw_at<SIGN>(tws, i * B) : d;
            v[i] = sel(h, dw, mine + other);
        }
        reg_dft3<SIGN, H, T>(v);
#pragma unroll
        for (int m = 0; m < H; ++m) {
            const int n1 = 2 * m + (int)h;
            lds[(n1 * B + k2) * LDP + ln] = v[m] * tw_at<SIGN>(tws, n1 * k2);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < B; ++kk) v[kk] = lds[(qa * B + kk) * LDP + ln];
        reg_dft<SIGN, B, T>(v);
        double acc[3] = {0.0, 0.0, 0.0};
        if (valid && s1) {
#pragma unroll
            for (int j = 0; j < B; ++j) {
                const int e = q + A * j;
                if (!(PRUNE && j >= B / 2) && e < n_out)
                    contig_out_pre<T, MODE, DOT>(v[j], up[j], ap[j], orow * n_out + e, out, acc);
            }
        }
        if constexpr (MODE == 1 && DOT != 0) contig_dot_parts<TY * NL, TY, DOT>(acc, tid, dot_parts, dot_lines, dot_nparts, sm);
    }
}

__device__ __forceinline__ void fold_index(int k, int L, int& kf, bool& flipped) {
    flipped = k > L / 2;
    kf = flipped ? L - k : k;
}

// Fused z pass with the four-step FFT: three components per column held in registers.  Logical
// block order (XCD-aware): right-hand side fastest, then x tiles and y rows in mirror pairs, so the
// blocks that read the same octant rows of G^ run together on one XCD.  The data occupy z < n3 <= L/2.
// a b + c with one rounding
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// g1 f1 + g2 f2 + g3 f3 as two chains of fused multiply-adds (12 operations instead of 16)
template <typename T>
__device__ __forceinline__ cpx<T> cdot3(cpx<T> g1, cpx<T> f1, cpx<T> g2, cpx<T> f2, cpx<T> g3, cpx<T> f3) {
    T re = g1.x * f1.x, im = g1.x * f1.y;
    re = fmadd(-g1.y, f1.y, re);
    im = fmadd(g1.y, f1.x, im);
    re = fmadd(g2.x, f2.x, re);
    im = fmadd(g2.x, f2.y, im);
    re = fmadd(-g2.y, f2.y, re);
    im = fmadd(g2.y, f2.x, im);
    re = fmadd(g3.x, f3.x, re);
    im = fmadd(g3.x, f3.y, im);
    re = fmadd(-g3.y, f3.y, re);
    im = fmadd(g3.y, f3.x, im);
    return {re, im};
}

// Lean forms (FP64): addresses split into a part common to the block (scalar registers) and the lane's
// byte offset in 32 bits, so that no per-element 64-bit arithmetic is needed (the host guarantees that
// (N1 - 1) ES + TX elements of the field and the whole table span less than 4 GiB); the 3 x 3 product as
// fused multiply-add chains; the first forward stage skips the known-zero half.  They cut the FP64
// kernel's vector instructions by 13 % and its time by 8 % at length 256, 6 right-hand sides; in FP32
// they cut the instructions as much but schedule worse (0.738 against 0.728 ms), so FP32 keeps the
// plain forms.
template <typename T, int L, int TX, bool HALF = false, int ZBS = 0>
__global__ __launch_bounds__((TX * ZSplit<T, L, HALF>::N1), (sizeof(T) == 4 ? (z_paired<T, L, HALF>() ? 2 : (L >= 512 ? 1 : 3)) : 1)) void k_fs_zgreen(cpx<T>* __restrict__ data, int nrhs, int L1,
                                                                    int L2, long long CS, long long RS, long long ES,
                                                                    int n3, GreenTabs<T> gt,
                                                                    const cpx<T>* __restrict__ tw, long long nb_real) {
    using F = ZSplit<T, L, HALF>;
    constexpr bool PAIRED = z_paired<T, L, HALF>();
    constexpr int zbs = ZBS;   // work buffer layout (zplane_offset), fixed at compile time
    __shared__ cpx<T> lds[L * TX];
    __shared__ cpx<T> tws[L];
    const long long lb = xcd_logical_block(blockIdx.x, nb_real);
    if (lb < 0) return;
    const int tid = threadIdx.x, t = tid % TX, q = tid / TX;
    stage_twiddles<T, L>(tws, tw, tid, TX * F::N1);
    const int ntx = L1 / TX;
    const int rhs = (int)(lb % nrhs);
    const cpx<T>* __restrict__ ghat = gt.g[rhs];   // this position's frequency
    const int xt = paired_row((int)((lb / nrhs) % ntx), ntx);
    const int y = paired_row((int)(lb / ((long long)nrhs * ntx)), L2);
    const int kx0 = xt * TX + t;
    constexpr bool LEAN = sizeof(T) == 8;
    // work buffer layout of zplane_offset: element e of a line at (e >> zbs) ZS + (e mod 2^zbs) L1, ZS the
    // z-block pitch; 2^zbs divides N1 (host), so thread q's part of that offset is the same for all its elements
    const long long ZS = ES << zbs;
    char* const ub = reinterpret_cast<char*>(data + (long long)rhs * RS + zrow_offset(y, zbs, L1) + (long long)xt * TX);
    const unsigned lane = ((unsigned)t + (unsigned)(q >> zbs) * (unsigned)ZS + (unsigned)(q & ((1 << zbs) - 1)) * (unsigned)L1) *
                          (unsigned)sizeof(cpx<T>);
    // element j of component c of this thread's line
    auto elem = [&](int c, int j) __attribute__((always_inline)) {
        if constexpr (LEAN)   // scalar base plus the lane offset
            return reinterpret_cast<cpx<T>*>(ub + (c * CS + (long long)((F::N1 >> zbs) * j) * ZS) * (long long)sizeof(cpx<T>) +
                                             lane);
        else
            return data + (long long)rhs * RS + zrow_offset(y, zbs, L1) + kx0 + c * CS +
                   zplane_offset(q + F::N1 * j, zbs, L2, L1);
    };
    cpx<T> v[3][F::N2];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < (LEAN ? F::N2 / 2 : F::N2); ++j) {
            const int e = q + F::N1 * j;
            // the field is streamed once: non-temporal loads and stores leave the caches to the table
            v[c][j] = (j < F::N2 / 2 && e < n3) ? load_nt(elem(c, j)) : cpx<T>{T(0), T(0)};
        }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) z_forward<T, L, TX, -1, PAIRED, LEAN>(v[c], lds, tws, t, q);

    const int O1 = L1 / 2 + 1, O2 = L2 / 2 + 1;
    int kx, ky;
    bool fx, fy;
    fold_index(kx0, L1, kx, fx);
    fold_index(y, L2, ky, fy);
    // half-space table: k_x > L1/2 reads the entry at -k
    const bool hneg = kx0 > L1 / 2;
    const int hx = hneg ? L1 - kx0 : kx0, hy = hneg ? (L2 - y) % L2 : y;
    const char* const gb = reinterpret_cast<const char*>(ghat);
    auto table_at = [&](int a, int b, int n, int c) __attribute__((always_inline)) {   // entry (a n + b) O1 + c
        if constexpr (LEAN)
            return reinterpret_cast<const cpx<T>*>(
                gb + (((unsigned)a * (unsigned)n + (unsigned)b) * (unsigned)O1 + (unsigned)c) * (unsigned)(6 * sizeof(cpx<T>)));
        else
            return ghat + (((long long)a * n + b) * O1 + c) * 6;
    };
#pragma unroll
    for (int i = 0; i < F::N2; ++i) {
        cpx<T> g[6];
        if constexpr (HALF) {
            const int kz0 = z_spectral_index<L, PAIRED>(q, i);
            const int hz = hneg ? (L - kz0) % L : kz0;
            load_g6(table_at(hz, hy, L2, hx), 0, g);
        } else {
            int kz;
            bool fz;
            fold_index(z_spectral_index<L, PAIRED>(q, i), L, kz, fz);
            load_g6(table_at(kz, ky, O2, kx), 0, g);
            if (fy != fz) g[3] = T(-1) * g[3];
            if (fx != fz) g[4] = T(-1) * g[4];
            if (fx != fy) g[5] = T(-1) * g[5];
        }
        const cpx<T> g11 = g[0], g22 = g[1], g33 = g[2], g23 = g[3], g13 = g[4], g12 = g[5];
        const cpx<T> f1 = v[0][i], f2 = v[1][i], f3 = v[2][i];
        if constexpr (LEAN) {
            v[0][i] = cdot3(g11, f1, g12, f2, g13, f3);
            v[1][i] = cdot3(g12, f1, g22, f2, g23, f3);
            v[2][i] = cdot3(g13, f1, g23, f2, g33, f3);
        } else {
            v[0][i] = g11 * f1 + g12 * f2 + g13 * f3;
            v[1][i] = g12 * f1 + g22 * f2 + g23 * f3;
            v[2][i] = g13 * f1 + g23 * f2 + g33 * f3;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) z_backward<T, L, TX, +1, PAIRED>(v[c], lds, tws, t, q);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < F::N2 / 2; ++j) {
            const int e = q + F::N1 * j;
            if (e < n3) store_nt(elem(c, j), v[c][j]);
        }
}

// Fused z pass for the lengths with a factor 3 (L = A x 16, A = 3, 6, 12: 48, 96, 192) with the octant table:
// an asymmetric four-step over 16 threads per column.  With n = n1 + A n2 and k = k2 + 16 k1 (n1, k1 < A;
// n2, k2 < 16),
//   X[k2 + 16 k1] = sum_{n1} W_A^{n1 k1} W_L^{n1 k2} sum_{n2} W_16^{n2 k2} x[n1 + A n2].
// Threads q < A run the length-16 DFT of the column's elements q + A n2 (n2 < 8: the data occupy z < L/2, so
// the upper half is zero) and the twiddles W_L^{q k2}; one LDS transpose gives thread q = k2 the A values of
// its length-A DFT (reg_dft3), whose outputs X[q + 16 k1] sit in slot k1 when the Green's table multiplies
// them.  The inverse runs the same steps backwards and threads q < A store their first 8 outputs.  The same
// register footprint (16 values of each component) and block (TX columns x 16 threads) as length 256.
template <typename T, int L, int TX, int ZBS>
__global__ __launch_bounds__(TX * 16, (sizeof(T) == 4 ? 3 : 1)) void k_fs_zgreen3(
    cpx<T>* __restrict__ data, int nrhs, int L1, int L2, long long CS, long long RS, int n3, GreenTabs<T> gt,
    const cpx<T>* __restrict__ tw, long long nb_real) {
    constexpr int B = 16, A = L / B;
    static_assert(A * B == L && (A == 3 || A == 6 || A == 12), "lengths 48, 96, 192");
    __shared__ cpx<T> lds[L * TX];
    __shared__ cpx<T> tws[L];
    const long long lb = xcd_logical_block(blockIdx.x, nb_real);
    if (lb < 0) return;
    const int tid = threadIdx.x, t = tid % TX, q = tid / TX;
    stage_twiddles<T, L>(tws, tw, tid, TX * B);
    const int ntx = L1 / TX;
    const int rhs = (int)(lb % nrhs);
    const cpx<T>* __restrict__ ghat = gt.g[rhs];   // this position's frequency
    const int xt = paired_row((int)((lb / nrhs) % ntx), ntx);
    const int y = paired_row((int)(lb / ((long long)nrhs * ntx)), L2);
    const int kx0 = xt * TX + t;
    cpx<T>* const col = data + (long long)rhs * RS + zrow_offset(y, ZBS, L1) + kx0;
    const bool s1 = q < A;   // a first-stage thread: element n1 = q of the line
    const int qa = s1 ? q : A - 1;
    cpx<T> v[3][B];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int e = q + A * j;
            v[c][j] = (s1 && j < B / 2 && e < n3) ? load_nt(&col[c * CS + zplane_offset(e, ZBS, L2, L1)])
                                                   : cpx<T>{T(0), T(0)};
        }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // every thread transforms (threads q >= A hold zeros and write nothing): no divergent merge
        reg_dft<-1, B, T, true>(v[c]);
#pragma unroll
        for (int k2 = 1; k2 < B; ++k2) v[c][k2] = v[c][k2] * tw_at<-1>(tws, qa * k2);
        if (s1) {
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) lds[(k2 * A + q) * TX + t] = v[c][k2];
        }
        __syncthreads();
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) v[c][n1] = lds[(q * A + n1) * TX + t];
#pragma unroll
        for (int n1 = A; n1 < B; ++n1) v[c][n1] = cpx<T>{T(0), T(0)};   // unused slots: no live registers
        __syncthreads();
        reg_dft3<-1, A, T>(v[c]);
    }

    const int O1 = L1 / 2 + 1, O2 = L2 / 2 + 1;
    int kx, ky;
    bool fx, fy;
    fold_index(kx0, L1, kx, fx);
    fold_index(y, L2, ky, fy);
#pragma unroll
    for (int i = 0; i < A; ++i) {
        int kz;
        bool fz;
        fold_index(q + B * i, L, kz, fz);
        cpx<T> g[6];
        load_g6(ghat, ((long long)kz * O2 + ky) * O1 + kx, g);
        if (fy != fz) g[3] = T(-1) * g[3];
        if (fx != fz) g[4] = T(-1) * g[4];
        if (fx != fy) g[5] = T(-1) * g[5];
        const cpx<T> g11 = g[0], g22 = g[1], g33 = g[2], g23 = g[3], g13 = g[4], g12 = g[5];
        const cpx<T> f1 = v[0][i], f2 = v[1][i], f3 = v[2][i];
        v[0][i] = g11 * f1 + g12 * f2 + g13 * f3;
        v[1][i] = g12 * f1 + g22 * f2 + g23 * f3;
        v[2][i] = g13 * f1 + g23 * f2 + g33 * f3;
    }

#pragma unroll
    for (int c = 0; c < 3; ++c) {
        reg_dft3<+1, A, T>(v[c]);
#pragma unroll
        for (int n1 = 1; n1 < A; ++n1) v[c][n1] = v[c][n1] * tw_at<+1>(tws, n1 * q);
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) lds[(n1 * B + q) * TX + t] = v[c][n1];
        __syncthreads();
        // threads q >= A read and transform row A - 1 again and store nothing
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) v[c][k2] = lds[(qa * B + k2) * TX + t];
        __syncthreads();
        reg_dft<+1, B, T>(v[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < B / 2; ++j) {
            const int e = q + A * j;
            if (s1 && e < n3) store_nt(&col[c * CS + zplane_offset(e, ZBS, L2, L1)], v[c][j]);
        }
}

// Fused z pass at length 384 = 24 x 16 with the octant table: the asymmetric four-step of k_fs_zgreen3 with the
// second stage split over thread pairs.  Threads q < 24 run the length-16 DFTs of elements q + 24 n2 (n2 < 8)
// and the twiddles W_384^{q k2}; after the LDS transpose thread p = 2 k2 + h holds the 12 values n1 = 2 m + h
// of line k2, runs a length-12 DFT, and the radix-2 step that joins the even (h = 0) and odd (h = 1) halves
// of the length-24 DFT exchanges values with the partner thread p ^ 1, TX lanes away in the same wavefront:
// thread p ends with X[k2 + 16 (i + 12 h)] in slot i.  The inverse runs the same steps backwards.  32 threads
// per column, 16 values of each component per thread.
template <typename T, int TX, int ZBS>
__global__ __launch_bounds__(TX * 32, (sizeof(T) == 4 ? 2 : 1)) void k_fs_zgreen3p(
    cpx<T>* __restrict__ data, int nrhs, int L1, int L2, long long CS, long long RS, int n3, GreenTabs<T> gt,
    const cpx<T>* __restrict__ tw, long long nb_real) {
    constexpr int L = 384, B = 16, A = 24, H = 12;
    static_assert(2 * TX <= 64, "partner lanes share a wavefront");
    __shared__ cpx<T> lds[L * TX];
    __shared__ cpx<T> tws[L];
    const long long lb = xcd_logical_block(blockIdx.x, nb_real);
    if (lb < 0) return;
    const int tid = threadIdx.x, t = tid % TX, q = tid / TX;
    stage_twiddles<T, L>(tws, tw, tid, TX * 32);
    const int ntx = L1 / TX;
    const int rhs = (int)(lb % nrhs);
    const cpx<T>* __restrict__ ghat = gt.g[rhs];
    const int xt = paired_row((int)((lb / nrhs) % ntx), ntx);
    const int y = paired_row((int)(lb / ((long long)nrhs * ntx)), L2);
    const int kx0 = xt * TX + t;
    cpx<T>* const col = data + (long long)rhs * RS + zrow_offset(y, ZBS, L1) + kx0;
    const bool s1 = q < A;       // a first-stage thread (element n1 = q)
    const int qa = s1 ? q : A - 1;
    const int k2 = q >> 1;       // second stage: line k2, half h
    const bool h = q & 1;
    cpx<T> v[3][B];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int e = q + A * j;
            v[c][j] = (s1 && j < B / 2 && e < n3) ? load_nt(&col[c * CS + zplane_offset(e, ZBS, L2, L1)])
                                                   : cpx<T>{T(0), T(0)};
        }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // every thread transforms (threads q >= 24 hold zeros and write nothing): no divergent merge
        reg_dft<-1, B, T, true>(v[c]);
#pragma unroll
        for (int kk = 1; kk < B; ++kk) v[c][kk] = v[c][kk] * tw_at<-1>(tws, qa * kk);
        if (s1) {
#pragma unroll
            for (int kk = 0; kk < B; ++kk) lds[(kk * A + q) * TX + t] = v[c][kk];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < H; ++m) v[c][m] = lds[(k2 * A + 2 * m + (int)h) * TX + t];
#pragma unroll
        for (int m = H; m < B; ++m) v[c][m] = cpx<T>{T(0), T(0)};
        __syncthreads();
        reg_dft3<-1, H, T>(v[c]);
#pragma unroll
        for (int i = 0; i < H; ++i) {
            cpx<T> mine = v[c][i];
            if (i > 0) mine = sel(h, mine * tw_at<-1>(tws, i * B), mine);
            const cpx<T> other = lane_xor<TX>(mine);
            v[c][i] = sel(h, other - mine, mine + other);
        }
    }

    const int O1 = L1 / 2 + 1, O2 = L2 / 2 + 1;
    int kx, ky;
    bool fx, fy;
    fold_index(kx0, L1, kx, fx);
    fold_index(y, L2, ky, fy);
#pragma unroll
    for (int i = 0; i < H; ++i) {
        int kz;
        bool fz;
        fold_index(k2 + B * (i + H * (int)h), L, kz, fz);
        cpx<T> g[6];
        load_g6(ghat, ((long long)kz * O2 + ky) * O1 + kx, g);
        if (fy != fz) g[3] = T(-1) * g[3];
        if (fx != fz) g[4] = T(-1) * g[4];
        if (fx != fy) g[5] = T(-1) * g[5];
        const cpx<T> g11 = g[0], g22 = g[1], g33 = g[2], g23 = g[3], g13 = g[4], g12 = g[5];
        const cpx<T> f1 = v[0][i], f2 = v[1][i], f3 = v[2][i];
        v[0][i] = g11 * f1 + g12 * f2 + g13 * f3;
        v[1][i] = g12 * f1 + g22 * f2 + g23 * f3;
        v[2][i] = g13 * f1 + g23 * f2 + g33 * f3;
    }

#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const cpx<T> mine = v[c][i];
            const cpx<T> other = lane_xor<TX>(mine);
            const cpx<T> d = other - mine;
            const cpx<T> dw = (i > 0) ? d * tw_at<+1>(tws, i * B) : d;
            v[c][i] = sel(h, dw, mine + other);
        }
        reg_dft3<+1, H, T>(v[c]);
#pragma unroll
        for (int m = 0; m < H; ++m) {
            const int n1 = 2 * m + (int)h;
            lds[(n1 * B + k2) * TX + t] = v[c][m] * tw_at<+1>(tws, n1 * k2);
        }
        __syncthreads();
        // threads q >= 24 read and transform row 23 again and store nothing
#pragma unroll
        for (int kk = 0; kk < B; ++kk) v[c][kk] = lds[(qa * B + kk) * TX + t];
        __syncthreads();
        reg_dft<+1, B, T>(v[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int j = 0; j < B / 2; ++j) {
            const int e = q + A * j;
            if (s1 && e < n3) store_nt(&col[c * CS + zplane_offset(e, ZBS, L2, L1)], v[c][j]);
        }
}

// z pass in registers where three components of N2 values fit (both precisions up to 512, paired at 512)
template <typename T, int L, bool HALF>
constexpr bool fs_z_ok() {
    if constexpr (!fs_ok<T, L>())
        return false;
    else
        return 3 * ZSplit<T, L, HALF>::N2 * (int)sizeof(cpx<T>) <= 3 * 32 * 8;
}

// ------------------------------------------------------------------------------------------
// host dispatch over the supported lengths

#define LS_FOR_LENGTHS(X) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

// LS_FFT=stockham in the environment selects the LDS Stockham kernels everywhere (both paths are
// kept under test); otherwise the register four-step kernels run wherever they fit.
bool use_fourstep() {
    static const bool fs = [] {
        const char* e = std::getenv("LS_FFT");
        return !(e && std::strcmp(e, "stockham") == 0);
    }();
    return fs;
}

// sm, lpr: the slot of each position and the lines per position, for the compact outputs of MODE 1 and 2
template <typename T, int SIGN, int MODE, bool PRUNE, int DOT = 0>
int launch_contig(Ctx* c, int L, cpx<T>* data, long long nlines, int D2, long long S1, long long S2, int n_in,
                  int n_out, const cpx<T>* tw, const cpx<T>* u, cpx<T>* out, const char* name, int variant = 0,
                  int zbs = 0, const SlotMap& sm = SlotMap{}, long long lpr = 1, int nrhs = 0) {
    c->prof.begin(c->stream, name, nrhs);
    const bool fs = variant == 0 && use_fourstep();
    if (DOT != 0 && !fs) return fail(LS_ERR_STATE, "fused inner products need the register four-step x pass");
    switch (L) {
#define CASE(LL)                                                                                             \
    case LL: {                                                                                               \
        if constexpr (LL == 48 || LL == 96 || LL == 192 || LL == 384) {                                      \
            if (fs) {                                                                                        \
                constexpr int TY = seg_cols<T>();                                                            \
                const long long nb = (nlines + TY - 1) / TY;                                                 \
                if constexpr (LL == 384)                                                                     \
                    hipLaunchKernelGGL((k_fs_contig3p<T, TY, SIGN, MODE, PRUNE, DOT>), dim3((unsigned)nb),   \
                                       dim3(TY * 32), 0, c->stream, data, nlines, D2, S1, S2, n_in, n_out,   \
                                       tw, u, out, (const cpx<T>*)c->dot.a, c->dot.parts, c->dot.lines,      \
                                       c->dot.nparts, zbs, sm, lpr);                                         \
                else                                                                                         \
                    hipLaunchKernelGGL((k_fs_contig3<T, LL, TY, SIGN, MODE, PRUNE, DOT>), dim3((unsigned)nb), \
                                       dim3(TY * 16), 0, c->stream, data, nlines, D2, S1, S2, n_in, n_out,   \
                                       tw, u, out, (const cpx<T>*)c->dot.a, c->dot.parts, c->dot.lines,      \
                                       c->dot.nparts, zbs, sm, lpr);                                         \
                break;                                                                                       \
            }                                                                                                \
        }                                                                                                    \
        if constexpr (fs_ok<T, LL>()) {                                                                      \
            if (fs) {                                                                                        \
                constexpr int TY = seg_cols<T>();                                                            \
                const long long nb = (nlines + TY - 1) / TY;                                                 \
                hipLaunchKernelGGL((k_fs_contig<T, LL, TY, SIGN, MODE, PRUNE, DOT>), dim3((unsigned)nb),             \
                                   dim3(fs_threads<T, LL>()), 0, c->stream, data, nlines, D2, S1, S2, n_in,  \
                                   n_out, tw, u, out, (const cpx<T>*)c->dot.a, c->dot.parts, c->dot.lines,   \
                                   c->dot.nparts, zbs, sm, lpr);                                             \
                break;                                                                                       \
            }                                                                                                \
        }                                                                                                    \
        if constexpr (DOT != 0) return fail(LS_ERR_STATE, "fused inner products need a register x pass");     \
        constexpr int TY = contig_lines<T, LL>();                                                            \
        const long long nb = (nlines + TY - 1) / TY;                                                         \
        hipLaunchKernelGGL((k_fft_contig<T, LL, TY, SIGN, MODE>), dim3((unsigned)nb), dim3(kThreads), 0,     \
                           c->stream, data, nlines, D2, S1, S2, n_in, n_out, tw, u, out, zbs, sm, lpr);      \
        break;                                                                                               \
    }
        LS_FOR_LENGTHS(CASE)
#undef CASE
        default:
            return fail(LS_ERR_ARG, "unsupported FFT length");
    }
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

// Strided passes at the powers of two from 64 to 256 and at 48, 96 and 192 take tiles of twice the columns (256-byte
// segments, twice the threads, the same 16 values per thread) where the x length allows: a plain copy with that
// access pattern moves 5.62 TB/s against 5.23 with 128-byte segments.  Measured on 6-RHS applies: FP32 y passes
// per chunk of 2 right-hand sides at 128^3 0.099 -> 0.097 ms (forward) and 0.113 -> 0.108 ms (inverse), y
// inverse at 64^3 0.047 -> 0.044 ms and at 96^3 0.128 -> 0.123 ms; FP64 per right-hand side at 128^3 0.111 ->
// 0.102 and 0.111 -> 0.103 ms, y inverse at 64^3 0.086 -> 0.077 ms and at 96^3 0.141 -> 0.126 ms.
template <typename T, int L>
constexpr bool strided_wide() {
    return L >= 64 && L <= 256 && (L & (L - 1)) == 0;
}
// the factor-3 kernel (k_fs_strided3)
template <typename T, int L>
constexpr bool strided3_wide() {
    return L == 48 || L == 96 || L == 192;
}

template <typename T, int SIGN, bool PRUNE>
int launch_strided(Ctx* c, int L, cpx<T>* data, int NX, int D2, int D1, long long S1, long long S2, long long ES,
                   int n_in, int n_out, const cpx<T>* tw, const char* name, int variant = 0, int nrhs = 0) {
    constexpr int TX = strided_cols<T>();
    static_assert(TX == seg_cols<T>(), "both strided kernels use 128-byte column tiles");
    if (NX % TX) return fail(LS_ERR_ARG, "x length not a multiple of the column tile");
    c->prof.begin(c->stream, name, nrhs);
    const bool fs = variant == 0 && use_fourstep();
    const bool wide = c->y_wide[sizeof(T) == 8 ? 0 : 1] != 0;
    switch (L) {
#define CASE(LL)                                                                                             \
    case LL: {                                                                                               \
        if constexpr (strided3_wide<T, LL>()) {                                                              \
            if (fs && wide && NX % (2 * TX) == 0) {                                                          \
                hipLaunchKernelGGL((k_fs_strided3<T, LL, 2 * TX, SIGN, PRUNE>), dim3(NX / (2 * TX), D2, D1),       \
                                   dim3(2 * TX * 16), 0, c->stream, data, S1, S2, ES, n_in, n_out, tw);      \
                break;                                                                                       \
            }                                                                                                \
        }                                                                                                    \
        if constexpr (LL == 48 || LL == 96 || LL == 192) {                                                   \
            if (fs) {                                                                                        \
                hipLaunchKernelGGL((k_fs_strided3<T, LL, TX, SIGN, PRUNE>), dim3(NX / TX, D2, D1),           \
                                   dim3(TX * 16), 0, c->stream, data, S1, S2, ES, n_in, n_out, tw);          \
                break;                                                                                       \
            }                                                                                                \
        }                                                                                                    \
        if constexpr (LL == 384) {                                                                           \
            if (fs) {                                                                                        \
                hipLaunchKernelGGL((k_fs_strided3p<T, TX, SIGN, PRUNE>), dim3(NX / TX, D2, D1),              \
                                   dim3(TX * 32), 0, c->stream, data, S1, S2, ES, n_in, n_out, tw);          \
                break;                                                                                       \
            }                                                                                                \
        }                                                                                                    \
        if constexpr (strided_wide<T, LL>()) {                                                               \
            if (fs && wide && NX % (2 * TX) == 0) {                                                          \
                hipLaunchKernelGGL((k_fs_strided<T, LL, 2 * TX, SIGN, PRUNE>), dim3(NX / (2 * TX), D2, D1),        \
                                   dim3(2 * fs_threads<T, LL>()), 0, c->stream, data, S1, S2, ES, n_in, n_out,   \
                                   tw);                                                                      \
                break;                                                                                       \
            }                                                                                                \
        }                                                                                                    \
        if constexpr (fs_ok<T, LL>()) {                                                                      \
            if (fs) {                                                                                        \
                hipLaunchKernelGGL((k_fs_strided<T, LL, TX, SIGN, PRUNE>), dim3(NX / TX, D2, D1),                    \
                                   dim3(fs_threads<T, LL>()), 0, c->stream, data, S1, S2, ES, n_in, n_out,   \
                                   tw);                                                                      \
                break;                                                                                       \
            }                                                                                                \
        }                                                                                                    \
        hipLaunchKernelGGL((k_fft_strided<T, LL, TX, SIGN>), dim3(NX / TX, D2, D1), dim3(kThreads), 0,        \
                           c->stream, data, S1, S2, ES, n_in, n_out, tw);                                    \
        break;                                                                                               \
    }
        LS_FOR_LENGTHS(CASE)
#undef CASE
        default:
            return fail(LS_ERR_ARG, "unsupported FFT length");
    }
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

// threads per block of the register z pass
template <typename T, int LL, bool HALF>
constexpr int z_threads() {
    return seg_cols<T>() * ZSplit<T, LL, HALF>::N1;
}
// Register z pass for one table layout (HALF) and work-buffer layout (c->zbs): 1 if launched, 0 if the
// register kernel does not apply (the caller takes the LDS kernel), -1 on a tile mismatch.
template <typename T, int LL, bool HALF>
int try_fs_z(Ctx* c, bool fs, cpx<T>* data, int nrhs, long long CS, long long RS, long long ES, const GreenTabs<T>& ghat,
             const cpx<T>* tw) {
    if constexpr (!HALF && (LL == 192 || (sizeof(T) == 4 && (LL == 48 || LL == 96)))) {
        // the asymmetric four-step (k_fs_zgreen3); the half-space table keeps the LDS kernel, and so does FP64
        // at 48 and 96, where it measured faster (6-RHS launches: 0.027 against 0.035 ms at 48, 0.129
        // against 0.131 ms at 96; at 192 the register kernel takes 0.80 ms against 1.24)
        if (fs) {
            constexpr int TX = seg_cols<T>();
            if (c->L1 % TX) return -1;
            const long long nb = (long long)nrhs * (c->L1 / TX) * c->L2;
            const unsigned nbl = (unsigned)((nb + 7) / 8 * 8);
            if (c->zbs)
                hipLaunchKernelGGL((k_fs_zgreen3<T, LL, TX, 3>), dim3(nbl), dim3(TX * 16), 0, c->stream, data, nrhs,
                                   c->L1, c->L2, CS, RS, c->n3, ghat, tw, nb);
            else
                hipLaunchKernelGGL((k_fs_zgreen3<T, LL, TX, 0>), dim3(nbl), dim3(TX * 16), 0, c->stream, data, nrhs,
                                   c->L1, c->L2, CS, RS, c->n3, ghat, tw, nb);
            return 1;
        }
        return 0;
    }
    if constexpr (!HALF && LL == 384) {
        // the paired asymmetric four-step (k_fs_zgreen3p); the half-space table keeps the LDS kernel
        if (fs) {
            constexpr int TX = seg_cols<T>();
            if (c->L1 % TX) return -1;
            const long long nb = (long long)nrhs * (c->L1 / TX) * c->L2;
            const unsigned nbl = (unsigned)((nb + 7) / 8 * 8);
            if (c->zbs)
                hipLaunchKernelGGL((k_fs_zgreen3p<T, TX, 3>), dim3(nbl), dim3(TX * 32), 0, c->stream, data, nrhs,
                                   c->L1, c->L2, CS, RS, c->n3, ghat, tw, nb);
            else
                hipLaunchKernelGGL((k_fs_zgreen3p<T, TX, 0>), dim3(nbl), dim3(TX * 32), 0, c->stream, data, nrhs,
                                   c->L1, c->L2, CS, RS, c->n3, ghat, tw, nb);
            return 1;
        }
        return 0;
    }
    if constexpr (fs_z_ok<T, LL, HALF>()) {
        // the register kernel needs 2^zbs to divide the threads per line
        if (fs && (z_threads<T, LL, HALF>() / seg_cols<T>()) % (1 << c->zbs) == 0) {
            constexpr int TX = seg_cols<T>();
            if (c->L1 % TX) return -1;
            const long long nb = (long long)nrhs * (c->L1 / TX) * c->L2;
            const unsigned nbl = (unsigned)((nb + 7) / 8 * 8);
            if (c->zbs)
                hipLaunchKernelGGL((k_fs_zgreen<T, LL, TX, HALF, 3>), dim3(nbl), dim3(z_threads<T, LL, HALF>()), 0,
                                   c->stream, data, nrhs, c->L1, c->L2, CS, RS, ES, c->n3, ghat, tw, nb);
            else
                hipLaunchKernelGGL((k_fs_zgreen<T, LL, TX, HALF, 0>), dim3(nbl), dim3(z_threads<T, LL, HALF>()), 0,
                                   c->stream, data, nrhs, c->L1, c->L2, CS, RS, ES, c->n3, ghat, tw, nb);
            return 1;
        }
    }
    return 0;
}
// LDS z pass for one work-buffer layout (ZBS, compile time), full or half table
template <typename T, int LL, int TX, int ZBS>
void launch_lds_z(Ctx* c, cpx<T>* data, int nrhs, long long CS, long long RS, long long ES, const GreenTabs<T>& ghat,
                  const cpx<T>* tw) {
    const dim3 grid(nrhs * (c->L1 / TX), c->L2, 1);
    if (c->green_half)
        hipLaunchKernelGGL((k_fft_zgreen<T, LL, TX, true, ZBS>), grid, dim3(kThreads), 0, c->stream, data, nrhs,
                           c->L1, c->L2, CS, RS, ES, c->n3, ghat, tw);
    else
        hipLaunchKernelGGL((k_fft_zgreen<T, LL, TX, false, ZBS>), grid, dim3(kThreads), 0, c->stream, data, nrhs,
                           c->L1, c->L2, CS, RS, ES, c->n3, ghat, tw);
}

template <typename T>
int launch_zgreen(Ctx* c, cpx<T>* data, int nrhs, const GreenTabs<T>& ghat, const cpx<T>* tw, int variant = 0,
                  int ntab = 1) {
    const int L1 = c->L1, L2 = c->L2, L = c->L3;
    const long long CS = (long long)c->n3 * L2 * L1;
    const long long RS = 3 * CS;
    const long long ES = (long long)L2 * L1;
    // the register kernel addresses a thread's line and the table with 32-bit byte offsets; larger
    // grids take the LDS kernel
    const long long table = c->green_half ? (long long)L * L2 * (L1 / 2 + 1)
                                          : (long long)(L / 2 + 1) * (L2 / 2 + 1) * (L1 / 2 + 1);
    const bool off32 = (33 * ES + seg_cols<T>()) * (long long)sizeof(cpx<T>) < (1LL << 32) &&
                       table * 6 * (long long)sizeof(cpx<T>) < (1LL << 32);
    c->prof.begin(c->stream, LS_PNAME(T, "fft_z_green"), nrhs, ntab);
    const bool fs = variant == 0 && use_fourstep() && off32;
    switch (L) {
#define CASE(LL)                                                                                              \
    case LL: {                                                                                                \
        const int reg = c->green_half ? try_fs_z<T, LL, true>(c, fs, data, nrhs, CS, RS, ES, ghat, tw)       \
                                      : try_fs_z<T, LL, false>(c, fs, data, nrhs, CS, RS, ES, ghat, tw);     \
        if (reg < 0) return fail(LS_ERR_ARG, "x length not a multiple of the z-pass tile");                  \
        if (reg > 0) break;                                                                                   \
        constexpr int TX = zpass_cols<T, LL>();                                                               \
        if (L1 % TX) return fail(LS_ERR_ARG, "x length not a multiple of the z-pass tile");                   \
        if (c->zbs)                                                                                           \
            launch_lds_z<T, LL, TX, 3>(c, data, nrhs, CS, RS, ES, ghat, tw);                                  \
        else                                                                                                  \
            launch_lds_z<T, LL, TX, 0>(c, data, nrhs, CS, RS, ES, ghat, tw);                                  \
        break;                                                                                                \
    }
        LS_FOR_LENGTHS(CASE)
#undef CASE
        default:
            return fail(LS_ERR_ARG, "unsupported FFT length");
    }
    c->prof.end(c->stream);
    LS_HIP(hipGetLastError());
    return LS_OK;
}

template <typename T>
const cpx<T>* twiddles(const Ctx* c, int L);
template <>
const z128* twiddles<double>(const Ctx* c, int L) { return c->twiddle128(L); }
template <>
const z64* twiddles<float>(const Ctx* c, int L) { return c->twiddle64(L); }

template <typename T>
const cpx<T>* green_table(const Ctx* c, int i);
template <>
const z128* green_table<double>(const Ctx* c, int i) { return c->ghat[i]; }
template <>
const z64* green_table<float>(const Ctx* c, int i) { return c->ghat32[i]; }

template <typename T>
GreenTabs<T> green_tabs(const Ctx* c, const RhsSet& set) {
    GreenTabs<T> g{};
    for (int r = 0; r < set.n; ++r) g.g[r] = green_table<T>(c, set.freq[r]);
    return g;
}

}  // namespace

// the smallest supported length (2^a or 3 * 2^a, 16..512) that holds the linear convolution of n cells
int supported_fft_length(int n) {
    static const int lengths[] = {16, 32, 48, 64, 96, 128, 192, 256, 384, 512};
    for (int L : lengths)
        if (L >= 2 * n - 1) return L;
    return 0;
}

// One pass of the apply (0 x forward, 1 y forward, 2 z with the Green multiply, 3 y inverse,
// 4 x inverse with the epilogue) with kernel variant 0 (register four-step) or 1 (LDS Stockham).
template <typename T>
int run_pass(Ctx* c, int pass, int variant, const RhsSet& set, cpx<T>* work, const cpx<T>* u, cpx<T>* Au,
             bool subtract_from_u) {
    const int N1 = c->n1, N2 = c->n2, N3 = c->n3, L1 = c->L1, L2 = c->L2, L3 = c->L3;
    const int nrhs = set.n;
    const long long rc = 3LL * nrhs;
    const long long lpr = 3LL * N3 * N2;   // x lines per position
    const long long plane = (long long)L2 * L1;
    // work buffer layout (zplane_offset): x lines run over z blocks (stride plane B) and the N2 B data rows of
    // a block (stride L1); y lines over z blocks and the B planes of a block, with elements B L1 apart
    const int zbs = c->zbs, B = 1 << zbs;
    const long long zblock = plane << zbs;
    switch (pass) {
        case 0:  // x forward on the N2 x N3 data lines
            return launch_contig<T, -1, 0, true>(c, L1, work, rc * N3 * N2, N2 * B, zblock, L1, N1, L1,
                                                 twiddles<T>(c, L1), nullptr, nullptr, LS_PNAME(T, "fft_x_fwd"), variant,
                                                 zbs, SlotMap{}, 1, nrhs);
        case 1:  // y forward on all L1 columns of the N3 data planes
            return launch_strided<T, -1, true>(c, L2, work, L1, B, (int)((rc * N3) >> zbs), zblock, L1, (long long)L1 * B,
                                               N2, L2, twiddles<T>(c, L2), LS_PNAME(T, "fft_y_fwd"), variant, nrhs);
        case 2:
            return launch_zgreen<T>(c, work, nrhs, green_tabs<T>(c, set), twiddles<T>(c, L3), variant,
                                    distinct_freqs(set));
        case 3:
            return launch_strided<T, +1, true>(c, L2, work, L1, B, (int)((rc * N3) >> zbs), zblock, L1, (long long)L1 * B,
                                               L2, N2, twiddles<T>(c, L2), LS_PNAME(T, "fft_y_inv"), variant, nrhs);
        default: {
            const SlotMap sm = slot_map(set);
            if (subtract_from_u && c->dot.mode == 1)
                return launch_contig<T, +1, 1, true, 1>(c, L1, work, rc * N3 * N2, N2 * B, zblock, L1, L1, N1,
                                                        twiddles<T>(c, L1), u, Au, LS_PNAME(T, "fft_x_inv_rv"), variant,
                                                        zbs, sm, lpr, nrhs);
            if (subtract_from_u && c->dot.mode == 2)
                return launch_contig<T, +1, 1, true, 2>(c, L1, work, rc * N3 * N2, N2 * B, zblock, L1, L1, N1,
                                                        twiddles<T>(c, L1), u, Au, LS_PNAME(T, "fft_x_inv_ts"), variant,
                                                        zbs, sm, lpr, nrhs);
            if (subtract_from_u)
                return launch_contig<T, +1, 1, true>(c, L1, work, rc * N3 * N2, N2 * B, zblock, L1, L1, N1,
                                                     twiddles<T>(c, L1), u, Au, LS_PNAME(T, "fft_x_inv_epi"), variant,
                                                     zbs, sm, lpr, nrhs);
            return launch_contig<T, +1, 2, true>(c, L1, work, rc * N3 * N2, N2 * B, zblock, L1, L1, N1,
                                                 twiddles<T>(c, L1), u, Au, LS_PNAME(T, "fft_x_inv_conv"), variant, zbs,
                                                 sm, lpr, nrhs);
        }
    }
}

// Right-hand sides per chunk of the x and y passes.  The x pass's output for a chunk is read by the y pass right
// after it; while it fits the device's memory-side cache (256 MiB on MI355X) the y pass reads it from there
// instead of HBM, and the same holds for the y inverse's output read by the x inverse.  Measured on 6-RHS
// applies at 128^3 (x output 101 MB per right-hand side in c64, 201 MB in c128): c64 2.10 -> 2.00 ms with
// chunks of 2 (2.06 ms with 1, 2.04 with 3), c128 4.70 -> 4.43 ms with chunks of 1; chunking the z pass as well
// was slower (2.09 ms), since its Green's table read is shared by the launch's right-hand sides.  A chunk
// larger than the cache gains nothing, so such sizes keep one launch per pass.
constexpr long long kMallBytes = 256ll << 20;
template <typename T>
int xy_chunk_rule(const Ctx* c, int nrhs) {
    const long long per = 3LL * c->n3 * c->n2 * c->L1 * (long long)sizeof(cpx<T>);
    if (per > kMallBytes) return nrhs;
    return (int)std::max(1LL, std::min<long long>(nrhs, kMallBytes / per));
}

// Au = u - Gconv(f) (subtract_from_u) or Au = Gconv(f), where f already sits in work.  The x and y passes run
// per chunk of right-hand-side positions (Ctx::xy_chunk, else xy_chunk_rule), the z pass over all of them.
template <typename T>
int fft_apply_passes(Ctx* c, const RhsSet& set, cpx<T>* work, const cpx<T>* u, cpx<T>* Au, bool subtract_from_u) {
    const int prec = sizeof(T) == 8 ? 0 : 1;
    const int ch = c->xy_chunk[prec] > 0 ? std::min(c->xy_chunk[prec], set.n) : xy_chunk_rule<T>(c, set.n);
    const long long pos = 3LL * c->n3 * c->L2 * c->L1;   // work elements per position
    auto chunk = [&](int a) {
        RhsSet s_;
        s_.n = std::min(ch, set.n - a);
        for (int i = 0; i < s_.n; ++i) s_.slot[i] = set.slot[a + i], s_.freq[i] = set.freq[a + i];
        return s_;
    };
    int rc_;
    for (int a = 0; a < set.n; a += ch) {
        const RhsSet s_ = chunk(a);
        for (int pass = 0; pass < 2; ++pass)
            if ((rc_ = run_pass<T>(c, pass, c->variant[prec][pass], s_, work + a * pos, u, Au, subtract_from_u)))
                return rc_;
    }
    if ((rc_ = run_pass<T>(c, 2, c->variant[prec][2], set, work, u, Au, subtract_from_u))) return rc_;
    for (int a = 0; a < set.n; a += ch) {
        const RhsSet s_ = chunk(a);
        for (int pass = 3; pass < 5; ++pass)
            if ((rc_ = run_pass<T>(c, pass, c->variant[prec][pass], s_, work + a * pos, u, Au, subtract_from_u)))
                return rc_;
    }
    return LS_OK;
}

// Time both kernel variants of every pass at the context's sizes (max_rhs right-hand sides, first
// frequency) and keep the faster; then, over the five passes together, the strided passes' column tiles (256
// or 128 bytes) and the right-hand sides per chunk of the x and y passes (the cache-size rule, 1, 2, 3 or all).
// The work buffer contents are scratch.
template <typename T>
int autotune_passes(Ctx* c) {
    const int prec = sizeof(T) == 8 ? 0 : 1;
    cpx<T>* work = (cpx<T>*)c->work;
    cpx<T>* out = (cpx<T>*)c->gs;
    const RhsSet set = RhsSet::uniform(c->max_rhs, 0);
    hipEvent_t a, b;
    LS_HIP(hipEventCreate(&a));
    LS_HIP(hipEventCreate(&b));
    int rc_ = LS_OK;
    // milliseconds of three runs of fn after one warm-up run
    auto timed = [&](auto fn, float& ms) -> int {
        int r = fn();
        if (r) return r;
        if (hipEventRecord(a, c->stream) != hipSuccess) return fail(LS_ERR_HIP, "autotune event");
        for (int k = 0; k < 3 && r == LS_OK; ++k) r = fn();
        if (r) return r;
        if (hipEventRecord(b, c->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess)
            return fail(LS_ERR_HIP, "autotune timing");
        return LS_OK;
    };
    // the kernel variant of every pass
    for (int pass = 0; pass < 5 && rc_ == LS_OK; ++pass) {
        float best = 0.f;
        for (int variant = 0; variant < 2 && rc_ == LS_OK; ++variant) {
            float ms = 0.f;
            rc_ = timed([&] { return run_pass<T>(c, pass, variant, set, work, out, out, false); }, ms);
            if (rc_ == LS_OK && (variant == 0 || ms < best)) {
                best = ms;
                c->variant[prec][pass] = variant;
            }
        }
    }
    // the strided passes' column tiles, then the chunk of the x and y passes, over all five passes
    auto passes = [&] { return fft_apply_passes<T>(c, set, work, out, out, false); };
    if (rc_ == LS_OK) {
        float ms1 = 0.f, ms0 = 0.f;
        c->y_wide[prec] = 1;
        rc_ = timed(passes, ms1);
        if (rc_ == LS_OK) {
            c->y_wide[prec] = 0;
            rc_ = timed(passes, ms0);
            c->y_wide[prec] = (rc_ == LS_OK && ms0 < ms1) ? 0 : 1;
        }
    }
    if (rc_ == LS_OK) {
        const int cands[] = {xy_chunk_rule<T>(c, set.n), 1, 2, 3, set.n};
        float best = 0.f;
        int pick = 0;
        for (int i = 0; i < 5 && rc_ == LS_OK; ++i) {
            const int ch = std::min(cands[i], set.n);
            bool seen = false;
            for (int k = 0; k < i; ++k) seen = seen || std::min(cands[k], set.n) == ch;
            if (seen) continue;
            c->xy_chunk[prec] = ch;
            float ms = 0.f;
            rc_ = timed(passes, ms);
            if (rc_ == LS_OK && (pick == 0 || ms < best)) {
                best = ms;
                pick = ch;
            }
        }
        c->xy_chunk[prec] = pick;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc_;
}

template int xy_chunk_rule<double>(const Ctx*, int);
template int xy_chunk_rule<float>(const Ctx*, int);
template int autotune_passes<double>(Ctx*);
template int autotune_passes<float>(Ctx*);

// In-place unnormalised forward 3-D FFT of one [L3][L2][L1] array (Green's table setup).
template <typename T>
int fft_full_3d_forward(Ctx* c, cpx<T>* buf) {
    const int L1 = c->L1, L2 = c->L2, L3 = c->L3;
    const long long plane = (long long)L2 * L1;
    int rc_ = launch_contig<T, -1, 0, false>(c, L1, buf, (long long)L3 * L2, L2, plane, L1, L1, L1, twiddles<T>(c, L1),
                                      nullptr, nullptr, "table_fft_x");
    if (rc_) return rc_;
    rc_ = launch_strided<T, -1, false>(c, L2, buf, L1, 1, L3, plane, 0, L1, L2, L2, twiddles<T>(c, L2), "table_fft_y");
    if (rc_) return rc_;
    return launch_strided<T, -1, false>(c, L3, buf, L1, L2, 1, 0, L1, plane, L3, L3, twiddles<T>(c, L3), "table_fft_z");
}

// Blocks per right-hand side of the x-inverse epilogue when the Bi-CGSTAB inner products can be fused
// into it (register four-step variant, whole wavefronts per block, whole blocks per right-hand side),
// else 0.
template <typename T>
int fused_dot_blocks(const Ctx* c) {
    const int prec = sizeof(T) == 8 ? 0 : 1;
    if (c->variant[prec][4] != 0 || !use_fourstep()) return 0;
    bool ok = false;
    switch (c->L1) {
#define CASE(LL)                                                         \
    case LL:                                                             \
        if constexpr (LL == 48 || LL == 96 || LL == 192 || LL == 384)   \
            ok = true;  /* 16 or 32 threads x 128-byte tiles */           \
        else if constexpr (fs_ok<T, LL>())                                \
            ok = fs_threads<T, LL>() % 64 == 0;                           \
        break;
        LS_FOR_LENGTHS(CASE)
#undef CASE
        default:
            ok = false;
    }
    constexpr int TY = seg_cols<T>();
    const long long lines = 3LL * c->n3 * c->n2;
    if (!ok || lines % TY != 0) return 0;
    return (int)(lines / TY);
}

template int fused_dot_blocks<double>(const Ctx*);
template int fused_dot_blocks<float>(const Ctx*);

template int fft_apply_passes<double>(Ctx*, const RhsSet&, z128*, const z128*, z128*, bool);
template int fft_apply_passes<float>(Ctx*, const RhsSet&, z64*, const z64*, z64*, bool);
template int fft_full_3d_forward<double>(Ctx*, z128*);

}  // namespace ls
