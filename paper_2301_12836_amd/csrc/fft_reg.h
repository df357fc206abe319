// Register-resident four-step FFT of one line of length L = N1 * N2 spread over N1 threads.
//
// With n = n1 + N1 n2 and k = k2 + N2 k1 (n1, k1 < N1; n2, k2 < N2):
//   X[k2 + N2 k1] = sum_{n1} W_N1^{n1 k1} W_L^{n1 k2} sum_{n2} W_N2^{n2 k2} x[n1 + N1 n2],
// so each thread q = n1 runs a length-N2 DFT on the elements it holds, applies the twiddles
// W_L^{q k2}, and one transpose through LDS hands every thread the N1 values of M = N2/N1 fixed k2
// for the length-N1 DFTs.  The inverse walks the same steps backwards, so
//   natural layout:  thread q holds x[q + N1 j],              j  < N2
//   spectral layout: thread q holds X[(q + N1 s) + N2 k1]     at v[s N1 + k1], s < M, k1 < N1.
// Columns: TX independent lines side by side (thread index t = tid % TX is the column), so
// global accesses for a fixed element are TX consecutive values.
#pragma once

#include <type_traits>

#include "fft_core.h"

namespace ls {

// cos(2 pi m / 32) for m = 0..8 (first quadrant); the rest by symmetry
constexpr double kCos32[9] = {1.0,
                                                  0.98078528040323044912618223613424,
                                                  0.92387953251128675612818318939679,
                                                  0.83146961230254523707878837761791,
                                                  0.70710678118654752440084436210485,
                                                  0.55557023301960222474283081394853,
                                                  0.38268343236508977172845998403040,
                                                  0.19509032201612826784828486847702,
                                                  0.0};

// e^{SIGN 2 pi i m / N} for N dividing 32, as a compile-time constant
template <int SIGN, int N, typename T>
__device__ __forceinline__ constexpr cpx<T> unit_root(int m) {
    const int q = ((m % N) + N) % N * (32 / N);   // index on the 32-point circle
    double c = 0.0, s = 0.0;
    if (q <= 8) {
        c = kCos32[q];
        s = kCos32[8 - q];
    } else if (q <= 16) {
        c = -kCos32[16 - q];
        s = kCos32[q - 8];
    } else if (q <= 24) {
        c = -kCos32[q - 16];
        s = -kCos32[24 - q];
    } else {
        c = kCos32[32 - q];
        s = -kCos32[q - 24];
    }
    return {T(c), T(SIGN * s)};
}

// In-register DFT of length N (2, 4, 8, 16, 32) with sign SIGN, natural order in and out.  HALF: the
// upper half of the input (v[j], j >= N/2) is zero and is not read; in the split n = a + 4 b every
// length-N/4 column then has the same zero upper half.
template <int SIGN, int N, typename T, bool HALF = false>
__device__ __forceinline__ void reg_dft(cpx<T>* v) {
    if constexpr (N <= 8) {
        if constexpr (HALF)
            SmallDft<SIGN, N, T>::run_half(v);
        else
            SmallDft<SIGN, N, T>::run(v);
    } else {
        constexpr int A = 4, B = N / A;   // n = a + A b, k = k2 + B k1
        cpx<T> tmp[N];
#pragma unroll
        for (int a = 0; a < A; ++a) {
            cpx<T> w[B];
#pragma unroll
            for (int b = 0; b < (HALF ? B / 2 : B); ++b) w[b] = v[a + A * b];
            reg_dft<SIGN, B, T, HALF>(w);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) tmp[a * B + k2] = (a * k2 == 0) ? w[k2] : w[k2] * unit_root<SIGN, N, T>(a * k2);
        }
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) {
            cpx<T> w[A];
#pragma unroll
            for (int a = 0; a < A; ++a) w[a] = tmp[a * B + k2];
            SmallDft<SIGN, A, T>::run(w);
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) v[k2 + B * k1] = w[k1];
        }
    }
}

// cos(2 pi m / 24) for m = 0..6 (first quadrant); with unit_root24 the roots of unity of orders 3, 6, 12, 24
constexpr double kCos24[7] = {1.0,
                              0.96592582628906828674974319972890,
                              0.86602540378443864676372317075294,
                              0.70710678118654752440084436210485,
                              0.5,
                              0.25881904510252076234889883762405,
                              0.0};

// e^{SIGN 2 pi i m / N} for N dividing 24, as a compile-time constant
template <int SIGN, int N, typename T>
__device__ __forceinline__ constexpr cpx<T> unit_root24(int m) {
    const int q = ((m % N) + N) % N * (24 / N);   // index on the 24-point circle
    double c = 0.0, s = 0.0;
    if (q <= 6) {
        c = kCos24[q];
        s = kCos24[6 - q];
    } else if (q <= 12) {
        c = -kCos24[12 - q];
        s = kCos24[q - 6];
    } else if (q <= 18) {
        c = -kCos24[q - 12];
        s = -kCos24[18 - q];
    } else {
        c = kCos24[24 - q];
        s = -kCos24[q - 18];
    }
    return {T(c), T(SIGN * s)};
}

// In-register DFT of length N = 3, 6 or 12 with sign SIGN, natural order in and out: with n = a + 3 b and
// k = k2 + B k1 (B = N / 3), a length-B DFT of each residue a, the twiddles W_N^{a k2}, then length-3 DFTs.
template <int SIGN, int N, typename T>
__device__ __forceinline__ void reg_dft3(cpx<T>* v) {
    if constexpr (N == 3) {
        SmallDft<SIGN, 3, T>::run(v);
    } else {
        constexpr int B = N / 3;
        static_assert(B == 2 || B == 4, "lengths 3, 6, 12");
        cpx<T> tmp[N];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cpx<T> w[B];
#pragma unroll
            for (int b = 0; b < B; ++b) w[b] = v[a + 3 * b];
            SmallDft<SIGN, B, T>::run(w);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2)
                tmp[a * B + k2] = (a * k2 == 0) ? w[k2] : w[k2] * unit_root24<SIGN, N, T>(a * k2);
        }
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) {
            cpx<T> w[3] = {tmp[k2], tmp[B + k2], tmp[2 * B + k2]};
            SmallDft<SIGN, 3, T>::run(w);
#pragma unroll
            for (int k1 = 0; k1 < 3; ++k1) v[k2 + B * k1] = w[k1];
        }
    }
}

template <int L>
struct FourStep {
    static constexpr int N1 = (L == 16) ? 4 : (L == 32) ? 4 : (L == 64) ? 8 : (L == 128) ? 8 : 16;
    static constexpr int N2 = L / N1;
    static constexpr int M = N2 / N1;
    static_assert(N1 * N2 == L && M * N1 == N2 && (M == 1 || M == 2), "unsupported length");
};

// twiddle W_L^{SIGN m} from the table e^{-2 pi i m / L}
template <int SIGN, typename T>
__device__ __forceinline__ cpx<T> tw_at(const cpx<T>* __restrict__ tw, int m) {
    cpx<T> w = tw[m];
    if constexpr (SIGN > 0) w.y = -w.y;
    return w;
}

// LDS slot of row r (the four-step index) of line or column t.  Plain: r TX + t, for kernels whose lanes run
// over t (columns).  SWZ, for kernels whose lanes run over the N1 threads q of a line (64 / N1 lines per
// wavefront): each line's L rows contiguous after a skew of N1 slots per line, with the low log2 N1 bits of the
// row XORed with the next log2 N1, so that the rows one access touches (r = N1 k2 + q when the forward writes,
// r = N1 (q + N1 s) + n1 when it reads, and the inverse's reverse steps) fall in distinct banks (at most two
// to a bank in the inverse's read at lengths 128 and 512).  With the plain padded layout the x passes took 24
// bank-conflict cycles per LDS instruction in FP32 and 10.5 in FP64 at length 256 (SQ_LDS_BANK_CONFLICT).  It
// uses (TX - 1)(L + N1) slots for TX - 1 lines: within the L TX the kernels allocate when (TX - 1) N1 <= L.
template <int L, int TX, bool SWZ>
__device__ __forceinline__ int fs_slot(int r, int t) {
    if constexpr (SWZ) {
        constexpr int N1 = FourStep<L>::N1, S = N1 == 16 ? 4 : N1 == 8 ? 3 : 2;
        static_assert((1 << S) == N1, "power-of-two split");
        return t * (L + N1) + (r & ~(N1 - 1)) + ((r & (N1 - 1)) ^ ((r >> S) & (N1 - 1)));
    } else {
        return r * TX + t;
    }
}

// natural -> spectral, one line per column.  lds: L * TX values, free on entry; free on exit.  HALF:
// the upper half of the line (slots j >= N2/2 of every thread) is zero and is not read.  SWZ: fs_slot.
template <typename T, int L, int TX, int SIGN, bool HALF = false, bool SWZ = false>
__device__ __forceinline__ void fs_forward(cpx<T>* v, cpx<T>* lds, const cpx<T>* __restrict__ tw, int t, int q) {
    using F = FourStep<L>;
    reg_dft<SIGN, F::N2, T, HALF>(v);
#pragma unroll
    for (int k2 = 1; k2 < F::N2; ++k2) v[k2] = v[k2] * tw_at<SIGN>(tw, q * k2);
#pragma unroll
    for (int k2 = 0; k2 < F::N2; ++k2) lds[fs_slot<L, TX, SWZ>(k2 * F::N1 + q, t)] = v[k2];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < F::M; ++s)
#pragma unroll
        for (int n1 = 0; n1 < F::N1; ++n1) v[s * F::N1 + n1] = lds[fs_slot<L, TX, SWZ>((q + F::N1 * s) * F::N1 + n1, t)];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < F::M; ++s) reg_dft<SIGN, F::N1, T>(v + s * F::N1);
}

// spectral -> natural (the reverse steps), same LDS contract.
template <typename T, int L, int TX, int SIGN, bool SWZ = false>
__device__ __forceinline__ void fs_backward(cpx<T>* v, cpx<T>* lds, const cpx<T>* __restrict__ tw, int t, int q) {
    using F = FourStep<L>;
#pragma unroll
    for (int s = 0; s < F::M; ++s) reg_dft<SIGN, F::N1, T>(v + s * F::N1);
#pragma unroll
    for (int s = 0; s < F::M; ++s)
#pragma unroll
        for (int n1 = 1; n1 < F::N1; ++n1)
            v[s * F::N1 + n1] = v[s * F::N1 + n1] * tw_at<SIGN>(tw, n1 * (q + F::N1 * s));
#pragma unroll
    for (int s = 0; s < F::M; ++s)
#pragma unroll
        for (int n1 = 0; n1 < F::N1; ++n1) lds[fs_slot<L, TX, SWZ>(n1 * F::N2 + q + F::N1 * s, t)] = v[s * F::N1 + n1];
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < F::N2; ++k2) v[k2] = lds[fs_slot<L, TX, SWZ>(q * F::N2 + k2, t)];
    __syncthreads();
    reg_dft<SIGN, F::N2, T>(v);
}

// index of the value held in slot i of thread q in the spectral layout
template <int L>
__device__ __forceinline__ int spectral_index(int q, int i) {
    using F = FourStep<L>;
    const int s = i / F::N1, k1 = i % F::N1;
    return (q + F::N1 * s) + F::N2 * k1;
}

// Paired four-step: N1 = 2 N2 threads per line, N2 values each (the same natural layout: thread p holds
// x[p + N1 j]).  It serves the z pass where the square split would hold 32 values of each of three
// components per thread (512 = 32 x 16 instead of 16 x 32).  After the first DFT and the transpose,
// thread p = 2 k2 + h holds the N2 inputs n1 = 2 m + h of the length-N1 DFT for k2 and transforms them;
// the radix-2 step that joins the two halves exchanges values with the partner thread p ^ 1, TX lanes
// away in the same wavefront.  Spectral layout: thread p holds X[k2 + N2 (i + N2 h)] at v[i].  Selections
// between the halves are made per real component (sel): a select of whole structs kept them in scratch.
template <int L>
struct FourStepPair {
    static constexpr int N2 = (L == 512) ? 16 : (L == 128) ? 8 : (L == 32) ? 4 : 0;
    static constexpr int N1 = 2 * N2;
    static_assert(N2 > 0 && N1 * N2 == L, "unsupported length");
};
template <typename T>
__device__ __forceinline__ cpx<T> sel(bool h, cpx<T> a, cpx<T> b) { return {h ? a.x : b.x, h ? a.y : b.y}; }
// The 32-bit value of lane (this lane XOR M) of the wavefront.  M = 1 and M = 8 stay inside a 16-lane row and
// are a DPP modifier on a VALU move (quad_perm [1, 0, 3, 2]; row_ror:8, a rotation by half a row), instead of a
// shuffle through the LDS crossbar (ds_bpermute): FP64 z pass 11.0 -> 8.8 ms at 384 and 21.2 -> 20.2 ms at 512
// (6 right-hand sides).  Other M take the crossbar: for M = 16, gfx950's v_permlane16_swap with a select per
// word measured slower in the FP32 z pass at 512 (9.9 -> 10.5 ms).  Lane layouts checked on the device.
template <int M>
__device__ __forceinline__ unsigned xor_lane_u32(unsigned x) {
    if constexpr (M == 1)
        return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
    else if constexpr (M == 8)
        return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false);
    else
        return (unsigned)__shfl_xor((int)x, M);
}
template <int M>
__device__ __forceinline__ float xor_lane(float x) {
    return __uint_as_float(xor_lane_u32<M>(__float_as_uint(x)));
}
template <int M>
__device__ __forceinline__ double xor_lane(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = xor_lane_u32<M>((unsigned)b), hi = xor_lane_u32<M>((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// the value of lane (this lane XOR M); every lane of the wavefront must take part
template <int M, typename T>
__device__ __forceinline__ cpx<T> lane_xor(cpx<T> a) { return {xor_lane<M>(a.x), xor_lane<M>(a.y)}; }
// the partner's value in the paired split of length L: the DPP exchange from length 384 up; at length 128
// (FP64 at 64^3) the crossbar measured faster (0.216 against 0.225-0.232 ms)
template <int M, int L, typename T>
__device__ __forceinline__ cpx<T> pair_partner(cpx<T> a) {
    if constexpr (L >= 384)
        return lane_xor<M>(a);
    else
        return {__shfl_xor(a.x, M), __shfl_xor(a.y, M)};
}
template <typename T, int L, int TX, int SIGN, bool HALF = false>
__device__ __forceinline__ void fsp_forward(cpx<T>* v, cpx<T>* lds, const cpx<T>* __restrict__ tw, int t, int p) {
    using F = FourStepPair<L>;
    static_assert(2 * TX <= 64, "partner lanes must share a wavefront");
    reg_dft<SIGN, F::N2, T, HALF>(v);
#pragma unroll
    for (int k2 = 1; k2 < F::N2; ++k2) v[k2] = v[k2] * tw_at<SIGN>(tw, p * k2);
#pragma unroll
    for (int k2 = 0; k2 < F::N2; ++k2) lds[(k2 * F::N1 + p) * TX + t] = v[k2];
    __syncthreads();
    const int k2 = p >> 1;
    const bool h = p & 1;
#pragma unroll
    for (int m = 0; m < F::N2; ++m) v[m] = lds[(k2 * F::N1 + 2 * m + (int)h) * TX + t];
    __syncthreads();
    reg_dft<SIGN, F::N2, T>(v);
#pragma unroll
    for (int i = 0; i < F::N2; ++i) {
        cpx<T> mine = v[i];
        if (i > 0) mine = sel(h, mine * tw_at<SIGN>(tw, i * F::N2), mine);
        const cpx<T> other = pair_partner<TX, L>(mine);
        v[i] = sel(h, other - mine, mine + other);
    }
}
template <typename T, int L, int TX, int SIGN>
__device__ __forceinline__ void fsp_backward(cpx<T>* v, cpx<T>* lds, const cpx<T>* __restrict__ tw, int t, int p) {
    using F = FourStepPair<L>;
    const int k2 = p >> 1;
    const bool h = p & 1;
#pragma unroll
    for (int i = 0; i < F::N2; ++i) {
        const cpx<T> mine = v[i];
        const cpx<T> other = pair_partner<TX, L>(mine);
        const cpx<T> d = other - mine;
        const cpx<T> dw = (i > 0) ? d * tw_at<SIGN>(tw, i * F::N2) : d;
        v[i] = sel(h, dw, mine + other);
    }
    reg_dft<SIGN, F::N2, T>(v);
#pragma unroll
    for (int m = 0; m < F::N2; ++m) {
        const int n1 = 2 * m + (int)h;
        lds[(n1 * F::N2 + k2) * TX + t] = v[m] * tw_at<SIGN>(tw, n1 * k2);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < F::N2; ++j) v[j] = lds[(p * F::N2 + j) * TX + t];
    __syncthreads();
    reg_dft<SIGN, F::N2, T>(v);
}
template <int L>
__device__ __forceinline__ int pair_spectral_index(int p, int i) {
    using F = FourStepPair<L>;
    return (p >> 1) + F::N2 * (i + F::N2 * (p & 1));
}
// The split the z pass uses for precision T, length L and table layout: paired at 512 with the octant
// table (with the half-space table the extra index work would spill, so that case keeps the square
// split), and at 128 in FP64 (measured at 64^3: FP64 0.249 -> 0.208 ms per 6-RHS launch, FP32 slower).
template <typename T, int L, bool HALF>
constexpr bool z_paired() {
    return (L == 512 || (L == 128 && sizeof(T) == 8)) && !HALF;
}
template <typename T, int L, bool HALF>
struct ZSplit : std::conditional_t<z_paired<T, L, HALF>(), FourStepPair<L>, FourStep<L>> {};
template <typename T, int L, int TX, int SIGN, bool PAIRED, bool HALF_IN = false>
__device__ __forceinline__ void z_forward(cpx<T>* v, cpx<T>* lds, const cpx<T>* __restrict__ tw, int t, int q) {
    if constexpr (PAIRED)
        fsp_forward<T, L, TX, SIGN, HALF_IN>(v, lds, tw, t, q);
    else
        fs_forward<T, L, TX, SIGN, HALF_IN>(v, lds, tw, t, q);
}
template <typename T, int L, int TX, int SIGN, bool PAIRED>
__device__ __forceinline__ void z_backward(cpx<T>* v, cpx<T>* lds, const cpx<T>* __restrict__ tw, int t, int q) {
    if constexpr (PAIRED)
        fsp_backward<T, L, TX, SIGN>(v, lds, tw, t, q);
    else
        fs_backward<T, L, TX, SIGN>(v, lds, tw, t, q);
}
template <int L, bool PAIRED>
__device__ __forceinline__ int z_spectral_index(int q, int i) {
    if constexpr (PAIRED)
        return pair_spectral_index<L>(q, i);
    else
        return spectral_index<L>(q, i);
}

// XCD-aware block order: hardware hands out workgroups round-robin over the 8 XCDs, so logical
// block b' = (b mod 8) * ceil(nb / 8) + b / 8 gives every XCD one contiguous range of logical
// blocks (neighbours in logical order then share that XCD's L2).  Returns -1 for padding blocks.
__device__ __forceinline__ long long xcd_logical_block(long long b, long long nb_real) {
    const long long per = (nb_real + 7) / 8;
    const long long lb = (b % 8) * per + b / 8;
    return lb < nb_real ? lb : -1;
}

}  // namespace ls
