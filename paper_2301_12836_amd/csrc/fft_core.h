// Device building blocks of the Stockham FFT used for the zero-padded convolutions of Eq 21.
//
// Lines of length L (2^a or 3 * 2^a) are held in LDS as s[e * LDP + t] (element e of line t,
// line index fastest).  Each stage reads R elements spaced L/R apart, applies the twiddles
// W_{Ns R}^{r k} (k = j mod Ns), a radix-R DFT in registers, and writes them back spaced Ns
// apart from (j / Ns) Ns R + k: the self-sorting (Stockham) form, so no bit reversal is needed.
// SIGN = -1 is the forward transform sum_n x_n e^{-2 pi i n k / L}, SIGN = +1 the unscaled inverse.
#pragma once

#include "common.h"

namespace ls {

template <int SIGN, typename T>
__device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {  // a * (SIGN * i)
    if constexpr (SIGN < 0)
        return {a.y, -a.x};
    else
        return {-a.y, a.x};
}

template <int SIGN, int R, typename T>
struct SmallDft;

// run_half (lengths 2, 4, 8): the same DFT when the upper half of the input (v[j], j >= R/2) is known
// to be zero; those elements are not read.
template <int SIGN, typename T>
struct SmallDft<SIGN, 2, T> {
    static __device__ __forceinline__ void run(cpx<T>* v) {
        const cpx<T> a = v[0];
        v[0] = a + v[1];
        v[1] = a - v[1];
    }
    static __device__ __forceinline__ void run_half(cpx<T>* v) { v[1] = v[0]; }
};

// X1,2 = a - (b + c)/2 +- SIGN i (sqrt(3)/2)(b - c)  (the cube roots of unity e^{SIGN 2 pi i/3})
template <int SIGN, typename T>
struct SmallDft<SIGN, 3, T> {
    static __device__ __forceinline__ void run(cpx<T>* v) {
        const cpx<T> t1 = v[1] + v[2];
        const cpx<T> t2 = v[0] - T(0.5) * t1;
        const cpx<T> t3 = mul_si<SIGN>(T(0.86602540378443864676) * (v[1] - v[2]));
        v[0] = v[0] + t1;
        v[1] = t2 + t3;
        v[2] = t2 - t3;
    }
};

template <int SIGN, typename T>
struct SmallDft<SIGN, 4, T> {
    static __device__ __forceinline__ void run(cpx<T>* v) {
        const cpx<T> t0 = v[0] + v[2], t1 = v[0] - v[2], t2 = v[1] + v[3];
        const cpx<T> t3 = mul_si<SIGN>(v[1] - v[3]);
        v[0] = t0 + t2;
        v[2] = t0 - t2;
        v[1] = t1 + t3;
        v[3] = t1 - t3;
    }
    static __device__ __forceinline__ void run_half(cpx<T>* v) {
        const cpx<T> a = v[0], b = v[1], sb = mul_si<SIGN>(v[1]);
        v[0] = a + b;
        v[2] = a - b;
        v[1] = a + sb;
        v[3] = a - sb;
    }
};

template <int SIGN, typename T>
struct SmallDft<SIGN, 8, T> {
    static __device__ __forceinline__ void run(cpx<T>* v) {
        cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
        SmallDft<SIGN, 4, T>::run(e);
        SmallDft<SIGN, 4, T>::run(o);
        combine(e, o, v);
    }
    static __device__ __forceinline__ void run_half(cpx<T>* v) {
        cpx<T> e[4] = {v[0], v[2]};
        cpx<T> o[4] = {v[1], v[3]};
        SmallDft<SIGN, 4, T>::run_half(e);
        SmallDft<SIGN, 4, T>::run_half(o);
        combine(e, o, v);
    }
    // v = the length-8 DFT from the length-4 DFTs of the even (e) and odd (o) elements
    static __device__ __forceinline__ void combine(const cpx<T>* e, const cpx<T>* o, cpx<T>* v) {
        const T r = T(0.70710678118654752440);
        const T s = T(SIGN);
        // W8 = (1 + SIGN i)/sqrt(2);  W8^2 = SIGN i;  W8^3 = W8^2 W8
        const cpx<T> o1 = {r * (o[1].x - s * o[1].y), r * (o[1].y + s * o[1].x)};
        const cpx<T> o2 = mul_si<SIGN>(o[2]);
        const cpx<T> o3 = mul_si<SIGN>(cpx<T>{r * (o[3].x - s * o[3].y), r * (o[3].y + s * o[3].x)});
        v[0] = e[0] + o[0];
        v[4] = e[0] - o[0];
        v[1] = e[1] + o1;
        v[5] = e[1] - o1;
        v[2] = e[2] + o2;
        v[6] = e[2] - o2;
        v[3] = e[3] + o3;
        v[7] = e[3] - o3;
    }
};

// the factor 3 first (at NS = 1 it needs no twiddles), then 8, 4, 2
template <int REM>
constexpr int pick_radix() {
    return (REM % 3 == 0) ? 3 : (REM % 8 == 0 && REM != 16) ? 8 : ((REM % 4 == 0) ? 4 : 2);
}

// One Stockham stage over NL lines of length L in LDS (leading dimension LDP), NT threads.
// Callers synchronise before the first stage; each stage ends with a barrier.
template <typename T, int L, int NL, int LDP, int NT, int SIGN, int NS, int R>
__device__ __forceinline__ void fft_stage(cpx<T>* s, const cpx<T>* __restrict__ tw, int tid) {
    constexpr int NB = NL * (L / R);
    constexpr int PER = (NB + NT - 1) / NT;
    cpx<T> v[PER][R];
#pragma unroll
    for (int it = 0; it < PER; ++it) {
        const int b = tid + it * NT;
        if (NB % NT == 0 || b < NB) {
            const int t = b % NL, j = b / NL;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = s[(j + r * (L / R)) * LDP + t];
            if constexpr (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cpx<T> w = tw[r * k * (L / (NS * R))];
                    if constexpr (SIGN > 0) w.y = -w.y;
                    v[it][r] = v[it][r] * w;
                }
            }
            SmallDft<SIGN, R, T>::run(v[it]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PER; ++it) {
        const int b = tid + it * NT;
        if (NB % NT == 0 || b < NB) {
            const int t = b % NL, j = b / NL;
            const int d = (j / NS) * NS * R + (j % NS);
#pragma unroll
            for (int r = 0; r < R; ++r) s[(d + r * NS) * LDP + t] = v[it][r];
        }
    }
    __syncthreads();
}

template <typename T, int L, int NL, int LDP, int NT, int SIGN, int NS = 1>
__device__ __forceinline__ void lds_fft(cpx<T>* s, const cpx<T>* __restrict__ tw, int tid) {
    if constexpr (NS < L) {
        constexpr int R = pick_radix<L / NS>();
        fft_stage<T, L, NL, LDP, NT, SIGN, NS, R>(s, tw, tid);
        lds_fft<T, L, NL, LDP, NT, SIGN, NS * R>(s, tw, tid);
    }
}

}  // namespace ls
