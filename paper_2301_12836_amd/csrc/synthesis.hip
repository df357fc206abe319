// Time-domain seismograms from the frequency-domain solutions: receiver sampling of solved fields and the
// inverse Fourier transform over the solved frequencies (the paper's frequency loop up to Nyquist followed
// by an inverse transform; Ricker source wavelet of its Tables 1 and 3).
//
// Conventions: time dependence e^{-i w t}, spectra S(w) = int s(t) e^{i w t} dt; a real medium gives
// u(-w) = conj u(w), so only w_k = 2 pi k / (nt dt) >= 0 is solved and
//   u(t_n) = (1/(nt dt)) sum_k c_k Re[S(w_k) U_k e^{-i w_k t_n}],  c_k = 1 for k = 0 or 2k = nt, else 2.
#include <cmath>

#include "common.h"

namespace ls {

namespace {

// out[r][m][c] = u[r][c][cell_m]
__global__ void k_sample(const z128* __restrict__ u, const int* __restrict__ rec, z128* __restrict__ out, int nrhs,
                         int nrec, int N1, int N2, int N3) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)nrhs * nrec * 3) return;
    const int c = (int)(q % 3), m = (int)((q / 3) % nrec), r = (int)(q / (3LL * nrec));
    const long long n = (long long)N1 * N2 * N3;
    const long long p = ((long long)rec[3 * m + 2] * N2 + rec[3 * m + 1]) * N1 + rec[3 * m];
    out[q] = u[((long long)r * 3 + c) * n + p];
}

// wavelet factor of each solved frequency: c_k S(w_k) / (nt dt), S the delayed Ricker spectrum
// (4 sqrt(pi) w^2 / wp^3) e^{-w^2/wp^2} e^{i w ts} (fp > 0) or 1 (fp <= 0: the traces of the fields)
__global__ void k_wavelet(const int* __restrict__ k, int nf, int nt, double dt, double fp, double ts,
                          z128* __restrict__ s) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nf) return;
    const double scale = ((k[q] == 0 || 2 * k[q] == nt) ? 1.0 : 2.0) / (nt * dt);
    if (fp <= 0.0) {
        s[q] = {scale, 0.0};
        return;
    }
    const double w = 2.0 * M_PI * k[q] / (nt * dt), wp = 2.0 * M_PI * fp;
    const double amp = scale * 4.0 * sqrt(M_PI) * w * w / (wp * wp * wp) * exp(-(w / wp) * (w / wp));
    double sn, cs;
    sincos(w * ts, &sn, &cs);
    s[q] = {amp * cs, amp * sn};
}

// traces[j][n] = sum_q Re[s_q U[q][j] e^{-2 pi i (k_q n mod nt) / nt}]
__global__ void k_traces(const z128* __restrict__ U, const z128* __restrict__ s, const int* __restrict__ k, int nf,
                         int ntr, int nt, double* __restrict__ tr) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long long)ntr * nt) return;
    const int n = (int)(q % nt), j = (int)(q / nt);
    double acc = 0.0;
    for (int f = 0; f < nf; ++f) {
        const z128 a = U[(long long)f * ntr + j] * s[f];
        const long long kn = ((long long)k[f] * n) % nt;
        double sn, cs;
        sincospi(2.0 * (double)kn / nt, &sn, &cs);
        acc += a.x * cs + a.y * sn;   // Re[a (cs - i sn)]
    }
    tr[q] = acc;
}

int ensure_ints(Ctx* c, int count) {
    if (count <= c->ints_cap) return LS_OK;
    if (c->ints) LS_HIP(hipFree(c->ints));
    c->ints = nullptr;
    c->ints_cap = 0;
    LS_HIP(hipMalloc((void**)&c->ints, sizeof(int) * (size_t)count));
    c->ints_cap = count;
    return LS_OK;
}

}  // namespace

int sample_launch(Ctx* c, const z128* u, int nrhs, const int* rec_host, int nrec, z128* out) {
    int rc = ensure_ints(c, 3 * nrec);
    if (rc) return rc;
    LS_HIP(hipMemcpyAsync(c->ints, rec_host, sizeof(int) * 3 * (size_t)nrec, hipMemcpyHostToDevice, c->stream));
    const long long m = (long long)nrhs * nrec * 3;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, c->stream, u, c->ints, out, nrhs, nrec,
                       c->n1, c->n2, c->n3);
    LS_HIP(hipGetLastError());
    LS_HIP(hipStreamSynchronize(c->stream));  // the staged receiver list may be replaced by the next call
    return LS_OK;
}

int synthesize_launch(Ctx* c, const z128* U, const int* k_host, int nf, int ntr, int nt, double dt, double fp, double ts,
                      double* traces) {
    // staging: k [nf] ints, then the nf complex wavelet factors (16-byte aligned)
    const int kints = (nf + 3) / 4 * 4;
    int rc = ensure_ints(c, kints + 4 * nf);
    if (rc) return rc;
    int* dk = c->ints;
    z128* ds = (z128*)(c->ints + kints);
    LS_HIP(hipMemcpyAsync(dk, k_host, sizeof(int) * (size_t)nf, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_wavelet, dim3((unsigned)((nf + 63) / 64)), dim3(64), 0, c->stream, dk, nf, nt, dt, fp, ts, ds);
    LS_HIP(hipGetLastError());
    const long long m = (long long)ntr * nt;
    hipLaunchKernelGGL(k_traces, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, c->stream, U, ds, dk, nf, ntr, nt,
                       traces);
    LS_HIP(hipGetLastError());
    LS_HIP(hipStreamSynchronize(c->stream));
    return LS_OK;
}

}  // namespace ls
