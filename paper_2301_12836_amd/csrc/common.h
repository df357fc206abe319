// Internal declarations shared by the library's translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ls.h"

namespace ls {

// ------------------------------------------------------------------------------------------
// complex arithmetic on interleaved (re, im) pairs, layout-compatible with complex128/complex64

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};
using z128 = cpx<double>;
using z64 = cpx<float>;

template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.x, -a.y}; }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
    return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}

// Non-temporal access for data a kernel streams once: the caches are left to data that is reused (the
// Green's tables, the contrast shared by neighbouring blocks).
template <typename T>
__device__ __forceinline__ cpx<T> load_nt(const cpx<T>* a) {
    return {__builtin_nontemporal_load(&a->x), __builtin_nontemporal_load(&a->y)};
}
template <typename T>
__device__ __forceinline__ void store_nt(cpx<T>* a, cpx<T> v) {
    __builtin_nontemporal_store(v.x, &a->x);
    __builtin_nontemporal_store(v.y, &a->y);
}

// Padded work buffer [rhs][component][z][y][x] with z planes in blocks of B = 2^zbs interleaved row by row:
// row y of plane z sits at (z / B) L2 B L1 + (y B + z mod B) L1, so the rows of one z block are
// contiguous and a z line spans N3 / B blocks instead of N3 planes (fewer pages per block of the z
// pass).  zbs = 0 is the plain [z][y][x] layout.
__host__ __device__ __forceinline__ long long zplane_offset(int z, int zbs, int L2, int L1) {
    return ((long long)(z >> zbs) * L2 << zbs) * L1 + (long long)(z & ((1 << zbs) - 1)) * L1;
}
__host__ __device__ __forceinline__ long long zrow_offset(int y, int zbs, int L1) {
    return ((long long)y << zbs) * L1;
}

// ------------------------------------------------------------------------------------------
// right-hand sides of one launch

constexpr int kMaxRhs = 64;   // largest batch of right-hand sides a context carries (ls_options.max_rhs)

// The systems one operator launch covers: launch position r (0 <= r < n) works on field slot slot[r] (the
// index into [.][3][N3][N2][N1] field arrays: fields, Krylov vectors, caller buffers) at frequency index
// freq[r]; the padded work buffer holds the positions contiguously.  One launch can so cover any subset
// of a batch (the systems still iterating) at any mix of frequencies, each position computing exactly
// what a launch of it alone computes.
struct RhsSet {
    int n = 0;
    int slot[kMaxRhs] = {};
    int freq[kMaxRhs] = {};
    // positions 0..n-1 on slots 0..n-1, all at one frequency
    static RhsSet uniform(int n, int freq) {
        RhsSet s;
        s.n = n;
        for (int r = 0; r < n && r < kMaxRhs; ++r) s.slot[r] = r, s.freq[r] = freq;
        return s;
    }
};

// per-position data handed to kernels by value (a captured graph records it with the launch)
struct SlotMap {
    int slot[kMaxRhs];
};
// per-position inverse diagonal blocks of the block-Jacobi preconditioner ([9][ncell] of the position's
// frequency; trans: apply the transposed blocks, for the transposed operator)
template <typename T>
struct PreTabs {
    const cpx<T>* m[kMaxRhs];
    int trans;
};
template <typename T>
struct SlotW2 {      // field slot and w^2 of each position (contrast kernels)
    int slot[kMaxRhs];
    T w2[kMaxRhs];
};

inline int distinct_freqs(const RhsSet& s) {
    int d = 0;
    for (int r = 0; r < s.n; ++r) {
        bool seen = false;
        for (int k = 0; k < r && !seen; ++k) seen = s.freq[k] == s.freq[r];
        d += seen ? 0 : 1;
    }
    return d;
}

inline SlotMap slot_map(const RhsSet& s) {
    SlotMap m{};
    for (int r = 0; r < s.n; ++r) m.slot[r] = s.slot[r];
    return m;
}

// ------------------------------------------------------------------------------------------
// error reporting

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define LS_HIP(call)                                         \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return ::ls::hip_fail(e_, #call); \
    } while (0)

// ------------------------------------------------------------------------------------------
// per-kernel event timing (enabled by ls_profile); family names carry the precision
#define LS_PNAME(T, base) (sizeof(T) == 8 ? base ".c128" : base ".c64")

struct Profiler {
    bool on = false;
    static constexpr int kMax = 16384;
    std::vector<hipEvent_t> ev;      // 2 per record
    std::vector<int> fam;            // family index per record
    std::vector<int> rhs, tabs;      // per record: right-hand sides the launch covers, distinct Green's tables it reads
    std::vector<std::string> names;  // family names
    int n = 0;
    int family(const char* name);
    void begin(hipStream_t s, const char* name, int nrhs = 0, int ntab = 0);
    void end(hipStream_t s);
    int open_family = -1, open_rhs = 0, open_tabs = 0;
    ~Profiler();
};

// ------------------------------------------------------------------------------------------
// context

struct Ctx {
    int n1 = 0, n2 = 0, n3 = 0;   // cells per axis (x, y, z)
    int L1 = 0, L2 = 0, L3 = 0;   // FFT lengths per axis (>= 2n - 1, supported sizes)
    int zbs = 0;                  // log2 of the z planes interleaved per block of the padded work buffer (below)
    long long ncell = 0;
    double h = 0;
    int mixed = 0;
    int green_mode = LS_GREEN_EXACT;
    bool green_half = false;      // k-space table over the half-space k_x <= L1/2 (backgrounds without the
                                  // three coordinate mirror planes) instead of the octant
    int max_rhs = 1;
    double rho0 = 0, alpha = 0, beta = 0;
    double fold21[21] = {0};      // C0 - C_iso, packed, added to every cell's contrast (zero for LS_GREEN_ANISO)
    double C0[36] = {0};          // background stiffness as given
    std::vector<double> omega;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;  // created when the caller passes the null stream (a blocking stream,
                                       // so it stays ordered with work on the legacy default stream)
    int flags = 0;
    int num_cu = 256;  // compute units of the device (block-count heuristics)
    int device = 0;    // the HIP device the context was set up on
    int taper = 0;     // absorbing-layer thickness in cells (0: off)
    int launch_rhs = 0;  // most systems one operator launch of a solve covers (0: all of them)
    int precond = 0;     // LS_PRECOND_*: preconditioner of the Bi-CGSTAB solves
    // FFT kernel variant per pass and precision: 0 register four-step, 1 LDS Stockham
    // passes: 0 x forward, 1 y forward, 2 z with Green multiply, 3 y inverse, 4 x inverse
    int variant[2][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
    // per precision (0 c128, 1 c64): right-hand sides per chunk of the x and y passes (0: the cache-size rule),
    // and whether the strided passes take 256-byte column tiles where the x length allows (1) or 128-byte ones
    int xy_chunk[2] = {0, 0};
    int y_wide[2] = {1, 1};

    // medium (folded contrast), FP64 and (mixed) FP32
    double* dc = nullptr;     // [21][ncell]
    double* drho = nullptr;   // [ncell]
    float* dc32 = nullptr;
    float* drho32 = nullptr;
    // the same contrast packed tile by tile for the fused contrast kernel (contrast_packed_elems): the 21
    // values of the cells of one xy tile on one z plane are contiguous, so a block reads one run per plane
    double* dcp = nullptr;
    float* dcp32 = nullptr;
    // values per cell in the packed copy: 9 when every cell's contrast has the orthotropic pattern (nonzero
    // only at 11, 12, 13, 22, 23, 33, 44, 55, 66: isotropic, VTI and orthorhombic media in the grid axes),
    // else 21
    int contrast_k = 21;

    // k-space Green's tables per frequency: octant [L3/2+1][L2/2+1][L1/2+1][6] (half-space
    // [L3][L2][L1/2+1][6] when green_half), already scaled by 1/(L1 L2 L3) so the inverse FFT needs no
    // normalisation
    std::vector<z128*> ghat;
    std::vector<z128*> greal;     // LS_GREEN_ANISO: h^3 G at the offsets of one octant, [N3][N2][N1][6] per frequency
                                  // (half-space: [2 N3 - 1][2 N2 - 1][N1][6])
    std::vector<z64*> ghat32;
    double* gl_nodes = nullptr;   // LS_GREEN_ANISO: Gauss-Legendre nodes and weights on [0, 1] (device)
    // block-Jacobi preconditioner (LS_PRECOND_BLOCK_JACOBI): inverse diagonal 3x3 blocks per frequency,
    // entry (a, b) of cell p at [(3 a + b) ncell + p], FP64 and (mixed) FP32; h^3 G at the offsets [-2, 2]^3
    // while they are built ([125][6])
    std::vector<z128*> minv;
    std::vector<z64*> minv32;
    z128* gloc = nullptr;

    // twiddle tables e^{-2 pi i m / L}, m < L, per distinct length
    std::vector<int> tw_len;
    std::vector<z128*> tw128;
    std::vector<z64*> tw64;

    // workspaces
    void* work = nullptr;       // padded FFT buffer [max_rhs][3][N3][L2][L1] (c128 size)
    void* tau = nullptr;        // Voigt stress scratch [max_rhs][6][ncell] (c128 size), split contrast only
    // Krylov vectors, c128 [max_rhs][3][ncell] each
    z128 *r = nullptr, *rhat = nullptr, *p = nullptr, *v = nullptr, *s = nullptr, *t = nullptr;
    z128 *xd = nullptr, *bd = nullptr;           // FP64 iterate / rhs copies for refinement
    z128 *ph = nullptr, *sh = nullptr;           // preconditioned directions M^-1 p, M^-1 s (block Jacobi only)
    z128* xbest = nullptr;       // best iterate of the FP64 solves [max_rhs][3][ncell]
    void* gs = nullptr;          // Gconv y scratch of the transposed operator [max_rhs][3][ncell] (c128 size)
    // c64 Krylov vectors for the inner solve of the mixed path
    z64 *r32 = nullptr, *rhat32 = nullptr, *p32 = nullptr, *v32 = nullptr, *s32 = nullptr, *t32 = nullptr,
        *x32 = nullptr, *b32 = nullptr;
    z64 *ph32 = nullptr, *sh32 = nullptr;
    double* partials = nullptr;  // reduction partials [max_rhs][kRedSlots][kRedBlocks]
    double* state = nullptr;     // BiCGSTAB scalars per right-hand side [max_rhs][kStateLen]
    void* stage = nullptr;       // small host/device staging area (8 KB)
    int* ints = nullptr;          // device staging for receiver lists and frequency indices (grown on demand)
    int ints_cap = 0;
    std::vector<std::vector<double>> history;  // per right-hand side: relative residual after each iteration of the last solve
    z128 *batch_b = nullptr, *batch_x = nullptr;  // [max_rhs][3][n] right-hand sides / solutions of ls_solve_batch (allocated on its first use)
    int bicgstab_l = 1;          // Krylov method: 1 Bi-CGSTAB (graph-captured), 2..4 BiCGSTAB(l)
    double* gpart = nullptr;     // BiCGSTAB(l) reduction partials [max_rhs][slots][kRedBlocks]
    std::vector<void*> kry128, kry64;  // BiCGSTAB(l) vectors beyond the six of Bi-CGSTAB, per precision
    // inner products fused into the x-inverse epilogue of the next forward operator application:
    // mode 1 = a^H (u - v), mode 2 = (u - v)^H u and ||u - v||^2; set by the solver around the call
    struct DotRequest {
        int mode = 0;
        const void* a = nullptr;
        double* parts = nullptr;
        long long lines = 1;   // x lines per right-hand side
        int nparts = 0;        // epilogue blocks per right-hand side
    } dot;
    double* dparts = nullptr;    // partials of the fused inner products [max_rhs][kRedSlots][blocks per RHS]
    double* red = nullptr;       // reduction results (device)
    double* red_host = nullptr;  // pinned host mirror
    long long bytes = 0;
    Profiler prof;

    const z128* twiddle128(int L) const;
    const z64* twiddle64(int L) const;
    size_t field_elems() const { return (size_t)3 * (size_t)ncell; }
};

// device allocation tracked in ctx->bytes
int dalloc(Ctx* c, void** p, size_t bytes);

// ------------------------------------------------------------------------------------------
// host launchers (each returns LS_OK or an error code)

// FFT passes over the padded buffer (positions of the set) ending in the compact fields Au (slots); see fft.hip
template <typename T>
int fft_apply_passes(Ctx* c, const RhsSet& set, cpx<T>* work, const cpx<T>* u, cpx<T>* Au, bool subtract_from_u);
template <typename T>
int fft_full_3d_forward(Ctx* c, cpx<T>* buf);
template <typename T>
int fused_dot_blocks(const Ctx* c);  // epilogue blocks per right-hand side if the dots can be fused, else 0
// right-hand sides per chunk of the x and y passes by the memory-side cache size (used when Ctx::xy_chunk is 0)
template <typename T>
int xy_chunk_rule(const Ctx* c, int nrhs);
template <typename T>
int autotune_passes(Ctx* c);
int supported_fft_length(int n);

// contrast kernels; see contrast.hip (fields indexed by slot, work and tau by position)
template <typename T>
int contrast_to_work(Ctx* c, const RhsSet& set, const cpx<T>* u, cpx<T>* work, cpx<T>* tau);
template <typename T>
int contrast_transposed_epilogue(Ctx* c, const RhsSet& set, const cpx<T>* g, const cpx<T>* y, cpx<T>* out,
                                 cpx<T>* tau);
template <typename T>
int to_work(Ctx* c, const RhsSet& set, const cpx<T>* f, cpx<T>* work);
int grad_contrast_launch(Ctx* c, int i_omega, const z128* u, const z128* mu, int nrhs, double* g21, double* grho);
int fold_background(Ctx* c, const double* dc_in, const double* drho_in, const double fold21[21]);
size_t contrast_packed_elems(const Ctx* c, bool fp32);   // elements of dcp (fp32 false) or dcp32
bool use_fused_contrast();  // false under LS_CONTRAST=split (the two-kernel contrast, which needs tau)
int conj_launch(Ctx* c, z128* a, long long m);
int sample_launch(Ctx* c, const z128* u, int nrhs, const int* rec_host, int nrec, z128* out);
int synthesize_launch(Ctx* c, const z128* U, const int* k_host, int nf, int ntr, int nt, double dt, double fp,
                      double ts, double* traces);
int grad_moment_launch(Ctx* c, int i_omega, const z128* mu, int nrhs, const int* src, const double* t0,
                       double* gM);
int strain_launch(Ctx* c, const z128* u, z128* eps, int nrhs);

// Green's tables and incident fields; see green.hip
int build_green_tables(Ctx* c);
int rhs_points_launch(Ctx* c, int i_omega, const int* cells, const double* forces, int npts, double t0,
                      z128* b);
int local_green_table(Ctx* c, int i_omega, z128* out);  // h^3 G at the offsets [-2, 2]^3, [125][6]

// block-Jacobi preconditioner; see precond.hip
int build_block_jacobi(Ctx* c);

// the LS matvec Au = u - Gconv B u, its transpose A^T y = y - B Gconv y, and Gconv f, for the systems of a
// set (fields indexed by slot); see capi.hip
template <typename T>
int apply_op(Ctx* c, const RhsSet& set, const cpx<T>* u, cpx<T>* Au);
template <typename T>
int apply_T_op(Ctx* c, const RhsSet& set, const cpx<T>* y, cpx<T>* ATy);
template <typename T>
int convolve_op(Ctx* c, const RhsSet& set, const cpx<T>* f, cpx<T>* out);

// solver (BiCGSTAB, mixed-precision refinement); see solver.hip.  System q (0 <= q < nrhs) is slot q of b,
// x0 and u_out, at frequency index freq[q].
int krylov_setup(Ctx* c);  // allocates what BiCGSTAB(l) needs beyond Bi-CGSTAB (called by ls_setup)
int solve_systems(Ctx* c, const int* freq, const z128* b, int nrhs, double tol, int maxit, int precision,
                  const z128* x0, z128* u_out, ls_info* info, bool transposed = false);

constexpr int kRedBlocks = 1024;  // fixed partial count: reductions are deterministic
constexpr int kRedSlots = 4;      // partial sums per right-hand side and pass
constexpr int kStateLen = 16;

}  // namespace ls
