// C ABI of the LS solver library: context set-up, the matvec pipeline, incident fields, solves,
// profiling.  See include/ls.h for the contract of every entry point.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <sys/stat.h>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "common.h"

struct ls_ctx : public ls::Ctx {};

namespace ls {

// ------------------------------------------------------------------------------------------
// errors

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return LS_ERR_HIP;
}

// ------------------------------------------------------------------------------------------
// profiler

int Profiler::family(const char* name) {
    for (size_t i = 0; i < names.size(); ++i)
        if (names[i] == name) return (int)i;
    names.emplace_back(name);
    return (int)names.size() - 1;
}

void Profiler::begin(hipStream_t s, const char* name, int nrhs, int ntab) {
    open_family = -1;
    if (!on || n >= kMax) return;
    open_family = family(name);
    open_rhs = nrhs;
    open_tabs = ntab;
    (void)hipEventRecord(ev[2 * n], s);
}

void Profiler::end(hipStream_t s) {
    if (open_family < 0) return;
    (void)hipEventRecord(ev[2 * n + 1], s);
    fam[n] = open_family;
    rhs[n] = open_rhs;
    tabs[n] = open_tabs;
    ++n;
    open_family = -1;
}

Profiler::~Profiler() {
    for (auto& e : ev) (void)hipEventDestroy(e);
}

// ------------------------------------------------------------------------------------------
// context helpers

int dalloc(Ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return LS_OK;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(LS_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    c->bytes += (long long)bytes;
    return LS_OK;
}

const z128* Ctx::twiddle128(int L) const {
    for (size_t i = 0; i < tw_len.size(); ++i)
        if (tw_len[i] == L) return tw128[i];
    return nullptr;
}

const z64* Ctx::twiddle64(int L) const {
    for (size_t i = 0; i < tw_len.size(); ++i)
        if (tw_len[i] == L) return tw64[i];
    return nullptr;
}

static void release(Ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    void* ptrs[] = {c->dc, c->drho, c->dc32, c->drho32, c->work, c->tau, c->r, c->rhat, c->p, c->v, c->s, c->t,
                    c->xd, c->bd, c->gs, c->r32, c->rhat32, c->p32, c->v32, c->s32, c->t32, c->x32, c->b32, c->partials,
                    c->state, c->stage, c->red, c->batch_b, c->batch_x, c->ints, c->gl_nodes, c->gpart, c->xbest, c->dparts,
                    c->gloc, c->ph, c->sh, c->ph32, c->sh32, c->dcp, c->dcp32};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    for (auto q : c->ghat) (void)hipFree(q);
    for (auto q : c->greal) (void)hipFree(q);
    for (auto q : c->kry128) (void)hipFree(q);
    for (auto q : c->kry64) (void)hipFree(q);
    for (auto q : c->ghat32) (void)hipFree(q);
    for (auto q : c->minv) (void)hipFree(q);
    for (auto q : c->minv32) (void)hipFree(q);
    for (auto q : c->tw128) (void)hipFree(q);
    for (auto q : c->tw64) (void)hipFree(q);
    if (c->red_host) (void)hipHostFree(c->red_host);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete static_cast<ls_ctx*>(c);
}

// ------------------------------------------------------------------------------------------
// the matvec

// work: the padded FFT buffer (set.n x 3 N3 L2 L1 values); tau: the stress scratch of the split contrast.
// Every value of work that a pass reads was written earlier in the same call, so it needs no clearing.
template <typename T>
int apply_op_in(Ctx* c, const RhsSet& set, const cpx<T>* u, cpx<T>* Au, cpx<T>* work, cpx<T>* tau) {
    int rc = contrast_to_work<T>(c, set, u, work, tau);
    if (rc) return rc;
    return fft_apply_passes<T>(c, set, work, u, Au, true);
}

template <typename T>
int apply_op(Ctx* c, const RhsSet& set, const cpx<T>* u, cpx<T>* Au) {
    return apply_op_in<T>(c, set, u, Au, (cpx<T>*)c->work, (cpx<T>*)c->tau);
}

template int apply_op<double>(Ctx*, const RhsSet&, const z128*, z128*);
template int apply_op<float>(Ctx*, const RhsSet&, const z64*, z64*);

// A^T y = y - B (Gconv y): Gconv and B are both symmetric, so the transpose applies the Green's
// convolution first and the contrast second
template <typename T>
int apply_T_op(Ctx* c, const RhsSet& set, const cpx<T>* y, cpx<T>* ATy) {
    cpx<T>* work = (cpx<T>*)c->work;
    cpx<T>* g = (cpx<T>*)c->gs;
    int rc = to_work<T>(c, set, y, work);
    if (rc) return rc;
    rc = fft_apply_passes<T>(c, set, work, nullptr, g, false);
    if (rc) return rc;
    return contrast_transposed_epilogue<T>(c, set, g, y, ATy, (cpx<T>*)c->tau);
}

template <typename T>
int convolve_op(Ctx* c, const RhsSet& set, const cpx<T>* f, cpx<T>* out) {
    int rc = to_work<T>(c, set, f, (cpx<T>*)c->work);
    if (rc) return rc;
    return fft_apply_passes<T>(c, set, (cpx<T>*)c->work, nullptr, out, false);
}

template int apply_T_op<double>(Ctx*, const RhsSet&, const z128*, z128*);
template int apply_T_op<float>(Ctx*, const RhsSet&, const z64*, z64*);
template int convolve_op<double>(Ctx*, const RhsSet&, const z128*, z128*);

// ------------------------------------------------------------------------------------------
// Allocation-free apply (ls_apply_noalloc): its padded work buffer is this file-scope device array, of
// which every GPU the library runs on holds its own copy until the process ends.  In host code the name
// `scratch` is only a stand-in for the symbol: its device address is looked up once per device
// (scratch_setup, called by ls_setup with the context's device current) and only that address is used.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Look up this device's copy of the array (once per device); the device must be current.
int scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(LS_ERR_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return LS_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(LS_ERR_HIP, std::string("scratch address lookup failed: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = ptr;
    return LS_OK;
}

void* scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_ptr[device];
}

}  // namespace ls

using namespace ls;

namespace {

int check_ctx(const ls_ctx* c) {
    if (!c) return fail(LS_ERR_ARG, "null context");
    return LS_OK;
}

int check_omega(const ls_ctx* c, int i) {
    if (i < 0 || i >= (int)c->omega.size()) return fail(LS_ERR_ARG, "frequency index out of range");
    return LS_OK;
}

int check_cell(const ls_ctx* c, const int* cell) {
    if (!cell) return fail(LS_ERR_ARG, "null cell index");
    const int n[3] = {c->n1, c->n2, c->n3};
    for (int a = 0; a < 3; ++a)
        if (cell[a] < 0 || cell[a] >= n[a]) return fail(LS_ERR_ARG, "cell index outside the grid");
    return LS_OK;
}

// the byte ranges [a, a + na) and [b, b + nb) intersect
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

// in and out of a field-to-field call (n_rhs fields of elem bytes per complex value) must be disjoint
int check_disjoint(const ls_ctx* c, const void* in, const void* out, int n_rhs, size_t elem, const char* what) {
    const size_t bytes = (size_t)n_rhs * c->field_elems() * elem;
    if (overlaps(in, bytes, out, bytes)) return fail(LS_ERR_ARG, std::string(what) + ": input and output overlap");
    return LS_OK;
}

// solves: b and u_out disjoint; x0 either u_out itself (an in-place warm start) or disjoint from it
int check_solve_buffers(const ls_ctx* c, const void* b, const void* x0, const void* u_out, int n_rhs) {
    int rc;
    if ((rc = check_disjoint(c, b, u_out, n_rhs, sizeof(z128), "solve (b, u_out)"))) return rc;
    if (x0 && x0 != u_out) {
        if ((rc = check_disjoint(c, x0, u_out, n_rhs, sizeof(z128), "solve (x0, u_out)"))) return rc;
    }
    return LS_OK;
}

// ------------------------------------------------------------------------------------------
// autotuner cache: one line per tuned configuration, "key v0 .. v9 c0 c1 w0 w1" (the FFT variant of every pass
// and precision, then per precision the right-hand sides per chunk of the x and y passes and the strided
// passes' tile choice), in the file LS_AUTOTUNE_CACHE names, else $HOME/.cache/lsvie/autotune.txt.  A missing
// or unreadable cache only means tuning again; a later line for the same key wins; lines of other formats
// (an older key version) are skipped.

std::string autotune_path() {
    if (const char* e = std::getenv("LS_AUTOTUNE_CACHE")) return e;
    const char* home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/lsvie/autotune.txt";
}

// everything the timings depend on: device, grid, FFT lengths, batch width, layout, table kind, precision
std::string autotune_key(const Ctx* c) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
    (void)hipGetLastError();
    for (char& ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    return "v2:" + arch + ":cu" + std::to_string(c->num_cu) + ":n" + std::to_string(c->n1) + "x" + std::to_string(c->n2) +
           "x" + std::to_string(c->n3) + ":L" + std::to_string(c->L1) + "x" + std::to_string(c->L2) + "x" +
           std::to_string(c->L3) + ":r" + std::to_string(c->max_rhs) + ":z" + std::to_string(c->zbs) + ":h" +
           std::to_string((int)c->green_half) + ":m" + std::to_string(c->mixed);
}

bool autotune_lookup(const std::string& key, Ctx* c) {
    FILE* f = std::fopen(autotune_path().c_str(), "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    int v[14];
    while (std::fgets(line, sizeof line, f)) {
        char k[400];
        int w[14];
        if (std::sscanf(line, "%399s %d %d %d %d %d %d %d %d %d %d %d %d %d %d", k, &w[0], &w[1], &w[2], &w[3], &w[4],
                        &w[5], &w[6], &w[7], &w[8], &w[9], &w[10], &w[11], &w[12], &w[13]) != 15 ||
            key != k)
            continue;
        bool ok = true;
        for (int q = 0; q < 10; ++q) ok = ok && (w[q] == 0 || w[q] == 1);
        for (int q = 10; q < 12; ++q) ok = ok && w[q] >= 1 && w[q] <= c->max_rhs;
        for (int q = 12; q < 14; ++q) ok = ok && (w[q] == 0 || w[q] == 1);
        if (ok) {
            std::copy(w, w + 14, v);
            found = true;
        }
    }
    std::fclose(f);
    if (found) {
        for (int p = 0; p < 2; ++p) {
            for (int q = 0; q < 5; ++q) c->variant[p][q] = v[5 * p + q];
            c->xy_chunk[p] = v[10 + p];
            c->y_wide[p] = v[12 + p];
        }
    }
    return found;
}

void autotune_store(const std::string& key, const Ctx* c) {
    const std::string path = autotune_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {   // create the directory chain (best effort)
        for (size_t i = 1; i <= slash; ++i)
            if (path[i] == '/' || i == slash) (void)mkdir(path.substr(0, i == slash ? slash : i).c_str(), 0755);
    }
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s", key.c_str());
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 5; ++q) std::fprintf(f, " %d", c->variant[p][q]);
    // a precision that was not tuned (c64 of an FP64-only context) stores the rule's choice of its chunk
    for (int p = 0; p < 2; ++p)
        std::fprintf(f, " %d", c->xy_chunk[p] > 0 ? c->xy_chunk[p]
                                                  : (p == 0 ? xy_chunk_rule<double>(c, c->max_rhs) : xy_chunk_rule<float>(c, c->max_rhs)));
    for (int p = 0; p < 2; ++p) std::fprintf(f, " %d", c->y_wide[p]);
    std::fprintf(f, "\n");
    std::fclose(f);
}

bool is_isotropic(const double* C) {
    double scale = 0;
    for (int i = 0; i < 36; ++i) scale = std::max(scale, std::fabs(C[i]));
    const double c11 = C[0], c44 = C[21], c12 = c11 - 2.0 * c44;
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) {
            double ref = 0;
            if (I < 3 && J < 3) ref = (I == J) ? c11 : c12;
            if (I >= 3 && I == J) ref = c44;
            if (std::fabs(C[I * 6 + J] - ref) > 1e-12 * scale) return false;
        }
    return true;
}

}  // namespace

namespace {

int check_moment(const ls_ctx* c, int i_omega, const double M[6], const int src[3], double t0) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega)) || (rc = check_cell(c, src))) return rc;
    if (!M) return fail(LS_ERR_ARG, "null moment tensor");
    for (int J = 0; J < 6; ++J)
        if (!std::isfinite(M[J])) return fail(LS_ERR_ARG, "non-finite moment tensor");
    if (!std::isfinite(t0)) return fail(LS_ERR_ARG, "non-finite rupture time");
    return LS_OK;
}

// incident field of a moment tensor into b (arguments already checked)
int rhs_moment_into(Ctx* c, int i_omega, const double M[6], const int src[3], double t0, z128* b) {
    // E^T (M delta_src): for each axis a and component c, row src_a of the 1-D difference matrix
    // D_a, weighted by the moment component of the Voigt pair (a, c)
    static const int voigt[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};
    const int n[3] = {c->n1, c->n2, c->n3};
    const double ih = 1.0 / c->h;
    std::map<std::array<int, 3>, std::array<double, 3>> pts;
    for (int a = 0; a < 3; ++a) {
        int cols[2];
        double coef[2];
        const int s = src[a];
        if (s == 0) {
            cols[0] = 0, coef[0] = -ih, cols[1] = 1, coef[1] = ih;
        } else if (s == n[a] - 1) {
            cols[0] = s, coef[0] = ih, cols[1] = s - 1, coef[1] = -ih;
        } else {
            cols[0] = s + 1, coef[0] = 0.5 * ih, cols[1] = s - 1, coef[1] = -0.5 * ih;
        }
        for (int cc = 0; cc < 3; ++cc) {
            const double m = M[voigt[a][cc]];
            if (m == 0.0) continue;
            for (int q = 0; q < 2; ++q) {
                std::array<int, 3> cell = {src[0], src[1], src[2]};
                cell[a] = cols[q];
                auto& f = pts[cell];
                f[cc] += m * coef[q];
            }
        }
    }
    std::vector<int> cells;
    std::vector<double> F;
    for (auto& kv : pts) {
        for (int a = 0; a < 3; ++a) cells.push_back(kv.first[a]);
        for (int a = 0; a < 3; ++a) F.push_back(kv.second[a]);
    }
    if (cells.empty()) {
        LS_HIP(hipMemsetAsync(b, 0, sizeof(z128) * c->field_elems(), c->stream));
        return LS_OK;
    }
    return rhs_points_launch(c, i_omega, cells.data(), F.data(), (int)pts.size(), t0, b);
}

}  // namespace

extern "C" {

const char* ls_last_error(void) { return g_last_error.c_str(); }

int ls_setup(const ls_grid* grid, const double C0[36], double rho0, const double* dC, const double* drho,
             const double* omega, int n_omega, const ls_options* opt, void* stream, ls_ctx** out) {
    if (!out) return fail(LS_ERR_ARG, "null output pointer");
    *out = nullptr;
    if (!grid || !C0 || !dC || !drho || !omega) return fail(LS_ERR_ARG, "null argument");
    for (int a = 0; a < 3; ++a)
        if (grid->n[a] < 2 || grid->n[a] > 256) return fail(LS_ERR_ARG, "grid size must be in [2, 256] per axis");
    if (!(grid->h > 0) || !std::isfinite(grid->h)) return fail(LS_ERR_ARG, "grid spacing must be positive");
    if (!(rho0 > 0) || !std::isfinite(rho0)) return fail(LS_ERR_ARG, "background density must be positive");
    if (n_omega < 1) return fail(LS_ERR_ARG, "need at least one frequency");
    for (int i = 0; i < n_omega; ++i)
        if (!(omega[i] > 0) || !std::isfinite(omega[i])) return fail(LS_ERR_ARG, "frequencies must be positive");
    double cmax = 0;
    for (int i = 0; i < 36; ++i) {
        if (!std::isfinite(C0[i])) return fail(LS_ERR_ARG, "non-finite background stiffness");
        cmax = std::max(cmax, std::fabs(C0[i]));
    }
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < I; ++J)
            if (std::fabs(C0[I * 6 + J] - C0[J * 6 + I]) > 1e-12 * cmax)
                return fail(LS_ERR_ARG, "background stiffness must be symmetric");
    ls_options o = {LS_PREC_C128, LS_GREEN_EXACT, 1, 0, 0, 1, LS_PRECOND_NONE, {0}};
    if (opt) o = *opt;
    if (o.bicgstab_l == 0) o.bicgstab_l = 1;
    if (o.bicgstab_l < 1 || o.bicgstab_l > 4) return fail(LS_ERR_ARG, "bicgstab_l must be in [1, 4] (0 means 1)");
    if (o.precision != LS_PREC_C128 && o.precision != LS_PREC_MIXED) return fail(LS_ERR_ARG, "bad precision");
    if (o.green_mode != LS_GREEN_EXACT && o.green_mode != LS_GREEN_PAPER_SUM && o.green_mode != LS_GREEN_ANISO)
        return fail(LS_ERR_ARG, "bad green_mode");
    // LS_GREEN_ANISO: a background with the three coordinate mirror planes (no coupling of normal and shear
    // strains or of different shears) keeps the octant table; any other takes the half-space table
    // (LS_GREEN_TABLE=half in the environment forces the half-space table, a test hook)
    bool half = false;
    if (o.green_mode == LS_GREEN_ANISO) {
        for (int I = 0; I < 6; ++I)
            for (int J = I + 1; J < 6; ++J)
                if (J >= 3 && std::fabs(C0[I * 6 + J]) > 1e-12 * cmax) half = true;
        const char* e = std::getenv("LS_GREEN_TABLE");
        if (e && std::strcmp(e, "half") == 0) half = true;
    }
    if (o.max_rhs < 1 || o.max_rhs > 64) return fail(LS_ERR_ARG, "max_rhs must be in [1, 64]");
    if (o.precond != LS_PRECOND_NONE && o.precond != LS_PRECOND_BLOCK_JACOBI) return fail(LS_ERR_ARG, "bad precond");
    if (o.precond != LS_PRECOND_NONE && o.bicgstab_l > 1)
        return fail(LS_ERR_ARG, "the block-Jacobi preconditioner works with Bi-CGSTAB (bicgstab_l = 1)");
    if (o.taper < 0 || 2 * o.taper > std::min(grid->n[0], std::min(grid->n[1], grid->n[2])))
        return fail(LS_ERR_ARG, "taper must be in [0, min(N)/2]");

    // isotropic reference and the anisotropic remainder folded into the contrast
    double c11, c44;
    if (is_isotropic(C0)) {
        c11 = C0[0];
        c44 = C0[21];
    } else {
        c11 = C0[14];
        c44 = 0.5 * (C0[21] + C0[28]);
    }
    if (!(c44 > 0) || !(c11 > c44)) return fail(LS_ERR_ARG, "reference medium needs C11 > C44 > 0");
    double Ciso[36] = {0};
    for (int I = 0; I < 3; ++I)
        for (int J = 0; J < 3; ++J) Ciso[I * 6 + J] = (I == J) ? c11 : c11 - 2.0 * c44;
    for (int I = 3; I < 6; ++I) Ciso[I * 6 + I] = c44;
    double fold21[21];
    for (int I = 0, q = 0; I < 6; ++I)
        for (int J = I; J < 6; ++J, ++q)
            fold21[q] = o.green_mode == LS_GREEN_ANISO ? 0.0 : C0[I * 6 + J] - Ciso[I * 6 + J];

    Ctx* c = new (std::nothrow) ls_ctx();
    if (!c) return fail(LS_ERR_OOM, "host allocation failed");
    c->n1 = grid->n[0];
    c->n2 = grid->n[1];
    c->n3 = grid->n[2];
    c->L1 = supported_fft_length(c->n1);
    c->L2 = supported_fft_length(c->n2);
    c->L3 = supported_fft_length(c->n3);
    // blocks of 8 z planes where a padded z line is 512 long (measured: the plain layout makes the z pass
    // miss the address-translation cache on 2 % of its requests there).  LS_ZBLOCK=0 keeps the plain layout
    // everywhere, LS_ZBLOCK=8 takes the blocked one wherever 8 divides N3 (both kept under test).
    {
        const char* e = std::getenv("LS_ZBLOCK");
        const bool off = e && std::strcmp(e, "0") == 0, force = e && std::strcmp(e, "8") == 0;
        c->zbs = (!off && (force || c->L3 >= 512) && c->n3 % 8 == 0) ? 3 : 0;
    }
    {
        // Operator launches inside a solve cover at most about 1.25 GiB of FP32 padded work buffer (6 systems
        // at 128^3, 1 at 256^3, all of a batch at 64^3): per system the apply costs the same from 6 systems a
        // launch upward, but in a 128^3 solve launches of 6 ran 2 % faster than launches of 48 (the passes
        // reread less of the previous pass's output from the Infinity Cache when the buffer is larger).
        // LS_LAUNCH_RHS in the environment overrides it (0: no cap).
        const long long per = 3LL * c->n3 * supported_fft_length(c->n2) * supported_fft_length(c->n1) * 8;
        c->launch_rhs = (int)std::max(1LL, (5LL << 28) / std::max(1LL, per));
        const char* e = std::getenv("LS_LAUNCH_RHS");
        if (e) c->launch_rhs = std::max(0, std::atoi(e));
    }
    c->ncell = (long long)c->n1 * c->n2 * c->n3;
    c->h = grid->h;
    c->mixed = o.precision == LS_PREC_MIXED;
    c->green_mode = o.green_mode;
    c->green_half = half;
    c->max_rhs = o.max_rhs;
    c->rho0 = rho0;
    std::copy(C0, C0 + 36, c->C0);
    c->alpha = std::sqrt(c11 / rho0);
    c->beta = std::sqrt(c44 / rho0);
    c->omega.assign(omega, omega + n_omega);
    c->stream = (hipStream_t)stream;
    c->flags = o.flags;
    c->taper = o.taper;
    c->bicgstab_l = o.bicgstab_l;
    c->precond = o.precond;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            c->device = dev;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
                c->num_cu = cus;
        }
        (void)hipGetLastError();
    }
    if (scratch_setup(c->device) != LS_OK) {
        const std::string msg = g_last_error;
        delete static_cast<ls_ctx*>(c);
        g_last_error = msg;
        return LS_ERR_HIP;
    }
    if (!c->stream) {
        // the legacy null stream cannot be captured into graphs: work on a private blocking stream,
        // which the runtime keeps ordered with the caller's work on the null stream
        if (hipStreamCreate(&c->own_stream) != hipSuccess) {
            (void)hipGetLastError();
            delete static_cast<ls_ctx*>(c);
            return fail(LS_ERR_HIP, "stream creation failed");
        }
        c->stream = c->own_stream;
    }

    const size_t n = (size_t)c->ncell;
    const size_t fe = 3 * n * (size_t)c->max_rhs;  // field elements of a batch
    const size_t oct = c->green_half ? (size_t)(c->L1 / 2 + 1) * c->L2 * c->L3
                                     : (size_t)(c->L1 / 2 + 1) * (c->L2 / 2 + 1) * (c->L3 / 2 + 1);
    int rc = LS_OK;
    auto A = [&](void** p, size_t bytes) {
        if (rc == LS_OK) rc = dalloc(c, p, bytes);
    };
    A((void**)&c->dc, 21 * n * sizeof(double));
    A((void**)&c->drho, n * sizeof(double));
    A((void**)&c->dcp, contrast_packed_elems(c, false) * sizeof(double));
    if (c->mixed) {
        A((void**)&c->dc32, 21 * n * sizeof(float));
        A((void**)&c->drho32, n * sizeof(float));
        A((void**)&c->dcp32, contrast_packed_elems(c, true) * sizeof(float));
    }
    c->ghat.assign(n_omega, nullptr);
    c->ghat32.assign(n_omega, nullptr);
    for (int i = 0; i < n_omega; ++i) {
        A((void**)&c->ghat[i], 6 * oct * sizeof(z128));
        if (c->mixed) A((void**)&c->ghat32[i], 6 * oct * sizeof(z64));
    }
    if (c->green_mode == LS_GREEN_ANISO) {
        c->greal.assign(n_omega, nullptr);
        const size_t nreal = c->green_half ? (size_t)c->n1 * (2 * c->n2 - 1) * (2 * c->n3 - 1) : n;
        for (int i = 0; i < n_omega; ++i) A((void**)&c->greal[i], 6 * nreal * sizeof(z128));
    }
    A(&c->work, (size_t)c->max_rhs * 3 * c->n3 * c->L2 * c->L1 * sizeof(z128));
    if (!use_fused_contrast()) A(&c->tau, (size_t)c->max_rhs * 6 * n * sizeof(z128));  // split contrast only
    z128** v128[] = {&c->r, &c->rhat, &c->p, &c->v, &c->s, &c->t};
    for (auto pp : v128) A((void**)pp, fe * sizeof(z128));
    A((void**)&c->bd, 3 * n * sizeof(z128));
    A((void**)&c->xbest, fe * sizeof(z128));
    A(&c->gs, fe * sizeof(z128));
    if (c->mixed) {
        z64** v64[] = {&c->r32, &c->rhat32, &c->p32, &c->v32, &c->s32, &c->t32, &c->x32, &c->b32};
        for (auto pp : v64) A((void**)pp, fe * sizeof(z64));
    }
    A((void**)&c->partials, (size_t)c->max_rhs * kRedSlots * kRedBlocks * sizeof(double));
    // fused inner products: at most 3 N3 N2 / 8 epilogue blocks per right-hand side (c128 tiles of 8 lines)
    A((void**)&c->dparts, (size_t)c->max_rhs * kRedSlots * (3 * (size_t)c->n3 * c->n2 / 8 + 1) * sizeof(double));
    A((void**)&c->state, (size_t)c->max_rhs * kStateLen * sizeof(double));
    // reductions: [0, 2 kRedBlocks) residual norms by slot, then per-slot scales, BiCGSTAB(l) coefficients and
    // per-slot squared tolerances, kRedBlocks doubles each
    A((void**)&c->red, 5 * kRedBlocks * sizeof(double));
    A(&c->stage, 8192);
    if (c->precond == LS_PRECOND_BLOCK_JACOBI) {
        c->minv.assign(n_omega, nullptr);
        c->minv32.assign(n_omega, nullptr);
        for (int i = 0; i < n_omega; ++i) {
            A((void**)&c->minv[i], 9 * n * sizeof(z128));
            if (c->mixed) A((void**)&c->minv32[i], 9 * n * sizeof(z64));
        }
        A((void**)&c->gloc, 125 * 6 * sizeof(z128));
        A((void**)&c->ph, fe * sizeof(z128));
        A((void**)&c->sh, fe * sizeof(z128));
        if (c->mixed) {
            A((void**)&c->ph32, fe * sizeof(z64));
            A((void**)&c->sh32, fe * sizeof(z64));
        }
    }
    if (rc == LS_OK && c->bicgstab_l > 1) rc = krylov_setup(c);
    if (rc == LS_OK) {
        const size_t hb = std::max<size_t>(4 * kRedBlocks, (size_t)c->max_rhs * kStateLen) * sizeof(double);
        if (hipHostMalloc((void**)&c->red_host, hb, hipHostMallocDefault) != hipSuccess) {
            c->red_host = nullptr;
            rc = fail(LS_ERR_OOM, "pinned host allocation failed");
        }
    }
    // twiddle tables e^{-2 pi i m / L} computed in FP64 on the host
    for (int L : {c->L1, c->L2, c->L3}) {
        if (rc || c->twiddle128(L)) continue;
        std::vector<z128> h128(L);
        std::vector<z64> h64(L);
        for (int m = 0; m < L; ++m) {
            const double ang = -2.0 * 3.14159265358979323846 * (double)m / (double)L;
            h128[m] = {std::cos(ang), std::sin(ang)};
            h64[m] = {(float)h128[m].x, (float)h128[m].y};
        }
        z128* d128 = nullptr;
        z64* d64 = nullptr;
        A((void**)&d128, L * sizeof(z128));
        A((void**)&d64, L * sizeof(z64));
        if (rc) {
            if (d128) (void)hipFree(d128);
            if (d64) (void)hipFree(d64);
            break;
        }
        c->tw_len.push_back(L);
        c->tw128.push_back(d128);
        c->tw64.push_back(d64);
        if (hipMemcpy(d128, h128.data(), L * sizeof(z128), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d64, h64.data(), L * sizeof(z64), hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(LS_ERR_HIP, "twiddle upload failed");
    }
    std::copy(fold21, fold21 + 21, c->fold21);
    if (rc == LS_OK) rc = fold_background(c, dC, drho, fold21);
    if (rc == LS_OK) rc = build_green_tables(c);
    if (rc == LS_OK) rc = build_block_jacobi(c);
    if (rc == LS_OK && (c->flags & LS_FLAG_AUTOTUNE)) {
        const std::string key = autotune_key(c);
        if (!autotune_lookup(key, c)) {
            if (hipMemsetAsync(c->work, 0, (size_t)c->max_rhs * 3 * c->n3 * c->L2 * c->L1 * sizeof(z128), c->stream) !=
                hipSuccess)
                rc = fail(LS_ERR_HIP, "autotune buffer clear failed");
            if (rc == LS_OK) rc = autotune_passes<double>(c);
            if (rc == LS_OK && c->mixed) rc = autotune_passes<float>(c);
            if (rc == LS_OK) autotune_store(key, c);
        }
    }
    if (rc == LS_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(LS_ERR_HIP, "setup synchronisation failed");
    if (rc) {
        const std::string msg = g_last_error;
        release(c);
        g_last_error = msg;
        return rc;
    }
    *out = static_cast<ls_ctx*>(c);
    return LS_OK;
}

void ls_destroy(ls_ctx* ctx) { release(ctx); }

int ls_set_contrast(ls_ctx* c, const double* dC, const double* drho) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (!dC || !drho) return fail(LS_ERR_ARG, "null argument");
    if ((rc = fold_background(c, dC, drho, c->fold21))) return rc;
    return build_block_jacobi(c);
}

int ls_precond_blocks(ls_ctx* c, int i_omega, void* minv) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega))) return rc;
    if (!minv) return fail(LS_ERR_ARG, "null argument");
    if (c->precond != LS_PRECOND_BLOCK_JACOBI) return fail(LS_ERR_STATE, "the context has no block-Jacobi preconditioner");
    LS_HIP(hipMemcpyAsync(minv, c->minv[i_omega], 9 * (size_t)c->ncell * sizeof(z128), hipMemcpyDeviceToDevice,
                          c->stream));
    return LS_OK;
}

int ls_apply(ls_ctx* c, int i_omega, const void* u, void* Au, int n_rhs) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega))) return rc;
    if (!u || !Au) return fail(LS_ERR_ARG, "null field pointer");
    if (n_rhs < 1 || n_rhs > c->max_rhs) return fail(LS_ERR_ARG, "n_rhs outside [1, max_rhs]");
    if ((rc = check_disjoint(c, u, Au, n_rhs, sizeof(z128), "ls_apply"))) return rc;
    return apply_op<double>(c, RhsSet::uniform(n_rhs, i_omega), (const z128*)u, (z128*)Au);
}

int ls_apply_noalloc(ls_ctx* c, int i_omega, const void* u, void* Au, int n_rhs) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega))) return rc;
    if (!u || !Au) return fail(LS_ERR_ARG, "null field pointer");
    if (n_rhs < 1 || n_rhs > c->max_rhs) return fail(LS_ERR_ARG, "n_rhs outside [1, max_rhs]");
    if ((rc = check_disjoint(c, u, Au, n_rhs, sizeof(z128), "ls_apply_noalloc"))) return rc;
    const size_t work = (size_t)n_rhs * 3 * c->n3 * c->L2 * c->L1 * sizeof(z128);
    const size_t tau = use_fused_contrast() ? 0 : (size_t)n_rhs * 6 * (size_t)c->ncell * sizeof(z128);
    const size_t work_al = (work + 255) / 256 * 256;
    if (work_al + tau > kScratchBytes)
        return fail(LS_ERR_ARG, "ls_apply_noalloc: " + std::to_string(work_al + tau) + " bytes of work buffer exceed the " +
                                    std::to_string(kScratchBytes) + "-byte scratch (3 N3 L2 L1 x 16 bytes per right-hand side)");
    char* base = static_cast<char*>(scratch_address(c->device));
    if (!base) return fail(LS_ERR_STATE, "scratch address not set up on the context's device");
    return apply_op_in<double>(c, RhsSet::uniform(n_rhs, i_omega), (const z128*)u, (z128*)Au, (z128*)base,
                               tau ? (z128*)(base + work_al) : nullptr);
}

int ls_apply_c64(ls_ctx* c, int i_omega, const void* u, void* Au, int n_rhs) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega))) return rc;
    if (!c->mixed) return fail(LS_ERR_STATE, "the FP32 operator needs a context built with LS_PREC_MIXED");
    if (!u || !Au) return fail(LS_ERR_ARG, "null field pointer");
    if (n_rhs < 1 || n_rhs > c->max_rhs) return fail(LS_ERR_ARG, "n_rhs outside [1, max_rhs]");
    if ((rc = check_disjoint(c, u, Au, n_rhs, sizeof(z64), "ls_apply_c64"))) return rc;
    return apply_op<float>(c, RhsSet::uniform(n_rhs, i_omega), (const z64*)u, (z64*)Au);
}

int ls_apply_T(ls_ctx* c, int i_omega, const void* y, void* ATy, int n_rhs) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega))) return rc;
    if (!y || !ATy) return fail(LS_ERR_ARG, "null field pointer");
    if (n_rhs < 1 || n_rhs > c->max_rhs) return fail(LS_ERR_ARG, "n_rhs outside [1, max_rhs]");
    if ((rc = check_disjoint(c, y, ATy, n_rhs, sizeof(z128), "ls_apply_T"))) return rc;
    return apply_T_op<double>(c, RhsSet::uniform(n_rhs, i_omega), (const z128*)y, (z128*)ATy);
}

int ls_convolve(ls_ctx* c, int i_omega, const void* f, void* out, int n_rhs) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega))) return rc;
    if (!f || !out) return fail(LS_ERR_ARG, "null field pointer");
    if (n_rhs < 1 || n_rhs > c->max_rhs) return fail(LS_ERR_ARG, "n_rhs outside [1, max_rhs]");
    return convolve_op<double>(c, RhsSet::uniform(n_rhs, i_omega), (const z128*)f, (z128*)out);
}

int ls_solve_T(ls_ctx* c, int i_omega, const void* b, int n_rhs, double tol, int maxit, int precision,
               const void* x0, void* x_out, ls_info* info) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega))) return rc;
    if (!b || !x_out) return fail(LS_ERR_ARG, "null field pointer");
    if (n_rhs < 1 || n_rhs > c->max_rhs) return fail(LS_ERR_ARG, "n_rhs outside [1, max_rhs]");
    if (!(tol > 0) || !(tol < 1)) return fail(LS_ERR_ARG, "tol must be in (0, 1)");
    if (maxit < 1) return fail(LS_ERR_ARG, "maxit must be >= 1");
    if (precision != LS_PREC_C128 && precision != LS_PREC_MIXED) return fail(LS_ERR_ARG, "bad precision");
    if (precision == LS_PREC_MIXED && !c->mixed)
        return fail(LS_ERR_STATE, "mixed precision needs a context built with LS_PREC_MIXED");
    if ((rc = check_solve_buffers(c, b, x0, x_out, n_rhs))) return rc;
    const std::vector<int> freq(n_rhs, i_omega);
    return solve_systems(c, freq.data(), (const z128*)b, n_rhs, tol, maxit, precision, (const z128*)x0, (z128*)x_out,
                         info, true);
}

int ls_grad_contrast(ls_ctx* c, int i_omega, const void* u, const void* mu, int n_rhs, double* g_dC, double* g_drho) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega))) return rc;
    if (!u || !mu || !g_dC || !g_drho) return fail(LS_ERR_ARG, "null pointer");
    if (n_rhs < 1) return fail(LS_ERR_ARG, "n_rhs must be >= 1");
    return grad_contrast_launch(c, i_omega, (const z128*)u, (const z128*)mu, n_rhs, g_dC, g_drho);
}

int ls_grad(ls_ctx* c, int i_omega, const void* u, const void* lam_bar, int n_rhs, const int* src, const double* t0,
            double* g_dC, double* g_drho, double* g_M) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega))) return rc;
    if (!u || !lam_bar || !g_dC || !g_drho) return fail(LS_ERR_ARG, "null pointer");
    if (n_rhs < 1 || n_rhs > c->max_rhs) return fail(LS_ERR_ARG, "n_rhs outside [1, max_rhs]");
    if (g_M) {
        if (!src || !t0) return fail(LS_ERR_ARG, "g_M needs the source cells and times");
        for (int r = 0; r < n_rhs; ++r) {
            if ((rc = check_cell(c, src + 3 * r))) return rc;
            if (!std::isfinite(t0[r])) return fail(LS_ERR_ARG, "non-finite source time");
        }
    }
    z128* mu = (z128*)c->gs;  // mu = conj(Gconv lam_bar), in the workspace of the transposed operator
    if ((rc = convolve_op<double>(c, RhsSet::uniform(n_rhs, i_omega), (const z128*)lam_bar, mu))) return rc;
    if ((rc = conj_launch(c, mu, 3 * c->ncell * n_rhs))) return rc;
    if ((rc = grad_contrast_launch(c, i_omega, (const z128*)u, mu, n_rhs, g_dC, g_drho))) return rc;
    if (g_M) return grad_moment_launch(c, i_omega, mu, n_rhs, src, t0, g_M);
    return LS_OK;
}


int ls_rhs_moment(ls_ctx* c, int i_omega, const double M[6], const int src[3], double t0, void* b) {
    int rc;
    if ((rc = check_moment(c, i_omega, M, src, t0))) return rc;
    if (!b) return fail(LS_ERR_ARG, "null argument");
    return rhs_moment_into(c, i_omega, M, src, t0, (z128*)b);
}

int ls_rhs_force(ls_ctx* c, int i_omega, const double F[3], const int cell[3], void* b) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega)) || (rc = check_cell(c, cell))) return rc;
    if (!F || !b) return fail(LS_ERR_ARG, "null argument");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(F[a])) return fail(LS_ERR_ARG, "non-finite force");
    return rhs_points_launch(c, i_omega, cell, F, 1, 0.0, (z128*)b);
}

int ls_solve(ls_ctx* c, int i_omega, const void* b, int n_rhs, double tol, int maxit, int precision, const void* x0,
             void* u_out, ls_info* info) {
    int rc;
    if ((rc = check_ctx(c)) || (rc = check_omega(c, i_omega))) return rc;
    if (!b || !u_out) return fail(LS_ERR_ARG, "null field pointer");
    if (n_rhs < 1 || n_rhs > c->max_rhs) return fail(LS_ERR_ARG, "n_rhs outside [1, max_rhs]");
    if (!(tol > 0) || !(tol < 1)) return fail(LS_ERR_ARG, "tol must be in (0, 1)");
    if (maxit < 1) return fail(LS_ERR_ARG, "maxit must be >= 1");
    if (precision != LS_PREC_C128 && precision != LS_PREC_MIXED) return fail(LS_ERR_ARG, "bad precision");
    if (precision == LS_PREC_MIXED && !c->mixed)
        return fail(LS_ERR_STATE, "mixed precision needs a context built with LS_PREC_MIXED");
    if ((rc = check_solve_buffers(c, b, x0, u_out, n_rhs))) return rc;
    const std::vector<int> freq(n_rhs, i_omega);
    return solve_systems(c, freq.data(), (const z128*)b, n_rhs, tol, maxit, precision, (const z128*)x0, (z128*)u_out,
                         info);
}

int ls_solve_multi(ls_ctx* c, const int* i_omega, const void* b, int n_rhs, double tol, int maxit, int precision,
                   const void* x0, void* u_out, ls_info* info) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (!i_omega || !b || !u_out) return fail(LS_ERR_ARG, "null argument");
    if (n_rhs < 1 || n_rhs > c->max_rhs) return fail(LS_ERR_ARG, "n_rhs outside [1, max_rhs]");
    for (int q = 0; q < n_rhs; ++q)
        if ((rc = check_omega(c, i_omega[q]))) return rc;
    if (!(tol > 0) || !(tol < 1)) return fail(LS_ERR_ARG, "tol must be in (0, 1)");
    if (maxit < 1) return fail(LS_ERR_ARG, "maxit must be >= 1");
    if (precision != LS_PREC_C128 && precision != LS_PREC_MIXED) return fail(LS_ERR_ARG, "bad precision");
    if (precision == LS_PREC_MIXED && !c->mixed)
        return fail(LS_ERR_STATE, "mixed precision needs a context built with LS_PREC_MIXED");
    if ((rc = check_solve_buffers(c, b, x0, u_out, n_rhs))) return rc;
    return solve_systems(c, i_omega, (const z128*)b, n_rhs, tol, maxit, precision, (const z128*)x0, (z128*)u_out,
                         info);
}

int ls_solve_moment(ls_ctx* c, int i_omega, const double M[6], const int src[3], double t0, double tol, int maxit,
                    int precision, const void* x0, void* u_out, ls_info* info) {
    int rc = ls_rhs_moment(c, i_omega, M, src, t0, c ? (void*)c->bd : nullptr);
    if (rc) return rc;
    return ls_solve(c, i_omega, c->bd, 1, tol, maxit, precision, x0, u_out, info);
}

int ls_solve_force(ls_ctx* c, int i_omega, const double F[3], const int cell[3], double tol, int maxit, int precision,
                   void* u_out, ls_info* info) {
    int rc = ls_rhs_force(c, i_omega, F, cell, c ? (void*)c->bd : nullptr);
    if (rc) return rc;
    return ls_solve(c, i_omega, c->bd, 1, tol, maxit, precision, nullptr, u_out, info);
}

}  // extern "C"

namespace {

bool soft_failure(int rc) { return rc == LS_ERR_NOT_CONVERGED || rc == LS_ERR_BREAKDOWN || rc == LS_ERR_NONFINITE; }

// One multi-right-hand-side solve of the jobs idx (all of context c, at any frequencies): incident fields
// into the context's batch buffer, one batched solve with each system at its own frequency, then each
// solution copied to its job.
int run_batch(Ctx* c, const ls_job* jobs, const std::vector<int>& idx, double tol, int maxit, int precision,
              ls_info* infos) {
    const size_t fe = c->field_elems();
    if (!c->batch_b || !c->batch_x) {
        int arc = dalloc(c, (void**)&c->batch_b, (size_t)c->max_rhs * fe * sizeof(z128));
        if (arc == LS_OK) arc = dalloc(c, (void**)&c->batch_x, (size_t)c->max_rhs * fe * sizeof(z128));
        if (arc != LS_OK) {   // leave neither half allocated, so the next call allocates both again
            for (z128** q : {&c->batch_b, &c->batch_x}) {
                if (*q) {
                    (void)hipFree(*q);
                    c->bytes -= (long long)((size_t)c->max_rhs * fe * sizeof(z128));
                }
                *q = nullptr;
            }
            return arc;
        }
    }
    const int nr = (int)idx.size();
    std::vector<int> freq(nr);
    int rc;
    for (int r = 0; r < nr; ++r) {
        const ls_job& j = jobs[idx[r]];
        freq[r] = j.i_omega;
        if ((rc = rhs_moment_into(c, j.i_omega, j.M, j.src, j.t0, c->batch_b + r * fe))) return rc;
    }
    std::vector<ls_info> inf(nr);
    rc = solve_systems(c, freq.data(), c->batch_b, nr, tol, maxit, precision, nullptr, c->batch_x, inf.data());
    if (rc != LS_OK && !soft_failure(rc)) return rc;
    for (int r = 0; r < nr; ++r) {
        LS_HIP(hipMemcpyAsync(jobs[idx[r]].u_out, c->batch_x + r * fe, fe * sizeof(z128), hipMemcpyDeviceToDevice,
                              c->stream));
        if (infos) infos[idx[r]] = inf[r];
    }
    LS_HIP(hipStreamSynchronize(c->stream));
    return rc;
}

}  // namespace

extern "C" {

int ls_solve_batch(ls_ctx* const* ctxs, int n_ctx, const ls_job* jobs, int n_jobs, double tol, int maxit,
                   int precision, ls_info* infos) {
    int rc;
    if (!ctxs || n_ctx < 1 || n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(LS_ERR_ARG, "bad batch arguments");
    if (!(tol > 0) || !(tol < 1)) return fail(LS_ERR_ARG, "tol must be in (0, 1)");
    if (maxit < 1) return fail(LS_ERR_ARG, "maxit must be >= 1");
    if (precision != LS_PREC_C128 && precision != LS_PREC_MIXED) return fail(LS_ERR_ARG, "bad precision");
    for (int i = 0; i < n_ctx; ++i) {
        if ((rc = check_ctx(ctxs[i]))) return rc;
        if (precision == LS_PREC_MIXED && !ctxs[i]->mixed)
            return fail(LS_ERR_STATE, "mixed precision needs contexts built with LS_PREC_MIXED");
        for (int k = 0; k < i; ++k)
            if (ctxs[k] == ctxs[i]) return fail(LS_ERR_ARG, "a context appears twice in the batch");
    }
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[j].ctx < 0 || jobs[j].ctx >= n_ctx) return fail(LS_ERR_ARG, "job context index out of range");
        if ((rc = check_moment(ctxs[jobs[j].ctx], jobs[j].i_omega, jobs[j].M, jobs[j].src, jobs[j].t0))) return rc;
        if (!jobs[j].u_out) return fail(LS_ERR_ARG, "null job output");
    }
    // plan: per context, its jobs ordered by frequency (stable within a frequency), in chunks of max_rhs;
    // a chunk mixes frequencies, each system at its own
    std::vector<std::vector<std::vector<int>>> plan(n_ctx);
    for (int i = 0; i < n_ctx; ++i) {
        std::vector<int> mine;
        for (int j = 0; j < n_jobs; ++j)
            if (jobs[j].ctx == i) mine.push_back(j);
        std::stable_sort(mine.begin(), mine.end(), [&](int a, int b) { return jobs[a].i_omega < jobs[b].i_omega; });
        for (size_t k = 0; k < mine.size(); k += (size_t)ctxs[i]->max_rhs)
            plan[i].emplace_back(mine.begin() + k, mine.begin() + std::min(mine.size(), k + (size_t)ctxs[i]->max_rhs));
    }
    // one worker per context with work, each driving its context's stream (the solves synchronise
    // for their convergence tests, so contexts on different streams overlap on the device)
    std::vector<int> codes(n_ctx, LS_OK);
    std::vector<std::string> msgs(n_ctx);
    auto work = [&](int i) {
        Ctx* c = ctxs[i];
        if (hipSetDevice(c->device) != hipSuccess) {
            (void)hipGetLastError();
            codes[i] = LS_ERR_HIP;
            msgs[i] = "hipSetDevice failed";
            return;
        }
        for (const auto& batch : plan[i]) {
            const int r = run_batch(c, jobs, batch, tol, maxit, precision, infos);
            if (r == LS_OK) continue;
            if (codes[i] == LS_OK || !soft_failure(r)) {
                codes[i] = r;
                msgs[i] = ls_last_error();
            }
            if (!soft_failure(r)) return;
        }
    };
    std::vector<int> active;
    for (int i = 0; i < n_ctx; ++i)
        if (!plan[i].empty()) active.push_back(i);
    if (active.size() == 1) {
        work(active[0]);
    } else if (!active.empty()) {
        std::vector<std::thread> th;
        for (int i : active) th.emplace_back(work, i);
        for (auto& t : th) t.join();
    }
    for (int i = 0; i < n_ctx; ++i)  // hard errors first, then the first unconverged context
        if (codes[i] != LS_OK && !soft_failure(codes[i])) return fail(codes[i], msgs[i]);
    for (int i = 0; i < n_ctx; ++i)
        if (codes[i] != LS_OK) return fail(codes[i], msgs[i]);
    return LS_OK;
}

int ls_sample(ls_ctx* c, const void* u, int n_rhs, const int* rec, int n_rec, void* out) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (!u || !out || !rec) return fail(LS_ERR_ARG, "null argument");
    if (n_rhs < 1 || n_rec < 1) return fail(LS_ERR_ARG, "n_rhs and n_rec must be >= 1");
    for (int m = 0; m < n_rec; ++m)
        if ((rc = check_cell(c, rec + 3 * m))) return rc;
    return sample_launch(c, (const z128*)u, n_rhs, rec, n_rec, (z128*)out);
}

int ls_synthesize(ls_ctx* c, const void* spectra, const int* k, int n_freq, int n_trace, int nt, double dt, double fp,
                  double ts, double* traces) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (!spectra || !k || !traces) return fail(LS_ERR_ARG, "null argument");
    if (n_freq < 1 || n_trace < 1 || nt < 2) return fail(LS_ERR_ARG, "n_freq, n_trace >= 1 and nt >= 2 required");
    if (!(dt > 0) || !std::isfinite(dt) || !std::isfinite(fp) || !std::isfinite(ts))
        return fail(LS_ERR_ARG, "dt must be positive; dt, fp, ts finite");
    for (int q = 0; q < n_freq; ++q)
        if (k[q] < 0 || 2 * k[q] > nt) return fail(LS_ERR_ARG, "frequency index outside [0, nt/2]");
    return synthesize_launch(c, (const z128*)spectra, k, n_freq, n_trace, nt, dt, fp, ts, traces);
}

int ls_strain(ls_ctx* c, const void* u, void* eps, int n_rhs) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (!u || !eps) return fail(LS_ERR_ARG, "null field pointer");
    if (n_rhs < 1) return fail(LS_ERR_ARG, "n_rhs must be >= 1");
    if (overlaps(u, (size_t)n_rhs * c->field_elems() * sizeof(z128), eps, 2 * (size_t)n_rhs * c->field_elems() * sizeof(z128)))
        return fail(LS_ERR_ARG, "ls_strain: u and eps overlap");
    return strain_launch(c, (const z128*)u, (z128*)eps, n_rhs);
}

int ls_residual_history(ls_ctx* c, int rhs, double* hist, int max_len) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    if (rhs < 0 || rhs >= (int)c->history.size()) return fail(LS_ERR_ARG, "no such right-hand side in the last solve");
    if (max_len < 0 || (max_len > 0 && !hist)) return fail(LS_ERR_ARG, "bad history buffer");
    const auto& h = c->history[rhs];
    for (int i = 0; i < max_len && i < (int)h.size(); ++i) hist[i] = h[i];
    return (int)h.size();
}

int ls_profile(ls_ctx* c, int enable) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    Profiler& P = c->prof;
    if (enable && P.ev.empty()) {
        P.ev.resize(2 * Profiler::kMax);
        P.fam.resize(Profiler::kMax);
        P.rhs.resize(Profiler::kMax);
        P.tabs.resize(Profiler::kMax);
        for (auto& e : P.ev) LS_HIP(hipEventCreate(&e));
    }
    P.on = enable != 0;
    return LS_OK;
}

int ls_profile_read(ls_ctx* c, char* names, int* counts, double* ms, long long* units, int n_max) {
    int rc;
    if ((rc = check_ctx(c))) return rc;
    Profiler& P = c->prof;
    LS_HIP(hipStreamSynchronize(c->stream));
    const size_t nf_ = P.names.size();
    std::vector<double> sum(nf_, 0.0);
    std::vector<int> cnt(nf_, 0);
    std::vector<long long> rsum(nf_, 0), tsum(nf_, 0);
    for (int i = 0; i < P.n; ++i) {
        float t = 0;
        LS_HIP(hipEventElapsedTime(&t, P.ev[2 * i], P.ev[2 * i + 1]));
        sum[P.fam[i]] += t;
        cnt[P.fam[i]] += 1;
        rsum[P.fam[i]] += P.rhs[i];
        tsum[P.fam[i]] += P.tabs[i];
    }
    const int nf = (int)nf_;
    for (int k = 0; k < nf && k < n_max; ++k) {
        if (names) {
            std::strncpy(names + 64 * k, P.names[k].c_str(), 63);
            names[64 * k + 63] = 0;
        }
        if (counts) counts[k] = cnt[k];
        if (ms) ms[k] = sum[k];
        if (units) {
            units[2 * k] = rsum[k];
            units[2 * k + 1] = tsum[k];
        }
    }
    P.n = 0;
    return nf;
}

long long ls_device_bytes(const ls_ctx* c) { return c ? c->bytes : 0; }

int ls_contrast_format(const ls_ctx* c) {
    if (!c) return fail(LS_ERR_ARG, "null context");
    return c->contrast_k;
}

int ls_kernel_variants(const ls_ctx* c, int* variants) {
    if (!c || !variants) return fail(LS_ERR_ARG, "null argument");
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 5; ++q) variants[p * 5 + q] = c->variant[p][q];
    return LS_OK;
}

int ls_kernel_schedule(const ls_ctx* c, int* schedule) {
    if (!c || !schedule) return fail(LS_ERR_ARG, "null argument");
    for (int p = 0; p < 2; ++p) {
        schedule[p] = c->xy_chunk[p] > 0 ? std::min(c->xy_chunk[p], c->max_rhs)
                                         : (p == 0 ? xy_chunk_rule<double>(c, c->max_rhs) : xy_chunk_rule<float>(c, c->max_rhs));
        schedule[2 + p] = c->y_wide[p];
    }
    return LS_OK;
}

}  // extern "C"
