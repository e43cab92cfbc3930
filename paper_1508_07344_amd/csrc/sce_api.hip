// Host runtime and C ABI of the spectral canonical electrostatic library.
// Owns the device buffers of a context, builds the mode tables, and orders
// the kernels of one pass (phase table -> deposit -> reduce/solve -> force)
// and of the leapfrog steps on the context's HIP stream.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sce.h"
#include "sce_internal.h"

using sce::Geom;

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct EventPair {
    hipEvent_t a, b;
};

// Scratch of sce_force_noalloc: one static array per GPU, resolved to a device
// address once per device (hipGetSymbolAddress at context creation) and only
// used through that address.  Every call on a GPU shares it.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Scratch buffers of one pass (deposit, solve, force) supplied by the caller
// of the pass instead of the context's own lazily sized buffers.
struct PassScratch {
    void *tab, *tabxy, *part, *rec, *fscr;
};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

struct sce_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool broken = false;

    double L = 1.0, width = 0.0, eps0 = 1.0;
    int dim = 3;  // 2: line charges, stored with x = 0 and (y, z) = their (x, y)
    // SCE_FIELD_TENT: tent field shapes on all of R^D, point particles, the
    // origin mode kept, no wrap (see sce_create_tent)
    int field = SCE_FIELD_DELTA;
    int kind = SCE_SHAPE_GAUSSIAN;
    int prec = SCE_PREC_FP64;
    int scheme = SCE_SCHEME_KDK;
    Geom g{};

    int64_t N = 0, cap = 0;
    double *pos = nullptr, *vel = nullptr, *q = nullptr, *m = nullptr, *F = nullptr,
           *phi = nullptr;
    void *tab = nullptr;        // z phase table, working precision
    size_t tab_bytes = 0;
    void *tabxy = nullptr;      // x/y phase tables, FP64
    size_t tabxy_bytes = 0;
    double *part = nullptr;
    size_t part_bytes = 0;
    double *Stab = nullptr, *Gtab = nullptr, *Ktab = nullptr;
    double2 *rho = nullptr, *psi = nullptr;
    void *ftab = nullptr, *psi0 = nullptr;
    // split-precision path: particle records, packed force fragments, row scales
    double *turns = nullptr;
    size_t turns_bytes = 0;
    void *wf = nullptr;
    float *wscr = nullptr;
    double qscale = 1.0;
    double *wpart = nullptr;
    int wblocks = 0;
    double *dscratch = nullptr;
    size_t dscratch_bytes = 0;
    double *fscratch = nullptr;  // line-group partial sums of the VALU force
    size_t fscratch_bytes = 0;
    double *dout = nullptr;
    // tent field shapes: weighted charges, envelope [4][N], force-kernel F and
    // P before the envelope, the mode cube (two buffers), the 1-D eigenbases
    double *qw = nullptr, *env = nullptr, *Fk = nullptr, *Pk = nullptr;
    double2 *cubeX = nullptr, *cubeY = nullptr;
    double *Vf = nullptr, *Vb = nullptr, *lam = nullptr;
    double env_max = 1.0;  // E(0), the largest envelope value
    // small systems: the stored modes as integer triplets and S^2 / (eps0 k^2 V),
    // for the single-workgroup multi-step kernel (|H| <= kSmallMaxH only)
    short4 *smodes = nullptr;
    double *sweight = nullptr;
    int64_t small_max_pairs = 1 << 16;  // largest N |H| stepped by that kernel (0: never)

    bool fields_valid = false;  // rho/psi/W/ftab correspond to the current positions
    bool force_valid = false;   // F corresponds to the current positions
    bool phi_valid = false;     // phi too (the split force leaves it out unless asked)
    int64_t step = 0;
    double time = 0.0;
    double q2sum = 0.0;
    double self_sum = 0.0;  // sum_H S^2 / |k|^2

    // Multi-step runs replay a captured HIP graph of graph_steps steps (0: launch
    // directly).  gen counts every change of a buffer, a kernel argument fixed
    // at capture or the stream; the graph is captured again when gen, dt or the
    // scheme differ from what it was captured with.
    int graph_steps = 8;
    uint64_t gen = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    uint64_t g_gen = 0;
    double g_dt = 0.0;
    int g_scheme = -1, g_len = 0;

    bool timing = false;
    std::vector<EventPair> ev_dep, ev_frc;
    std::vector<hipEvent_t> ev_pool;

    std::string err;
};

namespace {

sce_status fail(sce_ctx c, sce_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

sce_status hipfail(sce_ctx c, hipError_t e, const char *what)
{
    if (c) {
        c->broken = true;
        c->err = std::string(what) + ": " + hipGetErrorString(e);
    }
    return SCE_EDEVICE;
}

#define HIPCHK(c, expr)                                   \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return hipfail(c, _e, #expr); \
    } while (0)

// Device allocations sized by the caller's input: running out of memory is
// SCE_ENOMEM and leaves the context usable (the error is cleared); any other
// failure is a device error.
#define ALLOCCHK(c, expr)                                                               \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e == hipErrorOutOfMemory) {                                                \
            (void)hipGetLastError();                                                    \
            return fail(c, SCE_ENOMEM, std::string(#expr) + ": out of device memory");  \
        }                                                                               \
        if (_e != hipSuccess) return hipfail(c, _e, #expr);                             \
    } while (0)

Geom make_geom(int n, int dim)
{
    Geom g;
    g.n = n;
    g.M = 2 * n + 1;
    g.n1 = n + 1;
    g.lines = dim == 2 ? 1 : n + 1;
    g.R = (n + 1) + (g.lines - 1) * g.M;
    g.Rpad = (g.R + 63) / 64 * 64;
    g.P = (int64_t)g.R * g.M;
    g.H = g.P - (n + 1);
    // force table slots: a multiple of the widest register chunk (FP32's)
    const int c = sce::force_chunk(n, 4);
    g.nzp = (n + c - 1) / c * c;
    // covers the n_z groups of either deposit tiling (4 or 8 per group)
    g.zslots = 1 + (n + 7) / 8 * 8;
    return g;
}

double shape_factor(int kind, double a, double kx, double ky, double kz)
{
    if (kind == SCE_SHAPE_DELTA) return 1.0;
    if (kind == SCE_SHAPE_GAUSSIAN) return std::exp(-0.5 * (kx * kx + ky * ky + kz * kz) * a * a);
    auto sinc = [](double u) { return u == 0.0 ? 1.0 : std::sin(u) / u; };
    const double sx = sinc(0.5 * kx * a), sy = sinc(0.5 * ky * a), sz = sinc(0.5 * kz * a);
    return sx * sx * sy * sy * sz * sz;
}

size_t elem_bytes(int prec) { return prec == SCE_PREC_FP64 ? 8 : 4; }

void free_dev(void *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}
template <typename T>
void free_devp(T *&p)
{
    void *v = p;
    free_dev(v);
    p = nullptr;
}

template <typename T>
hipError_t dev_alloc(T *&p, size_t bytes)
{
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, bytes ? bytes : 16);
    p = (T *)v;
    return e;
}

// Stored modes exported through the ABI: H, preceded by the origin in a
// tent-field context; the origin sits just before H in the padded layout.
int64_t export_first(sce_ctx c) { return c->field == SCE_FIELD_TENT ? c->g.n : c->g.n1; }
int64_t export_count(sce_ctx c) { return c->field == SCE_FIELD_TENT ? c->g.H + 1 : c->g.H; }

// Box volume V = L^3, or the area A = L^2 of a two-dimensional context.
double box_measure(sce_ctx c) { return c->dim == 2 ? c->L * c->L : c->L * c->L * c->L; }

// Green tables for (row, |n_z|): S, G = S / (eps0 k^2 V), K = 1 / (eps0 k^2 V)
// (V = A in two dimensions; there k_x = 0 for every stored mode).
// Tent field shapes: S = 1 for every stored mode, the origin included, and
// G = K = 0: the reduce/solve kernel then leaves rho only, and the tent solve
// writes psi, the force table and the energy partials.
sce_status build_tables(sce_ctx c)
{
    const Geom &g = c->g;
    const size_t cnt = (size_t)g.R * g.n1;
    std::vector<double> S(cnt), G(cnt), K(cnt);
    const double f = kTwoPi / c->L, V = box_measure(c);
    double self = 0.0;
    for (int r = 0; r < g.R && c->field == SCE_FIELD_TENT; ++r)
        for (int nz = 0; nz <= g.n; ++nz) {
            const size_t i = (size_t)nz * g.R + r;  // [n_z][row]: rows fastest, as the reduce reads them
            S[i] = 1.0;
            G[i] = K[i] = 0.0;
        }
    for (int r = 0; r < g.R && c->field != SCE_FIELD_TENT; ++r) {
        int nx, ny;
        sce::row_nxny(r, g.n, nx, ny);
        for (int nz = 0; nz <= g.n; ++nz) {
            const size_t i = (size_t)nz * g.R + r;  // [n_z][row]: rows fastest, as the reduce reads them
            if (nx == 0 && ny == 0 && nz == 0) {
                S[i] = G[i] = K[i] = 0.0;
                continue;
            }
            const double kx = f * nx, ky = f * ny, kz = f * nz;
            const double k2 = kx * kx + ky * ky + kz * kz;
            const double s = shape_factor(c->kind, c->width, kx, ky, kz);
            S[i] = s;
            K[i] = 1.0 / (c->eps0 * k2 * V);
            G[i] = s * K[i];
            const int mult = (sce::in_half(nx, ny, nz) ? 1 : 0) +
                             ((nz > 0 && sce::in_half(nx, ny, -nz)) ? 1 : 0);
            self += mult * s * s / k2;
        }
    }
    c->self_sum = self;
    if (c->field != SCE_FIELD_TENT && g.H <= sce::kSmallMaxH) {
        std::vector<short4> md;
        std::vector<double> wt;
        md.reserve(g.H);
        wt.reserve(g.H);
        for (int r = 0; r < g.R; ++r) {
            int nx, ny;
            sce::row_nxny(r, g.n, nx, ny);
            for (int nz = -g.n; nz <= g.n; ++nz) {
                if (!sce::in_half(nx, ny, nz)) continue;
                const double kx = f * nx, ky = f * ny, kz = f * nz;
                const double k2 = kx * kx + ky * ky + kz * kz;
                const double s = shape_factor(c->kind, c->width, kx, ky, kz);
                short4 v;
                v.x = (short)nx;
                v.y = (short)ny;
                v.z = (short)nz;
                v.w = 0;
                md.push_back(v);
                wt.push_back(s * s / (c->eps0 * k2 * V));
            }
        }
        if (!c->smodes) {
            HIPCHK(c, dev_alloc(c->smodes, g.H * sizeof(short4)));
            HIPCHK(c, dev_alloc(c->sweight, g.H * sizeof(double)));
        }
        HIPCHK(c, hipMemcpy(c->smodes, md.data(), g.H * sizeof(short4), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->sweight, wt.data(), g.H * sizeof(double), hipMemcpyHostToDevice));
    }
    if (!c->Stab) {
        HIPCHK(c, dev_alloc(c->Stab, cnt * sizeof(double)));
        HIPCHK(c, dev_alloc(c->Gtab, cnt * sizeof(double)));
        HIPCHK(c, dev_alloc(c->Ktab, cnt * sizeof(double)));
    }
    HIPCHK(c, hipMemcpy(c->Stab, S.data(), cnt * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->Gtab, G.data(), cnt * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->Ktab, K.data(), cnt * sizeof(double), hipMemcpyHostToDevice));
    return SCE_OK;
}

// Tent tables.  The 1-D Gram integrals of tents of half-width dk centred at
// a dk, a = -n..n, have closed forms (c = a dk):
//   B(a,a) = 2 dk / 3,                  B(a,a+1) = dk / 6,
//   A(a,a) = (2/3) c^2 dk + dk^3 / 15,  A(a,a+1) = dk (c^2 / 6 + c dk / 6 + dk^2 / 20),
// zero beyond neighbours (B: int T T, A: int k^2 T T).  The generalised
// eigenproblem A v = lambda B v with V^T B V = I is solved by the Cholesky
// factor B = C C^T, cyclic Jacobi rotations on S = C^-1 A C^-T = W diag(lambda)
// W^T, and V = C^-T W; the tensor products of V then diagonalise the D-D
// matrix sum_d A (x) B (x) B (permuted).
sce_status tent_tables(sce_ctx c)
{
    const int n = c->g.n, M = c->g.M;
    const double dk = kTwoPi / c->L;
    std::vector<double> A((size_t)M * M, 0.0), B((size_t)M * M, 0.0);
    for (int i = 0; i < M; ++i) {
        const double ca = (i - n) * dk;
        B[i * M + i] = 2.0 * dk / 3.0;
        A[i * M + i] = 2.0 / 3.0 * ca * ca * dk + dk * dk * dk / 15.0;
        if (i + 1 < M) {
            B[i * M + i + 1] = B[(i + 1) * M + i] = dk / 6.0;
            A[i * M + i + 1] = A[(i + 1) * M + i] = dk * (ca * ca / 6.0 + ca * dk / 6.0 + dk * dk / 20.0);
        }
    }
    std::vector<double> C((size_t)M * M, 0.0);
    for (int j = 0; j < M; ++j) {
        double d = B[j * M + j];
        for (int k = 0; k < j; ++k) d -= C[j * M + k] * C[j * M + k];
        if (!(d > 0.0)) return fail(c, SCE_EDEVICE, "tent Gram matrix not positive definite");
        C[j * M + j] = std::sqrt(d);
        for (int i = j + 1; i < M; ++i) {
            double s = B[i * M + j];
            for (int k = 0; k < j; ++k) s -= C[i * M + k] * C[j * M + k];
            C[i * M + j] = s / C[j * M + j];
        }
    }
    // Y = C^-1 A, then S = C^-1 Y^T (= C^-1 A C^-T), symmetrised
    std::vector<double> Y((size_t)M * M), S((size_t)M * M), W((size_t)M * M, 0.0);
    for (int col = 0; col < M; ++col)
        for (int i = 0; i < M; ++i) {
            double s = A[i * M + col];
            for (int k = 0; k < i; ++k) s -= C[i * M + k] * Y[k * M + col];
            Y[i * M + col] = s / C[i * M + i];
        }
    for (int col = 0; col < M; ++col)
        for (int i = 0; i < M; ++i) {
            double s = Y[col * M + i];
            for (int k = 0; k < i; ++k) s -= C[i * M + k] * S[k * M + col];
            S[i * M + col] = s / C[i * M + i];
        }
    for (int i = 0; i < M; ++i)
        for (int j = i + 1; j < M; ++j) S[i * M + j] = S[j * M + i] = 0.5 * (S[i * M + j] + S[j * M + i]);
    for (int i = 0; i < M; ++i) W[i * M + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int p = 0; p < M; ++p) {
            dia += S[p * M + p] * S[p * M + p];
            for (int q = p + 1; q < M; ++q) off += S[p * M + q] * S[p * M + q];
        }
        if (off <= 1e-32 * dia) break;
        for (int p = 0; p < M; ++p)
            for (int q = p + 1; q < M; ++q) {
                const double apq = S[p * M + q];
                if (apq == 0.0) continue;
                const double th = (S[q * M + q] - S[p * M + p]) / (2.0 * apq);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < M; ++k) {
                    const double a = S[k * M + p], b = S[k * M + q];
                    S[k * M + p] = cs * a - sn * b;
                    S[k * M + q] = sn * a + cs * b;
                }
                for (int k = 0; k < M; ++k) {
                    const double a = S[p * M + k], b = S[q * M + k];
                    S[p * M + k] = cs * a - sn * b;
                    S[q * M + k] = sn * a + cs * b;
                }
                for (int k = 0; k < M; ++k) {
                    const double a = W[k * M + p], b = W[k * M + q];
                    W[k * M + p] = cs * a - sn * b;
                    W[k * M + q] = sn * a + cs * b;
                }
            }
    }
    std::vector<double> V((size_t)M * M), Vb((size_t)M * M), lam(M);
    for (int i = 0; i < M; ++i) lam[i] = S[i * M + i];
    for (int col = 0; col < M; ++col)
        for (int i = M - 1; i >= 0; --i) {
            double s = W[i * M + col];
            for (int k = i + 1; k < M; ++k) s -= C[k * M + i] * V[k * M + col];
            V[i * M + col] = s / C[i * M + i];
        }
    // check V^T B V = I and V^T A V = diag(lambda)
    double eb = 0.0, ea = 0.0, lmax = 0.0;
    for (int i = 0; i < M; ++i) lmax = std::fmax(lmax, std::fabs(lam[i]));
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            double sb = 0.0, sa = 0.0;
            for (int k = 0; k < M; ++k) {
                double bk = 0.0, ak = 0.0;
                for (int l = std::max(0, k - 1); l <= std::min(M - 1, k + 1); ++l) {
                    bk += B[k * M + l] * V[l * M + j];
                    ak += A[k * M + l] * V[l * M + j];
                }
                sb += V[k * M + i] * bk;
                sa += V[k * M + i] * ak;
            }
            eb = std::fmax(eb, std::fabs(sb - (i == j ? 1.0 : 0.0)));
            ea = std::fmax(ea, std::fabs(sa - (i == j ? lam[i] : 0.0)));
        }
    if (!(eb <= 1e-10 && ea <= 1e-10 * lmax))
        return fail(c, SCE_EDEVICE, "tent eigenbasis check failed");
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) Vb[j * M + i] = V[i * M + j];
    c->env_max = 1.0;
    for (int d = 0; d < c->dim; ++d) c->env_max *= dk / std::sqrt(kTwoPi);
    const size_t cube = (size_t)(c->dim == 2 ? 1 : M) * M * M;
    HIPCHK(c, dev_alloc(c->Vf, (size_t)M * M * sizeof(double)));
    HIPCHK(c, dev_alloc(c->Vb, (size_t)M * M * sizeof(double)));
    HIPCHK(c, dev_alloc(c->lam, (size_t)M * sizeof(double)));
    HIPCHK(c, dev_alloc(c->cubeX, cube * sizeof(double2)));
    HIPCHK(c, dev_alloc(c->cubeY, cube * sizeof(double2)));
    HIPCHK(c, hipMemcpy(c->Vf, V.data(), (size_t)M * M * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->Vb, Vb.data(), (size_t)M * M * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->lam, lam.data(), (size_t)M * sizeof(double), hipMemcpyHostToDevice));
    return SCE_OK;
}

// Buffers whose size depends on the precision (force table, psi0).
sce_status alloc_prec_buffers(sce_ctx c)
{
    c->gen++;
    free_dev(c->ftab);
    free_dev(c->psi0);
    const size_t eb = elem_bytes(c->prec == SCE_PREC_FP64 ? SCE_PREC_FP64 : SCE_PREC_FP32);
    const size_t fbytes = (size_t)c->g.R * c->g.nzp * 8 * eb;
    HIPCHK(c, hipMalloc(&c->ftab, fbytes));
    HIPCHK(c, hipMemset(c->ftab, 0, fbytes));
    HIPCHK(c, hipMalloc(&c->psi0, (size_t)c->g.R * 2 * eb));
    free_dev(c->wf);
    free_devp(c->wscr);
    if (c->prec == SCE_PREC_SPLIT_F16) {
        HIPCHK(c, hipMalloc(&c->wf, sce::force_pack_bytes(c->g)));
        HIPCHK(c, dev_alloc(c->wscr, sce::force_rowinfo_bytes(c->g)));
    }
    return SCE_OK;
}

sce_status ensure_particle_buffers(sce_ctx c, int64_t N)
{
    if (N <= c->cap) return SCE_OK;
    c->gen++;
    // no particles until every buffer of the new size exists
    c->N = 0;
    c->cap = 0;
    c->fields_valid = c->force_valid = c->phi_valid = false;
    free_devp(c->pos);
    free_devp(c->vel);
    free_devp(c->q);
    free_devp(c->m);
    free_devp(c->F);
    free_devp(c->phi);
    free_devp(c->qw);
    free_devp(c->env);
    free_devp(c->Fk);
    free_devp(c->Pk);
    if (c->field == SCE_FIELD_TENT) {
        ALLOCCHK(c, dev_alloc(c->qw, N * sizeof(double)));
        ALLOCCHK(c, dev_alloc(c->env, 4 * N * sizeof(double)));
        ALLOCCHK(c, dev_alloc(c->Fk, 3 * N * sizeof(double)));
        ALLOCCHK(c, dev_alloc(c->Pk, N * sizeof(double)));
    }
    ALLOCCHK(c, dev_alloc(c->pos, 3 * N * sizeof(double)));
    ALLOCCHK(c, dev_alloc(c->vel, 3 * N * sizeof(double)));
    ALLOCCHK(c, dev_alloc(c->q, N * sizeof(double)));
    ALLOCCHK(c, dev_alloc(c->m, N * sizeof(double)));
    ALLOCCHK(c, dev_alloc(c->F, 3 * N * sizeof(double)));
    ALLOCCHK(c, dev_alloc(c->phi, N * sizeof(double)));
    c->cap = N;
    return SCE_OK;
}

sce_status ensure_bytes(sce_ctx c, void *&p, size_t &have, size_t need)
{
    if (need <= have) return SCE_OK;
    c->gen++;
    free_dev(p);
    have = 0;
    ALLOCCHK(c, hipMalloc(&p, need));
    have = need;
    return SCE_OK;
}

hipEvent_t take_event(sce_ctx c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <typename T>
sce_status run_deposit(sce_ctx c, const PassScratch *ps)
{
    const Geom &g = c->g;
    const sce::DepositPlan pl = sce::plan_deposit(g, c->N, (int)sizeof(T));
    void *tab = ps ? ps->tab : nullptr, *tabxy = ps ? ps->tabxy : nullptr;
    double *part = ps ? (double *)ps->part : nullptr;
    if (!ps) {
        sce_status st = ensure_bytes(c, c->tab, c->tab_bytes, (size_t)c->N * 2 * g.zslots * sizeof(T));
        if (st) return st;
        st = ensure_bytes(c, c->tabxy, c->tabxy_bytes, (size_t)c->N * 2 * g.n1 * sizeof(double2));
        if (st) return st;
        size_t pb = c->part_bytes;
        void *pp = c->part;
        st = ensure_bytes(c, pp, pb, (size_t)pl.splits * g.n1 * 4 * g.Rpad * sizeof(double));
        c->part = (double *)pp;
        c->part_bytes = pb;
        if (st) return st;
        tab = c->tab;
        tabxy = c->tabxy;
        part = c->part;
    }
    const bool tent = c->field == SCE_FIELD_TENT;
    if (tent) HIPCHK(c, sce::launch_tent_prep(c->stream, c->pos, c->q, c->N, c->dim, c->L, c->qw, c->env));
    HIPCHK(c, sce::launch_phase_table<T>(c->stream, c->pos, c->N, g, c->L, (double2 *)tabxy,
                                         (T *)tab));
    EventPair ep{nullptr, nullptr};
    if (c->timing && !ps) {
        ep.a = take_event(c);
        ep.b = take_event(c);
        if (ep.a) HIPCHK(c, hipEventRecord(ep.a, c->stream));
    }
    HIPCHK(c, sce::launch_deposit<T>(c->stream, (const double2 *)tabxy, (const T *)tab,
                                     tent ? c->qw : c->q, c->N, g, pl, part));
    if (ep.a && ep.b) {
        HIPCHK(c, hipEventRecord(ep.b, c->stream));
        c->ev_dep.push_back(ep);
    }
    HIPCHK(c, sce::launch_reduce_solve<T>(c->stream, part, pl.splits, g, c->Stab, c->Gtab,
                                          c->Ktab, c->rho, c->psi, (T *)c->ftab, (T *)c->psi0,
                                          c->wpart, &c->wblocks));
    if (tent)
        HIPCHK(c, sce::launch_tent_solve<T>(c->stream, c->rho, g, c->dim, c->Vf, c->Vb, c->lam,
                                            c->eps0, c->cubeX, c->cubeY, c->psi, (T *)c->ftab,
                                            (T *)c->psi0, c->wpart, &c->wblocks));
    c->fields_valid = true;
    return SCE_OK;
}

template <typename T>
sce_status run_force(sce_ctx c, double kick, const PassScratch *ps)
{
    EventPair ep{nullptr, nullptr};
    if (c->timing && !ps) {
        ep.a = take_event(c);
        ep.b = take_event(c);
        if (ep.a) HIPCHK(c, hipEventRecord(ep.a, c->stream));
    }
    const bool tent = c->field == SCE_FIELD_TENT;
    const int lg = sce::force_line_groups(c->g, c->N, (int)sizeof(T));
    double *fscr = ps ? (double *)ps->fscr : c->fscratch;
    if (lg > 1 && !ps) {
        void *fs = c->fscratch;
        sce_status st = ensure_bytes(c, fs, c->fscratch_bytes, (size_t)lg * 4 * c->N * sizeof(double));
        c->fscratch = (double *)fs;
        if (st) return st;
        fscr = c->fscratch;
    }
    HIPCHK(c, sce::launch_force<T>(c->stream, c->pos, c->q, c->m, c->vel, (const T *)c->ftab,
                                   (const T *)c->psi0, c->g, c->L, c->N, tent ? 0.0 : kick,
                                   tent ? c->Fk : c->F, tent ? c->Pk : c->phi, fscr));
    if (ep.a && ep.b) {
        HIPCHK(c, hipEventRecord(ep.b, c->stream));
        c->ev_frc.push_back(ep);
    }
    if (tent)
        HIPCHK(c, sce::launch_tent_combine(c->stream, c->env, c->q, c->m, c->Fk, c->Pk, c->N, kick,
                                           c->vel, c->F, c->phi));
    c->force_valid = true;
    c->phi_valid = true;
    return SCE_OK;
}

sce_status run_deposit_split(sce_ctx c, const PassScratch *ps)
{
    const Geom &g = c->g;
    const sce::MfmaDepositPlan pl = sce::plan_deposit_mfma(g, c->N);
    float *rec = ps ? (float *)ps->rec : nullptr, *part = ps ? (float *)ps->part : nullptr;
    if (!ps) {
        void *tp = c->turns;
        sce_status st = ensure_bytes(c, tp, c->turns_bytes, sce::deposit_mfma_rec_bytes(c->N, g.n));
        c->turns = (double *)tp;
        if (st) return st;
        size_t pb = c->part_bytes;
        void *pp = c->part;
        st = ensure_bytes(c, pp, pb, (size_t)pl.splits * g.n1 * 4 * g.Rpad * sizeof(float));
        c->part = (double *)pp;
        c->part_bytes = pb;
        if (st) return st;
        rec = (float *)c->turns;
        part = (float *)c->part;
    }
    EventPair ep{nullptr, nullptr};
    if (c->timing && !ps) {
        ep.a = take_event(c);
        ep.b = take_event(c);
        if (ep.a) HIPCHK(c, hipEventRecord(ep.a, c->stream));
    }
    const bool tent = c->field == SCE_FIELD_TENT;
    if (tent) HIPCHK(c, sce::launch_tent_prep(c->stream, c->pos, c->q, c->N, c->dim, c->L, c->qw, c->env));
    HIPCHK(c, sce::launch_deposit_mfma(c->stream, c->pos, tent ? c->qw : c->q, c->N, g, c->L, pl,
                                       c->qscale, rec, part));
    if (ep.a && ep.b) {
        HIPCHK(c, hipEventRecord(ep.b, c->stream));
        c->ev_dep.push_back(ep);
    }
    HIPCHK(c, sce::launch_reduce_solve<float>(c->stream, (const float *)part, pl.splits, g, c->Stab, c->Gtab,
                                              c->Ktab, c->rho, c->psi, (float *)c->ftab,
                                              (float *)c->psi0, c->wpart, &c->wblocks));
    if (tent)
        HIPCHK(c, sce::launch_tent_solve<float>(c->stream, c->rho, g, c->dim, c->Vf, c->Vb, c->lam,
                                                c->eps0, c->cubeX, c->cubeY, c->psi,
                                                (float *)c->ftab, (float *)c->psi0, c->wpart,
                                                &c->wblocks));
    HIPCHK(c, sce::launch_force_pack(c->stream, (const float *)c->ftab, (const float *)c->psi0, g,
                                     reinterpret_cast<float4 *>(c->wscr), (_Float16 *)c->wf));
    c->fields_valid = true;
    return SCE_OK;
}

sce_status run_force_split(sce_ctx c, double kick, bool want_phi, const PassScratch *ps,
                           const sce::Drift &nd)
{
    EventPair ep{nullptr, nullptr};
    if (c->timing && !ps) {
        ep.a = take_event(c);
        ep.b = take_event(c);
        if (ep.a) HIPCHK(c, hipEventRecord(ep.a, c->stream));
    }
    const bool tent = c->field == SCE_FIELD_TENT;
    // the next step's half kick and drift ride in the force kernel, but for
    // the tent field, whose force is completed by the combine below
    HIPCHK(c, sce::launch_force_mfma(c->stream, c->pos, c->q, c->m, c->vel, (const _Float16 *)c->wf,
                                     reinterpret_cast<const float4 *>(c->wscr), c->g, c->L, c->N,
                                     tent ? 0.0 : kick, tent ? sce::Drift{} : nd, tent ? c->Fk : c->F,
                                     tent ? c->Pk : (want_phi ? c->phi : nullptr)));
    if (ep.a && ep.b) {
        HIPCHK(c, hipEventRecord(ep.b, c->stream));
        c->ev_frc.push_back(ep);
    }
    if (tent) {
        HIPCHK(c, sce::launch_tent_combine(c->stream, c->env, c->q, c->m, c->Fk, c->Pk, c->N, kick,
                                           c->vel, c->F, c->phi));
        if (nd.kick != 0.0 || nd.drift != 0.0)
            HIPCHK(c, sce::launch_kick_drift(c->stream, c->pos, c->vel, c->F, c->m, c->N, c->L, nd.kick,
                                             nd.drift, nd.wrap != 0));
    }
    c->force_valid = true;
    c->phi_valid = want_phi || tent;
    return SCE_OK;
}

// ps: caller-supplied scratch (sce_force_noalloc), or NULL for the
// context's own buffers, allocated or grown on demand.
sce_status deposit(sce_ctx c, const PassScratch *ps = nullptr)
{
    if (c->prec == SCE_PREC_FP64) return run_deposit<double>(c, ps);
    if (c->prec == SCE_PREC_FP32) return run_deposit<float>(c, ps);
    if (c->prec == SCE_PREC_SPLIT_F16) return run_deposit_split(c, ps);
    return fail(c, SCE_ENOTSUP, "precision not available");
}

// nd: the next leapfrog step's opening half kick and drift, applied after the
// force and its kick (inside the split-precision force kernel, else by a
// kick-drift launch); the fields and force are then those of the positions
// before the drift.
sce_status force(sce_ctx c, double kick, bool want_phi, const PassScratch *ps = nullptr,
                 const sce::Drift &nd = sce::Drift{})
{
    sce_status st;
    if (c->prec == SCE_PREC_SPLIT_F16) {
        st = run_force_split(c, kick, want_phi, ps, nd);
    } else {
        if (c->prec == SCE_PREC_FP64) st = run_force<double>(c, kick, ps);
        else if (c->prec == SCE_PREC_FP32) st = run_force<float>(c, kick, ps);
        else return fail(c, SCE_ENOTSUP, "precision not available");
        if (!st && (nd.kick != 0.0 || nd.drift != 0.0))
            HIPCHK(c, sce::launch_kick_drift(c->stream, c->pos, c->vel, c->F, c->m, c->N, c->L, nd.kick,
                                             nd.drift, nd.wrap != 0));
    }
    if (!st && nd.drift != 0.0) c->fields_valid = c->force_valid = c->phi_valid = false;
    return st;
}

// One pass of the hot path at the current positions: deposit, solve, force
// (+kick, and nd); the potential at the particles too when want_phi.
sce_status pass(sce_ctx c, double kick, bool want_phi = false, const PassScratch *ps = nullptr,
                const sce::Drift &nd = sce::Drift{})
{
    sce_status st = deposit(c, ps);
    if (st) return st;
    return force(c, kick, want_phi, ps, nd);
}

// Bytes of scratch one pass needs at the context's size and precision, laid
// out in ps from base (256-byte aligned pieces).  The deposit's tables and
// partials are dead once the solve has run, so the force's line-group
// partials reuse the same bytes.
size_t pass_scratch_layout(sce_ctx c, char *base, PassScratch *ps)
{
    const Geom &g = c->g;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t dep = 0, frc = 0;
    *ps = PassScratch{nullptr, nullptr, nullptr, nullptr, nullptr};
    if (c->prec == SCE_PREC_SPLIT_F16) {
        const sce::MfmaDepositPlan pl = sce::plan_deposit_mfma(g, c->N);
        const size_t rb = al(sce::deposit_mfma_rec_bytes(c->N, g.n));
        ps->rec = base;
        ps->part = base + rb;
        dep = rb + al((size_t)pl.splits * g.n1 * 4 * g.Rpad * sizeof(float));
    } else {
        const size_t eb = elem_bytes(c->prec);
        const sce::DepositPlan pl = sce::plan_deposit(g, c->N, (int)eb);
        const size_t tb = al((size_t)c->N * 2 * g.zslots * eb);
        const size_t xb = al((size_t)c->N * 2 * g.n1 * sizeof(double2));
        ps->tab = base;
        ps->tabxy = base + tb;
        ps->part = base + tb + xb;
        dep = tb + xb + al((size_t)pl.splits * g.n1 * 4 * g.Rpad * sizeof(double));
        const int lg = sce::force_line_groups(g, c->N, (int)eb);
        if (lg > 1) frc = al((size_t)lg * 4 * c->N * sizeof(double));
        ps->fscr = base;
    }
    return dep > frc ? dep : frc;
}

sce_status check_ready(sce_ctx c)
{
    if (!c) return SCE_EINVAL;
    if (c->broken) return fail(c, SCE_EDEVICE, "context unusable after a device error: " + c->err);
    HIPCHK(c, hipSetDevice(c->device));
    return SCE_OK;
}

sce_status copy_in(sce_ctx c, double *dst, const double *src, size_t bytes, int on_device)
{
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             c->stream));
    if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    return SCE_OK;
}

sce_status copy_out(sce_ctx c, double *dst, const double *src, size_t bytes, int on_device)
{
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
    if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    return SCE_OK;
}

}  // namespace

extern "C" {

const char *sce_status_string(sce_status s)
{
    switch (s) {
    case SCE_OK: return "ok";
    case SCE_EINVAL: return "invalid argument";
    case SCE_ENOMEM: return "out of memory";
    case SCE_EDEVICE: return "device error";
    case SCE_ESTATE: return "invalid state";
    case SCE_ENOTSUP: return "not supported";
    case SCE_EUNSTABLE: return "unstable (non-finite energy)";
    }
    return "unknown status";
}

const char *sce_last_error(sce_ctx c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

namespace {
// Device address of this GPU's static scratch (sce_force_noalloc), taken once
// per device with that device current; the array's name is never used as a
// device address in host code.
hipError_t resolve_noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipSuccess;  // sce_force_noalloc then refuses
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

sce_status create_ctx(double L, int32_t n_max, int32_t shape_kind, double shape_width, int dim,
                      int field, sce_ctx *out)
{
    if (!out) return SCE_EINVAL;
    *out = nullptr;
    if (!(L > 0.0) || !std::isfinite(L)) return SCE_EINVAL;
    if (n_max < 1 || n_max > 64) return SCE_EINVAL;
    if (shape_kind < SCE_SHAPE_DELTA || shape_kind > SCE_SHAPE_TENT) return SCE_EINVAL;
    if (!(shape_width >= 0.0) || !std::isfinite(shape_width)) return SCE_EINVAL;
    sce_ctx c = new (std::nothrow) sce_ctx_s();
    if (!c) return SCE_ENOMEM;
    c->L = L;
    c->kind = shape_kind;
    c->width = shape_width;
    c->dim = dim;
    c->field = field;
    c->g = make_geom(n_max, dim);
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = resolve_noalloc_scratch(c->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        return SCE_EDEVICE;
    }
    c->own_stream = true;
    sce_status st = build_tables(c);
    if (!st && field == SCE_FIELD_TENT) st = tent_tables(c);
    if (!st) {
        const Geom &g = c->g;
        if (dev_alloc(c->rho, g.P * sizeof(double2)) != hipSuccess ||
            dev_alloc(c->psi, g.P * sizeof(double2)) != hipSuccess ||
            dev_alloc(c->wpart, ((size_t)g.n1 * g.R / 64 + 2) * 2 * sizeof(double)) != hipSuccess ||
            dev_alloc(c->dout, 8 * sizeof(double)) != hipSuccess)
            st = SCE_ENOMEM;
    }
    if (!st) st = alloc_prec_buffers(c);
    if (st) {
        sce_destroy(c);
        return st;
    }
    *out = c;
    return SCE_OK;
}
}  // namespace

extern "C" {

sce_status sce_create(double L, int32_t n_max, int32_t shape_kind, double shape_width, sce_ctx *out)
{
    return create_ctx(L, n_max, shape_kind, shape_width, 3, SCE_FIELD_DELTA, out);
}

sce_status sce_create_2d(double L, int32_t n_max, int32_t shape_kind, double shape_width, sce_ctx *out)
{
    return create_ctx(L, n_max, shape_kind, shape_width, 2, SCE_FIELD_DELTA, out);
}

sce_status sce_create_tent(double L, int32_t n_max, int32_t dim, sce_ctx *out)
{
    if (dim != 2 && dim != 3) {
        if (out) *out = nullptr;
        return SCE_EINVAL;
    }
    return create_ctx(L, n_max, SCE_SHAPE_DELTA, 0.0, dim, SCE_FIELD_TENT, out);
}

sce_status sce_field_shape(sce_ctx c, int32_t *field)
{
    if (!c || !field) return SCE_EINVAL;
    *field = c->field;
    return SCE_OK;
}

sce_status sce_dimension(sce_ctx c, int32_t *dim)
{
    if (!c || !dim) return SCE_EINVAL;
    *dim = c->dim;
    return SCE_OK;
}

sce_status sce_set_options(sce_ctx c, double eps0, int32_t precision, int32_t scheme, void *hip_stream)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (!(eps0 > 0.0) || !std::isfinite(eps0)) return fail(c, SCE_EINVAL, "eps0 must be finite and > 0");
    if (precision < SCE_PREC_FP64 || precision > SCE_PREC_SPLIT_F16)
        return fail(c, SCE_EINVAL, "unknown precision");
    if (scheme != SCE_SCHEME_KDK && scheme != SCE_SCHEME_DKD) return fail(c, SCE_EINVAL, "unknown scheme");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const bool prec_changed = precision != c->prec;
    const bool eps_changed = eps0 != c->eps0;
    c->eps0 = eps0;
    c->prec = precision;
    c->scheme = scheme;
    if (hip_stream) {
        if (c->own_stream) HIPCHK(c, hipStreamDestroy(c->stream));
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    }
    if (eps_changed) {
        st = build_tables(c);
        if (st) return st;
    }
    if (prec_changed) {
        st = alloc_prec_buffers(c);
        if (st) return st;
        free_dev(c->tab);
        c->tab_bytes = 0;
    }
    c->fields_valid = c->force_valid = false;
    c->gen++;  // precision, stream and tables are captured by a step graph
    return SCE_OK;
}

sce_status sce_set_particles(sce_ctx c, int64_t N, const double *x, const double *v,
                             const double *q, const double *m, int32_t on_device)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (N < 1) return fail(c, SCE_EINVAL, "N must be >= 1");
    // the deposit's visiting order is a permutation of 32-bit indices (and
    // 2^32 particles would not fit in device memory anyway)
    if (N > (int64_t)0xFFFFFFFF) return fail(c, SCE_EINVAL, "N must be below 2^32");
    if (!x || !v || !q || !m) return fail(c, SCE_EINVAL, "NULL particle array");
    st = ensure_particle_buffers(c, N);
    if (st) return st;
    c->N = N;
    if (c->dim == 2) {
        // [2][N] in, stored as (0, x, y)
        HIPCHK(c, hipMemsetAsync(c->pos, 0, N * sizeof(double), c->stream));
        HIPCHK(c, hipMemsetAsync(c->vel, 0, N * sizeof(double), c->stream));
        if ((st = copy_in(c, c->pos + N, x, 2 * N * sizeof(double), on_device))) return st;
        if ((st = copy_in(c, c->vel + N, v, 2 * N * sizeof(double), on_device))) return st;
    } else {
        if ((st = copy_in(c, c->pos, x, 3 * N * sizeof(double), on_device))) return st;
        if ((st = copy_in(c, c->vel, v, 3 * N * sizeof(double), on_device))) return st;
    }
    if ((st = copy_in(c, c->q, q, N * sizeof(double), on_device))) return st;
    if ((st = copy_in(c, c->m, m, N * sizeof(double), on_device))) return st;
    // reject non-finite values and non-positive masses before anything uses them
    unsigned *flag = reinterpret_cast<unsigned *>(c->dout);
    unsigned bad = 0;
    HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(unsigned), c->stream));
    HIPCHK(c, sce::launch_check_particles(c->stream, c->pos, c->vel, c->q, c->m, N, flag));
    if (c->field != SCE_FIELD_TENT) HIPCHK(c, sce::launch_wrap(c->stream, c->pos, N, c->L));
    // sum q^2 for the self-energy (host copy of q)
    std::vector<double> hq(N);
    HIPCHK(c, hipMemcpyAsync(hq.data(), c->q, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&bad, flag, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad) {
        c->N = 0;
        c->gen++;
        c->fields_valid = c->force_valid = c->phi_valid = false;
        return fail(c, SCE_EINVAL, (bad & 1) ? "non-finite position, velocity or charge"
                                             : "every mass must be finite and > 0");
    }
    double s = 0.0, qmax = 0.0;
    for (double v_ : hq) {
        s += v_ * v_;
        qmax = std::fmax(qmax, std::fabs(v_));
    }
    c->q2sum = s;
    c->qscale = qmax > 0.0 ? qmax : 1.0;
    if (c->field == SCE_FIELD_TENT) c->qscale *= c->env_max;  // the deposit takes q E, E <= E(0)
    c->gen++;  // N, qscale and the particle buffers are captured by a step graph
    c->step = 0;
    c->time = 0.0;
    c->fields_valid = c->force_valid = false;
    return SCE_OK;
}

sce_status sce_get_particles(sce_ctx c, double *x, double *v, int32_t on_device)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (c->N < 1) return fail(c, SCE_ESTATE, "no particles set");
    const int64_t off = c->dim == 2 ? c->N : 0;
    const size_t bytes = (size_t)c->dim * c->N * sizeof(double);
    if (x && (st = copy_out(c, x, c->pos + off, bytes, on_device))) return st;
    if (v && (st = copy_out(c, v, c->vel + off, bytes, on_device))) return st;
    return SCE_OK;
}

sce_status sce_mode_count(sce_ctx c, int64_t *n_half)
{
    if (!c || !n_half) return SCE_EINVAL;
    *n_half = export_count(c);
    return SCE_OK;
}

sce_status sce_modes(sce_ctx c, int32_t *nxyz)
{
    if (!c || !nxyz) return SCE_EINVAL;
    const Geom &g = c->g;
    int64_t i = 0;
    for (int r = 0; r < g.R; ++r) {
        int nx, ny;
        sce::row_nxny(r, g.n, nx, ny);
        for (int nz = -g.n; nz <= g.n; ++nz) {
            const bool origin = nx == 0 && ny == 0 && nz == 0 && c->field == SCE_FIELD_TENT;
            if (!sce::in_half(nx, ny, nz) && !origin) continue;
            if (c->dim == 2) {
                nxyz[2 * i] = ny;
                nxyz[2 * i + 1] = nz;
            } else {
                nxyz[3 * i] = nx;
                nxyz[3 * i + 1] = ny;
                nxyz[3 * i + 2] = nz;
            }
            ++i;
        }
    }
    return i == export_count(c) ? SCE_OK : fail(c, SCE_EDEVICE, "mode count mismatch");
}

sce_status sce_deposit(sce_ctx c, double *rho, int32_t on_device)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (c->N < 1) return fail(c, SCE_ESTATE, "no particles set");
    if ((st = deposit(c))) return st;
    if (rho)
        return copy_out(c, rho, (const double *)(c->rho + export_first(c)),
                        export_count(c) * sizeof(double2), on_device);
    return SCE_OK;
}

sce_status sce_psi(sce_ctx c, double *psi, int32_t on_device)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (!c->fields_valid) return fail(c, SCE_ESTATE, "no current deposit");
    if (!psi) return fail(c, SCE_EINVAL, "NULL psi");
    return copy_out(c, psi, (const double *)(c->psi + export_first(c)),
                    export_count(c) * sizeof(double2), on_device);
}

sce_status sce_force(sce_ctx c, double *F, int32_t on_device)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (c->N < 1) return fail(c, SCE_ESTATE, "no particles set");
    if ((st = pass(c, 0.0))) return st;
    if (F)
        return copy_out(c, F, c->F + (c->dim == 2 ? c->N : 0), (size_t)c->dim * c->N * sizeof(double),
                        on_device);
    return SCE_OK;
}

sce_status sce_force_noalloc(sce_ctx c, double *F, int32_t on_device)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (c->N < 1) return fail(c, SCE_ESTATE, "no particles set");
    void *base = nullptr;
    if (c->device >= 0 && c->device < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch_ptr[c->device];
    }
    if (!base) return fail(c, SCE_ENOTSUP, "no static scratch on this device");
    PassScratch ps;
    const size_t need = pass_scratch_layout(c, (char *)base, &ps);
    if (need > kNoallocScratchBytes)
        return fail(c, SCE_EINVAL, "this pass needs " + std::to_string(need) +
                                       " bytes of scratch, above the static " +
                                       std::to_string(kNoallocScratchBytes) + " bytes");
    if ((st = pass(c, 0.0, false, &ps))) return st;
    if (F)
        return copy_out(c, F, c->F + (c->dim == 2 ? c->N : 0), (size_t)c->dim * c->N * sizeof(double),
                        on_device);
    return SCE_OK;
}

}  // extern "C"

namespace {

// k >= 1 kick-drift-kick steps: their launches on the context's stream.  A
// step's closing half kick and the next step's opening half kick and drift
// run in one pass after the force (same operations, same order as separate
// launches, so the states are bit for bit those of k single steps); the
// velocities are at an integer step only after the last one.
sce_status steps_kdk(sce_ctx c, double dt, int64_t k)
{
    sce_status st;
    const bool wrap = c->field != SCE_FIELD_TENT;
    if (!c->force_valid && (st = pass(c, 0.0))) return st;
    HIPCHK(c, sce::launch_kick_drift(c->stream, c->pos, c->vel, c->F, c->m, c->N, c->L, 0.5 * dt, dt, wrap));
    c->fields_valid = c->force_valid = c->phi_valid = false;
    sce::Drift nd;
    nd.kick = 0.5 * dt;
    nd.drift = dt;
    nd.wrap = wrap ? 1 : 0;
    for (int64_t i = 1; i < k; ++i)
        if ((st = pass(c, 0.5 * dt, false, nullptr, nd))) return st;
    if ((st = pass(c, 0.5 * dt))) return st;
    c->step += k;
    c->time += k * dt;
    return SCE_OK;
}

// One leapfrog step: its launches on the context's stream.
sce_status step_once(sce_ctx c, double dt)
{
    sce_status st;
    const bool wrap = c->field != SCE_FIELD_TENT;
    if (c->scheme == SCE_SCHEME_KDK) {
        return steps_kdk(c, dt, 1);
    } else {
        HIPCHK(c, sce::launch_kick_drift(c->stream, c->pos, c->vel, c->F, c->m, c->N, c->L,
                                         0.0, 0.5 * dt, wrap));
        if ((st = pass(c, dt))) return st;
        HIPCHK(c, sce::launch_kick_drift(c->stream, c->pos, c->vel, c->F, c->m, c->N, c->L,
                                         0.0, 0.5 * dt, wrap));
        c->fields_valid = c->force_valid = false;
    }
    c->step += 1;
    c->time += dt;
    return SCE_OK;
}

void drop_graph(sce_ctx c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->g_len = 0;
}

// Capture graph_steps steps of size dt into an executable graph.  The steps
// must have run once already (every buffer exists, the KDK force is
// current), so the captured launches are exactly those of a replayed step.
// No memset and no host synchronisation is recorded: a step is kernel
// launches only.
sce_status capture_steps(sce_ctx c, double dt)
{
    drop_graph(c);
    const int64_t step0 = c->step;
    const double time0 = c->time;
    const bool fv = c->fields_valid, cv = c->force_valid, pv = c->phi_valid;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    sce_status st = SCE_OK;
    if (c->scheme == SCE_SCHEME_KDK)
        st = steps_kdk(c, dt, c->graph_steps);
    else
        for (int i = 0; i < c->graph_steps && !st; ++i) st = step_once(c, dt);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->step = step0;
    c->time = time0;
    // flags as after the captured steps; restored if the capture fails
    if (st || e != hipSuccess) {
        c->fields_valid = fv;
        c->force_valid = cv;
        c->phi_valid = pv;
        if (g) (void)hipGraphDestroy(g);
        if (st) return st;
        return hipfail(c, e, "hipStreamEndCapture");
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hipfail(c, ei, "hipGraphInstantiate");
    }
    c->graph = g;
    c->gexec = x;
    c->g_gen = c->gen;
    c->g_dt = dt;
    c->g_scheme = c->scheme;
    c->g_len = c->graph_steps;
    return SCE_OK;
}

}  // namespace

extern "C" {

sce_status sce_step(sce_ctx c, double dt, int64_t n_steps)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (c->N < 1) return fail(c, SCE_ESTATE, "no particles set");
    if (!std::isfinite(dt)) return fail(c, SCE_EINVAL, "dt must be finite");
    if (n_steps < 0) return fail(c, SCE_EINVAL, "n_steps must be >= 0");
    if (c->smodes && c->field == SCE_FIELD_DELTA && c->prec == SCE_PREC_FP64 && !c->timing &&
        n_steps > 0 && c->N <= sce::kSmallMaxN && c->N * 3 * (c->g.n + 1) <= sce::kSmallMaxTab &&
        c->N * c->g.H <= c->small_max_pairs) {
        const bool kdk = c->scheme == SCE_SCHEME_KDK;
        if (kdk && !c->force_valid && (st = pass(c, 0.0))) return st;
        for (int64_t s = 0; s < n_steps;) {
            const int chunk = (int)std::min<int64_t>(n_steps - s, 4096);
            HIPCHK(c, sce::launch_step_small(c->stream, c->pos, c->vel, c->F, c->q, c->m, c->N,
                                             c->smodes, c->sweight, c->g, c->L, dt, chunk, kdk));
            s += chunk;
            c->step += chunk;
            c->time += chunk * dt;
        }
        c->fields_valid = false;
        c->force_valid = kdk;
        c->phi_valid = false;
        return SCE_OK;
    }
    int64_t s = 0;
    const int G = c->graph_steps;
    if (G > 0 && !c->timing && n_steps >= 2 * (int64_t)G) {
        if ((st = step_once(c, dt))) return st;
        ++s;
        if (!(c->gexec && c->g_gen == c->gen && c->g_dt == dt && c->g_scheme == c->scheme &&
              c->g_len == G)) {
            if ((st = capture_steps(c, dt))) return st;
        }
        for (; n_steps - s >= G; s += G) {
            HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
            c->step += G;
            c->time += G * dt;
        }
    }
    if (s < n_steps && c->scheme == SCE_SCHEME_KDK) return steps_kdk(c, dt, n_steps - s);
    for (; s < n_steps; ++s)
        if ((st = step_once(c, dt))) return st;
    return SCE_OK;
}

sce_status sce_set_small_step(sce_ctx c, int64_t max_pairs)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (max_pairs < 0 || max_pairs > ((int64_t)1 << 24))
        return fail(c, SCE_EINVAL, "max_pairs must be in 0..2^24");
    c->small_max_pairs = max_pairs;
    return SCE_OK;
}

sce_status sce_set_step_graph(sce_ctx c, int32_t steps_per_graph)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (steps_per_graph < 0 || steps_per_graph > 4096)
        return fail(c, SCE_EINVAL, "steps_per_graph must be in 0..4096");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->graph_steps = steps_per_graph;
    return SCE_OK;
}

sce_status sce_diagnostics(sce_ctx c, sce_diag *out, double *rho_abs)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (!out) return fail(c, SCE_EINVAL, "NULL output");
    if (c->N < 1) return fail(c, SCE_ESTATE, "no particles set");
    if (!(c->force_valid && c->fields_valid && c->phi_valid) && (st = pass(c, 0.0, true))) return st;
    const int nb = (int)((c->N + 255) / 256);
    void *ds = c->dscratch;
    st = ensure_bytes(c, ds, c->dscratch_bytes, (size_t)nb * 6 * sizeof(double));
    c->dscratch = (double *)ds;
    if (st) return st;
    HIPCHK(c, sce::launch_diag(c->stream, c->vel, c->q, c->m, c->phi, c->N, c->wpart, c->wblocks,
                               c->eps0 * box_measure(c), c->dscratch, c->dout));
    double h[8];
    HIPCHK(c, hipMemcpyAsync(h, c->dout, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out->step = c->step;
    out->time = c->time;
    out->kinetic = h[0];
    if (c->dim == 2) {
        out->momentum[0] = h[2];
        out->momentum[1] = h[3];
        out->momentum[2] = 0.0;
    } else {
        out->momentum[0] = h[1];
        out->momentum[1] = h[2];
        out->momentum[2] = h[3];
    }
    out->momentum_abs_sum = h[4];
    out->interaction = h[5];
    out->field = h[6];
    out->rho_abs_max = h[7];
    out->field_self = c->field == SCE_FIELD_TENT ? 0.0 : c->q2sum / (c->eps0 * box_measure(c)) * c->self_sum;
    out->total = out->kinetic + out->field;
    if (rho_abs) {
        const int64_t cnt = export_count(c);
        std::vector<double2> r(cnt);
        HIPCHK(c, hipMemcpyAsync(r.data(), c->rho + export_first(c), cnt * sizeof(double2),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < cnt; ++i) rho_abs[i] = std::hypot(r[i].x, r[i].y);
    }
    if (!std::isfinite(out->total)) return fail(c, SCE_EUNSTABLE, "non-finite energy");
    return SCE_OK;
}

namespace {
struct StateHeader {
    uint64_t magic;
    int64_t N;
    int64_t step;
    double time;
    double L;
    int32_t n_max;
    int32_t has_force;
    int32_t dim;
    int32_t field;
    int32_t kind;
    int32_t prec;
    double width;
    double eps0;
};
const uint64_t kMagic = 0x33454353484b5053ull;  // "SPKHSCE3"
}  // namespace

sce_status sce_get_state(sce_ctx c, void *buf, size_t *bytes)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (!bytes) return fail(c, SCE_EINVAL, "NULL size");
    if (c->N < 1) return fail(c, SCE_ESTATE, "no particles set");
    const size_t need = sizeof(StateHeader) + (size_t)c->N * 11 * sizeof(double);
    if (!buf) {
        *bytes = need;
        return SCE_OK;
    }
    if (*bytes < need) return fail(c, SCE_EINVAL, "buffer too small");
    StateHeader hd{kMagic, c->N, c->step, c->time, c->L, c->g.n, c->force_valid ? 1 : 0, c->dim,
                   c->field, c->kind, c->prec, c->width, c->eps0};
    std::memcpy(buf, &hd, sizeof(hd));
    double *d = (double *)((char *)buf + sizeof(hd));
    const size_t n3 = 3 * c->N * sizeof(double), n1 = c->N * sizeof(double);
    HIPCHK(c, hipMemcpyAsync(d, c->pos, n3, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(d + 3 * c->N, c->vel, n3, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(d + 6 * c->N, c->q, n1, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(d + 7 * c->N, c->m, n1, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(d + 8 * c->N, c->F, n3, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *bytes = need;
    return SCE_OK;
}

sce_status sce_set_state(sce_ctx c, const void *buf, size_t bytes)
{
    sce_status st = check_ready(c);
    if (st) return st;
    if (!buf || bytes < sizeof(StateHeader)) return fail(c, SCE_EINVAL, "bad checkpoint");
    StateHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (hd.magic != kMagic || hd.N < 1 || hd.L != c->L || hd.n_max != c->g.n || hd.dim != c->dim ||
        hd.field != c->field ||
        bytes < sizeof(hd) + (size_t)hd.N * 11 * sizeof(double))
        return fail(c, SCE_EINVAL, "checkpoint does not match this context");
    const double *d = (const double *)((const char *)buf + sizeof(hd));
    const int64_t N = hd.N;
    // the arrays are stored as (x, y, z); a 2-D context takes its (x, y) = stored (y, z)
    const int64_t off = c->dim == 2 ? N : 0;
    if ((st = sce_set_particles(c, N, d + off, d + 3 * N + off, d + 6 * N, d + 7 * N, 0))) return st;
    // the saved force belongs to the saved field: reuse it only when the shape,
    // its width, eps0 and the precision match; otherwise the next step
    // recomputes it
    const bool same_field = hd.kind == c->kind && hd.width == c->width && hd.eps0 == c->eps0 &&
                            hd.prec == c->prec;
    if (hd.has_force && same_field) {
        if ((st = copy_in(c, c->F, d + 8 * N, 3 * N * sizeof(double), 0))) return st;
        c->force_valid = true;
    }
    c->step = hd.step;
    c->time = hd.time;
    return SCE_OK;
}

sce_status sce_sync(sce_ctx c)
{
    sce_status st = check_ready(c);
    if (st) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SCE_OK;
}

sce_status sce_timing_enable(sce_ctx c, int32_t enable)
{
    sce_status st = check_ready(c);
    if (st) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->ev_dep) { c->ev_pool.push_back(p.a); c->ev_pool.push_back(p.b); }
    for (auto &p : c->ev_frc) { c->ev_pool.push_back(p.a); c->ev_pool.push_back(p.b); }
    c->ev_dep.clear();
    c->ev_frc.clear();
    c->timing = enable != 0;
    return SCE_OK;
}

sce_status sce_timing_read(sce_ctx c, double *deposit_ms, int64_t *deposit_launches,
                           double *force_ms, int64_t *force_launches)
{
    sce_status st = check_ready(c);
    if (st) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double td = 0.0, tf = 0.0;
    for (auto &p : c->ev_dep) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, p.a, p.b));
        td += ms;
    }
    for (auto &p : c->ev_frc) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, p.a, p.b));
        tf += ms;
    }
    if (deposit_ms) *deposit_ms = td;
    if (force_ms) *force_ms = tf;
    if (deposit_launches) *deposit_launches = (int64_t)c->ev_dep.size();
    if (force_launches) *force_launches = (int64_t)c->ev_frc.size();
    return SCE_OK;
}

void sce_destroy(sce_ctx c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto &p : c->ev_dep) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto &p : c->ev_frc) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    drop_graph(c);
    free_devp(c->pos);
    free_devp(c->vel);
    free_devp(c->q);
    free_devp(c->m);
    free_devp(c->F);
    free_devp(c->phi);
    free_dev(c->tab);
    free_dev(c->tabxy);
    free_devp(c->part);
    free_devp(c->Stab);
    free_devp(c->Gtab);
    free_devp(c->Ktab);
    free_devp(c->rho);
    free_devp(c->psi);
    free_dev(c->ftab);
    free_dev(c->psi0);
    free_dev(c->wf);
    free_devp(c->wscr);
    free_devp(c->turns);
    free_devp(c->wpart);
    free_devp(c->dscratch);
    free_devp(c->fscratch);
    free_devp(c->dout);
    free_devp(c->qw);
    free_devp(c->env);
    free_devp(c->Fk);
    free_devp(c->Pk);
    free_devp(c->cubeX);
    free_devp(c->cubeY);
    free_devp(c->Vf);
    free_devp(c->Vb);
    free_devp(c->lam);
    free_devp(c->smodes);
    free_devp(c->sweight);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
