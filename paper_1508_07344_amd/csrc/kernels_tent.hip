// Finite-width field shapes: tents Psi in k-space with point particles
// (Sections 3 and 4 of the paper).  The potential is expanded over
// f_s(x) = e^{i k_s.x} E(x), s in the full cube {-n..n}^D (s = 0 included),
// with the envelope E(x) = prod_d (2 pi)^(-1/2) dk sinc^2(dk x_d / 2).  So
//   deposit  rho_s = sum_j q_j E(x_j) e^{-i k_s.x_j}   (the ordinary type-1
//            sum with charges q_j E(x_j): the existing deposit kernels),
//   solve    M phi_s = rho_s / eps0, M_st = int |k|^2 Psi(k - k_s) Psi(k - k_t) dk
//            (the paper's K with the second index negated; M separates per
//            axis into tridiagonal 1-D matrices A (|k|^2-weighted) and B),
//   force    F_j = E_j F'_j - q_j grad E(x_j) P_j,  Phi_j = E_j P_j, where
//            F'_j = -q_j sum_s phi_s i k_s e^{i k_s.x_j} and
//            P_j = sum_s phi_s e^{i k_s.x_j} come from the existing force
//            kernels run on phi (zero mode stored as phi_0 / 2 in the force
//            table, so that the doubled half-space sum returns phi_0 once).
// The solve is exact: with V the B-orthonormal eigenvectors of A (A V = B V
// Lambda, V^T B V = I), M^-1 = V^(xD) diag(1 / sum_d lambda_d) V^T(xD), applied
// as D passes of V^T along the axes, a diagonal scale, and D passes of V.
//
// Cube layout: X[(a M + b) M + c], a = n_x + n (extent M in 3-D, 1 in 2-D where
// n_x = 0), b = n_y + n, c = n_z + n; complex FP64.

#include <hip/hip_runtime.h>

#include "sce_device.h"
#include "sce_internal.h"

namespace sce {

namespace {

constexpr double kTwoPiT = 6.283185307179586476925286766559;

// sinc(u) = sin(u) / u and its derivative (cos u - sinc u) / u; below
// |u| = 0.1 that difference cancels, so both come from their Taylor series
// (terms through u^12, truncation below 1e-22).
__device__ inline void sinc_d(double u, double &s, double &ds)
{
    if (fabs(u) < 0.1) {
        const double v = u * u;
        s = 1.0 + v * (-1.0 / 6 + v * (1.0 / 120 + v * (-1.0 / 5040 + v * (1.0 / 362880 +
            v * (-1.0 / 39916800 + v * (1.0 / 6227020800.0))))));
        ds = u * (-1.0 / 3 + v * (1.0 / 30 + v * (-1.0 / 840 + v * (1.0 / 45360 +
             v * (-1.0 / 3991680 + v * (1.0 / 518918400.0))))));
        return;
    }
    double sn, cs;
    sincos(u, &sn, &cs);
    s = sn / u;
    ds = (cs - s) / u;
}

}  // namespace

// Envelope, its gradient and the weighted charges.  env [4][N]: E, dE/dx,
// dE/dy, dE/dz; a 2-D context (stored x = 0) spans only y and z.
__global__ void __launch_bounds__(256)
k_tent_prep(const double *__restrict__ pos, const double *__restrict__ q, int64_t N, int dim,
            double dk, double *__restrict__ qw, double *__restrict__ env)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const double c = dk * 0.3989422804014326779399460599343819;  // dk / sqrt(2 pi)
    double e[3], de[3];
    for (int d = 0; d < 3; ++d) {
        if (d == 0 && dim == 2) {
            e[0] = 1.0;
            de[0] = 0.0;
            continue;
        }
        double s, ds;
        sinc_d(0.5 * dk * pos[d * N + j], s, ds);
        e[d] = c * s * s;
        de[d] = c * 2.0 * s * ds * 0.5 * dk;
    }
    const double E = e[0] * e[1] * e[2];
    env[j] = E;
    env[N + j] = de[0] * e[1] * e[2];
    env[2 * N + j] = e[0] * de[1] * e[2];
    env[3 * N + j] = e[0] * e[1] * de[2];
    qw[j] = q[j] * E;
}

// Full cube from the stored rows: a mode outside the stored half is the
// conjugate of its mirror image.
__global__ void __launch_bounds__(256)
k_tent_expand(const double2 *__restrict__ rho, int n, int Ma, double2 *__restrict__ X)
{
    const int M = 2 * n + 1;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)Ma * M * M) return;
    const int c = (int)(idx % M);
    const int b = (int)((idx / M) % M);
    const int a = (int)(idx / ((int64_t)M * M));
    int nx = Ma == 1 ? 0 : a - n, ny = b - n, nz = c - n;
    bool mirror = nx < 0 || (nx == 0 && ny < 0);
    if (mirror) {
        nx = -nx;
        ny = -ny;
        nz = -nz;
    }
    const int row = nx == 0 ? ny : (n + 1) + (nx - 1) * M + (ny + n);
    double2 v = rho[(int64_t)row * M + nz + n];
    if (mirror) v.y = -v.y;
    X[idx] = v;
}

// Y = Q applied along one axis: Y[.., i, ..] = sum_j Q[j M + i] X[.., j, ..].
// With lam != nullptr the result is divided by eps0 (lam_a + lam_b + lam_c)
// (lam_a left out in 2-D).
__global__ void __launch_bounds__(256)
k_tent_axis(const double2 *__restrict__ X, double2 *__restrict__ Y, const double *__restrict__ Q,
            int n, int Ma, int axis, const double *__restrict__ lam, double eps0)
{
    const int M = 2 * n + 1;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)Ma * M * M) return;
    const int c = (int)(idx % M);
    const int b = (int)((idx / M) % M);
    const int a = (int)(idx / ((int64_t)M * M));
    int i;
    int64_t base, stride;
    if (axis == 0) {
        i = a;
        base = (int64_t)b * M + c;
        stride = (int64_t)M * M;
    } else if (axis == 1) {
        i = b;
        base = (int64_t)a * M * M + c;
        stride = M;
    } else {
        i = c;
        base = ((int64_t)a * M + b) * M;
        stride = 1;
    }
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < M; ++j) {
        const double w = Q[j * M + i];
        const double2 x = X[base + j * stride];
        sr = fma(w, x.x, sr);
        si = fma(w, x.y, si);
    }
    if (lam) {
        const double d = eps0 * ((Ma == 1 ? 0.0 : lam[a]) + lam[b] + lam[c]);
        sr /= d;
        si /= d;
    }
    Y[idx] = make_double2(sr, si);
}

// Stored rows from the solved cube: psi on the padded layout (phi on the
// stored half and at the origin, zero elsewhere), the force table in the
// layout of the reduce/solve kernel (origin entered as phi_0 / 2), and the
// per-block partials of W = (1/2) sum_s phi_s conj(rho_s) over the cube and
// of max |rho|.
template <typename T>
__global__ void __launch_bounds__(256)
k_tent_pack(const double2 *__restrict__ X, const double2 *__restrict__ rho, int n, int R, int Ma,
            int nzp, double2 *__restrict__ psi, T *__restrict__ ftab, T *__restrict__ psi0,
            double *__restrict__ wpart)
{
    __shared__ double sh[8];
    const int n1 = n + 1, M = 2 * n + 1;
    const int64_t cell = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double w = 0.0, amax = 0.0;
    if (cell < (int64_t)n1 * R) {
        const int nz = (int)(cell / R);
        const int row = (int)(cell - (int64_t)nz * R);
        int nx, ny;
        row_nxny(row, n, nx, ny);
        const int64_t cb = ((int64_t)(Ma == 1 ? 0 : nx + n) * M + (ny + n)) * M + n;
        const int64_t rb = (int64_t)row * M + n;
        const bool origin = nx == 0 && ny == 0 && nz == 0;
        const bool hp = in_half(nx, ny, nz);
        const bool hm = nz > 0 && in_half(nx, ny, -nz);
        const double2 fp = X[cb + nz], fm = X[cb - nz];
        const double2 rp = rho[rb + nz], rm = rho[rb - nz];
        const double2 pp = (hp || origin) ? fp : make_double2(0.0, 0.0);
        const double2 pm = hm ? fm : make_double2(0.0, 0.0);
        psi[rb + nz] = pp;
        if (nz > 0) psi[rb - nz] = pm;
        if (hp) {
            w += fp.x * rp.x + fp.y * rp.y;
            amax = fmax(amax, sqrt(rp.x * rp.x + rp.y * rp.y));
        }
        if (hm) {
            w += fm.x * rm.x + fm.y * rm.y;
            amax = fmax(amax, sqrt(rm.x * rm.x + rm.y * rm.y));
        }
        if (origin) {
            w += 0.5 * (fp.x * rp.x + fp.y * rp.y);
            amax = fmax(amax, sqrt(rp.x * rp.x + rp.y * rp.y));
        }
        if (nz == 0) {
            const double h = origin ? 0.5 : 1.0;
            psi0[2 * row] = (T)(h * pp.x);
            psi0[2 * row + 1] = (T)(h * pp.y);
        } else {
            T *f = ftab + ((int64_t)row * nzp + (nz - 1)) * 8;
            const double sr = pp.x + pm.x, si = pp.y + pm.y;
            const double dr = pp.x - pm.x, di = pp.y - pm.y;
            f[0] = (T)sr;
            f[1] = (T)si;
            f[2] = (T)dr;
            f[3] = (T)di;
            f[4] = (T)(nz * dr);
            f[5] = (T)(nz * di);
            f[6] = (T)(nz * sr);
            f[7] = (T)(nz * si);
        }
    }
    // fixed-order block reductions (deterministic)
    for (int o = 32; o > 0; o >>= 1) {
        w += __shfl_xor(w, o, 64);
        amax = fmax(amax, __shfl_xor(amax, o, 64));
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[wv] = w;
        sh[4 + wv] = amax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        wpart[2 * blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        wpart[2 * blockIdx.x + 1] = fmax(fmax(sh[4], sh[5]), fmax(sh[6], sh[7]));
    }
}

// F_j = E_j F'_j - q_j grad E_j P_j, Phi_j = E_j P_j; optional kick v += a F / m.
__global__ void __launch_bounds__(256)
k_tent_combine(const double *__restrict__ env, const double *__restrict__ q,
               const double *__restrict__ m, const double *__restrict__ Fk,
               const double *__restrict__ Pk, int64_t N, double kick, double *__restrict__ vel,
               double *__restrict__ F, double *__restrict__ phi)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const double E = env[j], P = Pk[j], qj = q[j];
    double f[3];
    for (int d = 0; d < 3; ++d) f[d] = E * Fk[d * N + j] - qj * env[(d + 1) * N + j] * P;
    for (int d = 0; d < 3; ++d) F[d * N + j] = f[d];
    phi[j] = E * P;
    if (kick != 0.0) {
        const double a = kick / m[j];
        for (int d = 0; d < 3; ++d) vel[d * N + j] += a * f[d];
    }
}

hipError_t launch_tent_prep(hipStream_t s, const double *pos, const double *q, int64_t N, int dim,
                            double L, double *qw, double *env)
{
    const int64_t blocks = (N + 255) / 256;
    hipLaunchKernelGGL(k_tent_prep, dim3((unsigned)blocks), dim3(256), 0, s, pos, q, N, dim,
                       kTwoPiT / L, qw, env);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tent_solve(hipStream_t s, const double2 *rho, const Geom &g, int dim,
                             const double *Vf, const double *Vb, const double *lam, double eps0,
                             double2 *X, double2 *Y, double2 *psi, T *ftab, T *psi0,
                             double *wpart, int *wblocks)
{
    const int Ma = dim == 2 ? 1 : g.M;
    const int64_t cells = (int64_t)Ma * g.M * g.M;
    const unsigned cb = (unsigned)((cells + 255) / 256);
    hipLaunchKernelGGL(k_tent_expand, dim3(cb), dim3(256), 0, s, rho, g.n, Ma, X);
    // forward: V^T along each axis, the last pass divides by eps0 sum lambda
    const int first = dim == 2 ? 1 : 0;
    double2 *src = X, *dst = Y;
    for (int ax = first; ax < 3; ++ax) {
        hipLaunchKernelGGL(k_tent_axis, dim3(cb), dim3(256), 0, s, src, dst, Vf, g.n, Ma, ax,
                           ax == 2 ? lam : nullptr, eps0);
        double2 *t = src;
        src = dst;
        dst = t;
    }
    for (int ax = first; ax < 3; ++ax) {
        hipLaunchKernelGGL(k_tent_axis, dim3(cb), dim3(256), 0, s, src, dst, Vb, g.n, Ma, ax,
                           nullptr, eps0);
        double2 *t = src;
        src = dst;
        dst = t;
    }
    const int64_t pc = (int64_t)g.n1 * g.R;
    const int pb = (int)((pc + 255) / 256);
    *wblocks = pb;
    hipLaunchKernelGGL(k_tent_pack<T>, dim3(pb), dim3(256), 0, s, src, rho, g.n, g.R, Ma, g.nzp,
                       psi, ftab, psi0, wpart);
    return hipGetLastError();
}

hipError_t launch_tent_combine(hipStream_t s, const double *env, const double *q, const double *m,
                               const double *Fk, const double *Pk, int64_t N, double kick,
                               double *vel, double *F, double *phi)
{
    const int64_t blocks = (N + 255) / 256;
    hipLaunchKernelGGL(k_tent_combine, dim3((unsigned)blocks), dim3(256), 0, s, env, q, m, Fk, Pk,
                       N, kick, vel, F, phi);
    return hipGetLastError();
}

template hipError_t launch_tent_solve<float>(hipStream_t, const double2 *, const Geom &, int, const double *, const double *, const double *, double, double2 *, double2 *, double2 *, float *, float *, double *, int *);
template hipError_t launch_tent_solve<double>(hipStream_t, const double2 *, const Geom &, int, const double *, const double *, const double *, double, double2 *, double2 *, double2 *, double *, double *, double *, int *);

}  // namespace sce
