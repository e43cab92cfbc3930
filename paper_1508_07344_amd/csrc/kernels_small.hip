// Small periodic systems: one workgroup runs many leapfrog steps in one
// launch.  A step of a system with a few particles and a few thousand modes is
// otherwise bound by the latency of its five dependent kernels (about 4-5 us
// each); here every phase of the step (drift, phase tables, deposit, solve,
// force, kicks) is a stage of one kernel separated by workgroup barriers, and
// the particle state stays on chip between steps.  FP64 throughout.
//
// Per step, with the half space H given as integer triplets and the per-mode
// weight w_n = S(k_n)^2 / (eps0 |k_n|^2 V):
//   tables   T[j][d][m] = exp(2 pi i m x_jd / L), m = 0..n, each from its own
//            FP64 sincos of the exactly reduced phase (Section 8's per-axis
//            powers, here evaluated directly);
//   deposit  psi_n = w_n sum_j q_j conj(e_nj), e_nj = prod_d T[j][d][n_d]
//            (negative n_d by conjugation): psi = S rho / (eps0 k^2 V);
//   force    F_j = 2 q_j (2 pi / L) sum_n n Im(psi_n e_nj), the threads of a
//            particle summing interleaved slices of H, then a fixed-order
//            butterfly over the slices within each wave and, when a
//            particle spans several waves, a fixed-order sum of the waves'
//            partials (deterministic, one barrier);
//   kicks and drift as in the multi-kernel step (wrap into [0, L)).

#include <hip/hip_runtime.h>

#include "sce_device.h"
#include "sce_internal.h"

namespace sce {

namespace {

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline double wrap_small(double x, double L, double invL)
{
    double w = x - L * floor(x * invL);
    if (w >= L || w < 0.0) w = 0.0;
    return w;
}

}  // namespace

template <bool KDK>
__global__ void __launch_bounds__(kSmallThreads)
k_step_small(double *__restrict__ pos, double *__restrict__ vel, double *__restrict__ F,
             const double *__restrict__ q, const double *__restrict__ m, int N,
             const short4 *__restrict__ modes, const double *__restrict__ wmode, int H, int n,
             double L, double dt, int steps)
{
    // 158 KB of LDS: the mode list and weights are read every step, so they
    // are copied in once per launch
    __shared__ double2 psi[kSmallMaxH];
    __shared__ double2 tab[kSmallMaxTab];
    __shared__ short4 md[kSmallMaxH];
    __shared__ double wm[kSmallMaxH];
    __shared__ double xs[3][kSmallMaxN];
    __shared__ double qs[kSmallMaxN];
    __shared__ double red[3][kSmallMaxN];  // per particle, or per wave (at most 16)
    const int t = threadIdx.x;
    for (int h = t; h < H; h += kSmallThreads) {
        md[h] = modes[h];
        wm[h] = wmode[h];
    }
    const int n1 = n + 1;
    const double invL = 1.0 / L, kf = 6.283185307179586476925286766559 * invL;

    double x[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0}, f[3] = {0.0, 0.0, 0.0}, qj = 0.0, mj = 1.0;
    if (t < N) {
        for (int d = 0; d < 3; ++d) {
            x[d] = pos[d * N + t];
            v[d] = vel[d * N + t];
            f[d] = F[d * N + t];
        }
        qj = q[t];
        mj = m[t];
        qs[t] = qj;
    }
    // force slices: S threads per particle, S a power of two with N S <= kSmallThreads
    int S = 1;
    while (2 * S * N <= kSmallThreads) S *= 2;
    const int fj = t / S, fsl = t - (t / S) * S;
    const bool fown = fj < N;

    auto axis = [&](int j, int d, int k) {
        const double2 c = tab[(j * 3 + d) * n1 + (k < 0 ? -k : k)];
        return k < 0 ? make_double2(c.x, -c.y) : c;
    };
    auto phase = [&](int j, short4 mo) {
        double2 p = axis(j, 2, mo.z);
        if (mo.y) p = cmul(p, axis(j, 1, mo.y));
        if (mo.x) p = cmul(p, axis(j, 0, mo.x));
        return p;
    };
    // F of every particle at the positions x (threads t < N hold them)
    auto fields = [&]() {
        if (t < N)
            for (int d = 0; d < 3; ++d) xs[d][t] = x[d];
        __syncthreads();
        for (int e = t; e < N * 3 * n1; e += kSmallThreads) {
            const int j = e / (3 * n1), r = e - j * 3 * n1, d = r / n1, k = r - d * n1;
            double c, s;
            cis_turns(frac_mul(k, frac(xs[d][j] * invL)), c, s);
            tab[e] = make_double2(c, s);
        }
        __syncthreads();
        for (int h = t; h < H; h += kSmallThreads) {
            const short4 mo = md[h];
            double rr = 0.0, ri = 0.0;
            for (int j = 0; j < N; ++j) {
                const double2 p = phase(j, mo);
                rr = fma(qs[j], p.x, rr);
                ri = fma(-qs[j], p.y, ri);
            }
            const double w = wm[h];
            psi[h] = make_double2(w * rr, w * ri);
        }
        __syncthreads();
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        if (fown) {
            for (int h = fsl; h < H; h += S) {
                const short4 mo = md[h];
                const double2 p = phase(fj, mo), ps = psi[h];
                const double im = ps.x * p.y + ps.y * p.x;
                a0 = fma((double)mo.x, im, a0);
                a1 = fma((double)mo.y, im, a1);
                a2 = fma((double)mo.z, im, a2);
            }
        }
        // every lane takes part in the butterfly (lanes past N S carry zeros);
        // groups of S < 64 lanes are aligned, so offsets below S stay inside
        const int wsum = S < 64 ? S : 64;
        for (int o = wsum >> 1; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o, 64);
            a1 += __shfl_xor(a1, o, 64);
            a2 += __shfl_xor(a2, o, 64);
        }
        const bool head = S <= 64 ? (fown && fsl == 0) : ((t & 63) == 0);
        const int slot = S <= 64 ? fj : (t >> 6);
        if (head) {
            red[0][slot] = a0;
            red[1][slot] = a1;
            red[2][slot] = a2;
        }
        __syncthreads();
        if (t < N) {
            const int nw = S <= 64 ? 1 : S >> 6;  // the particle's waves
            const double c = 2.0 * qj * kf;
            for (int d = 0; d < 3; ++d) {
                double sum = 0.0;
                for (int i = 0; i < nw; ++i) sum += red[d][t * nw + i];
                f[d] = c * sum;
            }
        }
        __syncthreads();
    };

    for (int s = 0; s < steps; ++s) {
        if (KDK) {
            if (t < N) {
                const double a = 0.5 * dt / mj;
                for (int d = 0; d < 3; ++d) {
                    v[d] = fma(a, f[d], v[d]);
                    x[d] = wrap_small(x[d] + dt * v[d], L, invL);
                }
            }
            fields();
            if (t < N) {
                const double a = 0.5 * dt / mj;
                for (int d = 0; d < 3; ++d) v[d] = fma(a, f[d], v[d]);
            }
        } else {
            if (t < N)
                for (int d = 0; d < 3; ++d) x[d] = wrap_small(x[d] + 0.5 * dt * v[d], L, invL);
            fields();
            if (t < N) {
                const double a = dt / mj;
                for (int d = 0; d < 3; ++d) {
                    v[d] = fma(a, f[d], v[d]);
                    x[d] = wrap_small(x[d] + 0.5 * dt * v[d], L, invL);
                }
            }
        }
    }
    if (t < N) {
        for (int d = 0; d < 3; ++d) {
            pos[d * N + t] = x[d];
            vel[d * N + t] = v[d];
            F[d * N + t] = f[d];
        }
    }
}

hipError_t launch_step_small(hipStream_t s, double *pos, double *vel, double *F, const double *q,
                             const double *m, int64_t N, const short4 *modes, const double *wmode,
                             const Geom &g, double L, double dt, int steps, bool kdk)
{
    if (N < 1 || N > kSmallMaxN || g.H > kSmallMaxH || N * 3 * (g.n + 1) > kSmallMaxTab || steps < 1)
        return hipErrorInvalidValue;
    if (kdk)
        hipLaunchKernelGGL(k_step_small<true>, dim3(1), dim3(kSmallThreads), 0, s, pos, vel, F, q, m,
                           (int)N, modes, wmode, (int)g.H, g.n, L, dt, steps);
    else
        hipLaunchKernelGGL(k_step_small<false>, dim3(1), dim3(kSmallThreads), 0, s, pos, vel, F, q, m,
                           (int)N, modes, wmode, (int)g.H, g.n, L, dt, steps);
    return hipGetLastError();
}

}  // namespace sce
